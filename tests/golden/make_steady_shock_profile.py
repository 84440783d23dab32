"""Writes steady_shock_ma1.5_q343_n4_nx48.txt: the oracle's steady Ma = 1.5 shock profile.

Set-up of the paper's shock tubes (Sec. 4.2): D3Q343 (the degree-9 rule on r {0, +-1, +-2, +-3}),
Hermite order N = 4, Table 4 relaxation times with tau_20 from cells of half an upstream mean
free path, Rankine-Hugoniot end states, a tanh initial profile; 48 cells.  The FP64 oracle runs
until no cell's rho or theta changes by more than 1e-8 between samples 100 steps apart, and the
normalised profiles rho_hat, theta_hat (0 upstream, 1 downstream) and q_hat = q_x / (rho1
theta1^{3/2}) of the pre-collision state are written.  Only the oracle is called.

    python tests/golden/make_steady_shock_profile.py      # about 3 minutes on 8 cores
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from cases import D1Q7, shock_case  # noqa: E402

MACH, NX, EVERY, TOL = 1.5, 48, 100, 1e-8
OUT = os.path.join(HERE, "steady_shock_ma1.5_q343_n4_nx48.txt")


def main():
    case = shock_case(MACH, NX, D1Q7, 4)
    model, dom, st = case["model"], case["dom"], case["states"]
    f = O.equilibrium_f(case["fields"][0], case["fields"][1:4], case["fields"][4], model).reshape(-1, 1, 1, NX)
    ob = O.observables(f, model, dom)
    prev = np.stack([ob["rho"], ob["theta"]])
    steps = 0
    while True:
        for _ in range(EVERY):
            f = O.step(f, model, dom)
        steps += EVERY
        ob = O.observables(f, model, dom)
        now = np.stack([ob["rho"], ob["theta"]])
        change = float(np.abs(now - prev).max())
        prev = now
        if change < TOL:
            break
    rho_h = (ob["rho"] - st["rho1"]) / (st["rho2"] - st["rho1"])
    th_h = (ob["theta"] - st["theta1"]) / (st["theta2"] - st["theta1"])
    q_h = ob["q"][0] / (st["rho1"] * st["theta1"] ** 1.5)
    with open(OUT, "w") as fh:
        fh.write("# Steady Ma = 1.5 shock, D3Q343, N = 4, Nx = 48, Table 4 tau, cells of half an upstream mean\n")
        fh.write("# free path (Sec. 4.2); FP64 oracle run to a max change of rho, theta below 1e-8 per 100 steps.\n")
        fh.write(f"# written by make_steady_shock_profile.py; steps {steps}, last change {change:.3e}\n")
        fh.write("# x  rho_hat  theta_hat  q_hat\n")
        for x in range(NX):
            fh.write(f"{x} {rho_h[x]:.12e} {th_h[x]:.12e} {q_h[x]:.12e}\n")
    print(OUT, steps, change)


if __name__ == "__main__":
    main()
