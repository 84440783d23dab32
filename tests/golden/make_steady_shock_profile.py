"""Writes the oracle's steady shock profiles held in this folder, one file per case:

    steady_shock_ma1.5_q343_n4_nx48.txt          Ma 1.5, D3Q343, N = 4, Table 4 tau, 48 cells
    steady_shock_ma7_q729_n5_nx400.txt           Ma 7, D3Q729, N = 5, Table 4 tau, 400 cells
    steady_shock_ma3_q729_n5_nx300_lumped.txt    Ma 3, D3Q729, N = 5, one tau per order, 300 cells

Set-up of the paper's shock tubes (Sec. 4.2): D3Q343 is the degree-9 rule on r {0, +-1, +-2, +-3},
D3Q729 the degree-11 rule on r {0, +-1, +-2, +-3, +-5} (Table 3); relaxation times from Table 4
(or the lumped reading: 1, 3/2, 6/7, 108/163 per order) with tau_20 from cells of half an
upstream mean free path, Rankine-Hugoniot end states, a tanh initial profile.  The tubes are long
enough for the shock's tails to decay before the fixed ends: with 100 cells at Ma 3 the upstream
tail still reaches the inflow end (rho there 3e-7 above its Rankine-Hugoniot value) and the shock
creeps upstream at about 1e-6 cells per step instead of settling.  The FP64 oracle
runs until no cell's rho or theta changes by more than 1e-8 between samples 100 steps apart (or,
for a shock that still creeps, until that change has stayed constant below 1e-6 for 2000 steps;
the header gives the step count, which a comparison repeats), and the normalised profiles rho_hat, theta_hat (0 upstream, 1 downstream) and q_hat = q_x / (rho1
theta1^{3/2}) of the pre-collision state are written.  Only the oracle is called.

    python tests/golden/make_steady_shock_profile.py [case ...]   # all cases when none is named
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from cases import D1Q7, D1Q9, shock_case  # noqa: E402

EVERY, TOL, DRIFT = 100, 1e-8, 1e-6
# name: (Mach, Nx, stencil, N, relaxation table, description)
CASES = {
    "ma1.5_q343_n4_nx48": (1.5, 48, D1Q7, 4, None, "Steady Ma = 1.5 shock, D3Q343, N = 4, Nx = 48, Table 4 tau"),
    "ma7_q729_n5_nx400": (7.0, 400, D1Q9, 5, None, "Steady Ma = 7 shock, D3Q729, N = 5, Nx = 400, Table 4 tau"),
    "ma3_q729_n5_nx300_lumped": (3.0, 300, D1Q9, 5, O.tau_star_lumped(),
                                 "Steady Ma = 3 shock, D3Q729, N = 5, Nx = 300, one tau per order (lumped)"),
}


def path_of(name):
    return os.path.join(HERE, f"steady_shock_{name}.txt")


def run(name):
    mach, nx, stencil, N, table, desc = CASES[name]
    case = shock_case(mach, nx, stencil, N, table=table)
    model, dom, st = case["model"], case["dom"], case["states"]
    f = O.equilibrium_f(case["fields"][0], case["fields"][1:4], case["fields"][4], model).reshape(-1, 1, 1, nx)
    ob = O.observables(f, model, dom)
    prev = np.stack([ob["rho"], ob["theta"]])
    steps, history = 0, []
    while True:
        for _ in range(EVERY):
            f = O.step(f, model, dom)
        steps += EVERY
        ob = O.observables(f, model, dom)
        now = np.stack([ob["rho"], ob["theta"]])
        change = float(np.abs(now - prev).max())
        prev = now
        history.append(change)
        if steps % 2000 == 0:
            print(f"{name}: {steps} steps, change {change:.3e}", flush=True)
        if change < TOL:
            break
        # a shock that creeps at a constant rate (its tails still touch the fixed ends) never
        # meets TOL: stop once the change has stayed constant to 0.1 % over 2000 steps below DRIFT
        old = history[-21] if len(history) > 20 else None
        if old is not None and change < DRIFT and abs(change - old) < 1e-3 * change:
            break
    rho_h = (ob["rho"] - st["rho1"]) / (st["rho2"] - st["rho1"])
    th_h = (ob["theta"] - st["theta1"]) / (st["theta2"] - st["theta1"])
    q_h = ob["q"][0] / (st["rho1"] * st["theta1"] ** 1.5)
    with open(path_of(name), "w") as fh:
        fh.write(f"# {desc}, cells of half an upstream mean\n")
        fh.write("# free path (Sec. 4.2); FP64 oracle run to a max change of rho, theta below 1e-8 per 100 steps.\n"
                 if change < TOL else
                 "# free path (Sec. 4.2); FP64 oracle run until the change of rho, theta per 100 steps stayed constant\n")
        fh.write(f"# written by make_steady_shock_profile.py; steps {steps}, last change {change:.3e}\n")
        fh.write("# x  rho_hat  theta_hat  q_hat\n")
        for x in range(nx):
            fh.write(f"{x} {rho_h[x]:.12e} {th_h[x]:.12e} {q_h[x]:.12e}\n")
    print(path_of(name), steps, change, flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or list(CASES):
        run(n)
