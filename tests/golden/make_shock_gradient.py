"""Writes shock_gradient_ma3_q729_n5_nx600.txt and shock_target_ma3_q729_n5_nx600.txt: the FP64
oracle's misfit and its gradient with respect to the relaxation times for the calibration shock.

Set-up (Sec. 4.2 shock tube, Table 4 relaxation times): Ma = 3, D3Q729 (the degree-11 rule on
r {0, +-1, +-2, +-3, +-5}, Table 3), N = 5, Nx = 600 cells of half an upstream mean free path,
the tanh initial profile as the truncated equilibrium rounded to float32 (the state the HIP
library stores).  The target profiles rho*, theta*, q_x* are the oracle's pre-collision moments
after STEPS steps with the Table 4 times.  The misfit
    L = sum_x [s_rho^2 (rho - rho*)^2 + s_theta^2 (theta - theta*)^2 + s_q^2 (q_x - q_x*)^2],
s = 1/(rho2 - rho1), 1/(theta2 - theta1), 1/theta1^{3/2}, is taken at the relaxation times
perturbed by U[-0.2, 0.2] (seed 0, in the order of the sorted (n, m) keys), and each dL/dtau_nm
is a complex-step derivative of the oracle's forward (step 1e-30): exact to FP64 rounding, with
no difference step.  One process per relaxation time.  Only the oracle is called.

    python tests/golden/make_shock_gradient.py [steps]     # 3000 steps: ~6 minutes on 8 cores
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from cases import D1Q9, shock_case  # noqa: E402
from paper_2401_11086_amd import workloads as W  # noqa: E402

MACH, NX, N = 3.0, 600, 5
H_CS = 1e-30
KEYS = [(n, m) for n in range(2, N + 1) for m in range(n // 2 + 1) if (n, m) != (2, 1)]
GRAD = os.path.join(HERE, "shock_gradient_ma3_q729_n5_nx600.txt")
TARGET = os.path.join(HERE, "shock_target_ma3_q729_n5_nx600.txt")


def setup():
    case = shock_case(MACH, NX, D1Q9, N)
    f = O.equilibrium_f(case["fields"][0], case["fields"][1:4], case["fields"][4], case["model"])
    f0 = f.astype(np.float32).astype(np.float64).reshape(-1, 1, 1, NX)
    st = case["states"]
    scales = (1.0 / (st["rho2"] - st["rho1"]), 1.0 / (st["theta2"] - st["theta1"]), 1.0 / st["theta1"] ** 1.5)
    return case, f0, scales


def forward(case, f0, tau, steps):
    full = dict(case["model"].tau)
    full.update(tau)
    m = O.Model(vs=case["model"].vs, N=N, tau=full, shift=case["model"].shift, rho_ref=1.0)
    f = f0
    for _ in range(steps):
        f = O.step(f, m, case["dom"])
    return f, m


def _loss_job(args):
    key, steps, target, tau0 = args
    case, f0, scales = setup()
    tau = dict(tau0)
    if key is not None:
        tau[key] = complex(tau0[key], H_CS)
    f, m = forward(case, f0, tau, steps)
    L = O.shock_loss(f, m, case["dom"], target, scales)
    return key, (float(np.real(L)) if key is None else float(np.imag(L)) / H_CS)


def main(steps):
    case, f0, scales = setup()
    f, m = forward(case, f0, {}, steps)
    ob = O.observables(f, m, case["dom"])
    target = dict(rho=ob["rho"], theta=ob["theta"], q_x=ob["q"][0])
    tau0 = W.perturbed_taus({k: case["model"].tau[k] for k in KEYS}, seed=0, frac=0.2)
    jobs = [(k, steps, target, tau0) for k in [None] + KEYS]
    with mp.get_context("fork").Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        res = dict(pool.map(_loss_job, jobs))
    with open(TARGET, "w") as fh:
        fh.write(f"# Ma = 3 shock, D3Q729, N = 5, Nx = 600: oracle pre-collision rho, theta, q_x after {steps}\n")
        fh.write("# steps with the Table 4 relaxation times (written by make_shock_gradient.py)\n")
        fh.write("# x  rho  theta  q_x\n")
        for x in range(NX):
            fh.write(f"{x} {target['rho'][x]:.17e} {target['theta'][x]:.17e} {target['q_x'][x]:.17e}\n")
    with open(GRAD, "w") as fh:
        fh.write(f"# Ma = 3 shock, D3Q729, N = 5, Nx = 600, {steps} steps: FP64 oracle misfit L at the perturbed\n")
        fh.write("# relaxation times and its complex-step gradient (written by make_shock_gradient.py)\n")
        fh.write(f"steps {steps}\n")
        fh.write(f"loss {res[None]:.17e}\n")
        fh.write("# n m  tau_nm (perturbed, dt units)  dL/dtau_nm\n")
        for k in KEYS:
            fh.write(f"{k[0]} {k[1]} {tau0[k]:.17e} {res[k]:.17e}\n")
    print(GRAD, res, flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 3000)
