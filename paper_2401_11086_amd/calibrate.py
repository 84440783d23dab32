"""Calibrate relaxation times against shock profiles with the adjoint.

Workload: Ma = 3 shock, D3Q729 (D1Q9 degree 11), N = 5, Nx cells of half an
up-stream mean free path, `steps` steps from the tanh profile.  The target
rho, theta, q_x profiles are the forward run with the Table 4 times; the fit
starts from those times perturbed by +-20 % (seeded) and runs gradient
descent on log tau with Armijo backtracking.  The adjoint gradient at the
start is checked against central differences of the GPU forward.
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import _lib as C
from . import workloads as W
from .adjoint import ShockFit, tau_keys
from .lattice import Lattice
from .presets import tau_table
from .shocks import shock_domain


def build(mach=3.0, nx=600, steps=3000, every=100, order=5):
    ab, deg = [1, 2, 3, 5], 11
    c_l, _ = C.solve_quadrature(ab, deg)
    theta1 = {1.5: 0.714, 3.0: 0.333, 5.0: 0.167}.get(mach)
    st = C.shock_states(mach, theta1=theta1 or 0.0, theta2=0.0 if theta1 else 1.07, c_l=c_l)
    dom, fields, _ = shock_domain(mach, nx, c_l, theta2=st["theta2"])
    tau_true = tau_table("smrt", 1.0, order)
    lat = Lattice(ab, deg, order, tau_true, [dom], shift_k=(int(st["k"]), 0, 0), precision="fp64_contract")
    f0 = lat.equilibrium(torch.tensor(fields, dtype=torch.float64, device="cuda"))
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    cur = lat.step(fa, fb, steps)
    m = lat.moments(cur, C.MOM_BASIC | C.MOM_Q)
    target = torch.stack([m[0], m[4], m[5]]).contiguous()
    scales = (1.0 / (st["rho2"] - st["rho1"]), 1.0 / (st["theta2"] - st["theta1"]), 1.0 / st["theta1"] ** 1.5)
    fit = ShockFit(lat, f0, target, scales, steps, every)
    return lat, fit, tau_true


def loss_grad(fit, tau):
    fit.set_tau([tau[k] for k in fit.keys])
    L = fit.forward()
    g = fit.backward()
    return L, dict(zip(fit.keys, g))


def loss_only(fit, tau):
    fit.set_tau([tau[k] for k in fit.keys])
    return fit.forward()


def descend(fit, tau, iters, L0=None, g0=None, log=None):
    """Gradient descent on log tau with Armijo backtracking (step doubled after each accepted
    step, halved while the sufficient-decrease test fails): returns the final times and the
    misfit after every iteration (history[0] is the start)."""
    keys = fit.keys
    if L0 is None or g0 is None:
        L0, g0 = loss_grad(fit, tau)
    hist = [L0]
    L, g = L0, g0
    logt = {k: math.log(tau[k]) for k in keys}
    eta = 0.05 / max(abs(g[k] * tau[k]) for k in keys)
    for it in range(iters):
        gl = {k: g[k] * math.exp(logt[k]) for k in keys}
        gn2 = sum(v * v for v in gl.values())
        while True:
            trial = {k: logt[k] - eta * gl[k] for k in keys}
            Lt = loss_only(fit, {k: math.exp(v) for k, v in trial.items()})
            if Lt <= L - 1e-4 * eta * gn2 or eta < 1e-12:
                break
            eta *= 0.5
        logt = trial
        L, g = loss_grad(fit, {k: math.exp(v) for k, v in logt.items()})
        hist.append(L)
        eta *= 2.0
        if log is not None:
            log(it + 1, L)
    return {k: math.exp(v) for k, v in logt.items()}, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=600)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--fd-h", type=float, default=1e-4)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.time()
    lat, fit, tau_true = build(nx=args.nx, steps=args.steps, every=args.every)
    keys = fit.keys
    tau0 = W.perturbed_taus({k: tau_true[k] for k in keys}, seed=0, frac=0.2)
    tau = dict(tau0)
    L0, g0 = loss_grad(fit, tau)
    ta = time.time()
    _, _ = loss_grad(fit, tau)
    t_grad = time.time() - ta
    # central differences of the GPU forward, tau_nm (1 +- h)
    fd = {}
    for k in keys:
        tp, tm = dict(tau), dict(tau)
        tp[k] *= 1 + args.fd_h
        tm[k] *= 1 - args.fd_h
        fd[k] = (loss_only(fit, tp) - loss_only(fit, tm)) / (2 * args.fd_h * tau[k])
    gmax = max(abs(v) for v in g0.values())
    fd_err = {f"{n}{m}": abs(g0[(n, m)] - fd[(n, m)]) / gmax for (n, m) in keys}
    print(f"L0 = {L0:.6e}, adjoint vs FD max rel err {max(fd_err.values()):.2e}", file=sys.stderr, flush=True)
    tau_fit, hist = descend(fit, tau, args.iters, L0, g0,
                            log=lambda it, L: print(f"iter {it}: L = {L:.6e}", file=sys.stderr, flush=True))
    L = hist[-1]
    rel = {f"{n}{m}": (tau_fit[(n, m)] - tau_true[(n, m)]) / tau_true[(n, m)] for (n, m) in keys}
    rel0 = {f"{n}{m}": (tau0[(n, m)] - tau_true[(n, m)]) / tau_true[(n, m)] for (n, m) in keys}
    out = dict(workload=f"Ma=3 shock, Nx={args.nx}, D3Q729, N=5, {args.steps} steps, checkpoints every {args.every}",
               loss_start=L0, loss_end=L, loss_ratio=L / L0, iters=args.iters,
               grad_seconds=round(t_grad, 3), fd_h=args.fd_h, adjoint_vs_fd_rel=fd_err,
               tau_rel_error_start=rel0, tau_rel_error_end=rel, loss_history=hist,
               wall_s=round(time.time() - t0, 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
