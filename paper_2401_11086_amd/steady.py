"""Run shock tubes to a steady state.

The state is sampled every `every` steps; it is steady when at every node
the change of rho and theta since the previous sample is within
max(tol_abs, ulps * spacing(value)), the spacing being that of float32 (the
storage precision).  A shock between fixed ends is translation-neutral, so the
aligned shape is reported as well as the raw change.
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import _lib as C
from .lattice import Lattice
from .presets import tau_table
from .shocks import shock_domain


class MomentStepper:
    """Adapter that advances a moment state (lbsmrt_step_moment_state) behind the step / moments
    calls run_to_steady makes; moments are taken from the expanded populations."""

    def __init__(self, lat):
        self.lat = lat
        self.work = lat.new_moment_work()
        self.f = lat.new_state()

    def step(self, ma, mb, n):
        return self.lat.step_moment_state(ma, mb, self.work, n)

    def moments(self, m, mask):
        return self.lat.moments(self.lat.expand_state(m, out=self.f), mask)

    def sync(self):
        self.lat.sync()


def run_to_steady(lat, fa, fb, every=100, max_steps=400000, tol_abs=1e-8, ulps=8, progress=None):
    """lat: a Lattice (fa, fb population states) or a MomentStepper (fa, fb moment states)."""
    m = lat.moments(fa, C.MOM_BASIC)
    prev = torch.stack([m[0], m[4]]).cpu().numpy()
    steps = 0
    history = []
    while steps < max_steps:
        cur = lat.step(fa, fb, every)
        if cur is fb:
            fa, fb = fb, fa
        steps += every
        m = lat.moments(fa, C.MOM_BASIC)
        now = torch.stack([m[0], m[4]]).cpu().numpy()
        if not np.all(np.isfinite(now)):
            lat.sync()
            return dict(steps=steps, converged=False, diverged=True), fa
        change = np.abs(now - prev)
        bound = np.maximum(tol_abs, ulps * np.spacing(np.abs(now).astype(np.float32)).astype(np.float64))
        dmax = float(change.max())
        history.append(dmax)
        if progress and steps % (100 * every) == 0:
            progress(f"{steps} steps: max change {dmax:.3e}")
        if np.all(change <= bound):
            fired = "absolute 1e-8" if np.all(change <= tol_abs) else f"{ulps} float32 ulps"
            lat.sync()
            return dict(steps=steps, converged=True, diverged=False, max_change=dmax, criterion=fired), fa
        prev = now
    lat.sync()
    return dict(steps=steps, converged=False, diverged=False, max_change=history[-1] if history else None), fa


def shock_thickness(rho, st):
    """Maximum-slope thickness (rho2 - rho1) / max|d rho/dx| in cells."""
    return float((st["rho2"] - st["rho1"]) / np.abs(np.diff(rho)).max())


def main():
    ap = argparse.ArgumentParser(description="run one shock tube to a steady state on the GPU")
    ap.add_argument("--mach", type=float, default=3.0)
    ap.add_argument("--nx", type=int, default=1000)
    ap.add_argument("--tau", default="smrt", choices=["smrt", "lumped", "shakhov", "bgk", "reduced", "smrt_exact_kernel"])
    ap.add_argument("--stencil", default="d1q9", choices=["d1q7", "d1q9", "d1q17"])
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--lanes-per-node", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="lanes per node of the step kernel (0: the library's default)")
    ap.add_argument("--additive", action="store_true",
                    help="additive collision f* = g + R (a' - a) instead of the rebuild from the moments")
    ap.add_argument("--moment-state", action="store_true",
                    help="hold the state as the M moments of each node (lbsmrt_step_moment_state)")
    args = ap.parse_args()
    ab, deg = {"d1q7": ([1, 2, 3], 9), "d1q9": ([1, 2, 3, 5], 11),
               "d1q17": ([1, 2, 3, 4, 5, 6, 7, 9], 19)}[args.stencil]
    theta1 = {1.5: 0.714, 3.0: 0.333, 5.0: 0.167, 7.0: 0.071}.get(args.mach)
    c_l, _ = C.solve_quadrature(ab, deg)
    st = C.shock_states(args.mach, theta1=theta1 or 0.0, theta2=0.0 if theta1 else 1.07, c_l=c_l)
    dom, fields, _ = shock_domain(args.mach, args.nx, c_l, theta2=st["theta2"])
    k = int(st["k"])
    lat = Lattice(ab, deg, args.order, tau_table(args.tau, 1.0, args.order), [dom], shift_k=(k, 0, 0),
                  precision="fp64_contract", regularized=not args.additive)
    if args.lanes_per_node:
        lat.set_launch("direct", 0, 64, args.lanes_per_node)
    fields_t = torch.tensor(fields, dtype=torch.float64, device="cuda")
    if args.moment_state:
        stepper = MomentStepper(lat)
        fa, fb = lat.equilibrium_moments(fields_t), lat.new_moment_state()
    else:
        stepper = lat
        fa, fb = lat.equilibrium(fields_t), lat.new_state()
    t0 = time.time()
    res, fa = run_to_steady(stepper, fa, fb, max_steps=args.max_steps,
                            progress=lambda s: print(s, file=sys.stderr, flush=True))
    res["wall_s"] = round(time.time() - t0, 2)
    if res.get("converged"):
        m = stepper.moments(fa, C.MOM_BASIC | C.MOM_Q).cpu().numpy()
        res["shock_thickness_cells"] = round(shock_thickness(m[0], st), 3)
        res["max_theta"] = round(float(m[4].max()), 4)
        res["min_q_x"] = round(float(m[5].min()), 6)
    res.update(mach=args.mach, nx=args.nx, tau=args.tau, Q=lat.Q, N=lat.N, k=k, additive=args.additive,
               moment_state=args.moment_state,
               theta1=st["theta1"],
               theta2=st["theta2"], rho2=st["rho2"], launch=lat.launch_settings())
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
