"""Truncation order N = 4 against N = 5 on steady normal shocks (Sec. 4.2-4.3).

The paper runs every shock at both truncations with otherwise identical parameters and finds
that the fourth-order model departs from the fifth-order one first in the fourth moments, and
at higher Mach numbers in lower moments too.  This driver runs each Mach number at N = 4 and
N = 5 on the same D3Q729 velocity set (SMRT relaxation times of Table 4, cells of half an
upstream mean free path) to a steady state, aligns the two density profiles at their
rho_hat = 1/2 crossing, and reports the largest difference of each normalised profile:
rho_hat, theta_hat, q_x / (rho1 theta1^{3/2}), sigma_xx, and the fourth-moment quantities
R41_xx and R42 (scaled by rho1 theta1^2).

    python -m paper_2401_11086_amd.truncation --mach 1.5 3 5 --nx 400
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib as C
from .lattice import Lattice
from .presets import tau_table
from .shocks import shock_domain
from .steady import run_to_steady

THETA1 = {1.5: 0.714, 3.0: 0.333, 5.0: 0.167, 7.0: 0.071}   # Table 3


def _crossing(rho_hat):
    """x (cells) where rho_hat first reaches 1/2, linearly interpolated."""
    i = int(np.argmax(rho_hat >= 0.5))
    y0, y1 = rho_hat[i - 1], rho_hat[i]
    return i - 1 + (0.5 - y0) / (y1 - y0)


def steady_profiles(mach, order, nx, additive=False, max_steps=400000):
    ab, deg = [1, 2, 3, 5], 11
    c_l, _ = C.solve_quadrature(ab, deg)
    th1 = THETA1.get(mach)
    st = C.shock_states(mach, theta1=th1 or 0.0, theta2=0.0 if th1 else 1.07, c_l=c_l)
    dom, fields, _ = shock_domain(mach, nx, c_l, theta2=st["theta2"])
    lat = Lattice(ab, deg, order, tau_table("smrt", 1.0, order), [dom], shift_k=(int(st["k"]), 0, 0),
                  precision="fp64_contract", regularized=not additive)
    fa = lat.equilibrium(torch.tensor(fields, dtype=torch.float64, device="cuda"))
    try:
        res, fa = run_to_steady(lat, fa, lat.new_state(), max_steps=max_steps)
    except C.LbsmrtError as e:             # a node left the validity region (latched flag)
        if e.status != C.E_STATE:
            raise
        res = dict(steps=None, converged=False, diverged=True, left_validity_region=True)
    if res.get("diverged"):
        lat.close()
        return res, None
    mask = C.MOM_BASIC | C.MOM_SIGMA | C.MOM_Q | C.MOM_R41 | C.MOM_R42
    m = lat.moments(fa, mask).cpu().numpy()
    rho, th = m[0], m[4]
    r1, t1 = st["rho1"], st["theta1"]
    prof = {
        "rho": (rho - r1) / (st["rho2"] - r1),
        "theta": (th - t1) / (st["theta2"] - t1),
        "sigma_xx": m[5] / (r1 * t1),
        "q_x": m[11] / (r1 * t1 ** 1.5),
        "R41_xx": m[14] / (r1 * t1 ** 2),
        "R42": m[20] / (r1 * t1 ** 2),
    }
    lat.close()
    return res, prof


def compare(mach, nx, additive=False):
    out = {"mach": mach, "nx": nx, "additive": additive}
    profs = {}
    for order in (4, 5):
        t0 = time.time()
        res, prof = steady_profiles(mach, order, nx, additive)
        if res.get("diverged"):
            out[f"N{order}"] = {"steps": res["steps"], "diverged": True}
            continue
        out[f"N{order}"] = {"steps": res["steps"], "converged": res["converged"], "wall_s": round(time.time() - t0, 2),
                            "max_theta_hat": round(float(prof["theta"].max()), 4),
                            "min_q_x": round(float(prof["q_x"].min()), 5),
                            "min_R41_xx": round(float(prof["R41_xx"].min()), 5),
                            "max_R41_xx": round(float(prof["R41_xx"].max()), 5)}
        profs[order] = prof
    if len(profs) < 2:
        return out
    # align N = 4 onto N = 5 at the density crossing, compare on the interior
    dx = _crossing(profs[4]["rho"]) - _crossing(profs[5]["rho"])
    x = np.arange(nx, dtype=float)
    inner = slice(nx // 10, nx - nx // 10)
    out["shift_cells"] = round(float(dx), 3)
    out["max_abs_difference"] = {
        k: float(np.abs(np.interp(x + dx, x, profs[4][k]) - profs[5][k])[inner].max()) for k in profs[5]}
    return out


def main():
    ap = argparse.ArgumentParser(description="steady shocks at N = 4 and N = 5 on D3Q729")
    ap.add_argument("--mach", type=float, nargs="+", default=[1.5, 3.0, 5.0])
    ap.add_argument("--nx", type=int, default=400)
    ap.add_argument("--additive", action="store_true")
    args = ap.parse_args()
    for mach in args.mach:
        print(json.dumps(compare(mach, args.nx, args.additive)), flush=True)
        print(f"Ma {mach} done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
