"""Seeded synthetic inputs shared by the tests, the bench and the oracle legs.

Only random draws and input fields live here -- none of the method's
arithmetic (no equilibrium, no Rankine-Hugoniot, no collision).  Both the HIP
path and the oracle receive the same arrays from these functions.
"""
import numpy as np


def tanh_profile(nx, up, down, width=5.0, center=None):
    """Fields (rho, u_x, u_y, u_z, theta) of shape (5, nx) blending the up-stream
    state into the down-stream one with phi = (1 + tanh((x - x_c)/width)) / 2,
    x the cell index and x_c = nx/2.  up/down: (rho, u_x, theta)."""
    x = np.arange(nx, dtype=np.float64)
    xc = nx / 2.0 if center is None else center
    phi = 0.5 * (1.0 + np.tanh((x - xc) / width))
    out = np.zeros((5, nx))
    out[0] = up[0] + (down[0] - up[0]) * phi
    out[1] = up[1] + (down[1] - up[1]) * phi
    out[4] = up[2] + (down[2] - up[2]) * phi
    return out


def fourier_modes(seed=0, n_modes=16, kmax=8, amp=0.05, n_fields=5):
    """Random Fourier modes per field: integer wave-vectors k in {-kmax..kmax}^3
    with 1 <= |k| <= kmax, phases U[0, 2pi), per-mode amplitude amp/sqrt(n_modes)."""
    rng = np.random.default_rng(seed)
    ks = np.zeros((n_fields, n_modes, 3), dtype=np.int64)
    ph = np.zeros((n_fields, n_modes))
    for f in range(n_fields):
        j = 0
        while j < n_modes:
            k = rng.integers(-kmax, kmax + 1, size=3)
            nk = np.sqrt((k ** 2).sum())
            if 1.0 <= nk <= kmax:
                ks[f, j] = k
                j += 1
        ph[f] = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return ks, ph, amp / np.sqrt(n_modes)


def fourier_box(n, rho0=1.0, theta0=1.0, seed=0, n_modes=16, kmax=8, amp=0.05):
    """Fields (5, n^3), node order x fastest: rho/rho0 - 1, u/sqrt(theta0) and
    theta/theta0 - 1 each a sum of random Fourier modes on the periodic box."""
    ks, ph, a = fourier_modes(seed, n_modes, kmax, amp)
    x = np.arange(n) * (2.0 * np.pi / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    pert = np.zeros((5, n, n, n))
    for f in range(5):
        for j in range(n_modes):
            kx, ky, kz = ks[f, j]
            pert[f] += a * np.cos(kx * X + ky * Y + kz * Z + ph[f, j])
    out = np.empty((5, n ** 3))
    out[0] = rho0 * (1.0 + pert[0].reshape(-1))
    for k in range(3):
        out[1 + k] = np.sqrt(theta0) * pert[1 + k].reshape(-1)
    out[4] = theta0 * (1.0 + pert[4].reshape(-1))
    return out


def fourier_box_torch(n, device, rho0=1.0, theta0=1.0, seed=0, n_modes=16, kmax=8, amp=0.05):
    """fourier_box evaluated with torch float64 on `device` (same modes, same
    formula) for boxes too large to build quickly on the host."""
    import torch
    ks, ph, a = fourier_modes(seed, n_modes, kmax, amp)
    x = torch.arange(n, dtype=torch.float64, device=device) * (2.0 * np.pi / n)
    out = torch.empty((5, n ** 3), dtype=torch.float64, device=device)
    for f in range(5):
        acc = torch.zeros((n, n, n), dtype=torch.float64, device=device)
        for j in range(n_modes):
            kx, ky, kz = (int(v) for v in ks[f, j])
            acc += a * torch.cos(kz * x[:, None, None] + ky * x[None, :, None] + kx * x[None, None, :] + float(ph[f, j]))
        out[f] = acc.reshape(-1)
    out[0] = rho0 * (1.0 + out[0])
    out[1:4] *= np.sqrt(theta0)
    out[4] = theta0 * (1.0 + out[4])
    return out


def mach_sweep(n_shocks=64, seed=0, ma_lo=1.2, ma_hi=5.0, nx_lo=400, nx_hi=2000):
    """Batched shock draws: Ma ~ U[ma_lo, ma_hi], Nx ~ U{nx_lo..nx_hi}."""
    rng = np.random.default_rng(seed)
    ma = rng.uniform(ma_lo, ma_hi, size=n_shocks)
    nx = rng.integers(nx_lo, nx_hi + 1, size=n_shocks)
    return [(float(m), int(n)) for m, n in zip(ma, nx)]


def perturbed_taus(tau, seed=0, frac=0.2):
    """tau_nm * (1 + U[-frac, frac]) for every entry, in sorted key order."""
    rng = np.random.default_rng(seed)
    return {k: v * (1.0 + rng.uniform(-frac, frac)) for k, v in sorted(tau.items())}


def state_noise(shape, seed=0, amp=0.02):
    """Multiplicative noise factors 1 + amp*N(0,1) for perturbing a state."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.standard_normal(shape)
