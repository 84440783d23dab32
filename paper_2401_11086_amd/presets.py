"""Relaxation-time tables tau*_nm = tau_nm / tau_20 (Table 4 and the paper's variants)."""
from fractions import Fraction as F

_KEYS = [(2, 0), (3, 0), (3, 1), (4, 0), (4, 1), (4, 2), (5, 0), (5, 1), (5, 2)]

# Table 4, SMRT columns (Maxwell molecules)
SMRT = {(2, 0): F(1), (3, 0): F(2, 3), (3, 1): F(3, 2), (4, 0): F(432, 763), (4, 1): F(6, 7), (4, 2): F(3, 2),
        (5, 0): F(864, 1655), (5, 1): F(108, 163), (5, 2): F(1)}
# Table 4, Shakhov columns: tau_31 = tau_20 / Pr with Pr = 2/3, all others equal
SHAKHOV = {k: F(1) for k in _KEYS}
SHAKHOV[(3, 1)] = F(3, 2)
# single relaxation time
BGK = {k: F(1) for k in _KEYS}
# Sec. 4.3: SMRT with the two n = 4, m >= 1 parts forced to 6/7
REDUCED = dict(SMRT)
REDUCED[(4, 1)] = F(6, 7)
REDUCED[(4, 2)] = F(6, 7)
# one time per Hermite order (lumped): 1, 3/2 (keeps Pr = 2/3), 6/7, 108/163
LUMPED = {(n, m): {2: F(1), 3: F(3, 2), 4: F(6, 7), 5: F(108, 163)}[n] for (n, m) in _KEYS}

PRESETS = {"smrt": SMRT, "shakhov": SHAKHOV, "bgk": BGK, "reduced": REDUCED, "lumped": LUMPED}
# SMRT with the exact inverse-fifth-power kernel average (Sec. 2.1): tau*_40, tau*_50, tau*_51
# differ from Table 4 (whose kernel average is <sin^4 chi>/<sin^2 chi> = 7/9); computed on
# first use by the deflection-angle quadrature of wcu.py
_COMPUTED = {"smrt_exact_kernel": None}


def preset(name):
    """{(n, m): tau*_nm} of a named preset (Fractions for the tabulated ones, floats for the
    exact-kernel one)."""
    if name in PRESETS:
        return PRESETS[name]
    if name in _COMPUTED:
        if _COMPUTED[name] is None:
            from .wcu import tau_star_exact_kernel
            t = tau_star_exact_kernel(5)
            _COMPUTED[name] = {k: t[k] for k in _KEYS}
        return _COMPUTED[name]
    raise KeyError(f"unknown relaxation preset {name!r}; known: {sorted(PRESETS) + sorted(_COMPUTED)}")


def tau_table(name, tau20=1.0, N=5):
    """{(n, m): tau_nm} for n <= N from a preset scaled by tau_20."""
    return {k: float(v) * tau20 for k, v in preset(name).items() if k[0] <= N}
