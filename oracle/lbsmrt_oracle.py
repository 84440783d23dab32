"""Plain FP64 CPU oracle of the LB-SMRT scheme (Yan & Shan, arXiv 2401.11086).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
constant generator with the HIP library.

The method reaches a defined discrete result, so the oracle computes that same
scheme by the plainest route available, in float64 (complex128 when a caller
asks for complex-step derivatives):

* quadrature: its own root search on the even-moment equations (Sec. 4.2,
  Table 3; D1Qd rules made 3D by tensor product);
* local moments by direct summation, d_beta = sum_i g_i He_beta(v_i) with
  v_i = (c_i - u') / sqrt(theta) (Sec. 3, local expansion with rho absorbed);
* irreducible split on full 3^n symmetric tensors with explicit
  permutation-averaged symmetrisation (App. A, eq:IrrDecomp and eq:bd);
* relaxation d'^(n,m) = (1 - 1/tau_bar_nm) d^(n,m) for n >= 2 (eq:SMRT);
* return to the lattice frame by tensor Gauss-Hermite quadrature of the
  relaxed local expansion (exact: the integrand is omega times a polynomial
  of degree <= 2N);
* rebuild f_i = w_i sum_alpha a'_alpha He_alpha(c_i) / alpha!  (eq:fi with
  the 1/n! factor of eq:hermite1).

Readings of points the paper leaves open (each is a keyword argument):
  * tau_bar = tau + 1/2 (trapezoidal space-time discretisation) -- ``tau_offset_half``;
  * tau_nm(x) = tau_nm,ref * rho_ref / rho(x) (viscosity index 1 of Maxwell
    molecules, Sec. 4.2) -- ``tau_density_scaling``;
  * f rebuilt from its M moments each step (regularised), or corrected
    additively -- ``regularized``;
  * Rankine-Hugoniot temperature ratio with Ma^2 in the denominator
    (the printed equation has Ma; Table 3 is reproduced only with Ma^2);
  * eq:fi carries the 1/n! of eq:hermite1.

Pins (see tests/): quadrature against Table 3 c_l; Hermite tensors against
Table 1; projectors against Table 5 and the explicit n<=4 forms of App. A;
equilibrium moments against direct Gauss-Hermite integration of the
Maxwellian (App. B closed form); collision invariants (conservation, fixed
point, single-mode decay, BGK reduction); RH against Table 3.
Parity unpinned: steady shock profile shapes (no comparison data exists).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np
from numpy.polynomial import hermite_e as _herme

__all__ = [
    "QuadratureError", "StateError",
    "odd_double_factorial", "solve_d1_quadrature", "VelocitySet", "make_velocity_set",
    "hermite_1d", "multi_indices", "alpha_factorial",
    "full_basis_tensor", "components_of", "sym", "sym_product", "delta_power",
    "trace", "B_coef", "D_coef", "Q0", "irreducible_part", "irreducible_piece",
    "projector_matrices", "part_matrices", "trace_matrix",
    "TAU_STAR_SMRT", "TAU_STAR_SHAKHOV", "tau_star_lumped", "tau_star_bgk",
    "rankine_hugoniot", "shift_integer",
    "maxwellian_hermite_1d", "equilibrium_moments", "Model", "Domain",
    "equilibrium_f", "project", "reconstruct", "stream", "collide", "step",
    "observables", "shock_loss",
]


class QuadratureError(ValueError):
    """No real positive-weight rule exists for the requested stencil and degree."""


class StateError(ValueError):
    """A node left the validity region rho > 0, 0 < theta < 2 (Sec. 4.1)."""


# --------------------------------------------------------------------------------------
# Quadrature (Sec. 4.2: D1Qd-P1 rules, lattice constant c_l; Table 3)
# --------------------------------------------------------------------------------------

def odd_double_factorial(k: int) -> int:
    """(2k-1)!!: the 2k-th moment of the unit Gaussian; (-1)!! = 1."""
    out = 1
    for j in range(1, 2 * k, 2):
        out *= j
    return out


def _weights_for_r(abscissae, r, n_eq):
    """Weights (w_0, w_a1, ...) of the symmetric rule r*{0, +-a_j} that match the
    even Gaussian moments of orders 0, 2, ..., 2(n_eq-1).  Float64 version used
    to bracket roots."""
    p = len(abscissae)
    V = np.zeros((n_eq, p + 1))
    for k in range(n_eq):
        V[k, 0] = 1.0 if k == 0 else 0.0
        for j, a in enumerate(abscissae):
            V[k, j + 1] = 2.0 * (a * r) ** (2 * k)
    m = np.array([odd_double_factorial(k) for k in range(n_eq)], dtype=float)
    return np.linalg.solve(V, m)


def _moment_residual(abscissae, r, k_top):
    """Residual of the 2*k_top-th moment when the lower ones are matched."""
    w = _weights_for_r(abscissae, r, k_top)
    s = sum(2.0 * w[j + 1] * (a * r) ** (2 * k_top) for j, a in enumerate(abscissae))
    return s - odd_double_factorial(k_top)


def _mp_weights(abscissae, r, n_eq):
    """Same linear system in 50-digit arithmetic (the D1Q17 system is too
    ill-conditioned for float64 to reach full double accuracy)."""
    import mpmath as mp
    p = len(abscissae)
    V = mp.matrix(n_eq, p + 1)
    for k in range(n_eq):
        V[k, 0] = 1 if k == 0 else 0
        for j, a in enumerate(abscissae):
            V[k, j + 1] = 2 * (a * r) ** (2 * k)
    m = mp.matrix([odd_double_factorial(k) for k in range(n_eq)])
    return mp.lu_solve(V, m)


def _mp_residual(abscissae, r, k_top):
    w = _mp_weights(abscissae, r, k_top)
    return sum(2 * w[j + 1] * (a * r) ** (2 * k_top) for j, a in enumerate(abscissae)) - odd_double_factorial(k_top)


def solve_d1_quadrature(abscissae, degree, r_lo=0.02, r_hi=6.0, n_grid=12000):
    """Lattice constant r and weights of the 1D rule r*{0, +-a_1, ..., +-a_p}
    exact for polynomials of the given degree against exp(-x^2/2)/sqrt(2pi).

    Odd moments vanish by symmetry; the p+1 weights and r are fixed by the
    p+2 even moments 0..2(p+1).  Roots are bracketed on a float64 grid and
    refined by bisection in 50-digit arithmetic.  Among the real roots with
    every weight positive the smallest r is taken (it is the one Table 3
    prints).  Returns (r, w) with w[0] the weight of 0 and w[j] that of +-a_j.
    """
    import mpmath as mp
    abscissae = [int(a) for a in abscissae]
    p = len(abscissae)
    if sorted(set(abscissae)) != abscissae or abscissae[0] <= 0:
        raise ValueError("abscissae must be sorted distinct positive integers")
    if degree // 2 + 1 != p + 2:
        raise QuadratureError(f"{p} abscissae fix degree {2 * p + 3} (or {2 * p + 2}), not {degree}")
    k_top = p + 1
    grid = np.linspace(r_lo, r_hi, n_grid)
    res = np.array([_moment_residual(abscissae, r, k_top) for r in grid])
    with mp.workdps(50):
        for i in range(n_grid - 1):
            if not (res[i] * res[i + 1] < 0.0):
                continue
            lo, hi = mp.mpf(grid[i]), mp.mpf(grid[i + 1])
            flo = _mp_residual(abscissae, lo, k_top)
            for _ in range(120):
                mid = (lo + hi) / 2
                fm = _mp_residual(abscissae, mid, k_top)
                if (fm < 0) == (flo < 0):
                    lo, flo = mid, fm
                else:
                    hi = mid
            r = (lo + hi) / 2
            w = _mp_weights(abscissae, r, k_top)
            if all(w[j] > 0 for j in range(p + 1)):
                return float(r), np.array([float(w[j]) for j in range(p + 1)])
    raise QuadratureError(f"no positive-weight degree-{degree} rule on r*{{0,+-{abscissae}}}")


@dataclass
class VelocitySet:
    """3D tensor-product velocity set.  Population q = (ix*Q1 + iy)*Q1 + iz,
    where ix, iy, iz index the 1D integer set sorted ascending."""
    e1: np.ndarray          # 1D integers, ascending, length Q1
    c1: np.ndarray          # r * e1
    w1: np.ndarray          # 1D weights, same order
    r: float
    degree: int
    e: np.ndarray = field(init=False)   # (Q, 3) integers
    c: np.ndarray = field(init=False)   # (Q, 3)
    w: np.ndarray = field(init=False)   # (Q,)

    def __post_init__(self):
        Q1 = len(self.e1)
        idx = np.array(list(itertools.product(range(Q1), repeat=3)))
        self.e = self.e1[idx]
        self.c = self.c1[idx]
        self.w = self.w1[idx[:, 0]] * self.w1[idx[:, 1]] * self.w1[idx[:, 2]]

    @property
    def Q1(self):
        return len(self.e1)

    @property
    def Q(self):
        return len(self.e1) ** 3


def make_velocity_set(abscissae, degree) -> VelocitySet:
    r, w = solve_d1_quadrature(abscissae, degree)
    a = list(abscissae)
    e1 = np.array(sorted([-x for x in a] + [0] + a), dtype=np.int64)
    wmap = {0: w[0]}
    for j, x in enumerate(a):
        wmap[x] = w[j + 1]
        wmap[-x] = w[j + 1]
    w1 = np.array([wmap[int(x)] for x in e1])
    return VelocitySet(e1=e1, c1=r * e1.astype(float), w1=w1, r=r, degree=degree)


# --------------------------------------------------------------------------------------
# Hermite polynomials (Sec. 2.2, eq:hermite1): probabilists' He_n, tensor
# components H^(n)_alpha(xi) = prod_k He_{alpha_k}(xi_k)
# --------------------------------------------------------------------------------------

def hermite_1d(n_max: int, x):
    """He_0..He_{n_max} at x (any shape) -> array (..., n_max+1).
    He_{n+1}(x) = x He_n(x) - n He_{n-1}(x)."""
    x = np.asarray(x)
    out = np.empty(x.shape + (n_max + 1,), dtype=np.result_type(x, float))
    out[..., 0] = 1.0
    if n_max >= 1:
        out[..., 1] = x
    for n in range(1, n_max):
        out[..., n + 1] = x * out[..., n] - n * out[..., n - 1]
    return out


def multi_indices(N: int):
    """Multi-indices (a, b, c), |alpha| <= N, ordered by n = a+b+c, then a
    descending, then b descending."""
    out = []
    for n in range(N + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def alpha_factorial(alpha) -> int:
    return math.factorial(alpha[0]) * math.factorial(alpha[1]) * math.factorial(alpha[2])


def _order_slices(N):
    """Position range of each order n inside multi_indices(N)."""
    sl, start = [], 0
    for n in range(N + 1):
        cnt = (n + 1) * (n + 2) // 2
        sl.append(slice(start, start + cnt))
        start += cnt
    return sl


# --------------------------------------------------------------------------------------
# Full symmetric tensors and the irreducible decomposition (Sec. 2.2 and App. A)
# --------------------------------------------------------------------------------------

def _counts(idx_tuple):
    return (idx_tuple.count(0), idx_tuple.count(1), idx_tuple.count(2))


def full_basis_tensor(n: int, alpha) -> np.ndarray:
    """Rank-n full tensor whose entries are 1 where the index tuple has counts
    alpha and 0 elsewhere (the symmetric tensor with one distinct component)."""
    T = np.zeros((3,) * n)
    for t in itertools.product(range(3), repeat=n):
        if _counts(t) == tuple(alpha):
            T[t] = 1.0
    return T


def components_of(T: np.ndarray):
    """Distinct components of a symmetric rank-n tensor, in multi_indices order."""
    n = T.ndim
    out = []
    for (a, b, c) in [m for m in multi_indices(n) if sum(m) == n]:
        out.append(T[(0,) * a + (1,) * b + (2,) * c] if n > 0 else T[()])
    return np.array(out)


def from_components(n: int, comps) -> np.ndarray:
    T = np.zeros((3,) * n, dtype=np.result_type(np.asarray(comps), float))
    for k, alpha in enumerate([m for m in multi_indices(n) if sum(m) == n]):
        T = T + comps[k] * full_basis_tensor(n, alpha)
    return T


def sym(T: np.ndarray) -> np.ndarray:
    """Average of T over all permutations of its indices (Sec. 2.2)."""
    n = T.ndim
    if n <= 1:
        return T.copy()
    acc = np.zeros_like(T)
    perms = list(itertools.permutations(range(n)))
    for p in perms:
        acc = acc + np.transpose(T, p)
    return acc / len(perms)


def sym_product(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Symmetric product AB = sym(A (x) B), eq:symm."""
    return sym(np.multiply.outer(A, B))


def delta_power(m: int) -> np.ndarray:
    """delta^m, the m-fold symmetric product of the unit tensor (rank 2m)."""
    out = np.array(1.0)
    for _ in range(m):
        out = sym_product(out, np.eye(3))
    return out


def trace(T: np.ndarray, times: int = 1) -> np.ndarray:
    for _ in range(times):
        T = np.trace(T, axis1=0, axis2=1)
    return T


def _dfact(k: int) -> int:
    """k!! for odd k >= -1."""
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


def B_coef(n: int, m: int) -> Fraction:
    """B(n,m) of eq:bd."""
    return Fraction(math.factorial(n) * _dfact(2 * n - 4 * m + 1),
                    math.factorial(m) * 2 ** m * math.factorial(n - 2 * m) * _dfact(2 * n - 2 * m + 1))


def D_coef(n: int, m: int) -> Fraction:
    """D(n,m) of eq:bd."""
    return Fraction((-1) ** m * math.factorial(n) * _dfact(2 * n - 2 * m - 1),
                    math.factorial(m) * 2 ** m * math.factorial(n - 2 * m) * _dfact(2 * n - 1))


def Q0(l: int, X: np.ndarray) -> np.ndarray:
    """Traceless projector Q_0^(l) X = sum_k D(l,k) delta^k tr^k X (App. A)."""
    if l == 0:
        return np.array(X, dtype=float, copy=True)
    acc = np.zeros((3,) * l)
    for k in range(l // 2 + 1):
        tk = trace(X, k)
        term = tk if k == 0 else sym_product(delta_power(k), tk)
        acc = acc + float(D_coef(l, k)) * term
    return acc


def irreducible_part(T: np.ndarray, m: int) -> np.ndarray:
    """A^(n,m) = B(n,m) Q_0^(n-2m) tr^m A^(n): traceless, rank n-2m (App. A)."""
    n = T.ndim
    return float(B_coef(n, m)) * Q0(n - 2 * m, trace(T, m))


def irreducible_piece(T: np.ndarray, m: int) -> np.ndarray:
    """The rank-n term A^(n,m) delta^m of eq:IrrDecomp."""
    Anm = irreducible_part(T, m)
    if m == 0:
        return Anm
    return sym_product(Anm, delta_power(m))


_PROJ_CACHE: dict = {}
_PART_CACHE: dict = {}


def projector_matrices(n: int):
    """Matrices Pi_nm on the distinct components of rank-n symmetric tensors:
    comps(piece_m(T)) = Pi_nm @ comps(T).  Built once by applying the full-tensor
    decomposition to every basis tensor."""
    if n in _PROJ_CACHE:
        return _PROJ_CACHE[n]
    alphas = [a for a in multi_indices(n) if sum(a) == n]
    mats = []
    for m in range(n // 2 + 1):
        P = np.zeros((len(alphas), len(alphas)))
        for j, beta in enumerate(alphas):
            P[:, j] = components_of(irreducible_piece(full_basis_tensor(n, beta), m))
        mats.append(P)
    _PROJ_CACHE[n] = mats
    return mats


def trace_matrix(n: int):
    """Matrix mapping comps of a rank-n symmetric tensor to comps of its trace."""
    alphas = [a for a in multi_indices(n) if sum(a) == n]
    cols = [components_of(trace(full_basis_tensor(n, beta))) for beta in alphas]
    return np.stack(cols, axis=1)


def part_matrices(n: int):
    """Matrices mapping comps of a rank-n tensor to comps of its rank-(n-2m)
    irreducible parts A^(n,m)."""
    if n in _PART_CACHE:
        return _PART_CACHE[n]
    alphas = [a for a in multi_indices(n) if sum(a) == n]
    mats = []
    for m in range(n // 2 + 1):
        l = n - 2 * m
        dim = (l + 1) * (l + 2) // 2
        P = np.zeros((dim, len(alphas)))
        for j, beta in enumerate(alphas):
            P[:, j] = components_of(irreducible_part(full_basis_tensor(n, beta), m))
        mats.append(P)
    _PART_CACHE[n] = mats
    return mats


# --------------------------------------------------------------------------------------
# Relaxation times (Table 4, ratios tau_nm / tau_20)
# --------------------------------------------------------------------------------------

TAU_STAR_SMRT = {
    (2, 0): Fraction(1), (2, 1): Fraction(1),   # (2,1) multiplies an identically zero piece
    (3, 0): Fraction(2, 3), (3, 1): Fraction(3, 2),
    (4, 0): Fraction(432, 763), (4, 1): Fraction(6, 7), (4, 2): Fraction(3, 2),
    (5, 0): Fraction(864, 1655), (5, 1): Fraction(108, 163), (5, 2): Fraction(1),
}
TAU_STAR_SHAKHOV = {k: Fraction(1) for k in TAU_STAR_SMRT}
TAU_STAR_SHAKHOV[(3, 1)] = Fraction(3, 2)


def tau_star_bgk():
    return {k: Fraction(1) for k in TAU_STAR_SMRT}


def tau_star_lumped():
    """One tau per Hermite order: 1, 3/2 (keeps Pr = 2/3), 6/7 (the value the
    paper forces on n = 4), 108/163."""
    per_order = {2: Fraction(1), 3: Fraction(3, 2), 4: Fraction(6, 7), 5: Fraction(108, 163)}
    return {(n, m): per_order[n] for (n, m) in TAU_STAR_SMRT}


# --------------------------------------------------------------------------------------
# Shock set-up (Sec. 4.2, eq:rankine; Ma^2 in the temperature denominator)
# --------------------------------------------------------------------------------------

def rankine_hugoniot(Ma, gamma=5.0 / 3.0, theta1=None, theta2=None):
    """Up/down-stream states of a normal shock with rho1 = 1.  Give theta1 or theta2."""
    dens = (gamma + 1.0) * Ma ** 2 / ((gamma - 1.0) * Ma ** 2 + 2.0)
    tratio = ((2.0 * gamma * Ma ** 2 - gamma + 1.0) * ((gamma - 1.0) * Ma ** 2 + 2.0)
              / ((gamma + 1.0) ** 2 * Ma ** 2))
    if theta1 is None:
        theta1 = theta2 / tratio
    theta2 = theta1 * tratio
    u1 = Ma * math.sqrt(gamma * theta1)
    u2 = u1 / dens
    return dict(rho1=1.0, rho2=dens, u1=u1, u2=u2, theta1=theta1, theta2=theta2,
                u_mid=0.5 * (u1 + u2), u_half_diff=0.5 * (u1 - u2))


def shift_integer(u_mid, c_l):
    """Integer k with k*c_l closest to u_mid."""
    return int(math.floor(u_mid / c_l + 0.5))


# --------------------------------------------------------------------------------------
# Equilibrium (App. B closed form of the Maxwellian's Hermite coefficients)
# --------------------------------------------------------------------------------------

def maxwellian_hermite_1d(n_max, u, theta):
    """a^(n)(u, theta) = sum_k n! (theta-1)^k u^(n-2k) / (2^k k! (n-2k)!), n = 0..n_max,
    the 1D Hermite coefficients of a unit-density Maxwellian (App. B)."""
    u = np.asarray(u)
    theta = np.asarray(theta)
    out = np.zeros(np.broadcast(u, theta).shape + (n_max + 1,), dtype=np.result_type(u, theta, float))
    for n in range(n_max + 1):
        acc = 0.0
        for k in range(n // 2 + 1):
            acc = acc + (math.factorial(n) / (2 ** k * math.factorial(k) * math.factorial(n - 2 * k))
                         * (theta - 1.0) ** k * u ** (n - 2 * k))
        out[..., n] = acc
    return out


def equilibrium_moments(rho, u, theta, N):
    """Absolute Hermite coefficients of rho * Maxwellian(u, theta), |alpha| <= N.
    The 3D Maxwellian is a product over axes, so a_alpha = rho prod_k a^(alpha_k)(u_k).
    u has shape (3, ...).  Returns (M, ...)."""
    A = [maxwellian_hermite_1d(N, u[k], theta) for k in range(3)]
    out = [rho * A[0][..., a] * A[1][..., b] * A[2][..., c] for (a, b, c) in multi_indices(N)]
    return np.stack(out)


# --------------------------------------------------------------------------------------
# Model, domain and the step
# --------------------------------------------------------------------------------------

@dataclass
class Model:
    vs: VelocitySet
    N: int
    tau: dict                  # (n, m) -> tau_nm at rho_ref (time-step units)
    shift: tuple = (0, 0, 0)   # integer frame shift k; ubar = r * k
    rho_ref: float = 1.0
    tau_density_scaling: bool = True
    tau_offset_half: bool = True
    regularized: bool = True

    @property
    def M(self):
        return (self.N + 1) * (self.N + 2) * (self.N + 3) // 6

    @property
    def ubar(self):
        return self.vs.r * np.array(self.shift, dtype=float)

    def streaming_offsets(self):
        """Integer cell displacement of each population per step: e_i + k."""
        return self.vs.e + np.array(self.shift)[None, :]

    def hermite_matrix(self):
        """Hq[alpha, i] = He_alpha(c_i) (lattice frame, relative to ubar)."""
        H = hermite_1d(self.N, self.vs.c)          # (Q, 3, N+1)
        return np.array([H[:, 0, a] * H[:, 1, b] * H[:, 2, c] for (a, b, c) in multi_indices(self.N)])


@dataclass
class Domain:
    """Periodic box (bc_x = 0) or a 1D shock tube in x with fixed Maxwellian
    ends (bc_x = 1; ny = nz = 1, periodic in y and z), Sec. 4.2."""
    nx: int
    ny: int = 1
    nz: int = 1
    bc_x: int = 0
    state_in: tuple = None    # (rho, (ux, uy, uz), theta) left ghosts
    state_out: tuple = None   # right ghosts

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


def reconstruct(a, model: Model):
    """eq:fi with 1/alpha!:  f_i = w_i sum_alpha a_alpha He_alpha(c_i) / alpha!.
    a: (M, ...) -> f: (Q, ...)."""
    Hq = model.hermite_matrix()
    fact = np.array([alpha_factorial(al) for al in multi_indices(model.N)], dtype=float)
    R = (model.vs.w[:, None] * Hq.T) / fact[None, :]
    return np.tensordot(R, a, axes=(1, 0))


def project(g, model: Model):
    """eq:an:  a_alpha = sum_i g_i He_alpha(c_i).  g: (Q, ...) -> (M, ...)."""
    return np.tensordot(model.hermite_matrix(), g, axes=(1, 0))


def equilibrium_f(rho, u_lab, theta, model: Model):
    """Truncated discrete Maxwellian of (rho, u_lab, theta) in the frame moving with ubar."""
    u_rel = np.asarray(u_lab) - model.ubar.reshape((3,) + (1,) * (np.ndim(rho)))
    a = equilibrium_moments(np.asarray(rho), u_rel, np.asarray(theta), model.N)
    return reconstruct(a, model)


def _ghost_widths(model: Model):
    s = model.streaming_offsets()[:, 0]
    return max(0, int(s.max())), max(0, int(-s.min()))


def stream(fstar, model: Model, dom: Domain):
    """Pull streaming g_i(x) = f*_i(x - s_i), s_i = e_i + k.  fstar: (Q, nz, ny, nx).
    Periodic in y and z, and in x unless the domain is a shock tube, whose
    ghost cells hold the truncated Maxwellians of the end states."""
    Q = model.vs.Q
    s = model.streaming_offsets()
    if dom.bc_x == 1:
        gl, gr = _ghost_widths(model)
        rin, uin, tin = dom.state_in
        rout, uout, tout = dom.state_out
        fin = equilibrium_f(np.array(rin), np.array(uin, dtype=float), np.array(tin), model)
        fout = equilibrium_f(np.array(rout), np.array(uout, dtype=float), np.array(tout), model)
        ext = np.zeros(fstar.shape[:3] + (gl + dom.nx + gr,), dtype=np.result_type(fstar, fin))
        ext[..., gl:gl + dom.nx] = fstar
        ext[..., :gl] = fin[:, None, None, None]
        ext[..., gl + dom.nx:] = fout[:, None, None, None]
    g = np.empty(fstar.shape, dtype=np.result_type(fstar, float) if dom.bc_x == 0 else ext.dtype)
    for q in range(Q):
        sx, sy, sz = (int(v) for v in s[q])
        plane = fstar[q] if dom.bc_x == 0 else ext[q]
        plane = np.roll(plane, shift=(sz, sy), axis=(0, 1))
        if dom.bc_x == 0:
            g[q] = np.roll(plane, shift=sx, axis=2)
        else:
            g[q] = plane[..., gl - sx: gl - sx + dom.nx]
    return g


def _conserved(g, model: Model):
    """rho, u' (relative to ubar) and theta of the pre-collision populations."""
    c = model.vs.c
    rho = g.sum(axis=0)
    j = np.tensordot(c.T, g, axes=(1, 0))
    E = np.tensordot((c ** 2).sum(axis=1), g, axes=(0, 0))
    u = j / rho
    theta = (E - rho * (u ** 2).sum(axis=0)) / (3.0 * rho)
    return rho, u, theta


def _check_state(rho, theta):
    r = np.real(rho)
    t = np.real(theta)
    if not (np.all(np.isfinite(r)) and np.all(np.isfinite(t))):
        raise StateError("non-finite density or temperature")
    if np.any(r <= 0.0) or np.any(t <= 0.0) or np.any(t >= 2.0):
        raise StateError("node outside rho > 0, 0 < theta < 2")


def _local_moments(g, model: Model, u, theta):
    """d_beta = sum_i g_i He_beta((c_i - u')/sqrt(theta)), |beta| <= N (direct)."""
    vs, N = model.vs, model.N
    Q1 = vs.Q1
    sq = np.sqrt(theta)
    # v[k, j, node] = (c1_j - u'_k) / sqrt(theta)
    v = (vs.c1[None, :, None] - u[:, None, :]) / sq[None, None, :]
    H = hermite_1d(N, v)                       # (3, Q1, nodes, N+1)
    G = g.reshape(Q1, Q1, Q1, -1)              # (ix, iy, iz, node)
    full = np.einsum('xyzn,xna,ynb,znc->abcn', G, H[0], H[1], H[2], optimize=True)
    return np.stack([full[a, b, c] for (a, b, c) in multi_indices(N)])


def _omega(model: Model, rho):
    """1/tau_bar_nm at every node; tau may be real or complex (complex-step)."""
    out = {}
    scale = model.rho_ref / rho if model.tau_density_scaling else 1.0
    for (n, m), t in model.tau.items():
        t = complex(t) if isinstance(t, complex) else float(t)
        tbar = t * scale + (0.5 if model.tau_offset_half else 0.0)
        out[(n, m)] = 1.0 / tbar
    return out


def _relax(d, model: Model, rho):
    """eq:SMRT: d'^(n,m) = d^(n,m) - d^(n,m)/tau_bar_nm for n >= 2; n = 0, 1 unchanged."""
    N = model.N
    sl = _order_slices(N)
    om = _omega(model, rho)
    dp = d.astype(np.result_type(d, *om.values()))
    for n in range(2, N + 1):
        dn = d[sl[n]]
        new = dn.copy()
        for m, P in enumerate(projector_matrices(n)):
            new = new - om[(n, m)] * np.tensordot(P, dn, axes=(1, 0))
        dp[sl[n]] = new
    return dp


def _back_to_lattice(dp, model: Model, u, theta):
    """a'_alpha = int omega(v) [sum_beta d'_beta He_beta(v)/beta!] He_alpha(u' + sqrt(theta) v) dv,
    by the tensor Gauss-Hermite rule with N+2 nodes per axis (exact here)."""
    N = model.N
    x, wgh = _herme.hermegauss(N + 2)
    wgh = wgh / math.sqrt(2.0 * math.pi)
    Hv = hermite_1d(N, x)                              # (G, N+1)
    alphas = multi_indices(N)
    fact = np.array([alpha_factorial(al) for al in alphas], dtype=float)
    coef = dp / fact.reshape((-1,) + (1,) * (dp.ndim - 1))
    # F(v_g) on the 3D GH grid, per node
    Cfull = np.zeros((N + 1,) * 3 + dp.shape[1:], dtype=dp.dtype)
    for k, (a, b, c) in enumerate(alphas):
        Cfull[a, b, c] = coef[k]
    F = np.einsum('abcn,xa,yb,zc->xyzn', Cfull, Hv, Hv, Hv, optimize=True)
    sq = np.sqrt(theta)
    xi = u[:, None, :] + sq[None, None, :] * x[None, :, None]    # (3, G, nodes)
    Hxi = hermite_1d(N, xi)                                     # (3, G, nodes, N+1)
    W = F * wgh[:, None, None, None] * wgh[None, :, None, None] * wgh[None, None, :, None]
    full = np.einsum('xyzn,xna,ynb,znc->abcn', W, Hxi[0], Hxi[1], Hxi[2], optimize=True)
    return np.stack([full[a, b, c] for (a, b, c) in alphas])


def collide(g, model: Model):
    """SMRT collision of pre-collision populations g (Q, nodes) -> f* (Q, nodes)."""
    rho, u, theta = _conserved(g, model)
    _check_state(rho, theta)
    d = _local_moments(g, model, u, theta)
    dp = _relax(d, model, rho)
    ap = _back_to_lattice(dp, model, u, theta)
    if model.regularized:
        return reconstruct(ap, model)
    a = project(g, model)
    return g + reconstruct(ap - a, model)


def step(fstar, model: Model, dom: Domain):
    """One time step on the post-collision state f* (Q, nz, ny, nx): stream, then collide."""
    g = stream(fstar, model, dom)
    shp = g.shape
    out = collide(g.reshape(shp[0], -1), model)
    return out.reshape(shp)


def observables(fstar, model: Model, dom: Domain):
    """Macroscopic fields of the pre-collision populations (stream first), Sec. 4.3:
    rho, u (lab), theta, sigma = theta d^(2), q = theta^(3/2)/2 tr d^(3),
    m = d^(3,0)/D(3,0), R41 = d^(4,1)/D(4,1), R42 = d^(4,2)/D(4,2); d = local moments."""
    g = stream(fstar, model, dom)
    shp = g.shape
    g = g.reshape(shp[0], -1)
    rho, u, theta = _conserved(g, model)
    d = _local_moments(g, model, u, theta)
    sl = _order_slices(model.N)
    out = dict(rho=rho, u=u + model.ubar[:, None], theta=theta, d=d)
    out["sigma"] = theta[None, :] * d[sl[2]]
    out["q"] = 0.5 * theta[None, :] ** 1.5 * np.tensordot(trace_matrix(3), d[sl[3]], axes=(1, 0))
    out["m"] = np.tensordot(part_matrices(3)[0], d[sl[3]], axes=(1, 0)) / float(D_coef(3, 0))
    if model.N >= 4:
        out["R41"] = np.tensordot(part_matrices(4)[1], d[sl[4]], axes=(1, 0)) / float(D_coef(4, 1))
        out["R42"] = np.tensordot(part_matrices(4)[2], d[sl[4]], axes=(1, 0)) / float(D_coef(4, 2))
    return out


def shock_loss(fstar, model: Model, dom: Domain, target, scales):
    """L = sum_x sum_k s_k^2 (F_k(x) - F*_k(x))^2 over F = (rho, theta, q_x);
    target: dict of arrays, scales: (s_rho, s_theta, s_q)."""
    ob = observables(fstar, model, dom)
    F = (ob["rho"], ob["theta"], ob["q"][0])
    T = (target["rho"], target["theta"], target["q_x"])
    return sum(s ** 2 * ((f - t) ** 2).sum() for s, f, t in zip(scales, F, T))
