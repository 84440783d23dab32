"""Pins of the oracle's observables (Sec. 4.3 profiles) against their definitions.

The oracle computes sigma, q, m, R^(4,1), R^(4,2) from its local moments d (rho absorbed,
scaled velocity v = (xi - u)/sqrt(theta)).  Here the same quantities are rebuilt by routes
that share nothing with it:

* the tensorial velocity moments P = sum g c c, Q = sum g c c c, R = sum g c c c c of the
  peculiar velocity c = xi - u (Sec. 2.2, below eq:a), giving sigma = P - p delta (the
  (2,0) part, Sec. 2.2), q_i = Q_ikk / 2 (Sec. 2.2), and the rank-3 and rank-4 irreducible
  parts written out through P, Q, R;
* full 3^n Hermite tensors H^(n)(v) from the tensor recursion
  H^(n+1)_{i I} = v_i H^(n)_I - sum_{j in I} delta_{i j} H^(n-1)_{I \\ j}
  (not the oracle's products of 1D polynomials), contracted and made traceless by hand,
  with B(n,m), D(n,m) read from the Table 5 fixture (eq:bd).

Every state has theta far from 1 and a velocity away from the frame shift ubar (itself
nonzero), so a wrong power of theta, a dropped velocity shift or a wrong D(n,m) factor fails.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import oracle.lbsmrt_oracle as OM

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table5():
    out = {}
    with open(os.path.join(GOLD, "table5_bd.txt")) as fh:
        for ln in fh:
            if ln.strip() and not ln.startswith("#"):
                n, m, B, D = ln.split()
                out[(int(n), int(m))] = (float(Fraction(B)), float(Fraction(D)))
    return out


def _hermite_tensors(v, n_max):
    """Full Hermite tensors H^(0..n_max)(v) of one 3-vector v, by the tensor recursion."""
    eye = np.eye(3)
    H = [np.array(1.0), v.copy()]
    for n in range(1, n_max):
        nxt = np.multiply.outer(v, H[n])                    # v_i H^(n)_I, index i first
        for pos in range(n):                                # sum over j in I = (j_1..j_n)
            # delta_{i, j_pos} H^(n-1)_{I without j_pos}
            lower = H[n - 1]
            t = np.multiply.outer(eye, lower)               # axes (i, j_pos, rest...)
            order = [0] + list(range(2, 2 + pos)) + [1] + list(range(2 + pos, 1 + n))
            nxt = nxt - np.transpose(t, order)
        H.append(nxt)
    return H


def _comps(T):
    """Distinct components of a symmetric rank-n tensor: (a, b, c) with a+b+c = n, a then b
    descending, component T[0..0 1..1 2..2]."""
    n = T.ndim
    out = []
    for a in range(n, -1, -1):
        for b in range(n - a, -1, -1):
            out.append(T[(0,) * a + (1,) * b + (2,) * (n - a - b)])
    return np.array(out)


def _traceless3(T):
    """Traceless part of a symmetric rank-3 tensor: T - (delta t + perms)/5, t_k = T_kll."""
    t = np.einsum("kll->k", T)
    eye = np.eye(3)
    corr = (np.einsum("ij,k->ijk", eye, t) + np.einsum("ik,j->ijk", eye, t) + np.einsum("jk,i->ijk", eye, t))
    return T - corr / 5.0


def _dev(X):
    return X - np.trace(X) / 3.0 * np.eye(3)


def _random_state(model, rng, theta, du):
    """Positive non-equilibrium populations: |truncated Maxwellian of (1.3, ubar + du, theta)|,
    each population scaled by 1 + U(-0.35, 0.35)."""
    u_lab = model.ubar + np.asarray(du, dtype=float)
    f = np.abs(O.equilibrium_f(np.array(1.3), u_lab, np.array(theta), model))
    return f * (1.0 + rng.uniform(-0.35, 0.35, size=f.shape))


def _discrepancies(ob, g, model, tab):
    """Largest deviation of each oracle observable of one node from its direct definition."""
    vs = model.vs
    xi = vs.c + model.ubar[None, :]                  # lab-frame velocities
    rho = g.sum()
    u = (g[:, None] * xi).sum(axis=0) / rho
    c = xi - u
    th = (g * (c ** 2).sum(axis=1)).sum() / (3.0 * rho)
    P = np.einsum("i,ia,ib->ab", g, c, c)
    Qt = np.einsum("i,ia,ib,ic->abc", g, c, c, c)
    R = np.einsum("i,ia,ib,ic,id->abcd", g, c, c, c, c)
    p = np.trace(P) / 3.0
    assert abs(p - rho * th) < 1e-12 * p                 # p = rho theta
    # theta is far enough from 1 that a wrong power of it is seen: theta^(3/2) vs theta
    assert abs(th ** 1.5 - th) > 0.05 * th
    out = {"rho": abs(float(ob["rho"][0]) - rho) / rho,
           "u": float(np.abs(ob["u"][:, 0] - u).max()),
           "theta": abs(float(ob["theta"][0]) - th)}
    # sigma = P - p delta (the (2,0) part), q_i = Q_ikk / 2
    out["sigma"] = float(np.abs(ob["sigma"][:, 0] - _comps(P - p * np.eye(3))).max())
    out["q"] = float(np.abs(ob["q"][:, 0] - 0.5 * np.einsum("ikk->i", Qt)).max())
    # m = d^(3,0)/D(3,0): traceless part of Q / theta^(3/2), times B(3,0)/D(3,0)
    B30, D30 = tab[(3, 0)]
    out["m"] = float(np.abs(ob["m"][:, 0] - _comps(B30 / D30 * _traceless3(Qt) / th ** 1.5)).max())
    # the same through full Hermite tensors of v = c / sqrt(theta)
    v = c / np.sqrt(th)
    Hs = [_hermite_tensors(vi, 4) for vi in v]
    d3 = sum(gi * H[3] for gi, H in zip(g, Hs))
    d4 = sum(gi * H[4] for gi, H in zip(g, Hs))
    out["m_hermite"] = float(np.abs(ob["m"][:, 0] - _comps(B30 / D30 * _traceless3(d3))).max())
    # R^(4,1) = d^(4,1)/D(4,1) with d^(4,1) = B(4,1) dev(tr d^(4)); R^(4,2) = B(4,2) tr tr d^(4) / D(4,2)
    B41, D41 = tab[(4, 1)]
    B42, D42 = tab[(4, 2)]
    trd4 = np.einsum("ijkk->ij", d4)
    r41_h = B41 / D41 * _dev(trd4)
    r42_h = B42 / D42 * np.trace(trd4)
    # ... and through P and R: tr H^(4)(v) = v v (|v|^2 - 7) - delta (|v|^2 - 5), so
    # tr d^(4) = R_ijkk / theta^2 - 7 P_ij / theta + 2 rho delta, tr tr d^(4) = R_iijj / theta^2 - 15 rho
    Rkk = np.einsum("ijkk->ij", R)
    r41_m = B41 / D41 * _dev(Rkk / th ** 2 - 7.0 * P / th)
    r42_m = B42 / D42 * (np.trace(Rkk) / th ** 2 - 15.0 * rho)
    assert float(np.abs(r41_h - r41_m).max()) < 1e-10 and abs(r42_h - r42_m) < 1e-10 * max(1.0, abs(r42_m))
    out["R41"] = float(np.abs(ob["R41"][:, 0] - _comps(r41_m)).max())
    out["R42"] = abs(float(ob["R42"][0, 0]) - r42_m) / max(1.0, abs(r42_m))
    return out


TOL = {"rho": 1e-13, "u": 1e-13, "theta": 1e-13, "sigma": 1e-12, "q": 1e-12, "m": 1e-11, "m_hermite": 1e-11,
       "R41": 1e-10, "R42": 1e-10}


def _lattice(stencil, N, shift):
    vs = O.make_velocity_set(*stencil)
    return O.Model(vs=vs, N=N, tau={k: 1.0 for k in O.TAU_STAR_SMRT if k[0] <= N}, shift=shift)


@pytest.mark.parametrize("stencil,N,shift", [(([1, 2, 3], 9), 4, (1, 0, 0)),
                                              (([1, 2, 3, 5], 11), 5, (2, 0, 1))])
@pytest.mark.parametrize("theta,du", [(0.55, (0.35, -0.3, 0.2)), (1.45, (-0.4, 0.25, -0.3))])
def test_observables_match_direct_velocity_moments(stencil, N, shift, theta, du):
    tab = _table5()
    model = _lattice(stencil, N, shift)
    dom = O.Domain(nx=1, ny=1, nz=1, bc_x=0)             # one node: streaming is the identity
    rng = np.random.default_rng(11)
    for _ in range(3):
        f = _random_state(model, rng, theta, du)
        ob = O.observables(f.reshape(model.vs.Q, 1, 1, 1), model, dom)
        err = _discrepancies(ob, f.reshape(model.vs.Q), model, tab)
        for key, e in err.items():
            assert e < TOL[key], (key, e)


def _perturbed_D(n0, m0):
    orig = OM.D_coef

    def D(n, m):
        v = orig(n, m)
        return v * Fraction(101, 100) if (n, m) == (n0, m0) else v
    return D


@pytest.mark.parametrize("mutation,field", [("D30", "m"), ("D41", "R41"), ("D42", "R42"), ("theta", "sigma"),
                                            ("theta", "R42"), ("u", "q"), ("u", "m")])
def test_observables_pin_catches_planted_mistakes(monkeypatch, mutation, field):
    """Plant a mistake in the oracle (a D(n,m) factor off by 1 %, theta off by 1e-3 or u' off by
    1e-3 in the conserved moments) and check that the comparison above flags the affected field.
    (q = Q_ikk / 2 does not depend on theta: its theta powers cancel exactly.)"""
    tab = _table5()
    model = _lattice(([1, 2, 3], 9), 4, (1, 0, 0))
    dom = O.Domain(nx=1, ny=1, nz=1, bc_x=0)
    f = _random_state(model, np.random.default_rng(5), 0.55, (0.35, -0.3, 0.2))
    if mutation.startswith("D"):
        monkeypatch.setattr(OM, "D_coef", _perturbed_D(int(mutation[1]), int(mutation[2])))
    else:
        orig = OM._conserved

        def conserved(g, model):
            rho, u, theta = orig(g, model)
            if mutation == "theta":
                return rho, u, theta * (1.0 + 1e-3)
            return rho, u + 1e-3, theta
        monkeypatch.setattr(OM, "_conserved", conserved)
    ob = O.observables(f.reshape(model.vs.Q, 1, 1, 1), model, dom)
    err = _discrepancies(ob, f.reshape(model.vs.Q), model, tab)
    assert err[field] > 100 * TOL[field], (field, err[field])


def test_hermite_tensor_recursion_matches_explicit_rank4():
    """The test's own H^(4) against its explicit form v v v v - 6 sym(v v delta) + 3 sym(delta delta)."""
    rng = np.random.default_rng(3)
    v = rng.normal(size=3)
    H4 = _hermite_tensors(v, 4)[4]
    eye = np.eye(3)
    exp = np.einsum("i,j,k,l->ijkl", v, v, v, v)
    for (a, b, c, d) in [(0, 1, 2, 3), (0, 2, 1, 3), (0, 3, 1, 2), (1, 2, 0, 3), (1, 3, 0, 2), (2, 3, 0, 1)]:
        exp = exp - np.transpose(np.einsum("p,q,rs->pqrs", v, v, eye), np.argsort([a, b, c, d]))
    exp = exp + np.einsum("ij,kl->ijkl", eye, eye) + np.einsum("ik,jl->ijkl", eye, eye) + \
        np.einsum("il,jk->ijkl", eye, eye)
    np.testing.assert_allclose(H4, exp, atol=1e-12)
    # orthogonality in the Gaussian measure: <H^(4)_{xxxx}> = 0, <H^(4)_{xxxx}^2> = 4!
    xg, wg = np.polynomial.hermite_e.hermegauss(12)
    wg = wg / np.sqrt(2 * np.pi)
    vals = [_hermite_tensors(np.array([x, 0.3, -0.2]), 4)[4][0, 0, 0, 0] for x in xg]
    assert abs(np.dot(wg, vals)) < 1e-12
    assert abs(np.dot(wg, np.square(vals)) - 24.0) < 1e-10
