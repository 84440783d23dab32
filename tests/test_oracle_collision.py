"""Pins of the oracle's collision and step against invariants and closed forms
(eq:SMRT, eq:an, eq:fi, App. B) -- each built without the oracle's own route."""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as herme

import oracle as O


def _vs7():
    return O.make_velocity_set([1, 2, 3], 9)


def _vs9():
    return O.make_velocity_set([1, 2, 3, 5], 11)


def _model(vs, N, tau20=1.3, shift=(0, 0, 0), table=None, **kw):
    table = table or O.TAU_STAR_SMRT
    return O.Model(vs=vs, N=N, tau={k: float(v) * tau20 for k, v in table.items()}, shift=shift, **kw)


def _binom(n, k):
    return math.comb(n, k)


def _shift_local_to_absolute(d, u, theta, N):
    """Absolute coefficients of theta^{-3/2} omega(v) sum_beta d_beta He_beta(v)/beta!,
    v = (xi-u)/sqrt(theta), by the Hermite shift identity
    He_n(u + s y) = sum_k C(n,k) s^k He_k(y) A_{n-k}(u, s^2) with the App. B
    polynomials A_j(u, theta) = sum_k j! (theta-1)^k u^(j-2k) / (2^k k! (j-2k)!)."""
    alphas = O.multi_indices(N)
    pos = {a: i for i, a in enumerate(alphas)}
    A = [O.maxwellian_hermite_1d(N, u[k], theta) for k in range(3)]
    out = np.zeros(len(alphas))
    for i, al in enumerate(alphas):
        acc = 0.0
        for be in alphas:
            if all(be[k] <= al[k] for k in range(3)):
                c = 1.0
                for k in range(3):
                    c *= _binom(al[k], be[k]) * A[k][al[k] - be[k]]
                acc += c * theta ** (sum(be) / 2) * d[pos[be]]
        out[i] = acc
    return out


# ----------------------------------------------------------------------------- equilibrium

def test_appendix_b_maxwellian_coefficients_against_direct_integration():
    x, w = herme.hermegauss(60)
    w = w / math.sqrt(2 * math.pi)
    for u, th in [(0.0, 1.0), (0.7, 0.6), (-1.1, 1.4), (0.3, 0.25)]:
        # f(xi) = N(u, th); a_n = int f He_n = int omega(y) He_n(u + sqrt(th) y) dy
        Hn = O.hermite_1d(7, u + math.sqrt(th) * x)
        direct = (w[:, None] * Hn).sum(0)
        closed = O.maxwellian_hermite_1d(7, u, th)
        assert np.allclose(direct, closed, atol=1e-11)


@pytest.mark.parametrize("vsf,N", [(_vs7, 4), (_vs9, 5)])
def test_truncated_equilibrium_carries_the_maxwellian_moments(vsf, N):
    vs = vsf()
    model = _model(vs, N, shift=(1, 0, 0))
    rho, th = 1.3, 0.8
    u_lab = np.array([model.ubar[0] + 0.2, -0.3, 0.1])
    f = O.equilibrium_f(np.array(rho), u_lab, np.array(th), model)
    a = O.project(f, model)
    want = rho * _shift_local_to_absolute(np.eye(model.M)[0], u_lab - model.ubar, th, N)
    assert np.allclose(a, want, atol=1e-12)
    # conserved moments are those of the Maxwellian
    assert abs(f.sum() - rho) < 1e-13
    assert np.allclose(vs.c.T @ f / rho + model.ubar, u_lab, atol=1e-13)


# ----------------------------------------------------------------------------- collision

def _random_state(model, n_nodes, rng, amp=0.05):
    """Equilibria of random (rho, u, theta) times a random positive perturbation:
    not inside the M-dim Hermite space."""
    rho = 1 + 0.3 * rng.random(n_nodes)
    u = np.stack([model.ubar[k] + 0.3 * rng.standard_normal(n_nodes) for k in range(3)])
    th = 0.6 + 0.6 * rng.random(n_nodes)
    f = O.equilibrium_f(rho, u, th, model)
    return f * (1 + amp * rng.standard_normal(f.shape))


@pytest.mark.parametrize("vsf,N", [(_vs7, 4), (_vs9, 5)])
def test_collision_conserves_mass_momentum_energy(vsf, N):
    vs = vsf()
    model = _model(vs, N, tau20=0.9, shift=(1, 0, 0))
    g = _random_state(model, 16, np.random.default_rng(0))
    fs = O.collide(g, model)
    c = vs.c
    for wv in (np.ones(vs.Q), c[:, 0], c[:, 1], c[:, 2], (c ** 2).sum(1)):
        assert np.abs(wv @ fs - wv @ g).max() < 1e-13


@pytest.mark.parametrize("vsf,N", [(_vs7, 4), (_vs9, 5)])
def test_truncated_maxwellian_is_a_fixed_point(vsf, N):
    vs = vsf()
    model = _model(vs, N, tau20=2.0, shift=(1, 0, 0))
    rng = np.random.default_rng(1)
    rho = 1 + 0.3 * rng.random(8)
    u = np.stack([model.ubar[0] + 0.4 * rng.standard_normal(8), 0.2 * rng.standard_normal(8), 0 * rho])
    th = 0.5 + 0.8 * rng.random(8)
    f = O.equilibrium_f(rho, u, th, model)
    assert np.abs(O.collide(f, model) - f).max() < 1e-14 * 50


@pytest.mark.parametrize("N,n,m", [(4, 2, 0), (4, 3, 0), (4, 3, 1), (4, 4, 0), (4, 4, 1), (4, 4, 2),
                                   (5, 5, 0), (5, 5, 1), (5, 5, 2)])
def test_single_irreducible_mode_decays_by_one_minus_inverse_tau_bar(N, n, m):
    """A pure (n,m) perturbation of the local expansion relaxes by exactly
    (1 - 1/tau_bar_nm) in one collision (eq:SMRT), in a moving, non-unit-temperature frame."""
    vs = _vs7() if N == 4 else _vs9()
    model = _model(vs, N, tau20=1.7, shift=(0, 0, 0))
    rng = np.random.default_rng(100 * n + m)
    rho, th = 1.25, 0.85
    u = np.array([0.25, -0.15, 0.1])
    A = rng.standard_normal((3,) * n)
    A = sum(np.transpose(A, p) for p in __import__('itertools').permutations(range(n)))
    mode = O.components_of(O.irreducible_piece(A, m))
    mode = mode / np.abs(mode).max()
    eps = 1e-3
    alphas = O.multi_indices(N)
    sl = [i for i, a in enumerate(alphas) if sum(a) == n]
    d = np.zeros(model.M)
    d[0] = rho
    d[sl] = eps * mode
    g = O.reconstruct(_shift_local_to_absolute(d, u, th, N), model)[:, None]
    fs = O.collide(g, model)[:, 0]
    tbar = float(O.TAU_STAR_SMRT[(n, m)]) * 1.7 / rho + 0.5
    d_exp = d.copy()
    d_exp[sl] = (1 - 1 / tbar) * eps * mode
    want = _shift_local_to_absolute(d_exp, u, th, N)
    got = O.project(fs, model)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("vsf,N", [(_vs7, 4), (_vs9, 5)])
def test_equal_relaxation_times_reduce_to_bgk(vsf, N):
    """All tau equal: a' = (1 - omega) a + omega a_eq regardless of frame (Sec. 3)."""
    vs = vsf()
    model = _model(vs, N, tau20=1.4, shift=(1, 0, 0), table=O.tau_star_bgk())
    g = _random_state(model, 10, np.random.default_rng(5))
    rho = g.sum(0)
    u_rel = (vs.c.T @ g) / rho
    th = ((vs.c ** 2).sum(1) @ g - rho * (u_rel ** 2).sum(0)) / (3 * rho)
    a = O.project(g, model)
    aeq = O.equilibrium_moments(rho, u_rel, th, N)
    om = 1 / (1.4 / rho + 0.5)
    want = O.reconstruct((1 - om) * a + om * aeq, model)
    assert np.abs(O.collide(g, model) - want).max() < 1e-13


def _axis_permutation_of_populations(vs, perm):
    """Population index map for xi -> (xi[perm[0]], xi[perm[1]], xi[perm[2]])."""
    Q1 = vs.Q1
    idx = np.arange(vs.Q).reshape(Q1, Q1, Q1)
    return np.transpose(idx, perm).reshape(-1)


def test_collision_commutes_with_lattice_symmetries():
    vs = _vs7()
    model = _model(vs, 4, tau20=1.1)
    g = _random_state(model, 6, np.random.default_rng(7))
    fs = O.collide(g, model)
    for perm in [(1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        P = _axis_permutation_of_populations(vs, perm)
        assert np.abs(O.collide(g[P], model) - fs[P]).max() < 1e-14 * 100
    R = np.arange(vs.Q).reshape(vs.Q1, vs.Q1, vs.Q1)[::-1].reshape(-1)   # x -> -x
    assert np.abs(O.collide(g[R], model) - fs[R]).max() < 1e-14 * 100


def test_additive_and_rebuilt_forms_agree_inside_hermite_space():
    vs = _vs7()
    rng = np.random.default_rng(8)
    m1 = _model(vs, 4, tau20=1.2)
    m2 = _model(vs, 4, tau20=1.2, regularized=False)
    g = _random_state(m1, 5, rng)
    g_in = O.reconstruct(O.project(g, m1), m1)
    assert np.abs(O.collide(g_in, m1) - O.collide(g_in, m2)).max() < 1e-14 * 10
    assert np.abs(O.collide(g, m1) - O.collide(g, m2)).max() > 1e-6


def test_invalid_states_raise():
    vs = _vs7()
    model = _model(vs, 4)
    f = O.equilibrium_f(np.array([1.0]), np.zeros((3, 1)), np.array([2.2]), model)
    with pytest.raises(O.StateError):
        O.collide(f, model)
    with pytest.raises(O.StateError):
        O.collide(-O.equilibrium_f(np.array([1.0]), np.zeros((3, 1)), np.array([1.0]), model), model)
    bad = O.equilibrium_f(np.array([1.0]), np.zeros((3, 1)), np.array([1.0]), model)
    bad[3, 0] = np.nan
    with pytest.raises(O.StateError):
        O.collide(bad, model)


# ----------------------------------------------------------------------------- stream and shock

def test_stream_is_a_pull_by_e_plus_k_with_periodic_wrap():
    vs = _vs7()
    model = _model(vs, 4, shift=(1, 0, 0))
    dom = O.Domain(nx=9, ny=4, nz=3)
    rng = np.random.default_rng(9)
    f = rng.random((vs.Q, 3, 4, 9))
    g = O.stream(f, model, dom)
    s = model.streaming_offsets()
    for q in (0, 17, 200, vs.Q - 1):
        for (z, y, x) in [(0, 0, 0), (2, 3, 8), (1, 2, 4)]:
            assert g[q, z, y, x] == f[q, (z - s[q, 2]) % 3, (y - s[q, 1]) % 4, (x - s[q, 0]) % 9]


def _shock_setup(vs, N, Ma, nx, theta2=1.07):
    st = O.rankine_hugoniot(Ma, theta2=theta2)
    k = O.shift_integer(st["u_mid"], vs.r)
    tau20 = 2 * vs.r / math.sqrt(st["theta1"])
    model = _model(vs, N, tau20=tau20, shift=(k, 0, 0), rho_ref=1.0)
    dom = O.Domain(nx=nx, bc_x=1, state_in=(1.0, (st["u1"], 0, 0), st["theta1"]),
                   state_out=(st["rho2"], (st["u2"], 0, 0), st["theta2"]))
    x = np.arange(nx)
    phi = 0.5 * (1 + np.tanh((x - nx / 2) / 5))
    rho = 1 + (st["rho2"] - 1) * phi
    ux = st["u1"] + (st["u2"] - st["u1"]) * phi
    th = st["theta1"] + (st["theta2"] - st["theta1"]) * phi
    f = O.equilibrium_f(rho, np.stack([ux, 0 * ux, 0 * ux]), th, model).reshape(vs.Q, 1, 1, nx)
    return st, model, dom, f


def _interface_fluxes(f, model, dom, weight):
    """Discrete flux of sum_i weight_i f*_i through every interface x+1/2, ghosts included."""
    gl, gr = 8, 8
    fin = O.equilibrium_f(np.array(dom.state_in[0]), np.array(dom.state_in[1], float), np.array(dom.state_in[2]), model)
    fout = O.equilibrium_f(np.array(dom.state_out[0]), np.array(dom.state_out[1], float), np.array(dom.state_out[2]), model)
    ext = np.concatenate([np.repeat(fin[:, None], gl, 1), f[:, 0, 0, :], np.repeat(fout[:, None], gr, 1)], axis=1)
    s = model.streaming_offsets()[:, 0]
    out = []
    for xi in range(gl - 1, gl + dom.nx):          # interface between ext cells xi and xi+1
        tot = 0.0
        for q in range(model.vs.Q):
            if s[q] > 0:
                tot += weight[q] * ext[q, xi - s[q] + 1: xi + 1].sum()
            elif s[q] < 0:
                tot -= weight[q] * ext[q, xi + 1: xi + 1 - s[q]].sum()
        out.append(tot)
    return np.array(out)


@pytest.mark.slow
def test_steady_shock_has_constant_interface_fluxes_and_rankine_hugoniot_ends():
    vs = _vs7()
    st, model, dom, f = _shock_setup(vs, 4, 1.2, 24)
    for it in range(6000):
        f_new = O.step(f, model, dom)
        if it % 100 == 99 and np.abs(f_new - f).max() < 1e-13:
            f = f_new
            break
        f = f_new
    assert np.abs(O.step(f, model, dom) - f).max() < 1e-13
    xi_lab = vs.c + model.ubar[None, :]
    for wv in (np.ones(vs.Q), xi_lab[:, 0], 0.5 * (xi_lab ** 2).sum(1)):
        fl = _interface_fluxes(f, model, dom, wv)
        assert np.abs(fl - fl[0]).max() < 1e-10 * max(1.0, abs(fl[0]))
    # mass crossing an interface per step is rho u dt/dx = rho1 u1 / c_l up to the
    # discrete boundary layer at the ghost cells
    fl = _interface_fluxes(f, model, dom, np.ones(vs.Q))
    assert abs(fl[0] - st["rho1"] * st["u1"] / vs.r) < 5e-3 * fl[0]
    ob = O.observables(f, model, dom)
    # 24 cells hold only a few shock widths: the ends sit within a few percent of RH
    assert abs(ob["rho"][0] - 1.0) < 3e-2 and abs(ob["rho"][-1] - st["rho2"]) < 3e-2
    assert abs(ob["theta"][0] - st["theta1"]) < 3e-2 and abs(ob["theta"][-1] - st["theta2"]) < 3e-2


# ----------------------------------------------------------------------------- gradient

def test_complex_step_gradient_matches_central_differences():
    """dL/dtau_nm by complex-step through the oracle agrees with FD (h = 1e-4 relative)."""
    vs = _vs7()
    st, model, dom, f0 = _shock_setup(vs, 4, 1.2, 12)
    steps = 6
    target = O.observables(f0, model, dom)
    tgt = dict(rho=target["rho"] * 1.001, theta=target["theta"] * 0.999, q_x=target["q"][0] + 1e-3)
    scales = (1 / (st["rho2"] - 1), 1 / (st["theta2"] - st["theta1"]), 1 / st["theta1"] ** 1.5)

    def loss(tau):
        m = O.Model(vs=vs, N=4, tau=tau, shift=model.shift)
        f = f0
        for _ in range(steps):
            f = O.step(f, m, dom)
        return O.shock_loss(f, m, dom, tgt, scales)

    base = dict(model.tau)
    h = 1e-30
    for key in [(2, 0), (3, 0), (3, 1), (4, 0), (4, 1), (4, 2)]:
        tc = dict(base)
        tc[key] = complex(base[key], h)
        g_cs = loss(tc).imag / h
        tp, tm = dict(base), dict(base)
        tp[key] = base[key] * (1 + 1e-4)
        tm[key] = base[key] * (1 - 1e-4)
        g_fd = (loss(tp) - loss(tm)) / (2e-4 * base[key])
        assert abs(g_cs - g_fd) <= 1e-6 * max(abs(g_cs), 1e-12) + 1e-12, key
    tc = dict(base)
    tc[(2, 1)] = complex(base[(2, 1)], h)
    assert abs(loss(tc).imag / h) < 1e-10          # the (2,1) piece vanishes identically
