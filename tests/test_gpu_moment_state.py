"""Moment-state form of the periodic step (lbsmrt_step_moment_state) through the C ABI.

The regularised rebuild makes a post-collision state a function of its M moments, so the
moment-state step must agree with the population step on the expanded state (both FP32
state, different rounding points), and with the FP64 oracle.  Boxes with ragged sizes (not
multiples of the 256-wide rows or of the line chunks of the z and y passes), all four compiled
(stencil, N) pairs and a non-zero frame shift; one step at 256^3 over every node."""
import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

from cases import D1Q7, D1Q9, box_case

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_PROFILE = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _fields(shape, shift, r, seed):
    """Seeded random perturbation of a Maxwellian around u = r k (lab frame)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    f = np.empty((5, n))
    f[0] = 1.0 + 0.03 * rng.uniform(-1, 1, n)
    for k in range(3):
        f[1 + k] = r * shift[k] + 0.05 * rng.uniform(-1, 1, n)
    f[4] = 1.0 + 0.03 * rng.uniform(-1, 1, n)
    return f


def _lattice(stencil, N, shape, shift=(0, 0, 0), precision="fp64_contract", n_ref=32):
    from paper_2401_11086_amd import Lattice
    ab, deg = stencil
    vs = O.make_velocity_set(ab, deg)
    tau20 = 0.05 * n_ref * vs.r
    tau = {key: float(v) * tau20 for key, v in O.TAU_STAR_SMRT.items() if key[0] <= N}
    nx, ny, nz = shape
    lat = Lattice(ab, deg, N, tau, [dict(nx=nx, ny=ny, nz=nz, bc_x=0)], shift_k=shift, precision=precision)
    return lat, vs, tau


def _noisy_moments(torch, lat, fields, seed, amp=0.02):
    """Equilibrium moments with multiplicative noise on every moment of order >= 2."""
    m = lat.equilibrium_moments(torch.tensor(fields, dtype=torch.float64, device="cuda"))
    n = lat.n_nodes
    noise = torch.tensor(W.state_noise((lat.M - 4, n), seed=seed, amp=amp), dtype=torch.float32, device="cuda")
    m[4:, :n] *= noise
    return m


CASES = [
    ("q343_n4_20x12x30", D1Q7, 4, (20, 12, 30), (0, 0, 0)),
    ("q343_n3_9x8x7", D1Q7, 3, (9, 8, 7), (0, 0, 0)),
    ("q343_n4_shift_16x11x13", D1Q7, 4, (16, 11, 13), (1, 0, -1)),
    ("q729_n4_13x11x12", D1Q9, 4, (13, 11, 12), (0, 0, 0)),
    ("q729_n5_12x10x46", D1Q9, 5, (12, 10, 46), (0, 0, 0)),
    ("q343_n4_300x3x2", D1Q7, 4, (300, 3, 2), (0, 0, 0)),
    # rows of whole 64-lane waves: pass x takes its taps from the wave's own row values
    ("q343_n4_row_64x6x5", D1Q7, 4, (64, 6, 5), (0, 0, 0)),
    ("q343_n3_row_128x3x2", D1Q7, 3, (128, 3, 2), (0, 0, 0)),
    ("q729_n4_row_64x5x4", D1Q9, 4, (64, 5, 4), (0, 0, 0)),
    ("q729_n5_row_192x3x3", D1Q9, 5, (192, 3, 3), (0, 0, 0)),
    ("q343_n4_shift_64x5x4", D1Q7, 4, (64, 5, 4), (1, 0, 0)),
]


@pytest.mark.parametrize("name,stencil,N,shape,shift", CASES, ids=[c[0] for c in CASES])
def test_moment_state_matches_population_step(torch, name, stencil, N, shape, shift):
    lat, vs, _ = _lattice(stencil, N, shape, shift)
    n = lat.n_nodes
    m0 = _noisy_moments(torch, lat, _fields(shape, shift, vs.r, seed=3), seed=4)
    f0 = lat.expand_state(m0)
    fb = lat.new_state()
    steps = 3
    f_pop = lat.step(f0.clone(), fb, steps)
    mb, work = lat.new_moment_state(), lat.new_moment_work()
    m_out = lat.step_moment_state(m0, mb, work, steps)
    lat.sync()
    f_mom = lat.expand_state(m_out)
    torch.cuda.synchronize()
    a = f_mom[:, :n].double()
    b = f_pop[:, :n].double()
    err = float((a - b).abs().max() / b.abs().max())
    print(f"{name}: {steps} steps, moment state vs population state {err:.2e}")
    assert err < TOL_STEP, err


@pytest.mark.parametrize("stencil,N", [(D1Q7, 4), (D1Q9, 5)], ids=["q343_n4", "q729_n5"])
def test_moment_state_row_box_one_step_matches_oracle(torch, stencil, N):
    """A 64 x 4 x 3 box (whole 64-lane rows, the cross-lane form of pass x), one step from a noisy
    moment state, against the oracle's step of the expanded populations."""
    shape = (64, 4, 3)
    lat, vs, tau = _lattice(stencil, N, shape)
    n = lat.n_nodes
    m0 = _noisy_moments(torch, lat, _fields(shape, (0, 0, 0), vs.r, seed=11), seed=12)
    f0 = lat.expand_state(m0)
    m1 = lat.step_moment_state(m0, lat.new_moment_state(), lat.new_moment_work(), 1)
    lat.sync()
    g = lat.expand_state(m1)[:, :n].double().cpu().numpy()
    fo0 = f0[:, :n].double().cpu().numpy().reshape(-1, 3, 4, 64)
    model = O.Model(vs=vs, N=N, tau=tau, shift=(0, 0, 0))
    fo1 = O.step(fo0, model, O.Domain(nx=64, ny=4, nz=3, bc_x=0)).reshape(g.shape)
    err = float(np.abs(g - fo1).max() / np.abs(fo1).max())
    print(f"64x4x3 box, one moment-state step vs FP64 oracle: {err:.2e}")
    assert err < TOL_STEP, err


@pytest.mark.parametrize("stencil,N", [(D1Q7, 4), (D1Q9, 5)], ids=["q343_n4", "q729_n5"])
def test_moment_state_one_step_matches_oracle(torch, stencil, N):
    case = box_case(8, stencil, N, n_ref=32)
    lat, vs, _ = _lattice(stencil, N, (8, 8, 8))
    n = lat.n_nodes
    fields = W.fourier_box(8, seed=0)
    m0 = _noisy_moments(torch, lat, fields, seed=5)
    f0 = lat.expand_state(m0)
    mb, work = lat.new_moment_state(), lat.new_moment_work()
    m1 = lat.step_moment_state(m0, mb, work, 1)
    lat.sync()
    g = lat.expand_state(m1)[:, :n].double().cpu().numpy()
    fo0 = f0[:, :n].double().cpu().numpy().reshape(-1, 8, 8, 8)
    fo1 = O.step(fo0, case["model"], case["dom"]).reshape(g.shape)
    err = float(np.abs(g - fo1).max() / np.abs(fo1).max())
    print(f"one moment-state step vs FP64 oracle: {err:.2e}")
    assert err < TOL_STEP, err


def test_project_expand_round_trip(torch):
    lat, vs, _ = _lattice(D1Q7, 4, (10, 9, 8))
    n = lat.n_nodes
    m = _noisy_moments(torch, lat, _fields((10, 9, 8), (0, 0, 0), vs.r, seed=6), seed=7)
    f = lat.expand_state(m)
    m2 = lat.project_state(f)
    torch.cuda.synchronize()
    err = float((m2[:, :n] - m[:, :n]).abs().max() / m[:, :n].abs().max())
    assert err < 1e-6, err
    # the equilibrium moments are the projection of the population equilibrium
    fields = torch.tensor(_fields((10, 9, 8), (0, 0, 0), vs.r, seed=8), dtype=torch.float64, device="cuda")
    me = lat.equilibrium_moments(fields)
    mp = lat.project_state(lat.equilibrium(fields))
    torch.cuda.synchronize()
    err = float((me[:, :n] - mp[:, :n]).abs().max() / me[:, :n].abs().max())
    assert err < 1e-6, err


def test_box32_200_steps_moment_state_tracks_population_state(torch):
    """Fourier box of the 256^3 workload's recipe at 32^3, 200 steps: the two state forms stay
    within 1e-4 of each other on every moment (both FP32 states)."""
    from paper_2401_11086_amd import _lib as C
    lat, _, _ = _lattice(D1Q7, 4, (32, 32, 32), n_ref=32)
    n = lat.n_nodes
    fields = torch.tensor(W.fourier_box(32, seed=0), dtype=torch.float64, device="cuda")
    fa = lat.equilibrium(fields)
    ma = lat.project_state(fa)
    fb, mb, work = lat.new_state(), lat.new_moment_state(), lat.new_moment_work()
    f = lat.step(fa, fb, 200)
    m = lat.step_moment_state(ma, mb, work, 200)
    lat.sync()
    fm = lat.expand_state(m)
    a = lat.moments(f, C.MOM_ALAB)[:, :n]
    b = lat.moments(fm, C.MOM_ALAB)[:, :n]
    err = float((a - b).abs().max() / a.abs().max())
    print(f"200 steps: moment-state vs population-state lattice moments {err:.2e}")
    assert err < TOL_PROFILE, err


def test_moment_state_rejects_unsupported_contexts(torch):
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = C.solve_quadrature([1, 2, 3], 9)
    dom, _, _ = shock_domain(1.2, 40, c_l)
    dom["ny"] = 2                         # a shock tube two nodes wide: neither a line nor a box
    tau = {(2, 0): 1.0, (3, 0): 1.0, (3, 1): 1.0, (4, 0): 1.0, (4, 1): 1.0, (4, 2): 1.0}
    shock = Lattice([1, 2, 3], 9, 4, tau, [dom], shift_k=(1, 0, 0))
    m, mb, w = shock.new_moment_state(), shock.new_moment_state(), shock.new_moment_work()
    with pytest.raises(C.LbsmrtError) as e:
        shock.step_moment_state(m, mb, w, 1)
    assert e.value.status == C.E_UNSUPPORTED
    two = Lattice([1, 2, 3], 9, 4, tau, [dict(nx=8, ny=8, nz=8), dict(nx=4, ny=4, nz=4)])
    m, mb, w = two.new_moment_state(), two.new_moment_state(), two.new_moment_work()
    with pytest.raises(C.LbsmrtError) as e:
        two.step_moment_state(m, mb, w, 1)
    assert e.value.status == C.E_UNSUPPORTED
    box = Lattice([1, 2, 3], 9, 4, tau, [dict(nx=8, ny=8, nz=8)])
    m, w = box.new_moment_state(), box.new_moment_work()
    with pytest.raises(C.LbsmrtError) as e:
        box.step_moment_state(m, m, w, 1)            # m_a == m_b
    assert e.value.status == C.E_ARG
    with pytest.raises(C.LbsmrtError) as e:
        box.step_moment_state(m, w[: box.moment_state_len()[0]].view(box.M, -1), w, 1)   # m_b inside work
    assert e.value.status == C.E_ARG


def test_full_size_box_one_step_matches_population_step(torch):
    """256^3 D3Q343 box (the throughput workload), one step from the same state: every node against
    the population step, and 256 sampled nodes against the oracle's collision of the populations
    they pull (the moments of the expanded state carry the multiplicative noise of the other tests)."""
    from cases import gather_columns, pull_indices
    lat, vs, tau = _lattice(D1Q7, 4, (256, 256, 256), n_ref=256)
    n = lat.n_nodes
    fields = W.fourier_box_torch(256, "cuda", seed=0)
    ma = lat.equilibrium_moments(fields)
    del fields
    g = torch.Generator(device="cuda").manual_seed(9)
    ma[4:, :n] *= 1.0 + 0.02 * torch.randn((lat.M - 4, n), device="cuda", generator=g)
    fa = lat.expand_state(ma)
    fb = lat.new_state()
    lat.step(fa, fb, 1)
    mb, work = lat.new_moment_state(), lat.new_moment_work()
    lat.step_moment_state(ma, mb, work, 1)
    lat.sync()
    del work
    model = O.Model(vs=vs, N=4, tau=tau)
    nodes = np.random.default_rng(10).integers(0, n, size=256)
    ref = O.collide(gather_columns(torch, fa, pull_indices(model, (256, 256, 256), nodes)), model)
    lat.expand_state(mb, out=fa)
    torch.cuda.synchronize()
    got = fa[:, torch.tensor(nodes, device="cuda")].double().cpu().numpy()
    err_o = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"256^3 one moment-state step, 256 sampled nodes vs FP64 oracle: {err_o:.2e}")
    assert err_o < TOL_STEP, err_o
    torch.cuda.synchronize()
    worst, scale = 0.0, 0.0
    for q0 in range(0, lat.Q, 49):
        a = fa[q0:q0 + 49, :n]
        b = fb[q0:q0 + 49, :n]
        worst = max(worst, float((a - b).abs().max()))
        scale = max(scale, float(b.abs().max()))
    err = worst / scale
    print(f"256^3 one step: moment state vs population state {err:.2e}")
    assert err < TOL_STEP, err


# ---- line domains (ny = nz = 1): the x-stage alone, end states as ghosts ---------------------

def _line_lattice(domains, stencil, N, shift):
    from paper_2401_11086_amd import Lattice
    ab, deg = stencil
    vs = O.make_velocity_set(ab, deg)
    tau20 = 2.0 * vs.r / 0.6
    tau = {key: float(v) * tau20 for key, v in O.TAU_STAR_SMRT.items() if key[0] <= N}
    return Lattice(ab, deg, N, tau, domains, shift_k=shift, precision="fp64_contract")


def _shock_domains(machs_lengths, stencil):
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = C.solve_quadrature(*stencil)
    doms, fields, ks = [], [], []
    for Ma, nx in machs_lengths:
        d, fl, st = shock_domain(Ma, nx, c_l)
        doms.append(d)
        fields.append(fl)
        ks.append(int(st["k"]))
    return doms, np.concatenate(fields, axis=1), ks


LINE_CASES = [
    ("shock_q343_n4_ma1.2", D1Q7, 4, [(1.2, 200)]),
    ("shock_q729_n5_ma3", D1Q9, 5, [(3.0, 120)]),
    ("batch3_q729_n5", D1Q9, 5, [(1.5, 90), (3.0, 130), (2.2, 70)]),
    ("ring_q343_n4", D1Q7, 4, None),
]


def _line_case(stencil, N, spec):
    if spec is None:                                  # periodic ring of 50 nodes
        doms = [dict(nx=50, ny=1, nz=1, bc_x=0)]
        lat = _line_lattice(doms, stencil, N, (0, 0, 0))
        return lat, _fields((50, 1, 1), (0, 0, 0), lat.c_l, seed=31)
    doms, fields, ks = _shock_domains(spec, stencil)
    assert len(set(ks)) == 1
    return _line_lattice(doms, stencil, N, (ks[0], 0, 0)), fields


@pytest.mark.parametrize("name,stencil,N,spec", LINE_CASES, ids=[c[0] for c in LINE_CASES])
def test_line_moment_state_matches_population_step(torch, name, stencil, N, spec):
    lat, fields = _line_case(stencil, N, spec)
    n = lat.n_nodes
    assert lat.moment_state_len()[1] == 0           # line domains need no scratch
    m0 = _noisy_moments(torch, lat, fields, seed=32)
    f0 = lat.expand_state(m0)
    steps = 5
    f_pop = lat.step(f0.clone(), lat.new_state(), steps)
    m_out = lat.step_moment_state(m0, lat.new_moment_state(), lat.new_moment_work(), steps)
    lat.sync()
    f_mom = lat.expand_state(m_out)
    torch.cuda.synchronize()
    a, b = f_mom[:, :n].double(), f_pop[:, :n].double()
    err = float((a - b).abs().max() / b.abs().max())
    print(f"{name}: {steps} steps, line moment state vs population state {err:.2e}")
    assert err < TOL_STEP, err


def test_line_moment_state_one_step_matches_oracle(torch):
    from cases import oracle_state_from_gpu, shock_case
    case = shock_case(3.0, 64, D1Q9, 5)
    from paper_2401_11086_amd import Lattice
    lat = Lattice(precision="fp64_contract", **case["lat_kw"])
    m0 = _noisy_moments(torch, lat, case["fields"], seed=33)
    f0 = lat.expand_state(m0)
    m1 = lat.step_moment_state(m0, lat.new_moment_state(), lat.new_moment_work(), 1)
    lat.sync()
    g = lat.expand_state(m1)[:, :64].double().cpu().numpy()
    fo1 = O.step(oracle_state_from_gpu(f0.cpu().numpy(), case), case["model"], case["dom"])
    err = float(np.abs(g - fo1.reshape(g.shape)).max() / np.abs(fo1).max())
    print(f"Ma 3 shock, one line moment-state step vs FP64 oracle: {err:.2e}")
    assert err < TOL_STEP, err


def test_line_batch_equals_separate_contexts(torch):
    spec = [(1.5, 90), (3.0, 130), (2.2, 70)]
    lat, fields = _line_case(D1Q9, 5, spec)
    m0 = _noisy_moments(torch, lat, fields, seed=34)
    mb = lat.step_moment_state(m0.clone(), lat.new_moment_state(), lat.new_moment_work(), 7)
    lat.sync()
    off = 0
    for i, (Ma, nx) in enumerate(spec):
        one, fl = _line_case(D1Q9, 5, [(Ma, nx)])
        m1 = one.new_moment_state()
        m1[:, :nx] = m0[:, off:off + nx]
        out = one.step_moment_state(m1, one.new_moment_state(), one.new_moment_work(), 7)
        one.sync()
        assert torch.equal(out[:, :nx], mb[:, off:off + nx]), i
        off += nx


@pytest.mark.parametrize("stencil,N", [(D1Q7, 4), (D1Q9, 5)], ids=["q343_n4", "q729_n5"])
def test_line_lanes_per_node_agree(torch, stencil, N):
    """Eight lanes per node (one tap pair each, DPP group sums in FP64) against one lane per
    node (x-stage moments rounded to float32 before the collision): the same step up to that
    rounding and the order of the FP64 sums."""
    lat, fields = _line_case(stencil, N, [(3.0, 150)])
    n = lat.n_nodes
    m0 = _noisy_moments(torch, lat, fields, seed=35)
    outs = {}
    for lanes in (1, 8):
        lat.set_launch("direct", 0, 64, lanes)
        outs[lanes] = lat.step_moment_state(m0.clone(), lat.new_moment_state(), lat.new_moment_work(), 4)
        lat.sync()
    a, b = outs[1][:, :n].double(), outs[8][:, :n].double()
    err = float((a - b).abs().max() / a.abs().max())
    print(f"line moment state, 8 lanes vs 1 lane per node after 4 steps: {err:.2e}")
    assert err < 2e-6, err


def test_box_moment_state_conserves_mass_momentum_energy(torch):
    """Periodic box in the moment-state form, 50 steps: total mass, momentum and energy (the
    conserved moments summed over the box) change only by the float32 rounding of the stored
    fields, as in the population form with FP64 contractions."""
    lat, vs, _ = _lattice(D1Q7, 4, (16, 16, 16), n_ref=64)
    n = lat.n_nodes
    fields = torch.tensor(W.fourier_box(16, seed=1), dtype=torch.float64, device="cuda")
    m0 = lat.equilibrium_moments(fields)

    def totals(m):
        # rows 0..3 hold a_0 and the three first moments; 4, 7 and 9 the diagonal second moments
        t = m[:, :n].double().sum(dim=1)
        return torch.stack([t[0], t[1], t[2], t[3], t[4] + t[7] + t[9]])

    t0 = totals(m0)
    m = lat.step_moment_state(m0.clone(), lat.new_moment_state(), lat.new_moment_work(), 50)
    lat.sync()
    drift = ((totals(m) - t0).abs() / n).cpu().numpy()
    print(f"moment-state box, per-node drift of mass, momentum, energy over 50 steps: {drift}")
    # tap tables rounded to float32 break the exact sum rule of the taps and drift mass by ~6e-6
    assert np.all(drift < 1e-7), drift


UNIFORM_STATE = (1.1, (0.04, -0.03, 0.02), 0.97)     # rho, u, theta
UNIFORM_CASES = [
    ("box_q343_n4", D1Q7, 4, (12, 10, 9), 1),
    ("box_q729_n5", D1Q9, 5, (11, 9, 13), 1),
    ("ring_q343_n4", D1Q7, 4, (50, 1, 1), 1),
    ("ring_q729_n5", D1Q9, 5, (50, 1, 1), 1),
    ("tube_q729_n5", D1Q9, 5, "tube", 1),              # end states equal to the state
    ("tube_q729_n5_8lanes", D1Q9, 5, "tube", 8),
]


@pytest.mark.parametrize("name,stencil,N,shape,lanes", UNIFORM_CASES, ids=[c[0] for c in UNIFORM_CASES])
def test_uniform_state_is_a_fixed_point(torch, name, stencil, N, shape, lanes):
    """A uniform equilibrium is a fixed point of the step: the taps of every axis sum to the
    identity (the quadrature is exact to degree 2N) and the collision leaves an equilibrium
    where it is, so 100 steps move no moment by more than a few float32 ulps (the stored state
    is the float32 rounding of the equilibrium, which the first steps relax).  Tap tables
    rounded to float32 break the identity and move such a state by ~1e-7 of its moments per
    step, 1e-5 over these steps."""
    rho, u, theta = UNIFORM_STATE
    if shape == "tube":
        dom = dict(nx=70, ny=1, nz=1, bc_x=1, rho_in=rho, u_in=u, theta_in=theta, rho_out=rho, u_out=u,
                   theta_out=theta, tau_scale=1.0)
        lat = _line_lattice([dom], stencil, N, (0, 0, 0))
    else:
        lat, _, _ = _lattice(stencil, N, shape)
    if lanes > 1:
        lat.set_launch("direct", 0, 64, lanes)
    n = lat.n_nodes
    f = np.empty((5, n))
    f[0], f[1], f[2], f[3], f[4] = rho, u[0], u[1], u[2], theta
    m0 = lat.equilibrium_moments(torch.tensor(f, dtype=torch.float64, device="cuda"))
    m = lat.step_moment_state(m0.clone(), lat.new_moment_state(), lat.new_moment_work(), 100)
    lat.sync()
    a, b = m0[:, :n].double(), m[:, :n].double()
    err = float((b - a).abs().max() / a.abs().max())
    spread = float((b - b[:, :1]).abs().max() / a.abs().max())
    print(f"{name}: uniform equilibrium after 100 steps moved by {err:.2e}, non-uniformity {spread:.2e}")
    assert err < 1e-6, err
    assert spread == 0.0, spread       # every node sees the same arithmetic


@pytest.mark.parametrize("kind", ["line_batch", "box"])
def test_graph_mode_replays_match_direct(torch, kind):
    """The moment-state step in graph mode (8 steps captured) against direct launches, bitwise:
    three calls of 10 steps (one replay plus two direct steps each), eager work and
    synchronisations between them, every call's result compared; then a relaxation-time change
    must recapture (the replayed graph would hold the old times)."""
    if kind == "line_batch":
        lat, fields = _line_case(D1Q9, 5, [(1.5, 90), (3.0, 130), (2.2, 70)])
    else:
        lat, _, _ = _lattice(D1Q7, 4, (64, 6, 5))
        fields = _fields((64, 6, 5), (0, 0, 0), lat.c_l, seed=41)
    n = lat.n_nodes
    m0 = _noisy_moments(torch, lat, fields, seed=42)
    work = lat.new_moment_work()
    outs = {}
    for mode in ("direct", "graph"):
        lat.set_launch(mode, 0, 8, 0)
        ma, mb = m0.clone(), lat.new_moment_state()
        res = []
        for call in range(3):
            cur = lat.step_moment_state(ma, mb, work, 10)
            lat.sync()
            assert cur is ma                          # an even step count returns to m_a
            res.append(ma[:, :n].clone())
            torch.cuda.synchronize()
            _ = (ma[:, :n] * 2.0).sum().item()       # eager work between the replays
        if mode == "graph":
            tau = {k: v * 1.1 for k, v in lat.tau.items()}
            lat.set_tau(tau)
            cur = lat.step_moment_state(ma, mb, work, 10)
            lat.sync()
            res.append(ma[:, :n].clone())
            lat.set_tau({k: v / 1.1 for k, v in tau.items()})
        outs[mode] = res
    lat.set_launch("direct", 0, 8, 0)
    for a, b in zip(outs["direct"], outs["graph"]):
        assert torch.equal(a, b)
    # direct launches with the changed times from the same state as the graph's fourth call
    ma, mb = outs["direct"][-1].clone(), lat.new_moment_state()
    full = torch.zeros_like(m0)
    full[:, :n] = ma
    tau = {k: v * 1.1 for k, v in lat.tau.items()}
    lat.set_tau(tau)
    lat.step_moment_state(full, mb, work, 10)
    lat.sync()
    assert torch.equal(full[:, :n], outs["graph"][-1])
