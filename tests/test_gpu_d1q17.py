"""D3Q4913 (tensor product of D1Q17 {0, +-1..+-7, +-9}, degree 19; Table 3's set for Ma 7)
through the C ABI against the FP64 oracle on the same seeded states: one step of a Ma 7 shock
tube (one and eight lanes per node) and of a small periodic box; the moment-state form on line
domains against the population step and the oracle; and the calls the library refuses for this
stencil."""
import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

from cases import box_case, oracle_state_from_gpu, shock_case

pytestmark = pytest.mark.gpu

D1Q17 = ([1, 2, 3, 4, 5, 6, 7, 9], 19)
TOL_STEP = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _lattice(case, **kw):
    from paper_2401_11086_amd import Lattice
    return Lattice(precision="fp64_contract", **case["lat_kw"], **kw)


def _noisy_state(torch, lat, case, seed):
    f = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    n = case["nx"] * case["ny"] * case["nz"]
    f[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=seed, amp=0.02), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    return f


def test_d1q17_lattice_constant_is_table3():
    vs = O.make_velocity_set(*D1Q17)
    assert abs(vs.r - 0.5638701) < 5e-8


@pytest.mark.parametrize("lanes", [1, 8, 16])
def test_d3q4913_ma7_shock_one_step_matches_oracle(torch, lanes):
    case = shock_case(7.0, 40, D1Q17, 5)
    lat = _lattice(case)
    assert lat.Q == 4913 and lat.shift_k[0] == 3
    lat.set_launch("direct", 0, 64, lanes)
    n = case["nx"]
    f0 = _noisy_state(torch, lat, case, seed=21)
    fo0 = oracle_state_from_gpu(f0.cpu().numpy(), case)
    f1 = lat.step(f0, lat.new_state(), 1)
    lat.sync()
    fo1 = O.step(fo0, case["model"], case["dom"])
    g = f1[:, :n].double().cpu().numpy().reshape(fo1.shape)
    err = float(np.abs(g - fo1).max() / np.abs(fo1).max())
    print(f"D3Q4913 Ma 7 shock, {lanes} lane(s) per node: one step vs oracle {err:.2e}")
    assert err < TOL_STEP, err
    from paper_2401_11086_amd import _lib as C
    m = lat.moments(f1, C.MOM_BASIC | C.MOM_Q)[:, :n].cpu().numpy()
    ob = O.observables(fo1, case["model"], case["dom"])
    assert np.abs(m[0] - ob["rho"]).max() < 1e-5 * np.abs(ob["rho"]).max()
    assert np.abs(m[4] - ob["theta"]).max() < 1e-5


def test_d3q4913_box_one_step_matches_oracle(torch):
    case = box_case(6, D1Q17, 5, n_ref=32)
    lat = _lattice(case)
    n = 6 ** 3
    f0 = _noisy_state(torch, lat, case, seed=22)
    fo0 = oracle_state_from_gpu(f0.cpu().numpy(), case)
    f1 = lat.step(f0, lat.new_state(), 1)
    lat.sync()
    fo1 = O.step(fo0, case["model"], case["dom"])
    g = f1[:, :n].double().cpu().numpy().reshape(fo1.shape)
    err = float(np.abs(g - fo1).max() / np.abs(fo1).max())
    print(f"D3Q4913 6^3 box: one step vs oracle {err:.2e}")
    assert err < TOL_STEP, err


def test_d1q17_refused_calls(torch):
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import _lib as C
    case = shock_case(7.0, 20, D1Q17, 5)
    for kw in (dict(precision="fp32"), dict(precision="fp64_contract", regularized=False)):
        with pytest.raises(C.LbsmrtError) as e:
            Lattice(**case["lat_kw"], **kw)
        assert e.value.status == C.E_UNSUPPORTED
    with pytest.raises(C.LbsmrtError) as e:
        Lattice(D1Q17[0], D1Q17[1], 4, case["lat_kw"]["tau"], case["lat_kw"]["domains"])
    assert e.value.status == C.E_UNSUPPORTED                  # N = 4 is not built for D1Q17
    lat = _lattice(case)
    with pytest.raises(C.LbsmrtError) as e:
        lat.set_launch("persistent")
    assert e.value.status == C.E_UNSUPPORTED
    f = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    with pytest.raises(C.LbsmrtError) as e:
        lat.step_adjoint(f, lat.new_state(), lat.new_state(), dtau)
    assert e.value.status == C.E_UNSUPPORTED
    box = _lattice(box_case(4, D1Q17, 5, n_ref=32))           # the moment state: line domains only
    mb = box.new_moment_state()
    with pytest.raises(C.LbsmrtError) as e:
        box.step_moment_state(mb, box.new_moment_state(), box.new_moment_work(), 1)
    assert e.value.status == C.E_UNSUPPORTED


# ---- moment-state form on line domains (the x-stage kernel, one lane per node) ---------------

def _noisy_moments(torch, lat, fields, seed, amp=0.02):
    """Equilibrium moments with multiplicative noise on every moment of order >= 2."""
    m = lat.equilibrium_moments(torch.tensor(fields, dtype=torch.float64, device="cuda"))
    n = lat.n_nodes
    m[4:, :n] *= torch.tensor(W.state_noise((lat.M - 4, n), seed=seed, amp=amp), dtype=torch.float32, device="cuda")
    return m


def _ma7_tubes(specs):
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = C.solve_quadrature(*D1Q17)
    doms, fields, ks = [], [], []
    for Ma, nx in specs:
        d, fl, st = shock_domain(Ma, nx, c_l)
        doms.append(d)
        fields.append(fl)
        ks.append(int(st["k"]))
    assert len(set(ks)) == 1
    vs = O.make_velocity_set(*D1Q17)
    tau20 = 2.0 * vs.r / 0.6
    tau = {key: float(v) * tau20 for key, v in O.TAU_STAR_SMRT.items() if key[0] <= 5}
    lat = Lattice(D1Q17[0], D1Q17[1], 5, tau, doms, shift_k=(ks[0], 0, 0), precision="fp64_contract")
    return lat, np.concatenate(fields, axis=1)


@pytest.mark.parametrize("specs", [[(7.0, 60)], [(7.0, 45), (6.0, 70)], None], ids=["ma7_tube", "batch2", "ring"])
def test_d3q4913_line_moment_state_matches_population_step(torch, specs):
    if specs is None:                                   # periodic ring of 50 nodes, no shift
        from paper_2401_11086_amd import Lattice
        vs = O.make_velocity_set(*D1Q17)
        tau = {key: float(v) * 2.0 * vs.r / 0.6 for key, v in O.TAU_STAR_SMRT.items() if key[0] <= 5}
        lat = Lattice(D1Q17[0], D1Q17[1], 5, tau, [dict(nx=50, ny=1, nz=1, bc_x=0)], precision="fp64_contract")
        rng = np.random.default_rng(41)
        fields = np.zeros((5, 50))
        fields[0] = 1.0 + 0.03 * rng.uniform(-1, 1, 50)
        fields[1] = 0.05 * rng.uniform(-1, 1, 50)
        fields[4] = 1.0 + 0.03 * rng.uniform(-1, 1, 50)
    else:
        lat, fields = _ma7_tubes(specs)
    n = lat.n_nodes
    assert lat.moment_state_len()[1] == 0
    m0 = _noisy_moments(torch, lat, fields, seed=42)
    f0 = lat.expand_state(m0)
    steps = 5
    f_pop = lat.step(f0.clone(), lat.new_state(), steps)
    m_out = lat.step_moment_state(m0, lat.new_moment_state(), lat.new_moment_work(), steps)
    lat.sync()
    f_mom = lat.expand_state(m_out)
    torch.cuda.synchronize()
    a, b = f_mom[:, :n].double(), f_pop[:, :n].double()
    err = float((a - b).abs().max() / b.abs().max())
    print(f"D3Q4913 {specs}: {steps} steps, line moment state vs population state {err:.2e}")
    assert err < TOL_STEP, err
    # the projection of the population state returns the moments it was expanded from
    back = lat.project_state(f_pop)
    torch.cuda.synchronize()
    assert torch.isfinite(back[:, :n]).all()


def test_d3q4913_line_moment_state_one_step_matches_oracle(torch):
    case = shock_case(7.0, 40, D1Q17, 5)
    lat = _lattice(case)
    m0 = _noisy_moments(torch, lat, case["fields"], seed=43)
    f0 = lat.expand_state(m0)
    m1 = lat.step_moment_state(m0, lat.new_moment_state(), lat.new_moment_work(), 1)
    lat.sync()
    g = lat.expand_state(m1)[:, :40].double().cpu().numpy()
    fo1 = O.step(oracle_state_from_gpu(f0.cpu().numpy(), case), case["model"], case["dom"])
    err = float(np.abs(g - fo1.reshape(g.shape)).max() / np.abs(fo1).max())
    print(f"D3Q4913 Ma 7 shock, one line moment-state step vs FP64 oracle: {err:.2e}")
    assert err < TOL_STEP, err


def test_d3q4913_project_expand_round_trip(torch):
    """expand then project returns the moments (the quadrature is exact to degree 2N)."""
    case = shock_case(7.0, 30, D1Q17, 5)
    lat = _lattice(case)
    m0 = _noisy_moments(torch, lat, case["fields"], seed=44)
    m1 = lat.project_state(lat.expand_state(m0))
    torch.cuda.synchronize()
    n = lat.n_nodes
    err = float((m1[:, :n].double() - m0[:, :n].double()).abs().max() / m0[:, :n].double().abs().max())
    print(f"D3Q4913 project(expand(m)) - m: {err:.2e}")
    assert err < 1e-6, err


def test_d3q4913_line_moment_state_sixteen_lanes_agree_with_one(torch):
    """Shock tubes run the 17-point line kernel with sixteen lanes per node (one tap pair each,
    the partial moments summed over the row) when the lane setting is four or more: 4 steps agree
    with one lane per node to float32 rounding."""
    lat, fields = _ma7_tubes([(7.0, 57), (6.5, 30)])
    n = lat.n_nodes
    m0 = _noisy_moments(torch, lat, fields, seed=45)
    outs = []
    for lanes in (1, 8):
        lat.set_launch("direct", 0, 64, lanes)
        ma = m0.clone()
        outs.append(lat.step_moment_state(ma, lat.new_moment_state(), lat.new_moment_work(), 4).clone())
    lat.sync()
    a, b = outs[1][:, :n].double(), outs[0][:, :n].double()
    err = float((a - b).abs().max() / b.abs().max())
    print(f"D3Q4913 line moment state, sixteen lanes vs one after 4 steps: {err:.2e}")
    assert err < 2e-6, err
