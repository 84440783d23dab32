"""D3Q4913 (tensor product of D1Q17 {0, +-1..+-7, +-9}, degree 19; Table 3's set for Ma 7)
through the C ABI against the FP64 oracle on the same seeded states: one step of a Ma 7 shock
tube (one and eight lanes per node) and of a small periodic box, and the calls the library
refuses for this stencil."""
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


@pytest.mark.parametrize("lanes", [1, 8])
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
    for call in (lambda: lat.step_adjoint(f, lat.new_state(), lat.new_state(), dtau),
                 lambda: lat.project_state(f),
                 lambda: lat.expand_state(lat.new_moment_state())):
        with pytest.raises(C.LbsmrtError) as e:
            call()
        assert e.value.status == C.E_UNSUPPORTED
