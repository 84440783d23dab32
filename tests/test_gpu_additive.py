"""Additive collision f* = g + R (a' - a) (regularized = 0) through the C ABI, against the FP64
oracle's additive form on the same seeded states: shock tubes of both stencils and a periodic
box, one step from a state with content outside the Hermite span; conservation on the box;
and the combinations the library refuses."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

from cases import D1Q7, D1Q9, box_case, oracle_state_from_gpu, shock_case

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _additive(case):
    from paper_2401_11086_amd import Lattice
    case = dict(case)
    case["model"] = dataclasses.replace(case["model"], regularized=False)
    return case, Lattice(precision="fp64_contract", regularized=False, **case["lat_kw"])


def _noisy_state(torch, lat, case, seed):
    f = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    n = case["nx"] * case["ny"] * case["nz"]
    f[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=seed, amp=0.02), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    return f


CASES = {
    "shock_q343_n4_ma1.2": lambda: shock_case(1.2, 200, D1Q7, 4),
    "shock_q729_n5_ma3": lambda: shock_case(3.0, 64, D1Q9, 5),
    "box_q343_n4_10": lambda: box_case(10, D1Q7, 4, n_ref=32),
}


@pytest.mark.parametrize("name", list(CASES))
def test_additive_step_matches_oracle(torch, name):
    case, lat = _additive(CASES[name]())
    n = case["nx"] * case["ny"] * case["nz"]
    f0 = _noisy_state(torch, lat, case, seed=11)
    fo0 = oracle_state_from_gpu(f0.cpu().numpy(), case)
    f1 = lat.step(f0, lat.new_state(), 1)
    lat.sync()
    fo1 = O.step(fo0, case["model"], case["dom"])
    g = f1[:, :n].double().cpu().numpy().reshape(fo1.shape)
    err = float(np.abs(g - fo1).max() / np.abs(fo1).max())
    # the rebuilt collision from the same state differs by the non-Hermite part of g
    reg = O.step(fo0, dataclasses.replace(case["model"], regularized=True), case["dom"])
    gap = float(np.abs(reg - fo1).max() / np.abs(fo1).max())
    print(f"{name}: additive step vs oracle {err:.2e} (rebuilt collision differs by {gap:.2e})")
    assert err < TOL_STEP, err
    assert gap > 100 * TOL_STEP


def test_additive_box_conserves_mass_momentum_energy(torch):
    """Both collisions conserve mass, momentum and energy exactly; on the GPU both are limited by
    the float32 rounding of the stored state, so the additive path drifts no more than the
    rebuilt one from the same state."""
    from paper_2401_11086_amd import Lattice
    case, lat = _additive(box_case(12, D1Q7, 4, n_ref=32))
    reg = Lattice(precision="fp64_contract", **case["lat_kw"])
    n = case["nx"] * case["ny"] * case["nz"]
    f0 = _noisy_state(torch, lat, case, seed=12)
    e = torch.tensor(lat.e1d, dtype=torch.float64, device="cuda")
    Q1 = lat.Q1
    ex = e.repeat_interleave(Q1 * Q1)
    ey = e.repeat_interleave(Q1).repeat(Q1)
    ez = e.repeat(Q1 * Q1)

    def totals(f):
        g = f[:, :n].double().sum(dim=1)
        return torch.stack([g.sum(), (g * ex).sum(), (g * ey).sum(), (g * ez).sum(),
                            (g * (ex * ex + ey * ey + ez * ez)).sum()])

    t0 = totals(f0)
    drift = {}
    for name, ctx in (("additive", lat), ("rebuilt", reg)):
        cur = ctx.step(f0.clone(), ctx.new_state(), 10)
        ctx.sync()
        drift[name] = ((totals(cur) - t0).abs() / n).cpu().numpy()
    print(f"per-node drift of mass, momentum, energy over 10 steps: {drift}")
    assert np.all(drift["additive"] <= np.maximum(4 * drift["rebuilt"], 1e-9)), drift


def test_additive_combinations_refused(torch):
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import _lib as C
    case = shock_case(1.2, 40, D1Q7, 4)
    with pytest.raises(C.LbsmrtError) as e:
        Lattice(precision="fp32", regularized=False, **case["lat_kw"])
    assert e.value.status == C.E_UNSUPPORTED
    lat = Lattice(precision="fp64_contract", regularized=False, **case["lat_kw"])
    assert lat.launch_settings()["lanes_per_node"] == 1
    for kw in (dict(mode="persistent"), dict(mode="direct", lanes_per_node=8)):
        with pytest.raises(C.LbsmrtError) as e:
            lat.set_launch(**kw)
        assert e.value.status == C.E_UNSUPPORTED
    lat.set_launch("graph", graph_steps=4)   # graph replay of the additive kernel is allowed
    f = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    lam = lat.new_state()
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    with pytest.raises(C.LbsmrtError) as e:
        lat.step_adjoint(f, lam, lat.new_state(), dtau)
    assert e.value.status == C.E_UNSUPPORTED
    box = Lattice([1, 2, 3], 9, 4, case["lat_kw"]["tau"], [dict(nx=8, ny=8, nz=8)], regularized=False)
    with pytest.raises(C.LbsmrtError) as e:
        box.step_moment_state(box.new_moment_state(), box.new_moment_state(), box.new_moment_work(), 1)
    assert e.value.status == C.E_UNSUPPORTED


def test_additive_graph_replay_matches_direct(torch):
    case, lat = _additive(shock_case(1.2, 200, D1Q7, 4))
    f0 = _noisy_state(torch, lat, case, seed=13)
    a = lat.step(f0.clone(), lat.new_state(), 8)
    lat.sync()
    lat.set_launch("graph", graph_steps=4)
    b = lat.step(f0.clone(), lat.new_state(), 8)
    lat.sync()
    n = case["nx"]
    assert torch.equal(a[:, :n], b[:, :n])     # padding columns are never written
