"""The allocation-free adjoint entry point (lbsmrt_step_adjoint_noalloc) against
lbsmrt_step_adjoint: same kernels and summation order, so lam_t and the dL/dtau increment
must agree bit for bit.  Two calls in a row on the library's fixed scratch, the second on a
smaller context, then the size limit."""
import numpy as np
import pytest

from paper_2401_11086_amd import workloads as W

from cases import D1Q7, D1Q9, box_case, shock_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _setup(torch, case, seed):
    from paper_2401_11086_amd import Lattice
    lat = Lattice(precision="fp64_contract", **case["lat_kw"])
    n = lat.n_nodes
    f_t = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    f_t[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=seed, amp=0.02), dtype=torch.float32, device="cuda")
    lam_next = lat.new_state()
    lam_next.zero_()
    rng = np.random.default_rng(seed + 1)
    lam_next[:, :n] = torch.tensor(rng.standard_normal((lat.Q, n)).astype(np.float32), device="cuda")
    # a non-zero starting gradient: both entry points add their increment to it
    dtau0 = torch.tensor(rng.standard_normal(18), dtype=torch.float64, device="cuda")
    return lat, f_t, lam_next, dtau0


def _reference(lat, f_t, lam_next, dtau0):
    lam_t = lat.new_state()
    lam_t.fill_(7.0)
    dtau = dtau0.clone()
    lat.step_adjoint(f_t, lam_next, lam_t, dtau)
    return lam_t, dtau


def test_noalloc_adjoint_matches_allocating_entry_on_two_calls(torch):
    """First call on a 24^3 periodic D3Q343 box (N = 4, the 256-node adjoint work-groups, 54
    partial rows of 6), second on a 40-node D3Q729 shock tube (N = 5, several lanes per node,
    partial rows of 9): the second call reads none of the first call's scratch contents."""
    big = _setup(torch, box_case(24, D1Q7, 4, n_ref=16), seed=3)
    small = _setup(torch, shock_case(3.0, 40, D1Q9, 5), seed=4)
    assert small[0].n_nodes < big[0].n_nodes
    refs = [_reference(*big), _reference(*small)]
    torch.cuda.synchronize()
    outs = []
    for lat, f_t, lam_next, dtau0 in (big, small):       # two calls in a row on the shared scratch
        lam_t = lat.new_state()
        lam_t.fill_(7.0)
        dtau = dtau0.clone()
        lat.step_adjoint_noalloc(f_t, lam_next, lam_t, dtau)
        outs.append((lam_t, dtau))
    torch.cuda.synchronize()
    for (lat, _, _, dtau0), (lam_r, dtau_r), (lam_o, dtau_o) in zip((big, small), refs, outs):
        n = lat.n_nodes
        assert torch.equal(lam_o[:, :n], lam_r[:, :n]), lat.n_nodes
        assert torch.equal(dtau_o, dtau_r), (dtau_o.cpu().numpy(), dtau_r.cpu().numpy())
        assert torch.count_nonzero(dtau_o - dtau0).item() > 0          # an increment was added
    # once more on the big context after the small one: stale rows of the small call are not read
    lat, f_t, lam_next, dtau0 = big
    lam_t = lat.new_state()
    dtau = dtau0.clone()
    lat.step_adjoint_noalloc(f_t, lam_next, lam_t, dtau)
    torch.cuda.synchronize()
    assert torch.equal(lam_t[:, :lat.n_nodes], refs[0][0][:, :lat.n_nodes])
    assert torch.equal(dtau, refs[0][1])
    for ctx in (big, small):
        ctx[0].close()


def test_noalloc_adjoint_refuses_contexts_beyond_its_scratch(torch):
    """A 200^3 periodic D3Q729 box with N = 5 needs 125000 partial rows of 9 doubles, more than
    the 2^20 the fixed scratch holds: E_LIMIT before any launch, while the allocating entry
    point's context buffers are sized for it."""
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd import Lattice
    case = box_case(8, D1Q9, 5)
    kw = dict(case["lat_kw"])
    kw["domains"] = [dict(nx=200, ny=200, nz=200, bc_x=0)]
    lat = Lattice(precision="fp64_contract", **kw)
    buf = torch.zeros(16, dtype=torch.float32, device="cuda")
    other = torch.zeros(16, dtype=torch.float32, device="cuda")
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    with pytest.raises(C.LbsmrtError) as e:
        lat.step_adjoint_noalloc(buf, other, torch.zeros_like(buf), dtau)
    assert e.value.status == C.E_LIMIT
    assert torch.count_nonzero(dtau).item() == 0
    lat.close()
