"""Error behaviour of the C ABI on a live context (argument checks are synchronous and leave the
context usable), and relaxation-time updates under every launch mode."""
import ctypes

import numpy as np
import pytest

import oracle as O

from cases import D1Q7, shock_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _lat(case):
    from paper_2401_11086_amd import Lattice
    return Lattice(precision="fp64_contract", **case["lat_kw"])


def test_argument_errors_are_synchronous_and_harmless(torch):
    from paper_2401_11086_amd import _lib as C
    case = shock_case(1.2, 40, D1Q7, 4)
    lat = _lat(case)
    fa = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    fb = lat.new_state()
    lib, h = C.lib(), lat._h
    pa, pb = ctypes.c_void_p(fa.data_ptr()), ctypes.c_void_p(fb.data_ptr())
    assert lib.lbsmrt_step(h, pa, pa, 1, None) == C.E_ARG            # f_a == f_b
    assert lib.lbsmrt_step(h, pa, pb, 0, None) == C.E_ARG            # n_steps < 1
    assert lib.lbsmrt_step(h, None, pb, 1, None) == C.E_ARG
    assert lib.lbsmrt_set_launch(h, 7, 0, 64, 0) == C.E_ARG          # unknown mode
    assert lib.lbsmrt_set_launch(h, C.LAUNCH_DIRECT, 96, 64, 0) == C.E_ARG
    assert lib.lbsmrt_set_launch(h, C.LAUNCH_GRAPH, 0, 3, 0) == C.E_ARG   # odd graph_steps
    bad_tau = (ctypes.c_double * 18)(*([1.0] * 18))
    bad_tau[2 * 3 + 0] = -1.0
    assert lib.lbsmrt_set_tau(h, bad_tau) == C.E_ARG
    lam = lat.new_state()
    assert lib.lbsmrt_step_adjoint(h, pa, pa, pa, None, None) == C.E_ARG
    # the context still works and matches a fresh one
    ref = _lat(case)
    ra = ref.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    rb = ref.new_state()
    out = lat.step(fa, fb, 3)
    rout = ref.step(ra, rb, 3)
    lat.sync()
    ref.sync()
    n = lat.n_nodes
    assert torch.equal(out[:, :n], rout[:, :n])
    del lam


@pytest.mark.parametrize("mode", ["direct", "graph", "persistent"])
def test_set_tau_takes_effect_in_every_launch_mode(torch, mode):
    """After lbsmrt_set_tau the next steps use the new times (a captured graph is re-captured):
    one step against the oracle with the new times."""
    case = shock_case(1.2, 40, D1Q7, 4)
    lat = _lat(case)
    lat.set_launch(mode, 0, 2)
    fa = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    fb = lat.new_state()
    lat.step(fa, fb, 2)                    # captures (graph mode) with the old times
    lat.sync()
    new = {k: v * 1.7 for k, v in case["model"].tau.items()}
    lat.set_tau(new)
    f0 = fa.clone()
    out = lat.step(fa, fb, 2)
    lat.sync()
    model = O.Model(vs=case["model"].vs, N=4, tau=new, shift=case["model"].shift, rho_ref=1.0)
    n = lat.n_nodes
    fo = f0[:, :n].double().cpu().numpy().reshape(-1, 1, 1, n)
    for _ in range(2):
        fo = O.step(fo, model, case["dom"])
    g = out[:, :n].double().cpu().numpy().reshape(fo.shape)
    err = np.abs(g - fo).max() / np.abs(fo).max()
    print(f"{mode}: two steps after set_tau, max scaled error {err:.2e}")
    assert err < 1e-5


def test_empty_and_degenerate_domains_are_rejected(torch):
    from paper_2401_11086_amd import Lattice, LbsmrtError
    tau = {k: float(v) for k, v in O.TAU_STAR_SMRT.items() if k[0] <= 4}
    with pytest.raises(LbsmrtError):
        Lattice([1, 2, 3], 9, 4, tau, [])                                   # no domain
    with pytest.raises(LbsmrtError):
        Lattice([1, 2, 3], 9, 4, tau, [dict(nx=0, ny=4, nz=4)])             # empty domain
    with pytest.raises(LbsmrtError):
        Lattice([1, 2, 3], 9, 4, tau, [dict(nx=8, ny=8, nz=8, bc_x=2)])     # unknown boundary
    with pytest.raises(LbsmrtError):
        Lattice([1, 2, 3, 4], 11, 4, tau, [dict(nx=8, ny=8, nz=8)])         # no positive-weight rule


@pytest.mark.parametrize("precision,lpn", [("fp64_contract", 1), ("fp32", 1), ("fp64_contract", 8)])
def test_uniform_maxwellian_is_a_fixed_point(torch, precision, lpn):
    """A uniform truncated Maxwellian (moving, theta != 1) is unchanged by a step (eq:SMRT relaxes
    nothing at equilibrium), periodic box and shock tube with matching end states."""
    from paper_2401_11086_amd import Lattice
    tau = {k: float(v) * 1.3 for k, v in O.TAU_STAR_SMRT.items() if k[0] <= 4}
    rho, u, th = 1.3, (0.11, -0.05, 0.02), 0.9
    tube = dict(nx=37, bc_x=1, rho_in=rho, u_in=u, theta_in=th, rho_out=rho, u_out=u, theta_out=th)
    for doms, k in (([dict(nx=6, ny=5, nz=7)], (0, 0, 0)), ([tube], (0, 0, 0))):
        lat = Lattice([1, 2, 3], 9, 4, tau, doms, shift_k=k, precision=precision)
        if lpn > 1:
            if not any(d.get("bc_x", 0) for d in doms):
                continue
            lat.set_launch("direct", 0, 64, lpn)
        n = lat.n_nodes
        fields = torch.tensor(np.array([[rho] * n, [u[0]] * n, [u[1]] * n, [u[2]] * n, [th] * n]),
                              dtype=torch.float64, device="cuda")
        fa = lat.equilibrium(fields)
        fb = lat.new_state()
        out = lat.step(fa, fb, 1)
        lat.sync()
        err = float((out[:, :n].double() - fa[:, :n].double()).abs().max() / fa[:, :n].double().abs().max())
        print(f"{precision}, {lpn} lanes, {'tube' if doms[0].get('bc_x') else 'box'}: change {err:.2e}")
        assert err < 2e-6
