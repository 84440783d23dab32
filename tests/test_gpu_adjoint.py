"""The hand-written adjoint (lbsmrt_step_adjoint, lbsmrt_loss_seed) against
complex-step derivatives of the FP64 oracle on the same FP32 input state."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

from cases import D1Q7, D1Q9, box_case, oracle_state_from_gpu, shock_case

pytestmark = pytest.mark.gpu

H_CS = 1e-30


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _lattice(case, precision="fp64_contract"):
    from paper_2401_11086_amd import Lattice
    return Lattice(precision=precision, **case["lat_kw"])


def _state(torch, lat, case, seed):
    f = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    n = lat.n_nodes
    f[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=seed, amp=0.02), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    return f


def _flat(case, f_np):
    return f_np.reshape(f_np.shape[0], -1)


ADJ_CASES = {
    "shock_q343_n4": lambda: shock_case(1.2, 24, D1Q7, 4),
    "shock_q729_n5": lambda: shock_case(3.0, 20, D1Q9, 5),
    "box_q343_n4": lambda: box_case(5, D1Q7, 4, n_ref=16),
}


@pytest.mark.parametrize("name", list(ADJ_CASES))
def test_adjoint_step_matches_oracle_directional_derivatives(torch, name):
    """<lam_t, v> = <lam_{t+1}, J v> for random v, and dL/dtau_nm = <lam_{t+1}, df_{t+1}/dtau_nm>,
    with J v and df/dtau from complex-step derivatives of the oracle step."""
    case = ADJ_CASES[name]()
    lat = _lattice(case)
    n = lat.n_nodes
    f_t = _state(torch, lat, case, seed=11)
    fo = oracle_state_from_gpu(f_t.cpu().numpy(), case)
    rng = np.random.default_rng(5)
    lam_np = rng.standard_normal((lat.Q, n)).astype(np.float32)
    lam_next = lat.new_state()
    lam_next.zero_()
    lam_next[:, :n] = torch.tensor(lam_np, device="cuda")
    lam_t = lat.new_state()
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    lat.step_adjoint(f_t, lam_next, lam_t, dtau)
    lat.sync()
    lt = lam_t[:, :n].double().cpu().numpy()
    lam64 = lam_np.astype(np.float64)
    for seed in range(3):
        v = np.random.default_rng(100 + seed).standard_normal(fo.shape)
        Jv = O.step(fo + 1j * H_CS * v, case["model"], case["dom"]).imag / H_CS
        rhs = float((lam64 * _flat(case, Jv)).sum())
        lhs = float((lt * _flat(case, v)).sum())
        scale = float(np.abs(lt * _flat(case, v)).sum())
        assert abs(lhs - rhs) <= 1e-6 * scale + 1e-5 * abs(rhs), (seed, lhs, rhs, scale)
    g = dtau.view(6, 3).cpu().numpy()
    base = dict(case["model"].tau)
    for key in [k for k in sorted(base) if k[0] <= case["model"].N and k != (2, 1)]:
        tau_c = dict(base)
        tau_c[key] = complex(base[key], H_CS)
        m = O.Model(vs=case["model"].vs, N=case["model"].N, tau=tau_c, shift=case["model"].shift)
        dfdt = O.step(fo, m, case["dom"]).imag / H_CS
        rhs = float((lam64 * _flat(case, dfdt)).sum())
        assert abs(g[key] - rhs) <= 1e-4 * abs(rhs) + 1e-9, (key, g[key], rhs)


def _fit_case(torch, nx, steps, every, stencil=D1Q9, N=5, Ma=3.0):
    from paper_2401_11086_amd.adjoint import ShockFit
    case = shock_case(Ma, nx, stencil, N)
    lat = _lattice(case)
    f0 = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    st = case["states"]
    scales = (1.0 / (st["rho2"] - st["rho1"]), 1.0 / (st["theta2"] - st["theta1"]), 1.0 / st["theta1"] ** 1.5)
    # target: the oracle's FP64 forward with the Table 4 relaxation times
    fo0 = oracle_state_from_gpu(f0.cpu().numpy(), case)
    fo = fo0
    for _ in range(steps):
        fo = O.step(fo, case["model"], case["dom"])
    ob = O.observables(fo, case["model"], case["dom"])
    target = np.stack([ob["rho"], ob["theta"], ob["q"][0]])
    fit = ShockFit(lat, f0, torch.tensor(target, device="cuda"), scales, steps, every)
    return case, lat, fit, fo0, target, scales


def test_loss_and_gradient_through_many_steps_match_oracle(torch):
    """Ma = 3, D3Q729, N = 5, 40 cells, 30 steps with checkpoints every 10, relaxation
    times perturbed by +-20 %: L and dL/dtau against complex-step derivatives of the oracle."""
    from paper_2401_11086_amd.adjoint import SMRTShockLoss, tau_keys
    steps = 30
    case, lat, fit, fo0, target, scales = _fit_case(torch, 40, steps, 10)
    keys = tau_keys(5)
    tau0 = W.perturbed_taus({k: case["model"].tau[k] for k in keys}, seed=0, frac=0.2)
    tau_vec = torch.tensor([tau0[k] for k in keys], dtype=torch.float64, requires_grad=True)
    L = SMRTShockLoss.apply(tau_vec, fit)
    L.backward()
    g_gpu = tau_vec.grad.numpy()
    tgt = dict(rho=target[0], theta=target[1], q_x=target[2])

    def oracle_loss(tau):
        full = dict(case["model"].tau)
        full.update(tau)
        m = O.Model(vs=case["model"].vs, N=5, tau=full, shift=case["model"].shift)
        f = fo0
        for _ in range(steps):
            f = O.step(f, m, case["dom"])
        return O.shock_loss(f, m, case["dom"], tgt, scales)
    L_o = float(np.real(oracle_loss(tau0)))
    assert abs(float(L.detach()) - L_o) <= 1e-4 * L_o, (float(L.detach()), L_o)
    g_o = []
    for k in keys:
        t = dict(tau0)
        t[k] = complex(tau0[k], H_CS)
        g_o.append(oracle_loss(t).imag / H_CS)
    g_o = np.array(g_o)
    err = np.abs(g_gpu - g_o).max() / np.abs(g_o).max()
    print(f"L gpu {float(L.detach()):.6e} oracle {L_o:.6e}; grad rel err {err:.2e}")
    assert err < 1e-3, (g_gpu, g_o)


def test_gradient_is_independent_of_checkpoint_spacing(torch):
    from paper_2401_11086_amd.adjoint import tau_keys
    grads = []
    for every in (4, 100):
        case, lat, fit, fo0, target, scales = _fit_case(torch, 24, 12, every, D1Q7, 4, Ma=1.2)
        keys = tau_keys(4)
        fit.set_tau([case["model"].tau[k] * 1.1 for k in keys])
        fit.forward()
        grads.append(np.array(fit.backward()))
    assert np.array_equal(grads[0], grads[1])


def test_zero_misfit_gives_zero_loss_and_gradient(torch):
    """Target = the GPU's own forward moments at the same tau: L = 0 and dL/dtau = 0."""
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd.adjoint import ShockFit
    case = shock_case(1.2, 24, D1Q7, 4)
    lat = _lattice(case)
    f0 = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    cur = lat.step(fa, fb, 8)
    m = lat.moments(cur, C.MOM_BASIC | C.MOM_Q)
    target = torch.stack([m[0], m[4], m[5]]).contiguous()
    fit = ShockFit(lat, f0, target, (1.0, 1.0, 1.0), 8, 3)
    L = fit.forward()
    g = fit.backward()
    assert L < 1e-25, L
    assert max(abs(v) for v in g) < 1e-12, g


@pytest.mark.parametrize("name", ["shock_q343_n4", "shock_q729_n5"])
@pytest.mark.parametrize("lpn", [4, 8, 16])
def test_adjoint_split_lanes_match_one_lane(torch, name, lpn):
    """The adjoint step with each node's slabs split over four, eight or sixteen lanes against one
    lane per node: same lam_t up to the order of the FP64 sums, same dL/dtau."""
    case = ADJ_CASES[name]()
    lat = _lattice(case)
    n = lat.n_nodes
    f_t = _state(torch, lat, case, seed=13)
    lam_next = lat.new_state()
    lam_next.zero_()
    lam_next[:, :n] = torch.tensor(np.random.default_rng(6).standard_normal((lat.Q, n)), dtype=torch.float32,
                                   device="cuda")
    out = {}
    for k in (lpn, 1):
        lat.set_launch("direct", 0, 64, k)
        lam_t = lat.new_state()
        lam_t.zero_()
        dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
        lat.step_adjoint(f_t, lam_next, lam_t, dtau)
        lat.sync()
        out[k] = (lam_t[:, :n].double().clone(), dtau.clone())
    (l4, d4), (l1, d1) = out[lpn], out[1]
    err = float((l4 - l1).abs().max() / l1.abs().max())
    derr = float((d4 - d1).abs().max() / d1.abs().max())
    print(f"{name}, {lpn} lanes: lam_t {err:.2e}, dL/dtau {derr:.2e}")
    assert err < 1e-6
    assert derr < 1e-10


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_gradient():
    steps, loss, tau0, grad = None, None, {}, {}
    with open(os.path.join(GOLDEN, "shock_gradient_ma3_q729_n5_nx600.txt")) as fh:
        for ln in fh:
            w = ln.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "steps":
                steps = int(w[1])
            elif w[0] == "loss":
                loss = float(w[1])
            else:
                key = (int(w[0]), int(w[1]))
                tau0[key], grad[key] = float(w[2]), float(w[3])
    target = np.loadtxt(os.path.join(GOLDEN, "shock_target_ma3_q729_n5_nx600.txt"))[:, 1:].T.copy()
    return steps, loss, tau0, grad, target


def test_calibration_gradient_at_full_shape_matches_oracle(torch):
    """The calibration workload at its stated shape: Ma = 3, D3Q729, N = 5, Nx = 600, the full
    step count with checkpoints every 100 steps, relaxation times perturbed by +-20 % (seed 0).
    Misfit and every dL/dtau_nm from the checkpointed adjoint sweep against the FP64 oracle's
    complex-step gradient from the same float32 initial state (tests/golden, written by
    make_shock_gradient.py): each component within 1e-3 of the largest, L within 1e-4."""
    from paper_2401_11086_amd.adjoint import ShockFit, tau_keys
    steps, L_o, tau0, g_o, target = _golden_gradient()
    case = shock_case(3.0, 600, D1Q9, 5)
    lat = _lattice(case)
    n = lat.n_nodes
    f0 = lat.equilibrium(torch.tensor(case["fields"], dtype=torch.float64, device="cuda"))
    fo = O.equilibrium_f(case["fields"][0], case["fields"][1:4], case["fields"][4], case["model"])
    f0[:, :n] = torch.tensor(fo.astype(np.float32), device="cuda")
    st = case["states"]
    scales = (1.0 / (st["rho2"] - st["rho1"]), 1.0 / (st["theta2"] - st["theta1"]), 1.0 / st["theta1"] ** 1.5)
    fit = ShockFit(lat, f0, torch.tensor(target, device="cuda"), scales, steps, 100)
    keys = tau_keys(5)
    fit.set_tau([tau0[k] for k in keys])
    L = fit.forward()
    g = np.array(fit.backward())
    go = np.array([g_o[k] for k in keys])
    err = np.abs(g - go) / np.abs(go).max()
    print(f"{steps} steps: L gpu {L:.8e} oracle {L_o:.8e}; dL/dtau rel err per component " +
          ", ".join(f"{k[0]}{k[1]} {e:.1e}" for k, e in zip(keys, err)))
    assert abs(L - L_o) <= 1e-4 * L_o, (L, L_o)
    assert err.max() < 1e-3, (g, go)


def test_gradient_descent_fit_lowers_misfit(torch):
    """A reduced calibration (Ma = 3, D3Q729, N = 5, 100 cells, 300 steps, checkpoints every 100)
    against the oracle's target profiles: ten Armijo steps on log tau lower L at every iteration,
    by more than a factor four overall, and bring tau_20 and tau_31 (the times the rho, theta,
    q_x profiles identify best) closer to their Table 4 values."""
    from paper_2401_11086_amd.calibrate import descend
    steps = 300
    case, lat, fit, fo0, target, scales = _fit_case(torch, 100, steps, 100)
    keys = fit.keys
    true = {k: case["model"].tau[k] for k in keys}
    tau0 = W.perturbed_taus(true, seed=0, frac=0.2)
    tau_fit, hist = descend(fit, tau0, 10)
    print("L: " + ", ".join(f"{v:.3e}" for v in hist))
    assert all(b <= a for a, b in zip(hist, hist[1:])), hist
    assert hist[-1] < 0.25 * hist[0], hist
    for k in [(2, 0), (3, 1)]:
        assert abs(tau_fit[k] / true[k] - 1) < abs(tau0[k] / true[k] - 1), (k, tau0[k], tau_fit[k], true[k])
