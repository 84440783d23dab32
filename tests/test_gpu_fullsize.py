"""Parity at the benchmark sizes, in the launch configuration bench.py times:
256^3 D3Q343 box and the 64-shock D3Q729 Mach sweep.  The oracle computes the
sampled nodes one by one from the populations the GPU pulled."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

from cases import gather_columns, pull_indices

pytestmark = pytest.mark.gpu

TAU_STAR = {k: float(v) for k, v in O.TAU_STAR_SMRT.items()}
H_CS = 1e-30


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def box256(torch):
    from paper_2401_11086_amd import Lattice
    vs = O.make_velocity_set([1, 2, 3], 9)
    edge = 256
    tau = {k: v * 0.05 * edge * vs.r for k, v in TAU_STAR.items() if k[0] <= 4}
    lat = Lattice([1, 2, 3], 9, 4, tau, [dict(nx=edge, ny=edge, nz=edge)], precision="fp64_contract")
    fields = W.fourier_box_torch(edge, "cuda")
    f0 = lat.equilibrium(fields)
    del fields
    # a non-equilibrium state: multiplicative noise
    g = torch.Generator(device="cuda").manual_seed(3)
    f0[:, :lat.n_nodes] *= 1.0 + 0.02 * torch.randn((lat.Q, lat.n_nodes), device="cuda", generator=g)
    model = O.Model(vs=vs, N=4, tau=tau)
    yield lat, f0, model
    del f0
    torch.cuda.empty_cache()


def test_box256_step_at_sampled_nodes_matches_oracle(torch, box256):
    lat, f0, model = box256
    f1 = lat.new_state()
    lat.step(f0, f1, 1)
    lat.sync()
    rng = np.random.default_rng(7)
    nodes = rng.integers(0, lat.n_nodes, size=256)
    idx = pull_indices(model, (256, 256, 256), nodes)
    g = gather_columns(torch, f0, idx)
    ref = O.collide(g, model)
    got = f1[:, torch.tensor(nodes, device="cuda")].double().cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"256^3 box, 256 sampled nodes: max scaled error {err:.2e}")
    assert err < 1e-5


def test_box256_adjoint_localised_dot_product(torch, box256):
    """<lam_t, v> = <lam_{t+1}, J v> for v supported on one node's populations: J v is non-zero
    only at the <= 343 nodes those populations stream to, each computed by the oracle with a
    complex-step directional derivative of its collision."""
    lat, f0, model = box256
    n = lat.n_nodes
    lam_next = lat.new_state()
    g = torch.Generator(device="cuda").manual_seed(11)
    lam_next[:, :n] = torch.randn((lat.Q, n), device="cuda", generator=g)
    lam_t = lat.new_state()
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    lat.step_adjoint(f0, lam_next, lam_t, dtau)
    lat.sync()
    assert torch.isfinite(dtau).all()
    rng = np.random.default_rng(12)
    y0 = int(rng.integers(0, n))
    v = rng.standard_normal(lat.Q)
    lhs = float((lam_t[:, y0].double().cpu().numpy() * v).sum())
    # targets: node x_i = y0 + s_i receives population i of y0
    s = model.streaming_offsets()
    x0, yy, zz = y0 % 256, (y0 // 256) % 256, y0 // 65536
    tx = ((x0 + s[:, 0]) % 256) + 256 * (((yy + s[:, 1]) % 256) + 256 * ((zz + s[:, 2]) % 256))
    idx = pull_indices(model, (256, 256, 256), tx)
    gx = gather_columns(torch, f0, idx)                      # (Q, Q): pulled populations of each target node
    pert = np.zeros_like(gx, dtype=complex)
    pert[np.arange(lat.Q), np.arange(lat.Q)] = 1j * H_CS * v    # node i gets v_i on population i
    jv = O.collide(gx + pert, model).imag / H_CS
    lam_x = lam_next[:, torch.tensor(tx, device="cuda")].double().cpu().numpy()
    rhs = float((lam_x * jv).sum())
    scale = float(np.abs(lam_t[:, y0].double().cpu().numpy() * v).sum())
    print(f"adjoint dot product: {lhs:.8e} vs {rhs:.8e}")
    assert abs(lhs - rhs) <= 1e-6 * scale + 1e-5 * abs(rhs)


def test_mach_sweep_step_at_sampled_nodes_matches_oracle(torch):
    """The 64-shock D3Q729 N=5 sweep as bench.py runs it (one context, autotuned launch)."""
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.autotune import autotune
    from paper_2401_11086_amd.shocks import shock_domain
    ab, deg, N = [1, 2, 3, 5], 11, 5
    c_l, _ = solve_quadrature(ab, deg)
    doms, fields = [], []
    for Ma, nx in W.mach_sweep(64, seed=0):
        d, f, _ = shock_domain(Ma, nx, c_l)
        doms.append(d)
        fields.append(f)
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= N}
    lat = Lattice(ab, deg, N, tau, doms, shift_k=(2, 0, 0), precision="fp64_contract")
    fl = torch.tensor(np.concatenate(fields, axis=1), dtype=torch.float64, device="cuda")
    fa = lat.equilibrium(fl)
    fb = lat.new_state()
    autotune(lat, fa, fb, steps=10, use_cache=False)
    fa = lat.equilibrium(fl)
    n = lat.n_nodes
    fa[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=4), dtype=torch.float32, device="cuda")
    lat.step(fa, fb, 1)
    lat.sync()
    vs = O.make_velocity_set(ab, deg)
    rng = np.random.default_rng(8)
    worst = 0.0
    for i in rng.choice(64, size=12, replace=False):
        d = doms[i]
        nx, off = d["nx"], lat.domain_offset[i]
        model = O.Model(vs=vs, N=N, tau={k: v * d["tau_scale"] for k, v in tau.items()}, shift=(2, 0, 0))
        xs = np.unique(np.concatenate([[0, 1, nx - 2, nx - 1], rng.integers(0, nx, size=8)]))
        sx = model.streaming_offsets()[:, 0]
        src = xs[None, :] - sx[:, None]                  # (Q, n) x of the source
        inside = (src >= 0) & (src < nx)
        g = gather_columns(torch, fa, np.where(inside, off + src, off)).copy()
        fin = O.equilibrium_f(np.array(d["rho_in"]), np.array(d["u_in"]), np.array(d["theta_in"]), model)
        fout = O.equilibrium_f(np.array(d["rho_out"]), np.array(d["u_out"]), np.array(d["theta_out"]), model)
        g = np.where(src < 0, fin[:, None], np.where(src >= nx, fout[:, None], g))
        ref = O.collide(g, model)
        got = fb[:, torch.tensor(off + xs, device="cuda")].double().cpu().numpy()
        worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    print(f"Mach sweep, 12 shocks x ~12 sampled cells: max scaled error {worst:.2e}")
    assert worst < 1e-5
