"""Batched shocks in one context: launch modes agree bitwise with each other and
with separate per-shock contexts; graph replays are checked one by one."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2401_11086_amd import workloads as W

pytestmark = pytest.mark.gpu

TAU_STAR = {k: float(v) for k, v in O.TAU_STAR_SMRT.items()}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _batch(torch, draws, ab=(1, 2, 3), deg=9, N=4, k=1):
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = solve_quadrature(list(ab), deg)
    doms, fields = [], []
    for Ma, nx in draws:
        d, f, _ = shock_domain(Ma, nx, c_l)
        doms.append(d)
        fields.append(f)
    tau = {key: v for key, v in TAU_STAR.items() if key[0] <= N}
    lat = Lattice(list(ab), deg, N, tau, doms, shift_k=(k, 0, 0), precision="fp64_contract")
    fl = torch.tensor(np.concatenate(fields, axis=1), dtype=torch.float64, device="cuda")
    return lat, fl, doms, fields, tau


DRAWS = [(1.2, 37), (1.6, 64), (2.2, 91), (1.35, 50), (2.0, 130)]


def test_batched_equals_separate_contexts(torch):
    from paper_2401_11086_amd import Lattice
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    fa = lat.equilibrium(fl)
    fb = lat.new_state()
    cur = lat.step(fa, fb, 20)
    lat.sync()
    for i, (d, f) in enumerate(zip(doms, fields)):
        one = Lattice([1, 2, 3], 9, 4, tau, [d], shift_k=(1, 0, 0), precision="fp64_contract")
        ga = one.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda"))
        gb = one.new_state()
        gc = one.step(ga, gb, 20)
        one.sync()
        off, n = lat.domain_offset[i], d["nx"]
        assert torch.equal(cur[:, off:off + n], gc[:, :n]), i


def test_more_than_64_domains_locate_and_match_separate_contexts(torch):
    """A batch of 70 short shocks: every domain offset is reported (beyond the 64 held by
    lbsmrt_info), and every shock equals its own separate context bitwise."""
    from paper_2401_11086_amd import Lattice
    rng = np.random.default_rng(4)
    draws = [(float(rng.uniform(1.2, 2.4)), int(rng.integers(20, 60))) for _ in range(70)]
    lat, fl, doms, fields, tau = _batch(torch, draws)
    assert len(lat.domain_offset) == 70
    assert lat.domain_offset == list(np.cumsum([0] + [d["nx"] for d in doms[:-1]]))
    fa = lat.equilibrium(fl)
    fb = lat.new_state()
    cur = lat.step(fa, fb, 9)
    lat.sync()
    for i, (d, f) in enumerate(zip(doms, fields)):
        one = Lattice([1, 2, 3], 9, 4, tau, [d], shift_k=(1, 0, 0), precision="fp64_contract")
        one.set_launch("direct", 0, 2, lat.launch_settings()["lanes_per_node"])
        ga = one.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda"))
        gb = one.new_state()
        gc = one.step(ga, gb, 9)
        one.sync()
        off, n = lat.domain_offset[i], d["nx"]
        assert torch.equal(cur[:, off:off + n], gc[:, :n]), i
        one.close()
    lat.close()


@pytest.mark.parametrize("mode", ["graph", "persistent"])
def test_launch_modes_match_direct_bitwise(torch, mode):
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    f0 = lat.equilibrium(fl)
    ref_a, ref_b = lat.new_state(), lat.new_state()
    ref_a.copy_(f0)
    ref = lat.step(ref_a, ref_b, 13)
    lat.sync()
    lat.set_launch(mode, 0, 4)
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    out = lat.step(fa, fb, 13)
    lat.sync()
    n = lat.n_nodes
    assert torch.equal(out[:, :n], ref[:, :n])


def test_graph_replays_each_match_eager(torch):
    """Graph replays interleaved with eager work: every replay equals the eager result."""
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    f0 = lat.equilibrium(fl)
    ea, eb = lat.new_state(), lat.new_state()
    ea.copy_(f0)
    ga, gb = lat.new_state(), lat.new_state()
    ga.copy_(f0)
    lat_g, _, _, _, _ = _batch(torch, DRAWS)
    lat_g.set_launch("graph", 0, 4)
    n = lat.n_nodes
    for rep in range(5):
        lat.step(ea, eb, 4)          # eager reference, 4 steps -> back in ea
        lat_g.step(ga, gb, 4)        # one replay of the captured 4 steps
        junk = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
        lat.sync()
        lat_g.sync()
        assert torch.isfinite(junk)
        assert torch.equal(ga[:, :n], ea[:, :n]), rep


def test_batched_shock_matches_oracle_one_step(torch):
    """tau_scale per domain: one step of a two-shock batch against the oracle, per shock."""
    lat, fl, doms, fields, tau = _batch(torch, [(1.3, 40), (2.5, 60)])
    fa = lat.equilibrium(fl)
    n = lat.n_nodes
    fa[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=9), dtype=torch.float32, device="cuda")
    fb = lat.new_state()
    lat.step(fa, fb, 1)
    lat.sync()
    vs = O.make_velocity_set([1, 2, 3], 9)
    f0 = fa.cpu().numpy()
    f1 = fb.cpu().numpy()
    for i, d in enumerate(doms):
        off, nx = lat.domain_offset[i], d["nx"]
        model = O.Model(vs=vs, N=4, tau={k: v * d["tau_scale"] for k, v in tau.items()}, shift=(1, 0, 0))
        dom = O.Domain(nx=nx, bc_x=1, state_in=(d["rho_in"], d["u_in"], d["theta_in"]),
                       state_out=(d["rho_out"], d["u_out"], d["theta_out"]))
        fo = O.step(f0[:, off:off + nx].astype(np.float64).reshape(-1, 1, 1, nx), model, dom)
        g = f1[:, off:off + nx].reshape(fo.shape)
        assert np.abs(g - fo).max() / np.abs(fo).max() < 1e-5, i


@pytest.mark.parametrize("mode,block,lpn", [("direct", 64, 4), ("direct", 256, 4), ("graph", 128, 4),
                                            ("persistent", 64, 4), ("direct", 128, 2), ("persistent", 256, 2),
                                            ("direct", 64, 8), ("graph", 256, 8), ("persistent", 128, 8),
                                            ("direct", 64, 16), ("graph", 256, 16)])
def test_lanes_per_node(torch, mode, block, lpn):
    """lanes_per_node = 2, 4 or 8 (each node's x-slabs split over a group of lanes): 13 steps agree with
    lanes_per_node = 1 to float32 rounding (the FP64 projection sums run in another order), equal
    the direct launch with the same split bitwise, and leave the moment read-out unchanged."""
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    f0 = lat.equilibrium(fl)
    n = lat.n_nodes
    f0[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=21), dtype=torch.float32, device="cuda")
    lat.set_launch("direct", 64, 64, 1)
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 13)
    mom_ref = lat.moments(ref).clone()
    lat.set_launch("direct", block, 64, lpn)
    da, db = lat.new_state(), lat.new_state()
    da.copy_(f0)
    direct4 = lat.step(da, db, 13)
    lat.set_launch(mode, block, 4, lpn)
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    out = lat.step(fa, fb, 13)
    mom = lat.moments(ref)
    lat.sync()
    assert torch.equal(out[:, :n], direct4[:, :n])
    err = float((out[:, :n].double() - ref[:, :n].double()).abs().max() / ref[:, :n].double().abs().max())
    print(f"lanes_per_node {lpn} vs 1 after 13 steps ({mode}, {block}): {err:.2e}")
    assert err < 2e-6
    assert torch.equal(mom, mom_ref)


@pytest.mark.parametrize("lpn", [4, 8, 16])
def test_split_lanes_q729_one_step_matches_oracle(torch, lpn):
    """D3Q729, N = 5 (nine x-slabs over four lanes: 3, 2, 2, 2; over eight: 2, 1, ..., 1; over
    sixteen: one each on nine lanes, none on seven), one step from a perturbed state."""
    draws = [(3.0, 45), (1.5, 70)]
    lat, fl, doms, fields, tau = _batch(torch, draws, ab=(1, 2, 3, 5), deg=11, N=5, k=2)
    lat.set_launch("direct", 128, 64, lpn)
    fa = lat.equilibrium(fl)
    n = lat.n_nodes
    fa[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=23), dtype=torch.float32, device="cuda")
    fb = lat.new_state()
    lat.step(fa, fb, 1)
    lat.sync()
    vs = O.make_velocity_set([1, 2, 3, 5], 11)
    f0 = fa.cpu().numpy()
    f1 = fb.cpu().numpy()
    for i, d in enumerate(doms):
        off, nx = lat.domain_offset[i], d["nx"]
        model = O.Model(vs=vs, N=5, tau={k: v * d["tau_scale"] for k, v in tau.items()}, shift=(2, 0, 0))
        dom = O.Domain(nx=nx, bc_x=1, state_in=(d["rho_in"], d["u_in"], d["theta_in"]),
                       state_out=(d["rho_out"], d["u_out"], d["theta_out"]))
        fo = O.step(f0[:, off:off + nx].astype(np.float64).reshape(-1, 1, 1, nx), model, dom)
        g = f1[:, off:off + nx].reshape(fo.shape)
        err = np.abs(g - fo).max() / np.abs(fo).max()
        print(f"shock {i}: max scaled error {err:.2e}")
        assert err < 1e-5, i


def test_default_lanes_per_node(torch):
    """Shock contexts with FP64 contractions start with 8 lanes per node up to 8192 nodes (16 up to
    4096 for nine or more x-slabs), 4 up to 16384, then 1."""
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    assert lat.launch_settings() == {"mode": "direct", "block": 64, "lanes_per_node": 8}
    mid, _, _, _, _ = _batch(torch, [(1.5, 6000), (2.0, 6000)])
    assert mid.launch_settings() == {"mode": "direct", "block": 256, "lanes_per_node": 4}
    big, _, _, _, _ = _batch(torch, [(1.5, 9000), (2.0, 9000)])
    assert big.launch_settings() == {"mode": "direct", "block": 256, "lanes_per_node": 1}
    # nine x-slabs (D3Q729): sixteen lanes up to 4096 nodes
    q9, _, _, _, _ = _batch(torch, [(3.0, 600)], ab=(1, 2, 3, 5), deg=11, N=5, k=2)
    assert q9.launch_settings()["lanes_per_node"] == 16
    q9b, _, _, _, _ = _batch(torch, [(3.0, 3000), (2.0, 3000)], ab=(1, 2, 3, 5), deg=11, N=5, k=2)
    assert q9b.launch_settings()["lanes_per_node"] == 8


def test_four_lanes_per_node_rejected_where_unsupported(torch):
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd._lib import LbsmrtError
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= 4}
    box = Lattice([1, 2, 3], 9, 4, tau, [dict(nx=8, ny=8, nz=8)], precision="fp64_contract")
    with pytest.raises(LbsmrtError):
        box.set_launch("direct", 64, 64, 4)
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    with pytest.raises(LbsmrtError):
        lat.set_launch("direct", 64, 64, 3)


def _ring_lattice(torch, nxs):
    """Periodic line domains (D3Q343, N = 4, no shift, pull reach 3) from a seeded perturbed
    Maxwellian, in 64-node work-groups."""
    from paper_2401_11086_amd import Lattice
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= 4}
    doms = [dict(nx=n, ny=1, nz=1, bc_x=0) for n in nxs]
    lat = Lattice([1, 2, 3], 9, 4, tau, doms, precision="fp64_contract")
    lat.set_launch("direct", 64, 64, 1)
    n = lat.n_nodes
    fields = np.zeros((5, n))
    x = np.arange(n)
    fields[0] = 1.0 + 0.05 * np.sin(2 * np.pi * x / 37.0)
    fields[1] = 0.1 * np.cos(2 * np.pi * x / 53.0)
    fields[4] = 1.0 + 0.03 * np.sin(2 * np.pi * x / 29.0)
    f0 = lat.equilibrium(torch.tensor(fields, dtype=torch.float64, device="cuda"))
    f0[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=31), dtype=torch.float32, device="cuda")
    return lat, f0


# 320 = five full blocks (per-block progress); 257 = five blocks ending in one node, shorter than
# the reach (grid barrier); 150, 128, 40 = rings of three, two and one block; 259 ends in three
# nodes, as long as the reach (per-block progress) beside rings of four, three and one block
@pytest.mark.parametrize("nxs", [[320], [257], [150, 128, 40], [256, 259, 130, 64]])
def test_persistent_rings_match_direct_bitwise(torch, nxs):
    lat, f0 = _ring_lattice(torch, nxs)
    n = lat.n_nodes
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 17)
    lat.sync()
    lat.set_launch("persistent", 64, 4, 1)
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    for chunk in (5, 7, 5):                      # progress counters carried over calls
        out = lat.step(fa, fb, chunk)
        fa, fb = (out, fb if out is fa else fa)
    lat.sync()
    assert torch.equal(out[:, :n], ref[:, :n])
    lat.close()


def test_persistent_wait_give_up_is_reported(torch):
    """Line batch in the persistent launch: with every wait's target made unreachable from the host
    (and a short poll limit) the launch ends normally and lbsmrt_sync_status reports E_TIMEOUT;
    restored, the next launches match the direct launch bitwise again."""
    from paper_2401_11086_amd import _lib as C
    from paper_2401_11086_amd._lib import LbsmrtError
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    f0 = lat.equilibrium(fl)
    n = lat.n_nodes
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 6)
    lat.sync()
    lat.set_launch("persistent", 64, 4, 8)
    C.check(C.lib().lbsmrt_test_flow_wait(lat._h, 16, 1 << 30), "lbsmrt_test_flow_wait")
    ja, jb = lat.new_state(), lat.new_state()
    ja.copy_(f0)
    lat.step(ja, jb, 3)
    with pytest.raises(LbsmrtError) as e:
        lat.sync()
    assert e.value.status == C.E_TIMEOUT
    lat.sync()                                   # the status was cleared with the report
    C.check(C.lib().lbsmrt_test_flow_wait(lat._h, 1 << 22, 0), "lbsmrt_test_flow_wait")
    assert C.lib().lbsmrt_test_flow_wait(lat._h, 0, 0) == C.E_ARG
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    out = lat.step(fa, fb, 6)
    lat.sync()
    assert torch.equal(out[:, :n], ref[:, :n])


def test_persistent_box_ignores_wait_hook(torch):
    """A periodic box runs the persistent launch with the grid barrier: the wait hook changes nothing."""
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import _lib as C
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= 4}
    box = Lattice([1, 2, 3], 9, 4, tau, [dict(nx=16, ny=8, nz=8)], precision="fp64_contract")
    f0 = box.equilibrium(torch.tensor(_box_fields(16, 8, 8), dtype=torch.float64, device="cuda"))
    ra, rb = box.new_state(), box.new_state()
    ra.copy_(f0)
    ref = box.step(ra, rb, 4)
    box.sync()
    box.set_launch("persistent", 0, 4)
    C.check(C.lib().lbsmrt_test_flow_wait(box._h, 16, 1 << 30), "lbsmrt_test_flow_wait")
    fa, fb = box.new_state(), box.new_state()
    fa.copy_(f0)
    out = box.step(fa, fb, 4)
    box.sync()
    assert torch.equal(out, ref)


def _box_fields(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = np.zeros((5, nz, ny, nx))
    f[0] = 1.0 + 0.05 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)
    f[1] = 0.08 * np.sin(2 * np.pi * z / nz)
    f[2] = 0.05 * np.cos(2 * np.pi * x / nx)
    f[4] = 1.0 + 0.02 * np.cos(2 * np.pi * (x / nx + z / nz))
    return f.reshape(5, -1)


@pytest.mark.parametrize("block,lpn", [(64, 8), (128, 1)])
def test_persistent_q729_shocks_match_direct_bitwise(torch, block, lpn):
    """D3Q729 (N = 5, shift 2: pull reach 7) shock batch in the persistent launch with per-block
    progress, from a perturbed state: bitwise equal to direct launches after 11 steps."""
    lat, fl, doms, fields, tau = _batch(torch, [(3.0, 45), (1.5, 70), (4.5, 33)], ab=(1, 2, 3, 5), deg=11, N=5, k=2)
    lat.set_launch("direct", block, 64, lpn)
    f0 = lat.equilibrium(fl)
    n = lat.n_nodes
    f0[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=29), dtype=torch.float32, device="cuda")
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 11)
    lat.sync()
    lat.set_launch("persistent", block, 4, lpn)
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    out = lat.step(fa, fb, 11)
    lat.sync()
    assert torch.equal(out[:, :n], ref[:, :n])
    lat.close()


def test_persistent_interleaved_with_direct_launches(torch):
    """Persistent launches on a shock batch, then direct ones, then persistent again (the progress
    tables rebuilt): 5 + 4 + 6 steps bitwise equal to 15 direct steps."""
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    f0 = lat.equilibrium(fl)
    n = lat.n_nodes
    f0[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=33), dtype=torch.float32, device="cuda")
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 15)
    lat.sync()
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    cur, other = fa, fb
    for mode, k in (("persistent", 5), ("direct", 4), ("persistent", 6)):
        lat.set_launch(mode, 64, 4, 8)
        out = lat.step(cur, other, k)
        cur, other = (out, other if out is cur else cur)
    lat.sync()
    assert torch.equal(cur[:, :n], ref[:, :n])
    lat.close()


def test_sixteen_lanes_refused_for_the_persistent_launch(torch):
    from paper_2401_11086_amd._lib import LbsmrtError
    lat, fl, doms, fields, tau = _batch(torch, DRAWS)
    lat.set_launch("direct", 64, 4, 16)
    with pytest.raises(LbsmrtError):
        lat.set_launch("persistent", 64, 4, 0)
    with pytest.raises(LbsmrtError):
        lat.set_launch("persistent", 64, 4, 16)
    lat.set_launch("persistent", 64, 4, 8)


def test_persistent_mixed_tubes_and_rings_match_direct_bitwise(torch):
    """A shock context holding tubes and periodic rings (eight lanes per node, 8-node blocks):
    the persistent launch with per-block progress equals direct launches bitwise after 12 steps."""
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = solve_quadrature([1, 2, 3], 9)
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= 4}
    d1, f1, _ = shock_domain(1.5, 70, c_l)
    d2, f2, _ = shock_domain(2.2, 45, c_l)
    rings = [dict(nx=64, ny=1, nz=1, bc_x=0), dict(nx=37, ny=1, nz=1, bc_x=0)]
    ring_fields = []
    for r in rings:
        x = np.arange(r["nx"])
        g = np.zeros((5, r["nx"]))
        g[0] = 1.0 + 0.04 * np.sin(2 * np.pi * x / r["nx"])
        g[1] = c_l * 1 + 0.05 * np.cos(2 * np.pi * x / r["nx"])    # around the frame velocity k = 1
        g[4] = 1.0
        ring_fields.append(g)
    doms = [d1, rings[0], d2, rings[1]]
    lat = Lattice([1, 2, 3], 9, 4, tau, doms, shift_k=(1, 0, 0), precision="fp64_contract")
    fl = torch.tensor(np.concatenate([f1, ring_fields[0], f2, ring_fields[1]], axis=1), dtype=torch.float64,
                      device="cuda")
    lat.set_launch("direct", 64, 4, 8)
    f0 = lat.equilibrium(fl)
    n = lat.n_nodes
    f0[:, :n] *= torch.tensor(W.state_noise((lat.Q, n), seed=37), dtype=torch.float32, device="cuda")
    ra, rb = lat.new_state(), lat.new_state()
    ra.copy_(f0)
    ref = lat.step(ra, rb, 12)
    lat.sync()
    lat.set_launch("persistent", 64, 4, 8)
    fa, fb = lat.new_state(), lat.new_state()
    fa.copy_(f0)
    out = lat.step(fa, fb, 12)
    lat.sync()
    assert torch.equal(out[:, :n], ref[:, :n])
    lat.close()
