"""Host-side logic of the package that runs without a GPU: relaxation presets against Table 4,
the seeded input generators, the shock set-up, the autotuner's candidate list, the adjoint's
tau ordering and bench.py's traffic record.  (Shock states come from the library's host helper,
so the built library must be present, as for test_abi.py.)"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_smrt_and_shakhov_presets_are_table4():
    from paper_2401_11086_amd.presets import SHAKHOV, SMRT
    for model, n, m, t in _rows("table4_relaxation.txt"):
        table = SMRT if model == "SMRT" else SHAKHOV
        assert table[(int(n), int(m))] == Fraction(t), (model, n, m)


def test_derived_presets():
    from paper_2401_11086_amd.presets import BGK, LUMPED, REDUCED, SMRT, tau_table
    assert all(v == 1 for v in BGK.values())
    assert REDUCED[(4, 1)] == REDUCED[(4, 2)] == Fraction(6, 7)
    assert {k: v for k, v in REDUCED.items() if k not in ((4, 1), (4, 2))} == \
        {k: v for k, v in SMRT.items() if k not in ((4, 1), (4, 2))}
    for n in range(2, 6):                                  # one time per order
        assert len({v for (nn, _), v in LUMPED.items() if nn == n}) == 1
    assert LUMPED[(3, 0)] == Fraction(3, 2)                # keeps Pr = 2/3
    t = tau_table("smrt", 2.5, N=4)
    assert set(t) == {(2, 0), (3, 0), (3, 1), (4, 0), (4, 1), (4, 2)}
    assert t[(4, 0)] == pytest.approx(2.5 * 432 / 763)


def test_mach_sweep_is_seeded_and_in_range():
    from paper_2401_11086_amd import workloads as W
    a = W.mach_sweep(64, seed=0)
    b = W.mach_sweep(64, seed=0)
    c = W.mach_sweep(64, seed=1)
    assert a == b and a != c and len(a) == 64
    assert all(1.2 <= Ma <= 5.0 and 400 <= nx <= 2000 and int(nx) == nx for Ma, nx in a)


def test_fourier_modes_and_box():
    from paper_2401_11086_amd import workloads as W
    ks, ph, amp = W.fourier_modes(seed=0)
    norms = np.sqrt((ks ** 2).sum(axis=-1))
    assert ks.shape == (5, 16, 3) and norms.min() >= 1.0 and norms.max() <= 8.0
    assert np.all((ph >= 0) & (ph < 2 * np.pi)) and amp == pytest.approx(0.05 / 4)
    f = W.fourier_box(24, rho0=1.3, theta0=0.8)
    # every mode has a non-zero integer wave-vector below the Nyquist index: zero mean on the box
    assert f[0].mean() == pytest.approx(1.3, abs=1e-12)
    assert f[4].mean() == pytest.approx(0.8, abs=1e-12)
    assert np.abs(f[1:4].mean(axis=1)).max() < 1e-12
    assert np.abs(f[0] / 1.3 - 1).max() <= 16 * amp + 1e-12


def test_fourier_box_torch_matches_numpy():
    import torch
    from paper_2401_11086_amd import workloads as W
    a = W.fourier_box(12, rho0=1.1, theta0=0.9, seed=3)
    b = W.fourier_box_torch(12, "cpu", rho0=1.1, theta0=0.9, seed=3).numpy()
    assert np.abs(a - b).max() < 1e-13
    del torch


def test_tanh_profile_joins_the_end_states():
    from paper_2401_11086_amd import workloads as W
    f = W.tanh_profile(200, (1.0, 1.5, 0.7), (2.0, 0.75, 1.1))
    assert f.shape == (5, 200)
    assert f[0, 0] == pytest.approx(1.0, abs=1e-8) and f[0, -1] == pytest.approx(2.0, abs=1e-8)
    assert f[1, 0] == pytest.approx(1.5, abs=1e-8) and f[4, -1] == pytest.approx(1.1, abs=1e-8)
    assert np.all(f[2:4] == 0.0)
    assert f[0, 100] == pytest.approx(1.5)                 # centre of the blend


def test_theta2_interpolates_table3():
    from paper_2401_11086_amd.shocks import theta2_for
    rows = {float(r[0]): float(r[6]) for r in _rows("table3_implementation.txt")}
    for Ma in (1.5, 3.0, 5.0):
        assert theta2_for(Ma) == pytest.approx(rows[Ma])
    assert theta2_for(1.2) == pytest.approx(rows[1.5])
    assert theta2_for(2.25) == pytest.approx(0.5 * (rows[1.5] + rows[3.0]))
    assert theta2_for(9.0) == pytest.approx(rows[5.0])


def test_shock_domain_set_up():
    from paper_2401_11086_amd import solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    c_l, _ = solve_quadrature([1, 2, 3, 5], 11)
    dom, fields, st = shock_domain(3.0, 600, c_l)
    assert dom["bc_x"] == 1 and dom["nx"] == 600 and dom["ny"] == dom["nz"] == 1
    assert dom["tau_scale"] == pytest.approx(2 * c_l / math.sqrt(st["theta1"]))   # cells of l1 / 2
    assert dom["rho_in"] * dom["u_in"][0] == pytest.approx(dom["rho_out"] * dom["u_out"][0], rel=1e-12)
    assert fields[0, 0] == pytest.approx(st["rho1"], rel=1e-6) and fields[0, -1] == pytest.approx(st["rho2"], rel=1e-6)


def test_adjoint_tau_keys():
    from paper_2401_11086_amd.adjoint import tau_keys
    assert tau_keys(4) == [(2, 0), (3, 0), (3, 1), (4, 0), (4, 1), (4, 2)]
    assert len(tau_keys(5)) == 9 and (2, 1) not in tau_keys(5)


class _FakeLattice:
    def __init__(self, domains, precision):
        self.domains, self.precision = domains, precision


def test_autotune_candidates():
    from paper_2401_11086_amd.autotune import CANDIDATES, _candidates
    box = _FakeLattice([dict(nx=8, ny=8, nz=8)], "fp64_contract")
    tube32 = _FakeLattice([dict(nx=80, bc_x=1)], "fp32")
    tube64 = _FakeLattice([dict(nx=80, bc_x=1)], "fp64_contract")
    assert {c[2] for c in _candidates(box)} == {1}
    assert {c[2] for c in _candidates(tube32)} == {1}
    assert {c[2] for c in _candidates(tube64)} == {1, 2, 4, 8, 16}
    assert not any(c[0] == "persistent" and c[2] == 16 for c in _candidates(tube64))
    assert len(_candidates(tube64)) == len(CANDIDATES) == 42


def test_autotune_key_separates_geometries(monkeypatch):
    """A tuned choice for shock tubes must not be replayed on periodic domains of the same size
    (nor across domain shapes or collision forms)."""
    import types

    import paper_2401_11086_amd.autotune as A
    monkeypatch.setattr(A.torch.cuda, "get_device_properties", lambda dev: types.SimpleNamespace(
        name="gfx950", gcnArchName="gfx950"))

    def fake(domains, precision="fp64_contract", regularized=True):
        lat = _FakeLattice(domains, precision)
        lat.device, lat.Q, lat.N, lat.regularized = 0, 729, 5, regularized
        lat.n_nodes = sum(d["nx"] * d.get("ny", 1) * d.get("nz", 1) for d in domains)
        return lat
    tubes = fake([dict(nx=600, bc_x=1), dict(nx=424, bc_x=1)])
    rings = fake([dict(nx=600, bc_x=0), dict(nx=424, bc_x=0)])
    other = fake([dict(nx=500, bc_x=1), dict(nx=524, bc_x=1)])
    add = fake([dict(nx=600, bc_x=1), dict(nx=424, bc_x=1)], regularized=False)
    keys = {A._key(x) for x in (tubes, rings, other, add)}
    assert len(keys) == 4
    assert A._key(tubes) == A._key(fake([dict(nx=600, bc_x=1), dict(nx=424, bc_x=1)]))


def test_bench_traffic_record_is_keyed_by_sources(tmp_path, monkeypatch):
    import bench
    digest = bench.kernel_source_digest()
    assert len(digest) == 64 and digest == bench.kernel_source_digest()
    rec = tmp_path / "t.md"
    rec.write_text("- workload: box256_q343_n4\n"
                   f"- traffic_bytes_per_launch[fp64_contract]: 4.6e10\n- source_sha256: {digest}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(rec))
    assert bench.recorded_traffic("box256_q343_n4", "fp64_contract") == 4.6e10
    assert bench.recorded_traffic("box256_q343_n4", "fp32") is None
    rec.write_text(rec.read_text().replace(digest, "0" * 64))
    assert bench.recorded_traffic("box256_q343_n4", "fp64_contract") is None


def test_truncation_crossing_interpolates():
    from paper_2401_11086_amd.truncation import _crossing
    x = np.arange(50, dtype=float)
    rho_hat = np.clip((x - 10.3) / 20.0, 0.0, 1.0)      # reaches 1/2 at x = 20.3
    assert _crossing(rho_hat) == pytest.approx(20.3)


def test_bench_moment_state_bytes():
    import bench

    class _L:
        N, M = 4, 35
    b = bench.moment_state_bytes(_L)
    # 35 moment fields and 75 = 5 * 15 intermediate fields per node, FP32
    assert b == {"pass_z": 4.0 * 110, "pass_y": 8.0 * 75, "pass_x_collide": 4.0 * 110}
    assert sum(b.values()) == 1480.0
