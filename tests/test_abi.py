"""The C-ABI library loads, exports every declared entry point, and its host
helpers agree with the oracle (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "lbsmrt.h")).read()
    return sorted(set(re.findall(r"\b(lbsmrt_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2401_11086_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblbsmrt.so not built: run __graft_entry__.build()")
    return _lib


def test_library_exports_every_declared_symbol(lib):
    L = lib.lib()
    declared = _declared_symbols()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert set(lib.EXPORTED) == set(declared)


@pytest.mark.parametrize("ab,deg", [([1, 2, 3], 9), ([1, 2, 3, 5], 11), ([1, 2, 3, 4, 5, 6, 7, 9], 19)])
def test_library_quadrature_matches_oracle(lib, ab, deg):
    r, w = lib.solve_quadrature(ab, deg)
    ro, wo = O.solve_d1_quadrature(ab, deg)
    assert abs(r - ro) < 1e-13
    assert np.allclose(w, wo, rtol=1e-12, atol=1e-16)


def test_library_rejects_infeasible_stencil(lib):
    with pytest.raises(lib.LbsmrtError) as e:
        lib.solve_quadrature([1, 2, 3, 4], 11)
    assert e.value.status == lib.E_QUADRATURE
    with pytest.raises(lib.LbsmrtError) as e:
        lib.solve_quadrature([2, 1], 9)
    assert e.value.status == lib.E_ARG


@pytest.mark.parametrize("Ma,th1", [(1.5, 0.714), (3.0, 0.333), (5.0, 0.167), (7.0, 0.071)])
def test_library_shock_states_match_oracle(lib, Ma, th1):
    s = lib.shock_states(Ma, theta1=th1, c_l=0.6780039063343388)
    o = O.rankine_hugoniot(Ma, theta1=th1)
    for k in ("rho2", "u1", "u2", "theta2", "u_mid"):
        assert abs(s[k] - o[k]) < 1e-13 * max(1, abs(o[k]))
    assert int(s["k"]) == O.shift_integer(o["u_mid"], 0.6780039063343388)


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2401_11086_amd import Lattice
    with pytest.raises(RuntimeError):
        Lattice([1, 2, 3], 9, 4, {(2, 0): 1.0}, [dict(nx=4)])


def test_compiled_tap_tables_are_current(lib):
    """The compile-time FP64 tap tables of the moment-state kernels (ms_std_tables.hpp) hold
    exactly what their generator computes from the library's quadrature, and they satisfy the
    quadrature identity sum_e He_b(c_e) w_e He_a(c_e) / a! = delta_ab for a, b <= N (the
    quadrature is exact to degree 2N) to FP64 rounding, which the conservation of the
    moment-state step rests on."""
    import importlib.util
    path = os.path.join(ROOT, "paper_2401_11086_amd", "csrc")
    spec = importlib.util.spec_from_file_location("gen_ms_std_tables", os.path.join(path, "gen_ms_std_tables.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    text = open(os.path.join(path, "ms_std_tables.hpp")).read()
    for q1, N in ((7, 4), (9, 5)):
        he, rw = gen.table(q1)
        block = text[text.index(f"struct MsStdTables<{q1}>"):]
        for name, ref in (("He", he), ("Rw", rw)):
            m = re.search(name + r"\[\d+\]\[\d+\] = \{(.*?)\};\n", block)
            vals = [float.fromhex(v) for v in re.findall(r"-?0x[0-9a-f.]+p[+-]\d+", m.group(1))]
            assert vals == [v for row in ref for v in row], (q1, name)
        p = len(gen.STENCILS[q1][0])
        for b in range(N + 1):
            for a in range(N + 1):
                s = he[0][b] * rw[0][a] + sum((1 + (-1) ** (a + b)) * he[t][b] * rw[t][a] for t in range(1, p + 1))
                assert abs(s - (1.0 if a == b else 0.0)) < 1e-13, (q1, b, a, s)
