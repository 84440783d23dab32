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


def _decimal_rule(ab, deg, digits=60):
    """The positive-weight rule to `digits` decimal digits: bisection on r of the top even-moment
    residual, the weights from the lower moments by Gaussian elimination, all in Decimal (no
    float step, no library call)."""
    from decimal import Decimal as D, localcontext
    with localcontext() as ctx:
        ctx.prec = digits
        n, k_top = len(ab) + 1, len(ab) + 1
        dfact = [D(1)]
        for k in range(1, k_top + 1):
            dfact.append(dfact[-1] * (2 * k - 1))

        def weights(r):
            A = [[D(1 if k == 0 else 0)] + [2 * (D(a) * r) ** (2 * k) for a in ab] for k in range(n)]
            b = dfact[:n]
            for c in range(n):
                piv = max(range(c, n), key=lambda i: abs(A[i][c]))
                A[c], A[piv], b[c], b[piv] = A[piv], A[c], b[piv], b[c]
                for i in range(c + 1, n):
                    f = A[i][c] / A[c][c]
                    A[i] = [A[i][j] - f * A[c][j] for j in range(n)]
                    b[i] -= f * b[c]
            w = [D(0)] * n
            for i in range(n - 1, -1, -1):
                w[i] = (b[i] - sum(A[i][j] * w[j] for j in range(i + 1, n))) / A[i][i]
            return w

        def res(r):
            w = weights(r)
            return sum(2 * w[j + 1] * (D(a) * r) ** (2 * k_top) for j, a in enumerate(ab)) - dfact[k_top]

        r0 = D(repr(O.solve_d1_quadrature(ab, deg)[0]))      # bracket the oracle's root
        lo, hi = r0 * (1 - D("1e-9")), r0 * (1 + D("1e-9"))
        flo = res(lo)
        assert (flo < 0) != (res(hi) < 0)
        for _ in range(160):
            mid = (lo + hi) / 2
            fm = res(mid)
            if (fm < 0) == (flo < 0):
                lo, flo = mid, fm
            else:
                hi = mid
        r = (lo + hi) / 2
        return r, weights(r)


@pytest.mark.parametrize("ab,deg", [([1, 2, 3], 9), ([1, 2, 3, 5], 11), ([1, 2, 3, 4, 5, 6, 7, 9], 19)])
def test_library_quadrature_is_correctly_rounded(lib, ab, deg):
    """r and every weight equal the 60-digit rule rounded to double (the library bisects and
    solves in binary128, with basic operations only, so the rule is also the same on every host)."""
    r, w = lib.solve_quadrature(ab, deg)
    rd, wd = _decimal_rule(ab, deg)
    assert r == float(rd), (r, float(rd))
    assert list(w) == [float(x) for x in wd], (list(w), [float(x) for x in wd])


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
    for q1, N in ((7, 4), (9, 5), (17, 5)):
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
