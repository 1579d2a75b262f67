"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/svdp.h declares, and its host-only entry points (defaults,
workspace sizing, argument validation, the CANS coefficient scheduler) behave
as documented.  The scheduler is compared with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2609_32505_amd import _lib as L
    return L, L.load()


def _declared():
    with open(os.path.join(ROOT, "include", "svdp.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src))
    keywords = {"if", "for", "while", "sizeof", "return", "defined"}
    return sorted(n for n in names if n not in keywords and (n.startswith("svd") or n.startswith("polar")))


def test_header_functions_are_exported():
    L, lib = _lib()
    names = _declared()
    assert "svd_polar_fwd" in names and "polar_bwd" in names and len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in svdp.h but not exported"
        assert n in L.SIGNATURES, f"{n} has no ctypes signature in the binding"


def test_params_struct_matches_header_layout():
    L, lib = _lib()
    # the binding's struct must have the header's field order: defaults land
    # in the right fields
    p = L.default_params(3, 20, 10)
    assert (p.batch, p.m, p.n) == (3, 20, 10)
    assert (p.max_iters, p.pre_iters, p.refine_steps) == (50, 2, 2)
    assert p.delta == 0.99 and p.tol == 1e-5 and p.eps_qr == 1e-5
    assert p.jacobi_tol == 3e-3 and p.bf16_from == 0.2
    assert p.margin_max == 1.1 and p.margin_min == 1.0
    assert p.eps_K == 0.0 and p.user_bounds is None and p.probe is None
    assert p.eigh_off_tol == 6e-6 and p.eigh_restarts == 2 and p.jacobi_fro_tol == 3e-4 and p.poly == 0
    assert p.bf16_correct == 1


def _ws(p, op):
    L, lib = _lib()
    out = ctypes.c_size_t()
    st = lib.svdp_workspace_size(ctypes.byref(p), op, ctypes.byref(out))
    return st, out.value


def test_workspace_size_and_shape_validation():
    L, _ = _lib()
    st, nb = _ws(L.default_params(256, 512, 512), L.OP_SVD_FWD)
    assert st == 0 and nb > 4 * 256 * 512 * 512 * 4
    st2, nb2 = _ws(L.default_params(256, 512, 512), L.OP_SVD_BWD)
    assert st2 == 0 and 0 < nb2 < nb
    assert _ws(L.default_params(1, 4, 8), L.OP_SVD_FWD)[0] == 2          # m < n
    assert _ws(L.default_params(1, 8, 0), L.OP_SVD_FWD)[0] == 2          # n < 1
    assert _ws(L.default_params(70000, 8, 8), L.OP_SVD_FWD)[0] == 2      # batch too large
    assert _ws(L.default_params(1, 9000, 8193), L.OP_SVD_FWD)[0] == 2    # n too large
    assert _ws(L.default_params(1, 8, 8), 99)[0] == 1                    # unknown op
    assert _ws(L.default_params(1, 8, 8, max_iters=65), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, delta=1.5), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, precision=7), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, eigh_restarts=9), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, eigh_off_tol=-1.0), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, jacobi_fro_tol=-1.0), 0)[0] == 1
    assert _ws(L.default_params(0, 8, 8), L.OP_SVD_FWD)[0] == 0
    # divide and conquer: one matrix's worth (polar step, six n x n buffers and
    # the eigensolver's), independent of the batch
    st3, nb3 = _ws(L.default_params(1, 1024, 1024), L.OP_EIGH_DC)
    st4, nb4 = _ws(L.default_params(1, 1024, 1024), L.OP_EIGH)
    assert st3 == 0 and st4 == 0 and nb3 > nb4 + 6 * 1024 * 1024 * 4
    assert _ws(L.default_params(8, 1024, 1024), L.OP_EIGH_DC)[1] - nb3 < 1024
    # a single FP32 matrix from n = 2048 takes the SVD's EVD step by divide
    # and conquer: its forward workspace holds that solver's, which polar_fwd's,
    # the BF16 path's and a batch's do not
    one = _ws(L.default_params(1, 2048, 2048), L.OP_SVD_FWD)[1]
    dcw = _ws(L.default_params(1, 2048, 2048), L.OP_EIGH_DC)[1]
    assert one >= dcw + _ws(L.default_params(1, 2048, 2048), L.OP_POLAR_FWD)[1]
    assert _ws(L.default_params(1, 2048, 2048, precision=1), L.OP_SVD_FWD)[1] < one - dcw // 2
    assert _ws(L.default_params(2, 2048, 2048), L.OP_SVD_FWD)[1] < 2 * one - dcw
    assert _ws(L.default_params(1, 2047, 2047), L.OP_SVD_FWD)[1] < one - dcw // 2


def test_status_strings():
    L, lib = _lib()
    for code in range(6):
        assert lib.svdp_status_string(code).decode() == L.STATUS[code]


def test_null_handle_is_rejected_before_any_launch():
    L, lib = _lib()
    p = L.default_params(1, 8, 8)
    st = lib.svd_polar_fwd(None, ctypes.byref(p), 0, 8, 64, 0, 8, 64, 0, 8, 0, 8, 64, None, None, 0, None)
    assert st == 1
    assert "null" in lib.svdp_last_error().decode()


@pytest.mark.parametrize("delta,pre", [(0.99, 2), (0.9, 2), (0.999, 1)])
def test_conservative_schedule_matches_oracle(orc, delta, pre):
    from paper_2609_32505_amd import api
    tab, t = api.cans_table(0, 50, delta=delta, pre_iters=pre)
    ref = orc.cans_schedule_conservative(delta, pre, 50)
    np.testing.assert_allclose(tab, ref, rtol=1e-13, atol=1e-13)
    assert t == pytest.approx(orc.cans_preprocess_t(delta, pre), rel=1e-12)


@pytest.mark.parametrize("poly", [0, 1, 2])
@pytest.mark.parametrize("delta,pre", [(0.99, 2), (0.9, 1), (0.999, 3)])
def test_poly_table_matches_oracle(orc, poly, delta, pre):
    # the host Remez exchange (quintic) against the oracle's nonlinear solve
    # of the equioscillation system.  Where the interval is so narrow that the
    # minimax error nears FP64 rounding (E < 1e-12) the coefficients are no
    # longer determined by the problem, so each step is compared by what it
    # must achieve: its maximum error on the oracle's interval.
    from paper_2609_32505_amd import api
    tab, t = api.poly_table(poly, 40, delta=delta, pre_iters=pre)
    ref, t_ref = orc.poly_schedule_conservative(poly, delta, pre, 40)
    assert t == pytest.approx(t_ref, rel=1e-9, abs=0.0)
    if poly != 2:
        np.testing.assert_allclose(tab, ref, rtol=1e-12, atol=1e-13)
        return
    a, b = t_ref, 1.0
    for k in range(40):
        if k == pre:
            a, b = 1.0 - delta, 1.0 + delta
        c1, c3, c5, lo, hi = orc.cans5_poly(a, b)
        E = (hi - lo) / 2
        x = np.linspace(a, b, 20001)
        e_host = np.abs(1.0 - (tab[k, 0] * x + tab[k, 1] * x ** 3 + tab[k, 2] * x ** 5)).max()
        assert e_host <= E * (1 + 1e-6) + 1e-15, k
        if E > 1e-12:
            np.testing.assert_allclose(tab[k], ref[k], rtol=1e-7)
        a, b = lo, hi


def test_workspace_covers_quintic_buffer():
    # the quintic step needs one n x n buffer per matrix (P = c3 G + c5 G^2)
    L, _ = _lib()
    st0, nb0 = _ws(L.default_params(4, 300, 200), L.OP_SVD_FWD)
    st2, nb2 = _ws(L.default_params(4, 300, 200, poly=2), L.OP_SVD_FWD)
    assert st0 == 0 and st2 == 0 and nb2 - nb0 >= 0.99 * 4 * 200 * 200 * 4


def test_poly_argument_errors():
    L, lib = _lib()
    assert _ws(L.default_params(1, 8, 8, poly=4), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, poly=2, bound=1), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, poly=1, precision=1), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, poly=2), 0)[0] == 0


def test_bf16_correct_argument():
    L, lib = _lib()
    assert _ws(L.default_params(1, 8, 8, bf16_correct=2), 0)[0] == 1
    assert _ws(L.default_params(1, 8, 8, bf16_correct=0), 0)[0] == 0


@pytest.mark.parametrize("lo", [1e-6, 1e-3, 0.2, 1.0])
def test_interval_schedule_matches_oracle(orc, lo):
    from paper_2609_32505_amd import api
    tab, _ = api.cans_table(1, 30, lo=lo)
    ref, _ = orc.cans_schedule_interval(lo, 30)
    np.testing.assert_allclose(tab, ref, rtol=1e-13, atol=1e-13)


def test_schedule_argument_errors():
    L, lib = _lib()
    tab = (ctypes.c_double * 8)()
    assert lib.svdp_cans_table(0, 1.5, 2, 0.0, 4, tab, None) == 1
    assert lib.svdp_cans_table(1, 0.99, 2, 0.0, 4, tab, None) == 1
    assert lib.svdp_cans_table(2, 0.99, 2, 0.1, 4, tab, None) == 1
    assert lib.svdp_cans_table(1, 0.99, 2, 0.1, 4, None, None) == 1


def test_bench_refuses_more_than_one_gpu():
    # one GPU per box: --gpus N > 1 exits with a message before touching a GPU
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("lo", [1e-3, 1e-7, 0.3])
def test_pe_table_matches_oracle(orc, lo):
    # the host Remez exchange and exact interval images against the oracle's
    # equioscillation solve and grid images: same step count, each step's
    # polynomial as good as the oracle's on the oracle's cushioned interval
    from paper_2609_32505_amd import api
    tab = api.pe_table(lo)
    ref = orc.polar_express_schedule(lo)
    assert tab.shape == ref.shape
    # each step's polynomial against the oracle's on the oracle's interval: the
    # coefficients of a very narrow interval are not determined to FP64 by the
    # problem (the minimax error nears rounding), the values are
    l, u = lo, 1.0
    for k in range(len(ref)):
        last = k == len(ref) - 1
        f = 1.0 if last else 1.01
        x = np.linspace(l / f, u / f, 20001)
        ph = tab[k, 0] * x + tab[k, 1] * x ** 3 + tab[k, 2] * x ** 5
        pr = ref[k, 0] * x + ref[k, 1] * x ** 3 + ref[k, 2] * x ** 5
        assert np.abs(ph - pr).max() < 1e-8, k
        if u - l > 1e-3:
            np.testing.assert_allclose(tab[k], ref[k], rtol=1e-8)
        l, u = pr.min(), pr.max()


def test_pe_argument_errors():
    L, lib = _lib()
    tab = (ctypes.c_double * 192)()
    steps = ctypes.c_int32()
    assert lib.svdp_pe_table(0.0, 64, tab, ctypes.byref(steps)) == 1
    assert lib.svdp_pe_table(1e-3, 3, tab, ctypes.byref(steps)) == 1   # needs 8 steps
    assert lib.svdp_pe_table(1e-3, 8, tab, ctypes.byref(steps)) == 0 and steps.value == 8
    p = L.default_params(2, 10, 10, poly=L.POLY_PE, pe_lo=0.0)
    st, _ = _ws(p, L.OP_SVD_FWD)
    assert st == 1
    p = L.default_params(2, 10, 10, poly=L.POLY_PE, pe_lo=1e-3, precision=L.PREC_BF16)
    st, _ = _ws(p, L.OP_SVD_FWD)
    assert st == 1
