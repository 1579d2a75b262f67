"""The allocation-free backward (svd_polar_bwd_noalloc) against the
allocating svd_polar_bwd through the C ABI: same factors and gradients, two
calls in a row (the second with a smaller batch and shape), and the size
check of its static scratch."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2609_32505_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(L, h, p, U, S, V, dU, dS, dV, dA, stream):
    b, m, n = U.shape
    return L.load().svd_polar_bwd_noalloc(h.ptr, ctypes.byref(p), U.data_ptr(), n, m * n, S.data_ptr(), n,
                                          V.data_ptr(), n, n * n, dU.data_ptr(), n, m * n, dS.data_ptr(), n,
                                          dV.data_ptr(), n, n * n, dA.data_ptr(), n, m * n, stream)


def test_noalloc_backward_matches_workspace_backward():
    import torch
    from paper_2609_32505_amd import _lib as L, api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = api.Handle()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for call, (b, m, n, seed) in enumerate([(24, 256, 256, 201), (5, 150, 100, 202)]):
        _say(f"call {call}: {b} x {m} x {n}")
        A, _ = inputs.batch_with_spectra(seed, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-2, 1.0))
        rng = inputs.rng_for(seed, 7)
        dU, dS, dV = (torch.from_numpy(x.astype(np.float32)).cuda() for x in
                      (rng.standard_normal((b, m, n)), rng.standard_normal((b, n)), rng.standard_normal((b, n, n))))
        U, S, V, _ = api.svd_fwd(torch.from_numpy(A).cuda(), handle=h)
        eps = dict(eps_K=1e-8, eps_R=1e-6, eps_T=1e-4)
        ref = api.svd_bwd(U, S, V, dU, dS, dV, handle=h, **eps)
        p = L.default_params(b, m, n, **eps)
        dA = torch.full((b, m, n), float("nan"), device="cuda")
        st = _noalloc(L, h, p, U, S, V, dU, dS, dV, dA, stream)
        assert st == 0, L.load().svdp_last_error().decode()
        torch.cuda.synchronize()
        diff = (dA - ref).abs().max().item()
        scale = ref.abs().max().item()
        _say(f"  max |noalloc - workspace| = {diff:.3e} (|dA| max {scale:.3e})")
        assert torch.isfinite(dA).all() and diff <= 1e-6 * scale
    # beyond the static scratch: a clear error from the host-side size check,
    # before any launch (the pointers name a small live buffer, never read)
    p = L.default_params(2000, 512, 512)
    t = torch.zeros(16, device="cuda")
    q = t.data_ptr()
    st = L.load().svd_polar_bwd_noalloc(h.ptr, ctypes.byref(p), q, 512, 512 * 512, q, 512, q, 512, 512 * 512,
                                        None, 512, 512 * 512, None, 512, None, 512, 512 * 512, q, 512, 512 * 512,
                                        stream)
    msg = L.load().svdp_last_error().decode()
    _say(f"  oversized batch: status {st}, '{msg}'")
    assert st == 3 and "scratch" in msg
