"""Torch-facing wrappers of the C ABI: tensors in, tensors out.

PyTorch only provides device memory (outputs and the workspace) and the
current stream; every computation runs in ``libsvdp.so``.  All tensors are
CUDA float32, contiguous, batched as (batch, rows, cols) (a 2-D input is a
batch of one).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, load

_handles: dict = {}


class Handle:
    """Owns a library handle (predictor model + pinned read-back word)."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(load().svdp_create(ctypes.byref(h)), "svdp_create")
        self.ptr = h.value
        self.has_model = False

    def set_model(self, model: np.ndarray):
        model = np.ascontiguousarray(model, dtype=np.float32)
        if model.size != _lib.MODEL_FLOATS:
            raise ValueError(f"model must hold {_lib.MODEL_FLOATS} floats")
        check(load().svdp_set_model(self.ptr, model.ctypes.data), "svdp_set_model")
        self.has_model = True

    def __del__(self):
        try:
            if self.ptr:
                load().svdp_destroy(self.ptr)
        except Exception:
            pass


def default_handle(device=None) -> Handle:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    if dev not in _handles:
        with torch.cuda.device(dev):
            _handles[dev] = Handle()
    return _handles[dev]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else t.data_ptr()


def _req(t, name, ndim=None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{name} must be a CUDA float32 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _batched(t):
    return t if t.dim() == 3 else t.unsqueeze(0)


def _workspace(p, op, device):
    nbytes = ctypes.c_size_t()
    check(load().svdp_workspace_size(ctypes.byref(p), op, ctypes.byref(nbytes)), "workspace_size")
    return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=device)


def _info_tensor(batch, device):
    return torch.zeros((batch, 4), dtype=torch.int32, device=device)


def info_to_numpy(info: torch.Tensor) -> dict:
    """Split the (batch, 4) info records into named numpy arrays."""
    raw = info.cpu().numpy()
    return {"iters": raw[:, 0].copy(), "sweeps": raw[:, 1].copy(), "flags": raw[:, 2].copy(),
            "residual": raw[:, 3].copy().view(np.float32)}


def params(batch, m, n, **kw) -> _lib.Params:
    return _lib.default_params(batch, m, n, **kw)


def _prep_params(p, kw, batch, m, n, probe=None, user_bounds=None):
    if p is None:
        p = params(batch, m, n, **kw)
    else:
        p.batch, p.m, p.n = batch, m, n
    if probe is not None:
        p.probe = probe.data_ptr()
    if user_bounds is not None:
        p.user_bounds = user_bounds.data_ptr()
    return p


# ------------------------------------------------------------------ SVD

def svd_fwd(A, p=None, handle=None, probe=None, user_bounds=None, **kw):
    """U, S, V, info of A = U diag(S) V^T (Algorithm 1)."""
    A = _batched(_req(A, "A"))
    b, m, n = A.shape
    h = handle or default_handle()
    p = _prep_params(p, kw, b, m, n, _req(probe, "probe"), _req(user_bounds, "user_bounds"))
    U = torch.empty((b, m, n), device=A.device)
    S = torch.empty((b, n), device=A.device)
    V = torch.empty((b, n, n), device=A.device)
    info = _info_tensor(b, A.device)
    ws = _workspace(p, _lib.OP_SVD_FWD, A.device)
    check(load().svd_polar_fwd(h.ptr, ctypes.byref(p), A.data_ptr(), n, m * n, U.data_ptr(), n, m * n,
                               S.data_ptr(), n, V.data_ptr(), n, n * n, info.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream()), "svd_polar_fwd")
    return U, S, V, info


def svd_bwd(U, S, V, dU=None, dS=None, dV=None, p=None, handle=None, **kw):
    """dA of Algorithm 4 (dV is the gradient of V, not of V^T)."""
    U = _batched(_req(U, "U")); S = _req(S, "S"); V = _batched(_req(V, "V"))
    S = S if S.dim() == 2 else S.unsqueeze(0)
    b, m, n = U.shape
    dU = None if dU is None else _batched(_req(dU, "dU"))
    dS = None if dS is None else _req(dS, "dS")
    if dS is not None and dS.dim() == 1:
        dS = dS.unsqueeze(0)
    dV = None if dV is None else _batched(_req(dV, "dV"))
    h = handle or default_handle()
    p = _prep_params(p, kw, b, m, n)
    dA = torch.empty((b, m, n), device=U.device)
    ws = _workspace(p, _lib.OP_SVD_BWD, U.device)
    check(load().svd_polar_bwd(h.ptr, ctypes.byref(p), U.data_ptr(), n, m * n, S.data_ptr(), n,
                               V.data_ptr(), n, n * n, _p(dU), n, m * n, _p(dS), n, _p(dV), n, n * n,
                               dA.data_ptr(), n, m * n, ws.data_ptr(), ws.numel(), _stream()),
          "svd_polar_bwd")
    return dA


# ------------------------------------------------------------------ polar

def polar_fwd(A, cache=True, p=None, handle=None, probe=None, user_bounds=None, **kw):
    """W, H (A = W H) and, with cache, the eigenpairs (S, V) of H."""
    A = _batched(_req(A, "A"))
    b, m, n = A.shape
    h = handle or default_handle()
    p = _prep_params(p, kw, b, m, n, _req(probe, "probe"), _req(user_bounds, "user_bounds"))
    W = torch.empty((b, m, n), device=A.device)
    H = torch.empty((b, n, n), device=A.device)
    S = torch.empty((b, n), device=A.device) if cache else None
    V = torch.empty((b, n, n), device=A.device) if cache else None
    info = _info_tensor(b, A.device)
    ws = _workspace(p, _lib.OP_POLAR_FWD, A.device)
    check(load().polar_fwd(h.ptr, ctypes.byref(p), A.data_ptr(), n, m * n, W.data_ptr(), n, m * n,
                           H.data_ptr(), n, n * n, _p(S), n, _p(V), n, n * n, info.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream()), "polar_fwd")
    return W, H, S, V, info


def polar_bwd(A, H, S=None, V=None, dW=None, dH=None, p=None, handle=None, **kw):
    """dA of Algorithm 2; without (S, V) the eigendecomposition of H is computed first."""
    A = _batched(_req(A, "A"))
    b, m, n = A.shape
    H = None if H is None else _batched(_req(H, "H"))
    S = None if S is None else _req(S, "S")
    if S is not None and S.dim() == 1:
        S = S.unsqueeze(0)
    V = None if V is None else _batched(_req(V, "V"))
    dW = None if dW is None else _batched(_req(dW, "dW"))
    dH = None if dH is None else _batched(_req(dH, "dH"))
    h = handle or default_handle()
    p = _prep_params(p, kw, b, m, n)
    dA = torch.empty((b, m, n), device=A.device)
    ws = _workspace(p, _lib.OP_POLAR_BWD, A.device)
    check(load().polar_bwd(h.ptr, ctypes.byref(p), A.data_ptr(), n, m * n, _p(H), n, n * n, _p(S), n,
                           _p(V), n, n * n, _p(dW), n, m * n, _p(dH), n, n * n, dA.data_ptr(), n, m * n,
                           ws.data_ptr(), ws.numel(), _stream()), "polar_bwd")
    return dA


# ------------------------------------------------------------------ eigh

def eigh(H, p=None, handle=None, **kw):
    """lam (descending), V, info of symmetric H = V diag(lam) V^T."""
    H = _batched(_req(H, "H"))
    b, n, _ = H.shape
    h = handle or default_handle()
    p = _prep_params(p, kw, b, n, n)
    lam = torch.empty((b, n), device=H.device)
    V = torch.empty((b, n, n), device=H.device)
    info = _info_tensor(b, H.device)
    ws = _workspace(p, _lib.OP_EIGH, H.device)
    check(load().svdp_eigh(h.ptr, ctypes.byref(p), H.data_ptr(), n, n * n, lam.data_ptr(), n,
                           V.data_ptr(), n, n * n, info.data_ptr(), ws.data_ptr(), ws.numel(),
                           _stream()), "svdp_eigh")
    return lam, V, info


def eigh_dc(H, p=None, handle=None, **kw):
    """lam (descending), V, info of symmetric H = V diag(lam) V^T by one level
    of polar-based spectral divide and conquer (svdp_eigh_dc), one matrix at
    a time."""
    H = _batched(_req(H, "H"))
    b, n, _ = H.shape
    h = handle or default_handle()
    p = _prep_params(p, kw, b, n, n)
    lam = torch.empty((b, n), device=H.device)
    V = torch.empty((b, n, n), device=H.device)
    info = _info_tensor(b, H.device)
    ws = _workspace(p, _lib.OP_EIGH_DC, H.device)
    check(load().svdp_eigh_dc(h.ptr, ctypes.byref(p), H.data_ptr(), n, n * n, lam.data_ptr(), n,
                              V.data_ptr(), n, n * n, info.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream()), "svdp_eigh_dc")
    return lam, V, info


def eigh_bwd(lam, V, dlam=None, dV=None, p=None, handle=None, **kw):
    """dH of the symmetric EVD H = V diag(lam) V^T (the EVD pseudo-gradient
    theorem, regularised K with eps_K)."""
    V = _batched(_req(V, "V"))
    lam = _req(lam, "lam")
    lam = lam if lam.dim() == 2 else lam.unsqueeze(0)
    b, n, _ = V.shape
    dlam = None if dlam is None else _req(dlam, "dlam")
    if dlam is not None and dlam.dim() == 1:
        dlam = dlam.unsqueeze(0)
    dV = None if dV is None else _batched(_req(dV, "dV"))
    h = handle or default_handle()
    p = _prep_params(p, kw, b, n, n)
    dH = torch.empty((b, n, n), device=V.device)
    ws = _workspace(p, _lib.OP_EIGH_BWD, V.device)
    check(load().svdp_eigh_bwd(h.ptr, ctypes.byref(p), lam.data_ptr(), n, V.data_ptr(), n, n * n,
                               _p(dlam), n, _p(dV), n, n * n, dH.data_ptr(), n, n * n, ws.data_ptr(),
                               ws.numel(), _stream()), "svdp_eigh_bwd")
    return dH


# ------------------------------------------------------------------ predictor

def bound_features(A, probe, handle=None):
    A = _batched(_req(A, "A"))
    b, m, n = A.shape
    probe = _req(probe, "probe")
    h = handle or default_handle()
    p = params(b, m, n)
    F = torch.empty((b, 8), device=A.device)
    aux = torch.empty((b, 2), device=A.device)
    ws = _workspace(p, _lib.OP_FEATURES, A.device)
    check(load().svdp_bound_features(h.ptr, ctypes.byref(p), A.data_ptr(), n, m * n, probe.data_ptr(),
                                     F.data_ptr(), aux.data_ptr(), ws.data_ptr(), ws.numel(), _stream()),
          "svdp_bound_features")
    return F, aux


def spectral_features(s, z, m_over_n):
    s = _req(s, "s"); z = _req(z, "z"); m_over_n = _req(m_over_n, "m_over_n")
    rows, n = s.shape
    F = torch.empty((rows, 8), device=s.device)
    aux = torch.empty((rows, 2), device=s.device)
    check(load().svdp_spectral_features(s.data_ptr(), z.data_ptr(), rows, n, m_over_n.data_ptr(),
                                        F.data_ptr(), aux.data_ptr(), _stream()), "spectral_features")
    return F, aux


def training_targets(s, aux):
    """(log(max s / r_7), log(max s / min s)) per row (svdp_training_targets)."""
    s = _req(s, "s"); aux = _req(aux, "aux")
    rows, n = s.shape
    T = torch.empty((rows, 2), device=s.device)
    check(load().svdp_training_targets(s.data_ptr(), aux.data_ptr(), rows, n, T.data_ptr(), _stream()),
          "training_targets")
    return T


def feature_stats(F):
    """Column means and sample standard deviations (clamped at 1e-3) of F
    (rows x 8), by svdp_feature_stats."""
    F = _req(F, "F")
    mu = torch.empty(8, device=F.device)
    sd = torch.empty(8, device=F.device)
    check(load().svdp_feature_stats(F.data_ptr(), F.shape[0], mu.data_ptr(), sd.data_ptr(), _stream()),
          "feature_stats")
    return mu, sd


def mlp_fwd(P, X, mu=None, sd=None, keep_act=True):
    P = _req(P, "params"); X = _req(X, "X")
    rows = X.shape[0]
    out = torch.empty((rows, 2), device=X.device)
    act = torch.empty((rows, 128), device=X.device) if keep_act else None
    check(load().svdp_mlp_fwd(P.data_ptr(), _p(mu), _p(sd), X.data_ptr(), rows, out.data_ptr(), _p(act),
                              _stream()), "svdp_mlp_fwd")
    return out, act


def mlp_bwd(P, X, act, dout, mu=None, sd=None):
    rows = X.shape[0]
    dP = torch.empty(_lib.MLP_PARAMS, device=X.device)
    nbytes = int(load().svdp_mlp_bwd_ws_bytes(rows))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.device)
    check(load().svdp_mlp_bwd(P.data_ptr(), _p(mu), _p(sd), X.data_ptr(), act.data_ptr(), dout.data_ptr(),
                              rows, dP.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "svdp_mlp_bwd")
    return dP


def pinball(out, target, tau0, tau1):
    rows = out.shape[0]
    dout = torch.empty_like(out)
    loss = torch.zeros(1, device=out.device)
    check(load().svdp_pinball(out.data_ptr(), target.data_ptr(), rows, float(tau0), float(tau1),
                              dout.data_ptr(), loss.data_ptr(), _stream()), "svdp_pinball")
    return dout, loss


def adam_step(P, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    check(load().svdp_adam_step(P.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(), P.numel(),
                                float(lr), float(b1), float(b2), float(eps), int(t), _stream()),
          "svdp_adam_step")


def poly_table(poly, steps, delta=0.99, pre_iters=2):
    """Host coefficient table (steps, 3) of (c1, c3, c5) of the conservative
    schedule of iteration polynomial `poly` (POLY_CANS3, POLY_NS, POLY_CANS5)."""
    tab = (ctypes.c_double * (3 * steps))()
    t = ctypes.c_double()
    check(load().svdp_poly_table(poly, delta, pre_iters, steps, tab, ctypes.byref(t)), "poly_table")
    return np.array(tab[:]).reshape(steps, 3), t.value


def cans_table(kind, steps, delta=0.99, pre_iters=2, lo=1e-3):
    """Host coefficient table (steps, 2) of the library's scheduler."""
    tab = (ctypes.c_double * (2 * steps))()
    t = ctypes.c_double()
    check(load().svdp_cans_table(kind, delta, pre_iters, lo, steps, tab, ctypes.byref(t)), "cans_table")
    return np.array(tab[:]).reshape(steps, 2), t.value


def pe_table(lo=1e-3, max_steps=64):
    """Host Polar Express schedule from [lo, 1]: (steps, 3) array of
    (c1, c3, c5) with the 1.01 input damping folded in (all steps but the
    last)."""
    tab = (ctypes.c_double * (3 * max_steps))()
    steps = ctypes.c_int32()
    check(load().svdp_pe_table(float(lo), int(max_steps), tab, ctypes.byref(steps)), "pe_table")
    return np.array(tab[:3 * steps.value]).reshape(steps.value, 3)
