"""Edge cases, error paths and the autograd wrappers on the GPU."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2609_32505_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_32505_amd import api as _api
    return _api


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def test_tiny_shapes(api):
    _say("tiny shapes: 1x1, 7x1, 5x5 batch 3")
    for b, m, n in [(1, 1, 1), (2, 7, 1), (3, 5, 5), (1, 33, 32)]:
        A = inputs.rng_for(90, m * n).standard_normal((b, m, n)).astype(np.float32)
        U, S, V, info = api.svd_fwd(dev(A))
        Sh, Uh, Vh = (t.cpu().double().numpy() for t in (S, U, V))
        for i in range(b):
            _, So, _, _ = oracle.svd(A[i].astype(np.float64))
            np.testing.assert_allclose(Sh[i], So, rtol=1e-5, atol=1e-6 * So[0])
            np.testing.assert_allclose((Uh[i] * Sh[i]) @ Vh[i].T, A[i], atol=2e-5 * np.abs(A[i]).max())


def test_learned_tiny_shapes_and_zero_matrix(api):
    # the learned BF16 path (with its BF16 correction) on tiny shapes, and on
    # a batch holding an all-zero matrix beside ordinary ones: no non-finite
    # output, the zero matrix gives S = 0 with orthonormal completed U, V
    import torch
    from paper_2609_32505_amd import predictor
    h = api.Handle()
    h.set_model(predictor.load())
    _say("learned path: tiny shapes and a zero matrix")
    for b, m, n, zero in [(1, 1, 1, False), (2, 7, 1, False), (3, 5, 5, False), (3, 33, 32, True)]:
        A = inputs.rng_for(91, m * n).standard_normal((b, m, n)).astype(np.float32)
        if zero:
            A[1] = 0.0
            A[2] *= 1e3
        probe = dev(inputs.probe(92, b, n))
        U, S, V, info = api.svd_fwd(dev(A), handle=h, precision=1, bound=1, probe=probe)
        torch.cuda.synchronize()
        Sh, Uh, Vh = (t.cpu().double().numpy() for t in (S, U, V))
        inf = api.info_to_numpy(info)
        _say(f"  {b} x {m} x {n}: flags {inf['flags']}")
        assert np.all(np.isfinite(Sh)) and np.all(np.isfinite(Uh)) and np.all(np.isfinite(Vh))
        for i in range(b):
            if zero and i == 1:
                assert np.all(Sh[i] == 0.0)
                assert np.abs(Uh[i].T @ Uh[i] - np.eye(n)).max() < 1e-5
                continue
            _, So, _, _ = oracle.svd(A[i].astype(np.float64))
            assert np.abs(Sh[i] - So).max() / So[0] < 1e-3
            # BF16 level: on tall shapes the rounding of the iterate outside
            # A's column space is not corrected (1.4e-3 at 7 x 1)
            assert np.linalg.norm((Uh[i] * Sh[i]) @ Vh[i].T - A[i]) <= 1e-2 * np.linalg.norm(A[i])


def test_empty_batch_is_noop(api):
    import torch
    from paper_2609_32505_amd import _lib as L
    h = api.Handle()
    p = L.default_params(0, 8, 8)
    st = L.load().svd_polar_fwd(h.ptr, ctypes.byref(p), None, 8, 64, None, 8, 64, None, 8, None, 8, 64,
                                None, None, 0, None)
    assert st == 0


def test_rank_deficient_is_flagged_and_completed(api):
    # exactly rank-deficient in FP32: the last 28 columns are zero, so CANS
    # leaves those columns of W at zero (a partial isometry); the column
    # norms of U = W V expose it and Algorithm 1's QR step completes U to an
    # orthonormal matrix.  The completion is not unique: compared are the
    # singular values, the leading 20 singular vectors (against the FP64
    # oracle, up to sign) and the orthonormality of the whole U.
    _say("rank-deficient 64x48, rank 20 (zero columns)")
    rng = inputs.rng_for(91, 0)
    B = inputs.matrix_with_spectrum(rng, 64, 20, inputs.geometric(20, 10.0))
    A = np.concatenate([B, np.zeros((64, 28))], axis=1).astype(np.float32)
    s = np.concatenate([inputs.geometric(20, 10.0), np.zeros(28)])
    U, S, V, info = api.svd_fwd(dev(A[None]))
    inf = api.info_to_numpy(info)
    Sh = S.cpu().double().numpy()[0]
    Uh, Vh = U.cpu().double().numpy()[0], V.cpu().double().numpy()[0]
    np.testing.assert_allclose(Sh[:20], s[:20], atol=1e-5)
    assert np.abs(Sh[20:]).max() < 1e-5
    assert inf["flags"][0] & 8, "rank deficiency must be reported"
    orth = np.abs(Uh.T @ Uh - np.eye(48)).max()
    _say(f"  |U^T U - I| = {orth:.2e}")
    assert orth < 1e-5
    Uo, So, Vo, _ = oracle.svd(A.astype(np.float64))
    sg = np.sign(np.sum(Uh[:, :20] * Uo[:, :20], axis=0))
    assert np.abs(Uh[:, :20] * sg - Uo[:, :20]).max() < 1e-4
    rec = np.linalg.norm((Uh * Sh) @ Vh.T - A) / np.linalg.norm(A)
    assert rec < 1e-5


def test_rank_deficient_blocked_qr_1024(api):
    # above 512 columns the QR step runs blocked (64-column blocks projected
    # by GEMMs, CGS2 inside a block).  Two 1024^2 matrices: rank 100 and
    # rank 1023 (kappa 10 on the nonzero part).  The leading singular vectors
    # are compared with the generating Q1 (known, gaps >= 2%), the rest by
    # orthonormality, singular values and reconstruction.
    import torch
    n = 1024
    _say("rank-deficient 2 x 1024^2 (ranks 100 and 1023): blocked QR")
    As, Ss, Q1s = [], [], []
    for i, r in enumerate((100, 1023)):
        rng = inputs.rng_for(93, i)
        s = inputs.paper_kappa_rank(n, 10.0, r)
        Q1 = inputs.orthonormal(rng, n, n)
        Q2 = inputs.orthonormal(rng, n, n)
        As.append(((Q1 * s) @ Q2.T).astype(np.float32)); Ss.append(s); Q1s.append(Q1)
    A = np.stack(As)
    U, S, V, info = api.svd_fwd(dev(A))
    torch.cuda.synchronize()
    inf = api.info_to_numpy(info)
    Sh, Uh, Vh = (t.cpu().double().numpy() for t in (S, U, V))
    for i, r in enumerate((100, 1023)):
        orth = np.abs(Uh[i].T @ Uh[i] - np.eye(n)).max()
        orthv = np.abs(Vh[i].T @ Vh[i] - np.eye(n)).max()
        serr = np.abs(Sh[i] - Ss[i]).max() / Ss[i][0]
        rec = np.linalg.norm((Uh[i] * Sh[i]) @ Vh[i].T - A[i]) / np.linalg.norm(A[i])
        lead = np.abs(np.sum(Uh[i][:, :r] * Q1s[i][:, :r], axis=0)).min()
        _say(f"  rank {r}: flags {inf['flags'][i]}, |U^T U - I| {orth:.2e}, |V^T V - I| {orthv:.2e}, "
             f"sigma err {serr:.2e}, recon {rec:.2e}, min |<u_i, q_i>| over the leading {r}: {lead:.6f}")
        assert inf["flags"][i] & 8, "rank deficiency must be reported"
        assert orth < 1e-5 and orthv < 1e-5
        assert serr < 1e-5 and rec < 1e-5
        assert lead > 1 - 1e-4


def test_rank_deficient_blocked_qr_tall_and_learned(api):
    # the blocked QR step on a tall, exactly rank-deficient matrix: 1536 x 768
    # whose last 668 columns are zero (rank 100, kappa 10), on the
    # conservative path and on the learned BF16 path (a predictor model loaded;
    # a failed bound falls back to conservative CANS).  CANS leaves the zero
    # directions of W at zero, the column-norm test flags U and the QR step
    # completes it: U orthonormal, sigma against the generating spectrum, the
    # leading vectors against the generating Q1
    import torch
    from paper_2609_32505_amd import predictor
    m, n, r = 1536, 768, 100
    _say("1536 x 768 with 668 zero columns (rank 100): blocked QR, conservative and learned")
    rng = inputs.rng_for(94, 0)
    sr = inputs.paper_kappa_rank(r, 10.0)
    Q1 = inputs.orthonormal(rng, m, r)
    Q2 = inputs.orthonormal(rng, r, r)
    A = np.zeros((1, m, n), np.float32)
    A[0, :, :r] = (Q1 * sr) @ Q2.T
    s = np.concatenate([sr, np.zeros(n - r)])
    h = api.Handle()
    h.set_model(predictor.load())
    probe = torch.from_numpy(inputs.probe(17, 1, n)).cuda()
    for label, kw, tol_s in [("conservative", {}, 1e-5),
                             ("learned-bf16", dict(precision=1, bound=1, probe=probe), 1e-3)]:
        U, S, V, info = api.svd_fwd(dev(A), handle=h, **kw)
        torch.cuda.synchronize()
        inf = api.info_to_numpy(info)
        Uh, Sh, Vh = (t.cpu().double().numpy()[0] for t in (U, S, V))
        orth = np.abs(Uh.T @ Uh - np.eye(n)).max()
        serr = np.abs(Sh - s).max() / s[0]
        lead = np.abs(np.sum(Uh[:, :r] * Q1, axis=0)).min()
        rec = np.linalg.norm((Uh * Sh) @ Vh.T - A[0]) / np.linalg.norm(A[0])
        _say(f"  {label}: flags {inf['flags'][0]}, |U^T U - I| {orth:.2e}, sigma err {serr:.2e}, recon {rec:.2e}, "
             f"min |<u_i, q_i>| {lead:.6f}")
        assert inf["flags"][0] & 8
        assert orth < 1e-5 and serr < tol_s
        assert lead > 1 - (1e-4 if label == "conservative" else 1e-2)


def _eigh_backward_error(api, H, **kw):
    import torch
    lam, V, info = api.eigh(H, **kw)
    torch.cuda.synchronize()
    Hd = (0.5 * (H + H.transpose(-1, -2))).double()
    Vd, Ld = V.double(), lam.double()
    rec = torch.linalg.norm(Hd - (Vd * Ld[:, None, :]) @ Vd.transpose(-1, -2), dim=(1, 2)) / torch.linalg.norm(Hd, dim=(1, 2))
    return rec.cpu().numpy(), api.info_to_numpy(info)


def test_eigh_restarts_reach_fp32_floor_at_2048(api):
    # many FP32 block rotations leave a backward error that grows with n, and
    # one FP64 sweep does not finish a dense spectrum (kappa 10: 2048 values
    # in [1, 10]); the restarts (T = V^T H V re-formed and swept) must bring
    # |H - V diag(lam) V^T|_F / |H|_F to the 6e-6 tolerance
    import torch
    n = 2048
    _say("eigh 2048^2, eigenvalues geometric 10 .. 1: restarts off vs on")
    rng = inputs.rng_for(95, 0)
    Q = inputs.orthonormal(rng, n, n)
    H = torch.from_numpy(((Q * inputs.paper_kappa_rank(n, 10.0)) @ Q.T).astype(np.float32)[None]).cuda()
    r0, i0 = _eigh_backward_error(api, H, eigh_restarts=0)
    r2, i2 = _eigh_backward_error(api, H)
    _say(f"  no restart: {r0[0]:.2e} ({i0['sweeps'][0]} sweeps); default: {r2[0]:.2e} ({i2['sweeps'][0]} sweeps)")
    assert r2[0] < 8e-6 and r2[0] < r0[0]
    assert i2["sweeps"][0] <= i0["sweeps"][0] + 2


def test_eigh_restart_skips_rounding_level_cluster(api):
    # rank 100 at n = 1024: about 924 eigenvalues at rounding level.  Rotating
    # those pairs in a restart stirs the cluster and the restart converges only
    # linearly; restart sweeps leave pairs entirely below 2^-24 |H|_F alone,
    # and one restart reaches the tolerance
    import torch
    n = 1024
    _say("eigh of H = sym(W^T A), A 1024^2 of rank 100")
    rng = inputs.rng_for(93, 0)
    s = inputs.paper_kappa_rank(n, 10.0, 100)
    Q1 = inputs.orthonormal(rng, n, n)
    Q2 = inputs.orthonormal(rng, n, n)
    A = torch.from_numpy(((Q1 * s) @ Q2.T).astype(np.float32)[None]).cuda()
    W, H, _, _, _ = api.polar_fwd(A, cache=False)
    r0, i0 = _eigh_backward_error(api, H, eigh_restarts=0)
    r, inf = _eigh_backward_error(api, H)
    _say(f"  no restart: {r0[0]:.2e} ({i0['sweeps'][0]} sweeps); default: {r[0]:.2e} ({inf['sweeps'][0]} sweeps)")
    assert r[0] < 6e-6
    assert inf["sweeps"][0] <= i0["sweeps"][0] + 1


def test_numerically_rank_deficient_is_completed(api):
    # sigma down to 1e-9 relative: the smallest directions of W stay far
    # from unit norm after CANS, so U is orthogonalised by QR
    _say("96 x 64, sigma geometric 1 .. 1e-9")
    A, s = inputs.batch_with_spectra(97, 3, 96, 64, lambda r: inputs.geometric(64, 1e9))
    U, S, V, info = api.svd_fwd(dev(A))
    inf = api.info_to_numpy(info)
    Sh, Uh, Vh = (t.cpu().double().numpy() for t in (S, U, V))
    for i in range(3):
        orth = np.abs(Uh[i].T @ Uh[i] - np.eye(64)).max()
        serr = np.abs(Sh[i] - s[i]).max() / s[i][0]
        rec = np.linalg.norm((Uh[i] * Sh[i]) @ Vh[i].T - A[i]) / np.linalg.norm(A[i])
        _say(f"  b={i} flags={inf['flags'][i]} |U^T U - I|={orth:.2e} s_err={serr:.2e} recon={rec:.2e}")
        assert orth < 1e-5 and serr < 1e-5 and rec < 1e-5


def test_workspace_and_argument_errors(api):
    import torch
    from paper_2609_32505_amd import _lib as L
    h = api.Handle()
    A = torch.zeros((2, 16, 8), device="cuda")
    out = [torch.empty((2, 16, 8), device="cuda"), torch.empty((2, 8), device="cuda"),
           torch.empty((2, 8, 8), device="cuda")]
    p = L.default_params(2, 16, 8)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    st = L.load().svd_polar_fwd(h.ptr, ctypes.byref(p), A.data_ptr(), 8, 128, out[0].data_ptr(), 8, 128,
                                out[1].data_ptr(), 8, out[2].data_ptr(), 8, 64, None, ws.data_ptr(), 16, None)
    assert st == 3
    p2 = L.default_params(2, 16, 8, bound=1)
    h.set_model(np.zeros(L.MODEL_FLOATS, np.float32))
    st = L.load().svd_polar_fwd(h.ptr, ctypes.byref(p2), A.data_ptr(), 8, 128, out[0].data_ptr(), 8, 128,
                                out[1].data_ptr(), 8, out[2].data_ptr(), 8, 64, None, ws.data_ptr(), 16, None)
    assert st == 1 and "probe" in L.load().svdp_last_error().decode()
    st = L.load().svd_polar_fwd(h.ptr, ctypes.byref(p), A.data_ptr(), 4, 128, out[0].data_ptr(), 8, 128,
                                out[1].data_ptr(), 8, out[2].data_ptr(), 8, 64, None, ws.data_ptr(), 16, None)
    assert st == 1  # lda < n


def test_user_bound_too_small_falls_back(api):
    _say("user bound sigma_max at half the true value: fallback to conservative CANS")
    A, s = inputs.batch_with_spectra(92, 2, 96, 64, lambda r: inputs.log_uniform(r, 64, 1e-2, 1.0))
    ub = dev(np.stack([s[:, -1], 0.5 * s[:, 0]], axis=1))
    U, S, V, info = api.svd_fwd(dev(A), precision=1, bound=2, user_bounds=ub, margin_max=1.0)
    inf = api.info_to_numpy(info)
    assert np.all(inf["flags"] & 2), "fallback must be used"
    Sh = S.cpu().double().numpy()
    assert (np.abs(Sh - s).max(axis=1) / s[:, 0]).max() < 1e-5


def test_polar_bf16_corrected_with_fallback(api):
    # polar_fwd on the BF16 path with the eigenpairs cached (the BF16
    # correction on) and a user bound too small for matrix 1 only: matrix 1
    # falls back to conservative FP32 CANS (its W comes from the masked
    # copy of the rerun's iterate, its H from the rerun), the others keep the
    # corrected W and H; all against the FP64 oracle's polar factors
    _say("polar_fwd BF16, cached eigenpairs, one matrix falling back")
    b, n = 3, 128
    A, s = inputs.batch_with_spectra(95, b, n, n, lambda r: inputs.log_uniform(r, n, 1e-2, 1.0))
    bounds = np.stack([s[:, -1], s[:, 0]], axis=1)
    bounds[1, 1] *= 0.5
    W, H, S, V, info = api.polar_fwd(dev(A), cache=True, precision=1, bound=2, user_bounds=dev(bounds),
                                     margin_max=1.0)
    Wh, Hh, Sh, Vh = host(W), host(H), host(S), host(V)
    inf = api.info_to_numpy(info)
    assert [bool(f & 2) for f in inf["flags"]] == [False, True, False], inf["flags"]
    for i in range(b):
        Uo, So, Vo, _ = oracle.svd(A[i].astype(np.float64))
        Wo, Ho = oracle.polar_from_svd(Uo, So, Vo)
        werr = np.abs(Wh[i] - Wo).max()
        herr = np.abs(Hh[i] - Ho).max() / So[0]
        serr = np.abs(np.abs(Sh[i]) - So).max() / So[0]
        eig = np.abs((Vh[i] * Sh[i]) @ Vh[i].T - Hh[i]).max() / So[0]
        _say(f"  matrix {i} (fallback {bool(inf['flags'][i] & 2)}): W {werr:.2e}, H {herr:.2e}, S {serr:.2e}, "
             f"|V S V^T - H| {eig:.2e}")
        assert werr < 2e-4 and herr < 1e-5 and serr < 1e-5 and eig < 1e-5


def test_repeatable(api):
    A, _ = inputs.batch_with_spectra(93, 4, 100, 70, lambda r: inputs.log_uniform(r, 70, 1e-3, 1.0))
    r1 = [t.cpu().numpy() for t in api.svd_fwd(dev(A))[:3]]
    r2 = [t.cpu().numpy() for t in api.svd_fwd(dev(A))[:3]]
    for a, b in zip(r1, r2):
        np.testing.assert_array_equal(a, b)
    # the learned BF16 path too: its sketch features (|A|_F, column sums,
    # A^T x) are reduced in a fixed order, so the predicted interval, the
    # schedule and every output repeat bit for bit (ragged: 300 x 200)
    from paper_2609_32505_amd import predictor
    h = api.Handle()
    h.set_model(predictor.load())
    A, _ = inputs.batch_with_spectra(95, 6, 300, 200, lambda r: inputs.log_uniform(r, 200, 1e-4, 1.0))
    probe = dev(inputs.probe(96, 6, 200))
    F1, _ = api.bound_features(dev(A), probe, h)
    F2, _ = api.bound_features(dev(A), probe, h)
    np.testing.assert_array_equal(F1.cpu().numpy(), F2.cpu().numpy())
    outs = []
    for _ in range(2):
        U, S, V, info = api.svd_fwd(dev(A), handle=h, precision=1, bound=1, probe=probe)
        outs.append([t.cpu().numpy() for t in (U, S, V)] + [api.info_to_numpy(info)["iters"]])
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    # the benchmark's batch (256 x 512^2) on both paths, forward and backward:
    # every reduction that feeds a decision (stop tests, sweep and restart
    # tests, residual, column norms, features) runs in a fixed order
    import torch
    A, _ = inputs.square_loguniform(seed=2, batch=256, n=512)
    Ad = dev(A)
    probe = dev(inputs.probe(13, 256, 512))
    rng = np.random.default_rng(7)
    dU, dV = dev(rng.standard_normal((256, 512, 512))), dev(rng.standard_normal((256, 512, 512)))
    dS = dev(rng.standard_normal((256, 512)))
    for kw in (dict(), dict(precision=1, bound=1, probe=probe, fp64_sweeps=1, eigh_off_tol=1e-4,
                                jacobi_fro_tol=1e-3)):
        runs = []
        for _ in range(2):
            U, S, V, info = api.svd_fwd(Ad, handle=h, **kw)
            dA = api.svd_bwd(U, S, V, dU, dS, dV, handle=h)
            torch.cuda.synchronize()
            runs.append([t.cpu().numpy() for t in (U, S, V, info, dA)])
        for a, b in zip(runs[0], runs[1]):
            np.testing.assert_array_equal(a, b)
        _say(f"  256 x 512^2 {'learned' if kw else 'plain'}: two runs bit for bit equal")


def test_autograd_svd_and_polar(api):
    import torch
    from paper_2609_32505_amd import autograd
    _say("autograd wrappers")
    A, _ = inputs.batch_with_spectra(94, 2, 40, 24, lambda r: inputs.log_uniform(r, 24, 1e-1, 1.0))
    At = dev(A).requires_grad_(True)
    U, S, Vh = autograd.svd(At)
    rng = np.random.default_rng(3)
    gU, gS, gV = dev(rng.standard_normal(U.shape)), dev(rng.standard_normal(S.shape)), dev(rng.standard_normal(Vh.shape))
    loss = (U * gU).sum() + (S * gS).sum() + (Vh * gV).sum()
    loss.backward()
    ref = api.svd_bwd(U.detach(), S.detach(), Vh.detach().transpose(-1, -2).contiguous(), gU, gS,
                      gV.transpose(-1, -2).contiguous())
    np.testing.assert_allclose(At.grad.cpu().numpy(), ref.cpu().numpy(), rtol=1e-5, atol=1e-5)
    # polar: gradient of <G, W> + <K, H> against the oracle (Algorithm 2, eps = 0)
    A2 = dev(A).requires_grad_(True)
    W, H = autograd.polar(A2)
    G = rng.standard_normal(W.shape)
    K = rng.standard_normal(H.shape)
    ((W * dev(G)).sum() + (H * dev(K)).sum()).backward()
    g = A2.grad.cpu().double().numpy()
    for i in range(2):
        Uo, So, Vo, _ = oracle.svd(A[i].astype(np.float64))
        _, Ho = oracle.polar_from_svd(Uo, So, Vo)
        ref = oracle.polar_bwd(A[i], Ho, G[i], K[i])
        assert np.linalg.norm(g[i] - ref) / np.linalg.norm(ref) < 1e-4


def test_eigh_results_do_not_depend_on_stream_parts(api):
    # the eigensolver splits the batch over parallel streams; every matrix
    # runs the same kernels on its own data, so results are bitwise equal
    import os
    import torch
    _say("eigh 5 x 100^2 with 1, 2 and 4 stream parts")
    rng = inputs.rng_for(95, 0)
    lam0 = inputs.log_uniform(rng, 100, 1e-3, 1.0)
    Hs = np.stack([inputs.matrix_with_spectrum(inputs.rng_for(95, i + 1), 100, 100, lam0) for i in range(5)])
    Hs = 0.5 * (Hs + Hs.transpose(0, 2, 1))
    Hd = dev(Hs)
    out = []
    old = os.environ.get("SVDP_EIGH_PARTS")
    try:
        for parts in ("1", "2", "4"):
            os.environ["SVDP_EIGH_PARTS"] = parts
            h = api.Handle()
            lam, V, info = api.eigh(Hd, handle=h)
            torch.cuda.synchronize()
            out.append((lam.cpu().numpy(), V.cpu().numpy(), api.info_to_numpy(info)["sweeps"]))
    finally:
        if old is None:
            os.environ.pop("SVDP_EIGH_PARTS", None)
        else:
            os.environ["SVDP_EIGH_PARTS"] = old
    for lam, V, sw in out[1:]:
        np.testing.assert_array_equal(lam, out[0][0])
        np.testing.assert_array_equal(V, out[0][1])
        np.testing.assert_array_equal(sw, out[0][2])


def test_bound_far_too_narrow_hits_refinement_cap_and_falls_back(api):
    # user bounds claim kappa = 2 for matrices with kappa = 1e3: the bounded
    # schedule leaves the small singular values far from 1, the refinement
    # stop test does not pass within its cap, and conservative CANS reruns
    _say("user bounds with kappa 2 for kappa 1e3: refinement cap, fallback")
    A, s = inputs.batch_with_spectra(96, 3, 80, 64, lambda r: inputs.log_uniform(r, 64, 1e-3, 1.0))
    ub = dev(np.stack([0.5 * s[:, 0], s[:, 0]], axis=1))
    U, S, V, info = api.svd_fwd(dev(A), precision=1, bound=2, user_bounds=ub)
    inf = api.info_to_numpy(info)
    assert np.all(inf["flags"] & 2), "fallback must be used"
    assert not np.any(inf["flags"] & 1), "the conservative rerun converges"
    Sh = S.cpu().double().numpy()
    assert (np.abs(Sh - s).max(axis=1) / s[:, 0]).max() < 1e-5


def test_forward_host_syncs(api):
    # the forward passes enqueue their iteration control on the device: no
    # host synchronisation on the conservative path, one (the fallback test)
    # on the learned path, at n <= 512 (the QR step runs per matrix there)
    import torch
    from paper_2609_32505_amd import _lib as L, predictor
    h = api.Handle()
    h.set_model(predictor.load())
    A, _ = inputs.batch_with_spectra(98, 8, 256, 256, lambda r: inputs.log_uniform(r, 256, 1e-3, 1.0))
    Ad = dev(A)
    probe = dev(inputs.probe(99, 8, 256))
    lib = L.load()
    api.svd_fwd(Ad, handle=h)
    torch.cuda.synchronize()
    n0 = lib.svdp_host_syncs()
    U, S, V, info = api.svd_fwd(Ad, handle=h)
    n1 = lib.svdp_host_syncs()
    api.svd_fwd(Ad, handle=h, precision=1, bound=1, probe=probe)
    n2 = lib.svdp_host_syncs()
    W, H, _, _, _ = api.polar_fwd(Ad, handle=h, cache=False)
    n3 = lib.svdp_host_syncs()
    torch.cuda.synchronize()
    _say(f"  host syncs: conservative svd {n1 - n0}, learned svd {n2 - n1}, conservative polar {n3 - n2}")
    assert n1 - n0 == 0 and n2 - n1 <= 1 and n3 - n2 == 0
    # and the results are those of the oracle
    Sh = S.cpu().double().numpy()
    for i in (0, 7):
        So = oracle.svd(A[i].astype(np.float64))[1]
        assert np.abs(Sh[i] - So).max() / So[0] < 1e-5


def _householder_product(rng, n, k):
    """Q = (I - 2 v1 v1^T) ... (I - 2 vk vk^T) with random unit v_i, dense
    FP64, and the v_i."""
    Q = np.eye(n)
    vs = []
    for _ in range(k):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        Q -= 2.0 * np.outer(Q @ v, v)
        vs.append(v)
    return Q, vs


def test_max_size_8192(api):
    # the largest n the library accepts (8192), one matrix with a known SVD:
    # A = Q1 diag(s) Q2^T with Q1, Q2 products of four Householder
    # reflections (dense, exactly orthogonal, cheap to form at this size) and
    # s geometric from 1 to 1e-3.  Checked: sigma against s (normwise), the
    # reconstruction and orthogonality at the FP32 level, U and V against Q1
    # and Q2 on well separated columns.  The CANS stop test is normwise
    # (|dX|_F <= 1e-5 |X|_F), so at this n one direction may still be off by
    # up to about 1e-5 sqrt(n) when it passes; the column-norm test then flags
    # RANK_DEFICIENT and Algorithm 1's QR step completes that column, which is
    # allowed here (no other flag is)
    import torch
    n = 8192
    rng = inputs.rng_for(97, 0)
    s = inputs.geometric(n, 1e3)
    Q1, _ = _householder_product(rng, n, 4)
    Q2, v2 = _householder_product(rng, n, 4)
    # A = Q1 diag(s) Q2^T with Q2^T = H4 H3 H2 H1 applied as reflections
    # (O(n^2) each instead of an n^3 product)
    A = Q1 * s
    for v in reversed(v2):
        A -= 2.0 * np.outer(A @ v, v)
    A = A.astype(np.float32)
    _say(f"max size {n}^2 (plain FP32)")
    Ad = dev(A)[None]
    del A
    U, S, V, info = api.svd_fwd(Ad)
    torch.cuda.synchronize()
    inf = api.info_to_numpy(info)
    _say(f"  iters {inf['iters'][0]}, sweeps {inf['sweeps'][0]}, flags {inf['flags'][0]}")
    assert (inf["flags"][0] & ~8) == 0
    Sh = S[0].cpu().double().numpy()
    sig = np.abs(Sh - s).max() / s[0]
    Ud, Sd, Vd, Md = U[0].double(), S[0].double(), V[0].double(), Ad[0].double()
    rec = float(torch.linalg.norm(Md - (Ud * Sd) @ Vd.T) / torch.linalg.norm(Md))
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    orth = max(float(torch.linalg.norm(Ud.T @ Ud - eye)), float(torch.linalg.norm(Vd.T @ Vd - eye))) / np.sqrt(n)
    # columns whose singular value is separated from its neighbours by 1e-4 s_1
    sep = np.ones(n, bool)
    d = np.abs(np.diff(s)) / s[0]
    sep[:-1] &= d > 1e-4
    sep[1:] &= d > 1e-4
    idx = np.nonzero(sep)[0][:: max(1, int(sep.sum()) // 256)]
    Uh, Vh = U[0].cpu().double().numpy()[:, idx], V[0].cpu().double().numpy()[:, idx]
    sg = np.sign(np.sum(Vh * Q2[:, idx], axis=0))
    eu = float(np.abs(Uh * sg - Q1[:, idx]).max())
    ev = float(np.abs(Vh * sg - Q2[:, idx]).max())
    _say(f"  sigma error {sig:.2e}, reconstruction {rec:.2e}, orthogonality {orth:.2e}, "
         f"U {eu:.2e}, V {ev:.2e} on {len(idx)} separated columns")
    # the same normwise stop leaves sigma 6.5e-5 normwise here (4e-6 at
    # 4096^2); reconstruction 2.7e-5, orthogonality 1.2e-5, U and V 2.3e-3
    # on columns separated by 1e-4 s_1
    assert sig < 2e-4 and rec < 1e-4 and orth < 5e-5
    assert eu < 1e-2 and ev < 1e-2
