"""GPU parity of the HIP path against the FP64 oracle on small and ragged
shapes (several tiles plus a ragged tail).  Every call goes through the C ABI
(libsvdp.so) via the ctypes binding."""
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


def col_align(X, Xref):
    """signs that align the columns of X with those of Xref (batched)"""
    s = np.sign(np.sum(X * Xref, axis=-2, keepdims=True))
    s[s == 0] = 1.0
    return s


# ------------------------------------------------------------------ eigh

@pytest.mark.parametrize("n,batch", [(64, 2), (100, 3), (256, 2)])
def test_eigh_matches_oracle(api, n, batch):
    _say(f"eigh n={n} batch={batch}")
    Hs, lams = [], []
    for b in range(batch):
        rng = inputs.rng_for(100 + n, b)
        Q = inputs.orthonormal(rng, n, n)
        lam = np.sort(rng.uniform(-1.0, 2.0, n))[::-1]
        Hs.append(((Q * lam) @ Q.T).astype(np.float32))
    H = np.stack(Hs)
    lam_g, V_g, info = api.eigh(dev(H))
    lam_g, V_g = host(lam_g), host(V_g)
    inf = api.info_to_numpy(info)
    for b in range(batch):
        lo, Vo, _ = oracle.eigh(H[b].astype(np.float64))
        scale = np.abs(lo).max()
        err = np.abs(lam_g[b] - lo).max() / scale
        Vb = V_g[b] * col_align(V_g[b], Vo)
        # eigenvectors are compared where the gap to the neighbours exceeds
        # 1e-2 |H| (their conditioning is ~ eps |H| / gap)
        gap = np.abs(np.diff(lo)) / scale
        sep = np.ones(n, bool)
        sep[:-1] &= gap > 1e-2
        sep[1:] &= gap > 1e-2
        verr = np.abs(Vb - Vo)[:, sep].max() if sep.any() else 0.0
        orth = np.abs(V_g[b].T @ V_g[b] - np.eye(n)).max()
        recon = np.abs((V_g[b] * lam_g[b]) @ V_g[b].T - H[b]).max() / scale
        _say(f"  b={b} lam_err={err:.2e} V_err={verr:.2e} orth={orth:.2e} recon={recon:.2e} "
             f"sweeps={inf['sweeps'][b]} flags={inf['flags'][b]}")
        assert err < 2e-6
        assert orth < 2e-6
        assert recon < 4e-6
        assert verr < 1e-4


def test_eigh_diagonal_and_repeated(api):
    _say("eigh diagonal / repeated")
    n = 96
    d = np.linspace(3.0, -1.0, n)
    d[10] = d[11]  # exact tie
    rng = inputs.rng_for(7, 0)
    perm = rng.permutation(n)
    H = np.diag(d[perm]).astype(np.float32)
    lam, V, info = api.eigh(dev(H[None]))
    np.testing.assert_allclose(host(lam)[0], np.sort(d)[::-1], atol=1e-6)
    Vh = host(V)[0]
    np.testing.assert_allclose(np.abs(Vh).max(axis=0), 1.0, atol=1e-6)
    # repeated eigenvalue cluster in a rotated basis: compare the subspace
    Q = inputs.orthonormal(rng, 64, 64)
    lam0 = np.concatenate([[5.0, 5.0, 5.0], np.linspace(4.0, 1.0, 61)])
    H2 = ((Q * lam0) @ Q.T).astype(np.float32)
    lam2, V2, _ = api.eigh(dev(H2[None]))
    np.testing.assert_allclose(host(lam2)[0], lam0, atol=1e-5 * 5)
    P = host(V2)[0][:, :3]
    Po = Q[:, :3]
    s = np.linalg.svd(P.T @ Po, compute_uv=False)
    assert s.min() > 1 - 1e-5


# ------------------------------------------------------------------ SVD forward

def _svd_check(api, A, S_true=None, tol_s=1e-5, tol_uv=2e-3, **kw):
    U, S, V, info = api.svd_fwd(dev(A), **kw)
    U, S, V = host(U), host(S), host(V)
    inf = api.info_to_numpy(info)
    out = []
    for b in range(A.shape[0]):
        Uo, So, Vo, _ = oracle.svd(A[b].astype(np.float64))
        serr = np.abs(S[b] - So).max() / So[0]
        sg = col_align(V[b], Vo)
        Ub, Vb = U[b] * sg, V[b] * sg
        gap = np.abs(np.diff(So)) / So[0]
        sep = np.ones(len(So), bool)
        sep[:-1] &= gap > 1e-3
        sep[1:] &= gap > 1e-3
        uerr = np.abs(Ub - Uo)[:, sep].max() if sep.any() else 0.0
        verr = np.abs(Vb - Vo)[:, sep].max() if sep.any() else 0.0
        W, H = oracle.polar_from_svd(Uo, So, Vo)
        werr = np.abs(U[b] @ V[b].T - W).max()
        recon = np.linalg.norm((U[b] * S[b]) @ V[b].T - A[b]) / np.linalg.norm(A[b])
        orth = max(np.abs(U[b].T @ U[b] - np.eye(U.shape[2])).max(), np.abs(V[b].T @ V[b] - np.eye(U.shape[2])).max())
        _say(f"  b={b} s_err={serr:.2e} U_err={uerr:.2e} V_err={verr:.2e} W_err={werr:.2e} "
             f"recon={recon:.2e} orth={orth:.2e} iters={inf['iters'][b]} sweeps={inf['sweeps'][b]} "
             f"flags={inf['flags'][b]} res={inf['residual'][b]:.1e}")
        out.append((serr, uerr, verr, werr, recon, orth, inf["flags"][b]))
        assert serr < tol_s
        assert uerr < tol_uv and verr < tol_uv
    return out


def test_svd_single_64_fp32(api):
    _say("svd 1 x 64^2 fp32 conservative")
    A, _ = inputs.single_64()
    r = _svd_check(api, A)
    assert r[0][4] < 1e-5 and r[0][5] < 1e-5 and r[0][6] == 0


@pytest.mark.parametrize("b,m,n", [(3, 37, 20), (2, 130, 100), (2, 200, 200)])
def test_svd_ragged_fp32(api, b, m, n):
    _say(f"svd {b} x {m} x {n} fp32 conservative")
    A, _ = inputs.batch_with_spectra(50 + m, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-3, 1.0))
    _svd_check(api, A, tol_uv=5e-3)


@pytest.mark.parametrize("poly", [1, 2])
@pytest.mark.parametrize("b,m,n", [(3, 130, 100), (2, 200, 200)])
def test_svd_poly_variants_fp32(api, poly, b, m, n):
    # the iteration variants of the polar ablation (1: classical Newton-
    # Schulz, 2: the CANS quintic) against the FP64 oracle, and their step
    # counts against the CANS cubic on the same matrices
    _say(f"svd {b} x {m} x {n} fp32 conservative, poly {poly}")
    A, _ = inputs.batch_with_spectra(60 + m, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-3, 1.0))
    r = _svd_check(api, A, tol_uv=5e-3, poly=poly, max_iters=64)
    assert all(x[4] < 1e-5 and x[5] < 1e-5 and x[6] == 0 for x in r)
    _, _, _, i3 = api.svd_fwd(dev(A))
    _, _, _, ip = api.svd_fwd(dev(A), poly=poly, max_iters=64)
    it3, itp = api.info_to_numpy(i3)["iters"], api.info_to_numpy(ip)["iters"]
    _say(f"  iterations: cubic {it3}, poly {poly} {itp}")
    assert np.all(itp > it3) if poly == 1 else np.all(itp < it3)


@pytest.mark.parametrize("b,m,n", [(3, 130, 100), (2, 200, 200)])
def test_svd_polar_express_fp32(api, b, m, n):
    # Polar Express (poly 3) with its lower end below sigma_min / |A|_F: the
    # SVD against the FP64 oracle's Jacobi SVD, the polar factor against the
    # oracle's own FP64 Polar Express iterate, the step count against the
    # oracle's schedule
    import torch
    import oracle
    _say(f"svd {b} x {m} x {n} fp32, Polar Express")
    A, S = inputs.batch_with_spectra(65 + m, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-3, 1.0))
    lo = float(0.5 * (S[:, -1] / np.linalg.norm(S, axis=1)).min())
    r = _svd_check(api, A, tol_uv=5e-3, poly=3, pe_lo=lo, max_iters=64)
    assert all(x[4] < 1e-5 and x[5] < 1e-5 and x[6] == 0 for x in r)
    W, _, _, _, info = api.polar_fwd(dev(A), poly=3, pe_lo=lo, max_iters=64, cache=False)
    torch.cuda.synchronize()
    Wh = W.cpu().double().numpy()
    inf = api.info_to_numpy(info)
    for i in range(b):
        Wo, steps = oracle.polar_express_polar(A[i].astype(np.float64), lo)
        err = np.abs(Wh[i] - Wo).max()
        _say(f"  matrix {i}: {inf['iters'][i]} steps (oracle {steps}), W vs oracle Polar Express {err:.2e}")
        assert inf["iters"][i] == steps and err < 1e-4


def test_svd_bf16_user_bounds(api):
    # BF16 CANS from exact bounds, with the BF16 correction of the factors:
    # sigma to 1e-3 normwise, and the singular vectors of columns separated by
    # a gap of 1e-3 sigma_1 (their conditioning ~ error / gap) to 1e-2
    import torch
    _say("svd 4 x 256^2 bf16 user bounds")
    A, S = inputs.square_loguniform(seed=9, batch=4, n=256)
    So = np.stack([oracle.svd(a.astype(np.float64))[1] for a in A])
    ub = dev(np.stack([So[:, -1], So[:, 0]], axis=1))
    r = _svd_check(api, A, tol_s=1e-3, tol_uv=1e-2, precision=1, bound=2, user_bounds=ub)
    assert max(x[4] for x in r) < 1e-4   # reconstruction
    assert max(x[5] for x in r) < 1e-5   # orthogonality


@pytest.mark.parametrize("eps", [1e-8, 1e-6])
def test_polar_bwd_regularised_matches_oracle(api, eps):
    # Algorithm 2 with eps > 0 (eps_R = eps^(1/2), eps_T = eps^(1/4)): the
    # regularisers change the result by O(1) at these spectra (sigma down to
    # 1e-2), both from the cached eigenpairs and from a fresh eigendecomposition
    _say(f"polar bwd 2 x 80 x 48, eps {eps}")
    b, m, n = 2, 80, 48
    A, _ = inputs.batch_with_spectra(72, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-2, 1.0))
    _, eR, eT = oracle.paper_eps(eps)
    rng = inputs.rng_for(73, 0)
    dW = rng.standard_normal((b, m, n)).astype(np.float32)
    dH = rng.standard_normal((b, n, n)).astype(np.float32)
    Hs = np.stack([oracle.polar_from_svd(*oracle.svd(A[i].astype(np.float64))[:3])[1] for i in range(b)])
    H32 = Hs.astype(np.float32)
    lam, Vc, _ = api.eigh(dev(H32))
    for use_cache in (True, False):
        if use_cache:
            dA = host(api.polar_bwd(dev(A), None, lam, Vc, dev(dW), dev(dH), eps_R=eR, eps_T=eT))
        else:
            dA = host(api.polar_bwd(dev(A), dev(H32), None, None, dev(dW), dev(dH), eps_R=eR, eps_T=eT))
        for i in range(b):
            ref = oracle.polar_bwd(A[i], H32[i], dW[i], dH[i], eR, eT)
            ref0 = oracle.polar_bwd(A[i], H32[i], dW[i], dH[i], 0.0, 0.0)
            rel = np.linalg.norm(dA[i] - ref) / np.linalg.norm(ref)
            moved = np.linalg.norm(ref - ref0) / np.linalg.norm(ref)
            _say(f"  cache={use_cache} b={i} rel={rel:.2e} (regularisers move the gradient by {moved:.2e})")
            assert rel < 1e-4 and moved > 1e-2


# ------------------------------------------------------------------ backward

@pytest.mark.parametrize("eps", [0.0, 1e-8])
def test_svd_bwd_matches_oracle(api, eps):
    _say(f"svd bwd 3 x 96 x 64, eps={eps}")
    b, m, n = 3, 96, 64
    A, _ = inputs.batch_with_spectra(60, b, m, n, lambda r: inputs.clustered_pairs(n, first=4, step=8))
    rng = inputs.rng_for(61, 0)
    dU = rng.standard_normal((b, m, n)).astype(np.float32)
    dS = rng.standard_normal((b, n)).astype(np.float32)
    dV = rng.standard_normal((b, n, n)).astype(np.float32)
    eK, eR, eT = oracle.paper_eps(eps) if eps > 0 else (1e-12, 0.0, 0.0)
    Us, Ss, Vs = [], [], []
    for i in range(b):
        U, S, V, _ = oracle.svd(A[i].astype(np.float64))
        Us.append(U); Ss.append(S); Vs.append(V)
    U32, S32, V32 = (np.stack(x).astype(np.float32) for x in (Us, Ss, Vs))
    dA = host(api.svd_bwd(dev(U32), dev(S32), dev(V32), dev(dU), dev(dS), dev(dV), eps_K=eK, eps_R=eR, eps_T=eT))
    for i in range(b):
        M = (U32[i].astype(np.float64) * S32[i]) @ V32[i].T.astype(np.float64)
        ref = oracle.svd_bwd(M, U32[i], S32[i], V32[i], dU[i], dS[i], dV[i], eK, eR, eT)
        rel = np.linalg.norm(dA[i] - ref) / np.linalg.norm(ref)
        _say(f"  b={i} rel={rel:.2e} |ref|={np.linalg.norm(ref):.3e}")
        assert rel < 1e-4


def test_polar_fwd_bwd_matches_oracle(api):
    _say("polar fwd/bwd 2 x 80 x 48")
    b, m, n = 2, 80, 48
    A, _ = inputs.batch_with_spectra(70, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-2, 1.0))
    W, H, S, V, info = api.polar_fwd(dev(A), cache=True)
    W, H, S, V = host(W), host(H), host(S), host(V)
    rng = inputs.rng_for(71, 0)
    dW = rng.standard_normal((b, m, n)).astype(np.float32)
    dH = rng.standard_normal((b, n, n)).astype(np.float32)
    for i in range(b):
        Uo, So, Vo, _ = oracle.svd(A[i].astype(np.float64))
        Wo, Ho = oracle.polar_from_svd(Uo, So, Vo)
        _say(f"  b={i} W_err={np.abs(W[i]-Wo).max():.2e} H_err={np.abs(H[i]-Ho).max():.2e} "
             f"S_err={np.abs(S[i]-So).max():.2e}")
        assert np.abs(W[i] - Wo).max() < 1e-4
        assert np.abs(H[i] - Ho).max() < 1e-5
        assert np.abs(S[i] - So).max() < 1e-5
    # backward with the oracle's H (cache from the GPU and without cache)
    Hs = np.stack([oracle.polar_from_svd(*oracle.svd(A[i].astype(np.float64))[:3])[1] for i in range(b)])
    H32 = Hs.astype(np.float32)
    for use_cache in (True, False):
        if use_cache:
            lam, Vc, _ = api.eigh(dev(H32))
            dA = host(api.polar_bwd(dev(A), None, lam, Vc, dev(dW), dev(dH)))
        else:
            dA = host(api.polar_bwd(dev(A), dev(H32), None, None, dev(dW), dev(dH)))
        for i in range(b):
            ref = oracle.polar_bwd(A[i], H32[i], dW[i], dH[i], 0.0, 0.0)
            rel = np.linalg.norm(dA[i] - ref) / np.linalg.norm(ref)
            _say(f"  cache={use_cache} b={i} rel={rel:.2e}")
            assert rel < 1e-3


# ------------------------------------------------------------------ predictor pieces

def test_features_match_oracle(api):
    _say("features 3 x 70 x 50")
    b, m, n = 3, 70, 50
    A, _ = inputs.batch_with_spectra(80, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-3, 1.0))
    g = inputs.probe(80, b, n)
    F, aux = api.bound_features(dev(A), dev(g))
    F, aux = host(F), host(aux)
    for i in range(b):
        f, r7, fro = oracle.sketch_features(A[i], g[i])
        _say(f"  b={i} f_err={np.abs(F[i]-f).max():.2e}")
        np.testing.assert_allclose(F[i], f, atol=2e-4)
        np.testing.assert_allclose(aux[i], [r7, fro], rtol=1e-5)


@pytest.mark.parametrize("scale", [1e-3, 1e3, 1e5])
def test_features_scale_equivariant(api, scale):
    """The power sequence (A^T A)^k A g grows as sigma_1^(2k+1): at sigma_1 ~ 1e3
    and n = 2048 its squared norms exceed the FP32 range.  The features are
    ratios, so they must not depend on the scale of A; the sigma_max estimate
    and |A|_F scale with it.  Checked against the FP64 oracle at each scale."""
    _say(f"features 2 x 300 x 256 at scale {scale:g}")
    b, m, n = 2, 300, 256
    A, _ = inputs.batch_with_spectra(81, b, m, n, lambda r: inputs.log_uniform(r, n, 1e-3, 1.0))
    As = (A.astype(np.float64) * scale).astype(np.float32)
    g = inputs.probe(81, b, n)
    F, aux = api.bound_features(dev(As), dev(g))
    F, aux = host(F), host(aux)
    for i in range(b):
        f, r7, fro = oracle.sketch_features(As[i].astype(np.float64), g[i])
        _say(f"  b={i} f_err={np.abs(F[i] - f).max():.2e} aux {aux[i]} oracle {[r7, fro]}")
        assert np.all(np.isfinite(F[i])) and np.all(np.isfinite(aux[i]))
        np.testing.assert_allclose(F[i], f, atol=2e-4)
        np.testing.assert_allclose(aux[i], [r7, fro], rtol=1e-5)


def test_learned_path_large_scale_no_fallback(api):
    """A learned-path SVD of 1024 A equals 1024 times that of A, with the same
    schedule and no fallback: the features that pick the schedule are
    scale-free (a power-of-two scale keeps every FP32 value exactly scaled;
    before the power sequence was normalised its squared norms overflowed
    here)."""
    import torch
    from paper_2609_32505_amd import predictor
    _say("learned BF16 SVD of A and 1024 A, 4 x 512^2")
    A, s = inputs.square_loguniform(seed=82, batch=4, n=512)
    probe = dev(inputs.probe(82, 4, 512))
    h = api.Handle()
    h.set_model(predictor.load())
    out = []
    for c in (1.0, 1024.0):
        U, S, V, info = api.svd_fwd(dev(A * np.float32(c)), handle=h, precision=1, bound=1, probe=probe)
        torch.cuda.synchronize()
        inf = api.info_to_numpy(info)
        _say(f"  scale {c:g}: flags {inf['flags']}, iters {inf['iters']}")
        assert not np.any(inf["flags"] & 2)
        out.append((host(S) / c, inf["iters"]))
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert (np.abs(out[0][0] - out[1][0]).max(axis=1) / out[0][0][:, 0]).max() < 1e-5


def test_mlp_fwd_bwd_adam_match_oracle(api):
    import torch
    _say("mlp fwd/bwd/pinball/adam")
    rng = np.random.default_rng(90)
    P = (rng.standard_normal(oracle.N_PARAMS) * 0.2).astype(np.float32)
    X = rng.standard_normal((77, 8)).astype(np.float32)
    mu = rng.standard_normal(8).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, 8).astype(np.float32)
    T = rng.standard_normal((77, 2)).astype(np.float32)
    out, act = api.mlp_fwd(dev(P), dev(X), dev(mu), dev(sd))
    Xs = (X.astype(np.float64) - mu) / sd
    ref, cache = oracle.mlp_forward(P, Xs)
    np.testing.assert_allclose(host(out), ref, rtol=1e-5, atol=1e-5)
    dout, loss = api.pinball(out, dev(T), 0.9, 0.1)
    Lr, Gr = oracle.pinball_loss(host(out), T, [0.9, 0.1])
    np.testing.assert_allclose(host(dout), Gr, rtol=1e-6, atol=1e-9)
    assert float(loss.item()) == pytest.approx(Lr, rel=1e-5)
    dP = api.mlp_bwd(dev(P), dev(X), act, dout, dev(mu), dev(sd))
    gref = oracle.mlp_backward(P, cache, Gr)
    rel = np.linalg.norm(host(dP) - gref) / np.linalg.norm(gref)
    _say(f"  grad rel={rel:.2e}")
    assert rel < 1e-5
    p = dev(P); m1 = torch.zeros_like(p); v1 = torch.zeros_like(p)
    pn, mn, vn = P.astype(np.float64), np.zeros(P.size), np.zeros(P.size)
    for t in (1, 2, 3):
        api.adam_step(p, m1, v1, dP, t, 1e-3)
        pn, mn, vn = oracle.adam_step(pn, mn, vn, host(dP), t, 1e-3)
    np.testing.assert_allclose(host(p), pn, rtol=1e-6, atol=1e-7)


# ------------------------------------------------------------------ error handling

def test_errors_and_flags(api):
    import torch
    from paper_2609_32505_amd._lib import SvdpError
    _say("errors and flags")
    with pytest.raises(SvdpError, match="bad shape"):
        api.svd_fwd(torch.zeros((1, 4, 8), device="cuda"))
    with pytest.raises(SvdpError, match="no model"):
        api.svd_fwd(torch.zeros((1, 8, 8), device="cuda"), bound=1, handle=api.Handle(),
                    probe=torch.zeros((1, 8), device="cuda"))
    A = np.tile(np.eye(16, dtype=np.float32), (2, 1, 1))
    A[1, 3, 4] = np.nan
    U, S, V, info = api.svd_fwd(dev(A))
    inf = api.info_to_numpy(info)
    assert inf["flags"][0] == 0 and inf["flags"][1] & 16
    np.testing.assert_allclose(host(S)[0], 1.0, atol=1e-6)
    # one CANS step only: reported as not converged
    A2, _ = inputs.single_64()
    _, _, _, info2 = api.svd_fwd(dev(A2), max_iters=2)
    assert api.info_to_numpy(info2)["flags"][0] & 1


@pytest.mark.parametrize("eps", [0.0, 1e-8])
def test_eigh_bwd_matches_oracle(api, eps):
    # the EVD pseudo-gradient on the GPU's own eigenpairs vs the FP64 oracle
    _say(f"eigh bwd 3 x 96, eps_K={eps}")
    rng = inputs.rng_for(98, 0)
    X = rng.standard_normal((3, 96, 96))
    H = 0.5 * (X + X.transpose(0, 2, 1))
    lam, V, info = api.eigh(dev(H))
    dlam = rng.standard_normal((3, 96))
    dV = rng.standard_normal((3, 96, 96))
    dH = api.eigh_bwd(lam, V, dev(dlam), dev(dV), eps_K=eps).cpu().double().numpy()
    lh, Vh = lam.cpu().double().numpy(), V.cpu().double().numpy()
    for i in range(3):
        ref = oracle.eigh_bwd(lh[i], Vh[i], dlam[i], dV[i], eps_K=eps)
        rel = np.linalg.norm(dH[i] - ref) / np.linalg.norm(ref)
        _say(f"  b={i} rel={rel:.2e} |ref|={np.linalg.norm(ref):.3e} asym={np.abs(dH[i] - dH[i].T).max():.1e}")
        assert rel < 1e-4


def test_autograd_eigh(api):
    import torch
    from paper_2609_32505_amd import autograd
    _say("autograd eigh 2 x 40")
    rng = inputs.rng_for(99, 0)
    X = rng.standard_normal((2, 40, 40))
    H = dev(0.5 * (X + X.transpose(0, 2, 1))).requires_grad_(True)
    lam, V = autograd.eigh(H)
    g, G = rng.standard_normal((2, 40)), rng.standard_normal((2, 40, 40))
    ((lam * dev(g)).sum() + (V * dev(G)).sum()).backward()
    got = H.grad.cpu().double().numpy()
    lh, Vh = lam.detach().cpu().double().numpy(), V.detach().cpu().double().numpy()
    for i in range(2):
        ref = oracle.eigh_bwd(lh[i], Vh[i], g[i], G[i])
        assert np.linalg.norm(got[i] - ref) / np.linalg.norm(ref) < 1e-4
