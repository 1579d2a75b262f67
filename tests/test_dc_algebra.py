"""CPU checks of the algebra behind the spectral divide and conquer
(svdp_eigh_dc and the single-matrix SVD's EVD step), in float64 numpy: the
split by the sign of M - sigma I (the polar factor of the shifted matrix),
the rank k of P = (I + W) / 2, the subspace iteration step that squares W's
error in the basis, Newton-Schulz keeping each block's span, the
zero-padded batch's padding eigenpairs told apart by their weight, and the
SVD's order by |lambda| with the signs kept for U = W V diag(sgn).  These
test the method's steps, not the GPU code, whose parity runs under -m gpu."""
import numpy as np

from paper_2609_32505_amd import inputs


def _sym(rng, n, lam):
    Q = inputs.orthonormal(rng, n, n)
    return (Q * lam) @ Q.T, Q


def _polar(X):
    U, _, Vt = np.linalg.svd(X, full_matrices=False)
    return U @ Vt


def _split(M, W, Om, ns_steps=3):
    """One split as the library takes it: Y = [P Om1, (I - P) Om2], its
    blocks' polar factors, one subspace iteration step, Newton-Schulz on
    each block (the second projected twice against the first), T = Q^T M Q."""
    n = M.shape[0]
    k = int(round(0.5 * (n + np.trace(W))))
    P = 0.5 * (np.eye(n) + W)
    cs = np.where(np.arange(n) < k, 1.0, -1.0)
    Y = 0.5 * (Om + (W @ Om) * cs)
    Q = np.empty_like(Y)
    Q[:, :k] = _polar(Y[:, :k])
    Y2 = Y[:, k:].copy()
    for _ in range(2):
        Y2 -= Q[:, :k] @ (Q[:, :k].T @ Y2)
    Q[:, k:] = _polar(Y2)
    Y = 0.5 * (Q + (W @ Q) * cs)

    def ns(X):
        for _ in range(ns_steps):
            X = 1.5 * X - 0.5 * X @ (X.T @ X)
        return X
    Q[:, :k] = ns(Y[:, :k])
    Y2 = Y[:, k:].copy()
    for _ in range(2):
        Y2 -= Q[:, :k] @ (Q[:, :k].T @ Y2)
    Q[:, k:] = ns(Y2)
    T = Q.T @ M @ Q
    return k, P, Q, 0.5 * (T + T.T)


def test_split_reproduces_the_eigendecomposition():
    rng = inputs.rng_for(900, 0)
    n = 96
    lam = rng.uniform(-1.0, 2.0, n)
    M, _ = _sym(rng, n, lam)
    sigma = np.trace(M) / n
    W = _polar(M - sigma * np.eye(n))
    k, P, Q, T = _split(M, W, rng.uniform(-1.0, 1.0, (n, n)))
    assert k == int(np.sum(lam > sigma))
    assert np.abs(P @ P - P).max() < 1e-12
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
    assert np.linalg.norm(T[:k, k:]) < 1e-12 * np.linalg.norm(T)
    # the two pieces solved shifted by their means, eigenvalues descending
    # with the part above sigma first, V = Q diag(V1, V2)
    lams, Vs = [], []
    for blk in (T[:k, :k], T[k:, k:]):
        mu = np.trace(blk) / blk.shape[0]
        l, v = np.linalg.eigh(blk - mu * np.eye(blk.shape[0]))
        lams.append(l[::-1] + mu)
        Vs.append(v[:, ::-1])
    lam_dc = np.concatenate(lams)
    V = np.hstack([Q[:, :k] @ Vs[0], Q[:, k:] @ Vs[1]])
    assert np.all(np.diff(lam_dc) <= 0)
    assert np.abs(lam_dc - np.sort(lam)[::-1]).max() < 1e-12
    assert np.abs((V * lam_dc) @ V.T - M).max() < 1e-12


def test_subspace_step_squares_the_error_of_w():
    """CANS's iterates are odd polynomials of the symmetric shifted piece, so
    W = g(M) and its error sits in its eigenvalues: g(lam) = sign(lam)
    (1 - eps h) with h in (0, 1].  P's wrong-side eigenvalues are then
    eps h / 2.  The dropped coupling of a basis from one pass of P is first
    order in eps, after the subspace iteration step second order.  (An error
    that does not commute with M is not squared: the step converges to P's
    own invariant subspace, which it moves at first order.)"""
    rng = inputs.rng_for(901, 0)
    n = 80
    lam = np.concatenate([rng.uniform(-1.0, -0.3, n // 2), rng.uniform(0.3, 1.0, n - n // 2)])
    M, Qm = _sym(rng, n, lam)
    h = rng.uniform(0.1, 1.0, n)
    Om = rng.uniform(-1.0, 1.0, (n, n))
    out = []
    for eps in (1e-3, 1e-4):
        W = (Qm * (np.sign(lam) * (1.0 - eps * h))) @ Qm.T
        k = n - n // 2
        cs = np.where(np.arange(n) < k, 1.0, -1.0)
        Y = 0.5 * (Om + (W @ Om) * cs)
        Q1 = _polar(Y[:, :k])
        one = np.linalg.norm(Q1.T @ M @ (np.eye(n) - Q1 @ Q1.T)) / np.linalg.norm(M)
        _, _, Q, T = _split(M, W, Om)
        two = np.linalg.norm(T[:k, k:]) / np.linalg.norm(T)
        out.append((one, two))
    (o1, t1), (o2, t2) = out
    assert 5 < o1 / o2 < 20          # first order: 10x for 10x smaller eps
    assert t1 / t2 > 50              # second order: about 100x
    assert t1 < 0.1 * o1


def test_newton_schulz_keeps_the_span():
    rng = inputs.rng_for(902, 0)
    n, k = 60, 25
    B = _polar(rng.standard_normal((n, k)))
    X = B @ (np.eye(k) + 1e-3 * rng.standard_normal((k, k)))   # near orthonormal, span(B)
    for _ in range(3):
        X = 1.5 * X - 0.5 * X @ (X.T @ X)
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-12
    assert np.linalg.norm(X - B @ (B.T @ X)) < 1e-12


def test_zero_padded_piece_eigenpairs_are_told_apart_by_weight():
    """A piece of size s inside a zero-padded P x P matrix: the padding's
    eigenvectors live in rows s.. and the piece's have no weight there, so
    the rule 'weight over rows s.. above 1/2' drops exactly P - s columns
    and keeps the piece's eigenpairs in the solver's order."""
    rng = inputs.rng_for(903, 0)
    s, P = 37, 64
    lam = rng.uniform(-1.0, 1.0, s)
    lam[np.abs(lam) < 1e-3] = 0.5
    Ms, _ = _sym(rng, s, lam)
    Mp = np.zeros((P, P))
    Mp[:s, :s] = Ms
    lp, Vp = np.linalg.eigh(Mp)
    lp, Vp = lp[::-1], Vp[:, ::-1]
    pad = np.sum(Vp[s:, :] ** 2, axis=0) > 0.5
    assert pad.sum() == P - s
    keep = np.nonzero(~pad)[0]
    assert np.abs(lp[keep] - np.sort(lam)[::-1]).max() < 1e-12
    V = Vp[:s, keep]
    assert np.abs((V * lp[keep]) @ V.T - Ms).max() < 1e-12


def test_order_by_magnitude_keeps_the_svd():
    """The SVD's EVD step from a value-ordered decomposition of H = W^T A:
    S = |lambda| descending, signs kept, V's columns permuted alike, then
    U = W V diag(sgn) and A = U S V^T."""
    rng = inputs.rng_for(904, 0)
    n = 50
    A = rng.standard_normal((n, n))
    W = _polar(A)
    H = W.T @ A
    H = 0.5 * (H + H.T)
    l, V = np.linalg.eigh(H)
    l, V = l[::-1].copy(), V[:, ::-1].copy()
    l[-3:] *= -1.0        # rounding-level negatives of a (near) singular H
    H2 = (V * l) @ V.T
    order = np.lexsort((np.arange(n), -np.abs(l)))
    S, sgn, V2 = np.abs(l)[order], np.sign(l[order]), V[:, order]
    sgn[sgn == 0] = 1.0
    assert np.all(np.diff(S) <= 0)
    U = (W @ V2) * sgn
    assert np.abs((U * S) @ V2.T - W @ H2).max() < 1e-12
    assert np.abs(U.T @ U - np.eye(n)).max() < 1e-12


def test_an_error_that_does_not_commute_with_m_is_not_squared():
    """W off by a generic symmetric error eps E: the subspace iteration step
    converges to P's own invariant subspace, which E moves at first order,
    so the dropped coupling stays first order in eps (the split relies on W
    being a function of the shifted piece)."""
    rng = inputs.rng_for(901, 0)
    n = 80
    lam = np.concatenate([rng.uniform(-1.0, -0.3, n // 2), rng.uniform(0.3, 1.0, n - n // 2)])
    M, _ = _sym(rng, n, lam)
    W0 = _polar(M)
    E = rng.standard_normal((n, n))
    E = 0.5 * (E + E.T)
    E /= np.linalg.norm(E, 2)
    Om = rng.uniform(-1.0, 1.0, (n, n))
    t = []
    for eps in (1e-3, 1e-4):
        _, _, _, T = _split(M, W0 + eps * E, Om)
        t.append(np.linalg.norm(T[n - n // 2:, :n - n // 2]) / np.linalg.norm(T))
    assert 5 < t[0] / t[1] < 20
