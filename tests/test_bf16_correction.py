"""CPU check of the algebra behind the learned path's BF16 correction (the
first-order correction of a polar factor W = W_t (I + S), S skew): written
out in numpy from its derivation and checked against an exact SVD with a
planted skew error.  The GPU kernel is checked separately, against the FP64
oracle, by the learned-path GPU tests."""
import numpy as np
from scipy.linalg import expm


def _planted(n, delta, seed):
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.sort(10.0 ** rng.uniform(-3, 0, n))[::-1]
    A = (Q1 * s) @ Q2.T
    Sk = rng.standard_normal((n, n))
    Sk = (Sk - Sk.T) / 2
    Sk *= delta / np.abs(Sk).max()
    W = Q1 @ Q2.T @ expm(Sk)
    return A, s, W


def _factors(W, A):
    """Eigenpairs of sym(W^T A), sorted by |lambda| descending, and U = W V."""
    Y = W.T @ A
    lam, V = np.linalg.eigh((Y + Y.T) / 2)
    o = np.argsort(-np.abs(lam))
    lam, V = lam[o], V[:, o]
    return Y, lam, V, (W @ V) * np.sign(lam)


def _tie_sign(d):
    """sign(d_ij) for the pairwise shift; an exact tie (d = 0) gives the pair's
    two 2 x 2 eigenvalues in index order: +1 for i < j, -1 for i > j."""
    n = d.shape[0]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.where(d != 0, np.sign(d), np.where(i < j, 1.0, -1.0))


def _correct(Y, lam, V, W, reg_exp=-10, P=None):
    """S~_ij = -2 skew(P)_ij t_ij, t_ij = s/(s^2 + (2^reg lam_max)^2), s = lam_i + lam_j;
    U = W V (I - S~/2), V (I + S~/2); sigma_i = P_ii + 2 sum_j skew(P)_ij^2 t_ij
    - 1/4 sum_j S~_ij^2 lam_j + pairwise 2x2 shifts of the symmetric coupling."""
    if P is None:
        P = V.T @ Y @ V
    s = lam[:, None] + lam[None, :]
    reg = (2.0 ** reg_exp * np.abs(lam[0])) ** 2
    t = s / (s * s + reg)
    sk = (P - P.T) / 2
    st = -2 * sk * t
    e = (P + P.T) / 2
    np.fill_diagonal(e, 0.0)
    d = np.diag(P)[:, None] - np.diag(P)[None, :]
    hh = np.sqrt(d * d / 4 + e * e) + np.abs(d) / 2
    shift = np.where(hh > 0, _tie_sign(d) * e * e / np.where(hh > 0, hh, 1), 0.0)
    sig = np.abs(np.diag(P) + np.sum(2 * sk * sk * t, axis=1) - 0.25 * np.sum(st * st * lam[None, :], axis=1)
                 + np.sum(shift, axis=1))
    Mu = np.eye(len(lam)) - st / 2
    Uc = (W @ (V @ Mu)) * np.sign(lam)
    Vc = 2 * V - V @ Mu
    return Uc, np.minimum.accumulate(sig), Vc


def _recon(U, S, V, A):
    return np.linalg.norm((U * S) @ V.T - A) / np.linalg.norm(A)


def test_correction_removes_first_order_error():
    n = 96
    for delta in (2e-3, 5e-4):
        A, s, W = _planted(n, delta, seed=3)
        Y, lam, V, U = _factors(W, A)
        rec0 = _recon(U, np.abs(lam), V, A)
        rel0 = np.max(np.abs(np.abs(lam) - s) / s)
        Uc, Sc, Vc = _correct(Y, lam, V, W)
        rec1 = _recon(Uc, Sc, Vc, A)
        rel1 = np.max(np.abs(Sc - s) / s)
        orth = np.abs(Uc.T @ Uc - np.eye(n)).max()
        # first order removed: the reconstruction falls by at least 1 / (40 delta)
        assert rec0 > 0.2 * delta and rec1 < 40 * delta * rec0, (delta, rec0, rec1)
        # singular values relative to each value: second order removed
        assert rel1 < 0.05 * rel0 and rel1 < 2e-5, (delta, rel0, rel1)
        assert orth < delta * delta * 4


def test_correction_is_exact_without_error():
    # an exact polar factor: P is diagonal, the correction changes nothing
    n = 64
    A, s, W = _planted(n, 0.0, seed=4)
    Y, lam, V, U = _factors(W, A)
    Uc, Sc, Vc = _correct(Y, lam, V, W)
    assert np.abs(Uc - U).max() < 1e-10 and np.abs(Vc - V).max() < 1e-10
    np.testing.assert_allclose(Sc, s, rtol=1e-10)


def test_pairwise_shift_is_the_2x2_eigenvalue():
    # the symmetric-coupling shift for one pair is the exact 2 x 2 eigenvalue,
    # for both rows of the pair, including an exactly repeated diagonal
    for a, b, e in ((1.0, 0.5, 0.1), (1e-3, 0.99e-3, 3e-6), (2.0, 2.0 - 1e-9, 1e-5), (0.7, 0.7, 2e-4),
                    (0.7, 0.7, -2e-4)):
        P = np.array([[a, e], [e, b]])
        lam_true = np.sort(np.linalg.eigvalsh(P))[::-1]
        d = np.array([[0.0, a - b], [b - a, 0.0]])
        hh = np.sqrt(d * d / 4 + e * e) + np.abs(d) / 2
        sg = _tie_sign(d)
        got = [a + sg[0, 1] * e * e / hh[0, 1], b + sg[1, 0] * e * e / hh[1, 0]]
        assert abs(got[0] - lam_true[0]) <= 1e-12 * abs(lam_true[0]), (a, b, e, got, lam_true)
        assert abs(got[1] - lam_true[1]) <= 1e-12 * abs(lam_true[0]), (a, b, e, got, lam_true)


def test_correction_with_exactly_repeated_pair():
    # a planted skew error on a spectrum with an exactly repeated value: the
    # symmetric coupling left inside the pair must split into s + |e| and
    # s - |e|, not shift both values up
    n = 48
    rng = np.random.default_rng(11)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.sort(10.0 ** rng.uniform(-2, 0, n))[::-1]
    s[10] = s[11]
    A = (Q1 * s) @ Q2.T
    W = Q1 @ Q2.T
    Y = W.T @ A
    lam, V = np.linalg.eigh((Y + Y.T) / 2)
    o = np.argsort(-np.abs(lam))
    lam, V = lam[o], V[:, o]
    # a symmetric coupling e inside the repeated pair, with exactly equal
    # diagonal entries, as an eigensolver stopped early can leave it
    e = 1e-4 * s[10]
    P0 = V.T @ Y @ V
    P0[11, 11] = P0[10, 10]
    P0[10, 11] = P0[11, 10] = e
    Yp = V @ P0 @ V.T
    _, Sc, _ = _correct(Yp, np.diag(P0), V, W, P=P0)
    lam_true = np.sort(np.abs(np.linalg.eigvalsh((P0 + P0.T) / 2)))[::-1]
    assert abs(Sc[10] - lam_true[10]) < 1e-3 * e and abs(Sc[11] - lam_true[11]) < 1e-3 * e, (Sc[10:12], lam_true[10:12])
    # the rule that shifts both rows by +|e| would leave the smaller value 2|e| off
    assert abs(lam_true[10] - lam_true[11]) > 1.9 * e
