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


def _correct(Y, lam, V, W, reg_exp=-10):
    """S~_ij = -2 skew(P)_ij t_ij, t_ij = s/(s^2 + (2^reg lam_max)^2), s = lam_i + lam_j;
    U = W V (I - S~/2), V (I + S~/2); sigma_i = P_ii + 2 sum_j skew(P)_ij^2 t_ij
    - 1/4 sum_j S~_ij^2 lam_j + pairwise 2x2 shifts of the symmetric coupling."""
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
    shift = np.where(hh > 0, np.sign(d + (d == 0)) * e * e / np.where(hh > 0, hh, 1), 0.0)
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
    # the symmetric-coupling shift for one pair is the exact 2 x 2 eigenvalue
    for a, b, e in ((1.0, 0.5, 0.1), (1e-3, 0.99e-3, 3e-6), (2.0, 2.0 - 1e-9, 1e-5)):
        P = np.array([[a, e], [e, b]])
        lam_true = np.sort(np.linalg.eigvalsh(P))[::-1]
        d = a - b
        hh = np.sqrt(d * d / 4 + e * e) + abs(d) / 2
        got = a + np.sign(d + (d == 0)) * e * e / hh
        assert abs(got - lam_true[0]) <= 1e-12 * abs(lam_true[0])
