"""FP64 CPU oracle for differentiable SVD via polar decomposition.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark import this package.  The GPU library and its
Python binding never import it, and it imports nothing from them.

Contents (each function cites the passage of the paper it follows):

* C part (``oracle.c``, FP64, plain loops, built into ``liborc.so``):
  one-sided Jacobi SVD, two-sided Jacobi eigh, Algorithm 4 (SVD backward),
  Algorithm 2 (polar backward), the classical full-rank SVD backward.
* numpy part (FP64): the normalisation of the appendix on Newton-Schulz
  initialisation (Algorithm 3), the degree-3 CANS polynomial and its
  interval recursion, the CANS polar iteration, the iteration variants of
  the appendix's polar-iteration ablation (classical Newton-Schulz, the
  degree-5 interval-optimal polynomial, the Polar Express schedule), the
  symmetric EVD backward (the EVD pseudo-gradient theorem), and for the
  learned interval predictor its sketch features, training targets, feature
  standardisation and the small MLP (forward, backward, pinball loss, Adam).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, invariants, brute force or
finite differences, except where a docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liborc.so`` with gcc and OpenMP."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
               os.path.join(_HERE, "oracle.c"), "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.orc_svd.argtypes = [I, I, P, P, P, P]
        lib.orc_svd.restype = I
        lib.orc_eigh.argtypes = [I, P, P, P]
        lib.orc_eigh.restype = I
        lib.orc_svd_bwd.argtypes = [I, I, P, P, P, P, P, P, P, D, D, D, P]
        lib.orc_polar_bwd.argtypes = [I, I, P, P, P, P, D, D, P]
        lib.orc_townsend.argtypes = [I, I, P, P, P, P, P, P, P]
        lib.orc_svd_batch.argtypes = [I, I, I, P, P, P, P, P, I]
        lib.orc_svd_bwd_batch.argtypes = [I, I, I, P, P, P, P, P, P, P, D, D, D, P, I]
        lib.orc_num_threads.restype = I
        _lib = lib
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --------------------------------------------------------------------------
# SVD / eigh / polar factors
# --------------------------------------------------------------------------

def svd(A):
    """Thin SVD of one m x n matrix (m >= n) by one-sided Jacobi in FP64.

    Returns (U, S, V, sweeps) with S descending and V (not V^T); see the SVD
    definition next to the polar-decomposition definition of the paper.
    """
    A = _f64(A)
    m, n = A.shape
    U = np.zeros((m, n)); S = np.zeros(n); V = np.zeros((n, n))
    sw = _load().orc_svd(m, n, _ptr(A), _ptr(U), _ptr(S), _ptr(V))
    return U, S, V, sw


def svd_batch(A, threads: int = 0):
    """Batched ``svd`` over a (b, m, n) array, one matrix per OpenMP thread."""
    A = _f64(A)
    b, m, n = A.shape
    U = np.zeros((b, m, n)); S = np.zeros((b, n)); V = np.zeros((b, n, n))
    sw = np.zeros(b, dtype=np.int32)
    _load().orc_svd_batch(b, m, n, _ptr(A), _ptr(U), _ptr(S), _ptr(V), _ptr(sw), threads)
    return U, S, V, sw


def eigh(H):
    """Symmetric eigendecomposition by two-sided cyclic Jacobi in FP64.

    Returns (lam descending, V, sweeps) with H = V diag(lam) V^T.
    """
    H = _f64(H)
    n = H.shape[0]
    lam = np.zeros(n); V = np.zeros((n, n))
    sw = _load().orc_eigh(n, _ptr(H), _ptr(lam), _ptr(V))
    return lam, V, sw


def polar_from_svd(U, S, V):
    """W = U V^T and H = V Sigma V^T (the SVD-to-polar identity, Sec. 2)."""
    W = U @ V.T
    H = (V * S) @ V.T
    return W, H


# --------------------------------------------------------------------------
# backward passes
# --------------------------------------------------------------------------

def eigh_bwd(lam, V, dlam=None, dV=None, eps_K: float = 0.0):
    """Backward of the symmetric EVD H = V diag(lam) V^T: the EVD
    pseudo-gradient theorem (Section 4.2), literal, in FP64.
    K_ij = 1 / (lam_i - lam_j) when lam_i != lam_j and 0 otherwise; with
    eps_K > 0 the regularised K_ij = (lam_i - lam_j) / ((lam_i - lam_j)^2 + eps_K)
    of the same section (eps_K plays the role of eps^2).  Then
    S = K^T o (V^T dV - dV^T V) / 2 and dH = V (S + diag(dlam)) V^T."""
    lam = np.asarray(lam, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n = lam.shape[0]
    d = lam[:, None] - lam[None, :]
    if eps_K > 0:
        K = d / (d * d + eps_K)
    else:
        K = np.zeros((n, n))
        nz = d != 0
        K[nz] = 1.0 / d[nz]
    np.fill_diagonal(K, 0.0)
    P = np.zeros((n, n)) if dV is None else V.T @ np.asarray(dV, dtype=np.float64)
    S = 0.5 * K.T * (P - P.T)
    if dlam is not None:
        S = S + np.diag(np.asarray(dlam, dtype=np.float64))
    return V @ S @ V.T


def paper_eps(eps: float, k_exponent: str = "alg4"):
    """Map the paper's single eps to the three absolute regularisers.

    Algorithm 4 regularises K with eps^(1/2), R with eps^(1/2) and T with
    eps^(1/4); the main text writes K with eps^2.  ``k_exponent`` picks
    "alg4" (eps^(1/2)) or "main" (eps^2) for K.
    """
    eK = eps ** 0.5 if k_exponent == "alg4" else eps ** 2
    return eK, eps ** 0.5, eps ** 0.25


def svd_bwd(M, U, S, V, dU=None, dS=None, dV=None, eK=0.0, eR=0.0, eT=0.0):
    """Algorithm 4 backward, literal, FP64.  dV is the gradient of V."""
    M, U, S, V = _f64(M), _f64(U), _f64(S), _f64(V)
    dU, dS, dV = _f64(dU), _f64(dS), _f64(dV)
    m, n = M.shape
    dM = np.zeros((m, n))
    _load().orc_svd_bwd(m, n, _ptr(M), _ptr(U), _ptr(S), _ptr(V), _ptr(dU), _ptr(dS),
                        _ptr(dV), float(eK), float(eR), float(eT), _ptr(dM))
    return dM


def svd_bwd_batch(M, U, S, V, dU=None, dS=None, dV=None, eK=0.0, eR=0.0, eT=0.0,
                  threads: int = 0):
    M, U, S, V = _f64(M), _f64(U), _f64(S), _f64(V)
    dU, dS, dV = _f64(dU), _f64(dS), _f64(dV)
    b, m, n = M.shape
    dM = np.zeros((b, m, n))
    _load().orc_svd_bwd_batch(b, m, n, _ptr(M), _ptr(U), _ptr(S), _ptr(V), _ptr(dU),
                              _ptr(dS), _ptr(dV), float(eK), float(eR), float(eT),
                              _ptr(dM), threads)
    return dM


def polar_bwd(M, H, dW=None, dH=None, eR=0.0, eT=0.0):
    """Algorithm 2 (regularised polar backward), literal, FP64.

    With eR = eT = 0 it is the exact backward of the polar-decomposition
    theorem (full-rank M).
    """
    M, H, dW, dH = _f64(M), _f64(H), _f64(dW), _f64(dH)
    m, n = M.shape
    dM = np.zeros((m, n))
    _load().orc_polar_bwd(m, n, _ptr(M), _ptr(H), _ptr(dW), _ptr(dH), float(eR),
                          float(eT), _ptr(dM))
    return dM


def townsend_bwd(U, S, V, dU=None, dS=None, dV=None):
    """Classical full-rank SVD backward (existing-formulas appendix, k = n)."""
    U, S, V = _f64(U), _f64(S), _f64(V)
    dU, dS, dV = _f64(dU), _f64(dS), _f64(dV)
    m, n = U.shape
    dA = np.zeros((m, n))
    _load().orc_townsend(m, n, _ptr(U), _ptr(S), _ptr(V), _ptr(dU), _ptr(dS), _ptr(dV),
                         _ptr(dA))
    return dA


# --------------------------------------------------------------------------
# normalisation and the CANS polar iteration (FP64, numpy)
# --------------------------------------------------------------------------

def ns_normaliser(A):
    """sqrt(||A||_1 ||A||_inf), the bound on ||A||_2 used to scale X0
    (appendix on Newton-Schulz initialisation, Algorithm 3)."""
    A = np.asarray(A, dtype=np.float64)
    n1 = np.abs(A).sum(axis=0).max()    # max column abs sum
    ninf = np.abs(A).sum(axis=1).max()  # max row abs sum
    return float(np.sqrt(n1 * ninf))


def cans_poly(a: float, b: float):
    """Odd cubic p(x) = alpha x + beta x^3 closest to 1 in max norm on [a, b].

    The CANS polynomial is cited, not defined, in the paper; this reading
    takes the degree-3 Chebyshev-optimal (equioscillating) polynomial: the
    error 1 - p has equal magnitude E, alternating sign, at a, at the interior
    stationary point x* and at b.  Writing s = a^2 + ab + b^2: equal values
    at a and b give alpha = -beta s, stationarity gives x*^2 = s / 3, and
    p(a) + p(x*) = 2 gives beta = -2 / (ab(a + b) + 2 x*^3).
    Returns (alpha, beta, lo, hi) with [lo, hi] = [1 - E, 1 + E] the image
    interval.
    """
    a = float(a); b = float(b)
    s = a * a + a * b + b * b
    xs = np.sqrt(s / 3.0)
    beta = -2.0 / (a * b * (a + b) + 2.0 * xs ** 3)
    alpha = -beta * s
    lo = alpha * a + beta * a ** 3
    hi = alpha * xs + beta * xs ** 3
    return alpha, beta, lo, hi


def cans_preprocess_t(delta: float = 0.99, steps: int = 2):
    """Smallest t such that `steps` interval-optimal steps starting on [t, 1]
    land inside [1 - delta, 1 + delta] (CANS preprocessing, delta ablation
    appendix).  Found by bisection on t (the image error grows as t falls)."""
    def err(t):
        a, b = t, 1.0
        for _ in range(steps):
            _, _, a, b = cans_poly(a, b)
        return max(1.0 - a, b - 1.0)
    lo, hi = 1e-16, 1.0
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if err(mid) <= delta:
            hi = mid
        else:
            lo = mid
    return hi


def cans_schedule_conservative(delta: float = 0.99, pre_steps: int = 2, max_iters: int = 50):
    """Coefficient table of the conservative path: `pre_steps` optimal steps on
    [t, 1] (t from ``cans_preprocess_t``), then optimal steps on the interval
    recursion started at [1 - delta, 1 + delta] (Sec. 3 CANS hyperparameters;
    delta ablation appendix).  Returns a (max_iters, 2) array of (alpha, beta).
    """
    t = cans_preprocess_t(delta, pre_steps)
    out = []
    a, b = t, 1.0
    for _ in range(pre_steps):
        al, be, a, b = cans_poly(a, b)
        out.append((al, be))
    a, b = 1.0 - delta, 1.0 + delta
    while len(out) < max_iters:
        al, be, a, b = cans_poly(a, b)
        out.append((al, be))
    return np.array(out)


def cans_schedule_interval(lo: float, max_iters: int = 50):
    """Coefficients of interval-optimal steps started on [lo, 1] (learned or
    user bound path).  Returns (table (max_iters, 2), list of image errors)."""
    out, errs = [], []
    a, b = float(lo), 1.0
    for _ in range(max_iters):
        al, be, a, b = cans_poly(a, b)
        out.append((al, be))
        errs.append(max(1.0 - a, b - 1.0))
    return np.array(out), errs


def cans5_poly(a: float, b: float):
    """Odd quintic p(x) = c1 x + c3 x^3 + c5 x^5 closest to 1 in max norm on
    [a, b]: the degree-5 member of the interval-optimal family (the appendix's
    ablation of polar iterations; "higher-degree CANS").  Chebyshev's
    alternation theorem fixes it by equioscillation of the error 1 - p at four
    points a < x1 < x2 < b with signs (+, -, +, -), x1 and x2 stationary.
    Solved here as that nonlinear system in (c1, c3, c5, E, x1, x2) by
    Newton's method (scipy's hybrid solver).  A very narrow interval takes the
    limit q(x / x0) with q(u) = (15 u - 10 u^3 + 3 u^5) / 8 (p(x0) = 1,
    p'(x0) = p''(x0) = 0).  Returns (c1, c3, c5, lo, hi), [lo, hi] the image
    of [a, b]."""
    from scipy.optimize import fsolve
    a = float(a); b = float(b)
    if b - a <= 1e-6 * b:
        x0 = 0.5 * (a + b)
        c = (15.0 / (8.0 * x0), -10.0 / (8.0 * x0 ** 3), 3.0 / (8.0 * x0 ** 5))
        p = lambda x: c[0] * x + c[1] * x ** 3 + c[2] * x ** 5
        return c[0], c[1], c[2], p(a), p(b)

    def p(c, x):
        return c[0] * x + c[1] * x ** 3 + c[2] * x ** 5

    def dp(c, x):
        return c[0] + 3 * c[1] * x ** 2 + 5 * c[2] * x ** 4

    # work in u = x / b so that the system is scaled
    ua = a / b

    def eqs(z):
        c1, c3, c5, E, u1, u2 = z
        c = (c1, c3, c5)
        return [1 - p(c, ua) - E, 1 - p(c, u1) + E, 1 - p(c, u2) - E, 1 - p(c, 1.0) + E, dp(c, u1), dp(c, u2)]

    u1 = ua + (1 - ua) * 0.25
    u2 = ua + (1 - ua) * 0.75
    pts = np.array([ua, u1, u2, 1.0])
    M = np.stack([pts, pts ** 3, pts ** 5, np.array([1.0, -1.0, 1.0, -1.0])], axis=1)
    c1, c3, c5, E = np.linalg.solve(M, np.ones(4))
    import warnings
    with warnings.catch_warnings():
        # near-degenerate (very narrow) intervals stop short of xtol at FP64 rounding
        warnings.simplefilter("ignore", RuntimeWarning)
        z = fsolve(eqs, [c1, c3, c5, E, u1, u2], xtol=1e-13, maxfev=20000)
    c1, c3, c5, E, u1, u2 = z
    # back to x: p(x) = q(x / b)
    c = (c1 / b, c3 / b ** 3, c5 / b ** 5)
    xs = [a, u1 * b, u2 * b, b]
    vals = [p(c, x) for x in xs]
    return c[0], c[1], c[2], min(vals[0], vals[2]), max(vals[1], vals[3])


def cans5_preprocess_t(delta: float = 0.99, steps: int = 2):
    """Smallest t such that `steps` optimal quintic steps from [t, 1] land in
    [1 - delta, 1 + delta] (bisection on t, as for the cubic)."""
    def err(t):
        a, b = t, 1.0
        for _ in range(steps):
            *_, a, b = cans5_poly(a, b)
        return max(1.0 - a, b - 1.0)
    lo, hi = 1e-16, 1.0
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if err(mid) <= delta:
            hi = mid
        else:
            lo = mid
    return hi


def poly_schedule_conservative(poly: int, delta: float = 0.99, pre_steps: int = 2, max_iters: int = 50):
    """Coefficients (c1, c3, c5) per step of the conservative path for an
    iteration polynomial: 0 the CANS cubic (c5 = 0), 1 classical Newton-Schulz
    (1.5, -0.5, 0) throughout (no preprocessing), 2 the CANS quintic with its
    preprocessing on [t, 1] and the interval recursion from [1 - delta,
    1 + delta].  Returns (table (max_iters, 3), t)."""
    if poly == 1:
        return np.tile([1.5, -0.5, 0.0], (max_iters, 1)), 0.0
    if poly == 0:
        tab = cans_schedule_conservative(delta, pre_steps, max_iters)
        return np.concatenate([tab, np.zeros((max_iters, 1))], axis=1), cans_preprocess_t(delta, pre_steps)
    t = cans5_preprocess_t(delta, pre_steps)
    out = []
    a, b = t, 1.0
    for _ in range(min(pre_steps, max_iters)):
        c1, c3, c5, a, b = cans5_poly(a, b)
        out.append((c1, c3, c5))
    a, b = 1.0 - delta, 1.0 + delta
    while len(out) < max_iters:
        c1, c3, c5, a, b = cans5_poly(a, b)
        out.append((c1, c3, c5))
    return np.array(out), t


def polar_express_schedule(lo: float = 1e-3, max_steps: int = 64):
    """Polar Express (cited by the appendix's ablation of polar iterations;
    the paper states that its polynomial input is divided by 1.01 on every
    step but the last).  Reading of the published construction: X0 = A /
    |A|_F, so the singular values lie in [lo, 1]; step t takes the odd quintic
    closest to 1 in max norm on the cushioned interval [max(l_t, u_t / 10),
    u_t] (``cans5_poly``) and applies it to X / 1.01; [l_t+1, u_t+1] is the
    image of [l_t / 1.01, u_t / 1.01], read here off a dense grid of 2e5
    points plus the ends; once u - l <= 1e-4 one undamped step ends the
    schedule.  Returns a (steps, 3) array of (c1, c3, c5) with the damping
    folded in (c_k / 1.01^k)."""
    damp, cushion = 1.01, 0.1
    l, u = float(lo), 1.0
    out = []
    for _ in range(max_steps):
        c1, c3, c5, _, _ = cans5_poly(max(l, cushion * u), u)
        if u - l <= 1e-4:
            out.append((c1, c3, c5))
            return np.array(out)
        out.append((c1 / damp, c3 / damp ** 3, c5 / damp ** 5))
        xs = np.concatenate([np.linspace(l / damp, u / damp, 200001), [l / damp, u / damp]])
        v = c1 * xs + c3 * xs ** 3 + c5 * xs ** 5
        l, u = float(v.min()), float(v.max())
    raise ValueError("schedule longer than max_steps")


def polar_express_polar(A, lo: float = 1e-3):
    """The Polar Express iteration in FP64: X0 = A / |A|_F, then the fixed
    schedule of ``polar_express_schedule`` (no stop test).  Returns (W, steps)."""
    A = np.asarray(A, dtype=np.float64)
    X = A / np.linalg.norm(A)
    tab = polar_express_schedule(lo)
    for c1, c3, c5 in tab:
        G = X.T @ X
        X = c1 * X + X @ (c3 * G + c5 * (G @ G))
    return X, len(tab)


def poly_polar(A, table, tol: float = 1e-5, max_iters: int = 64):
    """Polar iteration in FP64 with per-step odd polynomials
    X <- c1 X + c3 X G + c5 X G^2, G = X^T X (rows of `table`), after the
    Algorithm 3 scaling, with the stop test of the CANS iteration.
    Returns (W, iterations)."""
    A = np.asarray(A, dtype=np.float64)
    X = A / ns_normaliser(A)
    it = 0
    for k in range(min(max_iters, len(table))):
        c1, c3, c5 = table[k]
        G = X.T @ X
        Xn = c1 * X + X @ (c3 * G + c5 * (G @ G))
        it = k + 1
        done = np.linalg.norm(Xn - X) <= tol * np.linalg.norm(Xn)
        X = Xn
        if done:
            break
    return X, it


def cans_polar(A, table, tol: float = 1e-5, scale: float | None = None, max_iters: int = 50):
    """CANS polar iteration in FP64 (Algorithm 1, normalise + preprocess +
    iterate): X0 = A / scale, then X <- alpha_k X + beta_k X (X^T X) with the
    k-th row of `table`, stopping when ||X_new - X||_F <= tol ||X_new||_F.
    The scale defaults to the 1-norm / inf-norm bound of Algorithm 3.
    Returns (W, iterations)."""
    A = np.asarray(A, dtype=np.float64)
    X = A / (ns_normaliser(A) if scale is None else scale)
    it = 0
    for k in range(min(max_iters, len(table))):
        al, be = table[k]
        Xn = al * X + be * (X @ (X.T @ X))
        it = k + 1
        done = np.linalg.norm(Xn - X) <= tol * np.linalg.norm(Xn)
        X = Xn
        if done:
            break
    return X, it


# --------------------------------------------------------------------------
# learned interval predictor: sketch features and MLP (FP64, numpy)
# --------------------------------------------------------------------------

N_FEAT = 8
HID = 64
N_OUT = 2
N_PARAMS = HID * N_FEAT + HID + HID * HID + HID + N_OUT * HID + N_OUT  # 4866


def _features_from_norms(F, norms, m, n):
    r = [norms[k] / norms[k - 1] for k in range(1, 8)]
    f = ([np.log(F / r[6])] + [np.log(r[k] / r[k + 1]) for k in range(1, 6)]
         + [np.log(n), np.log(m / n)])
    return np.array(f), r[6], F


def sketch_features(A, g):
    """Cheap sketch features of one m x n matrix with probe g (length n).

    Power sequence y0 = g, y1 = A y0, y2 = A^T y1, ... alternating up to y7;
    r_k = |y_k| / |y_{k-1}| (lower bounds on sigma_max that rise towards it).
    Features: log(|A|_F / r_7), log(r_k / r_{k+1}) for k = 2..6, log(n),
    log(m / n).  All are invariant to scaling A.  Returns (features, r_7,
    |A|_F).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    y = np.asarray(g, dtype=np.float64)
    norms = [np.linalg.norm(y)]
    for k in range(1, 8):
        y = A @ y if k % 2 == 1 else A.T @ y
        norms.append(np.linalg.norm(y))
    return _features_from_norms(np.linalg.norm(A), norms, m, n)


def spectral_features(s, z, m: int):
    """The same features for A = Q1 diag(s) Q2^T and g = Q2 z: then
    |y_k| = |s^k * z| exactly, so they depend only on (s, z)."""
    s = np.asarray(s, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = s.shape[0]
    norms = [np.linalg.norm(s ** k * z) for k in range(8)]
    return _features_from_norms(np.linalg.norm(s), norms, m, n)


def training_targets(s, r7):
    """Regression targets of the interval predictor for a spectrum s and its
    power-sequence estimate r_7: (log(sigma_max / r_7), log(sigma_max /
    sigma_min)), i.e. how far the cheap estimate sits below sigma_max and the
    log condition number; the learned bound of Section 3 is sigma_max <=
    r_7 exp(t_1), sigma_min >= sigma_max exp(-t_2).  sigma_min is clamped at
    1e-30 so that singular spectra give a finite target."""
    s = np.asarray(s, dtype=np.float64)
    smax = s.max()
    smin = max(s.min(), 1e-30)
    return np.array([np.log(smax / float(r7)), np.log(smax / smin)])


def feature_stats(F):
    """Standardisation of the predictor's inputs: per column of F (rows x 8)
    the mean and the sample standard deviation (divisor rows - 1), the latter
    clamped at 1e-3 so that a constant feature (log(m / n) on square-only
    data) does not divide by zero."""
    F = np.asarray(F, dtype=np.float64)
    rows = F.shape[0]
    mu = F.sum(axis=0) / rows
    var = ((F - mu) ** 2).sum(axis=0) / max(rows - 1, 1)
    return mu, np.maximum(np.sqrt(var), 1e-3)


def mlp_unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    def take(k, shape):
        nonlocal o
        v = p[o:o + k].reshape(shape); o += k
        return v
    W1 = take(HID * N_FEAT, (HID, N_FEAT)); b1 = take(HID, (HID,))
    W2 = take(HID * HID, (HID, HID)); b2 = take(HID, (HID,))
    W3 = take(N_OUT * HID, (N_OUT, HID)); b3 = take(N_OUT, (N_OUT,))
    return W1, b1, W2, b2, W3, b3


def mlp_forward(p, X):
    """8 -> 64 -> 64 -> 2 MLP with tanh hidden layers, rows of X are inputs.
    Returns (out (rows, 2), cache)."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    out = h2 @ W3.T + b3
    return out, (X, h1, h2)


def mlp_backward(p, cache, dout):
    """Gradient of sum(dout * out) with respect to the flat parameters
    (chain rule through the two tanh layers)."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(p)
    X, h1, h2 = cache
    dout = np.asarray(dout, dtype=np.float64)
    gW3 = dout.T @ h2; gb3 = dout.sum(0)
    d2 = (dout @ W3) * (1.0 - h2 ** 2)
    gW2 = d2.T @ h1; gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - h1 ** 2)
    gW1 = d1.T @ X; gb1 = d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def pinball_loss(out, target, taus):
    """Mean over rows of sum_j rho_tau_j(target_j - out_j) with
    rho_tau(u) = max(tau u, (tau - 1) u).  Returns (loss, dloss/dout)."""
    out = np.asarray(out, dtype=np.float64)
    u = np.asarray(target, dtype=np.float64) - out
    taus = np.asarray(taus, dtype=np.float64)[None, :]
    rows = out.shape[0]
    loss = np.maximum(taus * u, (taus - 1.0) * u).sum() / rows
    grad = np.where(u < 0, 1.0 - taus, -taus) / rows
    return loss, grad


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015) with bias correction; returns new
    (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
