"""Seeded synthetic inputs (FP64 generation, FP32 storage).

This module holds no arithmetic of the method: it only draws random matrices
with prescribed singular values, following the paper's matrix generation
scheme (appendix on implementation details: Gaussian matrices, thin QR
factors, M = Q1 Sigma Q2^T), and the spectra of the workloads.  Both the GPU
tests/benchmark and the oracle checks take their inputs from here.

Every generator takes an explicit seed; matrix i of a batch uses the PCG64
stream seeded with (seed, i), so any single matrix can be regenerated alone.
"""
from __future__ import annotations

import numpy as np


def rng_for(seed: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(index)]))


def orthonormal(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Thin Q (m x n, m >= n) of a Householder QR of an N(0,1) matrix, with
    column signs fixed so that diag(R) > 0 (Haar-distributed)."""
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def matrix_with_spectrum(rng: np.random.Generator, m: int, n: int, s) -> np.ndarray:
    """A = Q1 diag(s) Q2^T with Q1 m x n, Q2 n x n Haar (FP64)."""
    s = np.asarray(s, dtype=np.float64)
    Q1 = orthonormal(rng, m, n)
    Q2 = orthonormal(rng, n, n)
    return (Q1 * s) @ Q2.T


# ----------------------------------------------------------------- spectra

def geometric(n: int, kappa: float) -> np.ndarray:
    """s_i = kappa^(-(i-1)/(n-1)), i = 1..n: from 1 down to 1/kappa."""
    if n == 1:
        return np.ones(1)
    return kappa ** (-np.arange(n) / (n - 1.0))


def log_uniform(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """n values log-uniform in [lo, hi], sorted descending, with the two ends
    pinned to hi and lo exactly."""
    if n == 1:
        return np.array([hi])
    s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))
    s = np.sort(s)[::-1].copy()
    s[0], s[-1] = hi, lo
    return s


def clustered_pairs(n: int, kappa: float = 1e3, first: int = 8, step: int = 16,
                    gap: float = 1e-6) -> np.ndarray:
    """Geometric spectrum 1..1/kappa with disjoint pairs (i, i+1) at 1-based
    i = first, first + step, ...; pairs alternate between exactly equal and
    separated by `gap` (absolute)."""
    s = geometric(n, kappa)
    exact = True
    for i in range(first - 1, n - 1, step):
        s[i + 1] = s[i] if exact else s[i] - gap
        exact = not exact
    return s


def paper_kappa_rank(n: int, kappa: float, rank: int | None = None) -> np.ndarray:
    """The paper's kappa/rank scheme: Sigma_ii = kappa^((r - i)/(r - 1)) for
    i <= r (from kappa down to 1), 0 beyond the rank r."""
    r = n if rank is None else rank
    s = np.zeros(n)
    if r == 1:
        s[0] = 1.0
    else:
        i = np.arange(1, r + 1)
        s[:r] = kappa ** ((r - i) / (r - 1.0))
    return s


def paper_gap(n: int, gap: float) -> np.ndarray:
    """The paper's spectral-gap scheme: Sigma_ii = i for i < n and
    Sigma_nn = n - 1 + gap, returned in descending order."""
    s = np.arange(1, n + 1, dtype=np.float64)
    s[-1] = n - 1 + gap
    return np.sort(s)[::-1].copy()


# --------------------------------------------------------------- workloads

def batch_with_spectra(seed: int, batch: int, m: int, n: int, spectrum_fn):
    """Batch of FP32 matrices; spectrum_fn(rng) -> s (length n).  Returns
    (A float32 (batch, m, n), s float64 (batch, n))."""
    A = np.empty((batch, m, n), dtype=np.float32)
    S = np.empty((batch, n))
    for i in range(batch):
        rng = rng_for(seed, i)
        s = np.asarray(spectrum_fn(rng), dtype=np.float64)
        A[i] = matrix_with_spectrum(rng, m, n, s).astype(np.float32)
        S[i] = s
    return A, S


def generating_factors(seed: int, index: int, m: int, n: int, spectrum_fn):
    """(Q1, s, Q2) of matrix `index` of ``batch_with_spectra(seed, ...)``:
    the same draws in the same order, FP64."""
    rng = rng_for(seed, index)
    s = np.asarray(spectrum_fn(rng), dtype=np.float64)
    Q1 = orthonormal(rng, m, n)
    Q2 = orthonormal(rng, n, n)
    return Q1, s, Q2


def single_64(seed: int = 1):
    """One 64 x 64 matrix, geometric spectrum from 1 to 1e-3."""
    return batch_with_spectra(seed, 1, 64, 64, lambda r: geometric(64, 1e3))


def square_loguniform(seed: int = 2, batch: int = 256, n: int = 512,
                      lo: float = 1e-3, hi: float = 1.0):
    """Batch of n x n matrices, spectrum log-uniform in [lo, hi]."""
    return batch_with_spectra(seed, batch, n, n, lambda r: log_uniform(r, n, lo, hi))


def tall_loguniform(seed: int = 3, batch: int = 16, m: int = 4096, n: int = 1024,
                    lo: float = 1e-4, hi: float = 1.0):
    return batch_with_spectra(seed, batch, m, n, lambda r: log_uniform(r, n, lo, hi))


def low_rank_plus_noise(seed: int = 4, batch: int = 16, m: int = 4096, n: int = 1024,
                        rank: int = 64, noise: float = 1e-3):
    """A = Q1[:, :r] diag(s_sig) Q2[:, :r]^T + noise * N(0, 1), s_sig
    log-uniform in [0.1, 1].  Returns (A float32, s_sig float64 (batch, r))."""
    A = np.empty((batch, m, n), dtype=np.float32)
    S = np.empty((batch, rank))
    for i in range(batch):
        rng = rng_for(seed, i)
        s = log_uniform(rng, rank, 0.1, 1.0)
        Q1 = orthonormal(rng, m, rank)
        Q2 = orthonormal(rng, n, rank)
        A[i] = ((Q1 * s) @ Q2.T + noise * rng.standard_normal((m, n))).astype(np.float32)
        S[i] = s
    return A, S


def clustered_backward(seed: int = 5, batch: int = 64, n: int = 256):
    """Batch of n x n matrices with the clustered-pairs spectrum plus upstream
    gradients dU, dS, dV ~ N(0, 1) (FP32)."""
    A, S = batch_with_spectra(seed, batch, n, n, lambda r: clustered_pairs(n))
    rng = rng_for(seed, 1 << 20)
    dU = rng.standard_normal((batch, n, n)).astype(np.float32)
    dS = rng.standard_normal((batch, n)).astype(np.float32)
    dV = rng.standard_normal((batch, n, n)).astype(np.float32)
    return A, S, dU, dS, dV


def probe(seed: int, batch: int, n: int) -> np.ndarray:
    """Gaussian probe vectors for the sketch features (batch, n), FP32."""
    return rng_for(seed, 1 << 21).standard_normal((batch, n)).astype(np.float32)


# ------------------------------------------------- spectra for the predictor

def predictor_spectrum(rng: np.random.Generator, n: int, family: int):
    """One training/evaluation spectrum (length n, descending) for the learned
    interval predictor and its aspect ratio m/n.

    family 0: geometric with kappa log-uniform in [1e2, 1e6];
    family 1: Marchenko-Pastur-like: singular values of a Gaussian
              (n / c) x n matrix, c uniform in [0.25, 1], scaled by
              1/sqrt(n / c) -- returned as the Gaussian matrix itself
              (the caller computes its spectrum with the method);
    family 2: low-rank-plus-noise: 64 values log-uniform in [0.1, 1] on top
              of a noise floor, returned as a matrix as well.
    A global scale log-uniform in [1e-3, 1e3] multiplies everything.
    Returns (kind, payload, m): kind "s" with payload the spectrum, or kind
    "A" with payload an FP64 matrix whose spectrum is needed.
    """
    scale = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e3))))
    if family == 0:
        kappa = float(np.exp(rng.uniform(np.log(1e2), np.log(1e6))))
        return "s", scale * geometric(n, kappa), n
    if family == 1:
        c = float(rng.uniform(0.25, 1.0))
        m = int(round(n / c))
        return "A", scale * rng.standard_normal((m, n)) / np.sqrt(m), m
    s = log_uniform(rng, 64, 0.1, 1.0)
    m = n
    Q1 = orthonormal(rng, m, 64)
    Q2 = orthonormal(rng, n, 64)
    A = (Q1 * s) @ Q2.T + 1e-3 * rng.standard_normal((m, n))
    return "A", scale * A, m
