"""Training driver of the learned sigma-interval predictor.

The predictor maps the sketch features of a matrix (``svdp_bound_features``)
to (log(sigma_max / r_7), log(sigma_max / sigma_min)), from which the library
picks the CANS polynomials and step count (bound mode LEARNED); plain
conservative CANS is its fallback.  Every arithmetic step of training runs in
the library's kernels: spectral features, MLP forward/backward, the pinball
loss and Adam.  Python only draws the seeded spectra/probes and loops.

Training set: spectra of length 1024 from three families (geometric with
kappa log-uniform in [1e2, 1e7]; Marchenko-Pastur-like, i.e. singular values
of Gaussian (1024/c) x 1024 matrices computed by this library's SVD; rank-64
signal plus N(0, 1e-3^2) noise at m / n = 1, 2 and 4, also through this
library's SVD), each times
a global scale log-uniform in [1e-3, 1e3].  Features depend only on the
spectrum and a Gaussian probe (|y_k| = |s^k z| for bi-orthogonally invariant
matrices), so each row pairs a spectrum with a fresh probe, presented at
n = 512, 1024, 2048 or 4096 (decimated or geometrically interpolated) so
that the network sees how the power-step ratios scale with n.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import api, inputs

MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "bound_mlp.npy")
TAUS = (0.98, 0.98)  # upper quantiles: over-predict sigma_max and kappa (safe side)


def _resample(s: np.ndarray, n: int) -> np.ndarray:
    """Spectrum of length len(s) presented at length n (same range, same
    shape in log scale): decimation or geometric interpolation."""
    if n == len(s):
        return s
    x = np.linspace(0.0, 1.0, len(s))
    xn = np.linspace(0.0, 1.0, n)
    ls = np.log(np.maximum(s, 1e-300))
    return np.exp(np.interp(xn, x, ls))


def base_spectra_by_method(count_mp: int, count_lr: int, n: int, seed: int, device="cuda"):
    """Spectra of the two matrix families, computed by this library's SVD."""
    out = []
    aspect = [1.0, 0.75, 0.5, 0.25]
    per = max(1, count_mp // len(aspect))
    for gi, c in enumerate(aspect):
        m = int(round(n / c))
        G = np.stack([inputs.rng_for(seed, 1000 * gi + i).standard_normal((m, n)) / np.sqrt(m)
                      for i in range(per)]).astype(np.float32)
        _, S, _, _ = api.svd_fwd(torch.from_numpy(G).to(device))
        for s in S.cpu().double().numpy():
            out.append((np.abs(s), m / n, 1))
    # rank-64 signal plus N(0, 1e-3^2) noise, square and tall (m / n = 2, 4):
    # the noise floor of the spectrum, 1e-3 (sqrt(m) - sqrt(n)), rises with m / n
    lr_aspect = [1.0, 0.5, 0.25]
    for ai, c in enumerate(lr_aspect):
        m = int(round(n / c))
        A = []
        for i in range(ai, count_lr, len(lr_aspect)):
            rng = inputs.rng_for(seed + 1, i)
            sig = inputs.log_uniform(rng, 64, 0.1, 1.0)
            Q1 = inputs.orthonormal(rng, m, 64)
            Q2 = inputs.orthonormal(rng, n, 64)
            A.append(((Q1 * sig) @ Q2.T + 1e-3 * rng.standard_normal((m, n))).astype(np.float32))
        for k in range(0, len(A), 8):
            _, S, _, _ = api.svd_fwd(torch.from_numpy(np.stack(A[k:k + 8])).to(device))
            for s in S.cpu().double().numpy():
                out.append((np.abs(s), m / n, 2))
    return out


def training_rows(rows: int, n: int = 1024, seed: int = 0, bases=None, sizes=(512, 1024, 2048, 4096)):
    """Seeded (spectrum, probe, m/n) rows, grouped by presentation size.
    Returns {size: (s (r, size), z (r, size), m_over_n (r,))} as float32."""
    rng = np.random.default_rng(seed)
    groups = {k: ([], [], []) for k in sizes}
    for r in range(rows):
        fam = r % 3
        scale = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e3))))
        if fam == 0 or not bases:
            kappa = float(np.exp(rng.uniform(np.log(1e2), np.log(1e7))))
            s, mn = inputs.geometric(n, kappa), 1.0
        else:
            pool = [b for b in bases if b[2] == fam] or bases
            s, mn, _ = pool[int(rng.integers(len(pool)))]
        size = sizes[int(rng.integers(len(sizes)))]
        s = _resample(np.sort(s)[::-1] * scale, size)
        groups[size][0].append(s)
        groups[size][1].append(rng.standard_normal(size))
        groups[size][2].append(mn)
    out = {}
    for k, (S, Z, M) in groups.items():
        if S:
            out[k] = (np.asarray(S, np.float32), np.asarray(Z, np.float32), np.asarray(M, np.float32))
    return out


def features_targets(groups, device="cuda"):
    """Features (library kernel) and targets (log(smax / r7), log(smax / smin))."""
    Fs, Ts = [], []
    for size, (S, Z, M) in groups.items():
        s = torch.from_numpy(S).to(device)
        z = torch.from_numpy(Z).to(device)
        mn = torch.from_numpy(M).to(device)
        F, aux = api.spectral_features(s, z, mn)
        T = api.training_targets(s, aux)
        Fs.append(F)
        Ts.append(T)
    return torch.cat(Fs), torch.cat(Ts)


def train(F, T, steps: int = 3000, batch: int = 2048, lr: float = 2e-3, seed: int = 0,
          taus=TAUS, log_every: int = 0):
    """Train the 8-64-64-2 MLP with the library's kernels.  Returns the model
    vector (params + feature means + stds) as float32 numpy, and the losses."""
    dev = F.device
    mu, sd = api.feature_stats(F)
    g = torch.Generator(device="cpu").manual_seed(seed)
    P = torch.empty(4866)
    o = 0
    for fan_in, fan_out in ((8, 64), (64, 64), (64, 2)):
        P[o:o + fan_in * fan_out] = torch.randn(fan_in * fan_out, generator=g) / np.sqrt(fan_in)
        o += fan_in * fan_out
        P[o:o + fan_out] = 0.0
        o += fan_out
    P = P.to(dev)
    # start the output bias at the target means so the quantiles move from there
    # (the first two columns of T padded to 8 give their means)
    Tpad = torch.zeros((T.shape[0], 8), device=dev)
    Tpad[:, :2] = T
    P[4864:4866] = api.feature_stats(Tpad)[0][:2]
    m1 = torch.zeros_like(P)
    v1 = torch.zeros_like(P)
    rows = F.shape[0]
    losses = []
    for t in range(1, steps + 1):
        idx = torch.randint(0, rows, (min(batch, rows),), generator=g).to(dev)
        X = F[idx].contiguous()
        Y = T[idx].contiguous()
        out, act = api.mlp_fwd(P, X, mu, sd)
        dout, loss = api.pinball(out, Y, taus[0], taus[1])
        dP = api.mlp_bwd(P, X, act, dout, mu, sd)
        api.adam_step(P, m1, v1, dP, t, lr)
        if log_every and (t % log_every == 0 or t == 1):
            losses.append((t, float(loss.item())))
    model = torch.cat([P, mu, sd]).cpu().numpy().astype(np.float32)
    return model, losses


def evaluate(model, F, T):
    """Coverage of the quantile predictions: fraction of rows where the
    prediction is on the safe side of the target, per output."""
    P = torch.from_numpy(model[:4866]).to(F.device)
    mu = torch.from_numpy(model[4866:4874]).to(F.device)
    sd = torch.from_numpy(model[4874:4882]).to(F.device)
    out, _ = api.mlp_fwd(P, F.contiguous(), mu, sd, keep_act=False)
    cover = (out >= T).float().mean(dim=0).cpu().numpy()
    slack = (out - T).mean(dim=0).cpu().numpy()
    return cover, slack


def save(model, path=DEFAULT_MODEL):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(model, np.float32))


def load(path=DEFAULT_MODEL):
    return np.load(path, allow_pickle=False).astype(np.float32)


def main():
    import argparse
    import time
    ap = argparse.ArgumentParser(description="train the sigma-interval predictor on the GPU")
    ap.add_argument("--rows", type=int, default=100000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--bases", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    a = ap.parse_args()
    t0 = time.time()
    bases = base_spectra_by_method(a.bases, a.bases, 1024, a.seed + 17)
    print(f"base spectra by the method: {len(bases)} in {time.time() - t0:.1f}s", flush=True)
    groups = training_rows(a.rows, 1024, a.seed, bases)
    F, T = features_targets(groups)
    print(f"features {tuple(F.shape)} in {time.time() - t0:.1f}s", flush=True)
    model, losses = train(F, T, steps=a.steps, log_every=max(1, a.steps // 10))
    for t, l in losses:
        print(f"  step {t}: pinball {l:.4f}", flush=True)
    ev = training_rows(4000, 1024, a.seed + 99, bases)
    Fe, Te = features_targets(ev)
    cover, slack = evaluate(model, Fe, Te)
    print(f"held-out coverage {cover}, mean slack {slack}", flush=True)
    save(model, a.out)
    print(f"saved {a.out} ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main()
