"""The learned interval predictor on the GPU: its target and standardisation
kernels against the oracle, and a training run from a seed with the
library's kernels (features, targets, statistics, MLP forward/backward,
pinball loss, Adam) whose held-out coverage is checked."""
import sys
import time

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


def test_training_targets_match_oracle(api):
    # 301 rows (ragged against the 4-rows-per-workgroup grid), spectra of
    # length 77 with kappa up to 1e6, one exactly singular row
    _say("training targets")
    rows, n = 301, 77
    rng = inputs.rng_for(120, 0)
    S = np.stack([np.sort(inputs.log_uniform(rng, n, 10.0 ** -rng.uniform(1, 6), 1.0))[::-1]
                  * np.exp(rng.uniform(-5, 5)) for _ in range(rows)])
    S[7, -3:] = 0.0
    Z = rng.standard_normal((rows, n))
    mn = np.full(rows, 1.0)
    F, aux = api.spectral_features(dev(S), dev(Z), dev(mn))
    T = api.training_targets(dev(S), aux).cpu().double().numpy()
    Sf = S.astype(np.float32).astype(np.float64)
    for r in range(rows):
        r7 = oracle.spectral_features(Sf[r], Z[r].astype(np.float32), n)[1]
        ref = oracle.training_targets(Sf[r], r7)
        # FP32 power sequence against FP64: r_7 agrees to ~1e-6 relative
        np.testing.assert_allclose(T[r], ref, rtol=0, atol=2e-5, err_msg=f"row {r}")
    assert T[7, 1] == pytest.approx(np.log(Sf[7].max() / 1e-30), rel=1e-6)
    # empty input is a no-op
    api.training_targets(dev(np.zeros((0, n))), dev(np.zeros((0, 2))))


@pytest.mark.parametrize("rows", [1, 2, 255, 1000, 70001])
def test_feature_stats_match_oracle_and_repeat(api, rows):
    _say(f"feature stats rows={rows}")
    rng = inputs.rng_for(121, rows)
    F = rng.standard_normal((rows, 8)) * np.array([1, 2, 3, 0.1, 10, 1e-4, 1, 0]) + np.arange(8) * 3
    mu, sd = api.feature_stats(dev(F))
    mu_r, sd_r = oracle.feature_stats(F.astype(np.float32))
    np.testing.assert_allclose(mu.cpu().numpy(), mu_r, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(sd.cpu().numpy(), sd_r, rtol=1e-5, atol=1e-7)
    assert float(sd[7]) == pytest.approx(1e-3)  # constant column: the clamp
    mu2, sd2 = api.feature_stats(dev(F))
    np.testing.assert_array_equal(mu.cpu().numpy(), mu2.cpu().numpy())
    np.testing.assert_array_equal(sd.cpu().numpy(), sd2.cpu().numpy())


def test_predictor_trains_from_seed(api):
    # a reduced version of the shipped model's training run: base spectra
    # from this library's SVD (8 per matrix family at n = 256), 12000 rows,
    # 800 Adam steps; the 0.98-quantile outputs must cover >= 95% of a
    # held-out set drawn from another seed
    import torch
    from paper_2609_32505_amd import predictor
    t0 = time.time()
    bases = predictor.base_spectra_by_method(8, 8, 256, seed=31)
    _say(f"predictor: {len(bases)} base spectra in {time.time() - t0:.1f}s")
    F, T = predictor.features_targets(predictor.training_rows(12000, 256, 3, bases))
    model, losses = predictor.train(F, T, steps=800, log_every=100)
    _say(f"  losses {[(t, round(l, 4)) for t, l in losses]} ({time.time() - t0:.1f}s)")
    assert np.all(np.isfinite(model))
    assert losses[-1][1] < 0.5 * losses[0][1]
    Fe, Te = predictor.features_targets(predictor.training_rows(3000, 256, 1003, bases))
    cover, slack = predictor.evaluate(model, Fe, Te)
    _say(f"  held-out coverage {cover}, mean slack {slack}")
    assert cover[0] >= 0.95 and cover[1] >= 0.95
    # the sigma_max output: r_7 is already within a few percent of sigma_max
    # on these families, and the bound stays close (mean e^0.15 = 1.16 x);
    # the condition-number output uses its inputs: its mean slack is well
    # below that of the best constant bound (the training targets' own 0.98
    # quantile), measured 2.4 against 5.6
    Th, Teh = T.cpu().double().numpy(), Te.cpu().double().numpy()
    const_slack = [float(np.mean(np.quantile(Th[:, j], 0.98) - Teh[:, j])) for j in range(2)]
    _say(f"  constant 0.98-quantile bound: mean slack {const_slack}")
    assert 0.0 < slack[0] < 0.15 and slack[1] < 0.6 * const_slack[1]
    # every reduction in training is in a fixed order: the same seed gives
    # the same model bit for bit
    m1, _ = predictor.train(F, T, steps=30)
    m2, _ = predictor.train(F, T, steps=30)
    np.testing.assert_array_equal(m1, m2)
    torch.cuda.synchronize()
