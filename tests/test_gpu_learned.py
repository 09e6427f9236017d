"""Learned screening on the GPU: training kernels against the numpy FP64
reference, FP16 matrix-core inference against FP32/FP64, and the screened
build against the oracle (chosen-form bar 1e-6 au)."""
import sys

import numpy as np
import pytest

import mlp_ref as R
import oracle
import synth
from gpu_util import max_err, run_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, R.F)).astype(np.float32) * np.linspace(0.5, 3.0, R.F, dtype=np.float32)
    X[:, 11:] = 0.0
    y = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.5 * np.abs(X[:, 3]) - 8.0).astype(np.float32)
    return X, y


def test_mlp_gradient_matches_numpy_fp64():
    import paper_2102_02989_amd as P
    X, y = _data(3000, 0)
    params, _ = P.mlp_train(X, y, epochs=0, seed=1)       # initialisation only
    params, _ = P.mlp_train(X, y, params=params, epochs=2, batch=512, lr=3e-3, seed=2)  # move off the init
    _say("case mlp gradient")
    loss, g = P.mlp_grad(params, X, y, kappa=8.0)
    gref = R.grad(params, X, y, 8.0)
    lref = R.loss(params, X, y, 8.0)
    rel = float(np.abs(g - gref).max() / np.abs(gref).max())
    _say("  loss", loss, lref, "grad rel err", rel)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    assert rel <= 2e-5


def test_mlp_training_reduces_loss():
    import paper_2102_02989_amd as P
    X, y = _data(20000, 1)
    _say("case mlp training")
    params, hist = P.mlp_train(X, y, epochs=30, batch=1024, lr=3e-3, kappa=4.0, seed=3)
    _say("  loss per epoch", hist[0], hist[-1])
    assert hist[-1] < 0.2 * hist[0]
    assert R.loss(params, X, y, 4.0) == pytest.approx(float(hist[-1]), rel=1e-3)


def test_mlp_inference_fp16_and_fp32():
    import paper_2102_02989_amd as P
    X, y = _data(5000, 2)
    params, _ = P.mlp_train(X, y, epochs=5, batch=1024, lr=3e-3, seed=4)
    ref, _ = R.forward(params, X)
    p32 = P.mlp_predict(params, X, mode=0)
    p16 = P.mlp_predict(params, X, mode=1)
    e32, e16 = float(np.abs(p32 - ref).max()), float(np.abs(p16 - ref).max())
    _say("case mlp inference: fp32 err", e32, "fp16 mfma err", e16, "|pred| max", float(np.abs(ref).max()))
    assert e32 <= 1e-4 * max(1.0, float(np.abs(ref).max()))
    assert e16 <= 0.1


def _train_on(problems, seed=0):
    import paper_2102_02989_amd as P
    Xs, ys = [], []
    for p in problems:
        X, y = P.screen_log(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, sample_frac=1.0, seed=seed)
        Xs.append(X)
        ys.append(y)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    rng = np.random.default_rng(seed)
    val = rng.random(len(y)) < 0.2
    params, hist = P.mlp_train(X[~val], y[~val], epochs=40, batch=1024, lr=2e-3, kappa=8.0, seed=seed)
    margin = P.mlp_margin(params, X[val], y[val], quantile=1.0)
    return params, margin, len(y), hist


def test_learned_screening_tiny_vs_oracle():
    """Trained on magnitudes logged from two tiny cells, applied to a third:
    every element within the chosen-form bar of the oracle."""
    import paper_2102_02989_amd as P
    train = [synth.tiny_problem(kmesh=(1, 2, 2), omega=0.8, seed=s, diffuse=False) for s in (7, 8)]
    _say("case learned screening tiny: logging + training")
    params, margin, n, hist = _train_on(train)
    _say("  samples", n, "loss", hist[0], hist[-1], "margin", margin)
    p = synth.tiny_problem(kmesh=(1, 2, 2), omega=0.8, seed=9, diffuse=False)
    got, st = run_gpu(p, screening=P.SCREEN_LEARNED, mlp_weights=params, mlp_margin=margin)
    rig, st0 = run_gpu(p)
    ref = oracle.j3c(p)
    err, err0 = max_err(got, ref), max_err(rig, ref)
    _say("  err learned", err, "rigorous", err0, "candidates", st["n_screen_candidates"], "skipped",
         st["n_screen_skipped"], "terms", st["n_sr_terms"], "vs", st0["n_sr_terms"])
    assert st["n_screen_candidates"] > 0
    assert err <= 1e-6
