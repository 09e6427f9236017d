"""CPU pin of the numpy reference network used by the GPU training tests:
its hand-written backpropagation against central finite differences."""
import numpy as np

import mlp_ref as R


def _params(rng):
    p = np.zeros(R.NPARAM)
    p[R.OFF_MEAN:R.OFF_MEAN + R.F] = rng.normal(size=R.F)
    p[R.OFF_ISTD:R.OFF_ISTD + R.F] = rng.uniform(0.5, 2.0, R.F)
    p[R.OFF_W1:R.OFF_B3 + 1] = rng.normal(scale=0.3, size=R.NTRAIN)
    return p


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = _params(rng)
    X = rng.normal(size=(40, R.F))
    y = rng.normal(size=40)
    kappa = 8.0
    g = R.grad(p, X, y, kappa)
    h = 1e-6
    idx = np.concatenate([rng.choice(np.arange(R.OFF_W1, R.OFF_B3 + 1), 200, replace=False), [R.OFF_B3]])
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss(pp, X, y, kappa) - R.loss(pm, X, y, kappa)) / (2 * h)
        assert abs(fd - g[i - R.OFF_W1]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i - R.OFF_W1])


def test_asymmetric_weight():
    """kappa weights under-predictions only: shifting all targets above the
    predictions scales the loss by kappa exactly."""
    rng = np.random.default_rng(4)
    p = _params(rng)
    X = rng.normal(size=(10, R.F))
    pred, _ = R.forward(p, X)
    lo = R.loss(p, X, pred - 1.0, 5.0)   # predictions above targets: weight 1
    hi = R.loss(p, X, pred + 1.0, 5.0)   # predictions below targets: weight kappa
    assert abs(lo - 1.0) < 1e-12 and abs(hi - 5.0) < 1e-12
