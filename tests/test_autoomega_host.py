"""Host-side checks of the automatic choice of omega (no GPU): the planner's
work features behave as the paper's scaling analysis says they must (the
short-range work falls and the long-range work grows with omega, the q count
tracks the Gaussian-damped sphere), the chooser returns the argmin of the
committed cost model's predictions, and the committed model reproduces its
own measured rows."""
import json
import os

import numpy as np

import paper_2102_02989_amd as P
import synth

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2102_02989_amd", "data",
                     "cost_model.json")
OMEGAS = [0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5]


def test_features_follow_the_scaling_analysis():
    p = synth.config2()
    F = np.array([P.plan_features(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, p.g_thr) for om in OMEGAS])
    # SR work (feat 0, 7) decreases with omega (N_cell ~ omega^-3), LR work
    # (q count, transform candidates, contraction flops) increases
    assert np.all(np.diff(F[:, 0]) < 0) and np.all(np.diff(F[:, 7]) < 0)
    for j in (1, 2, 6):
        assert np.all(np.diff(F[:, j]) > 0)
    # the q sphere holds exp(-q^2/4w^2) >= g_thr: its volume grows like omega^3
    ratio = F[-1, 6] / F[3, 6]
    assert 0.7 * (1.5 / 0.3) ** 3 < ratio < 1.3 * (1.5 / 0.3) ** 3
    assert np.all(F[:, 8] == 1.0)
    # output and intermediate sizes do not depend on omega
    assert np.all(F[:, 4] == F[0, 4]) and np.all(F[:, 5] == F[0, 5])


def test_chooser_is_argmin_of_the_model():
    m = json.load(open(MODEL))
    coef = np.array(m["coef_fp64"])
    for mk in (synth.config1, synth.config2, synth.config3):
        p = mk()
        best, pred = P.choose_omega(p.cell, p.basis, p.aux, p.kmesh, p.thresh, coef, OMEGAS, g_thresh=p.g_thr)
        F = np.array([P.plan_features(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, p.g_thr) for om in OMEGAS])
        assert np.allclose(pred, F @ coef, rtol=1e-12)
        assert best == OMEGAS[int(np.argmin(pred))]


def test_committed_model_selects_near_the_measured_best():
    """On the measured rows (plain form), the omega the model picks for each
    workload builds within 15% of the fastest measured omega."""
    m = json.load(open(MODEL))
    coef = np.array(m["coef_fp64"])
    rows = m["rows"]
    for w in sorted(set(r["workload"] for r in rows)):
        rs = [r for r in rows if r["workload"] == w]
        pred = [np.dot(list(r["features"]) + [1.0] * (9 - len(r["features"])), coef) for r in rs]
        pick = rs[int(np.argmin(pred))]
        best = min(r["ms_fp64"] for r in rs)
        assert pick["ms_fp64"] <= 1.15 * best, (w, pick["omega"], pick["ms_fp64"], best)
