"""Host-side checks of the automatic choice of omega and alpha_cut (no GPU):
the planner's work features behave as the paper's scaling analysis says they
must (the short-range work falls and the long-range work grows with omega,
the q count tracks the Gaussian-damped sphere; the compact/diffuse split
moves work from the short range to the Eq. M15 spheres, which grow with
alpha_cut), the choosers return the argmin of the committed cost model's
predictions, and the committed model, fitted to measured builds with and
without the split, picks near the fastest measured point of each workload."""
import json
import os

import numpy as np

import paper_2102_02989_amd as P
import synth

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2102_02989_amd", "data",
                     "cost_model.json")
OMEGAS = [0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5]
ACUTS = [0.0, 0.1, 0.3, 1.0]


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


def test_split_features():
    """alpha_cut = 0 is the unsplit build; a larger cut leaves fewer compact
    primitives to the short range and widens the Eq. M15 q spheres."""
    p = synth.config2()
    F = np.array([P.plan_features(p.cell, p.basis, p.aux, p.kmesh, 0.3, p.thresh, p.g_thr, alpha_cut=a)
                  for a in ACUTS])
    assert np.all(np.diff(F[:, 0]) <= 0) and np.all(np.diff(F[:, 7]) <= 0)
    assert F[-1, 0] < F[0, 0]
    assert np.all(np.diff(F[:, 6]) > 0)  # q vectors: the M15 spheres grow with the cut
    assert np.all(F[:, 4] == F[0, 4]) and np.all(F[:, 5] == F[0, 5])


def test_joint_chooser_is_argmin_of_the_model():
    m = json.load(open(MODEL))
    coef = np.array(m["coef_fp64"])
    p = synth.config2()
    om = [0.2, 0.3, 0.5]
    bo, ba, pred = P.choose_params(p.cell, p.basis, p.aux, p.kmesh, p.thresh, coef, om, ACUTS, g_thresh=p.g_thr)
    F = np.array([[P.plan_features(p.cell, p.basis, p.aux, p.kmesh, o, p.thresh, p.g_thr, alpha_cut=a) @ coef
                   for a in ACUTS] for o in om])
    assert np.allclose(pred, F, rtol=1e-12)
    i, j = np.unravel_index(int(np.argmin(pred)), pred.shape)
    assert (bo, ba) == (om[i], ACUTS[j])
    # without the split among the candidates it is the omega chooser
    b1, p1 = P.choose_omega(p.cell, p.basis, p.aux, p.kmesh, p.thresh, coef, om, g_thresh=p.g_thr)
    b2, a2, p2 = P.choose_params(p.cell, p.basis, p.aux, p.kmesh, p.thresh, coef, om, [0.0], g_thresh=p.g_thr)
    assert b1 == b2 and a2 == 0.0 and np.allclose(p1, p2[:, 0], rtol=1e-12)


def test_committed_model_selects_near_the_measured_best():
    """On the measured rows (plain form, omega and alpha_cut candidates), the
    point the model picks for each workload builds within 15% of the fastest
    measured one."""
    m = json.load(open(MODEL))
    coef = np.array(m["coef_fp64"])
    rows = m["rows"]
    for w in sorted(set(r["workload"] for r in rows)):
        rs = [r for r in rows if r["workload"] == w]
        pred = [np.dot(list(r["features"]) + [1.0] * (9 - len(r["features"])), coef) for r in rs]
        pick = rs[int(np.argmin(pred))]
        best = min(r["ms_fp64"] for r in rs)
        assert pick["ms_fp64"] <= 1.15 * best, (w, pick["omega"], pick["ms_fp64"], best)
