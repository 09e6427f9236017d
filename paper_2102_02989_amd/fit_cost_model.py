"""Fit the cost model of the automatic choice of omega to measured builds.

For each workload and candidate omega the host planner's work features
(rsgdf_plan_features) are computed and the build is timed on the GPU, for the
plain form (FP64 contraction) and the FP32-contraction form.  Coefficients
are fitted per form by non-negative least squares on the relative error
(rows scaled by 1/t), time in ms = sum_i coef[i] feat[i] (feat[8] = 1, the
fixed cost of a build).  All arithmetic of
the builds runs in the library; this script sequences the calls, fits and
writes the result.

    python -m paper_2102_02989_amd.fit_cost_model --out paper_2102_02989_amd/data/cost_model.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OMEGAS = [0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5]
MAX_GEMM_FLOPS = 2.5e14  # skip (workload, omega) points whose FP64 contraction alone takes > ~5 s


def measure(workloads, omegas, reps=2):
    import torch

    import paper_2102_02989_amd as P
    rows = []
    for name, p in workloads:
        shape = (P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        for om in omegas:
            f = P.plan_features(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, p.g_thr)
            if f[2] > MAX_GEMM_FLOPS:
                continue
            rec = {"workload": name, "omega": om, "features": f.tolist()}
            for form, prec in (("fp64", P.FP64), ("fp32", P.FP32)):
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, out, g_thresh=p.g_thr,
                                lr_precision=prec)
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t0) * 1e3)
                rec[f"ms_{form}"] = min(ts)
            print(json.dumps(rec), flush=True)
            rows.append(rec)
        del out
        torch.cuda.empty_cache()
    return rows


def fit(rows, form):
    from scipy.optimize import nnls
    F = np.array([list(r["features"]) + [1.0] * (9 - len(r["features"])) for r in rows])
    t = np.array([r[f"ms_{form}"] for r in rows])
    scale = F.max(axis=0)
    scale[scale == 0] = 1.0
    A = (F / scale) / t[:, None]
    coef, _ = nnls(A, np.ones(len(t)))
    coef = coef / scale
    pred = F @ coef
    return coef, float(np.max(np.abs(pred / t - 1.0)))


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--data", help="reuse measured rows (JSON lines) instead of timing")
    a = ap.parse_args(argv)
    if a.data:
        rows = [json.loads(ln) for ln in open(a.data) if ln.strip().startswith("{")]
    else:
        wl = [("C1", synth.config1()), ("C2", synth.config2()), ("C3", synth.config3()), ("C5", synth.config5()),
              ("tiny 2x2x2", synth.tiny_problem(kmesh=(2, 2, 2), omega=0.5, diffuse=False))]
        rows = measure(wl, OMEGAS)
    model = {"features": ["sr_ops", "pairft_candidates", "gemm_flops", "kphase_elements", "out_elements",
                          "x_elements", "n_q", "sr_terms", "constant"], "rows": rows}
    for form in ("fp64", "fp32"):
        coef, worst = fit(rows, form)
        model[f"coef_{form}"] = coef.tolist()
        model[f"max_rel_err_{form}"] = worst
        print(f"{form}: coef {coef} max relative error {worst:.2f}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(model, fh, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
