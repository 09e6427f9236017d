"""Fit the cost model of the automatic choice of omega and alpha_cut to
measured builds.

For each workload and candidate omega (and, at a subset of the omegas, each
candidate alpha_cut of the compact/diffuse split) the host planner's work
features (rsgdf_plan_features_acut) are computed and the build is timed on
the GPU, for the plain form (FP64 contraction) and the FP32-contraction
form.  Coefficients
are fitted per form by non-negative least squares on the relative error
(rows scaled by 1/t), time in ms = sum_i coef[i] feat[i] (feat[8] = 1, the
fixed cost of a build).  All arithmetic of
the builds runs in the library; this script sequences the calls, fits and
writes the result.

    python -m paper_2102_02989_amd.fit_cost_model --out paper_2102_02989_amd/data/cost_model.json
    (or: --measure-only --workloads C1,C2 > rows.jsonl on the GPU, then
     --data rows.jsonl --out ... to fit the collected rows)
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
SPLIT_OMEGAS = [0.1, 0.3, 0.7]  # omegas at which the split is measured
ACUTS = [0.1, 0.3, 1.0]          # alpha_cut candidates of the split
MAX_GEMM_FLOPS = 2.5e14  # skip points whose FP64 contraction alone takes > ~5 s


def measure(workloads, omegas, reps=2, split_omegas=SPLIT_OMEGAS, acuts=ACUTS):
    import torch

    import paper_2102_02989_amd as P
    rows = []
    for name, p in workloads:
        shape = (P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        pts = [(om, 0.0) for om in omegas] + [(om, a) for om in split_omegas for a in acuts]
        # one untimed build first: the first call of a process sets up the device tables
        P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, out, g_thresh=p.g_thr)
        torch.cuda.synchronize()
        for om, acut in pts:
            f = P.plan_features(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, p.g_thr, alpha_cut=acut)
            if f[2] > MAX_GEMM_FLOPS:
                continue
            rec = {"workload": name, "omega": om, "alpha_cut": acut, "features": f.tolist()}
            for form, prec in (("fp64", P.FP64), ("fp32", P.FP32)):
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, om, p.thresh, out, g_thresh=p.g_thr,
                                lr_precision=prec, alpha_cut=acut)
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
    ap.add_argument("--out")
    ap.add_argument("--data", help="reuse measured rows (JSON lines) instead of timing")
    ap.add_argument("--measure-only", action="store_true", help="time and print the rows, fit nothing")
    ap.add_argument("--workloads", default="C1,C2,C3,C5,tiny 2x2x2")
    ap.add_argument("--reps", type=int, default=2, help="timed builds per point (the fastest counts)")
    a = ap.parse_args(argv)
    if a.data:
        rows = [json.loads(ln) for ln in open(a.data) if ln.strip().startswith("{")]
    else:
        makers = {"C1": synth.config1, "C2": synth.config2, "C3": synth.config3, "C5": synth.config5,
                  "tiny 2x2x2": lambda: synth.tiny_problem(kmesh=(2, 2, 2), omega=0.5, diffuse=False)}
        wl = [(w, makers[w]()) for w in a.workloads.split(",")]
        rows = measure(wl, OMEGAS, reps=a.reps)
        if a.measure_only:
            return
    if not a.out:
        ap.error("--out is required to fit")
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
