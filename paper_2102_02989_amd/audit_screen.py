"""Audit of learned screening: build j3c with the rigorous bounds only (the
full FP64 sum at the given threshold) and with the trained network, both on
the GPU, and report the largest absolute deviation, the fraction of
candidates the network dropped, the short-range terms and the build times.

    python -m paper_2102_02989_amd.audit_screen [--config c5] [--kmesh 4 4 4] [--margin M]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "screen_mlp.npz")


def audit(problem, weights=WEIGHTS, margin=None, lr_precision=0):
    import torch

    import paper_2102_02989_amd as P
    w = np.load(weights)
    margin = float(w["margin"]) if margin is None else float(margin)
    shape = (P.nkpairs(problem.kmesh), problem.aux.nfunc, problem.basis.nfunc, problem.basis.nfunc)
    res = {}
    outs = {}
    for form in ("rigorous", "learned"):
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        kw = dict(g_thresh=problem.g_thr, lr_precision=lr_precision)
        if form == "learned":
            kw.update(screening=P.SCREEN_LEARNED, mlp_weights=w["params"], mlp_margin=margin)
        P.build_j3c(problem.cell, problem.basis, problem.aux, problem.kmesh, problem.omega, problem.thresh, out,
                    **kw)  # warm-up
        _, st = P.build_j3c(problem.cell, problem.basis, problem.aux, problem.kmesh, problem.omega, problem.thresh,
                            out, **kw)
        torch.cuda.synchronize()
        res[form] = st
        outs[form] = out
    err = 0.0
    for k in range(shape[0]):  # per k-pair, to bound temporaries
        err = max(err, float((outs["learned"][k] - outs["rigorous"][k]).abs().max()))
    sl, sr = res["learned"], res["rigorous"]
    return {"workload": f"{problem.name} kmesh {'x'.join(map(str, problem.kmesh))}", "margin": margin,
            "max_abs_err": err, "candidates": sl["n_screen_candidates"], "skipped": sl["n_screen_skipped"],
            "skipped_frac": sl["n_screen_skipped"] / max(sl["n_screen_candidates"], 1),
            "sr_terms_rigorous": sr["n_sr_terms"], "sr_terms_learned": sl["n_sr_terms"],
            "t_sr_ms_rigorous": sr["t_sr_ms"], "t_sr_ms_learned": sl["t_sr_ms"],
            "t_total_ms_rigorous": sr["t_total_ms"], "t_total_ms_learned": sl["t_total_ms"]}


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c5", choices=["c2", "c5"])
    ap.add_argument("--kmesh", type=int, nargs=3, default=None)
    ap.add_argument("--margin", type=float, default=None)
    a = ap.parse_args(argv)
    if a.config == "c5":
        p = synth.config5(kmesh=a.kmesh or (4, 4, 4))
    else:
        p = synth.config2(kmesh=a.kmesh or (2, 2, 2))
    print(json.dumps(audit(p, margin=a.margin)), flush=True)


if __name__ == "__main__":
    main()
