"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle."""
import numpy as np


def run_gpu(problem, omega=None, thresh=None, **kw):
    import torch

    import paper_2102_02989_amd as P
    omega = problem.omega if omega is None else omega
    thresh = problem.thresh if thresh is None else thresh
    if "g_thresh" not in kw:
        kw["g_thresh"] = problem.g_thr
    out, stats = P.build_j3c(problem.cell, problem.basis, problem.aux, problem.kmesh, omega, thresh, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), stats


def aux_rows(problem, shells):
    off = problem.aux.offsets()
    rows = []
    for s in shells:
        rows.extend(range(off[s], off[s + 1]))
    return np.array(rows)


def max_err(a, b):
    return float(np.abs(a - b).max())
