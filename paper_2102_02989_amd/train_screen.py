"""Train the learned-screening network on magnitudes the method itself
generates (logged by the plain GPU short-range sum of the 2-atom Gamma cell,
the 8-atom cell on the 2x2x2 mesh at omega = 0.1 and on the 3x3x3 mesh at
omega = 1.5), then calibrate the margin on a held-out 20% as the largest
under-prediction.  All arithmetic runs in the library's kernels; this script
only sequences the calls and writes the result.

    python -m paper_2102_02989_amd.train_screen --out paper_2102_02989_amd/data/screen_mlp.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    import paper_2102_02989_amd as P
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--kappa", type=float, default=8.0)
    ap.add_argument("--frac", type=float, nargs=3, default=[1.0, 0.05, 0.02],
                    help="logged-candidate sample fractions of the three training cells")
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)

    problems = [synth.config1(), synth.config2(), synth.config3()]
    Xs, ys, src = [], [], []
    for i, (p, f) in enumerate(zip(problems, a.frac)):
        t = time.time()
        X, y = P.screen_log(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, sample_frac=f, seed=a.seed + i,
                            capacity=4_000_000)
        print(f"logged {p.name}: {len(y)} samples in {time.time() - t:.1f} s", flush=True)
        Xs.append(X)
        ys.append(y)
        src.append(np.full(len(y), i, np.int8))
    X, y, src = np.concatenate(Xs), np.concatenate(ys), np.concatenate(src)
    val = np.random.default_rng(a.seed).random(len(y)) < 0.2
    t = time.time()
    params, hist = P.mlp_train(X[~val], y[~val], epochs=a.epochs, batch=a.batch, lr=a.lr, kappa=a.kappa,
                               seed=a.seed)
    print(f"trained on {int((~val).sum())} samples in {time.time() - t:.1f} s; loss {hist[0]:.4g} -> {hist[-1]:.4g}",
          flush=True)
    margin = P.mlp_margin(params, X[val], y[val], quantile=1.0)
    m99 = P.mlp_margin(params, X[val], y[val], quantile=0.99)
    print(f"margin (max under-prediction on {int(val.sum())} held-out samples) {margin:.3f}; 99% quantile {m99:.3f}",
          flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.savez(a.out, params=params, margin=np.float64(margin), loss=hist, n_train=int((~val).sum()),
             n_val=int(val.sum()), sources=np.array([p.name for p in problems]),
             counts=np.bincount(src, minlength=3))
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
