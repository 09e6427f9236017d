"""Writes c3_blocks.npz: oracle j3c (SR - G0 + LR, FP64) of the 8-atom cell on
the 3x3x3 k-mesh at omega = 1.5 (about 2e4 q vectors per k12 class) for
sampled (aux shell, AO shell pair) blocks and a subset of the k-pairs.  Calls
only the oracle and the seeded input generators.  Run from the repository
root:  python tests/golden/make_c3_golden.py   (the oracle evaluates every pair transform
of each selected k-pair, so blocks with d shells would take hours at this size; those are
covered by the smaller parity cases)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

AUX = [3, 10, 15, 19]                        # s, p, d, f shells on atom 0
PAIRS = [(0, 13), (1, 7), (2, 3)]  # s-s across atoms (two), s-p on one atom
KPAIRS = list(range(0, 378, 13))             # 30 of the 378 k-pairs (k1 <= k2, row-major)


def main():
    p = synth.config3()
    t0 = time.time()
    full = oracle.j3c(p, aux_shells=AUX, pairs=PAIRS, kpairs=KPAIRS)
    xo, bo = p.aux.offsets(), p.basis.offsets()
    rows = np.concatenate([np.arange(xo[s], xo[s + 1]) for s in AUX])
    blocks = {}
    for (mu, nu) in PAIRS:
        blk = full[KPAIRS][:, rows][:, :, bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]]
        blocks[f"pair_{mu}_{nu}"] = blk
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_blocks.npz")
    np.savez_compressed(out, aux=np.array(AUX), pairs=np.array(PAIRS), kpairs=np.array(KPAIRS), rows=rows,
                        omega=p.omega, thresh=p.thresh, g_thr=p.g_thr, **blocks)
    print(f"wrote {out} in {time.time() - t0:.0f} s; max |j3c| {max(np.abs(b).max() for b in blocks.values()):.3e}")


if __name__ == "__main__":
    main()
