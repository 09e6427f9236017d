"""Writes c3_blocks.npz: oracle j3c (SR - G0 + LR, FP64) of the 8-atom cell on
the 3x3x3 k-mesh at omega = 1.5 (about 2e4 q vectors per k12 class) for
sampled (aux shell, AO shell pair) blocks and a subset of the k-pairs.  Calls
only the oracle and the seeded input generators.  Run from the repository
root:  python tests/golden/make_c3_golden.py [--set dd]

Set "sp" (c3_blocks.npz): s-s and s-p AO shell pairs on 30 of the 378 k-pairs.
Set "dd" (c3_blocks_dd.npz): d-d AO shell pairs on one atom and across atoms and
a p-s pair, against s, p, d and both f aux shells of atom 0, on 5 k-pairs (two
with k1 = k2, where the G = 0 term enters).  The oracle evaluates every pair
transform of each selected k-pair (about 2e4 q), which is what limits the
k-pairs of the d-d set."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SETS = {
    "sp": dict(aux=[3, 10, 15, 19],              # s, p, d, f shells on atom 0
               pairs=[(0, 13), (1, 7), (2, 3)],  # s-s across atoms (two), s-p on one atom
               kpairs=list(range(0, 378, 13)),   # 30 of the 378 k-pairs (k1 <= k2, row-major)
               file="c3_blocks.npz"),
    "dd": dict(aux=[3, 10, 15, 18, 19],             # s, p, d, f, f shells on atom 0
               pairs=[(5, 5), (5, 11), (3, 0)],     # d-d on one atom, d-d across atoms, p-s
               kpairs=[0, 1, 27, 200, 377],         # (k1, k2) = (0,0), (0,1), (1,1), (8,20), (26,26)
               file="c3_blocks_dd.npz"),
}


def main():
    which = sys.argv[sys.argv.index("--set") + 1] if "--set" in sys.argv else "sp"
    AUX, PAIRS, KPAIRS = SETS[which]["aux"], SETS[which]["pairs"], SETS[which]["kpairs"]
    p = synth.config3()
    t0 = time.time()
    full = oracle.j3c(p, aux_shells=AUX, pairs=PAIRS, kpairs=KPAIRS)
    xo, bo = p.aux.offsets(), p.basis.offsets()
    rows = np.concatenate([np.arange(xo[s], xo[s + 1]) for s in AUX])
    blocks = {}
    for (mu, nu) in PAIRS:
        blk = full[KPAIRS][:, rows][:, :, bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]]
        blocks[f"pair_{mu}_{nu}"] = blk
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), SETS[which]["file"])
    np.savez_compressed(out, aux=np.array(AUX), pairs=np.array(PAIRS), kpairs=np.array(KPAIRS), rows=rows,
                        omega=p.omega, thresh=p.thresh, g_thr=p.g_thr, **blocks)
    print(f"wrote {out} in {time.time() - t0:.0f} s; max |j3c| {max(np.abs(b).max() for b in blocks.values()):.3e}")


if __name__ == "__main__":
    main()
