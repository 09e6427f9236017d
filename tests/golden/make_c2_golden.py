"""Writes c2_blocks_dd.npz: oracle j3c (SR - G0 + LR, FP64) of the 8-atom cell
on the 2x2x2 k-mesh at omega = 0.1 for (aux shell, AO shell pair) blocks with
d-d AO pairs (one atom, two atoms) and a p-s pair against a d and both f aux
shells of atom 0 -- the angular-momentum classes up to L = l_P + l_a + l_b = 7
-- on all 36 k-pairs.  Calls only the oracle and the seeded input generators.
Run from the repository root:  python tests/golden/make_c2_golden.py
(about 5 minutes on 3 threads: the oracle's short-range sum at omega = 0.1 with
(f|dd) blocks)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

AUX = [14, 18, 19]                 # d, f, f shells on atom 0
PAIRS = [(5, 5), (5, 11), (3, 0)]  # d-d on atom 0, d-d across atoms 0 and 1, p-s on atom 0


def main():
    p = synth.config2()
    t0 = time.time()
    full = oracle.j3c(p, aux_shells=AUX, pairs=PAIRS)
    xo, bo = p.aux.offsets(), p.basis.offsets()
    rows = np.concatenate([np.arange(xo[s], xo[s + 1]) for s in AUX])
    blocks = {}
    for (mu, nu) in PAIRS:
        blocks[f"pair_{mu}_{nu}"] = full[:, rows][:, :, bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_blocks_dd.npz")
    np.savez_compressed(out, aux=np.array(AUX), pairs=np.array(PAIRS), kpairs=np.arange(36), rows=rows,
                        omega=p.omega, thresh=p.thresh, g_thr=p.g_thr, **blocks)
    print(f"wrote {out} in {time.time() - t0:.0f} s; max |j3c| {max(np.abs(b).max() for b in blocks.values()):.3e}")


if __name__ == "__main__":
    main()
