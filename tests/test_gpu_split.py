"""The compact/diffuse split at alpha_cut (the paper's Fig. 1): primitive
triples with a diffuse aux primitive or two diffuse AO primitives are
evaluated by the range-separation-free reciprocal sum of Eq. M15, the rest
by the range separation.  The j3c is the same quantity, so the bar is the
FP64 one against the oracle (1e-8 au): the tiny cells (every part,
Gamma and a 2x1x1 mesh), C1, and the 8-atom cell on the 2x2x2 mesh at full
size against the stored d-d blocks."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import aux_rows, max_err, run_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-8
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kmesh,acut", [((1, 1, 1), 1.0), ((2, 1, 1), 2.0), ((1, 2, 2), 0.8)])
def test_split_tiny(kmesh, acut):
    p = synth.tiny_problem(kmesh=kmesh, omega=0.8, diffuse=False)
    _say("case split tiny", kmesh, "alpha_cut", acut)
    got, st = run_gpu(p, alpha_cut=acut)
    ref = oracle.j3c(p)
    err = max_err(got, ref)
    _say(f"  max err {err:.3e} (max |ref| {np.abs(ref).max():.3e}), SR terms {st['n_sr_terms']}, q {st['n_g_total']}")
    assert err <= TOL


def test_split_c1():
    p = synth.config1()
    _say("case split C1 alpha_cut 0.5")
    got, st = run_gpu(p, alpha_cut=0.5)
    plain, st0 = run_gpu(p)
    sel = [0, 4, 6, 7, 12, 13]
    ref = oracle.j3c(p, aux_shells=sel)
    rows = aux_rows(p, sel)
    err = max_err(got[:, rows], ref[:, rows])
    _say(f"  max err {err:.3e}; SR terms {st['n_sr_terms']} (plain {st0['n_sr_terms']}), "
         f"build {st['t_total_ms']:.1f} ms (plain {st0['t_total_ms']:.1f})")
    assert err <= TOL


@pytest.mark.parametrize("acut", [0.3, 1.0])
def test_split_c2_dd_blocks(acut):
    import torch

    import paper_2102_02989_amd as P
    p = synth.config2()
    g = np.load(os.path.join(HERE, "golden", "c2_blocks_dd.npz"))
    bo = p.basis.offsets()
    rows = torch.as_tensor(g["rows"], device="cuda")
    out = torch.empty((P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc), dtype=torch.complex128,
                      device="cuda")
    _say("case split C2 alpha_cut", acut)
    res = {}
    for name, a in (("plain", 0.0), ("split", acut)):
        P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, out, g_thresh=p.g_thr, alpha_cut=a)
        _, st = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, out, g_thresh=p.g_thr, alpha_cut=a)
        torch.cuda.synchronize()
        sub = out.index_select(1, rows).cpu().numpy()
        err = max(float(np.abs(sub[:, :, bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]] - g[f"pair_{mu}_{nu}"]).max())
                  for mu, nu in g["pairs"])
        res[name] = (err, st)
        _say(f"  {name}: max err {err:.3e}, build {st['t_total_ms']:.0f} ms (SR {st['t_sr_ms']:.0f}, LR "
             f"{st['t_lr_ms']:.0f}), SR terms {st['n_sr_terms']}, q {st['n_g_total']}")
    assert res["split"][0] <= TOL
