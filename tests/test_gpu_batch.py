"""Batched builds: many cells in one merged short-range launch per class and
one captured HIP graph, against single-cell builds and the oracle; graph
replays against the eager result; the work-split autotuner."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import max_err, run_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _systems(problems):
    return [(p.cell, p.basis, p.aux, p.kmesh) for p in problems]


def test_batch_matches_single_and_oracle():
    """Three small cells in one batch equal their single-cell builds; the
    triclinic cell with d shells is checked against the oracle (3.5e-9 at
    thresh 1e-10)."""
    import paper_2102_02989_amd as P
    probs = [synth.tiny_problem(kmesh=(1, 1, 1), omega=0.7, seed=11, diffuse=False),
             synth.tiny_problem(kmesh=(1, 2, 2), omega=0.7, seed=12, diffuse=False),
             synth.config1(omega=0.7)]
    _say("case batch of 3 small cells")
    b = P.Batch(_systems(probs), 0.7, 1e-10, g_thresh=1e-12)
    st = b.run()
    for i, p in enumerate(probs):
        single, _ = run_gpu(p, omega=0.7, thresh=1e-10, g_thresh=1e-12)
        got = b.outs[i].cpu().numpy()
        d = max_err(got, single)
        _say("  cell", i, "batch vs single", d, "terms", st[i]["n_sr_terms"])
        assert d <= 1e-12
    ref = oracle.j3c(probs[1], omega=0.7, g_thr=1e-12)
    err = max_err(b.outs[1].cpu().numpy(), ref)
    _say("  vs oracle", err)
    assert err <= 1e-8
    b.close()


def test_batch_graph_replays():
    """Replays with eager work in between (the outputs are cleared and a
    single-cell build runs on the same stream) reproduce the first result."""
    import torch

    import paper_2102_02989_amd as P
    probs = [synth.tiny_problem(kmesh=(1, 2, 1), omega=0.8, seed=s, diffuse=False) for s in (21, 22)]
    _say("case batch graph replay")
    b = P.Batch(_systems(probs), 0.8, 1e-10, g_thresh=1e-12)
    b.run()
    first = [o.clone() for o in b.outs]
    for r in range(3):
        for o in b.outs:
            o.zero_()
        run_gpu(probs[0], omega=0.8, thresh=1e-10, g_thresh=1e-12)
        torch.cuda.synchronize()
        b.run()
        for i, o in enumerate(b.outs):
            assert torch.equal(o, first[i]), (r, i)
    b.close()


def test_batch_c4_cells_sampled():
    """The 64-cell uneven batch (2-16 atoms, meshes 1, 2^3, 3^3): one merged
    launch per class and one graph; sampled cells against single builds."""
    import torch

    import paper_2102_02989_amd as P
    probs = synth.config4_cells()
    _say("case C4 batch, 64 cells")
    b = P.Batch(_systems(probs), probs[0].omega, probs[0].thresh, g_thresh=probs[0].g_thr)
    st = b.run()
    torch.cuda.synchronize()
    _say("  batch wall ms", st[0]["t_total_ms"], "terms", sum(s["n_sr_terms"] for s in st))
    nat = [p.cell.natm for p in probs]
    picks = sorted({int(np.argmin(nat)), int(np.argmax(nat)), 8})
    for i in picks:
        p = probs[i]
        single, _ = run_gpu(p)
        got = b.outs[i].cpu().numpy()
        d = max_err(got, single)
        # and against oracle blocks: first and last aux shell, a same-shell and a
        # cross-cell AO pair, the first, a middle and the last k-pair
        nkp = got.shape[0]
        aux = [0, p.aux.nshell - 1]
        pairs = [(0, 0), (0, p.basis.nshell - 1)]
        kps = sorted({0, nkp // 2, nkp - 1})
        ref = oracle.j3c(p, aux_shells=aux, pairs=pairs, kpairs=kps)
        xo, bo = p.aux.offsets(), p.basis.offsets()
        e = 0.0
        for P_ in aux:
            for mu, nu in pairs:
                sl = (kps, slice(xo[P_], xo[P_ + 1]), slice(bo[mu], bo[mu + 1]), slice(bo[nu], bo[nu + 1]))
                e = max(e, float(np.abs(got[sl] - ref[sl]).max()))
        _say("  cell", i, "natm", p.cell.natm, "kmesh", p.kmesh, "batch vs single", d, "vs oracle", e)
        assert d <= 1e-12
        assert e <= 1e-8
    b.close()


def test_autotune_split():
    import paper_2102_02989_amd as P
    p = synth.tiny_problem(kmesh=(2, 2, 1), omega=0.5, seed=5, diffuse=False)
    _say("case autotune")
    split, ms = P.autotune_sr(p.cell, p.basis, p.aux, p.kmesh, 0.5, 1e-10)
    _say("  split", split.tolist())
    assert set(np.unique(split)).issubset({0.25, 0.5, 1.0, 2.0, 4.0})
    a, _ = run_gpu(p, omega=0.5, thresh=1e-10, sr_split=split)
    b, _ = run_gpu(p, omega=0.5, thresh=1e-10)
    assert max_err(a, b) <= 1e-12
