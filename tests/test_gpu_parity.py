"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, FP64 tolerance 1e-8 au (plain form)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import aux_rows, max_err, run_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("part", [oracle.PART_SR, oracle.PART_G0, oracle.PART_LR])
def test_tiny_gamma_parts(part):
    p = synth.tiny_problem(kmesh=(1, 1, 1), omega=0.7, diffuse=False)
    _say("case tiny gamma part", part)
    got, st = run_gpu(p, parts=part)
    ref = oracle.j3c(p, parts=part, g_thr=p.g_thr)
    err = max_err(got, ref)
    _say("  max err", err, "max |ref|", np.abs(ref).max(), st["n_sr_terms"])
    assert err <= TOL


def test_tiny_gamma_full():
    p = synth.tiny_problem(kmesh=(1, 1, 1), omega=0.7, diffuse=False)
    _say("case tiny gamma full")
    got, st = run_gpu(p)
    ref = oracle.j3c(p)
    err = max_err(got, ref)
    _say("  max err", err, st)
    assert err <= TOL


@pytest.mark.parametrize("kmesh", [(2, 1, 1), (1, 2, 2)])
def test_tiny_kmesh_full(kmesh):
    p = synth.tiny_problem(kmesh=kmesh, omega=0.8, diffuse=False)
    _say("case tiny kmesh", kmesh)
    got, st = run_gpu(p)
    ref = oracle.j3c(p)
    err = max_err(got, ref)
    _say("  max err", err, "max |ref|", np.abs(ref).max())
    assert err <= TOL


def test_config1_subset():
    """C1 (2-atom cubic cell, Gamma, omega = 0.1, thresh 1e-10): GPU builds the
    whole tensor; the oracle checks s, p and d aux rows on both atoms."""
    p = synth.config1()
    _say("case C1 subset")
    got, st = run_gpu(p)
    sel = [0, 4, 6, 7, 12, 13]
    ref = oracle.j3c(p, aux_shells=sel)
    rows = aux_rows(p, sel)
    err = max_err(got[:, rows], ref[:, rows])
    _say("  max err", err, "max |ref|", np.abs(ref).max(), "terms", st["n_sr_terms"], "t", st["t_total_ms"])
    assert err <= TOL


def _block_err(p, got, ref, aux_shells, pairs):
    xo, bo = p.aux.offsets(), p.basis.offsets()
    err = 0.0
    for P in aux_shells:
        for mu, nu in pairs:
            sl = (slice(None), slice(xo[P], xo[P + 1]), slice(bo[mu], bo[mu + 1]), slice(bo[nu], bo[nu + 1]))
            err = max(err, float(np.abs(got[sl] - ref[sl]).max()))
    return err


def test_config2_sampled_blocks():
    """C2 (8-atom cell, 3s2p1d / 8s6p4d2f, 2x2x2 mesh, omega 0.1, thresh 1e-10),
    the benchmark workload at full size in the benchmark's launch
    configuration; the oracle checks sampled (aux shell, AO shell pair) blocks
    for all 36 k-pairs: every aux l, same-atom and cross-atom pairs, s/p/d."""
    from paper_2102_02989_amd.chosen import chosen_options
    p = synth.config2()
    _say("case C2 sampled blocks")
    got, st = run_gpu(p)
    _say("  gpu", {k: st[k] for k in ("t_total_ms", "t_sr_ms", "t_fold_ms", "t_lr_ms", "n_sr_terms")})
    aux = [0, 8, 14, 18, 27, 40]  # s, p, d, f on atom 0; p, s on atoms 1, 2
    pairs = [(0, 0), (0, 6), (3, 10), (2, 5), (11, 4)]
    ref = oracle.j3c(p, aux_shells=aux, pairs=pairs)
    err = _block_err(p, got, ref, aux, pairs)
    _say("  max err", err, "max |ref|", np.abs(ref).max())
    assert err <= TOL
    # the chosen form (reduced-precision contraction, learned screening at the
    # calibrated margin) on the same blocks, bar 1e-6
    got_c, st_c = run_gpu(p, **chosen_options())
    err_c = _block_err(p, got_c, ref, aux, pairs)
    _say("  chosen form: max err", err_c, "candidates dropped", st_c["n_screen_skipped"])
    assert err_c <= 1e-6


def test_config2_dd_golden_blocks():
    """C2 at full size, plain and chosen forms, against stored oracle blocks
    (tests/golden/make_c2_golden.py): d-d AO pairs on one atom and across
    atoms and a p-s pair against a d and both f aux shells, all 36 k-pairs --
    the short-range classes up to (f|dd), L = 7, on their full-size work split."""
    import os

    from paper_2102_02989_amd.chosen import chosen_options
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_blocks_dd.npz")
    g = np.load(path)
    p = synth.config2()
    assert float(g["omega"]) == p.omega and float(g["thresh"]) == p.thresh
    rows = g["rows"]
    bo = p.basis.offsets()
    for name, kw, tol in (("plain", {}, TOL), ("chosen", chosen_options(), 1e-6)):
        _say("case C2 d-d golden blocks,", name)
        got, st = run_gpu(p, **kw)
        err = 0.0
        for mu, nu in g["pairs"]:
            blk = got[:, rows][:, :, bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]]
            err = max(err, float(np.abs(blk - g[f"pair_{mu}_{nu}"]).max()))
        _say(f"  max err {err:.3e}  t_sr {st['t_sr_ms']:.0f} ms")
        assert err <= tol, (name, err)


def test_config5_sampled_blocks():
    """The 16-atom cubic cell (a = 9) on the 4x4x4 mesh (2080 k-pairs, 54.5 GB
    output) at full size: sampled (aux shell, AO shell pair) blocks, s/p/d aux
    and same-atom and cross-atom s/p pairs, on k-pairs that include k1 = k2 ones
    (the G = 0 term) and the last pair."""
    p = synth.config5()
    _say("case C5 sampled blocks")
    aux = [0, 4, 6, 13, 20, 111]
    pairs = [(0, 0), (2, 5), (1, 30), (47, 47), (2, 2), (5, 17)]
    kps = [0, 1, 63, 64, 777, 1500, 2079]
    import torch

    import paper_2102_02989_amd as P
    out, st = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, g_thresh=p.g_thr)
    torch.cuda.synchronize()
    got = out[torch.as_tensor(kps, device=out.device)].cpu().numpy()  # the sampled k-pairs only
    del out
    _say("  gpu", {k: st[k] for k in ("t_total_ms", "t_sr_ms", "t_fold_ms", "t_lr_ms", "n_sr_terms")})
    ref = oracle.j3c(p, aux_shells=aux, pairs=pairs, kpairs=kps)
    err = _block_err(p, got, ref[kps], aux, pairs)
    _say("  max err", err, "max |ref|", np.abs(ref).max())
    assert err <= TOL
