"""The no-allocation entry point rsgdf_build_j3c_noalloc against the
allocating one, rsgdf_build_j3c_ex, through the C ABI: two calls in a row
(the second with a smaller input: the buffer keeps the first call's
contents), a build that needs more than the static scratch (a clear
RSGDF_ENOMEM, output untouched), and a call after that failure."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
TOL = 1e-8  # FP64 bar; both entry points run the same kernels


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(p, **kw):
    import torch

    import paper_2102_02989_amd as P
    shape = (P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
    ref = torch.empty(shape, dtype=torch.complex128, device="cuda")
    got = torch.full(shape, complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
    _, st_ref = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, ref, g_thresh=p.g_thr, **kw)
    _, st = P.build_j3c_noalloc(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, got, g_thresh=p.g_thr, **kw)
    torch.cuda.synchronize()
    err = float((got - ref).abs().max())
    return err, float(ref.abs().max()), st, st_ref


def test_noalloc_matches_allocating_entry_point():
    import torch

    import paper_2102_02989_amd as P
    p1 = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    p2 = synth.config1()  # smaller output than p1 (1 k-pair x 32 x 10 x 10)
    assert P.j3c_nbytes(p2.cell, p2.basis, p2.aux, p2.kmesh) < P.j3c_nbytes(p1.cell, p1.basis, p1.aux, p1.kmesh)
    for name, p, kw in (("tiny 2x1x1", p1, {}), ("C1", p2, {}),
                        ("C1 fp32 contraction", p2, dict(lr_precision=P.FP32))):
        _say("case noalloc", name)
        err, scale, st, st_ref = _pair(p, **kw)
        _say(f"  max |noalloc - alloc| {err:.3e} (max |V| {scale:.3e}); terms {st['n_sr_terms']} vs "
             f"{st_ref['n_sr_terms']}; {st['t_total_ms']:.1f} ms")
        assert err <= TOL, (name, err)
        assert st["n_sr_terms"] == st_ref["n_sr_terms"]
    # a build beyond the static buffer is refused with a clear error, before
    # anything is written to the output
    _say("case noalloc oversize (3x3x3 mesh at omega = 1.5)")
    p3 = synth.config3()
    big = torch.zeros(P.j3c_nbytes(p3.cell, p3.basis, p3.aux, p3.kmesh) // 16, dtype=torch.complex128,
                      device="cuda")
    with pytest.raises(P.RsgdfError) as ei:
        P.build_j3c_noalloc(p3.cell, p3.basis, p3.aux, p3.kmesh, p3.omega, p3.thresh, big, g_thresh=p3.g_thr)
    _say("  ", ei.value)
    assert ei.value.code == -3 and "static buffer" in str(ei.value)
    assert float(big.abs().max()) == 0.0
    del big
    torch.cuda.empty_cache()
    # and the entry point still works after that refusal
    _say("case noalloc after the refusal")
    err, _, _, _ = _pair(p1)
    _say(f"  max |noalloc - alloc| {err:.3e}")
    assert err <= TOL
