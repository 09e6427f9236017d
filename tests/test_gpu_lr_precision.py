"""Reduced-precision G-space contraction (FP32 and split-FP16x3 operands on the
matrix cores, FP32 accumulation) against the FP64 oracle; the pair and aux
transforms, the kernel weight and the Bloch sums stay FP64 in every form.
Bar: <= 1e-8 au for the FP64 form, <= 1e-6 au for the reduced forms."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import max_err, run_gpu

pytestmark = pytest.mark.gpu

FORMS = {"fp64": (0, 1e-8), "fp32": (1, 1e-6), "f16x3": (2, 1e-6)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("form", list(FORMS))
def test_lr_forms_tiny(form):
    """Triclinic 3-atom cell, 1x2x2 mesh, omega 0.8 (a few thousand q per
    class): long-range part only, whole tensor."""
    prec, tol = FORMS[form]
    p = synth.tiny_problem(kmesh=(1, 2, 2), omega=0.8, diffuse=False)
    _say("case tiny LR form", form)
    got, st = run_gpu(p, parts=oracle.PART_LR, lr_precision=prec)
    ref = oracle.j3c(p, parts=oracle.PART_LR)
    err = max_err(got, ref)
    _say("  max err", err, "max |ref|", np.abs(ref).max(), "N_G", st["n_g_total"])
    assert err <= tol


@pytest.mark.parametrize("form", ["fp32", "f16x3"])
def test_lr_forms_tiny_full(form):
    """Whole j3c (SR - G0 + LR) in the reduced forms, same tiny cell."""
    prec, tol = FORMS[form]
    p = synth.tiny_problem(kmesh=(1, 2, 2), omega=0.8, diffuse=False)
    _say("case tiny full form", form)
    got, _ = run_gpu(p, lr_precision=prec)
    ref = oracle.j3c(p)
    err = max_err(got, ref)
    _say("  max err", err)
    assert err <= tol


def test_small_classes_contracted_in_fp64():
    """A k12 class of at most 4 x 32 q is contracted in FP64 in every form (the
    reduced-precision kernels would take its innermost 32 q in FP64 on the
    vector ALUs anyway): on the 2x2x2 mesh at omega = 0.1 (56 q in 8 classes)
    the FP32 and split-FP16 forms give the FP64 form's long-range part bit for
    bit."""
    import torch

    import paper_2102_02989_amd as P
    p = synth.config2()
    shape = (P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
    outs = {}
    for name, prec in (("fp64", P.FP64), ("fp32", P.FP32), ("f16x3", P.F16X3)):
        _say("case C2 LR form", name)
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        _, st = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, out, g_thresh=p.g_thr,
                            lr_precision=prec, parts=P.PART_LR)
        torch.cuda.synchronize()
        _say("  N_G", st["n_g_total"])
        assert st["n_g_total"] <= 8 * 4 * 32
        outs[name] = out
    assert torch.equal(outs["fp32"], outs["fp64"])
    assert torch.equal(outs["f16x3"], outs["fp64"])
