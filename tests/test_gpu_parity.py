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
