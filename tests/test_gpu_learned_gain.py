"""What the trained screening network gains over the rigorous bounds alone:
on the 16-atom cell of the learned-screening workload (a = 9, random
positions, 2x2x2 mesh here; the 4x4x4 audit is run by
paper_2102_02989_amd.audit_screen), with the committed weights trained on
the other workloads' logs, at the network's calibrated margin (the chosen
form's setting), it must evaluate fewer short-range terms while staying
within the FP64 bar (1e-8 au) of the rigorous build."""
import sys

import pytest

import synth

pytestmark = pytest.mark.gpu


def test_learned_gain_c5_cell():
    from paper_2102_02989_amd.audit_screen import audit
    from paper_2102_02989_amd.chosen import network
    p = synth.config5(kmesh=(2, 2, 2))
    print("case learned gain, C5 cell 2x2x2", flush=True)
    _, margin = network()
    assert margin >= 0.0
    r = audit(p, margin=margin)
    print(" ", r, flush=True)
    sys.stdout.flush()
    assert r["candidates"] > 0
    assert r["sr_terms_learned"] < r["sr_terms_rigorous"]
    assert r["max_abs_err"] <= 1e-8
