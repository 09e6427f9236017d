"""The chosen form of the build: the options that the benchmark times and the
tests check against the oracle (one definition for both).

  * G-space contraction on reduced-precision matrix cores (default: each
    operand scaled per 64-q group by a power of two and split into two FP16
    numbers, three FP16 products per real product accumulated in FP32 over
    the group and promoted to FP64; the 32 innermost q of each k12 class in
    FP64);
  * learned screening with the committed network at its calibrated margin:
    the largest under-prediction (log10 units) on the held-out 20% of the
    training samples, so no held-out candidate above thresh would be dropped.

Boys, erfc, every Fourier transform, the kernel weight and the Bloch sums stay
FP64 in this form too.
"""
from __future__ import annotations

import os

import numpy as np

from .rsgdf import F16X3, FP32, FP64, SCREEN_LEARNED

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "screen_mlp.npz")
LR_FORMS = {"fp64": FP64, "fp32": FP32, "f16x3": F16X3}
CHOSEN_LR = "f16x3"


def network():
    """(parameters, calibrated margin) of the committed screening network."""
    d = np.load(WEIGHTS)
    return d["params"], float(d["margin"])


def chosen_options(lr: str = CHOSEN_LR) -> dict:
    """Keyword options of build_j3c for the chosen form."""
    params, margin = network()
    return dict(lr_precision=LR_FORMS[lr], screening=SCREEN_LEARNED, mlp_weights=params, mlp_margin=margin)
