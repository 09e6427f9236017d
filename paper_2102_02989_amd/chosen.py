"""The chosen form of the build: the options that the benchmark times and the
tests check against the oracle (one definition for both).

  * G-space contraction on reduced-precision matrix cores (default: operands
    rounded to FP32, FP32 products accumulated 16 q at a time and promoted to
    FP64; the 32 innermost q of each k12 class in FP64);
  * learned screening with the committed network at its calibrated margin:
    the largest under-prediction (log10 units) on the held-out 20% of the
    training samples, so no held-out candidate above thresh would be dropped.

Boys, erfc, every Fourier transform, the kernel weight and the Bloch sums stay
FP64 in this form too.
"""
from __future__ import annotations

import os

import numpy as np

from .rsgdf import BF16X3, FP32, FP64, SCREEN_LEARNED

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "screen_mlp.npz")
LR_FORMS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
CHOSEN_LR = "fp32"


def network():
    """(parameters, calibrated margin) of the committed screening network."""
    d = np.load(WEIGHTS)
    return d["params"], float(d["margin"])


def chosen_options(lr: str = CHOSEN_LR) -> dict:
    """Keyword options of build_j3c for the chosen form."""
    params, margin = network()
    return dict(lr_precision=LR_FORMS[lr], screening=SCREEN_LEARNED, mlp_weights=params, mlp_margin=margin)
