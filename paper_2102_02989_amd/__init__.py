"""MI355X (gfx950) range-separated Gaussian density fitting three-center
integrals (Ye & Berkelbach, arXiv 2102.02989).

The compute path is the native library ``librsgdf.so`` (HIP kernels behind a
C ABI, see ``include/rsgdf.h``); this package only marshals arguments.
"""
from .rsgdf import (  # noqa: F401
    PART_ALL,
    PART_G0,
    PART_LR,
    PART_SR,
    FP64,
    FP32,
    F16X3,
    Batch,
    autotune_sr,
    MLP_NFEAT,
    MLP_NPARAM,
    SCREEN_LEARNED,
    SCREEN_RIGOROUS,
    RsgdfError,
    build_j3c,
    release_cache,
    build_j2c,
    j2c_nbytes,
    df_solve,
    coulomb_direct,
    plan_features,
    choose_omega,
    choose_params,
    build_j3c_noalloc,
    NOALLOC_SCRATCH_MB,
    j3c_nbytes,
    library,
    library_path,
    mlp_grad,
    mlp_margin,
    mlp_predict,
    mlp_train,
    nkpairs,
    screen_log,
    version,
)
