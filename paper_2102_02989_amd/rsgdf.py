"""ctypes binding of librsgdf.so (argument marshalling only).

Every step of the computation runs in the native library; there is no
Python or CPU fallback.  Importing works without a GPU; calling
``build_j3c`` needs the library and a HIP device.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librsgdf.so")

RSGDF_OK = 0
ERRORS = {-1: "EINVAL", -2: "ESIZE", -3: "ENOMEM", -4: "EHIP", -5: "EUNSUPPORTED"}
FP64, FP32, F16X3 = 0, 1, 2
SCREEN_RIGOROUS, SCREEN_LEARNED = 0, 1
PART_SR, PART_G0, PART_LR = 1, 2, 4
PART_ALL = 7
MLP_NFEAT, MLP_NPARAM = 16, 5377
NOALLOC_SCRATCH_MB = 256  # RSGDF_NOALLOC_SCRATCH_MB


class RsgdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rsgdf error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Cell(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9), ("natm", ctypes.c_int32), ("coords", ctypes.c_void_p)]


class BasisT(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int32), ("shell_atom", ctypes.c_void_p), ("shell_l", ctypes.c_void_p),
                ("shell_nprim", ctypes.c_void_p), ("shell_ptr", ctypes.c_void_p), ("exps", ctypes.c_void_p),
                ("coefs", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("g_thresh", ctypes.c_double), ("lr_precision", ctypes.c_int32), ("screening", ctypes.c_int32),
                ("parts", ctypes.c_int32), ("sr_slices", ctypes.c_int32), ("mlp_weights", ctypes.c_void_p),
                ("mlp_margin", ctypes.c_double), ("sr_split", ctypes.c_void_p), ("alpha_cut", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("t_plan_ms", ctypes.c_double), ("t_sr_ms", ctypes.c_double), ("t_fold_ms", ctypes.c_double),
                ("t_lr_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("n_sr_terms", ctypes.c_int64),
                ("n_sr_shell_terms", ctypes.c_int64), ("n_sr_candidates", ctypes.c_int64),
                ("n_lr_terms", ctypes.c_int64), ("n_g_total", ctypes.c_int64), ("n_triplets", ctypes.c_int64),
                ("n_aux_batches", ctypes.c_int64), ("bytes_out", ctypes.c_int64), ("sr_flops", ctypes.c_double),
                ("t_lr_gemm_ms", ctypes.c_double), ("n_screen_candidates", ctypes.c_int64),
                ("n_screen_skipped", ctypes.c_int64), ("lr_gemm_flops", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Out(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("capacity_bytes", ctypes.c_int64), ("on_device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("nkpair", ctypes.c_int64), ("naux", ctypes.c_int64),
                ("nao", ctypes.c_int64), ("stats", ctypes.POINTER(Stats))]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load librsgdf.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RsgdfError(-5, f"native library missing: {_LIB_PATH} (run __graft_entry__.build())")
        # torch bundles a HIP runtime with the same soname (libamdhip64.so.7);
        # loading it first makes the library bind to that one, so that the
        # process holds a single HIP runtime whichever API is called first
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.rsgdf_j3c_nbytes.restype = ctypes.c_int64
        L.rsgdf_j3c_nbytes.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P]
        L.rsgdf_build_j3c.restype = ctypes.c_int
        L.rsgdf_build_j3c.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                      ctypes.c_double, ctypes.c_double, ctypes.POINTER(Out)]
        L.rsgdf_build_j3c_ex.restype = ctypes.c_int
        L.rsgdf_build_j3c_ex.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                         ctypes.c_double, ctypes.c_double, ctypes.POINTER(Options),
                                         ctypes.POINTER(Out)]
        L.rsgdf_j2c_nbytes.restype = ctypes.c_int64
        L.rsgdf_j2c_nbytes.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), P]
        L.rsgdf_build_j2c.restype = ctypes.c_int
        L.rsgdf_build_j2c.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), P, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(Options), ctypes.POINTER(Out)]
        L.rsgdf_df_solve.restype = ctypes.c_int
        L.rsgdf_df_solve.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P, P, P, P]
        L.rsgdf_coulomb_direct.restype = ctypes.c_int
        L.rsgdf_coulomb_direct.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                           ctypes.c_double, ctypes.c_double, ctypes.POINTER(Options), ctypes.c_int32,
                                           P, P, P, ctypes.POINTER(Stats)]
        L.rsgdf_plan_features.restype = ctypes.c_int
        L.rsgdf_plan_features.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.rsgdf_plan_features_acut.restype = ctypes.c_int
        L.rsgdf_plan_features_acut.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT),
                                               P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               P]
        L.rsgdf_choose_params.restype = ctypes.c_int
        L.rsgdf_choose_params.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                          ctypes.c_double, ctypes.c_double, P, ctypes.c_int32, P, ctypes.c_int32, P,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P]
        L.rsgdf_choose_omega.restype = ctypes.c_int
        L.rsgdf_choose_omega.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                         ctypes.c_double, ctypes.c_double, P, ctypes.c_int32, P,
                                         ctypes.POINTER(ctypes.c_double), P]
        L.rsgdf_build_j3c_noalloc.restype = ctypes.c_int
        L.rsgdf_build_j3c_noalloc.argtypes = L.rsgdf_build_j3c_ex.argtypes
        F = ctypes.c_float
        L.rsgdf_screen_log.restype = ctypes.c_int
        L.rsgdf_screen_log.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, P, P,
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P]
        L.rsgdf_mlp_train.restype = ctypes.c_int
        L.rsgdf_mlp_train.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, F, F,
                                      ctypes.c_uint64, ctypes.c_int32, P, P]
        L.rsgdf_mlp_grad.restype = ctypes.c_int
        L.rsgdf_mlp_grad.argtypes = [P, P, P, ctypes.c_int64, F, P, P, P]
        L.rsgdf_mlp_predict.restype = ctypes.c_int
        L.rsgdf_mlp_predict.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P, P]
        L.rsgdf_mlp_margin.restype = ctypes.c_int
        L.rsgdf_mlp_margin.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double), P]
        L.rsgdf_batch_create.restype = ctypes.c_int
        L.rsgdf_batch_create.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(Options), P, ctypes.POINTER(ctypes.c_void_p)]
        L.rsgdf_batch_run.restype = ctypes.c_int
        L.rsgdf_batch_run.argtypes = [ctypes.c_void_p]
        L.rsgdf_batch_destroy.restype = None
        L.rsgdf_batch_destroy.argtypes = [ctypes.c_void_p]
        L.rsgdf_build_j3c_batch.restype = ctypes.c_int
        L.rsgdf_build_j3c_batch.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                            ctypes.POINTER(Options), P]
        L.rsgdf_autotune_sr.restype = ctypes.c_int
        L.rsgdf_autotune_sr.argtypes = [ctypes.POINTER(Cell), ctypes.POINTER(BasisT), ctypes.POINTER(BasisT), P,
                                        ctypes.c_double, ctypes.c_double, P, P, P]
        L.rsgdf_release_cache.restype = ctypes.c_int
        L.rsgdf_release_cache.argtypes = []
        L.rsgdf_last_error.restype = ctypes.c_char_p
        L.rsgdf_version.restype = ctypes.c_char_p
        L.rsgdf_source_hash.restype = ctypes.c_char_p
        _check_fresh(L)
        _lib = L
    return _lib


def _check_fresh(L) -> None:
    """Refuse a library built from other sources than the ones in the tree:
    a stale build would test code that is not the committed one."""
    from . import build as _build
    if not os.path.isdir(_build.CSRC):
        return
    built, now = L.rsgdf_source_hash().decode(), _build.source_hash()
    if built != now:
        raise RsgdfError(-5, f"{_LIB_PATH} was built from other sources (library {built}, "
                             f"tree {now}); rebuild it with __graft_entry__.build()")


def version() -> str:
    return library().rsgdf_version().decode()


def release_cache() -> None:
    """Free the library's idle cached device blocks (rsgdf_release_cache).

    The large scratch buffers of a build are kept for the next one; call this
    to give their memory back to the device."""
    _check(library().rsgdf_release_cache())


class _Marshal:
    """Keeps the numpy arrays alive while the C structs point at them."""

    def __init__(self, cell, basis, aux, kmesh):
        self.keep = []
        lat = np.ascontiguousarray(cell.lattice, np.float64).reshape(9)
        crd = np.ascontiguousarray(cell.coords, np.float64)
        self.keep += [lat, crd]
        self.cell = Cell((ctypes.c_double * 9)(*lat.tolist()), int(crd.shape[0]), crd.ctypes.data)
        self.basis = self._basis(basis)
        self.aux = self._basis(aux)
        self.kmesh = np.ascontiguousarray(kmesh, np.int32)
        self.keep.append(self.kmesh)

    def _basis(self, b):
        arrs = [np.ascontiguousarray(b.shell_atom, np.int32), np.ascontiguousarray(b.shell_l, np.int32),
                np.ascontiguousarray(b.shell_nprim, np.int32), np.ascontiguousarray(b.shell_ptr, np.int32),
                np.ascontiguousarray(b.exps, np.float64), np.ascontiguousarray(b.coefs, np.float64)]
        self.keep += arrs
        return BasisT(len(arrs[1]), *[a.ctypes.data for a in arrs])


def _check(rc):
    if rc != RSGDF_OK:
        raise RsgdfError(rc, library().rsgdf_last_error().decode())


def j3c_nbytes(cell, basis, aux, kmesh) -> int:
    m = _Marshal(cell, basis, aux, kmesh)
    n = library().rsgdf_j3c_nbytes(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                   m.kmesh.ctypes.data)
    if n < 0:
        _check(int(n))
    return int(n)


def nkpairs(kmesh) -> int:
    nk = int(np.prod(kmesh))
    return nk * (nk + 1) // 2


def _options(g_thresh, lr_precision, screening, parts, sr_slices, mlp_weights, mlp_margin, sr_split, keep,
             alpha_cut=0.0):
    w = None if mlp_weights is None else _f32(mlp_weights, MLP_NPARAM)
    sp = None if sr_split is None else _f32(sr_split, 24)
    keep += [w, sp]
    return Options(-1.0 if g_thresh is None else float(g_thresh), int(lr_precision), int(screening), int(parts),
                   int(sr_slices), None if w is None else w.ctypes.data, float(mlp_margin),
                   None if sp is None else sp.ctypes.data, float(alpha_cut))


def build_j3c(cell, basis, aux, kmesh, omega, thresh, out=None, *, g_thresh=None, lr_precision=FP64,
              screening=SCREEN_RIGOROUS, parts=PART_ALL, sr_slices=0, mlp_weights=None, mlp_margin=0.0,
              sr_split=None, alpha_cut=0.0, stream=None, _noalloc=False):
    """Run rsgdf_build_j3c_ex.

    ``out``: a contiguous complex128 torch tensor on the GPU of shape
    [nkpair, naux, nao, nao] (allocated here if None), or a numpy complex128
    array (host output, staged through device memory by the library).
    ``stream``: a torch.cuda.Stream (defaults to the current stream).
    Returns (out, stats dict)."""
    m = _Marshal(cell, basis, aux, kmesh)
    nbytes = j3c_nbytes(cell, basis, aux, kmesh)
    shape = (nkpairs(kmesh), aux.nfunc, basis.nfunc, basis.nfunc)
    on_device = True
    if out is None:
        import torch
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
    if isinstance(out, np.ndarray):
        if _noalloc:
            raise ValueError("build_j3c_noalloc writes device memory only")
        if out.dtype != np.complex128 or not out.flags.c_contiguous or out.nbytes < nbytes:
            raise ValueError("host output must be a contiguous complex128 array of the full size")
        on_device = False
        ptr, cap = out.ctypes.data, out.nbytes
        sptr = None
    else:
        import torch
        if out.dtype != torch.complex128 or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("device output must be a contiguous complex128 CUDA tensor")
        ptr, cap = out.data_ptr(), out.numel() * 16
        if stream is None:
            stream = torch.cuda.current_stream(out.device)
        sptr = stream.cuda_stream
    stats = Stats()
    o = Out(ptr, cap, int(on_device), sptr, 0, 0, 0, ctypes.pointer(stats))
    keep = []
    opts = _options(g_thresh, lr_precision, screening, parts, sr_slices, mlp_weights, mlp_margin, sr_split, keep,
                    alpha_cut)
    fn = library().rsgdf_build_j3c_noalloc if _noalloc else library().rsgdf_build_j3c_ex
    rc = fn(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux), m.kmesh.ctypes.data, float(omega),
            float(thresh), ctypes.byref(opts), ctypes.byref(o))
    _check(rc)
    return out, stats.as_dict()


def build_j3c_noalloc(cell, basis, aux, kmesh, omega, thresh, out, *, stream=None, **options):
    """Run rsgdf_build_j3c_noalloc: the build of ``build_j3c`` with every
    device scratch buffer taken from the library's static per-GPU array (no
    device allocation in the call).  ``out`` must be a device tensor."""
    return build_j3c(cell, basis, aux, kmesh, omega, thresh, out, stream=stream, _noalloc=True, **options)


# ---- density fitting: two-center metric and the fitting solve ---------------

def j2c_nbytes(cell, aux, kmesh) -> int:
    m = _Marshal(cell, aux, aux, kmesh)
    n = library().rsgdf_j2c_nbytes(ctypes.byref(m.cell), ctypes.byref(m.aux), m.kmesh.ctypes.data)
    if n < 0:
        _check(int(n))
    return int(n)


def build_j2c(cell, aux, kmesh, omega, thresh, out=None, *, g_thresh=None, parts=PART_ALL, stream=None):
    """Run rsgdf_build_j2c: J^k [nk, naux, naux] complex128 (device tensor
    allocated here if ``out`` is None).  Returns (out, stats dict)."""
    import torch
    m = _Marshal(cell, aux, aux, kmesh)
    nk = int(np.prod(kmesh))
    if out is None:
        out = torch.empty((nk, aux.nfunc, aux.nfunc), dtype=torch.complex128, device="cuda")
    if out.dtype != torch.complex128 or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("output must be a contiguous complex128 CUDA tensor")
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    stats = Stats()
    o = Out(out.data_ptr(), out.numel() * 16, 1, stream.cuda_stream, 0, 0, 0, ctypes.pointer(stats))
    keep = []
    opts = _options(g_thresh, FP64, SCREEN_RIGOROUS, parts, 0, None, 0.0, None, keep)
    _check(library().rsgdf_build_j2c(ctypes.byref(m.cell), ctypes.byref(m.aux), m.kmesh.ctypes.data, float(omega),
                                     float(thresh), ctypes.byref(opts), ctypes.byref(o)))
    return out, stats.as_dict()


def df_solve(kmesh, j2c, j3c, out=None, *, stream=None):
    """Run rsgdf_df_solve: d with J^{k12} d = V per k-pair (Eq. M4).  ``j2c``
    [nk, naux, naux] and ``j3c`` [nkpair, naux, nao, nao] are complex128
    device tensors; ``out`` (default: a new tensor) may be ``j3c`` itself."""
    import torch
    for t in (j2c, j3c):
        if t.dtype != torch.complex128 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("inputs must be contiguous complex128 CUDA tensors")
    nk = int(np.prod(kmesh))
    naux = int(j2c.shape[-1])
    if j2c.shape != (nk, naux, naux) or j3c.shape[0] != nk * (nk + 1) // 2 or j3c.shape[1] != naux:
        raise ValueError("shape mismatch between kmesh, j2c and j3c")
    ncol = int(j3c[0, 0].numel())
    if out is None:
        out = torch.empty_like(j3c)
    if out.shape != j3c.shape or out.dtype != torch.complex128 or not out.is_contiguous():
        raise ValueError("out must match j3c")
    if stream is None:
        stream = torch.cuda.current_stream(j3c.device)
    km = np.ascontiguousarray(kmesh, np.int32)
    _check(library().rsgdf_df_solve(km.ctypes.data, naux, ncol, j2c.data_ptr(), j3c.data_ptr(), out.data_ptr(),
                                    stream.cuda_stream))
    return out


def coulomb_direct(cell, basis, aux, kmesh, omega, thresh, dm, vj=None, *, aux_group=0, g_thresh=None,
                   lr_precision=FP64, stream=None):
    """Run rsgdf_coulomb_direct: the density-fitted Coulomb matrix J(k)
    [nk, nao, nao] of the densities ``dm`` (complex128 device tensor, same
    shape) without storing the three-center integrals.  Returns (vj, stats)."""
    import torch
    m = _Marshal(cell, basis, aux, kmesh)
    if dm.dtype != torch.complex128 or not dm.is_contiguous() or not dm.is_cuda:
        raise ValueError("dm must be a contiguous complex128 CUDA tensor")
    if vj is None:
        vj = torch.empty_like(dm)
    if stream is None:
        stream = torch.cuda.current_stream(dm.device)
    keep = []
    opts = _options(g_thresh, lr_precision, SCREEN_RIGOROUS, PART_ALL, 0, None, 0.0, None, keep)
    stats = Stats()
    _check(library().rsgdf_coulomb_direct(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                          m.kmesh.ctypes.data, float(omega), float(thresh), ctypes.byref(opts),
                                          int(aux_group), dm.data_ptr(), vj.data_ptr(), stream.cuda_stream,
                                          ctypes.byref(stats)))
    return vj, stats.as_dict()


# ---- automatic choice of omega -----------------------------------------------

NFEATURES = 9


def plan_features(cell, basis, aux, kmesh, omega, thresh, g_thresh=None, alpha_cut=0.0) -> np.ndarray:
    """rsgdf_plan_features_acut: the cost-model features of one build (host only);
    alpha_cut = 0 means no compact/diffuse split."""
    m = _Marshal(cell, basis, aux, kmesh)
    f = np.zeros(NFEATURES, np.float64)
    _check(library().rsgdf_plan_features_acut(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                              m.kmesh.ctypes.data, float(omega), float(alpha_cut), float(thresh),
                                              -1.0 if g_thresh is None else float(g_thresh), f.ctypes.data))
    return f


def choose_params(cell, basis, aux, kmesh, thresh, coef, omegas, acuts, g_thresh=None):
    """rsgdf_choose_params: (best omega, best alpha_cut, predicted ms [len(omegas)][len(acuts)])."""
    m = _Marshal(cell, basis, aux, kmesh)
    om = np.ascontiguousarray(omegas, np.float64)
    ac = np.ascontiguousarray(acuts, np.float64)
    cf = np.ascontiguousarray(coef, np.float64)
    if cf.size != NFEATURES:
        raise ValueError(f"expected {NFEATURES} coefficients")
    pred = np.zeros((len(om), len(ac)), np.float64)
    bo, ba = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(library().rsgdf_choose_params(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                         m.kmesh.ctypes.data, float(thresh),
                                         -1.0 if g_thresh is None else float(g_thresh), om.ctypes.data, len(om),
                                         ac.ctypes.data, len(ac), cf.ctypes.data, ctypes.byref(bo), ctypes.byref(ba),
                                         pred.ctypes.data))
    return bo.value, ba.value, pred


def choose_omega(cell, basis, aux, kmesh, thresh, coef, omegas, g_thresh=None):
    """rsgdf_choose_omega: (best omega, predicted ms per candidate)."""
    m = _Marshal(cell, basis, aux, kmesh)
    om = np.ascontiguousarray(omegas, np.float64)
    cf = np.ascontiguousarray(coef, np.float64)
    if cf.size != NFEATURES:
        raise ValueError(f"expected {NFEATURES} coefficients")
    pred = np.zeros(len(om), np.float64)
    best = ctypes.c_double(0.0)
    _check(library().rsgdf_choose_omega(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                        m.kmesh.ctypes.data, float(thresh),
                                        -1.0 if g_thresh is None else float(g_thresh), om.ctypes.data, len(om),
                                        cf.ctypes.data, ctypes.byref(best), pred.ctypes.data))
    return best.value, pred


# ---- learned screening -------------------------------------------------------

def _f32(a, n=None):
    a = np.ascontiguousarray(a, np.float32)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} floats, got {a.size}")
    return a


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream


def screen_log(cell, basis, aux, kmesh, omega, thresh, *, sample_frac=1.0, seed=0, capacity=2_000_000, stream=None):
    """rsgdf_screen_log: (features [n,16] float32, targets [n] float32)."""
    m = _Marshal(cell, basis, aux, kmesh)
    n = ctypes.c_int64(0)
    for _ in range(2):
        feat = np.empty((max(capacity, 1), MLP_NFEAT), np.float32)
        tgt = np.empty(max(capacity, 1), np.float32)
        rc = library().rsgdf_screen_log(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                        m.kmesh.ctypes.data, float(omega), float(thresh), float(sample_frac),
                                        int(seed), feat.ctypes.data, tgt.ctypes.data, int(capacity),
                                        ctypes.byref(n), _stream_ptr(stream))
        if rc == -2:
            capacity = int(n.value)
            continue
        _check(rc)
        return feat[:n.value].copy(), tgt[:n.value].copy()
    _check(rc)


def mlp_train(X, y, *, params=None, epochs=20, batch=4096, lr=1e-3, kappa=8.0, seed=0, stream=None):
    """rsgdf_mlp_train: returns (params [MLP_NPARAM] float32, loss per epoch)."""
    X, y = _f32(X), _f32(y)
    init = params is None
    p = np.zeros(MLP_NPARAM, np.float32) if init else _f32(params, MLP_NPARAM).copy()
    hist = np.zeros(max(epochs, 1), np.float32)
    _check(library().rsgdf_mlp_train(p.ctypes.data, X.ctypes.data, y.ctypes.data, len(y), int(epochs), int(batch),
                                     float(lr), float(kappa), int(seed), int(init), hist.ctypes.data,
                                     _stream_ptr(stream)))
    return p, hist[:epochs]


def mlp_grad(params, X, y, *, kappa=8.0, stream=None):
    """rsgdf_mlp_grad: (loss, gradient over W1..b3 [5313])."""
    p, X, y = _f32(params, MLP_NPARAM), _f32(X), _f32(y)
    g = np.zeros(MLP_NPARAM - 64, np.float32)
    loss = np.zeros(1, np.float32)
    _check(library().rsgdf_mlp_grad(p.ctypes.data, X.ctypes.data, y.ctypes.data, len(y), float(kappa),
                                    g.ctypes.data, loss.ctypes.data, _stream_ptr(stream)))
    return float(loss[0]), g


def mlp_predict(params, X, *, mode=1, stream=None):
    """rsgdf_mlp_predict: mode 0 FP32, mode 1 FP16 matrix cores."""
    p, X = _f32(params, MLP_NPARAM), _f32(X)
    out = np.zeros(len(X), np.float32)
    _check(library().rsgdf_mlp_predict(p.ctypes.data, X.ctypes.data, len(X), int(mode), out.ctypes.data,
                                       _stream_ptr(stream)))
    return out


def mlp_margin(params, X, y, *, quantile=1.0, stream=None):
    """rsgdf_mlp_margin."""
    p, X, y = _f32(params, MLP_NPARAM), _f32(X), _f32(y)
    m = ctypes.c_double(0.0)
    _check(library().rsgdf_mlp_margin(p.ctypes.data, X.ctypes.data, y.ctypes.data, len(y), float(quantile),
                                      ctypes.byref(m), _stream_ptr(stream)))
    return m.value


# ---- batches and the work-split autotuner ------------------------------------

class Batch:
    """rsgdf_batch_create / run / destroy over a list of (cell, basis, aux,
    kmesh) with one shared omega, thresh and option set; outputs are device
    tensors allocated here (or passed in ``outs``).  ``run()`` replays the
    captured graph and returns the per-cell stats."""

    def __init__(self, systems, omega, thresh, *, outs=None, g_thresh=None, lr_precision=FP64,
                 screening=SCREEN_RIGOROUS, mlp_weights=None, mlp_margin=0.0, sr_split=None, stream=None):
        import torch
        self._keep = []
        n = len(systems)
        ms = [_Marshal(*s) for s in systems]
        self._keep.append(ms)
        self.cells = (Cell * n)(*[m.cell for m in ms])
        self.bases = (BasisT * n)(*[m.basis for m in ms])
        self.auxes = (BasisT * n)(*[m.aux for m in ms])
        km = np.ascontiguousarray([list(s[3]) for s in systems], np.int32).reshape(n, 3)
        self._keep.append(km)
        if outs is None:
            outs = [torch.empty((nkpairs(s[3]), s[2].nfunc, s[1].nfunc, s[1].nfunc), dtype=torch.complex128,
                                device="cuda") for s in systems]
        self.outs = outs
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stats = [Stats() for _ in range(n)]
        self.o = (Out * n)(*[Out(t.data_ptr(), t.numel() * 16, 1, stream.cuda_stream, 0, 0, 0,
                                 ctypes.pointer(self.stats[i])) for i, t in enumerate(outs)])
        self.opts = _options(g_thresh, lr_precision, screening, PART_ALL, 0, mlp_weights, mlp_margin, sr_split,
                             self._keep)
        h = ctypes.c_void_p(None)
        _check(library().rsgdf_batch_create(n, ctypes.addressof(self.cells), ctypes.addressof(self.bases),
                                            ctypes.addressof(self.auxes), km.ctypes.data, float(omega),
                                            float(thresh), ctypes.byref(self.opts), ctypes.addressof(self.o),
                                            ctypes.byref(h)))
        self._h = h

    def run(self):
        _check(library().rsgdf_batch_run(self._h))
        return [s.as_dict() for s in self.stats]

    def close(self):
        if self._h:
            library().rsgdf_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_sr(cell, basis, aux, kmesh, omega, thresh, *, stream=None):
    """rsgdf_autotune_sr: (split factors [24] float32, class times ms [24])."""
    m = _Marshal(cell, basis, aux, kmesh)
    split = np.ones(24, np.float32)
    ms = np.zeros(24, np.float64)
    _check(library().rsgdf_autotune_sr(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                       m.kmesh.ctypes.data, float(omega), float(thresh), split.ctypes.data,
                                       ms.ctypes.data, _stream_ptr(stream)))
    return split, ms
