"""Drive the host-only sanitizer build of the library (capi.cpp linked with
hip_host_stub.cpp under AddressSanitizer and UndefinedBehaviorSanitizer)
through every C-ABI entry point on the tiny, C1 and C2 inputs: planning,
validation, the short-range work split and aux batching, the long-range q
chunking, the batch planner, the two-center metric, the fitting solve, the
integral-direct consumer, the no-allocation entry point and the error paths.
No kernel runs; "device" buffers are host numpy arrays.

Usage: python drive.py LIBRARY  (run with the sanitizer runtime preloaded)."""
import ctypes
import os
import sys

sys.modules["torch"] = None  # the binding's optional torch import fails cleanly

import numpy as np  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import paper_2102_02989_amd.rsgdf as R  # noqa: E402

R._LIB_PATH = sys.argv[1]
import synth  # noqa: E402
from paper_2102_02989_amd.chosen import network  # noqa: E402

L = R.library()


def say(*a):
    print(*a, flush=True)


def out_struct(arr, on_device=1):
    stats = R.Stats()
    o = R.Out(arr.ctypes.data, arr.nbytes, on_device, None, 0, 0, 0, ctypes.pointer(stats))
    return o, stats


def build(p, name, *, keep_out=None, noalloc=False, **kw):
    m = R._Marshal(p.cell, p.basis, p.aux, p.kmesh)
    shape = (R.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
    out = keep_out if keep_out is not None else np.zeros(shape, np.complex128)
    o, stats = out_struct(out)
    keep = []
    opts = R._options(kw.get("g_thresh", p.g_thr), kw.get("lr_precision", R.FP64),
                      kw.get("screening", R.SCREEN_RIGOROUS), kw.get("parts", R.PART_ALL), 0,
                      kw.get("mlp_weights"), kw.get("mlp_margin", 0.0), kw.get("sr_split"), keep,
                      kw.get("alpha_cut", 0.0))
    fn = L.rsgdf_build_j3c_noalloc if noalloc else L.rsgdf_build_j3c_ex
    rc = fn(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux), m.kmesh.ctypes.data, float(p.omega),
            float(p.thresh), ctypes.byref(opts), ctypes.byref(o))
    say(f"  {name}: rc {rc}, triplets {stats.n_triplets}, aux batches {stats.n_aux_batches}, "
        f"q {stats.n_g_total}")
    if rc != 0:
        raise SystemExit(f"{name}: rc {rc}: {L.rsgdf_last_error()}")
    return out


def expect_error(name, rc):
    say(f"  error path {name}: rc {rc}")
    if rc >= 0:
        raise SystemExit(f"{name}: expected an error code, got {rc}")


def problem_set():
    return [("tiny 2x1x1", synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=True)),
            ("tiny 1x2x2", synth.tiny_problem(kmesh=(1, 2, 2), omega=0.6, diffuse=False)),
            ("C1", synth.config1()),
            ("C2", synth.config2())]


def main():
    params, margin = network()
    chosen = dict(lr_precision=R.F16X3, screening=R.SCREEN_LEARNED, mlp_weights=params, mlp_margin=margin)
    for name, p in problem_set():
        say("case", name)
        f = R.plan_features(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, g_thresh=p.g_thr)
        say("  plan features", np.array2string(np.asarray(f), precision=3))
        oms = np.array([0.1, 0.3, 0.8, 1.5])
        best, pred = R.choose_omega(p.cell, p.basis, p.aux, p.kmesh, p.thresh, np.ones(R.NFEATURES), oms,
                                    g_thresh=p.g_thr)
        say("  choose omega", best)
        out = build(p, "plain")
        for form, kw in (("fp32", dict(lr_precision=R.FP32)), ("chosen", chosen),
                         ("split", dict(alpha_cut=0.5)), ("sr only", dict(parts=R.PART_SR)),
                         ("lr only", dict(parts=R.PART_LR)), ("sr split x3", dict(sr_split=np.full(24, 3.0, np.float32)))):
            build(p, form, keep_out=out, **kw)
        if name != "C2":
            build(p, "noalloc", keep_out=out, noalloc=True)
            build(p, "noalloc chosen", keep_out=out, noalloc=True, **chosen)
        # two-center metric, fitting solve and the integral-direct consumer
        m = R._Marshal(p.cell, p.aux, p.aux, p.kmesh)
        nk = int(np.prod(p.kmesh))
        J = np.zeros((nk, p.aux.nfunc, p.aux.nfunc), np.complex128)
        o, _ = out_struct(J)
        keep = []
        opts = R._options(p.g_thr, R.FP64, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0, None, keep)
        rc = L.rsgdf_build_j2c(ctypes.byref(m.cell), ctypes.byref(m.aux), m.kmesh.ctypes.data, float(p.omega),
                               float(p.thresh), ctypes.byref(opts), ctypes.byref(o))
        say("  j2c rc", rc)
        if rc != 0:
            raise SystemExit(f"j2c: {L.rsgdf_last_error()}")
        if name != "C2":
            d = np.zeros_like(out)
            rc = L.rsgdf_df_solve(m.kmesh.ctypes.data, p.aux.nfunc, p.basis.nfunc ** 2, J.ctypes.data,
                                  out.ctypes.data, d.ctypes.data, None)
            say("  df solve rc", rc)
            if rc != 0:
                raise SystemExit(f"df solve: {L.rsgdf_last_error()}")
            dm = np.zeros((nk, p.basis.nfunc, p.basis.nfunc), np.complex128)
            vj = np.zeros_like(dm)
            mb = R._Marshal(p.cell, p.basis, p.aux, p.kmesh)
            st = R.Stats()
            rc = L.rsgdf_coulomb_direct(ctypes.byref(mb.cell), ctypes.byref(mb.basis), ctypes.byref(mb.aux),
                                        mb.kmesh.ctypes.data, float(p.omega), float(p.thresh), ctypes.byref(opts),
                                        4, dm.ctypes.data, J.ctypes.data, vj.ctypes.data, ctypes.byref(st))
            say("  coulomb direct rc", rc)
            if rc != 0:
                raise SystemExit(f"coulomb direct: {L.rsgdf_last_error()}")
        del out

    # batch planner: three cells of different sizes planned on worker threads
    say("case batch")
    systems = [problem_set()[i][1] for i in (0, 1, 2)]
    n = len(systems)
    ms = [R._Marshal(s.cell, s.basis, s.aux, s.kmesh) for s in systems]
    cells = (R.Cell * n)(*[m.cell for m in ms])
    bases = (R.BasisT * n)(*[m.basis for m in ms])
    auxes = (R.BasisT * n)(*[m.aux for m in ms])
    km = np.ascontiguousarray([list(s.kmesh) for s in systems], np.int32)
    outs = [np.zeros((R.nkpairs(s.kmesh), s.aux.nfunc, s.basis.nfunc, s.basis.nfunc), np.complex128)
            for s in systems]
    stats = [R.Stats() for _ in range(n)]
    o = (R.Out * n)(*[R.Out(a.ctypes.data, a.nbytes, 1, None, 0, 0, 0, ctypes.pointer(stats[i]))
                      for i, a in enumerate(outs)])
    keep = []
    opts = R._options(1e-12, R.FP64, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0, None, keep)
    h = ctypes.c_void_p(None)
    rc = L.rsgdf_batch_create(n, ctypes.addressof(cells), ctypes.addressof(bases), ctypes.addressof(auxes),
                              km.ctypes.data, 0.6, 1e-10, ctypes.byref(opts), ctypes.addressof(o), ctypes.byref(h))
    say("  batch create rc", rc)
    if rc != 0:
        raise SystemExit(f"batch: {L.rsgdf_last_error()}")
    for _ in range(2):
        rc = L.rsgdf_batch_run(h)
        say("  batch run rc", rc)
        if rc != 0:
            raise SystemExit(f"batch run: {L.rsgdf_last_error()}")
    L.rsgdf_batch_destroy(h)

    # the idle cached blocks of the builds above are freed
    rc = L.rsgdf_release_cache()
    say("case release cache rc", rc)
    if rc != 0:
        raise SystemExit(f"release cache: {L.rsgdf_last_error()}")

    # error paths: each is refused with a negative code and no access out of bounds
    say("case error paths")
    p = synth.config1()
    m = R._Marshal(p.cell, p.basis, p.aux, p.kmesh)
    small = np.zeros(4, np.complex128)
    o, _ = out_struct(small)
    keep = []
    opts = R._options(p.g_thr, R.FP64, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0, None, keep)
    args = (ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux), m.kmesh.ctypes.data)
    expect_error("capacity too small", L.rsgdf_build_j3c_ex(*args, 0.5, 1e-10, ctypes.byref(opts), ctypes.byref(o)))
    expect_error("omega <= 0", L.rsgdf_build_j3c_ex(*args, -1.0, 1e-10, ctypes.byref(opts), ctypes.byref(o)))
    expect_error("thresh nan", L.rsgdf_build_j3c_ex(*args, 0.5, float("nan"), ctypes.byref(opts), ctypes.byref(o)))
    bad = np.array([0, 1, 1], np.int32)
    expect_error("kmesh 0", L.rsgdf_build_j3c_ex(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux),
                                                 bad.ctypes.data, 0.5, 1e-10, ctypes.byref(opts), ctypes.byref(o)))
    full = np.zeros((R.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc), np.complex128)
    of, _ = out_struct(full)
    for what, opts_bad in (
            ("lr_precision 7", R._options(p.g_thr, 7, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0, None, keep)),
            ("screening 5", R._options(p.g_thr, R.FP64, 5, R.PART_ALL, 0, None, 0.0, None, keep)),
            ("learned without weights",
             R._options(p.g_thr, R.FP64, R.SCREEN_LEARNED, R.PART_ALL, 0, None, 0.0, None, keep)),
            ("alpha_cut < 0", R._options(p.g_thr, R.FP64, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0, None, keep,
                                          -1.0)),
            ("sr_split 0", R._options(p.g_thr, R.FP64, R.SCREEN_RIGOROUS, R.PART_ALL, 0, None, 0.0,
                                      np.zeros(24, np.float32), keep))):
        expect_error(what, L.rsgdf_build_j3c_ex(*args, 0.5, 1e-10, ctypes.byref(opts_bad), ctypes.byref(of)))
    o_host, _ = out_struct(full, on_device=0)
    expect_error("noalloc with host output",
                 L.rsgdf_build_j3c_noalloc(*args, 0.5, 1e-10, ctypes.byref(opts), ctypes.byref(o_host)))
    # malformed inputs, edited in the marshalled copies: the planner refuses them
    # (marshalled order: lattice, coords, AO atom / l / nprim / ptr / exps / coefs, the same for aux, kmesh)
    for what, edit in (("coordinate nan", lambda mm: mm.keep[1].__setitem__((0, 0), np.nan)),
                       ("AO atom index 99", lambda mm: mm.keep[2].__setitem__(0, 99)),
                       ("AO l = 3", lambda mm: mm.keep[3].__setitem__(0, 3)),
                       ("AO nprim 0", lambda mm: mm.keep[4].__setitem__(0, 0)),
                       ("aux l = 5", lambda mm: mm.keep[9].__setitem__(0, 5)),
                       ("aux exponent < 0", lambda mm: mm.keep[12].__setitem__(0, -1.0))):
        mm = R._Marshal(p.cell, p.basis, p.aux, p.kmesh)
        edit(mm)
        expect_error(what, L.rsgdf_build_j3c_ex(ctypes.byref(mm.cell), ctypes.byref(mm.basis), ctypes.byref(mm.aux),
                                                mm.kmesh.ctypes.data, 0.5, 1e-10, ctypes.byref(opts),
                                                ctypes.byref(of)))
    say("done")


if __name__ == "__main__":
    main()
