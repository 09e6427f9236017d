"""Benchmark: periodic RS-GDF three-center integrals (j3c) on one MI355X.

Workload (default): the 8-atom diamond-like cubic cell (a = 6.74 bohr),
Cartesian 3s2p1d AO (n_AO = 120) and 8s6p4d2f aux (n_aux = 560) Gaussian
bases drawn from a seeded generator, 3x3x3 k-mesh (378 k-pairs), omega = 1.5
(about 2.0e4 q vectors per k12 class, 5.5e5 in all), threshold 1e-10,
complex128 output (48.8 GB).  One step = one full three-center build into a
preallocated device buffer: host planning, short-range lattice sums, Bloch
fold, G = 0 term, aux and pair Fourier transforms and the G-space
contraction.

Two forms are timed on the same input:
  plain  : rsgdf_build_j3c, every stage FP64, rigorous screening;
  chosen : rsgdf_build_j3c_ex with the G-space contraction on reduced-
           precision matrix cores (each operand scaled per 64-q group by a
           power of two and split into two FP16 numbers, three FP16
           products per real product accumulated in FP32 over the group and
           promoted to FP64; the 32 innermost q of each class in FP64) and
           learned screening with the committed network at its calibrated
           margin (the largest under-prediction on held-out samples).  Boys,
           erfc, every transform and the Bloch sums stay FP64.
The chosen form is timed for --steps steps (after --warmup), the plain form
--plain-steps times; the chosen form's maximum absolute deviation from the
plain output is taken over the whole tensor.  Sub-records time both forms
once on the 2x2x2 workload (omega = 0.1) and the 16-atom 4x4x4 workload.

Prints one JSON line.  value = primitive integrals per second: the plain
build's (aux primitive, AO primitive, AO primitive, image pair) short-range
terms plus its (primitive pair, image, q) pair transforms, divided by the
chosen form's wall time per build.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR = 78.6e12  # 256 CU x 4 SIMD x 16 FP64 FMA lanes x 2 flop x 2.4 GHz
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "f16x3": 2.5e15}  # dense matrix-core peaks per operand type
LR_CHOICES = ("f16x3", "fp32", "fp64")
TRAFFIC_FILES = {  # committed FETCH_SIZE / WRITE_SIZE summaries, by kernel family and workload
    "sr": "sr3c_{}_traffic.json",
    "lr_gemm": "lr_gemm_{}_traffic.json",
}
KERNEL_SOURCES = {
    "sr": ("paper_2102_02989_amd/csrc/sr3c.hip", "paper_2102_02989_amd/csrc/device_math.h",
           "paper_2102_02989_amd/csrc/plan.h", "paper_2102_02989_amd/csrc/boys.h"),
    "lr_gemm": ("paper_2102_02989_amd/csrc/lr.hip", "paper_2102_02989_amd/csrc/kernels.h"),
}
TABLE_S3 = ("paper Table S3 (J+K CPU time per SCF cycle including DF initialisation, one core of an Intel Xeon "
            "Gold 6126 at 2.6 GHz, 16 GB): diamond/cc-pVDZ N_k = 3^3: GDF 1441.77 s, RSGDF 205.25 s; "
            "N_k = 2^3: GDF 855.27 s, RSGDF 79.43 s")


def source_hash(family):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(family, workload):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources changed since the counters were taken or they were
    taken on another workload."""
    try:
        with open(os.path.join(ROOT, "profiles", TRAFFIC_FILES[family].format(workload.lower()))) as fh:
            rec = json.load(fh)
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source_hash", rec.get("sr_source_hash")) != source_hash(family):
        return None
    if rec.get("workload", workload) != workload:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _class_pairs(problem):
    """One AO shell pair per (l_a, l_b) class: mu on atom 0, nu on atom 1."""
    b = problem.basis
    out = []
    for la in range(3):
        for lb in range(3):
            pr = next(((mu, nu) for mu in range(b.nshell) if b.shell_l[mu] == la and b.shell_atom[mu] == 0
                       for nu in range(b.nshell) if b.shell_l[nu] == lb and b.shell_atom[nu] == 1), None)
            if pr is not None:
                out.append(pr)
    return out


def _pair_weight(problem, mu, nu):
    b = problem.basis
    nc = lambda l: (l + 1) * (l + 2) // 2  # noqa: E731
    return float(b.shell_nprim[mu] * b.shell_nprim[nu] * nc(int(b.shell_l[mu])) * nc(int(b.shell_l[nu])))


def cpu_baseline(problem, gpu_terms):
    """The oracle (plain C, OpenMP) timed on the host cores on a bounded
    sample of the workload:
      short range + G = 0: the 20 aux shells of atom 0 (every l_P) against one
        AO shell pair per (l_a, l_b) class (9 pairs), all k-pairs;
      long range: the 16 s-s AO shell pairs with the fewest primitive
        pairs against every aux shell for one k-pair (k1 = 0, k2 = 1; about
        2.0e4 q);
      one thread: the short range of the s-s pair against the atom-0 aux
        shells, all k-pairs.
    value = the oracle's own primitive-integral count (short-range terms plus
    pair transforms) per second over the sample.  The full-build time is
    extrapolated per part by a work model (short range: primitive products x
    Cartesian block sizes over all (aux shell, AO pair); long range: primitive
    pairs x Cartesian block sizes over all AO pairs, times the k-pairs)."""

    import oracle
    ax, nkp = problem.aux, oracle.nkpairs(problem.kmesh)
    nc = lambda l: (l + 1) * (l + 2) // 2  # noqa: E731
    aux0 = [s for s in range(ax.nshell) if ax.shell_atom[s] == 0]
    cls_pairs = _class_pairs(problem)
    t0 = time.perf_counter()
    _, c_sr = oracle.j3c(problem, aux_shells=aux0, pairs=cls_pairs, parts=oracle.PART_SR | oracle.PART_G0,
                         return_counts=True)
    t_sr = time.perf_counter() - t0
    b = problem.basis
    lr_pairs = sorted(((mu, nu) for mu in range(b.nshell) for nu in range(b.nshell)
                       if b.shell_l[mu] + b.shell_l[nu] == 0), key=lambda pr: _pair_weight(problem, *pr))[:16]
    t0 = time.perf_counter()
    _, c_lr = oracle.j3c(problem, pairs=lr_pairs, kpairs=[1], parts=oracle.PART_LR, return_counts=True)
    t_lr = time.perf_counter() - t0
    # one-thread run in a child process (the thread count is fixed at load)
    code = ("import sys, time; sys.path.insert(0, %r); import oracle, synth, bench; p = synth.%s(); "
            "aux0 = [s for s in range(p.aux.nshell) if p.aux.shell_atom[s] == 0]; "
            "pr = bench._class_pairs(p)[0]; t = time.perf_counter(); "
            "_, c = oracle.j3c(p, aux_shells=aux0, pairs=[pr], parts=oracle.PART_SR | oracle.PART_G0, "
            "return_counts=True); print(int(c[0]), time.perf_counter() - t, oracle.num_threads())"
            % (ROOT, {"C1": "config1", "C2": "config2", "C3": "config3"}[problem.name]))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        n1, t1, th1 = r.stdout.split()[-3:]
        one = {"value": int(n1) / float(t1), "unit": "prim-integrals/s", "threads": int(th1),
               "sample": f"short range of AO pair {cls_pairs[0]} (s-s) x the {len(aux0)} aux shells of atom 0, "
                         f"all {nkp} k-pairs: {int(n1)} terms in {float(t1):.2f} s"}
    except (subprocess.SubprocessError, ValueError) as e:  # reported, not fatal
        one = {"error": str(e)}
    # work-model extrapolation to the full build
    aux_w_all = sum(ax.shell_nprim[s] * nc(int(ax.shell_l[s])) for s in range(ax.nshell))
    aux_w0 = sum(ax.shell_nprim[s] * nc(int(ax.shell_l[s])) for s in aux0)
    all_pairs = [(mu, nu) for mu in range(b.nshell) for nu in range(b.nshell)]
    w_all = sum(_pair_weight(problem, *pr) for pr in all_pairs)
    sr_full = t_sr * (aux_w_all * w_all) / (aux_w0 * sum(_pair_weight(problem, *pr) for pr in cls_pairs))
    lr_full = t_lr * nkp * w_all / sum(_pair_weight(problem, *pr) for pr in lr_pairs)
    n_sample = int(c_sr[0] + c_lr[1])
    ext = sr_full + lr_full
    return {"value": n_sample / (t_sr + t_lr), "unit": "prim-integrals/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{problem.name}: short range + G=0 of the {len(aux0)} aux shells of atom 0 x {len(cls_pairs)} "
                      f"AO shell pairs (one per (l_a, l_b) class), all {nkp} k-pairs: {int(c_sr[0])} terms in "
                      f"{t_sr:.2f} s; long range of {len(lr_pairs)} s-s AO shell pairs x all aux shells, k-pair "
                      f"(0, 1): {int(c_lr[1])} pair transforms in {t_lr:.2f} s",
            "one_thread": one,
            "extrapolated_build_s": ext, "extrapolated_sr_s": sr_full, "extrapolated_lr_s": lr_full,
            "sample_fraction_of_build": (t_sr + t_lr) / ext,
            "gpu_plain_prim_integrals": gpu_terms,
            "paper": TABLE_S3}


def max_abs_diff(a, b, chunk=8):
    import torch
    m = 0.0
    for i in range(0, a.shape[0], chunk):
        m = max(m, float((a[i:i + chunk] - b[i:i + chunk]).abs().max()))
    torch.cuda.synchronize()
    return m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1, help="timed plain builds (after the chosen ones)")
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c5"],
                    help="c3 (default): the 8-atom cell on the 3x3x3 mesh at omega = 1.5; c2: the same cell on "
                         "the 2x2x2 mesh at omega = 0.1; c5: the 16-atom cell on the 4x4x4 mesh; c1: the 2-atom cell")
    from paper_2102_02989_amd.chosen import CHOSEN_LR  # numpy and ctypes only: no device touched yet
    ap.add_argument("--lr", default=CHOSEN_LR, choices=LR_CHOICES, help="chosen form's contraction")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-sub", action="store_true", help="skip the sub-records of the other workloads")
    ap.add_argument("--form", default="both", choices=["both", "plain", "chosen"],
                    help="time the plain FP64 build, the chosen form, or both (value = chosen)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the timed steps, run one plain device copy of this many MiB (a known-size "
                         "reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus N > 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2102_02989_amd as P
    import synth

    from paper_2102_02989_amd.chosen import chosen_options
    P.library()  # fails loudly when the native library is missing
    forms = {"plain": dict(lr_precision=P.FP64), "chosen": chosen_options(args.lr)}
    margin = forms["chosen"]["mlp_margin"]
    makers = {"c1": synth.config1, "c2": synth.config2, "c3": synth.config3, "c5": synth.config5}

    def one_build(problem, form, out):
        _, st = P.build_j3c(problem.cell, problem.basis, problem.aux, problem.kmesh, problem.omega, problem.thresh,
                            out, g_thresh=problem.g_thr, **forms[form])
        return st

    def timed(problem, form, out, steps, warmup):
        for _ in range(warmup):
            one_build(problem, form, out)
        torch.cuda.synchronize()
        stats, each = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            stats.append(one_build(problem, form, out))
            torch.cuda.synchronize()
            each.append((time.perf_counter() - t1) * 1e3)
        total = (time.perf_counter() - t0) * 1e3
        return total / steps, stats, sorted(each)[len(each) // 2]

    def describe(problem, nkp):
        return (f"{problem.name}: {problem.cell.natm}-atom cubic cell a={problem.cell.lattice[0][0]:g}, n_AO="
                f"{problem.basis.nfunc}, n_aux={problem.aux.nfunc}, kmesh {'x'.join(map(str, problem.kmesh))} "
                f"({nkp} k-pairs), omega={problem.omega}, thresh={problem.thresh}")

    problem = makers[args.config]()
    shape = (P.nkpairs(problem.kmesh), problem.aux.nfunc, problem.basis.nfunc, problem.basis.nfunc)
    out_chosen = torch.empty(shape, dtype=torch.complex128, device="cuda")
    out_plain = torch.empty(shape, dtype=torch.complex128, device="cuda") if args.form == "both" else out_chosen
    res = {}
    if args.form in ("both", "chosen"):
        res["chosen"] = timed(problem, "chosen", out_chosen, args.steps, args.warmup)
    if args.form in ("both", "plain"):
        res["plain"] = timed(problem, "plain", out_plain, args.steps if args.form == "plain" else args.plain_steps,
                             args.warmup if args.form == "plain" else 0)
    head = "chosen" if "chosen" in res else "plain"
    ms, stats, _ = res[head]
    ref_stats = res["plain"][1][-1] if "plain" in res else stats[-1]
    n_terms = int(ref_stats["n_sr_terms"] + ref_stats["n_lr_terms"])
    value = n_terms / (ms * 1e-3)
    # roofline of the timed form's dominant kernel family, from HIP events on
    # the stream its kernels run on, averaged over the timed steps
    t_sr = sum(s["t_sr_ms"] for s in stats) / len(stats)
    t_gemm = sum(s["t_lr_gemm_ms"] for s in stats) / len(stats)
    lr_name = args.lr if head == "chosen" else "fp64"
    flops = stats[-1]["lr_gemm_flops"]
    achieved = flops / (t_gemm * 1e-3) if t_gemm > 0 else 0.0
    roof_gemm = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[lr_name] / 1e12, "unit": "TFLOP/s",
                 "frac": achieved / PEAK[lr_name], "traffic": recorded_traffic("lr_gemm", problem.name),
                 "kernel": (f"{'lr_gemm_f16x3_kernel' if lr_name == 'f16x3' else 'lr_gemm_tiled_kernel'} "
                            f"({lr_name} complex G-space contraction, all k12 classes of one build; flops = 8 per "
                            f"complex multiply-add" + (", the form issues 24 FP16 flops per complex multiply-add"
                                                       if lr_name == "f16x3" else "") + ")"),
                 "flops_per_launch": flops, "avg_launch_ms": t_gemm}
    flops = stats[-1]["sr_flops"]
    achieved = flops / (t_sr * 1e-3) if t_sr > 0 else 0.0
    roof_sr = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
               "frac": achieved / PEAK_FP64_VECTOR, "traffic": recorded_traffic("sr", problem.name),
               "kernel": "sr3c_kernel (the 24 angular-momentum classes of one build, on 3 side streams; flops = "
                         "image-loop terms plus the Hermite contractions)",
               "flops_per_launch": flops, "avg_launch_ms": t_sr}
    # the dominant kernel family by time; the other one is reported beside it
    roof, roof2 = (roof_gemm, roof_sr) if t_gemm > t_sr else (roof_sr, roof_gemm)
    cfg = {"workload": describe(problem, shape[0]), "form": head,
           "chosen": {"lr_precision": args.lr, "screening": "learned", "mlp_margin": margin,
                      "mlp_margin_rule": "largest under-prediction on the held-out 20% of the training samples",
                      "entry_point": "rsgdf_build_j3c_ex"} if head == "chosen" else None}
    for form, (fms, fst, med) in res.items():
        cfg[f"{form}_build_s"] = fms * 1e-3
        cfg[f"{form}_build_median_s"] = med * 1e-3
        cfg[f"{form}_phases_ms"] = {k: fst[-1][k] for k in ("t_plan_ms", "t_sr_ms", "t_fold_ms", "t_lr_ms",
                                                             "t_lr_gemm_ms", "t_total_ms")}
    if len(res) == 2:
        cfg["speedup_chosen_vs_plain"] = res["plain"][0] / res["chosen"][0]
        cfg["chosen_max_abs_err_vs_plain"] = max_abs_diff(out_chosen, out_plain)
    line = {
        "metric": "j3c build s per k-mesh + primitive integrals/s, chosen vs plain, err<=1e-6",
        "value": value,
        "unit": "prim-integrals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian bases and cells)",
        "config": cfg,
        "counts": {k: stats[-1][k] for k in ("n_sr_terms", "n_sr_shell_terms", "n_lr_terms", "n_g_total",
                                             "n_triplets", "n_screen_candidates", "n_screen_skipped")},
        "roofline": roof,
        "roofline_second": roof2,
        "cpu_baseline": None,
    }
    del out_chosen, out_plain
    torch.cuda.empty_cache()
    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calib_copy_bytes"] = n * 8
        del src, dst
        torch.cuda.empty_cache()
    if not args.no_sub and args.form == "both":
        subs = {}
        for name in ("c2", "c5"):
            if name == args.config:
                continue
            p = makers[name]()
            sh = (P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc)
            oc = torch.empty(sh, dtype=torch.complex128, device="cuda")
            op = torch.empty(sh, dtype=torch.complex128, device="cuda")
            mc, sc, _ = timed(p, "chosen", oc, 1, 0)
            mp, sp, _ = timed(p, "plain", op, 1, 0)
            subs[name] = {"workload": describe(p, sh[0]), "chosen_build_s": mc * 1e-3, "plain_build_s": mp * 1e-3,
                          "speedup_chosen_vs_plain": mp / mc, "chosen_max_abs_err_vs_plain": max_abs_diff(oc, op),
                          "plain_phases_ms": {k: sp[-1][k] for k in ("t_plan_ms", "t_sr_ms", "t_fold_ms", "t_lr_ms",
                                                                     "t_lr_gemm_ms")},
                          "prim_integrals_per_s": (sp[-1]["n_sr_terms"] + sp[-1]["n_lr_terms"]) / (mc * 1e-3)}
            del oc, op
            torch.cuda.empty_cache()
        cfg["sub_records"] = subs
    if not args.no_cpu and problem.name in ("C1", "C2", "C3"):
        line["cpu_baseline"] = cpu_baseline(problem, n_terms)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
