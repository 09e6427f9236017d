"""CPU FP64 oracle for the range-separated three-center integrals.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
it.  The C source (``oracle.c``) shares no code with the GPU library.

Functions follow the paper (arXiv 2102.02989):
  * ``j3c``    -- Eq. M12 (SR lattice sum, BvK fold of Eq. M14, G=0 term) plus
                  Eq. M10/M11 (LR reciprocal sum).
  * ``prim3c`` -- one isolated primitive integral (P|w|ab) with
                  w = 1/r, erf(wr)/r or erfc(wr)/r (Eq. M9).
  * ``boys``   -- Boys function F_m(T).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

COUL, ERF, ERFC = 0, 1, 2
PART_SR, PART_G0, PART_LR = 1, 2, 4
PART_M15 = 8  # the range-separation-free q sum of Eq. M15 (alone; omega and g_thr set the q sphere)
PART_ALL = PART_SR | PART_G0 | PART_LR


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        d, i = ctypes.c_double, ctypes.c_int
        P = ctypes.c_void_p
        L.orc_boys.restype = d
        L.orc_boys.argtypes = [i, d]
        L.orc_prim3c.restype = i
        L.orc_prim3c.argtypes = [i, d, i, d, P, i, d, P, i, d, P, P]
        L.orc_prim_ft.restype = i
        L.orc_prim_ft.argtypes = [i, i, d, P, P, P]
        L.orc_pair_ft.restype = i
        L.orc_pair_ft.argtypes = [i, i, d, P, i, i, d, P, P, P]
        L.orc_overlap.restype = d
        L.orc_overlap.argtypes = [i, i, d, P, i, i, d, P]
        L.orc_j3c.restype = i
        L.orc_j3c.argtypes = [P, i, P, i, P, P, P, P, P, P, i, P, P, P, P, P, P, P, d, d, d, i, i, i, P, i, P,
                              i, P, P, P]
        L.orc_j2c.restype = i
        L.orc_j2c.argtypes = [P, i, P, i, P, P, P, P, P, P, P, d, d, d, i, P, P]
        L.orc_num_threads.restype = i
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def boys(m: int, T: float) -> float:
    return lib().orc_boys(int(m), float(T))


def prim3c(kind, omega, lc, gc, C, la, ga, A, lb, gb, B):
    """Isolated primitive block (c|w|ab), shape [ncart(lc), ncart(la), ncart(lb)]."""
    nc = lambda l: (l + 1) * (l + 2) // 2
    out = np.zeros(nc(lc) * nc(la) * nc(lb))
    C, A, B = (np.ascontiguousarray(x, dtype=np.float64) for x in (C, A, B))
    rc = lib().orc_prim3c(kind, omega, lc, gc, _ptr(C), la, ga, _ptr(A), lb, gb, _ptr(B), _ptr(out))
    if rc:
        raise ValueError(f"orc_prim3c failed ({rc})")
    return out.reshape(nc(lc), nc(la), nc(lb))


def prim_ft(l, comp, g, C, q):
    C, q = (np.ascontiguousarray(x, dtype=np.float64) for x in (C, q))
    out = np.zeros(2)
    lib().orc_prim_ft(l, comp, g, _ptr(C), _ptr(q), _ptr(out))
    return complex(out[0], out[1])


def pair_ft(la, ca, ga, A, lb, cb, gb, B, q):
    A, B, q = (np.ascontiguousarray(x, dtype=np.float64) for x in (A, B, q))
    out = np.zeros(2)
    lib().orc_pair_ft(la, ca, ga, _ptr(A), lb, cb, gb, _ptr(B), _ptr(q), _ptr(out))
    return complex(out[0], out[1])


def overlap(la, ca, ga, A, lb, cb, gb, B):
    A, B = (np.ascontiguousarray(x, dtype=np.float64) for x in (A, B))
    return lib().orc_overlap(la, ca, ga, _ptr(A), lb, cb, gb, _ptr(B))


def nkpairs(kmesh, all_pairs=False):
    nk = int(np.prod(kmesh))
    return nk * nk if all_pairs else nk * (nk + 1) // 2


def j3c(problem, omega=None, cut=1e-15, g_thr=None, parts=PART_ALL, all_pairs=False, aux_shells=None,
        pairs=None, kpairs=None, return_counts=False):
    """Oracle three-center integrals for ``problem`` (a ``synth.Problem``).

    Returns complex128 [nkpair][naux][nao][nao]; k-pairs are k1 <= k2 in
    row-major upper-triangle order (or all ordered pairs with all_pairs=True).
    ``cut`` is the oracle's own per-term truncation (1s model with polynomial
    growth factors, see oracle.c); ``aux_shells``/``pairs``/``kpairs`` (k-pair
    indices) restrict the work (unselected entries stay zero)."""
    omega = problem.omega if omega is None else omega
    g_thr = problem.g_thr if g_thr is None else g_thr
    cell, bs, ax = problem.cell, problem.basis, problem.aux
    lat = np.ascontiguousarray(cell.lattice, np.float64).reshape(9)
    crd = np.ascontiguousarray(cell.coords, np.float64)
    km = np.asarray(problem.kmesh, np.int32)
    if aux_shells is None:
        aux_shells = np.arange(ax.nshell, dtype=np.int32)
    aux_shells = np.ascontiguousarray(aux_shells, np.int32)
    if pairs is None:
        psel, npsel = np.zeros(2, np.int32), -1
    else:
        psel = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1))
        npsel = len(psel) // 2
    if kpairs is None:
        ksel, nksel = np.zeros(1, np.int32), -1
    else:
        ksel = np.ascontiguousarray(np.asarray(kpairs, np.int32).reshape(-1))
        nksel = len(ksel)
    nkp = nkpairs(problem.kmesh, all_pairs)
    out = np.zeros((nkp, ax.nfunc, bs.nfunc, bs.nfunc), np.complex128)
    counts = np.zeros(2, np.int64)
    arrs = [bs.shell_atom, bs.shell_l, bs.shell_nprim, bs.shell_ptr, bs.exps, bs.coefs,
            ax.shell_atom, ax.shell_l, ax.shell_nprim, ax.shell_ptr, ax.exps, ax.coefs]
    arrs = [np.ascontiguousarray(a) for a in arrs]
    rc = lib().orc_j3c(_ptr(lat), cell.natm, _ptr(crd), bs.nshell, *[_ptr(a) for a in arrs[:6]], ax.nshell,
                       *[_ptr(a) for a in arrs[6:]], _ptr(km), float(omega), float(cut), float(g_thr), int(parts),
                       int(bool(all_pairs)), len(aux_shells), _ptr(aux_shells), npsel, _ptr(psel), nksel, _ptr(ksel),
                       _ptr(out), _ptr(counts))
    if rc:
        raise RuntimeError(f"orc_j3c failed ({rc})")
    if return_counts:
        return out, counts
    return out


def j2c(problem, omega=None, cut=1e-15, g_thr=None, parts=PART_ALL, return_counts=False):
    """Oracle two-center metric J^k_PQ (Eq. M5, q = 0 removed) of the aux basis
    for every k of the mesh: complex128 [nk][naux][naux], k in mesh order
    (j = (j1 n2 + j2) n3 + j3).  ``parts`` as for j3c (PART_M15 alone: the plain
    reciprocal-space sum)."""
    omega = problem.omega if omega is None else omega
    g_thr = problem.g_thr if g_thr is None else g_thr
    cell, ax = problem.cell, problem.aux
    lat = np.ascontiguousarray(cell.lattice, np.float64).reshape(9)
    crd = np.ascontiguousarray(cell.coords, np.float64)
    km = np.asarray(problem.kmesh, np.int32)
    nk = int(np.prod(problem.kmesh))
    out = np.zeros((nk, ax.nfunc, ax.nfunc), np.complex128)
    counts = np.zeros(2, np.int64)
    arrs = [np.ascontiguousarray(a) for a in (ax.shell_atom, ax.shell_l, ax.shell_nprim, ax.shell_ptr, ax.exps,
                                                ax.coefs)]
    rc = lib().orc_j2c(_ptr(lat), cell.natm, _ptr(crd), ax.nshell, *[_ptr(a) for a in arrs], _ptr(km), float(omega),
                       float(cut), float(g_thr), int(parts), _ptr(out), _ptr(counts))
    if rc:
        raise RuntimeError(f"orc_j2c failed ({rc})")
    if return_counts:
        return out, counts
    return out


def df_coefficients(J, V, kmesh, all_pairs=False):
    """The density-fitting coefficients of Eq. M4: solve J^{k12} d^{k1k2} = V^{k1k2}
    for every k-pair (k12 = k2 - k1 folded onto the mesh), by a Cholesky
    factorisation of each Hermitian positive-definite J^k and two triangular
    solves (numpy/scipy library routines).  J: [nk][naux][naux]; V:
    [nkpair][naux][nao][nao]; returns d with V's shape."""
    import scipy.linalg as sla
    n = tuple(int(x) for x in kmesh)
    pairs = kpair_list(n, all_pairs)
    d = np.empty_like(V)
    naux = V.shape[1]
    chol = {}
    for t, (k1, k2) in enumerate(pairs):
        j1 = np.unravel_index(k1, n)
        j2 = np.unravel_index(k2, n)
        c = int(np.ravel_multi_index(tuple((b - a) % m for a, b, m in zip(j1, j2, n)), n))
        if c not in chol:
            chol[c] = sla.cho_factor(J[c], lower=True)
        d[t] = sla.cho_solve(chol[c], V[t].reshape(naux, -1)).reshape(V.shape[1:])
    return d


def coulomb_df(problem, dm, cut=1e-15):
    """Density-fitted Coulomb matrix (Eq. M7 with k1 = k2, k3 = k4, and the
    fit of Eq. M4 at k12 = 0), written out from its definition:
        rho_Q = sum_k sum_{l s} V^{kk}_{Q l s} D^k_{s l},   J^0 c = rho,
        J_{m n}(k) = (1/Nk) sum_Q V^{kk}_{Q m n} c_Q,
    V from j3c (the k-pairs (k, k)), J^0 from j2c at Gamma, the solve by
    scipy's Cholesky factorisation.  dm: complex [nk][nao][nao]."""
    import copy

    import scipy.linalg as sla
    nk = int(np.prod(problem.kmesh))
    pairs = kpair_list(problem.kmesh)
    diag = [t for t, (k1, k2) in enumerate(pairs) if k1 == k2]
    V = j3c(problem, kpairs=diag, cut=cut)[diag]  # [nk][naux][nao][nao], k order
    g = copy.copy(problem)
    g.kmesh = (1, 1, 1)
    J0 = j2c(g, cut=cut)[0]
    rho = np.einsum("kqls,ksl->q", V, dm)
    c = sla.cho_solve(sla.cho_factor(J0, lower=True), rho)
    return np.einsum("kqmn,q->kmn", V, c) / nk


def num_threads() -> int:
    return lib().orc_num_threads()


def kpoints(problem):
    """Gamma-centred mesh k_j = sum_i (j_i/n_i) b_i, j = (j1 n2 + j2) n3 + j3."""
    A = np.asarray(problem.cell.lattice, float)
    B = 2 * np.pi * np.linalg.inv(A).T
    n = problem.kmesh
    ks = []
    for j0 in range(n[0]):
        for j1 in range(n[1]):
            for j2 in range(n[2]):
                ks.append(j0 / n[0] * B[0] + j1 / n[1] * B[1] + j2 / n[2] * B[2])
    return np.array(ks)


def kpair_list(kmesh, all_pairs=False):
    nk = int(np.prod(kmesh))
    return [(k1, k2) for k1 in range(nk) for k2 in (range(nk) if all_pairs else range(k1, nk))]


def unique_k12_count(n: int) -> int:
    """Number of distinct k2-k1 difference vectors on an n x n x n
    Gamma-centred mesh, counting k12 and -k12 once (Table S1, N_k12)."""
    diffs = set()
    r = range(-(n - 1), n)
    for a in r:
        for b in r:
            for c in r:
                v = (a, b, c)
                mv = (-a, -b, -c)
                diffs.add(min(v, mv))
    return len(diffs)
