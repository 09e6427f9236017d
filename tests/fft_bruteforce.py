"""Brute-force periodic three-center integrals on a real-space grid.

No analytic integral is used: Bloch sums of the Gaussians are sampled on a
uniform grid in the unit cell, transformed with numpy's FFT, and the
G=0-removed Coulomb kernel 4 pi/|G+k12|^2 is applied directly:

    V[k1,k2][P][mu][nu] = (4 pi/Omega) sum_{q = G + k12, q != 0}
                           conj(chi^_P(q)) rho^_{mu nu}(q) / |q|^2

with chi^(q) = int_Omega chi^{k12}(r) e^{-iq.r} dr and rho = conj(phi^{k1}_mu) phi^{k2}_nu
(paper Eqs. M1, M2, M6).  Valid for diffuse functions only (grid resolution).
"""
import itertools

import numpy as np


def cart_powers(l):
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def eval_bloch(basis, coords, lattice, k, pts, rcut):
    """phi^k(r) = sum_m e^{ik.m} phi(r - m) for every Cartesian function."""
    A = np.asarray(lattice)
    nmax = [int(np.ceil((rcut + np.linalg.norm(A.sum(0))) * np.linalg.norm(b) / (2 * np.pi))) + 1
            for b in 2 * np.pi * np.linalg.inv(A).T]
    out = []
    for s in range(basis.nshell):
        l = int(basis.shell_l[s])
        ctr = coords[basis.shell_atom[s]]
        p0 = basis.shell_ptr[s]
        ex = basis.exps[p0:p0 + basis.shell_nprim[s]]
        cf = basis.coefs[p0:p0 + basis.shell_nprim[s]]
        vals = np.zeros((len(cart_powers(l)), len(pts)), np.complex128)
        for m in itertools.product(*[range(-n, n + 1) for n in nmax]):
            mv = np.asarray(m) @ A
            d = pts - (ctr + mv)
            r2 = np.einsum("ij,ij->i", d, d)
            if r2.min() > rcut * rcut:
                continue
            rad = np.zeros(len(pts))
            for e, c in zip(ex, cf):
                rad += c * np.exp(-e * r2)
            ph = np.exp(1j * np.dot(k, mv))
            for ic, (i, j, kk) in enumerate(cart_powers(l)):
                vals[ic] += ph * rad * d[:, 0] ** i * d[:, 1] ** j * d[:, 2] ** kk
        out.append(vals)
    return np.concatenate(out, axis=0)


def j3c_fft(problem, ngrid=32, all_pairs=False, rcut=None):
    cell, bs, ax = problem.cell, problem.basis, problem.aux
    A = np.asarray(cell.lattice, float)
    B = 2 * np.pi * np.linalg.inv(A).T
    vol = abs(np.linalg.det(A))
    n = ngrid
    fr = np.stack(np.meshgrid(*[np.arange(n) / n] * 3, indexing="ij"), -1).reshape(-1, 3)
    pts = fr @ A
    amin = min(bs.exps.min(), ax.exps.min())
    if rcut is None:
        rcut = np.sqrt(36.0 / amin) + 2.0
    nm = problem.kmesh
    ks = []
    for j0 in range(nm[0]):
        for j1 in range(nm[1]):
            for j2 in range(nm[2]):
                ks.append(j0 / nm[0] * B[0] + j1 / nm[1] * B[1] + j2 / nm[2] * B[2])
    ks = np.array(ks)
    nk = len(ks)
    phis = [eval_bloch(bs, cell.coords, A, k, pts, rcut) for k in ks]
    g = np.fft.fftfreq(n, 1.0 / n)
    G = (np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)) @ B
    pairs = [(a, b) for a in range(nk) for b in (range(nk) if all_pairs else range(a, nk))]
    nao, naux = bs.nfunc, ax.nfunc
    out = np.zeros((len(pairs), naux, nao, nao), np.complex128)
    for t, (k1, k2) in enumerate(pairs):
        k12 = ks[k2] - ks[k1]
        chi = eval_bloch(ax, cell.coords, A, k12, pts, rcut)
        shift = np.exp(-1j * pts @ k12)
        chat = np.fft.fftn((chi * shift).reshape(naux, n, n, n), axes=(1, 2, 3)).reshape(naux, -1)
        chat *= vol / n ** 3
        q = G + k12
        q2 = np.einsum("ij,ij->i", q, q)
        w = np.zeros_like(q2)
        nz = q2 > 1e-14
        w[nz] = 4 * np.pi / vol / q2[nz]
        rho = (np.conj(phis[k1])[:, None, :] * phis[k2][None, :, :]).reshape(nao * nao, -1) * shift
        rhat = np.fft.fftn(rho.reshape(nao * nao, n, n, n), axes=(1, 2, 3)).reshape(nao * nao, -1)
        rhat *= vol / n ** 3
        out[t] = ((np.conj(chat) * w) @ rhat.T).reshape(naux, nao, nao)
    return out
