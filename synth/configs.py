"""Synthetic stand-ins for the paper's diamond / MgO / LiF workloads.

The paper's basis sets (cc-pVDZ, GTH-DZVP, cc-pVDZ-jkfit, even-tempered
auxiliary sets) and crystal geometries are not available, so every input is
drawn from a seeded generator with the shapes and exponent ranges of the
five benchmark configurations:

* C1: simple cubic 2-atom cell, a = 6.74 bohr, AO 2s1p (3 primitives each),
  aux 4s2p1d primitive shells, Gamma only, omega = 0.1.
* C2: 8-atom diamond-like cubic cell, AO 3s2p1d (3-6 primitives), aux
  8s6p4d2f primitive shells, 2x2x2 mesh, omega = 0.1.
* C3: the C2 cell and bases on a 3x3x3 mesh.
* C4: 64 uneven cells (2-16 atoms) with the C1 basis recipe per atom.
* C5: 16-atom cubic cell, a = 9.0 bohr, C1 bases, 4x4x4 mesh.

Basis arrays follow the C-ABI layout: per shell (atom, l, nprim, ptr) and
flat (exps, coefs).  Coefficients multiply bare Cartesian monomials
(x-Ax)^i (y-Ay)^j (z-Az)^k exp(-a r^2); a contracted shell is scaled so that
its x^l component has unit norm.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ANG_S, ANG_P, ANG_D, ANG_F = 0, 1, 2, 3


def cart_count(l: int) -> int:
    return (l + 1) * (l + 2) // 2


@dataclasses.dataclass
class Cell:
    lattice: np.ndarray  # (3,3) rows a1, a2, a3 in bohr
    coords: np.ndarray   # (natm,3) bohr

    @property
    def natm(self) -> int:
        return int(self.coords.shape[0])


@dataclasses.dataclass
class Basis:
    shell_atom: np.ndarray   # int32 [nshell]
    shell_l: np.ndarray      # int32 [nshell]
    shell_nprim: np.ndarray  # int32 [nshell]
    shell_ptr: np.ndarray    # int32 [nshell]
    exps: np.ndarray         # float64 [nprim_total]
    coefs: np.ndarray        # float64 [nprim_total]

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nfunc(self) -> int:
        return int(sum(cart_count(int(l)) for l in self.shell_l))

    def offsets(self) -> np.ndarray:
        out = np.zeros(self.nshell + 1, dtype=np.int64)
        for s, l in enumerate(self.shell_l):
            out[s + 1] = out[s] + cart_count(int(l))
        return out


@dataclasses.dataclass
class Problem:
    name: str
    cell: Cell
    basis: Basis
    aux: Basis
    kmesh: tuple
    omega: float
    thresh: float = 1e-10
    g_thr: float = 1e-12


def _x_norm2(l: int, exps: np.ndarray, coefs: np.ndarray) -> float:
    """Squared norm of the x^l component of a contracted Cartesian shell."""
    s = 0.0
    dfac = 1.0
    for k in range(2 * l - 1, 0, -2):
        dfac *= k
    for i in range(len(exps)):
        for j in range(len(exps)):
            a = exps[i] + exps[j]
            s += coefs[i] * coefs[j] * dfac / (2.0 * a) ** l * (math.pi / a) ** 1.5
    return s


class _ShellList:
    def __init__(self):
        self.atom, self.l, self.nprim, self.ptr = [], [], [], []
        self.exps, self.coefs = [], []

    def add(self, atom: int, l: int, exps, coefs):
        exps = np.asarray(exps, dtype=np.float64)
        coefs = np.asarray(coefs, dtype=np.float64)
        order = np.argsort(-exps)
        exps, coefs = exps[order], coefs[order]
        coefs = coefs / math.sqrt(_x_norm2(l, exps, coefs))
        self.atom.append(atom)
        self.l.append(l)
        self.nprim.append(len(exps))
        self.ptr.append(len(self.exps))
        self.exps.extend(exps.tolist())
        self.coefs.extend(coefs.tolist())

    def basis(self) -> Basis:
        return Basis(
            np.asarray(self.atom, np.int32), np.asarray(self.l, np.int32),
            np.asarray(self.nprim, np.int32), np.asarray(self.ptr, np.int32),
            np.asarray(self.exps, np.float64), np.asarray(self.coefs, np.float64))


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def _draw_atom_bases(rng, atom, ao_shells, ao_nprim, ao_range, aux_shells, aux_range, bs, ax):
    """Draw order per atom: AO shells in listed order (nprim, exponents,
    coefficients), then aux shells (exponents)."""
    for l in ao_shells:
        n = ao_nprim(rng)
        e = _log_uniform(rng, ao_range[0], ao_range[1], n)
        c = rng.normal(size=n)
        bs.add(atom, l, e, c)
    for l in aux_shells:
        e = _log_uniform(rng, aux_range[0], aux_range[1], 1)
        ax.add(atom, l, e, [1.0])


C1_AO = [ANG_S, ANG_S, ANG_P]
C1_AUX = [ANG_S] * 4 + [ANG_P] * 2 + [ANG_D]
C2_AO = [ANG_S] * 3 + [ANG_P] * 2 + [ANG_D]
C2_AUX = [ANG_S] * 8 + [ANG_P] * 6 + [ANG_D] * 4 + [ANG_F] * 2


def _c1_bases(rng, natm):
    bs, ax = _ShellList(), _ShellList()
    for atom in range(natm):
        _draw_atom_bases(rng, atom, C1_AO, lambda r: 3, (0.1, 10.0), C1_AUX, (0.2, 20.0), bs, ax)
    return bs.basis(), ax.basis()


def config1(omega: float = 0.1, seed: int = 0) -> Problem:
    a = 6.74
    cell = Cell(np.eye(3) * a, np.array([[0.0, 0.0, 0.0], [a / 4, a / 4, a / 4]]))
    rng = np.random.default_rng(seed)
    bs, ax = _c1_bases(rng, 2)
    return Problem("C1", cell, bs, ax, (1, 1, 1), omega)


def _diamond_cell(a=6.74):
    fr = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    fr = np.vstack([fr, fr + 0.25])
    return Cell(np.eye(3) * a, fr * a)


def _c2_bases(rng, natm):
    bs, ax = _ShellList(), _ShellList()
    for atom in range(natm):
        _draw_atom_bases(rng, atom, C2_AO, lambda r: int(r.integers(3, 7)), (0.05, 30.0),
                         C2_AUX, (0.2, 20.0), bs, ax)
    return bs.basis(), ax.basis()


def config2(omega: float = 0.1, seed: int = 0, kmesh=(2, 2, 2)) -> Problem:
    cell = _diamond_cell()
    rng = np.random.default_rng(seed)
    bs, ax = _c2_bases(rng, cell.natm)
    return Problem("C2", cell, bs, ax, tuple(kmesh), omega)


def config3(omega: float = 1.5, seed: int = 0) -> Problem:
    p = config2(omega=omega, seed=seed, kmesh=(3, 3, 3))
    p.name = "C3"
    return p


def _random_positions(rng, natm, a, dmin=2.0, max_tries=200000):
    pos = []
    tries = 0
    while len(pos) < natm:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling did not converge")
        f = rng.uniform(0.0, 1.0, 3)
        ok = True
        for g in pos:
            d = f - g
            d -= np.round(d)
            if np.linalg.norm(d * a) < dmin:
                ok = False
                break
        if ok:
            pos.append(f)
    return np.array(pos) * a


def config4_cells(ncell: int = 64):
    """64 uneven cells: nat ~ U{2..16}, simple cubic a ~ U[5,9] (redrawn so the
    packing fraction of 2-bohr spheres stays <= 0.3), C1 bases per atom, k-mesh
    from {1, 2^3, 3^3}."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(0).spawn(ncell)):
        rng = np.random.default_rng(ss)
        nat = int(rng.integers(2, 17))
        a = float(rng.uniform(5.0, 9.0))
        if nat * 4.19 / a ** 3 > 0.3:
            a = float(rng.uniform(max(5.0, (nat * 4.19 / 0.3) ** (1.0 / 3.0)), 9.0))
        pos = _random_positions(rng, nat, a)
        bs, ax = _c1_bases(rng, nat)
        km = [(1, 1, 1), (2, 2, 2), (3, 3, 3)][int(rng.integers(0, 3))]
        out.append(Problem(f"C4[{i}]", Cell(np.eye(3) * a, pos), bs, ax, km, 0.1))
    return out


def config5(seed: int = 0, kmesh=(4, 4, 4)) -> Problem:
    rng = np.random.default_rng(seed)
    a = 9.0
    pos = _random_positions(rng, 16, a)
    bs, ax = _c1_bases(rng, 16)
    return Problem("C5", Cell(np.eye(3) * a, pos), bs, ax, tuple(kmesh), 0.1)


def tiny_problem(kmesh=(1, 1, 1), omega=0.5, seed=7, diffuse=True) -> Problem:
    """A small triclinic 2-atom cell with s/p/d AO shells and s/p/d/f aux
    shells; with diffuse=True every exponent is <= 1.6 so a real-space grid
    resolves all functions (used by the brute-force FFT check)."""
    rng = np.random.default_rng(seed)
    lat = np.array([[3.6, 0.0, 0.0], [0.6, 3.4, 0.0], [0.3, 0.5, 3.8]])
    coords = np.array([[0.1, 0.2, 0.05], [1.9, 1.6, 2.1]])
    bs, ax = _ShellList(), _ShellList()
    hi = 1.6 if diffuse else 12.0
    ao = [(0, ANG_S, 2), (0, ANG_P, 2), (1, ANG_S, 1), (1, ANG_D, 2)]
    for atom, l, n in ao:
        bs.add(atom, l, _log_uniform(rng, 0.35, hi, n), rng.normal(size=n))
    aux = [(0, ANG_S), (0, ANG_P), (0, ANG_D), (1, ANG_S), (1, ANG_F)]
    for atom, l in aux:
        ax.add(atom, l, _log_uniform(rng, 0.3, hi, 1), [1.0])
    return Problem("tiny", Cell(lat, coords), bs.basis(), ax.basis(), tuple(kmesh), omega)


def nacl_problem(a: float = 8.0, alpha_aux: float = 6.0, alpha_ao: float = 3.0, omega: float = 0.5) -> Problem:
    """Rock salt in its 8-ion conventional cubic cell (nearest-neighbour
    distance a/2).  Every ion carries one aux s primitive normalised to unit
    charge, (alpha/pi)^{3/2} exp(-alpha r^2), and one AO s primitive whose
    square has unit charge, (2 alpha/pi)^{3/4} exp(-alpha r^2).  Ions 0-3
    (face-centred sites) are the cations, 4-7 (shifted by a/2 x) the anions.
    Gamma only."""
    fr = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    fr = np.vstack([fr, fr + np.array([0.5, 0.0, 0.0])])
    cell = Cell(np.eye(3) * a, fr * a)
    n = cell.natm
    idx = np.arange(n, dtype=np.int32)
    ones = np.ones(n, np.int32)
    zeros = np.zeros(n, np.int32)
    aux = Basis(idx, zeros, ones, idx.copy(), np.full(n, alpha_aux), np.full(n, (alpha_aux / math.pi) ** 1.5))
    ao = Basis(idx.copy(), zeros.copy(), ones.copy(), idx.copy(), np.full(n, alpha_ao),
               np.full(n, (2.0 * alpha_ao / math.pi) ** 0.75))
    return Problem("NaCl", cell, ao, aux, (1, 1, 1), omega)


NACL_CHARGES = np.array([1.0] * 4 + [-1.0] * 4)


def supercell(problem: Problem, reps) -> Problem:
    """The Born-von Karman supercell of ``problem``: lattice rows scaled by
    reps, atoms and shells repeated per cell c = (c1 r2 + c2) r3 + c3 (cell
    major, then the original order), Gamma only."""
    reps = tuple(int(r) for r in reps)
    lat = np.asarray(problem.cell.lattice, float)
    cells = [(i, j, k) for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])]
    natm = problem.cell.natm
    coords = np.vstack([problem.cell.coords + np.array(c, float) @ lat for c in cells])

    def tile(b: Basis) -> Basis:
        nprim_tot = len(b.exps)
        return Basis(np.concatenate([b.shell_atom + natm * i for i in range(len(cells))]).astype(np.int32),
                     np.tile(b.shell_l, len(cells)).astype(np.int32),
                     np.tile(b.shell_nprim, len(cells)).astype(np.int32),
                     np.concatenate([b.shell_ptr + nprim_tot * i for i in range(len(cells))]).astype(np.int32),
                     np.tile(b.exps, len(cells)), np.tile(b.coefs, len(cells)))

    sup = Cell(lat * np.array(reps, float)[:, None], coords)
    return Problem(problem.name + f"[{reps[0]}x{reps[1]}x{reps[2]} supercell]", sup, tile(problem.basis),
                   tile(problem.aux), (1, 1, 1), problem.omega, problem.thresh, problem.g_thr)
