"""Pins of the CPU oracle against things other than itself (paper closed
forms, mpmath, numerical quadrature, FFT brute force, exact invariants).

Each test names the passage of arXiv 2102.02989 it checks.
"""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from fft_bruteforce import j3c_fft

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Boys
@pytest.mark.parametrize("m", [0, 1, 2, 3, 5, 7, 9, 12])
def test_boys_vs_mpmath(m):
    """F_m(T) = gamma(m+1/2, T) / (2 T^{m+1/2}) (lower incomplete gamma)."""
    mpmath.mp.dps = 40
    for T in [0.0, 1e-12, 1e-6, 0.3, 1.0, 7.5, 25.0, 39.99, 40.01, 55.0, 120.0, 900.0]:
        if T == 0.0:
            ref = mpmath.mpf(1) / (2 * m + 1)
        else:
            ref = mpmath.gammainc(m + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (m + 0.5))
        got = oracle.boys(m, T)
        assert abs(got - float(ref)) <= 2e-15 * abs(float(ref)), (m, T, got, float(ref))


# ---------------------------------------------------- isolated integrals
def _ss_s_closed(kind, omega, gc, C, ga, A, gb, B):
    """Closed form of (s|w|ss) for unnormalised 1s primitives (Eqs. S3-S9,
    prefactor pi^3/(a_P p)^{3/2}; the printed (pi/4)^3 prefactor does not
    match quadrature).  The caller sets mpmath's working precision."""
    A, B, C = (mpmath.matrix([mpmath.mpf(x) for x in v]) for v in (A, B, C))
    ga, gb, gc, omega = (mpmath.mpf(x) for x in (ga, gb, gc, omega))
    p = ga + gb
    P = (ga * A + gb * B) / p
    ab2 = sum((A[i] - B[i]) ** 2 for i in range(3))
    R = mpmath.sqrt(sum((P[i] - C[i]) ** 2 for i in range(3)))
    eta1 = mpmath.sqrt(gc * p / (gc + p))
    eta2 = 1 / mpmath.sqrt(1 / eta1 ** 2 + 1 / omega ** 2)

    def g(eta):
        if R < mpmath.mpf("1e-30"):
            return 2 * eta / mpmath.sqrt(mpmath.pi)
        return mpmath.erf(eta * R) / R

    pref = mpmath.pi ** 3 / (gc * p) ** mpmath.mpf(1.5) * mpmath.exp(-ga * gb / p * ab2)
    val = {oracle.COUL: g(eta1), oracle.ERF: g(eta2), oracle.ERFC: g(eta1) - g(eta2)}[kind]
    return pref * val


@pytest.mark.parametrize("kind", [oracle.COUL, oracle.ERF, oracle.ERFC])
def test_ss_s_closed_form(kind):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    for _ in range(20):
        gc, ga, gb = np.exp(rng.uniform(np.log(0.05), np.log(30.0), 3))
        omega = float(np.exp(rng.uniform(np.log(0.05), np.log(3.0))))
        A, B, C = rng.normal(size=(3, 3)) * rng.uniform(0.0, 4.0)
        got = oracle.prim3c(kind, omega, 0, gc, C, 0, ga, A, 0, gb, B)[0, 0, 0]
        ref = float(_ss_s_closed(kind, omega, gc, C, ga, A, gb, B))
        # erfc = Coulomb - erf is formed as a difference: error relative to
        # the Coulomb magnitude
        scale = max(1.0, abs(float(_ss_s_closed(oracle.COUL, omega, gc, C, ga, A, gb, B))))
        assert abs(got - ref) <= 2e-14 * scale, (got, ref)
    # coincident centres: R -> 0 limit
    z = np.zeros(3)
    got = oracle.prim3c(kind, 0.4, 0, 0.7, z, 0, 0.9, z, 0, 1.3, z)[0, 0, 0]
    ref = float(_ss_s_closed(kind, 0.4, 0.7, z, 0.9, z, 1.3, z))
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_closed_form_vs_qspace_quadrature():
    """The corrected s-type prefactor pi^3/(a_P p)^{3/2} (Eq. S4 as printed
    carries (pi/4)^3) agrees with the isolated integral evaluated as a 1-D
    radial q-space quadrature: (1/2pi^2) int dq 4pi * w~(q) * sin(qR)/(qR) * Fc Fab."""
    gc, ga, gb, omega = 0.7, 0.6, 0.7, 0.4
    A = np.array([0.0, 0.0, 0.0]); B = np.array([0.0, 0.0, 0.0]); C = np.array([1.9, 0.0, 0.0])
    p = ga + gb
    R = 1.9
    pref = (math.pi / gc) ** 1.5 * (math.pi / p) ** 1.5

    def integrand(q, attenuated):
        w = 4 * math.pi / q ** 2 if q > 0 else 0.0
        if attenuated:
            w *= 1 - math.exp(-q * q / (4 * omega ** 2))
        s = math.sin(q * R) / (q * R) if q > 0 else 1.0
        return q * q / (2 * math.pi ** 2) * w * s * math.exp(-q * q / (4 * gc) - q * q / (4 * p))

    for kind, att in [(oracle.COUL, False), (oracle.ERFC, True)]:
        quad = pref * integrate.quad(lambda q: integrand(q, att), 0, 80, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
        got = oracle.prim3c(kind, omega, 0, gc, C, 0, ga, A, 0, gb, B)[0, 0, 0]
        assert abs(got - quad) <= 1e-12 * abs(quad), (kind, got, quad)


def _deriv_coefs(n, alpha):
    """(x-A)^n g = sum_j c_j d^j/dA^j g for a Gaussian g ~ exp(-alpha (x-A)^2):
    (x-A)^{n+1} g = (1/2alpha) [d/dA ((x-A)^n g) + n (x-A)^{n-1} g]."""
    F = [{0: mpmath.mpf(1)}]
    for k in range(n):
        nxt = {}
        for j, c in F[k].items():
            nxt[j + 1] = nxt.get(j + 1, 0) + c / (2 * alpha)
        if k >= 1:
            for j, c in F[k - 1].items():
                nxt[j] = nxt.get(j, 0) + k * c / (2 * alpha)
        F.append(nxt)
    return F[n]


def _cart(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


CLASSES = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (2, 1, 1), (2, 0, 2), (0, 2, 3), (2, 2, 0), (1, 2, 2),
           (2, 2, 3)]


@pytest.mark.parametrize("la,lb,lc", CLASSES)
def test_higher_l_vs_center_derivatives(la, lb, lc):
    """Cartesian blocks = centre derivatives of the s-type closed form
    (x-A)^n e^{-a(x-A)^2} generated from d/dA_x; derivatives by mpmath at 40
    digits.  Checks the oracle's Obara-Saika recurrences for every class of
    the benchmark bases (l_AO <= 2, l_aux <= 3) and the erfc operator."""
    mpmath.mp.dps = 40
    rng = np.random.default_rng(100 + 10 * la + 3 * lb + lc)
    ga, gb, gc = 0.9, 0.55, 1.3
    omega = 0.45
    A = rng.normal(size=3) * 0.8
    B = rng.normal(size=3) * 0.8
    C = rng.normal(size=3) * 0.8 + np.array([1.0, 0.5, -0.4])
    blk = oracle.prim3c(oracle.ERFC, omega, lc, gc, C, la, ga, A, lb, gb, B)
    scale = np.abs(blk).max()

    def f(*x):
        return _ss_s_closed(oracle.ERFC, omega, gc, x[6:9], ga, x[0:3], gb, x[3:6])

    x0 = [mpmath.mpf(v) for v in list(A) + list(B) + list(C)]
    comps = [(ic, ia, ib) for ic in range(len(_cart(lc))) for ia in range(len(_cart(la)))
             for ib in range(len(_cart(lb)))]
    nsel = 3 if la + lb + lc >= 6 else 8
    if len(comps) > nsel:
        idx = rng.choice(len(comps), nsel, replace=False)
        comps = [comps[i] for i in idx] + [comps[-1]]
    for ic, ia, ib in comps:
        pa, pb, pc = _cart(la)[ia], _cart(lb)[ib], _cart(lc)[ic]
        coef_lists = [_deriv_coefs(pa[d], mpmath.mpf(ga)) for d in range(3)] + \
                     [_deriv_coefs(pb[d], mpmath.mpf(gb)) for d in range(3)] + \
                     [_deriv_coefs(pc[d], mpmath.mpf(gc)) for d in range(3)]
        total = mpmath.mpf(0)

        def rec(i, orders, c):
            nonlocal total
            if i == 9:
                total += c * mpmath.diff(f, x0, tuple(orders))
                return
            for j, cj in coef_lists[i].items():
                rec(i + 1, orders + [j], c * cj)

        rec(0, [], mpmath.mpf(1))
        ref = float(total)
        assert abs(blk[ic, ia, ib] - ref) <= 1e-12 * max(scale, 1e-3), (ic, ia, ib, blk[ic, ia, ib], ref)


# ------------------------------------------------------ Fourier transforms
def test_fourier_transforms_vs_quadrature():
    """Aux and pair transforms (used in Eqs. M10, M11) and overlaps (Eq. M13c)
    against 1-D numerical quadrature of each Cartesian factor."""
    rng = np.random.default_rng(3)

    def q1(f):
        re = integrate.quad(lambda x: f(x).real, -40, 40, limit=400, epsabs=1e-15)[0]
        im = integrate.quad(lambda x: f(x).imag, -40, 40, limit=400, epsabs=1e-15)[0]
        return re + 1j * im

    for l in [0, 1, 2, 3]:
        g = float(rng.uniform(0.3, 3.0))
        C = rng.normal(size=3)
        q = rng.normal(size=3) * 2.0
        for comp, pw in enumerate(_cart(l)):
            ref = 1.0 + 0j
            for d in range(3):
                ref *= q1(lambda x: (x - C[d]) ** pw[d] * np.exp(-g * (x - C[d]) ** 2 - 1j * q[d] * x))
            got = oracle.prim_ft(l, comp, g, C, q)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
    for la, lb in [(0, 0), (1, 0), (1, 2), (2, 2)]:
        ga, gb = rng.uniform(0.3, 3.0, 2)
        A, B = rng.normal(size=(2, 3))
        q = rng.normal(size=3) * 1.5
        for ia, pa in enumerate(_cart(la)):
            for ib, pb in enumerate(_cart(lb)):
                ref = 1.0 + 0j
                ovl = 1.0
                for d in range(3):
                    fx = lambda x, d=d: ((x - A[d]) ** pa[d] * (x - B[d]) ** pb[d] *
                                         np.exp(-ga * (x - A[d]) ** 2 - gb * (x - B[d]) ** 2))
                    ref *= q1(lambda x, fx=fx, d=d: fx(x) * np.exp(-1j * q[d] * x))
                    ovl *= q1(lambda x, fx=fx: fx(x) + 0j).real
                got = oracle.pair_ft(la, ia, ga, A, lb, ib, gb, B, q)
                assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
                assert abs(oracle.overlap(la, ia, ga, A, lb, ib, gb, B) - ovl) <= 1e-12 * max(1.0, abs(ovl))


# ------------------------------------------------------ periodic, absolute
def test_periodic_gamma_vs_fft_bruteforce():
    """Full G=0-removed j3c (SR - G0 + LR, Eqs. M10-M13) at Gamma against a
    real-space-grid FFT evaluation that uses no analytic integral, on a
    triclinic 2-atom cell with s/p/d AO and s/p/d/f aux shells."""
    p = synth.tiny_problem(kmesh=(1, 1, 1), omega=0.7)
    ref = j3c_fft(p, ngrid=28)
    got = oracle.j3c(p, cut=1e-17)
    assert np.abs(got - ref).max() <= 1e-9, np.abs(got - ref).max()


@pytest.mark.slow
def test_periodic_kmesh_vs_fft_bruteforce():
    """As above on a 2x1x1 mesh, all ordered k-pairs: pins the Bloch phase
    convention (Eq. M1 -> e^{+ik2.n} in Eq. M11), the q = G + k12 set and the
    k1 = k2 restriction of the G=0 term."""
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.9)
    ref = j3c_fft(p, ngrid=26, all_pairs=True)
    got = oracle.j3c(p, all_pairs=True, cut=1e-17)
    assert np.abs(got - ref).max() <= 1e-9, np.abs(got - ref).max()


# ------------------------------------------------------ invariants
def test_omega_independence_gamma():
    """SR + LR - G0 does not depend on the range-separation parameter
    (Eq. M9 splits 1/r exactly; Eqs. M10 and M12 evaluate the two parts)."""
    p = synth.config1()
    sel = [0, 4, 6, 7, 13]  # s, p, d aux on both atoms
    V1 = oracle.j3c(p, omega=0.25, aux_shells=sel)
    V2 = oracle.j3c(p, omega=0.5, aux_shells=sel)
    assert np.abs(V1 - V2).max() <= 1e-10, np.abs(V1 - V2).max()
    assert np.abs(V1).max() > 0.1


def test_omega_independence_kmesh_and_hermiticity():
    """omega-independence with k1 != k2 (the LR phase sign and the G=0 term
    only on k1 = k2), Hermiticity V^{k2k1}_{P nu mu} = conj V^{k1k2}_{P mu nu},
    and a real, mu<->nu symmetric Gamma block (Eq. M6, M1)."""
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    V1 = oracle.j3c(p, omega=0.8, all_pairs=True)
    V2 = oracle.j3c(p, omega=1.2, all_pairs=True)
    assert np.abs(V1 - V2).max() <= 1e-10, np.abs(V1 - V2).max()
    nk = 2
    Vk = V1.reshape(nk, nk, *V1.shape[1:])
    herm = np.abs(Vk - np.conj(Vk.transpose(1, 0, 2, 4, 3))).max()
    assert herm <= 1e-12, herm
    g = Vk[0, 0]
    assert np.abs(g.imag).max() <= 1e-13
    assert np.abs(g - g.transpose(0, 2, 1)).max() <= 1e-12


def test_lattice_translation_phase():
    """Moving atom 1 by a lattice vector L multiplies the block by
    e^{+ik1.L} (AO mu on it), e^{-ik2.L} (AO nu on it), e^{+ik12.L} (aux P on it)."""
    p = synth.tiny_problem(kmesh=(1, 1, 2), omega=1.0, diffuse=False)
    V = oracle.j3c(p, all_pairs=True)
    L = p.cell.lattice[0] * 1 - p.cell.lattice[2]
    q = synth.tiny_problem(kmesh=(1, 1, 2), omega=1.0, diffuse=False)
    q.cell.coords = q.cell.coords.copy()
    q.cell.coords[1] += L
    W = oracle.j3c(q, all_pairs=True)
    ks = oracle.kpoints(p)
    on1_ao = np.repeat(p.basis.shell_atom == 1, [synth.cart_count(l) for l in p.basis.shell_l])
    on1_ax = np.repeat(p.aux.shell_atom == 1, [synth.cart_count(l) for l in p.aux.shell_l])
    for t, (k1, k2) in enumerate(oracle.kpair_list(p.kmesh, all_pairs=True)):
        k12 = ks[k2] - ks[k1]
        ph = (np.exp(1j * on1_ax * (k12 @ L))[:, None, None] * np.exp(1j * on1_ao * (ks[k1] @ L))[None, :, None] *
              np.exp(-1j * on1_ao * (ks[k2] @ L))[None, None, :])
        assert np.abs(W[t] - V[t] * ph).max() <= 1e-11


def test_truncation_convergence():
    """Tightening the oracle's per-term cutoff changes nothing above 1e-11
    (SI: screening error controlled by epsilon)."""
    p = synth.config1(omega=0.3)
    sel = [0, 6]
    V1 = oracle.j3c(p, aux_shells=sel, cut=1e-14)
    V2 = oracle.j3c(p, aux_shells=sel, cut=1e-16)
    V3 = oracle.j3c(p, aux_shells=sel, cut=1e-18)
    assert np.abs(V1 - V3).max() <= 2e-11
    assert np.abs(V2 - V3).max() <= 2e-13


# ------------------------------------------------------ bookkeeping
def test_table_s1_nk12_golden():
    """N_k12 column of Table S1: unique k2 - k1 up to inversion."""
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(GOLDEN, "table_s1_nk12.txt"))
            if ln.strip() and not ln.startswith("#")]
    for n, nk, nk12 in rows:
        assert n ** 3 == nk
        assert oracle.unique_k12_count(n) == nk12
        assert ((2 * n - 1) ** 3 + 1) // 2 == nk12


def test_kpair_counts():
    assert oracle.nkpairs((2, 2, 2)) == 36
    assert [oracle.nkpairs((n, n, n)) for n in range(1, 6)] == [1, 36, 378, 2080, 7875]


def test_selection_restricts_work_only():
    """aux shell, AO pair and k-pair selections return exactly the full
    result on the selected entries and zeros elsewhere."""
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    full = oracle.j3c(p)
    aux, pairs, kps = [1, 3], [(0, 3), (1, 1)], [0, 2]
    got = oracle.j3c(p, aux_shells=aux, pairs=pairs, kpairs=kps)
    xo, bo = p.aux.offsets(), p.basis.offsets()
    mask = np.zeros(full.shape, bool)
    for P in aux:
        for mu, nu in pairs:
            mask[kps, xo[P]:xo[P + 1], bo[mu]:bo[mu + 1], bo[nu]:bo[nu + 1]] = True
    assert np.array_equal(got[mask], full[mask])
    assert not np.any(got[~mask])


# ------------------------------------------------- the regime of the workloads
def test_truncation_convergence_omega01():
    """At omega = 0.1, the range separation of every benchmark workload, the
    erfc tail reaches R_c ~ 50 bohr; the oracle's own per-term cutoff (1e-15
    by default) must still be converged there (SI: the screening error is
    controlled by epsilon).  C1, an s and a d aux shell."""
    p = synth.config1()
    sel = [0, 6]
    V15 = oracle.j3c(p, aux_shells=sel, cut=1e-15)
    V18 = oracle.j3c(p, aux_shells=sel, cut=1e-18)
    assert np.abs(V15 - V18).max() <= 1e-11, np.abs(V15 - V18).max()
    assert np.abs(V18).max() > 0.1


def test_omega_independence_omega01_vs_03():
    """j3c at omega = 0.1 (a few q vectors, a long real-space tail) equals
    j3c at omega = 0.3 (Eq. M9 splits 1/r exactly)."""
    p = synth.config1()
    sel = [0, 6]
    V1 = oracle.j3c(p, omega=0.1, aux_shells=sel)
    V3 = oracle.j3c(p, omega=0.3, aux_shells=sel)
    assert np.abs(V1 - V3).max() <= 1e-10, np.abs(V1 - V3).max()


# ------------------------------------------------------ special cases
MADELUNG_NACL = 1.747564594633182  # rock-salt Madelung constant (nearest-neighbour distance units)


def test_nacl_madelung():
    """Rock salt with every ion a unit Gaussian charge (one aux function and
    one AO function whose square is that charge, both tight).  The
    G=0-removed j3c at Gamma gives the electrostatic energy per cell of the
    neutral periodic charge array, 1/2 sum_ij q_i q_j V[P_i; mu_j mu_j]; minus
    each ion's self-interaction (2/sqrt(pi)) eta_1 (the R -> 0 limit of Eq.
    S7's erf form) it is the point-charge Madelung energy, -alpha_M per ion
    pair over the nearest-neighbour distance.  Pins the absolute
    normalisation 4 pi/Omega of Eq. M10, the G=0 term of Eq. M12 and the
    lattice sums of Eq. M13a together."""
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    V = oracle.j3c(p, pairs=[(j, j) for j in range(8)], cut=1e-17)
    assert np.abs(V.imag).max() <= 1e-14
    V = V.real[0]
    q = synth.NACL_CHARGES
    Vd = np.array([[V[i, j, j] for j in range(8)] for i in range(8)])
    E = 0.5 * q @ Vd @ q
    eta1 = math.sqrt(6.0 * 6.0 / (6.0 + 6.0))  # aux exponent 6, AO square exponent 2 x 3
    self_energy = 0.5 * float(np.sum(q ** 2)) * 2.0 / math.sqrt(math.pi) * eta1
    r0 = 8.0 / 2
    assert abs((E - self_energy) - (-4 * MADELUNG_NACL / r0)) <= 1e-9, E - self_energy


def test_bvk_supercell_gamma_equals_kmesh():
    """The Gamma-point j3c of the 2x1x1 Born-von Karman supercell, Fourier
    transformed over the cell indices of mu and nu, equals the 2x1x1 k-mesh
    result:  V^{k1k2}_{P mu nu} = sum_{c1,c2} e^{-ik1.L_c1} e^{+ik2.L_c2}
    V^S[(0,P)][(c1,mu)][(c2,nu)]  (Eq. M14; the supercell's q = 0 maps to
    k12 = 0, Eq. M10)."""
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    Vk = oracle.j3c(p, all_pairs=True, cut=1e-17)
    S = synth.supercell(p, (2, 1, 1))
    VS = oracle.j3c(S, cut=1e-17)[0]
    nx, nf = p.aux.nfunc, p.basis.nfunc
    ks = oracle.kpoints(p)
    Lc = [np.zeros(3), np.asarray(p.cell.lattice[0], float)]
    for t, (k1, k2) in enumerate(oracle.kpair_list(p.kmesh, all_pairs=True)):
        ref = np.zeros((nx, nf, nf), complex)
        for c1 in range(2):
            for c2 in range(2):
                ref += (np.exp(-1j * ks[k1] @ Lc[c1]) * np.exp(1j * ks[k2] @ Lc[c2]) *
                        VS[:nx, c1 * nf:(c1 + 1) * nf, c2 * nf:(c2 + 1) * nf])
        assert np.abs(ref - Vk[t]).max() <= 1e-12, (t, np.abs(ref - Vk[t]).max())


def test_range_separation_free_sum_on_diffuse_basis():
    """Eq. M15: for diffuse functions the j3c is the plain reciprocal-space
    sum (4 pi/Omega) sum_{q != 0} chi~_P(-q) rho^(q)/q^2 with no range
    separation.  With a q sphere large enough for the transforms to decay
    it equals the range-separated result (SR - G0 + LR), at Gamma and with
    k1 != k2."""
    for kmesh in [(1, 1, 1), (2, 1, 1)]:
        p = synth.tiny_problem(kmesh=kmesh, omega=0.7, diffuse=True)
        Vrs = oracle.j3c(p, cut=1e-17, all_pairs=True)
        Vft = oracle.j3c(p, omega=1.2, g_thr=1e-12, parts=oracle.PART_M15, all_pairs=True)
        assert np.abs(Vft - Vrs).max() <= 1e-10, (kmesh, np.abs(Vft - Vrs).max())
        assert np.abs(Vrs).max() > 0.1


# ------------------------------------------------ two-center metric (Eq. M5)
def _two_center_closed(kind, omega, gc, C, ga, A):
    """(c | w | a) for unnormalised 1s primitives: pi^3/(a_c a_a)^{3/2} times
    erf(eta R)/R at eta1 = sqrt(a_c a_a/(a_c + a_a)) (Coulomb), at
    eta2 = (eta1^-2 + w^-2)^{-1/2} (erf), or their difference (erfc)."""
    A, C = (mpmath.matrix([mpmath.mpf(x) for x in v]) for v in (A, C))
    ga, gc, omega = (mpmath.mpf(x) for x in (ga, gc, omega))
    R = mpmath.sqrt(sum((A[i] - C[i]) ** 2 for i in range(3)))
    eta1 = mpmath.sqrt(gc * ga / (gc + ga))
    eta2 = 1 / mpmath.sqrt(1 / eta1 ** 2 + 1 / omega ** 2)

    def g(eta):
        return 2 * eta / mpmath.sqrt(mpmath.pi) if R < mpmath.mpf("1e-30") else mpmath.erf(eta * R) / R

    val = {oracle.COUL: g(eta1), oracle.ERF: g(eta2), oracle.ERFC: g(eta1) - g(eta2)}[kind]
    return mpmath.pi ** 3 / (gc * ga) ** mpmath.mpf(1.5) * val


@pytest.mark.parametrize("kind", [oracle.COUL, oracle.ERF, oracle.ERFC])
def test_two_center_primitive_closed_form(kind):
    """The oracle's two-center primitive integral (its three-center routine
    with the second orbital factor the constant 1) against the s-type closed
    form, and a (d|f) block against centre derivatives of it."""
    mpmath.mp.dps = 40
    rng = np.random.default_rng(21)
    for _ in range(15):
        gc, ga = np.exp(rng.uniform(np.log(0.05), np.log(30.0), 2))
        omega = float(np.exp(rng.uniform(np.log(0.05), np.log(3.0))))
        A, C = rng.normal(size=(2, 3)) * rng.uniform(0.0, 4.0)
        got = oracle.prim3c(kind, omega, 0, gc, C, 0, ga, A, 0, 0.0, A)[0, 0, 0]
        ref = float(_two_center_closed(kind, omega, gc, C, ga, A))
        scale = max(1.0, abs(float(_two_center_closed(oracle.COUL, omega, gc, C, ga, A))))
        assert abs(got - ref) <= 2e-14 * scale, (got, ref)
    if kind != oracle.ERFC:
        return
    la, lc, ga, gc, omega = 2, 3, 0.8, 1.1, 0.5
    A = np.array([0.3, -0.2, 0.5])
    C = np.array([1.2, 0.4, -0.7])
    blk = oracle.prim3c(oracle.ERFC, omega, lc, gc, C, la, ga, A, 0, 0.0, A)
    x0 = [mpmath.mpf(v) for v in list(A) + list(C)]
    for ic, ia in [(0, 0), (3, 1), (9, 5), (5, 2), (7, 4)]:
        pa, pc = _cart(la)[ia], _cart(lc)[ic]
        coef = [_deriv_coefs(pa[d], mpmath.mpf(ga)) for d in range(3)] + \
               [_deriv_coefs(pc[d], mpmath.mpf(gc)) for d in range(3)]
        total = mpmath.mpf(0)
        f = lambda *x: _two_center_closed(oracle.ERFC, omega, gc, x[3:6], ga, x[0:3])  # noqa: E731

        def rec(i, orders, c):
            nonlocal total
            if i == 6:
                total += c * mpmath.diff(f, x0, tuple(orders))
                return
            for j, cj in coef[i].items():
                rec(i + 1, orders + [j], c * cj)

        rec(0, [], mpmath.mpf(1))
        assert abs(blk[ic, ia, 0] - float(total)) <= 1e-12 * max(np.abs(blk).max(), 1e-3), (ic, ia)


def test_j2c_invariants():
    """J^k (Eq. M5 with the range separation of Eq. M9): omega-independent,
    Hermitian per k, positive definite (a Coulomb metric with q = 0 removed)."""
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    J1 = oracle.j2c(p)
    J2 = oracle.j2c(p, omega=1.3)
    assert np.abs(J1 - J2).max() <= 1e-10, np.abs(J1 - J2).max()
    for k in range(J1.shape[0]):
        assert np.abs(J1[k] - J1[k].conj().T).max() <= 1e-13
        assert np.linalg.eigvalsh(J1[k]).min() > 0.0
    assert np.abs(J1[0].imag).max() <= 1e-13  # Gamma: real symmetric


def test_j2c_range_separation_free_and_supercell():
    """Diffuse aux basis: J = the plain q sum of Eq. M15 with 4 pi/(Omega q^2);
    and the 2x1x1 supercell's Gamma metric, Fourier transformed over the cell
    index of Q, is J^k (Eq. M14 for two centres)."""
    pd = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.7, diffuse=True)
    Jrs = oracle.j2c(pd, cut=1e-17)
    Jft = oracle.j2c(pd, omega=1.4, g_thr=1e-12, parts=oracle.PART_M15)
    assert np.abs(Jrs - Jft).max() <= 1e-10, np.abs(Jrs - Jft).max()
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    J = oracle.j2c(p, cut=1e-17)
    JS = oracle.j2c(synth.supercell(p, (2, 1, 1)), cut=1e-17)[0]
    nx = p.aux.nfunc
    ks = oracle.kpoints(p)
    Lc = [np.zeros(3), np.asarray(p.cell.lattice[0], float)]
    for k in range(2):
        ref = sum(np.exp(1j * ks[k] @ Lc[c]) * JS[:nx, c * nx:(c + 1) * nx] for c in range(2))
        assert np.abs(ref - J[k]).max() <= 1e-12


def test_j2c_nacl_madelung():
    """Rock salt of unit Gaussian charges: 1/2 q^T J^Gamma q minus the ions'
    self-interactions (2/sqrt(pi)) sqrt(a a/(a + a)) is the Madelung energy."""
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    J = oracle.j2c(p, cut=1e-17)[0]
    assert np.abs(J.imag).max() <= 1e-14
    q = synth.NACL_CHARGES
    E = 0.5 * q @ J.real @ q
    self_energy = 0.5 * float(np.sum(q ** 2)) * 2.0 / math.sqrt(math.pi) * math.sqrt(6.0 * 6.0 / 12.0)
    assert abs((E - self_energy) - (-4 * MADELUNG_NACL / 4.0)) <= 1e-9, E - self_energy


def test_df_exact_fit():
    """Eq. M4 with a pair density the aux basis holds exactly: in the rock-salt
    cell every AO s function squared is its ion's aux function (cross-image
    products vanish below 1e-40 at these exponents), so
    V^{k1k2}[:, j, j] = J^{k12}[:, j] for every k-pair (the three-center and
    two-center oracles agree), and the fit returns the unit vector e_j."""
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    p.kmesh = (2, 1, 1)
    pairs = [(j, j) for j in range(8)]
    V = oracle.j3c(p, pairs=pairs, cut=1e-17)
    J = oracle.j2c(p, cut=1e-17)
    ks = oracle.kpair_list(p.kmesh)
    for t, (k1, k2) in enumerate(ks):
        c = (k2 - k1) % 2  # k12 on the 2x1x1 mesh
        for j in range(8):
            assert np.abs(V[t, :, j, j] - J[c][:, j]).max() <= 1e-12
    d = oracle.df_coefficients(J, V, p.kmesh)
    for t in range(len(ks)):
        for j in range(8):
            e = np.zeros(8)
            e[j] = 1.0
            assert np.abs(d[t, :, j, j] - e).max() <= 1e-10


def test_coulomb_df_madelung():
    """Integral-direct consumer oracle: with D^k = diag(q_j) in the rock-salt
    cell the electron density is sum_j q_j sum_m phi_j(r - m)^2 exactly (the
    k sum keeps m = n only), the fit is exact, and the Coulomb energy per
    cell (1/2Nk) sum_k Tr(D^k J(k)) is the Madelung energy plus the ions'
    self-interactions, on a 2x1x1 mesh."""
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    p.kmesh = (2, 1, 1)
    q = synth.NACL_CHARGES
    dm = np.array([np.diag(q).astype(complex)] * 2)
    J = oracle.coulomb_df(p, dm, cut=1e-17)
    E = 0.5 * np.einsum("knm,kmn->", dm, J).real / 2
    self_energy = 0.5 * float(np.sum(q ** 2)) * 2.0 / math.sqrt(math.pi) * math.sqrt(6.0 * 6.0 / 12.0)
    assert abs((E - self_energy) - (-4 * MADELUNG_NACL / 4.0)) <= 1e-9, E - self_energy
    for k in range(2):
        assert np.abs(J[k] - J[k].conj().T).max() <= 1e-12
