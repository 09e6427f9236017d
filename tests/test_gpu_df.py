"""GPU parity of the density-fitting pieces through the C ABI: the two-center
metric J^k (Eq. M5, range-separated like the three-center integrals) against
the oracle's orc_j2c, and the fitting solve of Eq. M4 against the oracle's
Cholesky solve on the same inputs.

Bars: J^k within 1e-8 au of the oracle (FP64 bar).  The solve is checked on
the GPU's own J and V (copied to the host), so it is compared with the same
linear system solved by scipy: the difference is bounded by the conditioning,
|d_gpu - d_ref| <= 1e-13 cond(J) max|d| (a backward-stable solve of each has a
forward error of a few units of cond(J) eps |d|), and the residual
|J d - V| <= 1e-12 max|V| * max(1, cond(J) 1e-4)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _j2c(p, **kw):
    import torch

    import paper_2102_02989_amd as P
    J, st = P.build_j2c(p.cell, p.aux, p.kmesh, p.omega, p.thresh, g_thresh=p.g_thr, **kw)
    torch.cuda.synchronize()
    return J, st


@pytest.mark.parametrize("part", [oracle.PART_SR | oracle.PART_G0, oracle.PART_LR, oracle.PART_ALL])
def test_j2c_tiny_parts(part):
    p = synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)
    _say("case J tiny 2x1x1 parts", part)
    J, st = _j2c(p, parts=part)
    ref = oracle.j2c(p, parts=part)
    err = float(np.abs(J.cpu().numpy() - ref).max())
    _say(f"  max err {err:.3e} (max |J| {np.abs(ref).max():.3e}), terms {st['n_sr_terms']}")
    assert err <= TOL


@pytest.mark.parametrize("name", ["C1", "C2", "tiny_1x2x2"])
def test_j2c_workloads(name):
    """C1 (Gamma, omega = 0.1), C2 (2x2x2, omega = 0.1: an erfc tail to ~50
    bohr, 160 aux shells up to f) and the triclinic tiny cell on a 1x2x2 mesh,
    whole J^k tensors."""
    p = {"C1": synth.config1, "C2": synth.config2,
         "tiny_1x2x2": lambda: synth.tiny_problem(kmesh=(1, 2, 2), omega=0.6, diffuse=False)}[name]()
    _say("case J", name)
    J, st = _j2c(p)
    ref = oracle.j2c(p)
    got = J.cpu().numpy()
    err = float(np.abs(got - ref).max())
    herm = max(float(np.abs(got[k] - got[k].conj().T).max()) for k in range(got.shape[0]))
    _say(f"  max err {err:.3e} (max |J| {np.abs(ref).max():.3e}), hermiticity {herm:.1e}, "
         f"SR {st['t_sr_ms']:.2f} ms, LR {st['t_lr_ms']:.2f} ms, terms {st['n_sr_terms']}")
    assert err <= TOL
    assert herm <= 1e-12


def test_j2c_nacl_madelung():
    """The GPU metric of the rock-salt cell of unit Gaussian charges gives the
    Madelung constant (1/2 q^T J q minus the self-interactions)."""
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    _say("case J NaCl Madelung")
    J, _ = _j2c(p)
    J = J.cpu().numpy()[0].real
    q = synth.NACL_CHARGES
    E = 0.5 * q @ J @ q - 0.5 * 8 * 2.0 / np.sqrt(np.pi) * np.sqrt(6.0 * 6.0 / 12.0)
    _say(f"  E - self = {E:.15f}, -alpha_M = {-1.747564594633182:.15f}")
    assert abs(E + 1.747564594633182) <= 1e-9


def _solve_case(p, inplace):
    import torch

    import paper_2102_02989_amd as P
    V, _ = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, g_thresh=p.g_thr)
    J, _ = _j2c(p)
    Vh, Jh = V.cpu().numpy(), J.cpu().numpy()
    d = P.df_solve(p.kmesh, J, V, out=V if inplace else None)
    torch.cuda.synchronize()
    dh = d.cpu().numpy()
    ref = oracle.df_coefficients(Jh, Vh, p.kmesh)
    cond = max(np.linalg.cond(Jh[k]) for k in range(Jh.shape[0]))
    err = float(np.abs(dh - ref).max())
    ks = oracle.kpair_list(p.kmesh)
    n = p.kmesh
    res = 0.0
    for t, (k1, k2) in enumerate(ks):
        j1, j2 = np.unravel_index(k1, n), np.unravel_index(k2, n)
        c = int(np.ravel_multi_index(tuple((b - a) % m for a, b, m in zip(j1, j2, n)), n))
        r = Jh[c] @ dh[t].reshape(dh.shape[1], -1) - Vh[t].reshape(Vh.shape[1], -1)
        res = max(res, float(np.abs(r).max()))
    return err, res, cond, float(np.abs(ref).max()), float(np.abs(Vh).max())


@pytest.mark.parametrize("name,inplace", [("tiny_2x1x1", False), ("tiny_2x1x1", True), ("C1", True)])
def test_df_solve(name, inplace):
    p = {"C1": synth.config1, "tiny_2x1x1": lambda: synth.tiny_problem(kmesh=(2, 1, 1), omega=0.8, diffuse=False)}[
        name]()
    _say("case DF solve", name, "in place" if inplace else "")
    err, res, cond, dmax, vmax = _solve_case(p, inplace)
    _say(f"  max |d_gpu - d_ref| {err:.3e} (max |d| {dmax:.3e}, cond(J) {cond:.2e}), residual {res:.3e}")
    assert err <= 1e-13 * cond * max(dmax, 1.0)
    assert res <= 1e-12 * vmax * max(1.0, cond * 1e-4)


def test_df_exact_fit_nacl():
    """Every AO square is an aux function in the rock-salt cell: the fit of
    rho_jj on the 2x1x1 mesh returns the unit vector e_j (Eq. M4)."""
    import torch

    import paper_2102_02989_amd as P
    p = synth.nacl_problem(a=8.0, alpha_aux=6.0, alpha_ao=3.0, omega=0.5)
    p.kmesh = (2, 1, 1)
    _say("case DF exact fit, rock salt 2x1x1")
    V, _ = P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, p.omega, p.thresh, g_thresh=p.g_thr)
    J, _ = _j2c(p)
    d = P.df_solve(p.kmesh, J, V)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    err = 0.0
    for t in range(d.shape[0]):
        for j in range(8):
            e = np.zeros(8)
            e[j] = 1.0
            err = max(err, float(np.abs(d[t, :, j, j] - e).max()))
    _say(f"  max |d[:, j, j] - e_j| {err:.3e}")
    assert err <= 1e-9


def test_df_singular_metric_reported():
    """The 8-atom cell's 8s6p4d2f aux set is nearly linearly dependent (the
    oracle's J^Gamma has condition number ~4e17): the solve refuses it with
    RSGDF_EINVAL naming the k index, and leaves d untouched."""
    import torch

    import paper_2102_02989_amd as P
    p = synth.config2()
    _say("case DF singular metric (C2)")
    J, _ = _j2c(p)
    V = torch.zeros((P.nkpairs(p.kmesh), p.aux.nfunc, p.basis.nfunc, p.basis.nfunc), dtype=torch.complex128,
                    device="cuda")
    d = torch.full_like(V, 7.0)
    with pytest.raises(P.RsgdfError) as ei:
        P.df_solve(p.kmesh, J, V, out=d)
    _say("  ", ei.value)
    assert ei.value.code == -1 and "singular" in str(ei.value)
    assert float((d - 7.0).abs().max()) == 0.0
