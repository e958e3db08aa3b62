"""GPU path (C ABI through the ctypes binding) against the FP64 CPU oracle.

Tolerances:
  * E (FP64): |E_gpu - E| <= 1e-12 max|E|  (both sides FP64; phases from the
    same integer k-vectors, erfc from two libraries: ~1e-15 observed).
  * E (FP32 / BF16 copies): |E_low - E| <= u |E| (1 + 1e-6) with the unit
    roundoff u = 2^-24 / 2^-8 of round-to-nearest.
  * b: <= 1e-12 max|b|.
  * q (FP64 CG to tol 1e-12): rel_2 <= 1e-9 per frame; mixed refinement to
    tol 1e-11: rel_2 <= 1e-8; |sum q + Q_sol| <= 1e-12 e.
The charge error bound follows from |dq| / |q| <= kappa(E) |r| / |b| with
kappa(E) ~ 62 (workload 1) and ~ 310 (workload 2), measured by the oracle.
"""
import math

import numpy as np
import pytest

from oracle import cpm as ocpm
from oracle import ewald as ew
from paper_2111_06704_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A, BETA, RC, EPS = wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, wl.KSPACE_EPS


def _cpm():
    from paper_2111_06704_amd import cpm
    cpm.lib()
    return cpm


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


class Case:
    def __init__(self, cfg, frames, store=("f32", "bf16"), jitter=0.0):
        cpm = _cpm()
        self.dev = _dev()
        self.geo, self.ipos, self.iq, self.chi = wl.workload(cfg, frames=frames)
        if jitter > 0:
            self.geo = wl.jitter(self.geo, jitter, 11 + cfg)
        self.km = ew.kmax_from_eps(BETA, EPS)
        g = self.geo
        print(f"[case] workload {cfg}: N={g.n} frames={frames}", flush=True)
        self.S = cpm.System(g.pos, g.box, A, BETA, RC, EPS, store=store)
        self.E = ew.ewald_matrix(g.pos, g.box, A, BETA, RC, self.km)
        self.bo, self.qso = ew.rhs(g.pos, A, self.ipos, self.iq, self.chi, g.box, BETA, RC, self.km)
        self.fac = ocpm.cholesky(self.E)
        _, self.d, _ = ocpm.neutralising_vector(self.fac, g.n)
        self.qo = ocpm.two_step(self.fac, self.bo, self.qso, self.d)
        self.t_ipos = torch.tensor(self.ipos, device=self.dev)
        self.t_iq = torch.tensor(self.iq, device=self.dev)
        self.t_chi = torch.tensor(self.chi, device=self.dev)


@pytest.fixture(scope="module")
def c1():
    return Case(1, 16)


@pytest.fixture(scope="module")
def c2():
    return Case(2, 16)


def _check_E(case):
    cpm = _cpm()
    E = case.E
    Eg = case.S.get_E(cpm.PREC_F64).cpu().numpy()
    assert np.max(np.abs(Eg - E)) <= 1e-12 * np.max(np.abs(E))
    assert np.array_equal(Eg, Eg.T)
    E32 = case.S.get_E(cpm.PREC_F32).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(E32 - E) <= 2.0 ** -24 * np.abs(E) * (1 + 1e-6) + 1e-300)
    E16 = case.S.get_E(cpm.PREC_BF16).float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(E16 - E) <= 2.0 ** -8 * np.abs(E) * (1 + 1e-6) + 1e-300)


def test_matrix_workload1(c1):
    _check_E(c1)


def test_matrix_workload2(c2):
    _check_E(c2)


def test_kvector_count(c1, c2):
    for c in (c1, c2):
        _, K, _ = ew.kvectors(c.geo.box, BETA, c.km)
        d = c.S.describe()
        assert d["n_kvec"] == len(K) and abs(d["kmax"] - c.km) < 1e-14


def _check_rhs(case):
    b, qsol = case.S.rhs(case.t_ipos, case.t_iq, case.t_chi)
    bg = b.cpu().numpy()
    assert np.max(np.abs(bg - case.bo)) <= 1e-12 * np.max(np.abs(case.bo))
    assert np.allclose(qsol.cpu().numpy(), case.qso, atol=0, rtol=0)
    return b, qsol


def test_rhs_workload1(c1):
    _check_rhs(c1)


def test_rhs_workload2(c2):
    _check_rhs(c2)


def test_rhs_without_ions(c1):
    b, qsol = c1.S.rhs(None, None, c1.t_chi)
    assert np.allclose(b.cpu().numpy()[0], c1.chi / ew.K_E, rtol=1e-15, atol=0)
    assert qsol.item() == 0.0


def test_rhs_is_deterministic(c1):
    b1, _ = c1.S.rhs(c1.t_ipos, c1.t_iq, c1.t_chi)
    b2, _ = c1.S.rhs(c1.t_ipos, c1.t_iq, c1.t_chi)
    assert torch.equal(b1, b2)


def test_dprime(c1, c2):
    for c in (c1, c2):
        dp, cele = c.S.dprime()
        dpo = ocpm.neutralising_vector(c.fac, c.geo.n)[0]
        assert np.max(np.abs(dp.cpu().numpy() - dpo)) <= 1e-11 * np.max(np.abs(dpo))
        assert abs(cele / np.sum(dpo) - 1) < 1e-11


@pytest.mark.parametrize("nf", [1, 5, 16, 17, 64, 70])
def test_matvec_all_precisions(c1, nf):
    cpm = _cpm()
    g = torch.Generator(device="cpu").manual_seed(nf)
    P = torch.randn(nf, c1.geo.n, dtype=torch.float64, generator=g).to(c1.dev)
    ref = P.cpu().numpy() @ c1.E.T
    scale = np.max(np.abs(P.cpu().numpy())) * np.max(np.sum(np.abs(c1.E), axis=1))
    for prec, tol in ((cpm.PREC_F64, 1e-14), (cpm.PREC_F32, 1e-6), (cpm.PREC_BF16, 1e-2)):
        V = c1.S.matvec(P, prec).cpu().numpy()
        assert np.max(np.abs(V - ref)) <= tol * scale, prec


def _solve_and_check(case, precision, tol, bound, **kw):
    cpm = _cpm()
    b, qsol = case.S.rhs(case.t_ipos, case.t_iq, case.t_chi)
    q, st = case.S.solve(b, qsol, tol=tol, precision=precision, **kw)
    qg = q.cpu().numpy()
    r2, rm = ocpm.rel_errors(qg, case.qo)
    print(f"[solve] prec={precision} rel2={r2.max():.2e} relmax={rm.max():.2e} "
          f"iters={st['iterations']} outer={st['outer']}", flush=True)
    assert r2.max() <= bound, r2.max()
    assert np.max(np.abs(qg.sum(1) + case.qso)) <= 1e-12
    assert st["max_abs_sum_q"] <= 1e-12
    assert st["max_rel_resid"] <= tol
    return q, st


def test_solve_fp64_workload1(c1):
    _solve_and_check(c1, _cpm().PREC_F64, 1e-12, 1e-9)


def test_solve_fp64_workload2(c2):
    _solve_and_check(c2, _cpm().PREC_F64, 1e-12, 1e-9)


@pytest.mark.parametrize("prec_name", ["f32", "bf16"])
@pytest.mark.parametrize("check_every", [1, 8])
def test_solve_mixed_workload1(c1, prec_name, check_every):
    cpm = _cpm()
    prec = {"f32": cpm.PREC_F32, "bf16": cpm.PREC_BF16}[prec_name]
    _solve_and_check(c1, prec, 1e-11, 1e-8, inner_tol=1e-3, check_every=check_every)


@pytest.mark.parametrize("prec_name", ["f32", "bf16"])
def test_solve_mixed_workload2(c2, prec_name):
    cpm = _cpm()
    prec = {"f32": cpm.PREC_F32, "bf16": cpm.PREC_BF16}[prec_name]
    _solve_and_check(c2, prec, 1e-11, 1e-8, inner_tol=1e-2)


def test_bench_step_workload2(c2):
    """The step bench.py times at workload 2 with its exact settings: FP32 E,
    the committed network's start, PCG-DC (g = 0.08 / A, r_cut 12 A),
    reliable-update factor 1e-4, checks every 4 iterations, tol 1e-11;
    charges of all 16 frames against the oracle's Cholesky solution."""
    cpm = _cpm()
    from paper_2111_06704_amd import warmstart
    S = cpm.System(c2.geo.pos, c2.geo.box, A, BETA, RC, EPS, store=("f32",))
    S.precond_dc(0.08, 12.0)
    warmstart.load_into(S, c2.geo, warmstart.weights_for(2))
    b, qsol = S.rhs(c2.t_ipos, c2.t_iq, c2.t_chi)
    q, st = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, warm_start=cpm.WARM_MLP,
                    inner_tol=1e-4, check_every=4, preconditioner=cpm.PRECOND_DC)
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), c2.qo)
    print(f"[bench-step] iterations {st['iterations']}, initial residual {st['initial_rel_resid']:.3f}")
    assert r2.shape == (16,) and r2.max() <= 1e-8
    assert st["max_abs_sum_q"] <= 1e-12
    assert st["fell_back"] == 0 and st["initial_rel_resid"] < 0.5
    S.close()


def test_jittered_geometry_workload1():
    """Every electrode atom displaced by U(-0.01, 0.01) A: no lattice symmetry
    left (the genericity check of the measurement). E, b and the FP64 and
    mixed solves against the oracle built for the same positions."""
    case = Case(1, 8, jitter=0.01)
    assert np.ptp(case.geo.pos[:, 2][case.geo.electrode == 0]) > 0.005
    _check_E(case)
    _check_rhs(case)
    _solve_and_check(case, _cpm().PREC_F64, 1e-12, 1e-9)
    _solve_and_check(case, _cpm().PREC_F32, 1e-11, 1e-8, inner_tol=1e-3, check_every=4)


def test_solve_ragged_frames(c1):
    """Frame counts that are not a multiple of 16 and exceed one 64-column block."""
    cpm = _cpm()
    ipos, iq = wl.ion_frames(c1.geo, 200, [wl.frame_seed(1, 100 + f) for f in range(70)])
    bo, qso = ew.rhs(c1.geo.pos, A, ipos, iq, c1.chi, c1.geo.box, BETA, RC, c1.km)
    qo = ocpm.two_step(c1.fac, bo, qso, c1.d)
    for nf in (1, 3, 70):
        b, qsol = c1.S.rhs(torch.tensor(ipos[:nf], device=c1.dev), torch.tensor(iq[:nf], device=c1.dev),
                           c1.t_chi)
        q, st = c1.S.solve(b, qsol, tol=1e-12, precision=cpm.PREC_F64)
        r2, _ = ocpm.rel_errors(q.cpu().numpy(), qo[:nf])
        assert r2.max() <= 1e-9 and len(st["frame_iters"]) == nf


def test_warm_chi_start(c1):
    cpm = _cpm()
    c1.S.set_warm_chi(c1.t_chi)
    b, qsol = c1.S.rhs(c1.t_ipos, c1.t_iq, c1.t_chi)
    q, st = c1.S.solve(b, qsol, tol=1e-12, warm_start=cpm.WARM_CHI)
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), c1.qo)
    assert r2.max() <= 1e-9


def test_not_converged_status(c1):
    cpm = _cpm()
    b, qsol = c1.S.rhs(c1.t_ipos, c1.t_iq, c1.t_chi)
    q, st = c1.S.solve(b, qsol, tol=1e-12, max_iter=3, check_every=1, allow_notconv=True)
    assert st["status"] == cpm.CPM_ENOTCONV
    # the returned iterate is still projected to the neutral subspace
    assert np.max(np.abs(q.cpu().numpy().sum(1) + c1.qso)) <= 1e-12


def test_capacitor_through_gpu():
    """Capacitor pin (Sec. III.C) on the GPU path: a = a0, 1 V, no electrolyte."""
    cpm = _cpm()
    dev = _dev()
    geo = wl.geometry(1)
    a0 = 2.93295072600296
    S = cpm.System(geo.pos, geo.box, a0, 0.3, ew.rcut_from_eps(0.3, 1e-12), 1e-12)
    chi = torch.tensor(wl.electrode_potential(geo), device=dev)
    b, qsol = S.rhs(None, None, chi)
    q, _ = S.solve(b, qsol, tol=1e-13)
    q = q.cpu().numpy()[0]
    na = int(np.sum(geo.electrode == 0))
    eps0 = 1.0 / (4 * math.pi * ew.K_E)
    q_cont = eps0 * (1 / 40.0 + 1 / 20.0) / geo.sheet_density
    assert np.ptp(q[:na]) / abs(q[:na].mean()) < 1e-9
    assert abs(q[:na].mean() / q_cont - 1) < 1e-5


def test_capacitor_with_slab_correction_through_gpu():
    """Slab geometry (Eq. 39): only the inner 40 A gap carries the field; at
    a = a0 the charge is the continuum eps0 dV / d1 per area."""
    cpm = _cpm()
    dev = _dev()
    geo = wl.geometry(1)
    a0 = 2.93295072600296
    S = cpm.System(geo.pos, geo.box, a0, 0.3, ew.rcut_from_eps(0.3, 1e-12), 1e-12, slab=True)
    chi = torch.tensor(wl.electrode_potential(geo), device=dev)
    b, qsol = S.rhs(None, None, chi)
    q, _ = S.solve(b, qsol, tol=1e-13)
    q = q.cpu().numpy()[0]
    na = int(np.sum(geo.electrode == 0))
    eps0 = 1.0 / (4 * math.pi * ew.K_E)
    assert np.ptp(q[:na]) / abs(q[:na].mean()) < 1e-9
    assert abs(q[:na].mean() / (eps0 / 40.0 / geo.sheet_density) - 1) < 1e-5


@pytest.mark.parametrize("cfg", [1, 2])
def test_slab_correction_charges(cfg):
    """Charges with the correction of Eq. 39 against the oracle's literal
    Eq. 39 matrix solved as the bordered system (Eq. 29): rel_2 <= 1e-9."""
    cpm = _cpm()
    dev = _dev()
    geo, ipos, iq, chi = wl.workload(cfg, frames=4)
    km = ew.kmax_from_eps(BETA, EPS)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, slab=True)
    b, qsol = S.rhs(torch.tensor(ipos, device=dev), torch.tensor(iq, device=dev),
                    torch.tensor(chi, device=dev))
    q, st = S.solve(b, qsol, tol=1e-12)
    EL = ew.ewald_matrix(geo.pos, geo.box, A, BETA, RC, km, slab=True)
    bl, qs = ew.rhs(geo.pos, A, ipos, iq, chi, geo.box, BETA, RC, km, slab=True)
    qo = np.array([ocpm.bordered(EL, bl[f], qs[f])[0] for f in range(len(qs))])
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), qo)
    assert r2.max() <= 1e-9
    assert st["max_abs_sum_q"] <= 1e-12


def test_point_charge_madelung_through_gpu():
    """SC and BCC Wigner constants (Supplementary Note) with point charges."""
    cpm = _cpm()
    _dev()
    beta = 5.0
    rc, km = ew.rcut_from_eps(beta, 1e-14), ew.kmax_from_eps(beta, 1e-14)
    S = cpm.System(np.array([[0.3, 0.2, 0.1]]), [1, 1, 1], math.inf, beta, rc, kmax_override=km)
    assert abs(S.get_E().item() + 2.837297479) < 1e-9
    S2 = cpm.System(np.array([[0.1, 0.1, 0.1], [0.6, 0.6, 0.6]]), [1, 1, 1], math.inf, beta, rc,
                    kmax_override=km)
    assert np.all(np.abs(S2.get_E().sum(1).cpu().numpy() / -3.63923345028097 - 1) < 1e-9)


def test_mixed_widths_literal():
    """Per-atom Gaussian widths, a point charge and an anisotropic box vs the
    literal term-by-term Eq. 22."""
    cpm = _cpm()
    _dev()
    rng = np.random.default_rng(3)
    box = np.array([5.0, 6.0, 7.5])
    pos = rng.random((5, 3)) * box
    a = np.array([1.2, 2.0, np.inf, 1.7, 3.0])
    km = ew.kmax_from_eps(0.9, 1e-10)
    rc = ew.rcut_from_eps(0.9, 1e-10)
    El = ew.ewald_matrix_literal(pos, box, a, 0.9, rc, km)
    S = cpm.System(pos, box, 1.0, 0.9, rc, kmax_override=km, per_atom_width=a)
    assert np.max(np.abs(S.get_E().cpu().numpy() - El)) <= 1e-12 * np.max(np.abs(El))


def test_invalid_inputs():
    cpm = _cpm()
    _dev()
    geo = wl.geometry(1)
    bad = geo.pos.copy()
    bad[3, 1] = np.nan
    with pytest.raises(cpm.CpmError) as e:
        cpm.System(bad, geo.box)
    assert e.value.status == cpm.CPM_EINVAL
    dup = geo.pos.copy()
    dup[5] = dup[4] + 1e-8
    with pytest.raises(cpm.CpmError) as e:
        cpm.System(dup, geo.box)
    assert e.value.status == cpm.CPM_EINVAL
    with pytest.raises(cpm.CpmError):
        cpm.System(geo.pos, geo.box, gauss_inv_width=-1.0)
    S = cpm.System(geo.pos, geo.box)           # no FP32 copy stored
    b = torch.zeros((1, geo.n), dtype=torch.float64, device="cuda")
    with pytest.raises(cpm.CpmError) as e:
        S.solve(b, torch.zeros(1, dtype=torch.float64, device="cuda"), precision=cpm.PREC_F32)
    assert e.value.status == cpm.CPM_EINVAL
    with pytest.raises(cpm.CpmError) as e:
        S.solve(b, torch.zeros(1, dtype=torch.float64, device="cuda"), warm_start=cpm.WARM_MLP)
    assert e.value.status == cpm.CPM_ESTATE


def test_rhs_many_ions_z_windows():
    """9000 ions per frame (the real-space sum then runs over the cell list of
    the ions) on workload 1's geometry, whose L_y = 14.76 A is below 2 r_cut,
    with ions placed across the periodic z boundary (z < 0, near 0, near L_z,
    > L_z): b of every atom against the oracle's Eq. 25, <= 1e-12 max|b|."""
    cpm = _cpm()
    dev = _dev()
    geo = wl.geometry(1)
    km = ew.kmax_from_eps(BETA, EPS)
    ipos, iq = wl.ion_frames(geo, 9000, [wl.frame_seed(1, 900 + f) for f in range(2)])
    lz = geo.box[2]
    rng = np.random.default_rng(77)
    for f in range(2):
        sel = rng.choice(9000, 800, replace=False)
        ipos[f, sel[:200], 2] = rng.uniform(-3.0, 0.0, 200)
        ipos[f, sel[200:400], 2] = rng.uniform(0.0, 3.0, 200)
        ipos[f, sel[400:600], 2] = rng.uniform(lz - 3.0, lz, 200)
        ipos[f, sel[600:], 2] = rng.uniform(lz, lz + 3.0, 200)
    chi = wl.electrode_potential(geo)
    print("[case] workload 1 geometry, 2 frames x 9000 ions", flush=True)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=())
    b, qsol = S.rhs(torch.tensor(ipos, device=dev), torch.tensor(iq, device=dev),
                    torch.tensor(chi, device=dev))
    bo, qso = ew.rhs(geo.pos, A, ipos, iq, chi, geo.box, BETA, RC, km)
    assert np.max(np.abs(b.cpu().numpy() - bo)) <= 1e-12 * np.max(np.abs(bo))
    assert np.array_equal(qsol.cpu().numpy(), qso)
    b2, _ = S.rhs(torch.tensor(ipos, device=dev), torch.tensor(iq, device=dev),
                  torch.tensor(chi, device=dev))
    assert torch.equal(b, b2)   # the sorted order is fixed: bitwise reproducible


@pytest.mark.parametrize("cfg,m,frames", [(1, 40000, 2), (2, 40000, 1)])
def test_rhs_beyond_one_sorting_workgroup(cfg, m, frames):
    """More than 32768 ions per frame (workload 5 has 200000): the cell list
    sorts each frame in several chunks. Ions are drawn over 1.5 box edges in
    x, y and z (positions outside [0, L) wrap). b of every atom against the
    oracle's Eq. 25, <= 1e-12 max|b|, Q_sol exact, and bitwise
    reproducible."""
    cpm = _cpm()
    dev = _dev()
    geo = wl.geometry(cfg)
    km = ew.kmax_from_eps(BETA, EPS)
    rng = np.random.default_rng(5000 + cfg)
    ipos = rng.random((frames, m, 3)) * geo.box * 1.5 - 0.25 * geo.box
    iq = np.where(np.arange(m) < m // 2, 1.0, -1.0)[None, :].repeat(frames, axis=0)
    iq[:, :7] = 2.0   # a charged frame
    chi = wl.electrode_potential(geo)
    print(f"[case] workload {cfg} geometry, {frames} frames x {m} ions", flush=True)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=())
    t_ipos, t_iq, t_chi = (torch.tensor(x, device=dev) for x in (ipos, iq, chi))
    b, qsol = S.rhs(t_ipos, t_iq, t_chi)
    bo, qso = ew.rhs(geo.pos, A, ipos, iq, chi, geo.box, BETA, RC, km)
    assert np.max(np.abs(b.cpu().numpy() - bo)) <= 1e-12 * np.max(np.abs(bo))
    assert np.array_equal(qsol.cpu().numpy(), qso)
    b2, _ = S.rhs(t_ipos, t_iq, t_chi)
    assert torch.equal(b, b2)


def test_indefinite_matrix_reports_not_spd():
    """Two point charges (a = inf) 0.8 A apart in a 6 A cube: the point-charge
    Ewald diagonal xi / L is negative and E has the eigenvalues -1.26 along
    (1, -1) and 0.31 along (1, 1). d' (along (1, 1)) still solves; a right-hand
    side mostly along (1, -1) makes the CG break down (p^T E p <= 0), and the
    solve returns CPM_ENOTSPD with a message."""
    cpm = _cpm()
    dev = _dev()
    pos = np.array([[1.0, 1.0, 1.0], [1.8, 1.0, 1.0]])
    box = np.array([6.0, 6.0, 6.0])
    km = ew.kmax_from_eps(0.8, 1e-12)
    E = ew.ewald_matrix(pos, box, np.inf, 0.8, ew.rcut_from_eps(0.8, 1e-12), km)
    assert np.min(np.linalg.eigvalsh(E)) < 0
    S = cpm.System(pos, box, math.inf, 0.8, ew.rcut_from_eps(0.8, 1e-12), kmax_override=km)
    b = torch.tensor([[1.3, -0.7]], dtype=torch.float64, device=dev)   # mostly along (1, -1)
    qs = torch.zeros((1,), dtype=torch.float64, device=dev)
    with pytest.raises(cpm.CpmError) as ei:
        S.solve(b, qs, tol=1e-10)
    assert ei.value.status == cpm.CPM_ENOTSPD
    assert "positive definite" in str(ei.value)


def test_allocation_failure_reports_enomem_and_leaves_no_state():
    """An E of n = 2^20 atoms (8.8 TB in FP64) cannot be allocated:
    cpm_build_E returns CPM_ENOMEM, frees what it took, and a normal system
    is built and solved correctly afterwards."""
    cpm = _cpm()
    dev = _dev()
    n = 1 << 20
    side = 102.4
    g = np.arange(128) * (side / 128)
    pos = np.stack(np.meshgrid(g, g, np.arange(64) * (side / 64), indexing="ij"), axis=-1).reshape(-1, 3)
    assert len(pos) == n
    free0 = torch.cuda.mem_get_info()[0]
    with pytest.raises(cpm.CpmError) as ei:
        cpm.System(pos, np.array([side, side, side]), A, BETA, RC, EPS)
    assert ei.value.status == cpm.CPM_ENOMEM
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    case = Case(1, 4, store=("f32",))
    _solve_and_check(case, cpm.PREC_F64, 1e-12, 1e-9)


@pytest.mark.parametrize("slab", [False, True])
def test_point_charge_simplification_capacitor_through_gpu(slab):
    """Point-charge simplification (Sec. III.C) on the GPU path: graphene
    point charges with the self-energy sqrt(2/pi) a0, 1 V, no electrolyte.
    At a0 the lattice term vanishes, so the sheets carry the continuum charge
    (3D periodic: eps0 dV (1/d1 + 1/d2); with Eq. 39: eps0 dV / d1) to the
    Ewald accuracy 1e-12; uniform per sheet to 1e-9."""
    cpm = _cpm()
    dev = _dev()
    geo = wl.geometry(1)
    a0 = 2.93295072600296
    S = cpm.System(geo.pos, geo.box, a0, 0.3, ew.rcut_from_eps(0.3, 1e-12), 1e-12, slab=slab,
                   point_charge_self=True)
    chi = torch.tensor(wl.electrode_potential(geo), device=dev)
    b, qsol = S.rhs(None, None, chi)
    q, _ = S.solve(b, qsol, tol=1e-13)
    q = q.cpu().numpy()[0]
    na = int(np.sum(geo.electrode == 0))
    eps0 = 1.0 / (4 * math.pi * ew.K_E)
    q_cont = eps0 * (1 / 40.0 if slab else (1 / 40.0 + 1 / 20.0)) / geo.sheet_density
    assert np.ptp(q[:na]) / abs(q[:na].mean()) < 1e-9
    assert abs(q[:na].mean() / q_cont - 1) < 1e-9


@pytest.mark.parametrize("cfg", [1, 2])
def test_point_charge_simplification_charges(cfg):
    """E, b and the FP64 and mixed charges of the point-charge simplification
    (a = 1.979 as self-energy width) against the oracle: E within 1e-12
    max|E| and exactly symmetric, b within 1e-12 max|b|, q (FP64, tol 1e-12)
    rel_2 <= 1e-9, q (FP32 + PCG-DC, tol 1e-11) rel_2 <= 1e-8."""
    cpm = _cpm()
    dev = _dev()
    geo, ipos, iq, chi = wl.workload(cfg, frames=4)
    km = ew.kmax_from_eps(BETA, EPS)
    print(f"[case] point-charge simplification, workload {cfg}", flush=True)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",), point_charge_self=True)
    E = ew.ewald_matrix_point_self(geo.pos, geo.box, A, BETA, RC, km)
    Eg = S.get_E(cpm.PREC_F64).cpu().numpy()
    assert np.max(np.abs(Eg - E)) <= 1e-12 * np.max(np.abs(E))
    assert np.array_equal(Eg, Eg.T)
    bo, qso = ew.rhs(geo.pos, np.inf, ipos, iq, chi, geo.box, BETA, RC, km)
    b, qsol = S.rhs(torch.tensor(ipos, device=dev), torch.tensor(iq, device=dev),
                    torch.tensor(chi, device=dev))
    assert np.max(np.abs(b.cpu().numpy() - bo)) <= 1e-12 * np.max(np.abs(bo))
    qo = ocpm.solve(E, bo, qso)
    q, _ = S.solve(b, qsol, tol=1e-12)
    assert ocpm.rel_errors(q.cpu().numpy(), qo)[0].max() <= 1e-9
    S.precond_dc(0.15, 7.0)
    q, st = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, inner_tol=1e-3, check_every=4,
                    preconditioner=cpm.PRECOND_DC)
    assert ocpm.rel_errors(q.cpu().numpy(), qo)[0].max() <= 1e-8
    assert st["max_abs_sum_q"] <= 1e-12
