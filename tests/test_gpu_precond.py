"""PCG-DC preconditioner (Sec. III.B.2, Eq. 36) through the C ABI against
the FP64 oracle.

  * P: the device apply z = P r (P built by the library on host threads, in
    FP64) equals the oracle's (P + P^T)/2 times r: |z - z_o| <= 1e-12 max|z_o|
    (same construction, two Cholesky implementations: ~1e-15 observed).
  * Solves with P: the same charges as the oracle's Cholesky solution to the
    bounds of the Jacobi solves (FP64 rel_2 <= 1e-9, mixed <= 1e-8), in
    fewer iterations than the Jacobi (plain) CG.
Workload 1 (L_y = 14.76 A < 2 r_cut) has neighbourhoods with two images of
one atom; workload 2 is the bench geometry.
"""
import json
import os

import numpy as np
import pytest

from oracle import cpm as ocpm
from oracle import ewald as ew
from oracle import precond as pc
from paper_2111_06704_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A, BETA, RC, EPS = wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, wl.KSPACE_EPS
PRM = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                  "paper_constants.json")))["pcg_dc_parameters"]
G, RDC = PRM["g"], PRM["rcut"]


class Case:
    def __init__(self, cfg, frames):
        from paper_2111_06704_amd import cpm
        cpm.lib()
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        self.cpm = cpm
        self.dev = torch.device("cuda:0")
        self.geo, self.ipos, self.iq, self.chi = wl.workload(cfg, frames=frames)
        g = self.geo
        print(f"[case] workload {cfg}: N={g.n} frames={frames}", flush=True)
        self.S = cpm.System(g.pos, g.box, A, BETA, RC, EPS, store=("f32", "bf16"))
        self.S.precond_dc(G, RDC)
        self.P = pc.dc_preconditioner(g.pos, g.box, A, G, RDC)
        km = ew.kmax_from_eps(BETA, EPS)
        E = ew.ewald_matrix(g.pos, g.box, A, BETA, RC, km)
        bo, qso = ew.rhs(g.pos, A, self.ipos, self.iq, self.chi, g.box, BETA, RC, km)
        self.E = E
        self.qo = ocpm.solve(E, bo, qso)
        self.b, self.qsol = self.S.rhs(torch.tensor(self.ipos, device=self.dev),
                                       torch.tensor(self.iq, device=self.dev),
                                       torch.tensor(self.chi, device=self.dev))


@pytest.fixture(scope="module")
def d1():
    return Case(1, 16)


@pytest.fixture(scope="module")
def d2():
    return Case(2, 16)


@pytest.mark.parametrize("which", ["d1", "d2"])
def test_apply_matches_oracle(which, request):
    c = request.getfixturevalue(which)
    rng = np.random.default_rng(7)
    for nf in (1, 16, 21):
        r = rng.standard_normal((nf, c.geo.n))
        z = c.S.precond_apply(torch.tensor(r, device=c.dev)).cpu().numpy()
        zo = r @ c.P.T
        assert np.max(np.abs(z - zo)) <= 1e-12 * np.max(np.abs(zo))


@pytest.mark.parametrize("which", ["d1", "d2"])
@pytest.mark.parametrize("prec_name", ["f64", "f32", "bf16"])
def test_solve_dc(which, prec_name, request):
    c = request.getfixturevalue(which)
    cpm = c.cpm
    prec = {"f64": cpm.PREC_F64, "f32": cpm.PREC_F32, "bf16": cpm.PREC_BF16}[prec_name]
    tol, bound = (1e-12, 1e-9) if prec_name == "f64" else (1e-11, 1e-8)
    q, st = c.S.solve(c.b, c.qsol, tol=tol, precision=prec, inner_tol=1e-2, check_every=4,
                      preconditioner=cpm.PRECOND_DC)
    q0, st0 = c.S.solve(c.b, c.qsol, tol=tol, precision=prec, inner_tol=1e-2, check_every=4)
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), c.qo)
    print(f"[dc] {which} {prec_name}: {st['iterations']} iterations vs {st0['iterations']} (Jacobi)")
    assert r2.max() <= bound
    assert st["max_abs_sum_q"] <= 1e-12
    assert st["iterations"] < 0.8 * st0["iterations"]


@pytest.mark.parametrize("which", ["d1", "d2"])
def test_block_form_matches_oracle(which, request):
    """The block-dense apply (tiles of 64 atoms over the union of their
    columns, on the FP64 matrix cores; the form of systems with 256 tiles or
    more) forced at these sizes: z = P r against the oracle's P (1e-12), with
    the Eq. 37 fill against with_gap(P, p_gap) (the oracle's sum of E^-1),
    and the FP32 solve against the oracle's charges."""
    c = request.getfixturevalue(which)
    cpm = c.cpm
    os.environ["CPM_PRECOND_BLOCK"] = "1"
    try:
        c.S.precond_dc(G, RDC)
    finally:
        del os.environ["CPM_PRECOND_BLOCK"]
    try:
        rng = np.random.default_rng(8)
        for nf in (1, 16, 40):
            r = rng.standard_normal((nf, c.geo.n))
            z = c.S.precond_apply(torch.tensor(r, device=c.dev)).cpu().numpy()
            zo = r @ c.P.T
            assert np.max(np.abs(z - zo)) <= 1e-12 * np.max(np.abs(zo))
        q, st = c.S.solve(c.b, c.qsol, tol=1e-11, precision=cpm.PREC_F32, inner_tol=1e-2,
                          check_every=4, preconditioner=cpm.PRECOND_DC)
        r2, _ = ocpm.rel_errors(q.cpu().numpy(), c.qo)
        assert r2.max() <= 1e-8 and st["max_abs_sum_q"] <= 1e-12
        gap = c.S.precond_gap(True)
        gap_o = pc.p_gap(c.P, float(np.linalg.inv(c.E).sum()))
        assert abs(gap - gap_o) <= 1e-9 * abs(gap_o)
        r = rng.standard_normal((3, c.geo.n))
        z = c.S.precond_apply(torch.tensor(r, device=c.dev)).cpu().numpy()
        zo = r @ pc.with_gap(c.P, gap_o).T
        assert np.max(np.abs(z - zo)) <= 1e-9 * np.max(np.abs(zo))
    finally:
        c.S.precond_dc(G, RDC)   # the default form for the other tests


def test_dc_requires_build():
    from paper_2111_06704_amd import cpm
    cpm.lib()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geo = wl.geometry(1)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS)
    b = torch.zeros((1, geo.n), dtype=torch.float64, device="cuda")
    qs = torch.zeros((1,), dtype=torch.float64, device="cuda")
    with pytest.raises(cpm.CpmError) as ei:
        S.solve(b, qs, preconditioner=cpm.PRECOND_DC)
    assert ei.value.status == cpm.CPM_ESTATE
    with pytest.raises(cpm.CpmError) as ei:
        S.precond_dc(0.0, 8.0)
    assert ei.value.status == cpm.CPM_EINVAL


@pytest.mark.parametrize("prec_name", ["f32", "bf16"])
def test_mixed_dc_on_electrode_indicators(d2, prec_name):
    """Right-hand sides that are nearly eigenvectors of E (the indicator of
    each electrode: the FP64 solve converges in ~16 iterations) under FP32
    or BF16 storage, PCG-DC, checks every 8 iterations and reliable-update
    factor 1e-3. The recursive residual falls below the storage's accuracy
    within one batch; the solver must notice that its recursion stopped
    tracking the true residual (a stalled batch, a true residual above the
    previous one) and restart the direction instead of diverging. Charges
    against the oracle's Cholesky two-step solution (Eq. 35) with Q_sol = 0."""
    c = d2
    cpm = c.cpm
    prec = {"f32": cpm.PREC_F32, "bf16": cpm.PREC_BF16}[prec_name]
    ind = np.stack([(c.geo.electrode == a) for a in range(2)]).astype(np.float64)
    b = torch.tensor(ind, device=c.dev)
    qs = torch.zeros(2, dtype=torch.float64, device=c.dev)
    q, st = c.S.solve(b, qs, tol=1e-11, precision=prec, inner_tol=1e-3, check_every=8,
                      preconditioner=cpm.PRECOND_DC, max_iter=2000)
    qo = ocpm.solve(c.E, ind, 0.0)
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), qo)
    print(f"[indicator] {prec_name}: {st['iterations']} iterations, {st['outer']} true residuals")
    assert r2.max() <= 1e-8
    assert st["iterations"] < 200
