"""Workload 3 at full size (N = 32768 electrode atoms, 64 frames of 20000
ions, FP32 copy of E, the mixed-precision solve with the settings bench.py
times) against the FP64 oracle on sampled outputs and on properties that
hold at any size.

The oracle cannot form the 32768 x 32768 matrix here, so it checks:
  * E: sampled entries against the literal sum of Eq. 22 (every image with
    d < r_cut, the full K set): |E_gpu - E| <= 1e-12 max|E|; sampled
    diagonal blocks are exactly symmetric; the FP32 copy is the
    round-to-nearest of the FP64 matrix.
  * b: sampled atoms of the first and last frame against the oracle's
    Eq. 25: <= 1e-12 max|b|.
  * q: the constrained minimum of Eq. 28 is the point where E q - b is the
    same constant (the Lagrange multiplier) on every atom and sum q = -Q_sol.
    At every atom of frames 0 and 63 (and of frame 5 for PCG-DC) the oracle
    evaluates (E q)_i matrix-free and b_i itself; the spread of (E q)_i - b_i
    is bounded by twice the residual the solve stops at, |b - E q_b| <=
    1e-11 |b| (bound used: 2e-10 |b|_2, which also covers the oracle's own
    rounding). sum q + Q_sol <= 1e-12 e. The mixed solve and the FP64 solve
    agree to rel_2 <= 1e-8 (a supplement).
"""
import numpy as np
import pytest

from oracle import ewald as ew
from paper_2111_06704_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A, BETA, RC, EPS = wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, wl.KSPACE_EPS


@pytest.fixture(scope="module")
def big():
    from paper_2111_06704_amd import cpm
    cpm.lib()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    geo, ipos, iq, chi = wl.workload(3)
    print(f"[case] workload 3: N={geo.n} frames={ipos.shape[0]} ions={ipos.shape[1]}", flush=True)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",))
    t_chi = torch.tensor(chi, device=dev)
    b, qsol = S.rhs(torch.tensor(ipos, device=dev), torch.tensor(iq, device=dev), t_chi)
    S.set_warm_chi(t_chi)
    q, st = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, warm_start=cpm.WARM_CHI,
                    inner_tol=1e-2, check_every=8)
    q64, st64 = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F64)
    print(f"[case] mixed: {st['iterations']} iterations, FP64: {st64['iterations']}", flush=True)
    return dict(cpm=cpm, S=S, geo=geo, ipos=ipos, iq=iq, chi=chi, b=b.cpu().numpy(),
                qsol=qsol.cpu().numpy(), q=q.cpu().numpy(), st=st, q64=q64.cpu().numpy(),
                km=ew.kmax_from_eps(BETA, EPS))


def _samples(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, k, replace=False))


def test_matrix_sampled_entries(big):
    cpm, S, geo = big["cpm"], big["S"], big["geo"]
    E = S.get_E(cpm.PREC_F64)
    rng = np.random.default_rng(31)
    ii = rng.integers(0, geo.n, 24)
    jj = rng.integers(0, geo.n, 24)
    diag = _samples(geo.n, 6, 32)
    near = _samples(geo.n - 1, 6, 33)
    pairs = list(zip(ii, jj)) + [(i, i) for i in diag] + [(i, i + 1) for i in near]
    vals = E[torch.tensor([p[0] for p in pairs]), torch.tensor([p[1] for p in pairs])].cpu().numpy()
    ref = np.array([ew.ewald_entry_literal(geo.pos[i], geo.pos[j], geo.box, A, A, BETA, RC, big["km"],
                                           same_atom=(i == j)) for i, j in pairs])
    scale = float(np.max(np.abs(ref)))
    assert np.max(np.abs(vals - ref)) <= 1e-12 * scale
    # exact symmetry of sampled blocks, including blocks across the diagonal
    for i0, j0 in ((0, 0), (12288, 4096), (32768 - 512, 16384)):
        blk = E[i0:i0 + 512, j0:j0 + 512]
        tb = E[j0:j0 + 512, i0:i0 + 512].T
        assert torch.equal(blk, tb)
    # the FP32 copy is the rounding of the FP64 matrix
    E32 = S.get_E(cpm.PREC_F32)
    for r0 in range(0, geo.n, 8192):
        assert torch.equal(E32[r0:r0 + 8192], E[r0:r0 + 8192].float())
    del E, E32


def test_rhs_sampled_atoms(big):
    geo = big["geo"]
    at = _samples(geo.n, 8, 34)
    for f in (0, 63):
        bo, qso = ew.rhs(geo.pos[at], A, big["ipos"][f], big["iq"][f], big["chi"][at], geo.box,
                         BETA, RC, big["km"])
        assert np.max(np.abs(big["b"][f, at] - bo)) <= 1e-12 * np.max(np.abs(bo))
        assert big["qsol"][f] == qso


def _stationarity_spread(big, q, f):
    """max over all atoms of |(E q - b)_i - mean|, with (E q)_i and b_i from
    the oracle (matrix-free potentials and direct Ewald through per-axis
    factors of exp(iK.r)); the constrained minimum of Eq. 28 has E q - b
    uniform (Eq. 29)."""
    geo = big["geo"]
    u = ew.potentials_factored(geo.pos, A, q, geo.box, BETA, RC, big["km"])
    bo, qso = ew.rhs_factored(geo.pos, A, big["ipos"][f], big["iq"][f], big["chi"], geo.box,
                              BETA, RC, big["km"])
    assert np.max(np.abs(big["b"][f] - bo)) <= 1e-12 * np.max(np.abs(bo))
    dev = u - bo
    return float(np.max(np.abs(dev - np.mean(dev))))


def test_charges_stationary_and_neutral(big):
    """Every atom of frames 0 and 63: the spread of E q - b is bounded by
    twice the stopping residual, 2e-11 |b|_2 (bound used: 2e-10 |b|_2, which
    also covers the oracle's own rounding)."""
    q = big["q"]
    for f in (0, 63):
        spread = _stationarity_spread(big, q[f], f)
        print(f"[kkt] frame {f}: spread {spread:.3e} over {big['geo'].n} atoms, "
              f"|b|_2 {np.linalg.norm(big['b'][f]):.3e}")
        assert spread <= 2e-10 * np.linalg.norm(big["b"][f])
    assert np.max(np.abs(q.sum(axis=1) + big["qsol"])) <= 1e-12
    assert big["st"]["max_abs_sum_q"] <= 1e-12


def test_mixed_matches_fp64(big):
    q, q64 = big["q"], big["q64"]
    rel = np.linalg.norm(q - q64, axis=1) / np.linalg.norm(q64, axis=1)
    assert rel.max() <= 1e-8


def test_pcg_dc_at_full_size(big):
    """PCG-DC (g = 0.083 / A, r_cut = 8 A) on the same frames: the charges of
    the FP64 Jacobi solve to rel_2 <= 1e-8, stationarity at every atom of frame 5,
    fewer iterations."""
    cpm, S, geo = big["cpm"], big["S"], big["geo"]
    S.precond_dc(0.083, 8.0)
    b = torch.tensor(big["b"], device="cuda")
    qsol = torch.tensor(big["qsol"], device="cuda")
    q, st = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, warm_start=cpm.WARM_CHI,
                    inner_tol=1e-2, check_every=8, preconditioner=cpm.PRECOND_DC)
    q = q.cpu().numpy()
    print(f"[dc] workload 3: {st['iterations']} iterations vs {big['st']['iterations']} (Jacobi)")
    rel = np.linalg.norm(q - big["q64"], axis=1) / np.linalg.norm(big["q64"], axis=1)
    assert rel.max() <= 1e-8
    assert st["iterations"] < big["st"]["iterations"]
    spread = _stationarity_spread(big, q[5], 5)
    assert spread <= 2e-10 * np.linalg.norm(big["b"][5])


def test_bench_step_settings(big):
    """The combination bench.py times at this workload: FP32 E, the committed
    four-layer network's start, PCG-DC with g = 0.08 / A and r_cut = 14 A
    (the block-dense apply on the matrix cores) with the coarse space of
    14 A patches, reliable-update factor 1e-3, checks every 4 iterations.
    All 64 frames within rel_2 1e-8 of the FP64 solve, stationarity at every
    atom of frame 17, sum q + Q_sol <= 1e-12 e."""
    from paper_2111_06704_amd import warmstart
    cpm, S, geo = big["cpm"], big["S"], big["geo"]
    S.precond_dc(0.08, 14.0)
    assert S.precond_coarse(14.0) == 480
    warmstart.load_into(S, geo, warmstart.weights_for(3))
    b = torch.tensor(big["b"], device="cuda")
    qsol = torch.tensor(big["qsol"], device="cuda")
    q, st = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, warm_start=cpm.WARM_MLP,
                    inner_tol=1e-3, check_every=4, preconditioner=cpm.PRECOND_DC)
    q = q.cpu().numpy()
    print(f"[bench settings] workload 3: {st['iterations']} iterations, "
          f"{st['outer']} true residuals, fell back: {st['fell_back']}", flush=True)
    rel = np.linalg.norm(q - big["q64"], axis=1) / np.linalg.norm(big["q64"], axis=1)
    assert rel.max() <= 1e-8
    assert np.max(np.abs(q.sum(axis=1) + big["qsol"])) <= 1e-12
    S.precond_coarse(0.0)
    spread = _stationarity_spread(big, q[17], 17)
    assert spread <= 2e-10 * np.linalg.norm(big["b"][17])
