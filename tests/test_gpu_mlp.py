"""GPU warm-start network (cpm_mlp_* through the C ABI) against the FP64 oracle.

Tolerances: the kernels run in FP32, the oracle in FP64. Features are
rounded to FP32 on both sides (|diff| <= 1 ulp); forward outputs agree to
1e-5 relative to the output scale; gradients to 1e-4 relative to their
norm (FP32 accumulation over the batch); one Adam step moves each parameter
by at most lr, and agrees to 1e-4 lr.
"""
import numpy as np
import pytest

from oracle import cpm as ocpm
from oracle import ewald as ew
from oracle import features as ft
from oracle import mlp as omlp
from paper_2111_06704_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A, BETA, RC, EPS = wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, wl.KSPACE_EPS


def _cpm():
    from paper_2111_06704_amd import cpm
    cpm.lib()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return cpm


@pytest.fixture(scope="module")
def sys1():
    cpm = _cpm()
    geo = wl.geometry(1)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",))
    S.mlp_init(geo.layer, geo.n_layers, 0.3, wl.BOND, 0.01)
    return geo, S


def _params(seed):
    from paper_2111_06704_amd import warmstart
    th = warmstart.init_params(seed).astype(np.float64)
    th[omlp.NIN * omlp.NH: omlp.NIN * omlp.NH + omlp.NH] = np.random.default_rng(seed).standard_normal(64) * 0.1
    return th


def test_neighbours_match_oracle(sys1):
    geo, S = sys1
    nbr_o, _ = ft.neighbours(geo.pos, geo.box)
    assert np.array_equal(S.mlp_neighbours(), nbr_o)


def test_neighbours_jittered_graphite():
    cpm = _cpm()
    geo = wl.jitter(wl.geometry(2), 0.01, 3)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS)
    S.mlp_init(geo.layer, geo.n_layers, 0.3, wl.BOND, 0.01)
    nbr_o, _ = ft.neighbours(geo.pos, geo.box)
    assert np.array_equal(S.mlp_neighbours(), nbr_o)


def test_features_match_oracle(sys1):
    geo, S = sys1
    rng = np.random.default_rng(1)
    b = rng.standard_normal((3, geo.n)) * 0.2 + 0.05
    feat = S.mlp_features(torch.tensor(b, device="cuda")).cpu().numpy()
    nbr, dist = ft.neighbours(geo.pos, geo.box)
    Xo = ft.features(b, nbr, dist, geo.layer, geo.n_layers, 0.3, wl.BOND).astype(np.float32)
    assert np.max(np.abs(feat - Xo) / np.maximum(np.abs(Xo), 1e-6)) <= 2.4e-7


def test_forward_and_gradient(sys1):
    geo, S = sys1
    th = _params(3)
    S.mlp_set_params(th.astype(np.float32))
    rng = np.random.default_rng(2)
    for rows in (1, 31, 32, 33, 1000):
        X = rng.standard_normal((rows, 26)).astype(np.float32)
        t = rng.standard_normal(rows).astype(np.float32)
        Xt = torch.tensor(X, device="cuda")
        y = S.mlp_forward(Xt).cpu().numpy()
        yo = omlp.forward(th.astype(np.float32).astype(np.float64), X.astype(np.float64))
        assert np.max(np.abs(y - yo)) <= 1e-5 * max(1.0, np.max(np.abs(yo)))
        loss, g = S.mlp_loss_grad(Xt, torch.tensor(t, device="cuda"))
        lo, go = omlp.loss_grad(th.astype(np.float32).astype(np.float64), X.astype(np.float64),
                                t.astype(np.float64))
        assert abs(loss - lo) <= 1e-5 * max(1.0, lo)
        g = g.cpu().numpy()
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_adam_step(sys1):
    geo, S = sys1
    th = _params(4).astype(np.float32)
    S.mlp_set_params(th)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 26)).astype(np.float32)
    t = rng.standard_normal(300).astype(np.float32)
    lr = 1e-3
    S.mlp_train_step(torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"), lr=lr)
    th_gpu = S.mlp_get_params()
    _, go = omlp.loss_grad(th.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    th_o, _, _ = omlp.adam_step(th.astype(np.float64), np.zeros_like(go), np.zeros_like(go), go, 1, lr)
    # the first Adam step moves every parameter with a non-negligible gradient by ~lr
    big = np.abs(go) > 1e-3 * np.max(np.abs(go))
    assert np.max(np.abs(th_gpu - th_o)[big]) <= 1e-4 * lr + 1e-7


def test_training_reduces_loss_and_start_residual():
    """Train on 96 solver-generated frames of workload 1 (seeds disjoint from
    the evaluation frames) and check that the loss falls and the network
    start has a smaller initial residual than the zero start."""
    cpm = _cpm()
    from paper_2111_06704_amd import warmstart
    geo = wl.geometry(1)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",))
    chi = torch.tensor(wl.electrode_potential(geo), device="cuda")
    seeds = [wl.train_seed(t) for t in range(96)]
    b_all, q_all = warmstart.generate(S, geo, seeds, 200, chi)
    bs, qs = warmstart.scales(b_all, q_all)
    warmstart.init_network(S, geo, bs, qs)
    S.mlp_set_params(warmstart.init_params(7))
    losses = warmstart.train(S, b_all, q_all, epochs=6, batch=1024, lr=3e-3, lr_final=3e-4, seed=8)
    assert losses[-1] < 0.5 * losses[0]
    _, ipos, iq, chi_np = wl.workload(1)
    b, qsol = S.rhs(torch.tensor(ipos, device="cuda"), torch.tensor(iq, device="cuda"), chi)
    q0, st0 = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F64, warm_start=cpm.WARM_ZERO)
    q1, st1 = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F64, warm_start=cpm.WARM_MLP)
    print(f"[warm] initial residual {st1['initial_rel_resid']:.3f}, iterations {st1['iterations']} vs {st0['iterations']}")
    assert st1["initial_rel_resid"] < 0.8
    assert st1["iterations"] <= st0["iterations"]
    km = ew.kmax_from_eps(BETA, EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, A, BETA, RC, km)
    bo, qso = ew.rhs(geo.pos, A, ipos, iq, chi_np, geo.box, BETA, RC, km)
    qo = ocpm.solve(E, bo, qso)
    r2, _ = ocpm.rel_errors(q1.cpu().numpy(), qo)
    assert r2.max() <= 1e-8


def test_broken_network_falls_back(sys1):
    """A network with NaN weights gives a rejected start; the solve still
    returns the correct charges from a zero start."""
    cpm = _cpm()
    geo, S = sys1
    th = _params(9).astype(np.float32)
    th[5] = np.nan
    S.mlp_set_params(th)
    _, ipos, iq, chi = wl.workload(1, frames=4)
    b, qsol = S.rhs(torch.tensor(ipos, device="cuda"), torch.tensor(iq, device="cuda"),
                    torch.tensor(chi, device="cuda"))
    q, st = S.solve(b, qsol, tol=1e-12, warm_start=cpm.WARM_MLP)
    assert st["fell_back"] == 1
    km = ew.kmax_from_eps(BETA, EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, A, BETA, RC, km)
    bo, qso = ew.rhs(geo.pos, A, ipos, iq, chi, geo.box, BETA, RC, km)
    r2, _ = ocpm.rel_errors(q.cpu().numpy(), ocpm.solve(E, bo, qso))
    assert r2.max() <= 1e-9


def test_solver_warm_start_matches_oracle():
    """The start cpm_solve takes with the network: the fused inference kernel
    (inputs formed from b inside the kernel, both layers on the FP32 matrix
    cores), the neutral shift sum(q0) = -Q_sol and the Lagrange shift
    x0 = q0 + mu0 d', mu0 = mean(b - E q0) (Eq. 29-31), against the oracle's
    features -> FP64 forward pass -> the same shifts with its Cholesky d'.
    Workload 1 with 7 frames (2016 rows: the last 64-row tile is partial),
    the committed workload-2 network. x0 within 2e-5 max|x0| (FP32 network);
    r0 = b - E x0 of the GPU's own x0 within 1e-12 |b| (FP64)."""
    cpm = _cpm()
    from paper_2111_06704_amd import warmstart
    geo, ipos, iq, chi = wl.workload(1, frames=7)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",))
    warmstart.load_into(S, geo, warmstart.DEFAULT_PATH)
    z = np.load(warmstart.DEFAULT_PATH, allow_pickle=False)
    b, qsol = S.rhs(torch.tensor(ipos, device="cuda"), torch.tensor(iq, device="cuda"),
                    torch.tensor(chi, device="cuda"))
    x0, r0 = S.warm_start(b, qsol, cpm.WARM_MLP)
    x0, r0, bn, qs = (t.cpu().numpy() for t in (x0, r0, b, qsol))
    km = ew.kmax_from_eps(BETA, EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, A, BETA, RC, km)
    dprime, _, _ = ocpm.neutralising_vector(ocpm.cholesky(E), geo.n)
    nbr, dist = ft.neighbours(geo.pos, geo.box)
    X = ft.features(bn, nbr, dist, geo.layer, geo.n_layers, float(z["b_scale"]), float(z["r_scale"]))
    q0 = omlp.forward(z["params"].astype(np.float64), X).reshape(7, geo.n) * float(z["q_scale"])
    q0 -= ((q0.sum(axis=1) + qs) / geo.n)[:, None]
    mu0 = np.mean(bn - q0 @ E, axis=1)
    x0o = q0 + mu0[:, None] * dprime[None, :]
    assert np.max(np.abs(x0 - x0o)) <= 2e-5 * np.max(np.abs(x0o))
    assert np.max(np.abs(x0.sum(axis=1) + qs - mu0 * dprime.sum())) <= 1e-4 * np.max(np.abs(x0o))
    assert np.max(np.linalg.norm(r0 - (bn - x0 @ E), axis=1) / np.linalg.norm(bn, axis=1)) <= 1e-12


def test_learned_start_gain_workload2():
    """What the trained network gains over the method without it, at the
    settings bench.py times at workload 2 (FP32 E, PCG-DC g = 0.08 / A with
    r_cut 12 A, reliable-update factor 1e-4, checks every 4 iterations, tol
    1e-11), on the 16 evaluation frames (seeds disjoint from the training
    frames): a smaller initial residual and strictly fewer iterations than
    both the zero start and the free q_chi start."""
    cpm = _cpm()
    from paper_2111_06704_amd import warmstart
    geo, ipos, iq, chi = wl.workload(2)
    S = cpm.System(geo.pos, geo.box, A, BETA, RC, EPS, store=("f32",))
    S.precond_dc(0.08, 12.0)
    t_chi = torch.tensor(chi, device="cuda")
    S.set_warm_chi(t_chi, preconditioner=cpm.PRECOND_DC)
    warmstart.load_into(S, geo, warmstart.DEFAULT_PATH)
    b, qsol = S.rhs(torch.tensor(ipos, device="cuda"), torch.tensor(iq, device="cuda"), t_chi)
    st = {}
    for name, ws in (("zero", cpm.WARM_ZERO), ("chi", cpm.WARM_CHI), ("mlp", cpm.WARM_MLP)):
        _, st[name] = S.solve(b, qsol, tol=1e-11, precision=cpm.PREC_F32, warm_start=ws,
                              inner_tol=1e-4, check_every=4, preconditioner=cpm.PRECOND_DC)
        print(f"[gain] {name}: {st[name]['iterations']} iterations, initial residual "
              f"{st[name]['initial_rel_resid']:.3f}")
    assert st["mlp"]["fell_back"] == 0
    for other in ("zero", "chi"):
        assert st["mlp"]["initial_rel_resid"] < st[other]["initial_rel_resid"]
        assert st["mlp"]["iterations"] < st[other]["iterations"]
