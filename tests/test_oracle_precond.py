"""Pins of the PCG-DC preconditioner oracle (Sec. III.B.2, Eq. 36-37).

What fixes the construction: the neighbourhood count the paper prints for
its Fig. 2 chain; the limit where every local matrix is the whole E (then
the column fill of step 2 must give E^-1 exactly); the closed form for
g -> 0 (Eq. 36 has no off-diagonal then); Eq. 37's p_gap restores the sum
of E^-1; and preconditioned CG with P reaching the Cholesky solution in
fewer iterations than plain CG. Which P is best is a heuristic: parity
unpinned beyond these properties.
"""
import json
import math
import os

import numpy as np

from oracle import cpm as ocpm
from oracle import ewald as ew
from oracle import precond as pc
from paper_2111_06704_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _small_system(n=12, seed=3):
    rng = np.random.default_rng(seed)
    box = np.array([9.0, 10.0, 11.0])
    while True:
        pos = rng.random((n, 3)) * box
        d = np.linalg.norm(pos[:, None] - pos[None], axis=2) + np.eye(n) * 10
        if d.min() > 1.0:
            return pos, box


def test_fig2_chain_neighbourhood():
    g = GOLD["fig2_chain"]
    L = g["box"]
    x = np.arange(g["n_atoms"]) * (L / g["n_atoms"])
    pos = np.stack([x, np.full_like(x, L / 2), np.full_like(x, L / 2)], axis=1)
    nb = pc.neighbourhood(pos, np.array([L, L, L]), g["rcut"])
    assert all(len(jj) + 1 == g["n_cut"] for jj, _ in nb)


def test_whole_matrix_limit_gives_inverse():
    """Local matrices equal to all of E (every atom once): P = E^-1."""
    pos, box = _small_system()
    km = ew.kmax_from_eps(0.5, 1e-8)
    E = ew.ewald_matrix(pos, box, 1.2, 0.5, 6.0, km)
    n = len(pos)
    nbhd = [(np.array([j for j in range(n) if j != t]), None) for t in range(n)]

    def local(tau, jj, pp):
        ix = np.concatenate([[tau], jj])
        return E[np.ix_(ix, ix)]

    P = pc.dc_columns(n, nbhd, local)
    Einv = np.linalg.inv(E)
    assert np.max(np.abs(P - Einv)) <= 1e-12 * np.max(np.abs(Einv))


def test_eq36_limits():
    X = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 2.0, 0], [3.0, 3.0, 0]])
    a = np.full(4, 1.979)
    rc = 5.0
    M = pc.local_matrix(X, a, 0.083, rc)
    assert np.array_equal(M, M.T)
    assert np.allclose(np.diag(M), math.sqrt(2 / math.pi) * 1.979, rtol=0, atol=1e-15)
    # continuity at the cutoff: the coupling vanishes as r -> r_cut
    Y = np.array([[0.0, 0, 0], [rc * (1 - 1e-9), 0, 0]])
    assert abs(pc.local_matrix(Y, a[:2], 0.083, rc)[0, 1]) <= 1e-9
    # g -> 0: no off-diagonal coupling, P = diag(1 / (sqrt(2/pi) a))
    geo = wl.geometry(1)
    P = pc.dc_preconditioner(geo.pos, geo.box, 1.979, 1e-14, 8.0)
    assert np.max(np.abs(P - np.eye(geo.n) / (math.sqrt(2 / math.pi) * 1.979))) <= 1e-12


def test_images_symmetry_and_definiteness():
    """Workload 1 (L_y = 14.76 A < 2 r_cut): some neighbourhoods hold two images
    of one atom; the symmetrised P is symmetric positive definite."""
    geo = wl.geometry(1)
    prm = GOLD["pcg_dc_parameters"]
    nb = pc.neighbourhood(geo.pos, geo.box, prm["rcut"])
    assert any(len(np.unique(jj)) < len(jj) for jj, _ in nb)
    P = pc.dc_preconditioner(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, prm["g"], prm["rcut"])
    assert np.array_equal(P, P.T)
    assert np.linalg.eigvalsh(P)[0] > 0


def test_p_gap_restores_sum_of_inverse():
    pos, box = _small_system(16, 5)
    km = ew.kmax_from_eps(0.5, 1e-8)
    E = ew.ewald_matrix(pos, box, 1.2, 0.5, 6.0, km)
    P = pc.dc_preconditioner(pos, box, 1.2, 0.083, 3.0)
    assert np.count_nonzero(P == 0) > 0
    s = float(np.linalg.inv(E).sum())
    gap = pc.p_gap(P, s)
    assert abs(pc.with_gap(P, gap).sum() - s) <= 1e-12 * abs(s)


def test_pcg_reaches_cholesky_solution_faster():
    geo, ipos, iq, chi = wl.workload(1, frames=1)
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, km)
    b, _ = ew.rhs(geo.pos, wl.GAUSS_INV_WIDTH, ipos, iq, chi, geo.box, wl.EWALD_SPLIT, wl.RCUT, km)
    b = b[0]
    import scipy.linalg as sla
    xo = sla.cho_solve(ocpm.cholesky(E), b)
    prm = GOLD["pcg_dc_parameters"]
    P = pc.dc_preconditioner(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, prm["g"], prm["rcut"])
    x1, k1 = pc.pcg(E, b, P, 1e-12)
    x0, k0 = pc.pcg(E, b, np.eye(geo.n) / E[0, 0], 1e-12)
    assert np.linalg.norm(x1 - xo) <= 1e-9 * np.linalg.norm(xo)
    assert k1 < 0.7 * k0


def test_images_of_one_atom_add_up():
    """Two images of atom 1 in the neighbourhood of atom 0: their entries of
    the column of M^-1 add up in P (step 2). With M = I + c 1 1^T (m x m),
    M^-1 e_0 = e_0 - c / (1 + c m) 1."""
    c = 0.1
    nbhd = [(np.array([1, 1]), None), (np.array([0]), None)]

    def local(tau, jj, pp):
        m = len(jj) + 1
        return np.eye(m) + c * np.ones((m, m))

    P = pc.dc_columns(2, nbhd, local)
    assert math.isclose(P[1, 0], -2 * c / (1 + 3 * c), rel_tol=1e-14)
    assert math.isclose(P[0, 0], 1 - c / (1 + 3 * c), rel_tol=1e-14)
    assert math.isclose(P[0, 1], -c / (1 + 2 * c), rel_tol=1e-14)


# ---- PCG-Normal / PCG-Full (sparsified E^-1, Sec. III.B.2)

def _w1_inverse():
    geo = wl.geometry(1)
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, km)
    return geo, E, np.linalg.inv(E)


def test_sparse_inverse_pattern_by_brute_force():
    """The kept pairs are those with an image closer than rcut, found here by
    looping over the 27 neighbouring images of every pair."""
    pos, box = _small_system(10, seed=5)
    Einv = np.arange(100, dtype=np.float64).reshape(10, 10) + 1.0
    P = pc.sparse_inverse(Einv, pos, box, 4.0)
    for i in range(10):
        for j in range(10):
            dmin = min(np.linalg.norm(pos[j] + np.array([a, b, c]) * box - pos[i])
                       for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
            want = Einv[i, j] if (i == j or dmin < 4.0) else 0.0
            assert P[i, j] == want


def test_sparse_inverse_limits():
    """A cutoff beyond every pair distance keeps E^-1 (preconditioned CG then
    converges in one iteration); one below the nearest-neighbour distance
    keeps its diagonal only."""
    geo, E, Einv = _w1_inverse()
    far = float(np.linalg.norm(geo.box))
    P = pc.sparse_inverse(Einv, geo.pos, geo.box, far)
    assert np.array_equal(P, Einv)
    b = np.random.default_rng(4).standard_normal(geo.n)
    _, it = pc.pcg(E, b, P, 1e-10)
    assert it == 1
    D = pc.sparse_inverse(Einv, geo.pos, geo.box, 0.5 * wl.BOND)
    assert np.array_equal(D, np.diag(np.diag(Einv)))


def test_sparse_inverse_gap_and_fig6_order():
    """Eq. 37 restores the sum of E^-1; a longer cutoff needs no more
    iterations (Fig. 6a: Full before Normal at 8, 4, 2 A), and every one of
    them fewer than plain CG."""
    geo, E, Einv = _w1_inverse()
    P8 = pc.sparse_inverse(Einv, geo.pos, geo.box, 8.0)
    s = float(Einv.sum())
    assert abs(pc.with_gap(P8, pc.p_gap(P8, s)).sum() - s) <= 1e-10 * abs(s)
    b = wl.electrode_potential(geo) / ew.K_E + 0.05 * np.random.default_rng(9).standard_normal(geo.n)
    _, it_cg = pc.pcg(E, b, np.eye(geo.n), 1e-10)
    its = [pc.pcg(E, b, pc.sparse_inverse(Einv, geo.pos, geo.box, rc), 1e-10)[1]
           for rc in (2.0, 4.0, 8.0, 12.0)]
    assert all(a >= c for a, c in zip(its, its[1:])), its
    assert its[0] < it_cg, (its, it_cg)


# ---- coarse-space (two-level) correction: not in the paper; pinned by its
# closed forms


def test_coarse_patches_of_workload1():
    """Two sheets of 6 x 6 four-atom cells in a 25.56 x 14.757 A box: an edge
    of 8 A gives 3 x 2 bins per sheet (floor(L / 8 + 1/2)), 12 patches of 24
    atoms; displacing every atom by up to 0.01 A keeps each sheet one slab
    (12 patches, none across the sheets) and moves only atoms within 0.01 A
    of a bin edge; one bin per slab gives the two sheets."""
    geo = wl.geometry(1)
    pid = pc.coarse_patches(geo.pos, geo.box, 8.0)
    assert pid.max() + 1 == 12
    assert np.all(np.bincount(pid) == 24)
    # one patch never spans both sheets
    for t in range(12):
        assert len(np.unique(geo.layer[pid == t])) == 1
    jit = wl.jitter(geo, 0.01, 5)
    pj = pc.coarse_patches(jit.pos, jit.box, 8.0)
    assert pj.max() + 1 == 12
    for t in range(12):
        assert len(np.unique(geo.layer[pj == t])) == 1
    moved = np.nonzero(pid != pj)[0]
    assert len(moved) > 0   # the lattice has atoms on the bin edges
    w = np.mod(geo.pos[moved, :2], geo.box[:2])
    edges = [geo.box[0] / 3, geo.box[1] / 2]
    near = np.zeros(len(moved), dtype=bool)
    for d, e in enumerate(edges):
        frac = w[:, d] / e
        near |= np.abs(frac - np.round(frac)) * e <= 0.0101
    assert near.all()
    one = pc.coarse_patches(geo.pos, geo.box, 1e3)
    assert np.array_equal(one, geo.layer.astype(np.int64))


def _w1_dc():
    geo = wl.geometry(1)
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    E = ew.ewald_matrix(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, km)
    prm = GOLD["pcg_dc_parameters"]
    P = pc.dc_preconditioner(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, prm["g"], prm["rcut"])
    return geo, E, P


def test_two_level_exact_on_coarse_space_and_definite():
    """M = P_D^T P P_D + Q maps E Z to Z exactly (M E Z = Z: the coarse modes
    converge in one step), is symmetric and positive definite."""
    geo, E, P = _w1_dc()
    pid = pc.coarse_patches(geo.pos, geo.box, 8.0)
    M = pc.two_level(P, E, pid)
    Z = np.zeros((geo.n, pid.max() + 1))
    Z[np.arange(geo.n), pid] = 1.0
    assert np.max(np.abs(M @ E @ Z - Z)) <= 1e-10
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(M).min() > 0.0


def test_two_level_limits():
    """An exact local solve (P = E^-1) stays exact, and one patch per atom
    (Z = I) gives Q = E^-1 whatever P is."""
    geo, E, P = _w1_dc()
    Einv = np.linalg.inv(E)
    pid = pc.coarse_patches(geo.pos, geo.box, 8.0)
    assert np.max(np.abs(pc.two_level(Einv, E, pid) - Einv)) <= 1e-9 * np.max(np.abs(Einv))
    each = np.arange(geo.n)
    assert np.max(np.abs(pc.two_level(P, E, each) - Einv)) <= 1e-9 * np.max(np.abs(Einv))


def test_two_level_reaches_cholesky_solution_faster():
    """PCG with the two-level P reaches the Cholesky solution (1e-9) in fewer
    iterations than with P alone."""
    geo, ipos, iq, chi = wl.workload(1, frames=1)
    _, E, P = _w1_dc()
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    b, _ = ew.rhs(geo.pos, wl.GAUSS_INV_WIDTH, ipos, iq, chi, geo.box, wl.EWALD_SPLIT, wl.RCUT, km)
    b = b[0]
    import scipy.linalg as sla
    xo = sla.cho_solve(ocpm.cholesky(E), b)
    M = pc.two_level(P, E, pc.coarse_patches(geo.pos, geo.box, 8.0))
    x1, k1 = pc.pcg(E, b, M, 1e-12)
    _, k0 = pc.pcg(E, b, P, 1e-12)
    assert np.linalg.norm(x1 - xo) <= 1e-9 * np.linalg.norm(xo)
    assert k1 < k0, (k1, k0)


def test_coarse_patch_counts_of_the_large_workloads():
    """The patch counts the parity tests and the bench rely on, from the rule's
    closed form: 8 graphite layers (one slab each) times nx x ny bins with
    nx = floor(L_x / edge + 1/2): 6 x 10 bins of 14 A at N = 32768 (480
    patches) and 17 x 30 bins of 9 A at N = 131072 (4080 patches), none
    empty, each within one layer."""
    for cfg, edge, nx, ny in ((3, 14.0, 6, 10), (5, 9.0, 17, 30)):
        geo = wl.geometry(cfg)
        assert int(math.floor(geo.box[0] / edge + 0.5)) == nx
        assert int(math.floor(geo.box[1] / edge + 0.5)) == ny
        pid = pc.coarse_patches(geo.pos, geo.box, edge)
        m = int(pid.max()) + 1
        assert m == geo.n_layers * nx * ny
        counts = np.bincount(pid, minlength=m)
        assert counts.min() > 0 and counts.sum() == geo.n
        first = np.zeros(m, dtype=np.int64)
        first[pid] = geo.layer
        assert np.all(first[pid] == geo.layer)   # one layer per patch
