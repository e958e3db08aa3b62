"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test states the passage of arXiv 2111.06704 (or the mathematical fact)
that pins it. None of them re-types the oracle's own formula: they compare
against printed constants, closed forms, a literal term-by-term evaluation,
brute-force image sums, invariances or independent solution routes.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import erf, erfc

from oracle import cpm, ewald as ew
from paper_2111_06704_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
TIGHT = 1e-14


def _params(beta, eps=TIGHT):
    return beta, ew.rcut_from_eps(beta, eps), ew.kmax_from_eps(beta, eps)


def _lattice_2d(kind, nx, ny, R):
    s3 = math.sqrt(3.0)
    if kind == "sq":
        cell, basis = np.array([R, R]), np.array([[0.0, 0.0]])
    elif kind == "hex":
        cell, basis = np.array([R, s3 * R]), np.array([[0.0, 0.0], [R / 2, s3 / 2 * R]])
    elif kind == "kagome":
        cell = np.array([2 * R, 2 * s3 * R])
        basis = np.array([[0, 0], [R, 0], [R / 2, s3 / 2 * R], [R, s3 * R], [0, s3 * R],
                          [1.5 * R, 1.5 * s3 * R]], dtype=float)
    else:
        cell = np.array([3 * R, s3 * R])
        basis = np.array([[0, 0], [R, 0], [1.5 * R, s3 / 2 * R], [2.5 * R, s3 / 2 * R]])
    pts = np.concatenate([basis + np.array([i, j]) * cell for i in range(nx) for j in range(ny)])
    return pts, cell * np.array([nx, ny]), len(basis) / (cell[0] * cell[1])


# --- P1, P2: 3D Madelung constants (Supplementary Note on the Madelung constant)

@pytest.mark.parametrize("beta", [4.0, 6.5])
def test_sc_madelung_constant(beta):
    """One point charge in a unit cube: e_11 = xi (SC Wigner constant)."""
    b, rc, km = _params(beta)
    E = ew.ewald_matrix(np.array([[0.3, 0.2, 0.1]]), [1.0, 1.0, 1.0], np.inf, b, rc, km)
    ref = GOLD["madelung_sc"]["value"]
    assert abs(E[0, 0] - ref) < 1e-9
    # the same entry written out term by term over the full K set
    El = ew.ewald_matrix_literal(np.array([[0.3, 0.2, 0.1]]), [1.0, 1.0, 1.0], np.inf, b, rc, km)
    assert abs(El[0, 0] - E[0, 0]) < 1e-13


def test_bcc_fcc_madelung_constants():
    """Row sums of E x L for the conventional BCC (2 charges) and FCC (4
    charges) cells equal U^BCC and U^FCC; FCC under the digit reading in
    tests/golden/paper_constants.json."""
    b, rc, km = _params(5.0)
    bcc = np.array([[0, 0, 0], [0.5, 0.5, 0.5]]) + 0.1
    fcc = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) + 0.1
    rb = ew.ewald_matrix(bcc, [1, 1, 1], np.inf, b, rc, km).sum(1)
    rf = ew.ewald_matrix(fcc, [1, 1, 1], np.inf, b, rc, km).sum(1)
    assert np.all(np.abs(rb / GOLD["madelung_bcc"]["value"] - 1) < 1e-9)
    assert np.all(np.abs(rf / GOLD["madelung_fcc_reading"]["value"] - 1) < 1e-9)
    assert np.all(np.abs(rf - GOLD["madelung_fcc_printed"]["value"]) > 4.9e-4)
    # scaling: a cell of edge L gives the constant / L
    rb2 = ew.ewald_matrix(bcc * 3.0, [3, 3, 3], np.inf, b / 3, rc * 3, km / 3).sum(1)
    assert np.allclose(rb2 * 3.0, rb, rtol=1e-12, atol=0)


# --- P4: 2D Wigner lattices with a planar neutralising background (Table 1)

@pytest.mark.parametrize("kind,nx,ny", [("sq", 4, 3), ("hex", 4, 2), ("kagome", 2, 2), ("gra", 2, 3)])
def test_2d_lattice_row_sums(kind, nx, ny):
    """One periodic sheet of unit point charges in an L_z-periodic box: the
    potential at a site is pi n L_z / 3 (planar average of a charged sheet
    plus uniform background, zero cell mean) minus U^LATT / R (Table 1)."""
    R = 1.0
    p2, L2, dens = _lattice_2d(kind, nx, ny, R)
    lz = 7.0
    pos = np.column_stack([p2, np.full(len(p2), 2.0)])
    b, rc, km = _params(2.0)
    E = ew.ewald_matrix(pos, [L2[0], L2[1], lz], np.inf, b, rc, km)
    pred = math.pi * dens * lz / 3.0 - GOLD["lattice_2d_unit_bond"][kind] / R
    assert np.max(np.abs(E.sum(1) - pred)) < 5e-11


def test_gaussian_graphene_sheet_row_sum():
    """Graphene sheet of Gaussian charges (R = 1.42, a = 1.979): the row sum
    is the point-charge value of Table 1 plus the Gaussian self-energy
    sqrt(2/pi) a (Eq. 6) minus the erfc(a_ij d)/d screening of the in-sheet
    neighbours (Eq. 20 with a_ij = a / sqrt 2)."""
    R, a = GOLD["gra_bond"]["value"], 1.979
    p2, L2, dens = _lattice_2d("gra", 3, 4, R)
    lz = 20.0
    pos = np.column_stack([p2, np.full(len(p2), 5.0)])
    b, rc, km = _params(0.8)
    E = ew.ewald_matrix(pos, [L2[0], L2[1], lz], a, b, rc, km)
    aij = a / math.sqrt(2.0)
    # direct neighbour sum of the Gaussian screening over in-plane images
    shifts = np.array([[i, j] for i in range(-3, 4) for j in range(-3, 4)]) * L2
    d = np.linalg.norm((p2[None, :, :] - p2[0] + shifts[:, None, :]).reshape(-1, 2), axis=1)
    d = d[d > 0]
    screen = np.sum(erfc(aij * d) / d)
    pred = (math.pi * dens * lz / 3.0 - GOLD["lattice_2d_unit_bond"]["gra"] / R
            + math.sqrt(2.0 / math.pi) * a - screen)
    assert np.max(np.abs(E.sum(1) - pred)) < 1e-10


# --- P5: parallel-plate capacitor (Sec. III.C)

@pytest.mark.parametrize("a", [1.979, 2.93295072600296])
def test_capacitor_charge(a):
    """Two graphene sheets at +-dV/2 (d1 = 40, d2 = 20, 3D periodic, no
    electrolyte). By symmetry each sheet carries a uniform charge +-q with
    q = (dV/k_e) / (4 pi n d1 d2 / L_z + 2 delta), delta = sqrt(2/pi) a -
    U^GRA / R - sum_j erfc(a_ij r_ij) / r_ij. At a = a^0 (Sec. III.C) the
    Gaussian self-energy cancels U^GRA / R and the charge matches the
    continuum capacitor eps0 A dV (1/d1 + 1/d2)."""
    geo = wl.geometry(1)
    b, rc, km = _params(0.3, 1e-12)
    E = ew.ewald_matrix(geo.pos, geo.box, a, b, rc, km)
    bvec = wl.electrode_potential(geo) / ew.K_E
    q = cpm.solve(E, bvec, 0.0)
    na = int(np.sum(geo.electrode == 0))
    qa, qb = q[:na], q[na:]
    assert np.ptp(qa) / abs(qa.mean()) < 1e-9 and np.ptp(qb) / abs(qb.mean()) < 1e-9
    assert abs(qa.mean() + qb.mean()) < 1e-15
    R = GOLD["gra_bond"]["value"]
    aij = a / math.sqrt(2.0)
    _, _, d = ew.real_space_pairs(geo.pos[:1], geo.pos[:na], geo.box, 12.0)
    delta = math.sqrt(2 / math.pi) * a - GOLD["lattice_2d_unit_bond"]["gra"] / R - np.sum(erfc(aij * d) / d)
    lz, d1, d2 = geo.box[2], 40.0, 20.0
    qf = (1.0 / ew.K_E) / (4 * math.pi * geo.sheet_density * d1 * d2 / lz + 2 * delta)
    assert abs(qa.mean() / qf - 1) < 1e-9
    if a == GOLD["gra_alpha0"]["value"]:
        eps0 = 1.0 / (4 * math.pi * ew.K_E)          # e / (V A)
        q_cont = eps0 * 1.0 * (1 / d1 + 1 / d2) / geo.sheet_density
        assert abs(qa.mean() / q_cont - 1) < 1e-5


# --- P6: independence of the Ewald splitting (Sec. II.B: the partition is arbitrary)

def test_split_independence():
    rng = np.random.default_rng(11)
    box = np.array([7.0, 8.5, 9.0])
    pos = rng.random((7, 3)) * box
    a = rng.uniform(1.0, 3.0, 7)
    Es = [ew.ewald_matrix(pos, box, a, *_params(bt, 1e-15)) for bt in (0.5, 0.7, 1.0)]
    scale = np.max(np.abs(Es[0]))
    for E in Es[1:]:
        assert np.max(np.abs(E - Es[0])) < 1e-11 * scale


# --- P7: brute-force image sums (Eq. 8-10, 17 without splitting; tinfoil)

def test_brute_force_energy():
    """For neutral, dipole-free charges the spherical sum over images of
    q_i q_j erf(a_ij d)/d (Eq. 5), with the Gaussian self-energy (Eq. 6),
    converges to 1/2 q^T E q."""
    rng = np.random.default_rng(5)
    box = np.array([6.0, 7.0, 8.0])
    n = 6
    pos = rng.random((n, 3)) * box
    a = np.full(n, 1.5)
    q = rng.standard_normal(n)
    A = np.vstack([np.ones(n), pos.T])
    q = q - A.T @ np.linalg.solve(A @ A.T, A @ q)
    E = ew.ewald_matrix(pos, box, a, *_params(0.6))
    u_ewald = 0.5 * q @ E @ q
    aij = a[0] / math.sqrt(2.0)
    rmax = 400.0
    nm = [int(rmax / box[d]) + 1 for d in range(3)]
    g = np.stack(np.meshgrid(*[np.arange(-m, m + 1) for m in nm], indexing="ij"), -1).reshape(-1, 3)
    Rn = g * box
    Rn = Rn[np.linalg.norm(Rn, axis=1) < rmax]
    u = 0.0
    for i in range(n):
        for j in range(n):
            dd = np.linalg.norm(pos[i] - pos[j] + Rn, axis=1)
            nz = dd > 0
            u += 0.5 * q[i] * q[j] * np.sum(erf(aij * dd[nz]) / dd[nz])
        u += q[i] * q[i] * aij / math.sqrt(math.pi)
    assert abs(u / u_ewald - 1) < 2e-8


# --- P8: symmetric positive definite (Eq. 14: U = 1/2 q^T E q, E symmetric)

def test_workload1_matrix_spd():
    geo = wl.geometry(1)
    E = ew.ewald_matrix(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT,
                        ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS))
    assert np.max(np.abs(E - E.T)) < 1e-14 * np.max(np.abs(E))
    cpm.cholesky(E)
    lam = np.linalg.eigvalsh(E)
    assert lam[0] > 0.4 and lam[-1] / lam[0] < 100


# --- literal Eq. 22 vs the factorised sum (mixed widths, half K set)

def test_literal_matches_factorised():
    rng = np.random.default_rng(3)
    box = np.array([5.0, 6.0, 7.5])
    pos = rng.random((5, 3)) * box
    a = np.array([1.2, 2.0, np.inf, 1.7, 3.0])
    p = _params(0.9, 1e-10)
    El = ew.ewald_matrix_literal(pos, box, a, *p)
    Ef = ew.ewald_matrix(pos, box, a, *p)
    assert np.max(np.abs(El - Ef)) < 1e-12 * np.max(np.abs(El))


# --- P9, P10: neutral solution, gauge invariance, three routes (Eq. 29-35)

def _small_system(seed=2, n=12):
    rng = np.random.default_rng(seed)
    box = np.array([9.0, 10.0, 11.0])
    pos = rng.random((n, 3)) * box
    E = ew.ewald_matrix(pos, box, 1.979, *_params(0.7, 1e-12))
    b = rng.standard_normal(n)
    return E, b


def test_three_routes_agree():
    E, b = _small_system()
    for qsol in (0.0, 0.7):
        q2 = cpm.solve(E, b, qsol)
        qbord, mu = cpm.bordered(E, b, qsol)
        S, d = cpm.s_matrix(E)
        qs = S @ b - qsol * d
        assert abs(q2.sum() + qsol) < 1e-12
        assert np.max(np.abs(q2 - qbord)) < 1e-12 * np.max(np.abs(qbord))
        assert np.max(np.abs(q2 - qs)) < 1e-11 * np.max(np.abs(qbord))
        # the Lagrange shift mu makes E q = b - mu 1 (Eq. 29)
        assert np.max(np.abs(E @ q2 - (b - mu))) < 1e-11 * np.max(np.abs(b))
    # S annihilates uniform shifts (Eq. 33: S 1 = 0)
    assert np.max(np.abs(S @ np.ones(len(b)))) < 1e-12


def test_gauge_invariance():
    E, b = _small_system(4)
    q0 = cpm.solve(E, b, 0.0)
    q1 = cpm.solve(E, b + 3.7, 0.0)                        # chi -> chi + c 1
    q2 = cpm.solve(E + 0.9 * np.ones_like(E), b, 0.0)       # E -> E + c 1 1^T
    assert np.max(np.abs(q1 - q0)) < 1e-12 * np.max(np.abs(q0))
    assert np.max(np.abs(q2 - q0)) < 1e-12 * np.max(np.abs(q0))


def test_not_spd_detected():
    E, _ = _small_system(6)
    with pytest.raises(cpm.NotSPD):
        cpm.cholesky(E - 2.0 * np.eye(len(E)) * np.max(np.abs(E)))


# --- P11: point-charge limit (end of Sec. II.C)

def test_point_charge_limit():
    rng = np.random.default_rng(8)
    box = np.array([8.0, 8.0, 8.0])
    pos = rng.random((4, 3)) * box
    p = _params(0.8, 1e-13)
    Eg = ew.ewald_matrix(pos, box, 1e4, *p)
    Ep = ew.ewald_matrix(pos, box, np.inf, *p)
    off = ~np.eye(4, dtype=bool)
    assert np.max(np.abs((Eg - Ep)[off])) < 1e-12
    assert np.allclose(np.diag(Eg - Ep), math.sqrt(2 / math.pi) * 1e4, rtol=1e-13)


# --- P12 and Fig. 1: the matrix-inversion construction (Sec. III.B.1, S10-S13)

def test_fig1_three_charges():
    L = 1.0
    s = GOLD["fig1_spacing"]["value"] * L
    pos = np.array([[0.4, 0.5, 0.5], [0.4 + s, 0.5, 0.5], [0.4 + 2 * s, 0.5, 0.5]])
    p = _params(6.0)
    E = ew.ewald_matrix(pos, [L, L, L], np.inf, *p)
    xi = GOLD["madelung_sc"]["value"]
    assert np.allclose(np.diag(E), xi, atol=1e-9)
    # hollow matrix + xi 1 1^T with Coulomb increments 1/r at r << L (S7)
    assert abs(E[0, 1] - xi - 1 / s) < 1e-3 and abs(E[0, 2] - xi - 1 / (2 * s)) < 1e-3
    Q, Qinv = cpm.charge_matrix(3)
    assert np.allclose(np.diag(Q), 3.0) and np.allclose(Q[~np.eye(3, dtype=bool)], -1.0)
    g = GOLD["fig1_qtilde_inverse"]
    assert np.allclose(np.diag(Qinv), g["diag"]) and np.allclose(Qinv[~np.eye(3, dtype=bool)], g["offdiag"])
    assert np.allclose(Q @ Qinv, np.eye(3), atol=1e-15)
    Em = cpm.matrix_from_potentials(lambda qv: ew.potentials(pos, np.inf, qv, [L] * 3, *p), 3)
    assert np.max(np.abs(Em - E)) < 1e-11 * np.max(np.abs(E))


def test_matrix_inversion_route_gaussian():
    rng = np.random.default_rng(9)
    box = np.array([10.0, 11.0, 12.0])
    pos = rng.random((9, 3)) * box
    a = rng.uniform(1.0, 3.0, 9)
    p = _params(0.6, 1e-12)
    E = ew.ewald_matrix(pos, box, a, *p)
    Em = cpm.matrix_from_potentials(lambda qv: ew.potentials(pos, a, qv, box, *p), 9)
    assert np.max(np.abs(Em - E)) < 1e-12 * np.max(np.abs(E))


# --- Eq. 25: the electrolyte potential equals the electrode-ion block of E

def test_electrolyte_potential_is_cross_block():
    rng = np.random.default_rng(12)
    box = np.array([9.0, 10.0, 14.0])
    pe = rng.random((6, 3)) * box
    pi_ = rng.random((5, 3)) * box
    qi = np.array([1.0, -1.0, 1.0, -1.0, 1.0])
    a = rng.uniform(1.2, 2.5, 6)
    p = _params(0.6, 1e-12)
    bsol = ew.electrolyte_potential(pe, a, pi_, qi, box, *p)
    Efull = ew.ewald_matrix(np.vstack([pe, pi_]), box, np.concatenate([a, np.full(5, np.inf)]), *p)
    assert np.max(np.abs(bsol - Efull[:6, 6:] @ qi)) < 1e-12
    # and the literal entries e_iI
    lit = np.array([sum(qi[I] * ew.ewald_entry_literal(pe[i], pi_[I], box, a[i], np.inf, *p)
                        for I in range(5)) for i in range(6)])
    assert np.max(np.abs(bsol - lit)) < 1e-12
    # batched frames equal single frames
    b2 = ew.electrolyte_potential(pe, a, np.stack([pi_, pi_[::-1]]), np.stack([qi, qi[::-1]]), box, *p)
    assert np.allclose(b2[0], bsol, rtol=0, atol=1e-15) and np.allclose(b2[1], bsol, rtol=0, atol=1e-13)


# --- workload generator shapes

@pytest.mark.parametrize("cfg,n", [(1, 288), (2, 4608), (3, 32768), (5, 131072)])
def test_workload_sizes(cfg, n):
    geo = wl.geometry(cfg)
    assert geo.n == n
    assert np.all(geo.pos >= -1e-12) and np.all(geo.pos < geo.box)
    # no coincident atoms: nearest in-layer distance is the bond length
    if n <= 4608:
        _, _, d = ew.real_space_pairs(geo.pos, geo.pos, geo.box, 1.5)
        assert abs(d.min() - wl.BOND) < 1e-9


# --- slab geometry: boundary correction of Eq. 39 (Sec. IV.A)

@pytest.mark.parametrize("a", [1.979, 2.93295072600296])
def test_capacitor_charge_with_slab_correction(a):
    """With the correction of Eq. 39 the field of the periodic replicas is
    removed: only the inner gap d1 carries the field, q = (dV/k_e) /
    (4 pi n d1 + 2 delta) with the same lattice term delta as in 3D
    periodicity, and at a = a^0 the continuum eps0 dV / d1 per area. The
    result does not depend on the vacuum: the same sheets in a cell twice as
    tall give the same charge. E with the correction is solved by the
    bordered system (Eq. 29), which does not need E to be definite."""
    geo = wl.geometry(1)
    b, rc, km = _params(0.3, 1e-12)
    na = int(np.sum(geo.electrode == 0))
    R = GOLD["gra_bond"]["value"]
    aij = a / math.sqrt(2.0)
    _, _, d = ew.real_space_pairs(geo.pos[:1], geo.pos[:na], geo.box, 12.0)
    delta = math.sqrt(2 / math.pi) * a - GOLD["lattice_2d_unit_bond"]["gra"] / R - np.sum(erfc(aij * d) / d)
    d1 = 40.0
    qf = (1.0 / ew.K_E) / (4 * math.pi * geo.sheet_density * d1 + 2 * delta)
    charges = []
    for lz in (geo.box[2], 2 * geo.box[2]):
        box = np.array([geo.box[0], geo.box[1], lz])
        km = ew.kmax_from_eps(b, 1e-12)
        E = ew.ewald_matrix(geo.pos, box, a, b, rc, km, slab=True)
        bvec = wl.electrode_potential(geo) / ew.K_E
        q, _ = cpm.bordered(E, bvec, 0.0)
        qa, qb = q[:na], q[na:]
        assert np.ptp(qa) / abs(qa.mean()) < 1e-9 and abs(qa.mean() + qb.mean()) < 1e-15
        assert abs(qa.mean() / qf - 1) < 1e-8
        charges.append(qa.mean())
    assert abs(charges[1] / charges[0] - 1) < 1e-8
    if a == GOLD["gra_alpha0"]["value"]:
        eps0 = 1.0 / (4 * math.pi * ew.K_E)
        assert abs(charges[0] / (eps0 / d1 / geo.sheet_density) - 1) < 1e-5


def test_slab_correction_equals_dipole_energy():
    """On neutral charge sets the correction of Eq. 39 adds (2 pi / V) M_z^2
    (M_z the dipole along z) to the energy q^T E q / 2."""
    rng = np.random.default_rng(21)
    box = np.array([8.0, 9.0, 30.0])
    pos = rng.random((9, 3)) * box
    q = rng.standard_normal(9)
    q -= q.mean()
    B = ew.slab_term(pos[:, 2][:, None], pos[:, 2][None, :], box)
    mz = float(q @ pos[:, 2])
    assert abs(0.5 * q @ B @ q - 2 * math.pi / np.prod(box) * mz * mz) <= 1e-12 * mz * mz


@pytest.mark.parametrize("qsol", [0.0, 2.0])
def test_slab_correction_positive_definite_form(qsol):
    """The charges of the literal Eq. 39 system (bordered solve) are those of
    the definite form E + (4 pi / V) z z^T with right-hand side
    chi/k_e - b_sol - (4 pi / V) M1 z, M1 = sum_I q_I z_I (the correction
    restricted to sum q = -Q_sol), also for a charged electrolyte."""
    geo = wl.geometry(1)
    b, rc, km = _params(0.3, 1e-8)
    rng = np.random.default_rng(5)
    m = 20
    ipos = np.stack([rng.random(m) * geo.box[0], rng.random(m) * geo.box[1],
                     geo.ion_zlo + rng.random(m) * (geo.ion_zhi - geo.ion_zlo)], axis=1)
    iq = np.where(np.arange(m) < m // 2, 1.0, -1.0)
    iq[0] += qsol
    chi = wl.electrode_potential(geo)
    a = wl.GAUSS_INV_WIDTH
    EL = ew.ewald_matrix(geo.pos, geo.box, a, b, rc, km, slab=True)
    bl, qs = ew.rhs(geo.pos, a, ipos, iq, chi, geo.box, b, rc, km, slab=True)
    ql, _ = cpm.bordered(EL, bl, qs)
    vol = float(np.prod(geo.box))
    z = np.mod(geo.pos[:, 2], geo.box[2])
    E0 = ew.ewald_matrix(geo.pos, geo.box, a, b, rc, km)
    b0, _ = ew.rhs(geo.pos, a, ipos, iq, chi, geo.box, b, rc, km)
    m1 = float(iq @ np.mod(ipos[:, 2], geo.box[2]))
    qs2 = cpm.solve(E0 + 4 * math.pi / vol * np.outer(z, z), b0 - 4 * math.pi / vol * m1 * z, qs)
    assert np.max(np.abs(qs2 - ql)) <= 1e-10 * np.max(np.abs(ql))


# --- factored structure factor (exp(i K.r) as a product of per-axis factors)

def test_structure_factor_matches_direct_sum():
    """The structure factor of Eq. 23 from per-axis factor tables equals the
    literal sum_j q_j exp(i K.r_j) over every k-vector of a box (positions
    also outside [0, L), several particle chunks)."""
    rng = np.random.default_rng(91)
    box = np.array([13.0, 17.5, 31.0])
    pos = rng.random((301, 3)) * box * 1.4 - 0.2 * box
    q = rng.standard_normal(301)
    n, K, _ = ew.kvectors(box, 0.3, ew.kmax_from_eps(0.3, 1e-6), half=True)
    S = ew.structure_factor(pos, q, box, n, chunk=64)
    direct = np.array([np.sum(q * np.exp(1j * (pos @ k))) for k in K])
    assert np.max(np.abs(S - direct)) <= 1e-12 * np.max(np.abs(direct))
    # and its back-projection sum_K w_K Re(exp(-i K.r) S_K) at other points
    _, _, w = ew.kvectors(box, 0.3, ew.kmax_from_eps(0.3, 1e-6), half=True)
    pts = rng.random((37, 3)) * box
    back = ew.reciprocal_potential(pts, S, n, w, box, chunk=16)
    lit = np.array([np.sum(w * (np.exp(-1j * (K @ r)) * direct).real) for r in pts])
    assert np.max(np.abs(back - lit)) <= 1e-12 * np.max(np.abs(lit))


def test_factored_potentials_and_rhs_match_direct_routines():
    """At workload 1 the factored routines (used for workload 5 checks) give the
    electrode potentials of ``potentials`` and the right-hand side of ``rhs``
    at sampled atoms to 1e-12 of their scale."""
    geo, ipos, iq, chi = wl.workload(1, frames=1)
    rng = np.random.default_rng(92)
    q = rng.standard_normal(geo.n)
    q -= q.mean()
    at = np.sort(rng.choice(geo.n, 20, replace=False))
    p = (wl.EWALD_SPLIT, wl.RCUT, ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS))
    u = ew.potentials(geo.pos, wl.GAUSS_INV_WIDTH, q, geo.box, *p, at=at)
    uf = ew.potentials_factored(geo.pos, wl.GAUSS_INV_WIDTH, q, geo.box, *p, at=at)
    assert np.max(np.abs(uf - u)) <= 1e-12 * np.max(np.abs(u))
    uall = ew.potentials(geo.pos, wl.GAUSS_INV_WIDTH, q, geo.box, *p)
    ufall = ew.potentials_factored(geo.pos, wl.GAUSS_INV_WIDTH, q, geo.box, *p)
    assert np.max(np.abs(ufall - uall)) <= 1e-12 * np.max(np.abs(uall))
    b, qs = ew.rhs(geo.pos[at], wl.GAUSS_INV_WIDTH, ipos[0], iq[0], chi[at], geo.box, *p)
    bf, qsf = ew.rhs_factored(geo.pos[at], wl.GAUSS_INV_WIDTH, ipos[0], iq[0], chi[at], geo.box, *p)
    assert np.max(np.abs(bf - b)) <= 1e-12 * np.max(np.abs(b))
    assert qsf == qs


# --- point-charge simplification with the Gaussian self-energy (Sec. III.C)

@pytest.mark.parametrize("slab", [False, True])
def test_point_charge_simplification_capacitor(slab):
    """Point charges on graphene plus the self-energy sqrt(2/pi) a^0: the lattice
    term of the capacitor, delta = sqrt(2/pi) a^0 - U^GRA / R (no screening
    sum for point charges), vanishes exactly at a^0 (Table 1: U^GRA =
    sqrt(2/pi) a^0 R / R), so each sheet carries the continuum charge:
    eps0 dV (1/d1 + 1/d2) per area under 3D periodicity, eps0 dV / d1 with
    the correction of Eq. 39."""
    geo = wl.geometry(1)
    b, rc, km = _params(0.3, 1e-12)
    a0 = GOLD["gra_alpha0"]["value"]
    R = GOLD["gra_bond"]["value"]
    assert abs(math.sqrt(2 / math.pi) * a0 - GOLD["lattice_2d_unit_bond"]["gra"] / R) < 1e-12
    E = ew.ewald_matrix_point_self(geo.pos, geo.box, a0, b, rc, km, slab=slab)
    bvec = wl.electrode_potential(geo) / ew.K_E
    q, _ = cpm.bordered(E, bvec, 0.0)
    na = int(np.sum(geo.electrode == 0))
    qa = q[:na]
    assert np.ptp(qa) / abs(qa.mean()) < 1e-9 and abs(qa.mean() + q[na:].mean()) < 1e-15
    eps0 = 1.0 / (4 * math.pi * ew.K_E)          # e / (V A)
    lz, d1, d2 = geo.box[2], 40.0, 20.0
    q_cont = eps0 * (1 / d1 if slab else (1 / d1 + 1 / d2)) / geo.sheet_density
    assert abs(qa.mean() / q_cont - 1) < 1e-9


def test_point_charge_simplification_is_unscreened_gaussian_matrix():
    """The simplified matrix equals the Gaussian matrix of Eq. 22 plus the
    screening terms sum_images erfc(a_ij d) / d that the point charges drop
    (the literal entries of both), and equals the classic point-charge matrix
    (a = inf) plus sqrt(2/pi) a_i on the diagonal."""
    rng = np.random.default_rng(23)
    box = np.array([6.0, 7.0, 8.0])
    pos = rng.random((5, 3)) * box
    a = rng.uniform(1.5, 3.0, 5)
    p = _params(0.7, 1e-13)
    Es = ew.ewald_matrix_point_self(pos, box, a, *p)
    for i in range(5):
        for j in range(5):
            lit_g = ew.ewald_entry_literal(pos[i], pos[j], box, a[i], a[j], *p, same_atom=(i == j))
            lit_p = ew.ewald_entry_literal(pos[i], pos[j], box, np.inf, np.inf, *p, same_atom=(i == j))
            aij = 1.0 / math.sqrt(1 / a[i] ** 2 + 1 / a[j] ** 2)
            screen = 0.0
            for sx in range(-3, 4):
                for sy in range(-3, 4):
                    for sz in range(-3, 4):
                        if i == j and sx == sy == sz == 0:
                            continue
                        d = np.linalg.norm(pos[i] - pos[j] + np.array([sx, sy, sz]) * box)
                        if d < p[1]:
                            screen += erfc(aij * d) / d
            self_e = math.sqrt(2 / math.pi) * a[i] if i == j else 0.0
            assert abs(Es[i, j] - (lit_p + self_e)) < 1e-12
            assert abs(Es[i, j] - (lit_g + screen)) < 1e-11
