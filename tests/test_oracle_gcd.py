"""Pins of the GCD / capacitance-matrix oracle (Supplementary Eq. S14-S24).

None of the checks re-types the oracle's formula: they compare the two-step
route against a bordered Lagrange solve and a null-space minimisation of the
energy of Eq. S14, against the closed-form parallel-plate capacitor of
Sec. III.C, against the constant-potential two-step solution (Eq. 35), and
against the identities and symmetries the capacitance matrix must obey.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import erfc

from oracle import cpm, ewald as ew, gcd
from paper_2111_06704_amd import workloads as wl
from tests.test_oracle import GOLD, _params


def _capacitor_E(a):
    geo = wl.geometry(1)
    b, rc, km = _params(0.3, 1e-12)
    return geo, ew.ewald_matrix(geo.pos, geo.box, a, b, rc, km)


def _spd(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((n, n))
    return X @ X.T + n * np.eye(n), rng


def test_gcd_matches_null_space_minimum():
    """Minimising 1/2 q^T E q - b^T q over {q : L q = Q} (Eq. S14) directly,
    with q = q_0 + N y and N a basis of the null space of L, gives the same
    charges as the two-step route, and E q - b is constant per electrode and
    equal to Delta mu_a (Eq. S15)."""
    n, m = 9, 3
    E, rng = _spd(n, 11)
    labels = np.array([0, 1, 2, 0, 1, 2, 0, 0, 2])
    b = rng.standard_normal(n)
    Q = np.array([0.7, -1.3, 0.2])
    L = np.zeros((m, n))
    for i, a in enumerate(labels):
        L[a, i] = 1.0
    q0 = np.linalg.lstsq(L, Q, rcond=None)[0]
    N = sla.null_space(L)
    y = np.linalg.solve(N.T @ E @ N, N.T @ (b - E @ q0))
    q_ref = q0 + N @ y
    grad = E @ q_ref - b
    for a in range(m):
        assert np.ptp(grad[labels == a]) < 1e-12
    q, dmu = gcd.gcd_two_step(cpm.cholesky(E), b, labels, m, Q)
    assert np.max(np.abs(q - q_ref)) < 1e-12
    assert np.max(np.abs(dmu - [grad[labels == a][0] for a in range(m)])) < 1e-12
    for a in range(m):
        assert abs(np.sum(q[labels == a]) - Q[a]) < 1e-12


def test_gcd_two_step_equals_bordered_on_capacitor():
    """Eq. S16-S20 (two-step, Cholesky) and the bordered Lagrange system
    (LU) agree for electrolyte-like right-hand sides on the graphene
    capacitor, for several frames at once."""
    geo, E = _capacitor_E(GOLD["gra_alpha0"]["value"])
    n = E.shape[0]
    rng = np.random.Generator(np.random.PCG64(5))
    b = 0.05 * rng.standard_normal((3, n)) + wl.electrode_potential(geo) / ew.K_E
    Q = rng.uniform(-2, 2, size=(3, 2))
    q, dmu = gcd.gcd_two_step(cpm.cholesky(E), b, geo.electrode, 2, Q)
    for f in range(3):
        qr, mr = gcd.gcd_bordered(E, b[f], geo.electrode, 2, Q[f])
        assert np.max(np.abs(q[f] - qr)) < 1e-11 * np.max(np.abs(qr))
        assert np.max(np.abs(dmu[f] - mr)) < 1e-11 * np.max(np.abs(mr))


def test_gcd_reproduces_constant_potential_solution():
    """Taking Q_a as the electrode totals of the constant-potential charges
    (Eq. 35, with Q_sol != 0) gives back those charges, and Delta mu is the
    same on every electrode: the neutrality multiplier of Eq. 29."""
    geo, E = _capacitor_E(1.979)
    n = E.shape[0]
    rng = np.random.Generator(np.random.PCG64(9))
    b = wl.electrode_potential(geo) / ew.K_E + 0.02 * rng.standard_normal(n)
    qsol = 0.37
    q_cp = cpm.solve(E, b, qsol)
    Q = np.array([q_cp[geo.electrode == a].sum() for a in range(2)])
    assert abs(Q.sum() + qsol) < 1e-12
    q, dmu = gcd.gcd_two_step(cpm.cholesky(E), b, geo.electrode, 2, Q)
    assert np.max(np.abs(q - q_cp)) < 1e-12 * np.max(np.abs(q_cp)) + 1e-15
    _, mu = cpm.bordered(E, b, qsol)
    # bordered: E q + mu 1 = b, i.e. Delta mu = -mu on every electrode
    assert np.max(np.abs(dmu + mu)) < 1e-10 * abs(mu)


def test_capacitance_matrix_identities():
    """C_E is symmetric positive definite, its entries sum to
    C_ele = 1^T E^-1 1 (the sum over both electrode indices covers every
    atom pair), and the two mirror-equivalent sheets have C_aa = C_bb. The
    paper's C_ab < 0 holds for finite electrodes in open space; under 3D
    periodicity the neutralising background is the third electrode and
    C_ab comes out positive here, so its sign is not pinned."""
    geo, E = _capacitor_E(GOLD["gra_alpha0"]["value"])
    fac = cpm.cholesky(E)
    C, A = gcd.capacitance_matrix(fac, geo.electrode, 2)
    assert np.max(np.abs(C - C.T)) < 1e-11 * np.max(np.abs(C))
    assert np.all(np.linalg.eigvalsh(C) > 0)
    _, _, c_ele = cpm.neutralising_vector(fac, E.shape[0])
    assert abs(C.sum() - c_ele) < 1e-10 * abs(C[0, 0])
    assert abs(C[0, 0] - C[1, 1]) < 1e-10 * C[0, 0]
    # q^{Delta mu} = A Delta u_E (the note after Eq. S24) is E^-1 Delta u
    dmu = np.array([0.3, -0.1])
    du = np.where(geo.electrode == 0, dmu[0], dmu[1])
    assert np.max(np.abs(A @ dmu - np.linalg.solve(E, du))) < 1e-11 * np.max(np.abs(A @ dmu))


@pytest.mark.parametrize("a", [1.979, 2.93295072600296])
def test_joint_capacitance_of_plate_capacitor(a):
    """With b = 0 and Q = (+Q, -Q), the sheets carry the uniform charges of
    the closed-form capacitor (Sec. III.C): per atom q = (1 V / k_e) /
    (4 pi n d1 d2 / L_z + 2 delta), the multipliers differ by exactly 1 V /
    k_e, and C(Q, -Q) = |C_E| / C_ele (Eq. S21) equals Q / (V_a - V_b)."""
    geo, E = _capacitor_E(a)
    na = int(np.sum(geo.electrode == 0))
    R = GOLD["gra_bond"]["value"]
    aij = a / math.sqrt(2.0)
    _, _, d = ew.real_space_pairs(geo.pos[:1], geo.pos[:na], geo.box, 12.0)
    delta = math.sqrt(2 / math.pi) * a - GOLD["lattice_2d_unit_bond"]["gra"] / R - np.sum(erfc(aij * d) / d)
    qf = (1.0 / ew.K_E) / (4 * math.pi * geo.sheet_density * 40.0 * 20.0 / geo.box[2] + 2 * delta)
    Qa = na * qf
    fac = cpm.cholesky(E)
    q, dmu = gcd.gcd_two_step(fac, np.zeros(E.shape[0]), geo.electrode, 2, [Qa, -Qa])
    assert np.max(np.abs(q[:na] / qf - 1)) < 1e-9 and np.max(np.abs(q[na:] / qf + 1)) < 1e-9
    assert abs((dmu[0] - dmu[1]) * ew.K_E - 1.0) < 1e-9
    C, _ = gcd.capacitance_matrix(fac, geo.electrode, 2)
    cj = gcd.joint_capacitance(C)
    qb, mb = gcd.gcd_bordered(E, np.zeros(E.shape[0]), geo.electrode, 2, [Qa, -Qa])
    assert abs(cj / (Qa / (mb[0] - mb[1])) - 1) < 1e-9
    assert abs(cj / (Qa * ew.K_E) - 1) < 1e-9
