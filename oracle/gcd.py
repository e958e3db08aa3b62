"""Galvanostatic charge-discharge constraint and the capacitance coefficient
matrix (Supplementary Note, Eq. S14-S24), in plain FP64 (oracle; test
infrastructure only).

With M electrodes and a prescribed total charge Q_a on each electrode a,
minimising the energy of Eq. S14 gives E q = b + Delta u (Eq. S15), where
Delta u_i = Delta mu_a for every atom i of electrode a. Two independent
computations of the same charges:
  * the bordered Lagrange system [[E, -L^T], [L, 0]] [q; Delta mu] = [b; Q]
    with L the M x N electrode indicator (the constraints of Eq. S14);
  * the two-step route of Eq. S16-S20: q_b = E^-1 b, A = E^-1 [b^1 .. b^M]
    with b^h the indicator of electrode h (Eq. S22-S23), C_ab = sum over the
    atoms of a of A[:, b] (Eq. S24), Delta mu = C^-1 (Q - L q_b) (Eq. S20),
    q = q_b + A Delta mu (Eq. S17).
The joint capacitance of two electrodes carrying +Q and -Q is
C(Q, -Q) = det C_E / C_ele with C_ele = 1^T E^-1 1 (Eq. S21).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def indicator(labels, m):
    """M x N matrix L with L[a, i] = 1 if atom i belongs to electrode a."""
    labels = np.asarray(labels)
    L = np.zeros((m, len(labels)))
    L[labels, np.arange(len(labels))] = 1.0
    return L


def coefficient_solutions(factor, labels, m):
    """A = E^-1 [b^1 .. b^M] (Eq. S22-S23); factor is a Cholesky factor of E."""
    return sla.cho_solve(factor, indicator(labels, m).T)


def capacitance_matrix(factor, labels, m):
    """C_E[a, b] = sum over the atoms of a of A[:, b] (Eq. S24) and A."""
    A = coefficient_solutions(factor, labels, m)
    return indicator(labels, m) @ A, A


def gcd_two_step(factor, b, labels, m, Q):
    """Charges under the total-charge constraints by Eq. S16-S20; b (N,) or
    (F, N), Q (M,) or (F, M). Returns (q, Delta mu)."""
    C, A = capacitance_matrix(factor, labels, m)
    L = indicator(labels, m)
    b2 = np.atleast_2d(b)
    Q2 = np.atleast_2d(Q)
    qb = sla.cho_solve(factor, b2.T).T
    dmu = np.linalg.solve(C, (Q2 - qb @ L.T).T).T
    q = qb + dmu @ A.T
    return (q[0], dmu[0]) if np.ndim(b) == 1 else (q, dmu)


def gcd_bordered(E, b, labels, m, Q):
    """The same charges from the bordered Lagrange system of Eq. S14-S15."""
    n = E.shape[0]
    L = indicator(labels, m)
    K = np.zeros((n + m, n + m))
    K[:n, :n] = E
    K[:n, n:] = -L.T
    K[n:, :n] = L
    rhs = np.concatenate([np.asarray(b, dtype=np.float64), np.asarray(Q, dtype=np.float64)])
    sol = np.linalg.solve(K, rhs)
    return sol[:n], sol[n:]


def joint_capacitance(C):
    """C(Q, -Q) of two electrodes (Eq. S21): det C_E / (sum of all C_ab)."""
    return float(np.linalg.det(C) / np.sum(C))
