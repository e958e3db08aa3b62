"""Constrained electrode-charge solve in plain FP64 (oracle; test infrastructure only).

Sec. III.A of the paper: minimising the energy functional (Eq. 28) under
sum(q) + Q_sol = 0 gives E q = b - mu_c 1 (Eq. 29-30). The solution is
computed three ways:
  * two-step (Eq. 35): q_b = E^-1 b, d' = E^-1 1 (S9), d = d' / 1^T d' (S8),
    q = q_b - (1^T q_b + Q_sol) d;
  * the bordered Lagrange system [[E, 1], [1^T, 0]] [q; mu] = [b; -Q_sol]
    (Eq. 29 with the constraint of Eq. 28);
  * the S matrix of Eq. 33, S = E^-1 (I - 1 d^T), q = S b - Q_sol d (Eq. 34).
E^-1 is applied through a Cholesky factorisation (LAPACK dpotrf / dpotrs),
which also certifies that E is symmetric positive definite.

The matrix-inversion construction of E (Sec. III.B.1, S10-S13) is provided
as ``matrix_from_potentials``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotSPD(RuntimeError):
    pass


def cholesky(E):
    """Lower Cholesky factor of E; raises NotSPD if E is not positive definite."""
    try:
        return sla.cho_factor(E, lower=True, check_finite=True)
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc


def neutralising_vector(factor, n):
    """d' = E^-1 1 (S9), C_ele = 1^T d' and d = d' / C_ele (S8, Eq. 32)."""
    dp = sla.cho_solve(factor, np.ones(n))
    c_ele = float(np.sum(dp))
    return dp, dp / c_ele, c_ele


def two_step(factor, b, qsol, d):
    """q = q_b - (1^T q_b + Q_sol) d with q_b = E^-1 b (Eq. 35).

    b may be (N,) or (F, N) with qsol scalar or (F,)."""
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        qb = sla.cho_solve(factor, b)
        return qb - (np.sum(qb) + float(qsol)) * d
    qb = sla.cho_solve(factor, b.T).T
    qsol = np.broadcast_to(np.asarray(qsol, dtype=np.float64), (b.shape[0],))
    return qb - (np.sum(qb, axis=1) + qsol)[:, None] * d[None, :]


def solve(E, b, qsol):
    """Electrode charges for b (N,) or (F, N) by the two-step method."""
    f = cholesky(E)
    _, d, _ = neutralising_vector(f, E.shape[0])
    return two_step(f, b, qsol, d)


def bordered(E, b, qsol):
    """Solve [[E, 1], [1^T, 0]] [q; mu] = [b; -Q_sol] by LU (Eq. 29)."""
    n = E.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = E
    A[:n, n] = 1.0
    A[n, :n] = 1.0
    rhs = np.concatenate([np.asarray(b, dtype=np.float64), [-float(qsol)]])
    x = sla.solve(A, rhs)
    return x[:n], x[n]


def s_matrix(E):
    """S = E^-1 (I - 1 d^T) (Eq. 33) and d, through the explicit inverse."""
    n = E.shape[0]
    Einv = np.linalg.inv(E)
    d = Einv @ np.ones(n)
    d /= np.sum(d)
    S = Einv @ (np.eye(n) - np.outer(np.ones(n), d))
    return S, d


def charge_matrix(n):
    """Q~ = (N+1) I - 1 1^T and its inverse (I + 1 1^T) / (N+1) (S10-S12)."""
    Q = (n + 1.0) * np.eye(n) - np.ones((n, n))
    Qinv = (np.eye(n) + np.ones((n, n))) / (n + 1.0)
    return Q, Qinv


def matrix_from_potentials(potential_fn, n):
    """E = U~ Q~^-1 where column j of U~ is the potential produced by charge
    configuration column j of Q~ (Sec. III.B.1, steps 1-4)."""
    Q, Qinv = charge_matrix(n)
    U = np.column_stack([potential_fn(Q[:, j]) for j in range(n)])
    return U @ Qinv


def rel_errors(q, q_ref):
    """Per-frame rel_2 = |q - q_ref|_2 / |q_ref|_2 and
    rel_max = max|q - q_ref| / max|q_ref|."""
    q = np.atleast_2d(q)
    q_ref = np.atleast_2d(q_ref)
    r2 = np.linalg.norm(q - q_ref, axis=1) / np.linalg.norm(q_ref, axis=1)
    rm = np.max(np.abs(q - q_ref), axis=1) / np.max(np.abs(q_ref), axis=1)
    return r2, rm
