"""Divide-and-conquer preconditioner of Sec. III.B.2 (PCG-DC, Eq. 36-37) in
plain FP64 (oracle; test infrastructure only).

Construction (Sec. III.B.2, steps 1-3): for each electrode atom tau
  1. take tau and its neighbourhood, every atom (periodic image) within r_cut
     of tau, and form the local matrix M_tau of Eq. 36 over them:
     diagonal sqrt(2/pi) a_i, off-diagonal erfc(g r)/r - erfc(g r_cut)/r for
     r < r_cut and 0 beyond, with r the distance between the two images;
  2. invert M_tau; the column of M_tau^-1 that belongs to tau is written into
     column tau of P (entries of two images of one atom add up), every other
     entry of the column is zero;
  3. repeat for every atom.
Optionally the zeros of P are replaced by p_gap (Eq. 37), the mean of the
removed entries of E^-1: p_gap = (1^T E^-1 1 - sum_ij P_ij) / n_zero.

PCG-Normal and PCG-Full (Sec. III.B.2) sparsify E^-1 itself by the
real-space distance of the two charges: p_ij = (E^-1)_ij when the pair is
closer than a cutoff, 0 otherwise (Full: the cutoff of the neighbour list;
Normal: a shorter preset r_cut).

Not in the paper: a coarse-space (two-level) correction of any of these P,
in the balancing Neumann-Neumann form (Mandel, Commun. Numer. Methods Eng.
9, 233 (1993)): with Z the indicator columns of patches of atoms, E_c =
Z^T E Z, Q = Z E_c^-1 Z^T and P_D = I - E Q, the preconditioner is
P_D^T P P_D + Q. Patches: z-slabs (sorted z, a new slab where two
consecutive values differ by more than 1 A) split into nx x ny in-plane
bins, nx = max(1, floor(L_x / edge + 1/2)). Its pins are closed forms
(exact on the coarse space, E^-1 from an exact P or from one patch per atom).

Readings (the paper is silent or ambiguous):
  * the neighbourhood includes atoms at exactly r_cut (Fig. 2: N_cut = 21 for
    a chain of spacing 1.5 A at r_cut = 15 A counts the atoms at 15 A); their
    Eq. 36 coupling to tau is zero;
  * P filled column by column is not symmetric; CG uses (P + P^T) / 2;
  * PCG-Normal / Full: the distance of a pair is that of the nearest images
    (E^-1 has one entry per pair), pairs strictly closer than the cutoff are
    kept, the diagonal always.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree
from scipy.special import erfc


def neighbourhood(pos, box, rcut):
    """For every atom: (indices, image positions) of all atoms, periodic
    images included, with distance <= rcut (the atom itself at n = 0
    excluded), ordered by index and then by image."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    nr = [int(math.ceil(rcut / box[d])) + 1 for d in range(3)]
    shifts = np.array([[a, b, c] for a in range(-nr[0], nr[0] + 1)
                       for b in range(-nr[1], nr[1] + 1)
                       for c in range(-nr[2], nr[2] + 1)], dtype=np.float64) * box
    imgs = (pos[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    idx = np.tile(np.arange(len(pos)), len(shifts))
    tree = cKDTree(imgs)
    out = []
    for i in range(len(pos)):
        js = np.array(sorted(tree.query_ball_point(pos[i], rcut * (1 + 1e-12))), dtype=np.int64)
        d = np.linalg.norm(imgs[js] - pos[i], axis=1)
        js = js[(d > 1e-9) & (d <= rcut)]
        order = np.lexsort((js, idx[js]))          # by atom index, then image
        js = js[order]
        out.append((idx[js], imgs[js]))
    return out


def local_matrix(X, a, g, rcut):
    """Eq. 36 over the points X (first row tau), inverse widths a."""
    X = np.asarray(X, dtype=np.float64)
    d = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=2)
    M = np.zeros_like(d)
    off = (d > 0) & (d < rcut)
    M[off] = (erfc(g * d[off]) - erfc(g * rcut)) / d[off]
    M[np.diag_indices(len(X))] = math.sqrt(2.0 / math.pi) * np.asarray(a, dtype=np.float64)
    return M


def dc_columns(n, nbhd, local):
    """P filled column by column (step 2): nbhd[tau] = (indices, positions),
    local(tau, indices, positions) -> M_tau with tau first."""
    P = np.zeros((n, n))
    for tau in range(n):
        jj, pp = nbhd[tau]
        M = local(tau, jj, pp)
        e = np.zeros(len(M))
        e[0] = 1.0
        col = np.linalg.solve(M, e)               # column of M_tau^-1 belonging to tau
        P[tau, tau] += col[0]
        np.add.at(P[:, tau], jj, col[1:])
    return P


def dc_preconditioner(pos, box, a, g, rcut, symmetric=True):
    """P of PCG-DC for atoms pos (inverse widths a), screening g, cutoff rcut."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    nbhd = neighbourhood(pos, box, rcut)

    def local(tau, jj, pp):
        X = np.vstack([pos[tau][None, :], pp])
        return local_matrix(X, np.concatenate([[a[tau]], a[jj]]), g, rcut)

    P = dc_columns(n, nbhd, local)
    return 0.5 * (P + P.T) if symmetric else P


def min_image_distances(pos, box):
    """Distance of every pair of atoms to the nearest periodic image (n x n)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.round(d / box)
    return np.linalg.norm(d, axis=2)


def sparse_inverse(Einv, pos, box, rcut):
    """PCG-Normal / PCG-Full P: the entries of E^-1 of the pairs closer than
    rcut (nearest images) and the diagonal; zero elsewhere."""
    keep = min_image_distances(pos, box) < rcut
    np.fill_diagonal(keep, True)
    return np.where(keep, Einv, 0.0)


def p_gap(P, sum_einv):
    """Eq. 37: mean of the entries of E^-1 removed by the sparsification;
    sum_einv = 1^T E^-1 1."""
    n_zero = int(np.count_nonzero(P == 0.0))
    return (sum_einv - float(P.sum())) / n_zero if n_zero else 0.0


def with_gap(P, gap):
    """P with its zeros replaced by gap (Eq. 37)."""
    Q = P.copy()
    Q[P == 0.0] = gap
    return Q


def pcg(E, b, P, tol, max_iter=10000):
    """Textbook preconditioned CG on E x = b with preconditioner P (dense),
    stopped on the true residual |b - E x| <= tol |b|. Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = P @ r
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for k in range(1, max_iter + 1):
        v = E @ p
        alpha = rz / (p @ v)
        x += alpha * p
        r -= alpha * v
        if np.linalg.norm(b - E @ x) <= tol * bn:
            return x, k
        z = P @ r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter


def coarse_patches(pos, box, edge, slab_gap=1.0):
    """Patch index of every atom (numbered by slab, x bin, y bin; empty bins
    dropped): z-slabs from the sorted z (a new slab where two consecutive
    values differ by more than slab_gap), each split into nx x ny bins of
    the box, nx = max(1, floor(L_x / edge + 1/2)). Positions are wrapped
    into the box first (fmod, then one shift)."""
    box = np.asarray(box, dtype=np.float64)
    w = np.fmod(np.asarray(pos, dtype=np.float64), box)
    w = np.where(w < 0, w + box, w)
    w = np.where(w >= box, w - box, w)
    n = len(w)
    order = np.argsort(w[:, 2], kind="stable")
    slab = np.zeros(n, dtype=np.int64)
    slab[order] = np.concatenate([[0], np.cumsum(np.diff(w[order, 2]) > slab_gap)])
    nx = max(1, int(math.floor(box[0] / edge + 0.5)))
    ny = max(1, int(math.floor(box[1] / edge + 0.5)))
    bx = np.minimum(nx - 1, np.floor(w[:, 0] / box[0] * nx).astype(np.int64))
    by = np.minimum(ny - 1, np.floor(w[:, 1] / box[1] * ny).astype(np.int64))
    key = (slab * nx + bx) * ny + by
    _, pid = np.unique(key, return_inverse=True)
    return pid.astype(np.int64)


def two_level(P, E, pid):
    """Balancing Neumann-Neumann two-level preconditioner on top of P:
    Z = indicator columns of the patches pid, E_c = Z^T E Z,
    Q = Z E_c^-1 Z^T, P_D = I - E Q; returns P_D^T P P_D + Q (dense)."""
    n = E.shape[0]
    m = int(pid.max()) + 1
    Z = np.zeros((n, m))
    Z[np.arange(n), pid] = 1.0
    Ec = Z.T @ E @ Z
    Q = Z @ np.linalg.solve(Ec, Z.T)
    PD = np.eye(n) - E @ Q
    return PD.T @ P @ PD + Q
