"""Per-atom inputs of the warm-start network (oracle; test infrastructure only).

Definition (the library follows the same one; it is not from the paper, which
warm-starts from the previous MD step instead, Sec. III.A Eq. 26):
  * neighbours: the 12 nearest other electrode atoms under the minimum
    image, ordered by distance, then by azimuth about +z measured from +x
    in [0, 2 pi), then by index; distance and azimuth are compared after
    rounding to 1e-6 (A, rad);
  * inputs of atom i in a frame with right-hand side b:
      [ (b_i - mean b) / b_scale, layer_i / (n_layers - 1),
        (b_j - mean b) / b_scale for the 12 neighbours j,
        r_ij / r_scale for the same neighbours ].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

NNB = 12


def _keys(dv):
    d = np.sqrt(np.sum(dv * dv, axis=-1))
    az = np.arctan2(dv[..., 1], dv[..., 0])
    az = np.where(az < 0, az + 2 * math.pi, az)
    return d, np.round(d * 1e6).astype(np.int64), np.round(az * 1e6).astype(np.int64)


def min_image(dv, box):
    box = np.asarray(box, dtype=np.float64)
    return dv - box * np.round(dv / box)


def neighbours(pos, box, k=NNB, candidates=40):
    """(N, k) neighbour indices and (N, k) distances."""
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    n = len(pos)
    tree = cKDTree(pos, boxsize=np.asarray(box, dtype=np.float64))
    kk = min(candidates, n)
    _, idx = tree.query(pos, k=kk)
    nbr = np.empty((n, k), dtype=np.int64)
    dist = np.empty((n, k))
    for i in range(n):
        cand = idx[i][idx[i] != i]
        dv = min_image(pos[cand] - pos[i], box)
        d, kd, ka = _keys(dv)
        order = np.lexsort((cand, ka, kd))
        # every candidate tied with the k-th must be present for the order to be exact
        assert kk == n or kd[order[k - 1]] < kd[order[-1]], "too few neighbour candidates"
        nbr[i] = cand[order[:k]]
        dist[i] = d[order[:k]]
    return nbr, dist


def neighbours_brute(pos, box, k=NNB):
    """Same list by comparing every pair (small N only)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    nbr = np.empty((n, k), dtype=np.int64)
    for i in range(n):
        dv = min_image(pos - pos[i], box)
        d, kd, ka = _keys(dv)
        j = np.arange(n)
        keep = j != i
        order = np.lexsort((j[keep], ka[keep], kd[keep]))
        nbr[i] = j[keep][order[:k]]
    return nbr


def features(b, nbr, dist, layer, n_layers, b_scale, r_scale):
    """(F*N, 26) float64 inputs for frames b (F, N); row = frame * N + atom."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    f, n = b.shape
    bc = (b - b.mean(axis=1, keepdims=True)) / b_scale
    lay = np.asarray(layer, dtype=np.float64) / (n_layers - 1) if n_layers > 1 else np.zeros(n)
    out = np.empty((f, n, 2 + 2 * NNB))
    out[:, :, 0] = bc
    out[:, :, 1] = lay[None, :]
    out[:, :, 2:2 + NNB] = bc[:, nbr]
    out[:, :, 2 + NNB:] = (np.asarray(dist) / r_scale)[None, :, :]
    return out.reshape(f * n, 2 + 2 * NNB)
