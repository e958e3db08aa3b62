"""Gaussian-charge Ewald sums in plain FP64 (oracle; test infrastructure only).

Follows Sec. II of the paper:
  * Gaussian pair potential erf(a_ij r)/r with a_ij^-2 = a_i^-2 + a_j^-2
    (Sec. II.A, Eq. 5) and self-energy 2 a_ii / sqrt(pi) (Eq. 6);
  * the Gaussian Ewald potential (Sec. II.C, Eq. 20) and the matrix entries
    e_ij (Eq. 22-23): real-space sum over images of
    [erfc(beta d) - erfc(a_ij d)] / d, reciprocal sum
    (4 pi / V) sum_{K != 0} exp(-K^2 / 4 beta^2) / K^2 cos(K . r_ij), the
    background constant -pi / (V beta^2) and, on the diagonal,
    -2 beta / sqrt(pi) + 2 a_ii / sqrt(pi);
  * the point-charge limit a -> inf (end of Sec. II.C): the erfc(a d) terms
    vanish and the Gaussian self-energy is dropped, which is the classic
    Ewald matrix of Eq. 15;
  * the electrolyte potential b_sol,i = sum_I q_I e_iI(a_i) (Sec. III.A,
    Eq. 25), point-Gaussian mixing a_iI = a_i (Sec. II.A).

Reading of Eq. 23: the reciprocal prefactor is (4 pi / V) times
exp(-K^2/4 beta^2)/K^2, i.e. (1/V) phi_hat(K; beta), as in Eq. 13, 16 and
20; the extra 4 pi printed in Eq. 23 is taken as a typo.

A point charge is given an inverse width of ``numpy.inf``.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.spatial import cKDTree
from scipy.special import erfc, erfcinv

K_E = 14.3996454784      # e^2 / (4 pi eps0) in V * A / e


def mix_width(ai, aj):
    """a_ij = (a_i^-2 + a_j^-2)^(-1/2) (Sec. II.A, after Eq. 5); inf = point."""
    ai = np.asarray(ai, dtype=np.float64)
    aj = np.asarray(aj, dtype=np.float64)
    with np.errstate(divide="ignore"):
        s = 1.0 / ai ** 2 + 1.0 / aj ** 2
        return np.where(s > 0, 1.0 / np.sqrt(np.where(s > 0, s, 1.0)), np.inf)


def kmax_from_eps(beta: float, eps: float) -> float:
    """Spherical reciprocal cutoff with exp(-K_max^2 / 4 beta^2) = eps.

    The paper leaves the k-space truncation to standard error estimators
    (end of Sec. II.C); this is the reading used throughout."""
    return 2.0 * beta * math.sqrt(math.log(1.0 / eps))


def rcut_from_eps(beta: float, eps: float) -> float:
    """Real-space cutoff with erfc(beta r_cut) = eps."""
    return float(erfcinv(eps)) / beta


def kvectors(box, beta: float, kmax: float, half: bool = True):
    """Reciprocal lattice vectors K = 2 pi (n_x/L_x, n_y/L_y, n_z/L_z), K != 0,
    |K| <= kmax (Sec. II.B, after Eq. 11), and their weights.

    half=True keeps one of each +-K pair (n_x > 0, or n_x = 0 and n_y > 0, or
    n_x = n_y = 0 and n_z > 0) and doubles the weight, using
    cos(K.r) = cos(-K.r). Weight w_K = m (4 pi / V) exp(-K^2 / 4 beta^2) / K^2
    with m = 2 for the half set and 1 for the full set (Eq. 13 / 20).
    Returns (n (M,3) int, K (M,3) float, w (M,) float)."""
    box = np.asarray(box, dtype=np.float64)
    vol = float(np.prod(box))
    nmax = [int(math.floor(kmax * box[d] / (2.0 * math.pi))) for d in range(3)]
    ax = [np.arange(-nmax[d], nmax[d] + 1) for d in range(3)]
    nx, ny, nz = np.meshgrid(*ax, indexing="ij")
    n = np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1)
    K = 2.0 * math.pi * n / box
    k2 = np.sum(K * K, axis=1)
    keep = (k2 > 0) & (k2 <= kmax * kmax)
    if half:
        pos_half = (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | \
                   ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))
        keep &= pos_half
    n, K, k2 = n[keep], K[keep], k2[keep]
    mult = 2.0 if half else 1.0
    w = mult * (4.0 * math.pi / vol) * np.exp(-k2 / (4.0 * beta * beta)) / k2
    return n, K, w


class _Phases:
    """cos and sin of the phases K.r of a set of points for chunks of K, in
    float64 on PyTorch's multi-threaded CPU kernels, with the work arrays
    allocated once (large structure-factor sums)."""

    def __init__(self, rows, chunk):
        self.ph = np.empty((rows, chunk))
        self.c = np.empty((rows, chunk))
        self.s = np.empty((rows, chunk))

    def __call__(self, r, Kc):
        m = Kc.shape[0]
        ph, c, s = self.ph[:, :m], self.c[:, :m], self.s[:, :m]
        np.matmul(r, Kc.T, out=ph)
        t = torch.from_numpy(ph)
        torch.cos(t, out=torch.from_numpy(c))
        torch.sin(t, out=torch.from_numpy(s))
        return c, s


def _image_range(box, rcut):
    return [int(math.ceil(rcut / box[d])) + 1 for d in range(3)]


def _pair_potential_real(d, beta, aij):
    """[erfc(beta d) - erfc(a_ij d)] / d, the real-space summand of Eq. 20."""
    gauss = np.where(np.isinf(aij), 0.0, erfc(np.where(np.isinf(aij), 0.0, aij) * d))
    return (erfc(beta * d) - gauss) / d


def ewald_entry_literal(ri, rj, box, ai, aj, beta, rcut, kmax, same_atom=False):
    """One entry e_ij of Eq. 22 written out term by term (small cases only).

    Real space: every image n (n = 0 excluded for the self entry) with
    |r_ij + n L| < rcut. Reciprocal: the full set of K != 0 with |K| <= kmax
    and cos(K . r_ij)."""
    box = np.asarray(box, dtype=np.float64)
    vol = float(np.prod(box))
    rij = np.asarray(ri, dtype=np.float64) - np.asarray(rj, dtype=np.float64)
    aij = float(mix_width(ai, aj))
    e = 0.0
    nr = _image_range(box, rcut + float(np.max(np.abs(rij))))
    for a in range(-nr[0], nr[0] + 1):
        for b in range(-nr[1], nr[1] + 1):
            for c in range(-nr[2], nr[2] + 1):
                if same_atom and a == 0 and b == 0 and c == 0:
                    continue
                v = rij + np.array([a, b, c]) * box
                d = math.sqrt(float(v @ v))
                if d < rcut:
                    e += float(_pair_potential_real(d, beta, aij))
    _, K, w = kvectors(box, beta, kmax, half=False)
    e += float(np.sum(w * np.cos(K @ rij)))
    e -= math.pi / (vol * beta * beta)
    if same_atom:
        e -= 2.0 * beta / math.sqrt(math.pi)
        if not math.isinf(aij):
            e += 2.0 * aij / math.sqrt(math.pi)
    return e


def ewald_matrix_literal(pos, box, a, beta, rcut, kmax):
    """E built entry by entry with ``ewald_entry_literal`` (N <= ~20)."""
    pos = np.asarray(pos, dtype=np.float64)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (len(pos),))
    n = len(pos)
    E = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            E[i, j] = ewald_entry_literal(pos[i], pos[j], box, a[i], a[j], beta, rcut, kmax,
                                          same_atom=(i == j))
    return E


def slab_term(za, zb, box):
    """Boundary correction of Eq. 39 between charges at heights za and zb
    (cell coordinates in [0, L_z)): -(2 pi / V) [(z_a - z_b)^2 + L_z^2 / 6].
    The first part cancels the net dipole of the periodic slab (Yeh and
    Berkowitz), the second the non-neutral slab (Ballenegger); z is the
    non-periodic direction (Sec. IV.A)."""
    box = np.asarray(box, dtype=np.float64)
    vol = float(np.prod(box))
    za = np.mod(np.asarray(za, dtype=np.float64), box[2])
    zb = np.mod(np.asarray(zb, dtype=np.float64), box[2])
    return -(2.0 * math.pi / vol) * ((za - zb) ** 2 + box[2] ** 2 / 6.0)


def real_space_pairs(pos_a, pos_b, box, rcut):
    """All (i, j, d) with d = |r_a,i - r_b,j + n L| < rcut over every image n.

    Pairs at exactly d = 0 (an atom with itself, n = 0) are removed."""
    box = np.asarray(box, dtype=np.float64)
    nr = _image_range(box, rcut)
    shifts = np.array([[a, b, c] for a in range(-nr[0], nr[0] + 1)
                       for b in range(-nr[1], nr[1] + 1)
                       for c in range(-nr[2], nr[2] + 1)], dtype=np.float64) * box
    pb = np.mod(np.asarray(pos_b, dtype=np.float64), box)
    pa = np.mod(np.asarray(pos_a, dtype=np.float64), box)
    # keep only image copies that can be within rcut of the box
    imgs = (pb[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    idx = np.tile(np.arange(len(pb)), len(shifts))
    lo, hi = -rcut, box + rcut
    inside = np.all((imgs > lo) & (imgs < hi), axis=1)
    imgs, idx = imgs[inside], idx[inside]
    ta, tb = cKDTree(pa), cKDTree(imgs)
    sdm = ta.sparse_distance_matrix(tb, rcut, output_type="ndarray")
    i = sdm["i"].astype(np.int64)
    j = idx[sdm["j"]]
    d = sdm["v"]
    keep = (d > 0.0) & (d < rcut)
    return i[keep], j[keep], d[keep]


def reciprocal_gram(pos_a, pos_b, K, w, chunk=2048):
    """sum_K w_K [cos(K.r_a) cos(K.r_b) + sin(K.r_a) sin(K.r_b)]
    = sum_K w_K cos(K.(r_a - r_b)), accumulated over chunks of K."""
    pos_a = np.asarray(pos_a, dtype=np.float64)
    pos_b = np.asarray(pos_b, dtype=np.float64)
    out = np.zeros((len(pos_a), len(pos_b)))
    for k0 in range(0, len(K), chunk):
        Kc, wc = K[k0:k0 + chunk], w[k0:k0 + chunk]
        pa = pos_a @ Kc.T
        pb = pos_b @ Kc.T
        out += (np.cos(pa) * wc) @ np.cos(pb).T
        out += (np.sin(pa) * wc) @ np.sin(pb).T
    return out


def ewald_matrix(pos, box, a, beta, rcut, kmax, slab=False):
    """The Gaussian Ewald matrix E of Eq. 22 for electrode atoms ``pos``
    (slab: plus the boundary correction of Eq. 39 on every entry).

    Same sum as ``ewald_matrix_literal``; the reciprocal part uses the half
    K set and the identity cos(K.(ri - rj)) = cos cos + sin sin."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    vol = float(np.prod(box))
    _, K, w = kvectors(box, beta, kmax, half=True)
    E = reciprocal_gram(pos, pos, K, w)
    i, j, d = real_space_pairs(pos, pos, box, rcut)
    aij = mix_width(a[i], a[j])
    np.add.at(E, (i, j), _pair_potential_real(d, beta, aij))
    E -= math.pi / (vol * beta * beta)
    aii = mix_width(a, a)
    diag = -2.0 * beta / math.sqrt(math.pi) + np.where(np.isinf(aii), 0.0,
                                                        2.0 * np.where(np.isinf(aii), 0.0, aii)
                                                        / math.sqrt(math.pi))
    E[np.arange(n), np.arange(n)] += diag
    if slab:
        E += slab_term(pos[:, 2][:, None], pos[:, 2][None, :], box)
    return E


def ewald_matrix_point_self(pos, box, a, beta, rcut, kmax, slab=False):
    """The point-charge simplification of Sec. III.C: the electrode charges
    interact as classic point charges (the matrix of Eq. 15, i.e. Eq. 22
    without its erfc(a_ij d) screening terms, which for graphene at a^0 are
    below 3.2e-5 of the pair term, last column of Table 1), and each keeps
    the non-singular self-energy sqrt(2/pi) a_i of a Gaussian charge on the
    diagonal (U^GRA = sqrt(2/pi) a^0). The electrolyte acts on them as
    point charges too: ``electrolyte_potential`` / ``rhs`` with a = inf."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    E = ewald_matrix(pos, box, np.inf, beta, rcut, kmax, slab)
    E[np.arange(n), np.arange(n)] += math.sqrt(2.0 / math.pi) * a
    return E


def electrolyte_potential(pos, a, ion_pos, ion_q, box, beta, rcut, kmax, slab=False):
    """b_sol,i = sum_I q_I e_iI(a_i) (Eq. 25).

    e_iI is Eq. 22 for a Gaussian electrode charge and a point ion: mixing
    width a_i, real-space [erfc(beta d) - erfc(a_i d)]/d over images with
    d < rcut, the reciprocal sum and the background -pi/(V beta^2).
    ion_pos (M, 3) and ion_q (M,) for one frame, or (F, M, 3) and (F, M) for
    F frames (then the result is (F, N))."""
    pos = np.asarray(pos, dtype=np.float64)
    ion_pos = np.asarray(ion_pos, dtype=np.float64)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    single = ion_pos.ndim == 2
    if single:
        ion_pos, ion_q = ion_pos[None], ion_q[None]
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    nf = ion_pos.shape[0]
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    vol = float(np.prod(box))
    _, K, w = kvectors(box, beta, kmax, half=True)
    out = np.zeros((nf, n))
    chunk = 2048
    pe, pi = _Phases(n, chunk), _Phases(ion_pos.shape[1], chunk)
    for k0 in range(0, len(K), chunk):
        Kc, wc = K[k0:k0 + chunk], w[k0:k0 + chunk]
        ce, se = pe(pos, Kc)
        for f in range(nf):
            ci, si = pi(ion_pos[f], Kc)
            sc = ion_q[f] @ ci                    # Re S(K) = sum_I q_I cos(K.r_I)
            ss = ion_q[f] @ si                    # Im S(K)
            out[f] += ce @ (wc * sc) + se @ (wc * ss)
    for f in range(nf):
        i, I, d = real_space_pairs(pos, ion_pos[f], box, rcut)
        np.add.at(out[f], i, ion_q[f][I] * _pair_potential_real(d, beta, a[i]))
        out[f] -= math.pi / (vol * beta * beta) * float(np.sum(ion_q[f]))
        if slab:
            out[f] += slab_term(pos[:, 2][:, None], ion_pos[f][:, 2][None, :], box) @ ion_q[f]
    return out[0] if single else out


def rhs(pos, a, ion_pos, ion_q, chi_volts, box, beta, rcut, kmax, slab=False):
    """b = chi - b_sol (Eq. 25) with chi converted from volts to e/A, and
    Q_sol = sum_I q_I, for one frame ((N,), float) or F frames ((F, N), (F,))."""
    bsol = electrolyte_potential(pos, a, ion_pos, ion_q, box, beta, rcut, kmax, slab)
    chi = np.asarray(chi_volts, dtype=np.float64) / K_E
    return chi - bsol, np.sum(np.asarray(ion_q, dtype=np.float64), axis=-1)


def potentials(pos, a, q, box, beta, rcut, kmax, at=None):
    """Matrix-free potentials u_i = sum_j e_ij q_j of a charge configuration q
    on the electrode atoms (the per-atom derivative of Eq. 21), at the atoms
    ``at`` (default: all).

    Reciprocal part through the structure factor S(K) = sum_j q_j exp(iK.r_j)
    (accumulated over chunks of K), real part through the pair list, then
    background and self terms."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    idx = np.arange(n) if at is None else np.asarray(at, dtype=np.int64)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    vol = float(np.prod(box))
    _, K, w = kvectors(box, beta, kmax, half=True)
    u = np.zeros(len(idx))
    chunk = 2048
    phases = _Phases(n, chunk)
    for k0 in range(0, len(K), chunk):
        Kc, wc = K[k0:k0 + chunk], w[k0:k0 + chunk]
        c, s = phases(pos, Kc)
        sr, si = q @ c, q @ s                     # S(K)
        u += c[idx] @ (wc * sr) + s[idx] @ (wc * si)   # sum_K w Re(exp(-iK.r_i) S(K))
    i, j, d = real_space_pairs(pos[idx], pos, box, rcut)
    u += np.bincount(i, weights=q[j] * _pair_potential_real(d, beta, mix_width(a[idx][i], a[j])),
                     minlength=len(idx))
    u -= math.pi / (vol * beta * beta) * float(np.sum(q))
    aii = mix_width(a[idx], a[idx])
    selfc = -2.0 * beta / math.sqrt(math.pi) + np.where(np.isinf(aii), 0.0,
                                                         2.0 * np.where(np.isinf(aii), 0.0, aii)
                                                         / math.sqrt(math.pi))
    u += selfc * q[idx]
    return u


def structure_factor(pos, q, box, n, chunk=16384):
    """S(K) = sum_j q_j exp(i K.r_j) for the k-vectors K = 2 pi n / L of the
    integer triplets n (M, 3) (Eq. 23's structure factor, the sum whose real
    and imaginary parts the reciprocal terms of Eq. 21-22 and 25 contract).

    Uses the exact identity exp(i K.r) = exp(2 pi i n_x x / L_x)
    exp(2 pi i n_y y / L_y) exp(2 pi i n_z z / L_z): per-axis factor tables of
    every particle, and for each chunk of particles one complex matrix
    product over them,
        T[n_y, (n_x, n_z)] = sum_j Y_j(n_y) [q_j X_j(n_x) Z_j(n_z)],
    from which the entries of the requested triplets are read. Same sum as
    the direct cos / sin evaluation of ``potentials``, in another order; it
    costs particles x (distinct n_x) x (distinct n_z) products instead of
    particles x k-vectors phases."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = np.asarray(n, dtype=np.int64)
    vals = [np.unique(n[:, d]) for d in range(3)]
    ix = [np.searchsorted(vals[d], n[:, d]) for d in range(3)]
    nxv, nyv, nzv = (len(v) for v in vals)
    T = np.zeros((nyv, nxv * nzv), dtype=np.complex128)
    for j0 in range(0, len(pos), chunk):
        u = pos[j0:j0 + chunk] / box
        X, Y, Z = (np.exp(2j * math.pi * np.outer(u[:, d], vals[d])) for d in range(3))
        XZ = (q[j0:j0 + chunk, None] * X)[:, :, None] * Z[:, None, :]
        T += Y.T @ XZ.reshape(len(u), nxv * nzv)
    return T[ix[1], ix[0] * nzv + ix[2]]


def reciprocal_potential(pos_at, S, n, w, box, chunk=16384):
    """sum_K w_K Re(exp(-i K.r) S(K)) at the points pos_at for the k-vectors of
    the integer triplets n (the reciprocal sums of Eq. 21 and 25 given the
    structure factor S), through the per-axis factors of exp(-i K.r):
        G[r, n_y] = sum_{n_z} conj(Z_r(n_z)) W[n_x, n_y, n_z],  W = w S on the
        (n_x, n_y, n_z) grid (zero off the k-set),
    then the sums over n_y and n_x with conj(Y_r) and conj(X_r)."""
    pos_at = np.asarray(pos_at, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = np.asarray(n, dtype=np.int64)
    vals = [np.unique(n[:, d]) for d in range(3)]
    ix = [np.searchsorted(vals[d], n[:, d]) for d in range(3)]
    W = np.zeros((len(vals[0]), len(vals[1]), len(vals[2])), dtype=np.complex128)
    W[ix[0], ix[1], ix[2]] = np.asarray(w) * np.asarray(S)
    out = np.empty(len(pos_at))
    for r0 in range(0, len(pos_at), chunk):
        u = pos_at[r0:r0 + chunk] / box
        X, Y, Z = (np.exp(-2j * math.pi * np.outer(u[:, d], vals[d])) for d in range(3))
        acc = np.zeros(len(u), dtype=np.complex128)
        for a in range(len(vals[0])):
            G = Z @ W[a].T                      # (points, n_y)
            acc += X[:, a] * np.sum(Y * G, axis=1)
        out[r0:r0 + chunk] = acc.real
    return out


def potentials_factored(pos, a, q, box, beta, rcut, kmax, at=None):
    """The potentials of ``potentials`` at the atoms ``at`` (default: all),
    with the reciprocal part from ``structure_factor`` and
    ``reciprocal_potential`` (large systems)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    idx = np.arange(n) if at is None else np.asarray(at, dtype=np.int64)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    vol = float(np.prod(box))
    nv, _, w = kvectors(box, beta, kmax, half=True)
    u = reciprocal_potential(pos[idx], structure_factor(pos, q, box, nv), nv, w, box)
    i, j, d = real_space_pairs(pos[idx], pos, box, rcut)
    u += np.bincount(i, weights=q[j] * _pair_potential_real(d, beta, mix_width(a[idx][i], a[j])),
                     minlength=len(idx))
    u -= math.pi / (vol * beta * beta) * float(np.sum(q))
    aii = mix_width(a[idx], a[idx])
    selfc = -2.0 * beta / math.sqrt(math.pi) + np.where(np.isinf(aii), 0.0,
                                                         2.0 * np.where(np.isinf(aii), 0.0, aii)
                                                         / math.sqrt(math.pi))
    return u + selfc * q[idx]


def rhs_factored(pos, a, ion_pos, ion_q, chi_volts, box, beta, rcut, kmax):
    """b = chi - b_sol and Q_sol of ``rhs`` for one frame at the atoms ``pos``
    (any subset of the electrode), with the ion structure factor from
    ``structure_factor`` (large ion counts)."""
    pos = np.asarray(pos, dtype=np.float64)
    ion_pos = np.asarray(ion_pos, dtype=np.float64)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (len(pos),))
    vol = float(np.prod(box))
    nv, _, w = kvectors(box, beta, kmax, half=True)
    bsol = reciprocal_potential(pos, structure_factor(ion_pos, ion_q, box, nv), nv, w, box)
    i, I, d = real_space_pairs(pos, ion_pos, box, rcut)
    bsol += np.bincount(i, weights=ion_q[I] * _pair_potential_real(d, beta, a[i]),
                        minlength=len(pos))
    qsol = float(np.sum(ion_q))
    bsol -= math.pi / (vol * beta * beta) * qsol
    return np.asarray(chi_volts, dtype=np.float64) / K_E - bsol, qsol
