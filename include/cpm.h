/* cpm.h - C ABI of the constant-potential electrode-charge library (gfx950).
 *
 * The library computes electrode charges of the Gaussian-charge constant
 * potential method (SR-CPM) of Li, Wang, Liu, Jiang, arXiv 2111.06704:
 *
 *   cpm_build_E  assembles the dense Gaussian Ewald interaction matrix E over
 *                the N electrode atoms (Sec. II.C, Eq. 22-23) and the
 *                neutralising vector d' = E^-1 1 (Supplementary Eq. S8-S9);
 *   cpm_rhs      forms b = chi - b_sol for F electrolyte frames, where b_sol
 *                is the potential of the electrolyte point charges on the
 *                Gaussian electrode charges (Sec. III.A, Eq. 25);
 *   cpm_solve    solves E q_b = b by block conjugate gradients and enforces
 *                electroneutrality sum(q) = -Q_sol with the two-step
 *                post-treatment q = q_b - (1^T q_b + Q_sol) d (Eq. 34-35);
 *   cpm_mlp_*    a per-atom network that predicts a CG starting point.
 *
 * Conventions (all entry points):
 *   - Units: lengths in Angstrom, charges in e, applied potentials chi in
 *     volts. E is in Gaussian units (1/Angstrom); b is in e/Angstrom
 *     (chi is divided by k_e = 14.3996454784 V A / e inside cpm_rhs).
 *   - "Gaussian inverse width" a_i is the paper's alpha_i (Eq. 4); the Ewald
 *     splitting parameter beta is the paper's eta (Eq. 12-13).
 *   - Arrays are row-major, FP64 unless stated. Pointers named *_dev are
 *     device pointers (HBM of the current HIP device), *_host are host
 *     pointers. The caller owns every buffer it passes; the library copies
 *     what it keeps. A cpm_system owns its device memory until cpm_free.
 *   - Work is enqueued on the stream given to cpm_build_E (or cpm_set_stream).
 *     Calls that return host-side results (info structs, losses)
 *     synchronise that stream. cpm_rhs shares no device memory with the
 *     solve calls: a cpm_rhs enqueued on one stream may run while a solve
 *     runs on another, but two cpm_rhs calls on one system must not overlap
 *     (they share the structure-factor scratch).
 *   - Atom order in and out is the caller's order.
 *   - No exception or abort crosses the ABI. On failure a call returns a
 *     negative cpm_status and cpm_last_error() describes it (thread-local).
 */
#ifndef CPM_H
#define CPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPM_OK = 0,
  CPM_EINVAL = -1,    /* invalid argument (NaN/Inf, sizes, coincident atoms, ...) */
  CPM_ENOMEM = -2,    /* a device allocation failed; the system is unchanged      */
  CPM_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed              */
  CPM_ENOTSPD = -4,   /* CG breakdown p^T E p <= 0: E is not positive definite   */
  CPM_ENOTCONV = -5,  /* tolerance not reached within max_iter; outputs hold the
                         last projected iterate                                   */
  CPM_ESTATE = -6     /* call out of order (e.g. no network loaded)             */
} cpm_status;

typedef struct cpm_system cpm_system;   /* opaque */

/* Storage precisions of E. FP64 is always kept: it defines the residual.
   CPM_PROFILE_BUILD additionally times the assembly contraction (see
   cpm_profile_read). */
enum { CPM_STORE_F32 = 1u, CPM_STORE_BF16 = 2u, CPM_PROFILE_BUILD = 4u };

typedef struct {
  /* Gaussian inverse width a_i of each electrode charge in 1/A (Eq. 4).
     Either a pointer to N host values (gauss_inv_width_per_atom) or, when it
     is NULL, the single value gauss_inv_width for every atom. Mixing
     a_ij = (a_i^-2 + a_j^-2)^-1/2 (Eq. 5); a_ii = a_i / sqrt 2 (Eq. 6). */
  double gauss_inv_width;
  const double *gauss_inv_width_per_atom;
  double ewald_split;    /* beta > 0 in 1/A (the paper's eta, Eq. 12-13)         */
  double rcut;           /* real-space cutoff in A: images with d < rcut count  */
  double kspace_eps;     /* reciprocal cutoff K_max = 2 beta sqrt(ln(1/eps))     */
  double kmax_override;  /* > 0: use this K_max (1/A) instead of kspace_eps      */
  unsigned store_mask;   /* CPM_STORE_F32 | CPM_STORE_BF16: extra copies of E   */
  /* 1: slab geometry, z not periodic: the boundary correction of Eq. 39,
     e_ij += -(2 pi / V) [(z_i - z_j)^2 + L_z^2 / 6], on E and on the
     electrode-ion terms of b. On the neutral subspace it equals the dipole
     energy (2 pi / V) M_z^2, so the library stores the definite matrix
     E + (4 pi / V) z z^T and cpm_rhs returns b - (4 pi / V) M1 z with
     M1 = sum_I q_I z_I (z in [0, L_z)); cpm_solve then gives exactly the
     charges of the Eq. 39 system (they differ from it only by multiples of
     1 on the right-hand side and by terms that vanish for sum q = -Q_sol). */
  int slab_correction;
  /* 1: the point-charge simplification of Sec. III.C: electrode charges
     interact with each other and with the ions as classic point charges
     (the erfc(a d) screening terms of Eq. 22 and 25 are dropped) and keep
     the Gaussian self-energy sqrt(2/pi) a_i on the diagonal of E (for
     graphene, a_i = a^0 = 2.93295 /A makes it the lattice potential gap
     U^GRA). Needs finite a_i. The PCG-DC matrices keep their Eq. 36 form. */
  int point_charge_self;
} cpm_params;

/* Assemble E for n electrode atoms. The neutralising vector d' = E^-1 1
 * (S9) is solved on first use by cpm_solve / cpm_get_dprime /
 * cpm_set_warm_chi, which return its CPM_ENOTSPD / CPM_ENOTCONV (E of point
 * charges alone, a = inf, is in general not positive definite).
 *   pos_host  (n, 3) positions in an orthorhombic box [0, box_d); values
 *             outside are wrapped.
 *   box_host  (3,) box edges in A, > 0. The box is 3D periodic (tinfoil,
 *             Sec. II.B after Eq. 14).
 *   stream    hipStream_t (may be NULL for the default stream).
 * E_ij (i != j) = sum over images n with d = |r_ij + n L| < rcut of
 *   [erfc(beta d) - erfc(a_ij d)] / d
 *   + sum_{K != 0, |K| <= K_max} (4 pi / V) exp(-K^2 / 4 beta^2) / K^2 cos(K.r_ij)
 *   - pi / (V beta^2);
 * E_ii adds -2 beta / sqrt(pi) + 2 a_ii / sqrt(pi) and takes n != 0 images
 * only (Eq. 22-23, with the reciprocal prefactor of Eq. 13).
 * Errors: CPM_EINVAL for n < 1, non-finite input, box <= 0, beta <= 0,
 * a_i <= 0, rcut <= 0, eps outside (0, 1), two atoms closer than 1e-6 A
 * (minimum image); CPM_ENOMEM.
 * On error *out is set to NULL and nothing is leaked. */
cpm_status cpm_build_E(const double *pos_host, int64_t n, const double *box_host,
                       const cpm_params *params, void *stream, cpm_system **out);

/* Release every device and host resource of s (NULL is a no-op). */
void cpm_free(cpm_system *s);

/* Change the stream later calls enqueue on. */
cpm_status cpm_set_stream(cpm_system *s, void *stream);

/* Problem facts: n atoms, number of half-space k-vectors, K_max used, memory
   held on the device (bytes). Any pointer may be NULL. */
cpm_status cpm_describe(const cpm_system *s, int64_t *n, int64_t *n_kvec, double *kmax,
                        int64_t *device_bytes);

/* Right-hand side for f electrolyte frames of m point charges each (Eq. 25):
 *   b[f, i] = chi_i / k_e - sum_I q_fI e_iI(a_i),   Q_sol[f] = sum_I q_fI,
 * where e_iI is Eq. 22 between Gaussian electrode charge i (width a_i) and
 * point charge I (mixing width a_iI = a_i, Sec. II.A).
 *   ion_pos_dev (f, m, 3), ion_q_dev (f, m), chi_dev (n,) in volts,
 *   b_out_dev (f, n), qsol_out_dev (f,) - all device pointers.
 * m may be 0 (then b = chi / k_e and Q_sol = 0). An ion exactly on an
 * electrode site uses the limit 2 (a_i - beta) / sqrt(pi) of the real-space
 * term. Errors: CPM_EINVAL for NULL pointers, f < 1, m < 0. */
cpm_status cpm_rhs(cpm_system *s, const double *ion_pos_dev, const double *ion_q_dev,
                   int64_t m, int64_t f, const double *chi_dev, double *b_out_dev,
                   double *qsol_out_dev);

/* cpm_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result, with the scratch of the structure factors, partial sums and
 * ion cell lists in a fixed device array of 4 Mi doubles (32 MiB) that the
 * library holds on each GPU it runs on until the process ends, instead of
 * memory allocated on the system. No hipMalloc, hipFree or allocating
 * library call, and no memset node. The partial sums are then fewer when
 * the usual split would not fit (a different summation order: b agrees
 * with cpm_rhs to rounding, and bitwise when the usual split fits).
 * Errors: those of cpm_rhs, and CPM_EINVAL when even the least split needs
 * more scratch (the message gives both sizes; e.g. 2 n_k f doubles of
 * structure factors alone). Calls that overlap on one GPU share the array
 * and race: serialise them (one stream, or events). */
cpm_status cpm_rhs_noalloc(cpm_system *s, const double *ion_pos_dev, const double *ion_q_dev,
                           int64_t m, int64_t f, const double *chi_dev, double *b_out_dev,
                           double *qsol_out_dev);

enum { CPM_PREC_F64 = 0, CPM_PREC_F32 = 1, CPM_PREC_BF16 = 2 };
enum { CPM_WARM_ZERO = 0, CPM_WARM_CHI = 1, CPM_WARM_MLP = 2 };
enum { CPM_PRECOND_JACOBI = 0, CPM_PRECOND_DC = 1 };

typedef struct {
  double tol;          /* stop when |b - E q_b|_2 <= tol |b|_2 (true FP64 residual) */
  int max_iter;        /* total CG iterations (inner iterations for mixed)          */
  int precision;       /* CPM_PREC_*: storage of E in the CG matvec. F32/BF16 run
                          iterative refinement: inner FP32 CG on the rounded E,
                          FP64 residual b - E q on the FP64 E                      */
  int warm_start;      /* CPM_WARM_*: zero, the no-electrolyte solution q_chi, or
                          the network prediction                                   */
  double inner_tol;    /* reliable-update factor (mixed): the FP64 true residual
                          replaces the recursive one once the latter has fallen by
                          this factor, e.g. 1e-2                                   */
  int check_every;     /* iterations between the device-side convergence checks
                          (>= 1). FP32 / BF16 replace the recursive residual only
                          at a check: with the coarse correction (about tenfold
                          per iteration) keep it at 2-4, as longer intervals let
                          the recursion run orders past the reliable-update
                          point and can cost many iterations                  */
  int preconditioner;  /* CPM_PRECOND_JACOBI (diag E) or CPM_PRECOND_DC (the
                          system's sparse P, Sec. III.B.2: the PCG-DC matrix of
                          cpm_precond_dc or the sparsified inverse of
                          cpm_precond_sparse_inverse, whichever was built last,
                          with the Eq. 37 fill when cpm_precond_gap enabled it,
                          and the coarse correction of cpm_precond_coarse)      */
} cpm_solve_opts;

typedef struct {
  int iterations;      /* CG iterations (max over frames; inner for mixed)         */
  int outer;           /* refinement steps (mixed) / true-residual restarts (F64)  */
  double max_rel_resid;/* max over frames of |b - E q_b| / |b| at exit             */
  double initial_rel_resid; /* max over frames of the relative residual at start   */
  double max_abs_sum_q;/* max over frames of |sum(q) + Q_sol| after projection     */
  double warm_ms;      /* GPU time of the warm start (network, shifts and the FP64
                          residual of the start), from HIP events               */
  double solve_ms;     /* wall time of the whole call                              */
  int fell_back;       /* 1 if the warm start of some frame was rejected (it did not
                          lower the energy x.E x / 2 - x.b below zero's)         */
  /* optional per-frame outputs (host arrays of length f, may be NULL) */
  int *frame_iters;
  double *frame_rel_resid;
} cpm_solve_info;

/* Electrode charges for f right-hand sides.
 *   b_dev (f, n), qsol_dev (f,), q_out_dev (f, n): device pointers.
 * q_out[f] = q_b - (1^T q_b + Q_sol[f]) d with E q_b = b[f] (Eq. 35),
 * d = d' / 1^T d'. Errors: CPM_EINVAL (pointers, f < 1, tol <= 0, unknown
 * precision or preconditioner, precision not stored), CPM_ESTATE
 * (CPM_WARM_MLP without a network, CPM_PRECOND_DC before cpm_precond_dc),
 * CPM_ENOTSPD (breakdown), CPM_ENOTCONV (q_out then holds the projected last
 * iterate). info may be NULL. */
cpm_status cpm_solve(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                     const cpm_solve_opts *opts, double *q_out_dev, cpm_solve_info *info);

/* ---- PCG-DC preconditioner (Sec. III.B.2, Eq. 36) --------------------------
 * For every atom tau: the local matrix M_tau of Eq. 36 over tau and every atom
 * image within rcut of it (distance <= rcut),
 *   m_ii = sqrt(2/pi) a_i,
 *   m_ij = [erfc(g r_ij) - erfc(g rcut)] / r_ij  (r_ij < rcut), 0 otherwise,
 * with r_ij the distance of the two images; the column of M_tau^-1 belonging
 * to tau becomes column tau of P (entries of images of one atom add up, zero
 * beyond rcut). The solver uses the symmetric part (P + P^T) / 2. Built once
 * per system: the neighbourhoods on host threads, the local matrices and
 * their FP64 Cholesky factorisations on the device (rocSOLVER, batched);
 * kept on the device in a block-dense form (tiles of 64 atoms over the
 * union of their columns) that cpm_solve applies with CPM_PRECOND_DC on the
 * FP64 matrix cores. The paper's choice for graphene electrodes is
 * g = 0.083 / A, rcut = 8 A. Errors: CPM_EINVAL (g or rcut not finite and
 * > 0, point-charge atoms), CPM_ENOTSPD (a local matrix is not positive
 * definite), CPM_ENOMEM, CPM_EDEVICE. */
cpm_status cpm_precond_dc(cpm_system *s, double screening_g, double rcut);

/* z = P r for f vectors, r_dev and z_dev (f, n) device arrays: the solver's
   own apply kernel (tests), with the Eq. 37 fill when it is on. CPM_ESTATE
   before a preconditioner is built. */
cpm_status cpm_precond_apply(cpm_system *s, const double *r_dev, int64_t f, double *z_dev);

/* ---- PCG-Normal / PCG-Full (Sec. III.B.2) ---------------------------------
 * P = E^-1 sparsified by distance: p_ij = (E^-1)_ij for every pair whose
 * nearest images are strictly closer than rcut, and the diagonal; 0
 * elsewhere. E^-1 = S + d' d'^T / C_ele from the matrix-inversion path
 * (cpm_mi_build first; S symmetrised entry by entry). PCG-Normal takes a
 * preset rcut, PCG-Full the cutoff of the neighbour list. The result
 * replaces the system's sparse preconditioner (the one CPM_PRECOND_DC
 * applies) in the same block-dense form. Errors: CPM_EINVAL (rcut not finite and
 * > 0), CPM_ESTATE (no cpm_mi_build), CPM_ENOMEM, CPM_EDEVICE. */
cpm_status cpm_precond_sparse_inverse(cpm_system *s, double rcut);

/* Eq. 37: enable != 0 fills the zeros of the current sparse preconditioner
 * with p_gap = (1^T E^-1 1 - sum_ij p_ij) / n_zero, the mean of the entries of
 * E^-1 that the sparsification removed (1^T E^-1 1 = 1^T d' = C_ele, solved
 * here if needed; n_zero = n^2 - the stored entries); enable = 0 removes the
 * fill. Applied as z = (P - p_gap on the pattern of P) r + p_gap (1^T r) 1.
 * A negative p_gap can make P indefinite: a solve then stops with
 * CPM_ENOTSPD (r^T P r <= 0). gap_out (may be NULL) receives p_gap (0 when
 * disabled). Errors: CPM_EINVAL, CPM_ESTATE (no preconditioner), the d'
 * solve's errors. */
cpm_status cpm_precond_gap(cpm_system *s, int enable, double *gap_out);

/* ---- coarse-space correction of the sparse preconditioner -----------------
 * Not in the paper: a second level on top of the sparse P of Sec. III.B.2
 * (the balancing Neumann-Neumann form of two-level preconditioning; Mandel,
 * Commun. Numer. Methods Eng. 9, 233 (1993)). Z (n x m) holds the indicator
 * columns of m patches of atoms: the atoms are split into z-slabs (sorted z,
 * a new slab wherever two consecutive values differ by more than 1 A) and
 * each slab into nx x ny in-plane bins of the box, nx = max(1, floor(L_x /
 * edge + 1/2)) and likewise ny; empty bins are dropped. With E_c = Z^T E Z,
 * Q = Z E_c^-1 Z^T and P_D = I - E Q, CPM_PRECOND_DC then applies
 *   z = P_D^T P P_D r + Q r,
 * which is symmetric positive definite for every SPD P, maps E Z exactly to
 * Z (the coarse modes converge in one step) and equals E^-1 when P does.
 * A local P leaves the long-wavelength modes of E at large eigenvalues;
 * the coarse solve removes them. E Z is kept in FP32 (m x n_pad floats)
 * and E_c^-1 in FP64 (m_pad^2 doubles); each apply adds two products with
 * E Z on the FP32 matrix cores and two with E_c^-1 on the FP64 ones.
 * edge > 0: builds the space for that in-plane patch edge (A) and keeps it
 * until replaced or disabled (it does not depend on P, so rebuilding P
 * keeps it); edge <= 0: disables it. m_out (may be NULL) receives m.
 * CPM_EINVAL and CPM_ESTATE leave the current coarse space as it was; a
 * build that fails later (CPM_ENOMEM, CPM_EDEVICE, CPM_ENOTSPD) leaves the
 * system without one.
 * Errors: CPM_EINVAL (edge not finite, more than 8192 patches), CPM_ESTATE
 * (no sparse preconditioner built), CPM_ENOTSPD (E_c not positive
 * definite), CPM_ENOMEM, CPM_EDEVICE. */
cpm_status cpm_precond_coarse(cpm_system *s, double edge, int64_t *m_out);

/* ---- matrix-inversion path (Sec. III.B.1 MI; Eq. 33-35) -------------------
 * cpm_mi_build forms S = E^-1 (I - 1 d^T) (Eq. 33), symmetric, whose column
 * j is the two-step charge vector (Eq. 35) of the unit right-hand side e_j
 * with Q_sol = 0: it runs cpm_solve on the n unit vectors, 64 at a time, with
 * the caller's opts (tolerance, precision, preconditioner; the warm start is
 * ignored), and keeps S on the device (n_pad^2 doubles). The error of S is
 * that of those solves. cpm_mi_solve then gives q = S b - Q_sol d for f
 * frames with one block product (b_dev, q_out_dev (f, n), qsol_dev (f,)
 * device arrays; enqueued on the stream, not synchronised).
 * Errors: CPM_EINVAL, CPM_ENOMEM, the solve's errors (build); CPM_ESTATE
 * (cpm_mi_solve before cpm_mi_build). */
cpm_status cpm_mi_build(cpm_system *s, const cpm_solve_opts *opts);
cpm_status cpm_mi_solve(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                        double *q_out_dev);

/* ---- galvanostatic charge-discharge (Supplementary Note, Eq. S14-S24) -----
 * Electrode a carries a prescribed total charge Q_a; minimising the energy of
 * Eq. S14 under these constraints gives E q = b + Delta u, Delta u_i =
 * Delta mu_a for the atoms i of electrode a (Eq. S15).
 * cpm_gcd_build: labels_host (n,) int32, the electrode of each atom (caller's
 * atom order), every one of the m electrodes (1 <= m <= 64) non-empty. Solves
 * E a^h = b^h for the m indicator vectors b^h (Eq. S22-S23) with the block
 * solver and the caller's opts (tolerance on |b^h - E a^h| / |b^h|,
 * precision, preconditioner; the warm start is ignored), keeps
 * A = (a^1 .. a^m) (m n doubles) on the device, sums it per electrode into
 * the capacitance coefficients C_ab = sum over the atoms of a of a^b_i
 * (Eq. S24), symmetrises C_E (it is symmetric up to the solve error), and
 * factors it on the device. Outputs (host): C_out_host (m, m) row-major in
 * units of e per (V / k_e); det_out = |C_E| and joint_out = C(Q, -Q) =
 * |C_E| / sum_ab C_ab (Eq. S21; NaN unless m = 2), either may be NULL. A later
 * build replaces the previous one. info as for cpm_solve (max_abs_sum_q 0).
 * Errors: CPM_EINVAL (NULL, m, a label outside [0, m), an empty electrode,
 * the opts), CPM_ESTATE (CPM_PRECOND_DC before cpm_precond_dc), CPM_ENOMEM,
 * CPM_ENOTSPD (C_E not positive definite), the solve's errors.
 * cpm_gcd_solve: b_dev (f, n), Q_dev (f, m) the totals Q_a per frame,
 * q_out_dev (f, n), dmu_out_dev (f, m) or NULL: device arrays. q_b = E^-1 b
 * by the block solver (opts as above), Delta mu = C_E^-1 (Q - L q_b)
 * (Eq. S18-S20) and q = q_b + A Delta mu (Eq. S17). The system's E is used as
 * built (with the boundary correction of Eq. 39 when it was requested; the
 * constraint then fixes the totals, not the dipole). Synchronous.
 * info->max_abs_sum_q = max over frames and electrodes of |sum_a q - Q_a|.
 * Errors: CPM_EINVAL, CPM_ESTATE (before cpm_gcd_build), CPM_ENOTCONV (q_out
 * then holds the shifted last iterate), the solve's errors. */
cpm_status cpm_gcd_build(cpm_system *s, const int32_t *labels_host, int32_t m,
                         const cpm_solve_opts *opts, double *C_out_host, double *det_out,
                         double *joint_out, cpm_solve_info *info);
cpm_status cpm_gcd_solve(cpm_system *s, const double *b_dev, const double *Q_dev, int64_t f,
                         const cpm_solve_opts *opts, double *q_out_dev, double *dmu_out_dev,
                         cpm_solve_info *info);

/* Copy E (caller's atom order) into dst_dev with leading dimension ld >= n,
   in the requested precision (FP64 double, FP32 float, BF16 uint16 bits).
   CPM_EINVAL if that precision is not stored. */
cpm_status cpm_get_E(const cpm_system *s, int precision, void *dst_dev, int64_t ld);

/* Copy the block E[row0 : row0 + rows, col0 : col0 + cols] into dst_dev
   (rows x cols, leading dimension ld >= cols) in the requested precision:
   inspection of matrices too large to copy whole (N = 131072: 137 GB).
   CPM_EINVAL if the block leaves [0, n)^2 or that precision is not stored. */
cpm_status cpm_get_E_block(const cpm_system *s, int precision, int64_t row0, int64_t col0,
                           int64_t rows, int64_t cols, void *dst_dev, int64_t ld);

/* Copy d' = E^-1 1 (S9) into dst_dev (n,) and return C_ele = 1^T d'. */
cpm_status cpm_get_dprime(cpm_system *s, double *dst_dev, double *c_ele);

/* Block matrix product V = E P for f vectors, P and V (f, n) row-major
   device arrays (one vector per row), E in the requested precision (FP32/BF16 products accumulate
   in FP32 and are returned widened to FP64). The CG's own matvec. */
cpm_status cpm_matvec(cpm_system *s, int precision, const double *p_dev, int64_t f,
                      double *v_dev);

/* ---- learned warm start --------------------------------------------------
 * A per-atom multilayer perceptron 26 -> 64 -> 64 -> 1 with SiLU activations
 * predicts each atom's charge from its own b_i - mean(b), its layer index and
 * its 12 nearest electrode neighbours' (b_j - mean(b), r_ij). Neighbours are
 * ordered by distance, then azimuth about +z from +x, then index, using the
 * minimum image; distances and angles are compared after rounding to 1e-6.
 * The prediction is shifted to sum(q0) = -Q_sol, and the CG start is
 * q_b0 = q0 + mu0 d' with mu0 = mean(b - E q0) (the Lagrange shift of
 * Eq. 29-31). A start that does not lower the energy x.E x / 2 - x.b below
 * that of x = 0 (equivalently: whose E-norm error, the norm CG reduces, is
 * not below the zero start's) is discarded (zero start). Feature layout per atom: [b_i - mean, layer/(L-1),
 * 12 x (b_j - mean), 12 x r_ij], with b scaled by 1/b_scale and r by 1/r_scale;
 * the output is multiplied by q_scale. */
#define CPM_MLP_IN 26
#define CPM_MLP_HIDDEN 64
#define CPM_MLP_NPARAM (CPM_MLP_IN * CPM_MLP_HIDDEN + CPM_MLP_HIDDEN + \
                        CPM_MLP_HIDDEN * CPM_MLP_HIDDEN + CPM_MLP_HIDDEN + CPM_MLP_HIDDEN + 1)

/* Parameter vector layout (float32, CPM_MLP_NPARAM values):
   W1 (26 x 64, row-major: input-major), b1 (64), W2 (64 x 64), b2 (64),
   W3 (64), b3 (1). Layer: h = silu(x W + b). */

/* Set the 12-neighbour list from the geometry given at build (computed on
   the host) and the layer index of each atom (n ints, host; n_layers >= 1). */
cpm_status cpm_mlp_init(cpm_system *s, const int32_t *layer_host, int32_t n_layers,
                        float b_scale, float r_scale, float q_scale);

/* Copy the neighbour list (n, 12) int32 to host (for tests). */
cpm_status cpm_mlp_neighbours(const cpm_system *s, int32_t *nbr_host);

/* Load / read parameters (host float32, CPM_MLP_NPARAM values). Setting
   resets the Adam moments. */
cpm_status cpm_mlp_set_params(cpm_system *s, const float *params_host);
cpm_status cpm_mlp_get_params(const cpm_system *s, float *params_host);

/* Features (f*n, 26) float32 of f frames of b (device) into feat_out_dev. */
cpm_status cpm_mlp_features(cpm_system *s, const double *b_dev, int64_t f, float *feat_out_dev);

/* Network output y (rows,) float32 for feature rows (rows, 26) (device). */
cpm_status cpm_mlp_forward(cpm_system *s, const float *feat_dev, int64_t rows, float *y_out_dev);

/* Loss and gradient of the mean squared error L = mean((y - t)^2) over rows
   (device features and targets, targets already divided by q_scale); the
   gradient (CPM_MLP_NPARAM floats) goes to grad_out_dev, the loss to *loss. */
cpm_status cpm_mlp_loss_grad(cpm_system *s, const float *feat_dev, const float *target_dev,
                             int64_t rows, float *grad_out_dev, double *loss);

/* One Adam step (Kingma & Ba 2015; beta1, beta2, eps, bias correction) with
   learning rate lr on the loss of one mini-batch; returns the batch loss
   before the step. */
cpm_status cpm_mlp_train_step(cpm_system *s, const float *feat_dev, const float *target_dev,
                              int64_t rows, float lr, float beta1, float beta2, float eps,
                              double *loss);

/* One pass over f frames of (b, q) pairs (device, (f, n) each; q is the
   solver's neutral charge): rows are visited in the order perm_dev (f*n
   int64 row ids, row = frame * n + atom), batch rows per Adam step. Features
   and targets (q / q_scale) are gathered on the device. mean_loss receives
   the mean of the batch losses. */
cpm_status cpm_mlp_train_epoch(cpm_system *s, const double *b_dev, const double *q_dev, int64_t f,
                               const int64_t *perm_dev, int64_t batch, float lr, float beta1,
                               float beta2, float eps, double *mean_loss);

/* Precompute q_chi, the neutral solution without electrolyte (b = chi / k_e,
   Q_sol = 0), used by CPM_WARM_CHI. chi_dev (n,) volts; opts as cpm_solve. */
cpm_status cpm_set_warm_chi(cpm_system *s, const double *chi_dev, const cpm_solve_opts *opts);

/* The CG start cpm_solve takes for warm_start (CPM_WARM_CHI or CPM_WARM_MLP)
   and f frames of b (device, (f, n)) and Q_sol (device, (f,)), before its
   acceptance test: x0_out_dev (f, n) = q0 + mu0 d' with q0 the network's
   prediction (times q_scale) or q_chi, shifted to sum(q0) = -Q_sol, and
   mu0 = mean(b - E q0) (Eq. 29-31); r0_out_dev (f, n) = b - E x0 in FP64.
   The same kernels as cpm_solve (inspection and tests).
   Errors: CPM_EINVAL, CPM_ESTATE (network or q_chi not set), d' errors. */
cpm_status cpm_warm_start(cpm_system *s, int warm_start, const double *b_dev,
                          const double *qsol_dev, int64_t f, double *x0_out_dev,
                          double *r0_out_dev);

/* ---- live kernel timing ----------------------------------------------------
 * While enabled, the library brackets launches of the block matrix product
 * (per storage precision of E), of the assembly contraction and of the ion
 * structure factors of cpm_rhs with HIP events on its stream and records
 * each launch's algorithmic work:
 *   matvec: bytes s*n*n (E) + 2 * s_v * n * cols (P read, V written),
 *           s = 8/4/2 for FP64/FP32/BF16 E, s_v = 8 (FP64) or 4 (FP32 vectors);
 *   assembly: flops 4 * n_k * n (n + 1) / 2 for a chunk of n_k k-vectors;
 *   structure factors: flops 4 * n_k * m * f (one complex multiply-add of
 *           q e^{iK.r} per k-vector, ion and frame) for f frames of m ions.
 * cpm_profile_enable(s, on) starts a new window (clears earlier records):
 * on = 0 stops timing, on = 1 times every launch, on = k > 1 times every
 * k-th launch of each kind (the bracketing
 * launch costs the host ~10 us more than a plain one; sampling keeps that
 * out of the throughput being measured); cpm_profile_read synchronises the
 * stream and sums each kind over the timed launches. */
typedef struct {
  int64_t launches[5];   /* index: CPM_PREC_F64, CPM_PREC_F32, CPM_PREC_BF16, 3 = assembly,
                            4 = structure factors                                         */
  double ms[5];          /* summed kernel time (ms) between the events                    */
  double work[5];        /* summed algorithmic bytes (matvec) or flops (the others)       */
} cpm_profile_info;

cpm_status cpm_profile_enable(cpm_system *s, int on);
cpm_status cpm_profile_read(cpm_system *s, cpm_profile_info *out);

/* ---- diagnostics ---------------------------------------------------------- */
const char *cpm_status_str(cpm_status st);
const char *cpm_last_error(void);   /* thread-local message of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */
