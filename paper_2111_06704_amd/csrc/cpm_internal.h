// Internal declarations shared by the HIP translation units of libcpm.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cpm.h"

namespace cpm {

constexpr int kColGroup = 16;  // CG works on column groups of 16 right-hand sides
constexpr double kCoulombVA = 14.3996454784;   // e^2/(4 pi eps0) in V*A/e

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// thread-local error message
void set_error(const std::string &msg);
const char *last_error();

struct Kset {
  int64_t nk = 0;              // number of half-space vectors
  int nmax[3] = {0, 0, 0};
  std::vector<int32_t> n;      // nk*3 integer triplets
  std::vector<double> w;       // nk weights 2 (4 pi / V) exp(-K^2/4 beta^2) / K^2
  // The vectors are ordered by (n_x, n_y, n_z), so each (n_x, n_y) column is
  // a contiguous range of consecutive n_z. Runs split every column into
  // pieces of at most kRun vectors: runs[2r] = first index, runs[2r+1] = length.
  std::vector<int32_t> runs;
  int64_t nruns = 0;
  // info[4k..4k+3] = n_x, n_y, n_z, 1 if k starts a run (else 0)
  std::vector<int32_t> info;
  // (n_x, n_y) columns for the structure-factor product, sorted by their
  // largest |n_z| (descending) and padded to a multiple of kSfTile:
  // cols[4c..4c+3] = n_x, n_y, m = largest |n_z| (-1: padding), k index of
  // n_z = 0 (the column (0, 0) holds n_z = 1..m only: k index of n_z = 0 is
  // one before its first vector)
  std::vector<int32_t> cols;
  int64_t ncols = 0, ncols_pad = 0;
  int smax = 0;                // largest |n_z|
};

constexpr int kSfTile = 64;    // columns per workgroup of the structure-factor product

// electrode atoms on at most kMaxPlanes exact z-planes (graphite layers)
// take the factored back-projection; its n_z sums keep a table of
// |n_z| <= kMaxPlaneS per plane in LDS; kPlaneTile atoms per wave tile
constexpr int kMaxPlanes = 64;
constexpr int kMaxPlaneS = 1023;
constexpr int kPlaneTile = 16;
constexpr int kRun = 24;       // longest run of consecutive n_z (phase recurrence length)

// Half-space reciprocal vectors with |K| <= kmax, K != 0 (host).
Kset make_kset(const double box[3], double beta, double kmax);

struct Workspace {            // CG scratch, grown on demand
  int64_t cols = 0;           // padded number of columns the buffers hold
  int splits = 0;
  void *x = nullptr, *r = nullptr, *p = nullptr, *z = nullptr, *v = nullptr;  // n_pad*cols (double)
  void *vpart = nullptr;      // splits*n_pad*cols (double)
  // FP32 vectors of the inner CG, separate from the FP64 ones so that their
  // padding rows (>= n) are always zero
  void *xf = nullptr, *rf = nullptr, *pf = nullptr, *zf = nullptr, *vf = nullptr;
  double *rt = nullptr;       // n_pad*cols double: r with the 16 columns of a group interleaved
  double *partial = nullptr;  // dot partial sums: 2*nblk*cols
  double *bpart = nullptr;    // per-workgroup dot partials of the preconditioner apply
  double *scal = nullptr;     // per-column scalars, see cg.hip
  double *red = nullptr;      // 3*64 doubles: reduced dot partials (p.v; r.r and r.z)
  double *sum_err = nullptr;  // MAX_COLS doubles: |sum q + Q_sol| per column after the projection
  double *rsum = nullptr;     // MAX_COLS doubles: 1^T r per column (the Eq. 37 gap term)
  double *bx = nullptr;       // n_pad*cols double: right-hand sides / outer iterate
  double *bres = nullptr;     // n_pad*cols double: outer residual
  int *flags = nullptr;       // device status words
  int *hstat = nullptr;       // pinned host copies of the status words (ring of kStatusSlots)
  double *hfin = nullptr;     // pinned host copy of the final per-column scalars, then the
                              // projection's |sum q + Q_sol| per column
  int *hfl = nullptr;         // pinned host copy of the final status words
  int hit = 0;                // iterations enqueued by the last solve (for messages)
  hipEvent_t ev[2] = {nullptr, nullptr};
  size_t bytes = 0;
};
constexpr int kStatusSlots = 2;

// device buffer of a system that keeps its largest size: per-call scratch
// (warm starts, per-frame means, error words) without an allocation per call
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct Precond {              // sparse PCG preconditioner P
  bool ready = false;
  int kind = 0;               // 0: PCG-DC (P + P^T) / 2 (Eq. 36); 1: E^-1 sparsified by distance
  double g = 0, rcut = 0;     // screening and cutoff of Eq. 36 (kind 0), cutoff (kind 1)
  int width = 0;              // entries per ELL row (padded with (i, 0))
  int max_local = 0;          // largest local matrix
  int64_t nnz = 0;
  // device ELL form (systems below kPcBlockTiles tiles): column of entry k
  // of the row of atom atom_order[t] at t * width + k, value (minus gap on
  // the real entries when the gap is on)
  int32_t *idx = nullptr;
  double *val = nullptr;
  int64_t bytes = 0;           // device memory held
  // Eq. 37: the zeros of P filled with gap (0: off); applied as
  // z = (P - gap on its pattern) r + gap (1^T r) 1
  double gap = 0.0;
  double sum_p = 0.0;         // sum of the entries of P (without the gap)
  // host ELL form without the gap: row t is the row of atom atom_order[t],
  // entry k (column, value) at t * width + k, h_len[t] real entries
  std::vector<int32_t> h_idx;
  std::vector<double> h_val;
  std::vector<int32_t> h_len;
  // block-dense form (from kPcBlockTiles tiles on): tile t holds the kPcTile ELL
  // rows t kPcTile .. (atom_order positions) over U_t, the sorted union of
  // their columns padded to a multiple of 4 with its first column:
  // U_t = uidx[uoff[t] .. uoff[t + 1]), entry (row, k) of the tile at
  // blk[(uoff[t] + k) * kPcTile + row] (P minus gap on its pattern, zero
  // off it and in the padding)
  int64_t ntiles = 0;
  int64_t *uoff = nullptr;
  int32_t *uidx = nullptr;
  double *blk = nullptr;
  std::vector<int64_t> h_uoff;
  std::vector<int32_t> h_uidx;
};
constexpr int kPcTile = 64;
// the block-dense form from this many tiles on (N >= 16384); below, the ELL
// form (one wavefront per row) keeps more of the chip busy
constexpr int64_t kPcBlockTiles = 256;
void free_precond(Precond &p);

// Coarse-space correction of the sparse preconditioner P (two-level,
// balancing Neumann-Neumann form): Z holds the indicator columns of m
// patches of atoms (z-slabs split into in-plane bins), E_c = Z^T E Z, and
// the apply is z = P_D^T P P_D r + Z E_c^-1 Z^T r with P_D = I - E Z E_c^-1 Z^T.
// The local P resolves the short-range response, the coarse solve the
// long-wavelength modes that a local P leaves at large eigenvalues.
struct Coarse {
  bool ready = false;
  double edge = 0.0;            // in-plane patch edge (A)
  int64_t m = 0, mp = 0;        // patches, and padded to kCoarseAlign
  int nslab = 0;
  int32_t *pid = nullptr;       // n: patch of atom i
  int32_t *perm = nullptr;      // n: atoms grouped by patch, increasing index in a patch
  int32_t *off = nullptr;       // mp + 1: patch t is perm[off[t] .. off[t + 1]) (empty past m)
  float *az = nullptr;          // mp x ld: az[t * ld + i] = (E Z)_it (zero padding)
  double *eci = nullptr;        // mp x mp: E_c^-1 (zero padding)
  int ks = 0;                   // atom slices of the Z^T-side product
  int64_t kslice = 0;
  // scratch for up to 64 columns: row-interleaved u = P_D r and w = P u
  // (layout of the residual copy rt), coarse vectors (cols x mp), the
  // slice partials of (E Z)^T w
  double *ut = nullptr, *wt = nullptr;
  double *c1 = nullptr, *g1 = nullptr, *dg = nullptr;
  float *g1f = nullptr, *c2p = nullptr;
  int64_t bytes = 0;
};
constexpr int kCoarseAlign = 256;     // patches per workgroup of the Z^T-side product
constexpr int kCoarseCols = 64;       // columns of the coarse scratch (the solver's most)
constexpr int64_t kMaxCoarse = 8192;  // most patches (E_c^-1: 512 MB)
constexpr double kSlabGap = 1.0;      // z gap (A) that starts a new slab
void free_coarse(Coarse &c);

struct Gcd {                 // capacitance coefficients (Supplementary Eq. S22-S24)
  bool ready = false;
  int m = 0;                  // electrodes
  int32_t *labels = nullptr;  // n: electrode of each atom
  double *A = nullptr;        // m * n: A[h * n + i] = (E^-1 b^h)_i
  double *mats = nullptr;     // 2 m^2 + 4: C_E (symmetrised), C_E^-1, then |C_E|,
                              // sum of C_E, C(Q, -Q), factor status
  int64_t bytes = 0;
};

struct Mlp {
  bool ready = false;
  int32_t *nbr = nullptr;     // n*12
  float *nbr_r = nullptr;     // n*12 distances
  int32_t *layer = nullptr;   // n
  int32_t n_layers = 1;
  float b_scale = 1.f, r_scale = 1.f, q_scale = 1.f;
  float *params = nullptr;    // CPM_MLP_NPARAM
  float *adam_m = nullptr, *adam_v = nullptr;
  float *grad = nullptr;      // CPM_MLP_NPARAM
  float *gpart = nullptr;     // per-tile gradient partials
  int64_t gpart_tiles = 0;
  double *loss = nullptr;     // device loss scalar(s)
  int64_t step = 0;
  float *feat = nullptr;      // feature scratch for the warm start
  float *yout = nullptr;
  int64_t feat_rows = 0;
  bool params_set = false;
};

// Live kernel timing: HIP events around every launch of the profiled
// kernels (block matrix product per storage precision, and the assembly
// contraction), enabled per system.
struct Profile {
  bool enabled = false;
  int stride = 1;            // time every stride-th block-product launch of each kind
  int64_t seen[5] = {0, 0, 0, 0, 0};
  // whether this launch of the block product (kind 0..2) is to be timed
  bool sample(int kind) { return enabled && (seen[kind]++ % stride) == 0; }
  struct Rec {
    int kind;              // 0..2: matvec FP64/FP32/BF16, 3: assembly contraction,
                           // 4: ion structure factors of the right-hand side
    double work;           // algorithmic bytes (matvec) or flops (assembly) of the launch
    hipEvent_t a, b;
    int mark = -1;         // slot in marks: 1 if the launch did its work, 0 if it was gated off
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  static constexpr int kMarks = 1 << 16;
  int *marks = nullptr;    // device, kMarks ints (allocated when profiling is enabled)
  int next_mark = 0;
  // a mark slot for a gated launch (nullptr when none is left)
  int *take_mark(Rec &r) {
    if (!marks || next_mark >= kMarks) return nullptr;
    r.mark = next_mark++;
    return marks + r.mark;
  }
  hipEvent_t get();
  // new record; its events are passed to hipExtLaunchKernelGGL, which
  // stamps them as part of the kernel dispatch (no extra queue packets)
  Rec &add(int kind, double work);
  void reset();
};

}  // namespace cpm

struct cpm_system {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0, ld = 0;      // ld = padded leading dimension (multiple of 128)
  double box[3] = {0, 0, 0};
  double vol = 0, beta = 0, rcut = 0, kmax = 0;
  bool slab = false;          // boundary correction of Eq. 39 (definite form)
  cpm::Kset kset;
  double *pos = nullptr;      // n*3 device
  double *width = nullptr;    // n device (Gaussian inverse widths)
  // n device: widths of the real-space pair screening erfc(a d) (width, or
  // +inf everywhere under the point-charge simplification: then its own array)
  double *rs_width = nullptr;
  bool point_self = false;    // point-charge simplification (Sec. III.C)
  int32_t *kn = nullptr;      // nk*3 device
  double *kw = nullptr;       // nk device
  int32_t *kinfo = nullptr;   // nk*4 device (Kset::info)
  int32_t *krun = nullptr;    // nruns*2 device (Kset::runs)
  int32_t *kcol = nullptr;    // ncols_pad*4 device (Kset::cols)
  int32_t *atom_order = nullptr;  // n device: atoms in compact spatial tiles (real-space sums)
  // the atoms' z-planes when there are at most kMaxPlanes of them (else
  // nplanes = 0): z / L_z per plane, and tiles of kPlaneTile atoms of one
  // plane each (atom -1 pads a plane's last tile)
  int nplanes = 0;
  int64_t plane_ntiles = 0;
  double *plane_uz = nullptr;
  int32_t *plane_tile = nullptr;  // plane_ntiles: plane of the tile
  int32_t *plane_atom = nullptr;  // plane_ntiles * kPlaneTile
  double *E64 = nullptr;      // ld*ld device (rows >= n and cols >= n are zero)
  float *E32 = nullptr;
  uint16_t *E16 = nullptr;
  double *dinv = nullptr;     // ld: 1/E_ii (zero in padding)
  double *dprime = nullptr;   // ld: E^-1 1
  double *dvec = nullptr;     // ld: d' / C_ele
  double c_ele = 0;
  bool dprime_ready = false;
  double *qchi = nullptr;     // ld: neutral charges without electrolyte (warm start)
  double *erfc_tab = nullptr; // piecewise polynomial of erfc (cpm::kErfcTab doubles)
  double *S = nullptr;        // ld*ld: S = E^-1 (I - 1 d^T) of the MI path (Eq. 33), or null
  bool qchi_ready = false;
  double *rhs_S = nullptr;    // structure-factor scratch
  int64_t rhs_S_elems = 0;
  std::vector<double> pos_host;   // n*3 wrapped positions (host copy)
  cpm::Workspace ws;
  cpm::Mlp mlp;
  cpm::Precond pc;
  cpm::Coarse cz;
  cpm::Gcd gcd;
  std::vector<double> width_host;   // n Gaussian inverse widths (host copy)
  mutable cpm::Profile prof;   // timing only: recorded from const paths too
  hipEvent_t warm_ev[2] = {nullptr, nullptr};   // brackets of the warm start (its time)
  // per-call scratch, grown on demand and kept: the warm start and its
  // residual (2 f n), E q0 of its neutral shift (f n), per-frame means (f),
  // and small values of one call (per-frame errors, flags, loss history,
  // the right-hand side of q_chi)
  cpm::DevBuf buf_warm, buf_eq, buf_mean, buf_aux;
  int64_t device_bytes = 0;
};

namespace cpm {

// device pointer to at least `bytes` bytes of b, grown (after the stream has
// drained, so no enqueued work still reads the old buffer) when too small;
// nullptr with CPM_ENOMEM in *rc when the allocation fails
void *grow_buf(cpm_system *s, DevBuf &b, size_t bytes, cpm_status *rc);

// ---- assembly.hip
// A (ld rows, kdim = 2 * k-vectors-per-chunk columns, column-blocked by 16):
// sqrt(w) cos / sin of the chunk's k-vectors k0 .. k0 + kc - 1
hipError_t launch_phase_matrix(hipStream_t st, const double *pos, int64_t n, int64_t ld,
                               const double box[3], const int32_t *kn, const double *kw,
                               int64_t k0, int64_t kc, int64_t kdim, double *A);
// lower-triangular tile list of the contraction (pairs ti >= tj, in the
// order the kernel walks them) for T = ld / 128 tile rows
std::vector<int32_t> syrk_tile_order(int64_t T);
hipError_t launch_syrk_lower(hipStream_t st, const double *A, int64_t kdim,
                             const int32_t *tiles, int64_t ld, double *E, int64_t lde,
                             bool accumulate, hipEvent_t ev_start, hipEvent_t ev_stop);
// width: the Gaussian self-energy of the diagonal; rs_width: the screening
// of the real-space pair terms (the same array unless the point-charge
// simplification sets it to +inf)
hipError_t launch_finalize(hipStream_t st, const double *pos, const double *width,
                           const double *rs_width, int64_t n, int64_t ld, const double box[3],
                           double beta, double rcut, bool slab, double *E64, float *E32,
                           uint16_t *E16);

// ---- rhs.hip
// erfc on [0, 6.5): kErfcIntervals intervals of width 1/8, kErfcTerms
// Taylor coefficients each (about the midpoint, in units of the width)
constexpr int kErfcIntervals = 52;
constexpr int kErfcTerms = 12;
constexpr int kErfcTab = kErfcIntervals * kErfcTerms;
void erfc_table(double *out);
int64_t rhs_scratch_elems(const cpm_system *s, int64_t m, int64_t f);
// scratch of the plan limited to limit doubles (fewer partial buffers), and
// the static scratch of cpm_rhs_noalloc: its size and this device's address
int64_t rhs_scratch_elems_capped(const cpm_system *s, int64_t m, int64_t f, int64_t limit);
int64_t rhs_static_scratch_elems();
hipError_t rhs_static_scratch(double **ptr);
// limit > 0: the plan whose scratch fits limit doubles (as sized by
// rhs_scratch_elems_capped)
hipError_t launch_rhs(hipStream_t st, const cpm_system *s, const double *ion_pos,
                      const double *ion_q, int64_t m, int64_t f, const double *chi,
                      double *S, double *b_out, double *qsol_out, int64_t limit = 0);

// ---- cg.hip
void release_workspace(cpm_system *s);
// q_out = E^-1 b for f frames; with project the two-step neutralisation of
// Eq. 35 follows (qsol_dev required), without it q_out is the raw solution
// and qsol_dev is not read
// r0_dev (with x0_dev, may be null): b - E x0 already known (FP64)
cpm_status solve_block(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                       const cpm_solve_opts &o, double *q_out_dev, cpm_solve_info *info,
                       const double *x0_dev, bool project = true, const double *r0_dev = nullptr);
cpm_status solve_dprime(cpm_system *s, double tol, int max_iter);
cpm_status matvec_cols(cpm_system *s, int precision, const double *p_dev, int64_t f,
                       double *v_dev);
// V = M P with an ld x ld FP64 matrix M instead of E (precision CPM_PREC_F64)
cpm_status matvec_cols_with(cpm_system *s, int precision, const double *M64, const double *p_dev,
                            int64_t f, double *v_dev);
// z = P r (PCG-DC preconditioner) for f vectors (f, n), the CG's own apply kernel
cpm_status precond_cols(cpm_system *s, const double *r_dev, int64_t f, double *z_dev);
// slices of the coarse Z^T-side product for mp padded patches
void coarse_slices(int64_t ld, int64_t mp, int &ks, int64_t &kslice);
hipError_t launch_diag_inverse(hipStream_t st, const double *E, int64_t n, int64_t ld,
                               double *dinv);

// ---- api.hip
// checks *opts against the system (tolerance, iterations, precision stored,
// preconditioner built) and fills defaults; the warm start is not checked
cpm_status check_solve_opts(const cpm_system *s, const cpm_solve_opts *opts, cpm_solve_opts *o);

// ---- gcd.hip
void free_gcd(Gcd &g);

// ---- mlp.hip
// x0 (f, n): the start; r0 (f, n) or null: its FP64 residual b - E x0
cpm_status warm_start_impl(cpm_system *s, bool use_mlp, const double *b, const double *qsol,
                           int64_t f, double *x0, double *r0 = nullptr);
hipError_t launch_mlp_forward(hipStream_t st, const float *params, const float *feat,
                              int64_t rows, float *y);

}  // namespace cpm

#define CPM_HIP_CHECK(expr)                                                   \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      cpm::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));     \
      return CPM_EDEVICE;                                                     \
    }                                                                         \
  } while (0)
