// Block conjugate gradients on the dense Ewald matrix and the two-step
// electroneutrality post-treatment (Sec. III.A, Eq. 31-35; Sec. III.B.2).
//
// Up to 64 right-hand sides run as independent CG recurrences that share
// one matrix product V = E P per iteration (E streamed once for all of
// them). Vectors are stored frame-major: column c of a block is a
// contiguous array of ld values; rows >= n stay zero (E's padded columns
// are zero, and 0 * NaN would not be).
//
// One Jacobi-preconditioned iteration is three kernels:
//   block product        v = E p as k-slice partials (16 columns: the
//     row-split kernel, waves over rows, the P slice in LDS; 32..64 columns
//     of an FP64 E: the streamed-P FP64 kernel; 32..64 columns of an FP32 /
//     BF16 E: the split-bf16 kernel). MFMA blocks of 16x16
//     (v_mfma_f64_16x16x4f64 for FP64 E, v_mfma_f32_16x16x4f32 for FP32 and
//     BF16 E, products accumulated in FP32). Lane l supplies A[l % 16][l / 16]
//     and B[l / 16][l % 16]; the k slots of the MFMA are mapped to 32
//     contiguous bytes of an E row per lane, so E and P are read with wide,
//     coalesced loads. Each workgroup also reduces its share of p.v.
//   cg_update_kernel     v = sum of the slices; alpha = r.z / p.v;
//                        x += alpha p; r -= alpha v;
//                        z = M^-1 r (Jacobi, M = diag E); partial r.r, r.z.
//   cg_direction_kernel  beta = r'.z' / r.z; p = z + beta p.
// With PCG-DC (Sec. III.B.2) the update is cg_update_pc_kernel (it also
// writes the row-interleaved copy of r) and precond_kernel computes z = P r
// and the partial r.r, r.z before the direction kernel.
// All dots are FP64 and reduced in a fixed order (bitwise reproducible).
//
// Control runs on the device: every check_every iterations a one-wave
// kernel decides per column whether the true residual is due (converged
// recursively, reliable-update point, or iteration limit); the FP64
// residual kernels that follow are gated by that decision and exit at once
// when it is negative, and a second control kernel retires converged
// columns. The host only enqueues batches ahead of the GPU and reads a
// status word one batch behind, so the queue never drains while the solve
// runs; kernels of a batch enqueued after the last column converged exit
// at once.
//
// Precision: x, r, z are FP64 in every mode. FP64 mode streams the FP64 E.
// FP32 / BF16 modes stream the rounded E (p and v in FP32) and use true-
// residual updates: whenever the recursive residual has fallen by the factor
// inner_tol below the last true residual (or meets the tolerance), r is
// replaced by the true FP64 residual b - E x computed on the FP64 E. FP32
// continues with the same search direction (a reliable update); BF16
// restarts it from the new residual, i.e. iterative refinement with an
// inner CG on the BF16 matrix. Convergence is always decided on the true
// FP64 residual.
#include "cpm_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>

namespace cpm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int RED_THREADS = 256;
constexpr int MAX_COLS = 64;
constexpr int64_t CHUNK = 256;    // rows per block of the vector kernels
// partial sums that the workgroups of one vector kernel may re-reduce in
// total before a separate reduction launch is cheaper
constexpr int64_t kRedLoads = (int64_t)1 << 22;

// scalar fields (struct of arrays, cols entries each): r.z (two slots), r.r,
// |b|^2, active flag, last true residual norm, relative true residual,
// iterations, initial relative residual, start-discarded flag
enum {
  S_RZ0 = 0, S_RZ1 = 1, S_RR = 2, S_BN2 = 3, S_ACT = 4, S_RT = 5, S_RES = 6, S_IT = 7,
  S_INIT = 8, S_FB = 9, S_HOLD0 = 10, S_HOLD1 = 11, S_RST = 12, S_RPREV = 13,
  S_EN = 14,   // x0 . (b + r0) of a warm start: > 0 iff it lowers the energy
  S_NFIELDS = 15
};
// status words (ints): breakdown flag and column, debug doubles (ints 2..5),
// true residual due, any column active, non-finite residual seen, number of
// true-residual updates, a start was discarded, largest recursive residual
enum {
  F_BREAK = 0, F_COL = 1, F_NEED = 6, F_ANY = 7, F_NONFINITE = 8, F_UPDATES = 9, F_FELLBACK = 10,
  F_RMAX = 12,   // (double, words 12-13) largest relative residual of the active columns at the
                 // last check: the true one when the check took it, else the recursive one
  F_NWORDS = 16
};

template <typename T> struct Mv;
template <> struct Mv<double> {
  using VT = double;
  using Acc = d4;
  static constexpr int VEC = 4;
  __device__ static inline Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  struct Raw { double v[VEC]; };
  __device__ static inline void load(const double *p, Raw &o) {
    const double4 v = *reinterpret_cast<const double4 *>(p);
    o.v[0] = v.x; o.v[1] = v.y; o.v[2] = v.z; o.v[3] = v.w;
  }
  __device__ static inline double elem(const Raw &o, int t) { return o.v[t]; }
  // output row of register v in lane group g: D[4v + g][lane % 16]
  __device__ static inline int out_row(int g, int v) { return 4 * v + g; }
};
template <> struct Mv<float> {
  using VT = float;
  using Acc = f4;
  static constexpr int VEC = 8;
  __device__ static inline Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  struct Raw { float v[VEC]; };
  __device__ static inline void load(const float *p, Raw &o) {
    const float4 v0 = *reinterpret_cast<const float4 *>(p);
    const float4 v1 = *reinterpret_cast<const float4 *>(p + 4);
    o.v[0] = v0.x; o.v[1] = v0.y; o.v[2] = v0.z; o.v[3] = v0.w;
    o.v[4] = v1.x; o.v[5] = v1.y; o.v[6] = v1.z; o.v[7] = v1.w;
  }
  __device__ static inline float elem(const Raw &o, int t) { return o.v[t]; }
  // output row of register v in lane group g: D[4g + v][lane % 16]
  __device__ static inline int out_row(int g, int v) { return 4 * g + v; }
};
template <> struct Mv<uint16_t> {   // bf16 storage, widened to FP32
  using VT = float;
  using Acc = f4;
  static constexpr int VEC = 16;
  __device__ static inline Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // raw bf16 pairs stay packed in registers until the MFMA needs them
  struct Raw { uint32_t w[8]; };
  __device__ static inline void load(const uint16_t *p, Raw &o) {
    const uint4 v0 = *reinterpret_cast<const uint4 *>(p);
    const uint4 v1 = *reinterpret_cast<const uint4 *>(p + 8);
    o.w[0] = v0.x; o.w[1] = v0.y; o.w[2] = v0.z; o.w[3] = v0.w;
    o.w[4] = v1.x; o.w[5] = v1.y; o.w[6] = v1.z; o.w[7] = v1.w;
  }
  __device__ static inline float elem(const Raw &o, int t) {
    const uint32_t w = o.w[t >> 1];
    return __uint_as_float((t & 1) ? (w & 0xffff0000u) : (w << 16));
  }
  __device__ static inline int out_row(int g, int v) { return 4 * g + v; }
};

template <typename VT, int VEC> __device__ inline void load_vec(const VT *p, VT (&o)[VEC]) {
#pragma unroll
  for (int q = 0; q < VEC; q += 4) {
    if constexpr (sizeof(VT) == 8) {
      const double4 v = *reinterpret_cast<const double4 *>(p + q);
      o[q] = v.x; o[q + 1] = v.y; o[q + 2] = v.z; o[q + 3] = v.w;
    } else {
      const float4 v = *reinterpret_cast<const float4 *>(p + q);
      o[q] = v.x; o[q + 1] = v.y; o[q + 2] = v.z; o[q + 3] = v.w;
    }
  }
}

// Block product for 16 columns with the rows split over the waves: grid
// (row blocks of MR_WAVES x 16 rows, k slices). The workgroup first copies
// its slice of P (16 columns x kslice) into LDS; each wave then streams its
// own 16 rows of E over the slice (U load stages in flight) and takes the B
// operands from LDS, so P is read from L2 once per workgroup and no
// reduction across waves is needed:
//   part[s][c][row] = sum_{k in slice s} E[row][k] P[c][k]
//   pv_part[s][workgroup][c] = sum over the workgroup's rows of P[c][row] part[s][c][row]
constexpr int MR_WAVES = 8;
extern __shared__ double mv_lds[];

template <typename T> constexpr int mr_pad() { return 4; }   // keeps 32-byte alignment of LDS rows
// longest k slice whose P copy fits 64 KB of LDS (a multiple of the k step)
template <typename T> constexpr int64_t mr_kmax() {
  constexpr int64_t kb = 4 * Mv<T>::VEC;
  return ((65536 / (16 * (int64_t)sizeof(typename Mv<T>::VT))) - mr_pad<T>()) / kb * kb;
}
// the P copy plus the static p.v buffer stay far inside the 160 KB of LDS a
// workgroup can hold (a launch asking for more than exists is not rejected
// reliably)
template <typename T> constexpr bool mr_lds_fits() {
  return sizeof(typename Mv<T>::VT) * 16 * (mr_kmax<T>() + mr_pad<T>()) +
             sizeof(double) * MR_WAVES * 16 <= 65536 + 4096;
}
static_assert(mr_lds_fits<double>() && mr_lds_fits<float>() && mr_lds_fits<uint16_t>(),
              "LDS of the 16-column product");

template <typename T>
__global__ __launch_bounds__(64 * MR_WAVES) void block_matvec_rows_kernel(
    const T *__restrict__ E, int64_t ld, const typename Mv<T>::VT *__restrict__ P,
    typename Mv<T>::VT *__restrict__ part, int64_t kslice, int64_t split_stride,
    double *__restrict__ pv_part, const int *__restrict__ gate, int *__restrict__ mark) {
  using M = Mv<T>;
  using VT = typename M::VT;
  using Acc = typename M::Acc;
  constexpr int VEC = M::VEC;
  constexpr int KB = 4 * VEC;
  constexpr int U = 4;
  const bool first = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  if (gate != nullptr && *gate == 0) {
    if (mark != nullptr && first) *mark = 0;
    return;
  }
  if (mark != nullptr && first) *mark = 1;
  VT *ps = reinterpret_cast<VT *>(mv_lds);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t wtile = (int64_t)blockIdx.x * MR_WAVES + wave;
  const int64_t r0 = wtile * 16;
  const int64_t sl = blockIdx.y;
  const int64_t k0 = sl * kslice;
  const int64_t kn = min(kslice, ld - k0);   // a multiple of KB
  const int64_t pstride = kslice + mr_pad<T>();
  const int64_t nsteps = kn / KB;
  const T *erow = E + (r0 + lr) * ld + k0 + lg * VEC;
  // E ring: slot u holds step st0 + u. The loads of the prologue and of the
  // main loop are unconditional (the prologue's clamped to the last step) so
  // that the loop body is one straight path: the compiler then waits only
  // for the oldest slot (vmcnt 2 (U - 1)) instead of draining every load in
  // flight at the top of each iteration.
  typename M::Raw ea[U];
#pragma unroll
  for (int u = 0; u < U; ++u) M::load(erow + min<int64_t>(u, nsteps - 1) * KB, ea[u]);
  // P of the wave's own rows for the p.v partial, loaded now so that the
  // loads are complete when the epilogue needs them
  const VT *pc = P + (int64_t)lr * ld + r0;
  VT pown[4];
  if (pv_part != nullptr)
#pragma unroll
    for (int v = 0; v < 4; ++v) pown[v] = pc[M::out_row(lg, v)];
  // P slice into LDS (16-byte pieces; kn / PV < 2^31)
  constexpr int PV = 16 / sizeof(VT);
  const int q = (int)(kn / PV);
  for (int t = threadIdx.x; t < 16 * q; t += 64 * MR_WAVES) {
    const int c = t / q, kk = (t - c * q) * PV;
    *reinterpret_cast<uint4 *>(ps + c * pstride + kk) =
        *reinterpret_cast<const uint4 *>(P + c * ld + k0 + kk);
  }
  __syncthreads();
  Acc acc[2] = {Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}};
  const VT *pl = ps + lr * pstride + lg * VEC;
  auto step = [&](const typename M::Raw &e, int64_t st) {
    VT pb[VEC];
    load_vec<VT, VEC>(pl + st * KB, pb);
#pragma unroll
    for (int t = 0; t < VEC; ++t) acc[t & 1] = M::mfma(M::elem(e, t), pb[t], acc[t & 1]);
  };
  int64_t st0 = 0;
  for (; st0 + 2 * U <= nsteps; st0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      step(ea[u], st0 + u);
      M::load(erow + (st0 + u + U) * KB, ea[u]);
      // keep the refill here: scheduled after the last slot, all U refills
      // would go out together and the ring would drain every iteration
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the last U .. 2U - 1 steps (fewer when nsteps < U)
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (st0 + u < nsteps) {
      step(ea[u], st0 + u);
      if (st0 + u + U < nsteps) M::load(erow + (st0 + u + U) * KB, ea[u]);
    }
  st0 += U;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (st0 + u < nsteps) step(ea[u], st0 + u);
  // lane (lr, lg) holds rows out_row(lg, v) of column lr
  VT *out = part + sl * split_stride + (int64_t)lr * ld + r0;
  VT sv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) sv[v] = acc[0][v] + acc[1][v];
#pragma unroll
  for (int v = 0; v < 4; ++v) out[M::out_row(lg, v)] = sv[v];
  if (pv_part == nullptr) return;
  double pv = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) pv += (double)pown[v] * (double)sv[v];
  pv += __shfl_xor(pv, 16, 64);
  pv += __shfl_xor(pv, 32, 64);
  __shared__ double pvs[MR_WAVES][16];
  if (lg == 0) pvs[wave][lr] = pv;
  __syncthreads();
  if (threadIdx.x < 16) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < MR_WAVES; ++w) t += pvs[w][threadIdx.x];
    pv_part[(sl * gridDim.x + blockIdx.x) * 16 + threadIdx.x] = t;
  }
}

// ---- FP64 block product for 32..64 columns: P streamed through LDS
//
// With 64 columns the FP64 product does 128 flops per E entry and is bound
// by the FP64 matrix cores; what has to be avoided is re-reading P for every
// 16-row tile. Workgroup = 4 waves x F64_RW row tiles of 16 rows (F64_ROWS
// rows) and one k slice; per chunk of F64_KC columns of E the workgroup
// copies the matching 16 NG x F64_KC block of P into LDS once (double
// buffered, one barrier per chunk) and every wave takes its B operands from
// there while its own E rows stream from HBM (F64_U chunks in flight).
// v_mfma_f64_16x16x4f64: lane (lr, lg) supplies A = E[row lr][k 4 lg + t]
// and B = P[column lr][k 4 lg + t] for t = 0..3 of each 16-k step.
constexpr int F64_RW = 2;
constexpr int F64_ROWS = 4 * 16 * F64_RW;   // rows per workgroup
constexpr int F64_KC = 32;                  // k per chunk
constexpr int F64_PR = F64_KC + 4;          // LDS row length of the P chunk (doubles)
constexpr int F64_U = 2;                    // E chunks in flight per wave

template <int NG>
__global__ __launch_bounds__(256) void block_matvec_f64s_kernel(
    const double *__restrict__ E, int64_t ld, const double *__restrict__ P,
    double *__restrict__ part, int64_t kslice, int64_t split_stride,
    double *__restrict__ pv_part, const int *__restrict__ gate, int *__restrict__ mark) {
  constexpr int COLS = 16 * NG;
  __shared__ __align__(16) double ps[2][COLS][F64_PR];
  __shared__ double pvs[4][COLS];
  const bool first = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  if (gate != nullptr && *gate == 0) {
    if (mark != nullptr && first) *mark = 0;
    return;
  }
  if (mark != nullptr && first) *mark = 1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t tile = blockIdx.x, sl = blockIdx.y;
  const int64_t row0 = tile * F64_ROWS + wave * 16 * F64_RW;
  const int64_t kbeg = sl * kslice;
  const int64_t kend = min(ld, kbeg + kslice);
  const int nch = (int)((kend - kbeg) / F64_KC);
  // P loader: thread -> (column tid / 4, 8 consecutive k); 64 columns x 32 k per chunk
  const int pcol = tid >> 2, pk = (tid & 3) * 8;
  const bool ploader = pcol < COLS;
  const double *pbase = P + (int64_t)(ploader ? pcol : 0) * ld + kbeg + pk;
  // E: row tile a, chunk u holds k = 16 s + 4 lg + t for s = 0, 1
  // row tile a starts erow_stride * a after erow0
  const double *erow0 = E + (row0 + lr) * ld + kbeg + lg * 4;
  const int64_t erow_stride = 16 * ld;
  double4 ring[F64_U][F64_RW][2];
#pragma unroll
  for (int u = 0; u < F64_U; ++u)
    if (u < nch)
#pragma unroll
      for (int a = 0; a < F64_RW; ++a)
#pragma unroll
        for (int st = 0; st < 2; ++st)
          ring[u][a][st] = *reinterpret_cast<const double4 *>(erow0 + a * erow_stride + u * F64_KC + st * 16);
  double4 pn0 = make_double4(0, 0, 0, 0), pn1 = pn0;
  if (nch > 0 && ploader) {
    pn0 = *reinterpret_cast<const double4 *>(pbase);
    pn1 = *reinterpret_cast<const double4 *>(pbase + 4);
    *reinterpret_cast<double4 *>(&ps[0][pcol][pk]) = pn0;
    *reinterpret_cast<double4 *>(&ps[0][pcol][pk + 4]) = pn1;
  }
  __syncthreads();
  d4 acc[F64_RW][NG];
#pragma unroll
  for (int a = 0; a < F64_RW; ++a)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[a][g] = d4{0, 0, 0, 0};
  // one chunk with E from ring slot U (a compile-time index, so that the
  // ring stays in registers)
  auto chunk = [&](auto slot, int ch) {
    constexpr int U = decltype(slot)::value;
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more && ploader) {
      pn0 = *reinterpret_cast<const double4 *>(pbase + (int64_t)(ch + 1) * F64_KC);
      pn1 = *reinterpret_cast<const double4 *>(pbase + (int64_t)(ch + 1) * F64_KC + 4);
    }
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const double4 b = *reinterpret_cast<const double4 *>(&ps[buf][g * 16 + lr][st * 16 + lg * 4]);
#pragma unroll
        for (int a = 0; a < F64_RW; ++a) {
          const double4 e = ring[U][a][st];
          acc[a][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.x, b.x, acc[a][g], 0, 0, 0);
          acc[a][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.y, b.y, acc[a][g], 0, 0, 0);
          acc[a][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.z, b.z, acc[a][g], 0, 0, 0);
          acc[a][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(e.w, b.w, acc[a][g], 0, 0, 0);
        }
      }
    if (ch + F64_U < nch) {
#pragma unroll
      for (int a = 0; a < F64_RW; ++a)
#pragma unroll
        for (int st = 0; st < 2; ++st)
          ring[U][a][st] =
              *reinterpret_cast<const double4 *>(erow0 + a * erow_stride + (int64_t)(ch + F64_U) * F64_KC + st * 16);
    }
    if (more && ploader) {
      *reinterpret_cast<double4 *>(&ps[buf ^ 1][pcol][pk]) = pn0;
      *reinterpret_cast<double4 *>(&ps[buf ^ 1][pcol][pk + 4]) = pn1;
    }
    __syncthreads();
  };
  static_assert(F64_U == 2, "two ring slots");
  for (int ch0 = 0; ch0 < nch; ch0 += F64_U) {
    chunk(std::integral_constant<int, 0>(), ch0);
    if (ch0 + 1 < nch) chunk(std::integral_constant<int, 1>(), ch0 + 1);
  }
  // lane (lr, lg) holds rows 4 v + lg of column lr of each tile
  double *out = part + sl * split_stride;
  double pv[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    pv[g] = 0.0;
    const int64_t c = g * 16 + lr;
#pragma unroll
    for (int a = 0; a < F64_RW; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + a * 16 + 4 * v + lg;
        out[c * ld + row] = acc[a][g][v];
        if (pv_part) pv[g] += P[c * ld + row] * acc[a][g][v];
      }
  }
  if (pv_part == nullptr) return;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    pv[g] += __shfl_xor(pv[g], 16, 64);
    pv[g] += __shfl_xor(pv[g], 32, 64);
    if (lg == 0) pvs[wave][g * 16 + lr] = pv[g];
  }
  __syncthreads();
  if (tid < COLS)
    pv_part[(sl * gridDim.x + tile) * COLS + tid] =
        ((pvs[0][tid] + pvs[1][tid]) + pvs[2][tid]) + pvs[3][tid];
}

// ---- block product on bf16 matrix cores (32..64 columns, FP32 or BF16 E)
//
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] for j = 0..7 and receives D[4 (l / 16) + v][l % 16]
// in register v. An FP32 value x is split exactly into three bf16 parts
// x = x0 + x1 + x2 (round to nearest, then the remainders, each exact in
// FP32); the product of an FP32 E and an FP32 P keeps the six part products
// whose orders add up to at most 2, which leaves an error of the order of
// FP32 rounding. A BF16 E is one part (three products with the parts of P).
// Workgroup: 4 waves x SP_RW row tiles of 16 rows (SP_ROWS rows) and one k
// slice; per chunk of SP_KC columns of E the workgroup splits the matching
// P chunk into LDS once (double buffered), each wave streams its own E rows.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int SP_RW = 2;                     // row tiles per wave
constexpr int SP_ROWS = 4 * 16 * SP_RW;      // rows per workgroup
constexpr int SP_KC = 32;                    // k per chunk (one MFMA depth)
constexpr int SP_PR = SP_KC + 8;             // LDS row length of a P part (bf16, padded)
// E chunks in flight per wave: 2 up to 32 columns (three waves per SIMD fit
// beside the FP64 sums: 12.3 ms against 14.4 with 4 at N = 131072), 4 for 64
template <int NG> constexpr int sp_ring() { return NG <= 2 ? 2 : 4; }

__device__ inline uint32_t cvt_bf16x2(float a, float b) {
  const f2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// 8 FP32 values -> three bf16 parts (4 packed words each), x = x0 + x1 + x2
__device__ inline void split3(const float (&x)[8], uint32_t (&w0)[4], uint32_t (&w1)[4],
                              uint32_t (&w2)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float a = x[2 * j], b = x[2 * j + 1];
    w0[j] = cvt_bf16x2(a, b);
    const float ra = a - bf16_lo(w0[j]), rb = b - bf16_hi(w0[j]);
    w1[j] = cvt_bf16x2(ra, rb);
    const float sa = ra - bf16_lo(w1[j]), sb = rb - bf16_hi(w1[j]);
    w2[j] = cvt_bf16x2(sa, sb);
  }
}

__device__ inline bf16x8 as_bf16x8(const uint32_t (&w)[4]) {
  const uint4 u = make_uint4(w[0], w[1], w[2], w[3]);
  return __builtin_bit_cast(bf16x8, u);
}
__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ inline f4 mfma_bf16(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename T> struct Sp;
template <> struct Sp<float> {
  static constexpr int EP = 3;
  struct Raw { float v[8]; };
  __device__ static inline void load(const float *p, Raw &o) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    o.v[0] = a.x; o.v[1] = a.y; o.v[2] = a.z; o.v[3] = a.w;
    o.v[4] = b.x; o.v[5] = b.y; o.v[6] = b.z; o.v[7] = b.w;
  }
  // acc += E P over one chunk for one 16 x 16 block, small products first
  __device__ static inline f4 madd(const Raw &e, const bf16x8 (&pp)[3], f4 acc) {
    uint32_t w0[4], w1[4], w2[4];
    split3(e.v, w0, w1, w2);
    const bf16x8 e0 = as_bf16x8(w0), e1 = as_bf16x8(w1), e2 = as_bf16x8(w2);
    acc = mfma_bf16(e2, pp[0], acc);
    acc = mfma_bf16(e1, pp[1], acc);
    acc = mfma_bf16(e0, pp[2], acc);
    acc = mfma_bf16(e1, pp[0], acc);
    acc = mfma_bf16(e0, pp[1], acc);
    return mfma_bf16(e0, pp[0], acc);
  }
};
template <> struct Sp<uint16_t> {
  static constexpr int EP = 1;
  struct Raw { uint4 w; };
  __device__ static inline void load(const uint16_t *p, Raw &o) {
    o.w = *reinterpret_cast<const uint4 *>(p);
  }
  __device__ static inline f4 madd(const Raw &e, const bf16x8 (&pp)[3], f4 acc) {
    const bf16x8 a = as_bf16x8(e.w);
    acc = mfma_bf16(a, pp[2], acc);
    acc = mfma_bf16(a, pp[1], acc);
    return mfma_bf16(a, pp[0], acc);
  }
};

template <typename T, int NG>
__global__ __launch_bounds__(256) void block_matvec_split_kernel(
    const T *__restrict__ E, int64_t ld, const float *__restrict__ P, float *__restrict__ part,
    int64_t kslice, int64_t split_stride, double *__restrict__ pv_part,
    const int *__restrict__ gate, int *__restrict__ mark) {
  using SP = Sp<T>;
  constexpr int COLS = 16 * NG;
  constexpr int SP_U = sp_ring<NG>();
  // one LDS buffer: the P parts during the k loop, the output tile after it
  constexpr int PS_BYTES = 2 * 3 * COLS * SP_PR * 2;
  constexpr int OUT_BYTES = COLS * (SP_ROWS + 1) * 4;
  __shared__ __align__(16) unsigned char smem[PS_BYTES > OUT_BYTES ? PS_BYTES : OUT_BYTES];
  auto ps = reinterpret_cast<uint16_t(*)[3][COLS][SP_PR]>(smem);
  auto outs = reinterpret_cast<float(*)[SP_ROWS + 1]>(smem);

  const bool first = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  if (gate != nullptr && *gate == 0) {
    if (mark != nullptr && first) *mark = 0;
    return;
  }
  if (mark != nullptr && first) *mark = 1;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t tile = blockIdx.x, sl = blockIdx.y;
  const int64_t row0 = tile * SP_ROWS;
  const int64_t kbeg = sl * kslice;
  const int64_t kend = min(ld, kbeg + kslice);
  const int nch = (int)((kend - kbeg) / SP_KC);

  // P loader: thread -> (column, 8 consecutive k)
  const int pcol = tid >> 2, pk = (tid & 3) * 8;
  const bool ploader = pcol < COLS;
  const float *pbase = P + (int64_t)(ploader ? pcol : 0) * ld + pk;
  auto load_p = [&](int64_t k0, float (&x)[8]) {
    const float4 a = *reinterpret_cast<const float4 *>(pbase + k0);
    const float4 b = *reinterpret_cast<const float4 *>(pbase + k0 + 4);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
  };
  auto store_p = [&](int buf, const float (&x)[8]) {
    uint32_t w0[4], w1[4], w2[4];
    split3(x, w0, w1, w2);
    *reinterpret_cast<uint4 *>(&ps[buf][0][pcol][pk]) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    *reinterpret_cast<uint4 *>(&ps[buf][1][pcol][pk]) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    *reinterpret_cast<uint4 *>(&ps[buf][2][pcol][pk]) = make_uint4(w2[0], w2[1], w2[2], w2[3]);
  };

  const T *erow[SP_RW];
#pragma unroll
  for (int a = 0; a < SP_RW; ++a) erow[a] = E + (row0 + wave * 16 * SP_RW + a * 16 + lr) * ld + kbeg + lg * 8;

  // the matrix cores accumulate in FP32 over SP_U chunks, then the sums move
  // to FP64 registers: a running FP32 sum over a k slice of ~40000 would
  // carry ~1e-6 of |v| in rounding (slower CG), the flushed one ~1e-7
  f4 acc[SP_RW][NG];
  d4 accd[SP_RW][NG];
#pragma unroll
  for (int a = 0; a < SP_RW; ++a)
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      acc[a][g] = f4{0, 0, 0, 0};
      accd[a][g] = d4{0.0, 0.0, 0.0, 0.0};
    }

  typename SP::Raw ring[SP_U][SP_RW];
#pragma unroll
  for (int u = 0; u < SP_U; ++u)
    if (u < nch) {
#pragma unroll
      for (int a = 0; a < SP_RW; ++a) SP::load(erow[a] + u * SP_KC, ring[u][a]);
    }
  if (nch > 0 && ploader) {
    float x[8];
    load_p(kbeg, x);
    store_p(0, x);
  }
  __syncthreads();

  for (int ch0 = 0; ch0 < nch; ch0 += SP_U) {
#pragma unroll
    for (int u = 0; u < SP_U; ++u) {
      const int ch = ch0 + u;
      if (ch < nch) {
        const int buf = u & 1;   // SP_U is even, so buf == ch & 1
        float xn[8];
        const bool more = ch + 1 < nch;
        if (more && ploader) load_p(kbeg + (int64_t)(ch + 1) * SP_KC, xn);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          bf16x8 pp[3];
#pragma unroll
          for (int q = 0; q < 3; ++q)
            pp[q] = as_bf16x8(*reinterpret_cast<const uint4 *>(&ps[buf][q][g * 16 + lr][lg * 8]));
#pragma unroll
          for (int a = 0; a < SP_RW; ++a) acc[a][g] = SP::madd(ring[u][a], pp, acc[a][g]);
        }
        if (ch + SP_U < nch) {
#pragma unroll
          for (int a = 0; a < SP_RW; ++a) SP::load(erow[a] + (int64_t)(ch + SP_U) * SP_KC, ring[u][a]);
        }
        if (more && ploader) store_p(buf ^ 1, xn);
        __syncthreads();
      }
    }
#pragma unroll
    for (int a = 0; a < SP_RW; ++a)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[a][g][v] += (double)acc[a][g][v];
        acc[a][g] = f4{0, 0, 0, 0};
      }
  }

  // this workgroup's partial product through LDS: coalesced rows per column
#pragma unroll
  for (int a = 0; a < SP_RW; ++a)
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        outs[g * 16 + lr][wave * 16 * SP_RW + a * 16 + 4 * lg + v] = (float)accd[a][g][v];
  __syncthreads();
  float *out = part + sl * split_stride;
  for (int c = tid / SP_ROWS; c < COLS; c += 256 / SP_ROWS) {
    const int r = tid % SP_ROWS;
    out[(int64_t)c * ld + row0 + r] = outs[c][r];
  }
  if (pv_part) {
    // p.v share of the workgroup's rows: 4 threads per column, fixed order
    constexpr int RPT = SP_ROWS / 4;
    if (tid < COLS * 4) {
      const int c = tid >> 2, r0 = (tid & 3) * RPT;
      const float *pc = P + (int64_t)c * ld + row0 + r0;
      double s = 0.0;
      for (int r = 0; r < RPT; ++r) s += (double)pc[r] * (double)outs[c][r0 + r];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      if ((tid & 3) == 0) pv_part[(sl * gridDim.x + tile) * COLS + c] = s;
    }
  }
}

// Sum over the block (RED_THREADS = 4 waves): butterfly within each wave,
// then the four wave sums in a fixed order; every thread gets the result.
// red must hold 4 doubles and not be reused by the caller before the next
// __syncthreads.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double *red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// sum of v[b * stride + off] over b = b0, b0 + step, ... < nb in a fixed
// order, sixteen loads in flight (clamped indices keep the loads unconditional)
__device__ inline double strided_sum(const double *__restrict__ v, int nb, int b0, int step,
                                     int64_t stride, int64_t off) {
  double s = 0.0;
  for (int b = b0; b < nb; b += 16 * step) {
    double t[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int bb = b + m * step;
      t[m] = v[(int64_t)(bb < nb ? bb : nb - 1) * stride + off];
      if (bb >= nb) t[m] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) s += t[m];
  }
  return s;
}

// sum of the k-slice partial products of element idx (fixed order)
template <typename VT>
__device__ inline double sum_slices(const VT *__restrict__ part, int slices, int64_t stride,
                                    int64_t idx) {
  double v = 0.0;
  for (int s0 = 0; s0 < slices; s0 += 8) {
    VT t[8];   // eight loads in flight; clamped indices keep them unconditional
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int sl = s0 + m;
      t[m] = part[(int64_t)(sl < slices ? sl : slices - 1) * stride + idx];
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (s0 + m < slices) v += (double)t[m];
  }
  return v;
}

// r = b - E x (k-slice partials of the FP64 product); partial[blk][c][0] = |r|^2.
__global__ __launch_bounds__(RED_THREADS) void residual_kernel(
    const double *__restrict__ vpart, int slices, int64_t stride, const double *__restrict__ b,
    double *__restrict__ r, int64_t ld, int64_t n, int cols, double *__restrict__ partial,
    const int *__restrict__ gate) {
  __shared__ double red[3][4];
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  const int64_t i0 = (int64_t)blk * CHUNK;
  const int64_t i1 = min(n, i0 + CHUNK);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
    const int64_t idx = (int64_t)c * ld + i;
    const double ri = b[idx] - sum_slices(vpart, slices, stride, idx);
    r[idx] = ri;
    acc += ri * ri;
  }
  acc = block_sum(acc, red[0]);
  if (threadIdx.x == 0) partial[((int64_t)blk * cols + c) * 2] = acc;
}

// partial[blk][c][0] = sum of squares of a over the block's rows
__global__ __launch_bounds__(RED_THREADS) void sumsq_kernel(const double *__restrict__ a,
                                                            int64_t ld, int64_t n, int cols,
                                                            double *__restrict__ partial) {
  __shared__ double red[3][4];
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  const int64_t i0 = (int64_t)blk * CHUNK;
  const int64_t i1 = min(n, i0 + CHUNK);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
    const double ai = a[(int64_t)c * ld + i];
    acc += ai * ai;
  }
  acc = block_sum(acc, red[0]);
  if (threadIdx.x == 0) partial[((int64_t)blk * cols + c) * 2] = acc;
}

// partial[blk][c][0] = block's share of x . (b + r): with r = b - E x,
// x . (b + r) = 2 x.b - x.E x = -2 (x.E x / 2 - x.b), so it is positive
// exactly when x lowers the energy x.E x / 2 - x.b below that of x = 0
__global__ __launch_bounds__(RED_THREADS) void start_energy_kernel(
    const double *__restrict__ x, const double *__restrict__ b, const double *__restrict__ r,
    int64_t ld, int64_t n, int cols, double *__restrict__ partial) {
  __shared__ double red[3][4];
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  const int64_t i0 = (int64_t)blk * CHUNK;
  const int64_t i1 = min(n, i0 + CHUNK);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
    const int64_t idx = (int64_t)c * ld + i;
    acc += x[idx] * (b[idx] + r[idx]);
  }
  acc = block_sum(acc, red[0]);
  if (threadIdx.x == 0) partial[((int64_t)blk * cols + c) * 2] = acc;
}

// scal[field][c] = sum over blocks of partial[blk][c][0]
__global__ void sum_partials_kernel(const double *__restrict__ partial, int nblk, int cols,
                                    double *__restrict__ scal, int field,
                                    const int *__restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int c = threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((int64_t)b * cols + c) * 2];
  scal[field * cols + c] = s;
}

// z = M^-1 r; if set_p, p = z; partial r.r and r.z (active columns only).
template <typename VT>
__global__ __launch_bounds__(RED_THREADS) void cg_refresh_kernel(
    const double *__restrict__ r, double *__restrict__ z, VT *__restrict__ p,
    const double *__restrict__ dinv, int64_t ld, int64_t n, int cols,
    const double *__restrict__ scal, double *__restrict__ partial, int set_p,
    const int *__restrict__ gate) {
  __shared__ double red[3][4];
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  const bool act = scal[S_ACT * cols + c] != 0.0;
  const bool sp = set_p || scal[S_RST * cols + c] != 0.0;
  double arr = 0.0, arz = 0.0;
  if (act) {
    const int64_t i0 = (int64_t)blk * CHUNK;
    const int64_t i1 = min(n, i0 + CHUNK);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
      const int64_t idx = (int64_t)c * ld + i;
      const double ri = r[idx];
      const double zi = ri * dinv[i];
      z[idx] = zi;
      if (sp) p[idx] = (VT)zi;
      arr += ri * ri;
      arz += ri * zi;
    }
  }
  arr = block_sum(arr, red[1]);
  arz = block_sum(arz, red[2]);
  if (threadIdx.x == 0) {
    partial[((int64_t)blk * cols + c) * 2] = arr;
    partial[((int64_t)blk * cols + c) * 2 + 1] = arz;
  }
}

// Index of entry (block b, column c) of a partial array of nb blocks and
// width values per entry: row-major part[b][c][width] (cmajor = 0) or
// column-major part[c][b][width] (the PCG-DC dots). With nb = 1 both agree.
__device__ inline int64_t part_at(int64_t b, int64_t c, int nb, int cols, int width, int cmajor) {
  return cmajor ? (c * nb + b) * width : (b * cols + c) * width;
}

// out[c][w] = sum over b of part(b, c)[w] (w < width) in a fixed order: one
// workgroup per column. Serves the update and direction kernels when
// re-reducing all partials in each of their workgroups would cost more
// than this extra launch (large systems).
__global__ __launch_bounds__(RED_THREADS) void sum_cols_kernel(const double *__restrict__ part,
                                                               int nb, int cols, int width,
                                                               int cmajor,
                                                               double *__restrict__ out) {
  __shared__ double red[3][4];
  const int c = blockIdx.x;
  const int64_t bstride = cmajor ? width : (int64_t)cols * width;
  for (int w = 0; w < width; ++w) {
    const double v = strided_sum(part, nb, threadIdx.x, RED_THREADS, bstride,
                                 part_at(0, c, nb, cols, width, cmajor) + w);
    const double t = block_sum(v, red[w % 3]);
    if (threadIdx.x == 0) out[c * width + w] = t;
  }
}

// Reduce (rr, rz) partials into the scalars of active columns.
// one workgroup per column
__global__ __launch_bounds__(RED_THREADS) void set_scalars_kernel(
    const double *__restrict__ partial, int nblk, int cols, int cmajor, double *__restrict__ scal,
    int slot, const int *__restrict__ gate) {
  __shared__ double red[3][4];
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.x;
  if (scal[S_ACT * cols + c] == 0.0) return;
  if (threadIdx.x == 0) scal[S_RST * cols + c] = 0.0;   // the refresh has applied it
  double rr = 0.0, rz = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RED_THREADS) {
    const int64_t o = part_at(b, c, nblk, cols, 2, cmajor);
    rr += partial[o];
    rz += partial[o + 1];
  }
  rr = block_sum(rr, red[0]);
  rz = block_sum(rz, red[1]);
  if (threadIdx.x == 0) {
    scal[S_RR * cols + c] = rr;
    scal[(S_RZ0 + slot) * cols + c] = rz;
  }
}

// Jacobi path: alpha = rz / p.v; x += alpha p; r -= alpha v; z = M^-1 r and
// the partial rr, rz.
template <typename VT>
__global__ __launch_bounds__(RED_THREADS) void cg_update_kernel(
    double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
    const VT *__restrict__ p, const VT *__restrict__ vpart, int slices, int64_t stride,
    const double *__restrict__ dinv, int64_t ld, int64_t n, int cols, int npv,
    const double *__restrict__ pv_part,
    const double *__restrict__ scal, int slot, double *__restrict__ partial,
    int *__restrict__ flags) {
  __shared__ double red[3][4];
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  const bool act = scal[S_ACT * cols + c] != 0.0 && scal[(S_HOLD0 + slot) * cols + c] == 0.0;
  double arr = 0.0, arz = 0.0;
  if (act) {
    double pv = 0.0;
    for (int b = threadIdx.x; b < npv; b += RED_THREADS) pv += pv_part[(int64_t)b * cols + c];
    pv = block_sum(pv, red[0]);
    const double rz = scal[(S_RZ0 + slot) * cols + c];
    double alpha = 0.0;
    if (pv > 0.0 && isfinite(pv)) {
      alpha = rz / pv;
    } else if (blk == 0 && threadIdx.x == 0) {
      flags[0] = 1;   // breakdown: p^T E p <= 0
      flags[1] = c;
      double *dbg = reinterpret_cast<double *>(flags + 2);
      dbg[0] = pv;
      dbg[1] = rz;
    }
    const int64_t i0 = (int64_t)blk * CHUNK;
    const int64_t i1 = min(n, i0 + CHUNK);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
      const int64_t idx = (int64_t)c * ld + i;
      x[idx] += alpha * (double)p[idx];
      const double ri = r[idx] - alpha * sum_slices(vpart, slices, stride, idx);
      r[idx] = ri;
      const double zi = ri * dinv[i];
      z[idx] = zi;
      arr += ri * ri;
      arz += ri * zi;
    }
  }
  arr = block_sum(arr, red[1]);
  arz = block_sum(arz, red[2]);
  if (threadIdx.x == 0) {
    partial[((int64_t)blk * cols + c) * 2] = arr;
    partial[((int64_t)blk * cols + c) * 2 + 1] = arz;
  }
}

// PCG-DC path of the update: alpha = rz / p.v; x += alpha p; r -= alpha v,
// and r also into its row-interleaved copy rt (layout of rows_kernel).
// Workgroup = 16 rows x one column group of 16; thread t takes column t / 16
// and row t % 16 (column-major accesses in 128-byte pieces); the tile goes
// through LDS so that its rt rows are written as 2 KB of whole lines.
constexpr int UP_ROWS = 16;
template <typename VT>
__global__ __launch_bounds__(RED_THREADS) void cg_update_pc_kernel(
    double *__restrict__ x, double *__restrict__ r, const VT *__restrict__ p,
    const VT *__restrict__ vpart, int slices, int64_t stride, int64_t ld, int64_t n, int cols,
    int npv, const double *__restrict__ pv_part, const double *__restrict__ scal, int slot,
    int *__restrict__ flags, double *__restrict__ rt) {
  __shared__ double pvr[16][kColGroup + 1];
  __shared__ double alpha_s[kColGroup];
  __shared__ double tile[UP_ROWS][kColGroup + 1];
  const int g = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * UP_ROWS;
  // p.v of the group's columns: 16 threads per column over the partials
  {
    const int c = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int col = g * kColGroup + c;
    pvr[part][c] = strided_sum(pv_part, npv, part, 16, cols, col);
  }
  __syncthreads();
  if (threadIdx.x < kColGroup) {
    const int c = threadIdx.x, col = g * kColGroup + c;
    double pv = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) pv += pvr[q][c];
    const double rz = scal[(S_RZ0 + slot) * cols + col];
    double alpha = 0.0;
    if (scal[S_ACT * cols + col] != 0.0 && scal[(S_HOLD0 + slot) * cols + col] == 0.0) {
      if (pv > 0.0 && isfinite(pv)) {
        alpha = rz / pv;
      } else if (blockIdx.x == 0) {
        flags[0] = 1;   // breakdown: p^T E p <= 0
        flags[1] = col;
        double *dbg = reinterpret_cast<double *>(flags + 2);
        dbg[0] = pv;
        dbg[1] = rz;
      }
    }
    alpha_s[c] = alpha;
  }
  __syncthreads();
  const int c = threadIdx.x >> 4, rr = threadIdx.x & 15;
  const int col = g * kColGroup + c;
  const int64_t i = r0 + rr;
  const int64_t idx = (int64_t)col * ld + i;
  double ri = 0.0;
  if (i < n) {
    ri = r[idx];
    if (scal[S_ACT * cols + col] != 0.0 && scal[(S_HOLD0 + slot) * cols + col] == 0.0) {
      const double alpha = alpha_s[c];
      x[idx] += alpha * (double)p[idx];
      ri -= alpha * sum_slices(vpart, slices, stride, idx);
      r[idx] = ri;
    }
  }
  tile[rr][c] = ri;
  __syncthreads();
  rt[((int64_t)g * ld + r0) * kColGroup + threadIdx.x] = tile[threadIdx.x >> 4][threadIdx.x & 15];
}

// Row-interleaved copy of the residual for the PCG-DC apply: column group g
// (16 columns) holds entry (i, c) at rt[(g * ld + i) * 16 + c], so that the
// 16 columns of one atom are one 128-byte line. src has column stride cs and
// fc valid columns of n rows; rows >= n and columns >= fc are written as 0.
// 64 rows x 16 columns per workgroup, transposed through LDS.
constexpr int RT_ROWS = 64;
__global__ __launch_bounds__(RED_THREADS) void rows_kernel(const double *__restrict__ src,
                                                           int64_t cs, int64_t n, int fc,
                                                           double *__restrict__ rt, int64_t ld,
                                                           const int *__restrict__ gate) {
  __shared__ double tile[kColGroup][RT_ROWS + 1];
  if (gate != nullptr && *gate == 0) return;
  const int64_t r0 = (int64_t)blockIdx.x * RT_ROWS;
  const int g = blockIdx.y;
  for (int t = threadIdx.x; t < kColGroup * RT_ROWS; t += RED_THREADS) {
    const int c = t / RT_ROWS, rr = t % RT_ROWS;
    const int64_t i = r0 + rr;
    const int col = g * kColGroup + c;
    tile[c][rr] = (col < fc && i < n) ? src[(int64_t)col * cs + i] : 0.0;
  }
  __syncthreads();
  double *out = rt + ((int64_t)g * ld + r0) * kColGroup;
  for (int t = threadIdx.x; t < kColGroup * RT_ROWS; t += RED_THREADS) {
    const int rr = t / kColGroup, c = t % kColGroup;
    if (r0 + rr < ld) out[t] = tile[c][rr];
  }
}

// 1^T r per column (fixed order): rsum[c] = sum_i r[c * cs + i], zero for
// c >= fc; the Eq. 37 term of the preconditioner apply
__global__ __launch_bounds__(RED_THREADS) void colsum_kernel(const double *__restrict__ r,
                                                            int64_t cs, int64_t n, int fc,
                                                            double *__restrict__ rsum,
                                                            const int *__restrict__ gate) {
  __shared__ double red[4];
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.x;
  double acc = 0.0;
  if (c < fc)
    for (int64_t i = threadIdx.x; i < n; i += RED_THREADS) acc += r[(int64_t)c * cs + i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) rsum[c] = acc;
}

// Preconditioner apply for small systems (fewer than kPcBlockTiles tiles of
// the block-dense form, whose few workgroups would leave most of the chip
// idle): z = P r with P in row-major ELL form whose
// row t is the row of atom order[t] (entry k at t * width + k), r in the
// row-interleaved layout of rows_kernel. One wavefront per row (rows taken
// in the spatial order) and column group (grid.y); lane = 8 e + h takes
// entries k = e, e + 8, ... and the column pair (2h, 2h + 1), so every
// gather of the wavefront reads eight whole 128-byte lines. Each wavefront
// stages its row of P in LDS with all its loads in flight at once (the ELL
// row does not depend on order[t], so that load overlaps them), and the
// vector memory path then serves only the gathers. The eight entry lanes of
// each pair are summed by shuffles in a fixed order. Active columns only
// (scal == nullptr: all); set_p: p = z. bpart (may be null): per workgroup
// and column (r.r, r.z), column-major (bpart[(c * gridDim.x + block) * 2 +
// {0, 1}]) so that the kernels summing one column read it contiguously.
constexpr int PC_ROWS = 4;                  // rows (waves) per workgroup
constexpr int PC_THREADS = 64 * PC_ROWS;
constexpr int PC_CHUNK = 256;               // entries per row staged at a time
constexpr int PC_PER_LANE = PC_CHUNK / 64;

template <typename VT>
__global__ __launch_bounds__(PC_THREADS) void precond_kernel(
    const double *__restrict__ rt, double *__restrict__ z, VT *__restrict__ p,
    const int32_t *__restrict__ pidx, const double *__restrict__ pval, int width,
    const int32_t *__restrict__ order, int64_t ld, int64_t n, int cols,
    const double *__restrict__ scal, int slot, double *__restrict__ bpart, int set_p,
    double gap, const double *__restrict__ rsum, const int *__restrict__ gate,
    double *__restrict__ zt) {
  __shared__ double red[PC_ROWS][kColGroup][2];
  __shared__ double sval[PC_ROWS][PC_CHUNK];
  __shared__ int32_t sidx[PC_ROWS][PC_CHUNK];
  if (gate != nullptr && *gate == 0) return;
  const int g = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = lane >> 3, h = lane & 7;
  const int64_t t = (int64_t)blockIdx.x * PC_ROWS + wave;
  const bool live = t < n;
  const int64_t i = live ? (int64_t)order[t] : -1;
  const int32_t *ix = pidx + (live ? t : 0) * width;
  const double *vx = pval + (live ? t : 0) * width;
  const double *rg = rt + (int64_t)g * ld * kColGroup;
  const int c0 = g * kColGroup + 2 * h;
  const bool act0 = scal == nullptr || (scal[S_ACT * cols + c0] != 0.0 &&
                                         scal[(S_HOLD0 + slot) * cols + c0] == 0.0);
  const bool act1 = scal == nullptr || (scal[S_ACT * cols + c0 + 1] != 0.0 &&
                                         scal[(S_HOLD0 + slot) * cols + c0 + 1] == 0.0);
  double2 ri = make_double2(0.0, 0.0);
  double a0 = 0.0, a1 = 0.0;
  for (int k0 = 0; k0 < width; k0 += PC_CHUNK) {
    const int cw = min(PC_CHUNK, width - k0);
    int32_t li[PC_PER_LANE];
    double lv[PC_PER_LANE];
#pragma unroll
    for (int u = 0; u < PC_PER_LANE; ++u) {
      const int k = lane + 64 * u;
      li[u] = 0;
      lv[u] = 0.0;
      if (live && k < cw) {
        li[u] = ix[k0 + k];
        lv[u] = vx[k0 + k];
      }
    }
    if (k0 == 0 && i >= 0) ri = *reinterpret_cast<const double2 *>(rg + i * kColGroup + 2 * h);
    if (k0 > 0) __syncthreads();
#pragma unroll
    for (int u = 0; u < PC_PER_LANE; ++u) {
      const int k = lane + 64 * u;
      if (k < cw) {
        sidx[wave][k] = li[u];
        sval[wave][k] = lv[u];
      }
    }
    __syncthreads();
    if (i >= 0) {
#pragma unroll 4
      for (int k = e; k < cw; k += 8) {
        const int64_t j = sidx[wave][k];
        const double v = sval[wave][k];
        const double2 x = *reinterpret_cast<const double2 *>(rg + j * kColGroup + 2 * h);
        a0 += v * x.x;
        a1 += v * x.y;
      }
    }
  }
#pragma unroll
  for (int off = 8; off < 64; off <<= 1) {
    a0 += __shfl_xor(a0, off, 64);
    a1 += __shfl_xor(a1, off, 64);
  }
  // lanes 0..7 hold columns (2h, 2h + 1)
  if (zt != nullptr) {
    // raw output (the coarse correction's inner apply): every column, in the
    // row-interleaved layout, no dots
    if (lane < 8 && i >= 0) {
      const double add0 = rsum != nullptr ? gap * rsum[c0] : 0.0;
      const double add1 = rsum != nullptr ? gap * rsum[c0 + 1] : 0.0;
      double *o = zt + ((int64_t)g * ld + i) * kColGroup + 2 * h;
      o[0] = a0 + add0;
      o[1] = a1 + add1;
    }
    return;
  }
  if (lane < 8) {
    double d[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (i >= 0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // the Eq. 37 fill: P's zeros hold gap, its pattern P - gap
        const double zi = (u ? a1 : a0) + (rsum != nullptr ? gap * rsum[c0 + u] : 0.0);
        const double rv = u ? ri.y : ri.x;
        if (u ? act1 : act0) {
          const int64_t idx = (int64_t)(c0 + u) * ld + i;
          z[idx] = zi;
          if (set_p || (scal != nullptr && scal[S_RST * cols + c0 + u] != 0.0)) p[idx] = (VT)zi;
          d[u][0] = rv * rv;
          d[u][1] = rv * zi;
        }
      }
    }
    if (bpart != nullptr) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        red[wave][2 * h + u][0] = d[u][0];
        red[wave][2 * h + u][1] = d[u][1];
      }
    }
  }
  if (bpart == nullptr) return;
  __syncthreads();
  if (threadIdx.x < 2 * kColGroup) {
    const int c = threadIdx.x >> 1, s2 = threadIdx.x & 1;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < PC_ROWS; ++w) v += red[w][c][s2];
    bpart[((int64_t)(g * kColGroup + c) * gridDim.x + blockIdx.x) * 2 + s2] = v;
  }
}

// Preconditioner apply (Sec. III.B.2): z = P r with P in its block-dense
// form: tile t (one workgroup) holds the kPcTile rows of atoms
// order[t kPcTile ..] over U_t, the union of their columns, so z of the tile
// is the product [64 rows x |U_t|] . [|U_t| x cols] on the FP64 matrix cores
// and every row of r is read once per tile (where a row-by-row sparse
// product reads it once per entry). Wave w takes rows 16 w .. 16 w + 15 and
// every column group; per step of 4 entries of U_t lane (lr, lg) gives
// A = P(row lr, U_t[k + lg]) and, per group g, B = r(U_t[k + lg], column
// 16 g + lr) from the row-interleaved copy rt (16 columns of an atom in one
// 128-byte line). Active columns only (scal == nullptr: all); set_p: p = z;
// with the Eq. 37 fill z += gap (1^T r). bpart (may be null): per tile and
// column (r.r, r.z), column-major (bpart[(c * gridDim.x + tile) * 2 +
// {0, 1}]), summed in a fixed order.
template <typename VT, int NG>
__global__ __launch_bounds__(256) void precond_block_kernel(
    const double *__restrict__ rt, double *__restrict__ z, VT *__restrict__ p,
    const int64_t *__restrict__ uoff, const int32_t *__restrict__ uidx,
    const double *__restrict__ blk, const int32_t *__restrict__ order, int64_t ld, int64_t n,
    int cols, const double *__restrict__ scal, int slot, double *__restrict__ bpart, int set_p,
    double gap, const double *__restrict__ rsum, const int *__restrict__ gate,
    double *__restrict__ zt) {
  __shared__ double red[4][16 * NG][2];
  if (gate != nullptr && *gate == 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t tile = blockIdx.x;
  const int64_t k0 = uoff[tile], K = uoff[tile + 1] - k0;
  const int32_t *U = uidx + k0;
  const double *A = blk + k0 * kPcTile + wave * 16 + lr;
  d4 acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t k = lg; k < K; k += 4) {
    const double a = A[k * kPcTile];
    const int64_t j = U[k];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const double b = rt[((int64_t)g * ld + j) * kColGroup + lr];
      acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[g], 0, 0, 0);
    }
  }
  // D[i][j] (row i of the wave's 16, column j of the group) in lane
  // j + 16 (i % 4), register i / 4
  if (zt != nullptr) {
    // raw output (the coarse correction's inner apply): every column, in the
    // row-interleaved layout, no dots
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const double add = rsum != nullptr ? gap * rsum[g * 16 + lr] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t t = tile * kPcTile + wave * 16 + 4 * v + lg;
        if (t < n) zt[((int64_t)g * ld + order[t]) * kColGroup + lr] = acc[g][v] + add;
      }
    }
    return;
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int c = g * 16 + lr;
    const bool act = scal == nullptr || (scal[S_ACT * cols + c] != 0.0 &&
                                         scal[(S_HOLD0 + slot) * cols + c] == 0.0);
    const bool rst = set_p || (scal != nullptr && scal[S_RST * cols + c] != 0.0);
    const double add = rsum != nullptr ? gap * rsum[c] : 0.0;
    double rr = 0.0, rz = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t t = tile * kPcTile + wave * 16 + 4 * v + lg;
      if (t < n && act) {
        const int64_t i = order[t];
        const double zi = acc[g][v] + add;
        const int64_t idx = (int64_t)c * ld + i;
        z[idx] = zi;
        if (rst) p[idx] = (VT)zi;
        const double ri = rt[((int64_t)g * ld + i) * kColGroup + lr];
        rr += ri * ri;
        rz += ri * zi;
      }
    }
    if (bpart != nullptr) {
      rr += __shfl_xor(rr, 16, 64);
      rz += __shfl_xor(rz, 16, 64);
      rr += __shfl_xor(rr, 32, 64);
      rz += __shfl_xor(rz, 32, 64);
      if (lg == 0) {
        red[wave][c][0] = rr;
        red[wave][c][1] = rz;
      }
    }
  }
  if (bpart == nullptr) return;
  __syncthreads();
  if (threadIdx.x < 2 * 16 * NG) {
    const int c = threadIdx.x >> 1, s2 = threadIdx.x & 1;
    const double v = ((red[0][c][s2] + red[1][c][s2]) + red[2][c][s2]) + red[3][c][s2];
    bpart[((int64_t)c * gridDim.x + tile) * 2 + s2] = v;
  }
}

// ---- coarse-space correction (two-level, balancing Neumann-Neumann form)
// z = P_D^T P P_D r + Q r with Q = Z E_c^-1 Z^T, P_D = I - E Q, Z the
// indicator columns of the patches, applied as
//   g1 = E_c^-1 Z^T r,  u = r - (E Z) g1,  w = P u,
//   g2 = E_c^-1 (E Z)^T w,  z = w + Z (g1 - g2).
// Z^T r and Z y are sums and broadcasts over the patches' atoms; the two
// products with E Z (kept as FP32 (E Z)^T, patch-major, atoms contiguous)
// run on the FP32 matrix cores, the two with E_c^-1 on the FP64 ones.

// c1[c * mp + t] = sum of r over the atoms of patch t (fixed order), from the
// row-interleaved rt: one wavefront per patch; lane (lr, lg) takes column lr
// of every group and the patch's atoms lg, lg + 4, ...
template <int NG>
__global__ __launch_bounds__(256) void coarse_restrict_kernel(
    const double *__restrict__ rt, int64_t ld, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ off, int64_t mp, double *__restrict__ c1,
    const int *__restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t t = (int64_t)blockIdx.x * 4 + wave;
  const int32_t k1 = off[t + 1];
  double acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = 0.0;
  for (int32_t k = off[t] + lg; k < k1; k += 4) {
    const int64_t i = perm[k];
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[g] += rt[((int64_t)g * ld + i) * kColGroup + lr];
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    acc[g] += __shfl_xor(acc[g], 16, 64);
    acc[g] += __shfl_xor(acc[g], 32, 64);
    if (lg == 0) c1[(int64_t)(g * kColGroup + lr) * mp + t] = acc[g];
  }
}

// out = E_c^-1 in for 16 NG columns on the FP64 matrix cores: out[c * mp + t]
// = sum_s eci[s * mp + t] in[c * mp + s] (E_c^-1 is symmetric). Workgroup:
// 16 patches t and every column; its four waves split s in quarters and add
// their results in LDS in a fixed order. Lane (lr, lg) gives A = eci(s + lg,
// t0 + lr) and, per group, B = in(column 16 g + lr, s + lg). mode 0: g1 = out
// and its FP32 copy g1f; mode 1: dg = g1 - out.
template <int NG>
__global__ __launch_bounds__(256) void coarse_solve_kernel(
    const double *__restrict__ eci, int64_t mp, const double *__restrict__ in,
    double *__restrict__ g1, float *__restrict__ g1f, double *__restrict__ dg, int mode,
    const int *__restrict__ gate) {
  __shared__ double red[4][NG][4][64];
  if (gate != nullptr && *gate == 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t t0 = (int64_t)blockIdx.x * 16;
  const int64_t q = mp / 4, s0 = wave * q;
  d4 acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t s = s0 + lg; s < s0 + q; s += 4) {
    const double a = eci[s * mp + t0 + lr];
#pragma unroll
    for (int g = 0; g < NG; ++g)
      acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, in[(int64_t)(g * 16 + lr) * mp + s], acc[g],
                                                    0, 0, 0);
  }
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][g][v][lane] = acc[g][v];
  __syncthreads();
  for (int e = threadIdx.x; e < NG * 256; e += 256) {
    const int g = e >> 8, v = (e >> 6) & 3, l = e & 63;
    const double val =
        ((red[0][g][v][l] + red[1][g][v][l]) + red[2][g][v][l]) + red[3][g][v][l];
    // D[i][j] in lane j + 16 (i % 4), register i / 4
    const int64_t t = t0 + 4 * v + (l >> 4);
    const int64_t o = (int64_t)(g * 16 + (l & 15)) * mp + t;
    if (mode == 0) {
      g1[o] = val;
      g1f[o] = (float)val;
    } else {
      dg[o] = g1[o] - val;
    }
  }
}

// u = r - (E Z) g1 into the row-interleaved ut, on the FP32 matrix cores,
// as the product g1^T (E Z)^T: workgroup = 64 atoms, its four waves split
// the patches in quarters and add their sums in LDS in a fixed order. Per
// step of 4 patches lane (lr, lg) loads (E Z)^T(patch t + lg, atoms i0 + 4 lr
// .. + 3) as one float4 and gives A = g1f(column 16 g + lr, patch t + lg);
// product j of a group takes B = the j-th of those atoms, so it holds
// D[row 4 lg + v][column lr] = column 16 g + 4 lg + v of atom i0 + 4 lr + j
// in register v. Rows past n stay 0 (az and rt are 0 there).
template <int NG>
__global__ __launch_bounds__(256) void coarse_prolong_kernel(
    const float *__restrict__ az, const float *__restrict__ g1f, int64_t mp,
    const double *__restrict__ rt, int64_t ld, double *__restrict__ ut,
    const int *__restrict__ gate) {
  __shared__ float red[3][NG][4][4][64];
  if (gate != nullptr && *gate == 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t q = mp / 4, t0 = wave * q;
  f4 acc[NG][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  const float *B = az + i0 + 4 * lr;
#pragma unroll 2
  for (int64_t t = t0 + lg; t < t0 + q; t += 4) {
    const f4 b4 = *reinterpret_cast<const f4 *>(B + t * ld);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float a = g1f[(int64_t)(g * 16 + lr) * mp + t];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[g][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b4[j], acc[g][j], 0, 0, 0);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave - 1][g][j][v][lane] = acc[g][j][v];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float sum = ((acc[g][j][v] + red[0][g][j][v][lane]) + red[1][g][j][v][lane]) +
                          red[2][g][j][v][lane];
        const int64_t o = ((int64_t)g * ld + i0 + 4 * lr + j) * kColGroup + 4 * lg + v;
        ut[o] = rt[o] - (double)sum;
      }
}

// Slice partials of (E Z)^T w on the FP32 matrix cores: c2p[(k * cols + c) *
// mp + t] = sum over the atoms i of slice k of az(t, i) w(i, c), w from the
// row-interleaved wt. Workgroup: kCoarseAlign patches (wave w: 64 of them,
// four row blocks of 16) and one slice of kslice atoms (a multiple of 16).
// Per 16 atoms lane (lr, lg) loads az(patch tb + 16 rb + lr, atoms i + 4 lg
// .. + 3) as one float4; step j (0..3) takes k = lg as the atom i + 4 lg + j,
// with B = w(i + 4 lg + j, column 16 g + lr).
template <int NG>
__global__ __launch_bounds__(256) void coarse_gather_kernel(
    const float *__restrict__ az, const double *__restrict__ wt, int64_t ld, int64_t mp,
    int64_t kslice, int cols, float *__restrict__ c2p, const int *__restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t tb = (int64_t)blockIdx.x * kCoarseAlign + wave * 64;
  const int64_t i0 = (int64_t)blockIdx.y * kslice;
  const int64_t i1 = min(ld, i0 + kslice);
  f4 acc[4][NG];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[rb][g] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t i = i0; i < i1; i += 16) {
    f4 a[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      a[rb] = *reinterpret_cast<const f4 *>(az + (tb + 16 * rb + lr) * ld + i + 4 * lg);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const float b = (float)wt[((int64_t)g * ld + i + 4 * lg + j) * kColGroup + lr];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc[rb][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][j], b, acc[rb][g], 0, 0, 0);
      }
  }
  float *out = c2p + (int64_t)blockIdx.y * cols * mp;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(int64_t)(g * 16 + lr) * mp + tb + 16 * rb + 4 * lg + v] = acc[rb][g][v];
}

// c[e] = sum over the ks slices of c2p (FP64, in slice order), e < count
__global__ __launch_bounds__(256) void coarse_sum_kernel(const float *__restrict__ c2p, int ks,
                                                         int64_t count, double *__restrict__ c,
                                                         const int *__restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  double v = 0.0;
  for (int k = 0; k < ks; ++k) v += (double)c2p[(int64_t)k * count + e];
  c[e] = v;
}

// 1^T u per column of the row-interleaved ut (fixed order): the Eq. 37 term
// of the inner apply
__global__ __launch_bounds__(RED_THREADS) void colsum_rt_kernel(const double *__restrict__ ut,
                                                               int64_t ld, int64_t n,
                                                               double *__restrict__ rsum,
                                                               const int *__restrict__ gate) {
  __shared__ double red[4];
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.x, g = c / kColGroup, cc = c % kColGroup;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RED_THREADS)
    acc += ut[((int64_t)g * ld + i) * kColGroup + cc];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) rsum[c] = acc;
}

// z = w + Z dg (dg = g1 - g2) for the active columns, p = z where a column
// restarts (or set_p), and per workgroup of 64 atoms and column the partial
// (r.r, r.z) into bpart, column-major like the local apply kernels (r from
// the row-interleaved rt). Wave q takes the columns 4 q .. 4 q + 3 of every
// group, lane = atom; the wave sums of the dots run in a fixed order.
template <typename VT>
__global__ __launch_bounds__(256) void coarse_finish_kernel(
    const double *__restrict__ wt, const double *__restrict__ dg,
    const int32_t *__restrict__ pid, const double *__restrict__ rt, int64_t ld, int64_t n,
    int cols, int64_t mp, double *__restrict__ z, VT *__restrict__ p,
    const double *__restrict__ scal, int slot, double *__restrict__ bpart, int set_p,
    const int *__restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < n;
  const int64_t t = live ? pid[i] : 0;
  for (int c0 = 4 * q; c0 < cols; c0 += 16) {
    const int g = c0 / kColGroup;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u;
      const bool act = scal == nullptr || (scal[S_ACT * cols + c] != 0.0 &&
                                           scal[(S_HOLD0 + slot) * cols + c] == 0.0);
      const bool rst = set_p || (scal != nullptr && scal[S_RST * cols + c] != 0.0);
      double rr = 0.0, rz = 0.0;
      if (live && act) {
        const int64_t o = ((int64_t)g * ld + i) * kColGroup + (c % kColGroup);
        const double zi = wt[o] + dg[(int64_t)c * mp + t];
        const int64_t idx = (int64_t)c * ld + i;
        z[idx] = zi;
        if (rst && p != nullptr) p[idx] = (VT)zi;
        const double ri = rt[o];
        rr = ri * ri;
        rz = ri * zi;
      }
      if (bpart != nullptr) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          rr += __shfl_xor(rr, off, 64);
          rz += __shfl_xor(rz, off, 64);
        }
        if (lane == 0) {
          bpart[((int64_t)c * gridDim.x + blockIdx.x) * 2] = rr;
          bpart[((int64_t)c * gridDim.x + blockIdx.x) * 2 + 1] = rz;
        }
      }
    }
  }
}

// beta = rz' / rz; p = z + beta p; block 0 stores rz' in the other slot and
// rr, and counts the iteration.
// Hold: a column whose recursive residual has fallen kHold below the level at
// which the next control step takes a true residual (half the tolerance, or
// the reliable-update factor below the last true residual) does no further
// iteration until that step: below it the recursion only drifts (FP32 p
// underflows, an exactly zero residual gives p = 0) and p^T E p can reach 0.
// The hold flag of the next iteration goes to the other slot (S_HOLD0 +
// slot ^ 1), so no workgroup reads a flag this launch writes; the control
// step clears both.
constexpr double kHold = 1e-3;
// r.z = r^T P r <= 0 for r != 0 means that the preconditioner is not
// positive definite (possible with the Eq. 37 fill): breakdown word 2.
template <typename VT>
__global__ __launch_bounds__(RED_THREADS) void cg_direction_kernel(
    VT *__restrict__ p, const double *__restrict__ z, int64_t ld, int64_t n, int cols, int nblk,
    const double *__restrict__ partial, int cmajor, double *__restrict__ scal, int slot, double tol,
    double ru, int *__restrict__ flags) {
  __shared__ double red[3][4];
  const int c = blockIdx.y;
  const int blk = blockIdx.x;
  if (scal[S_ACT * cols + c] == 0.0) return;
  if (scal[(S_HOLD0 + slot) * cols + c] != 0.0) {
    if (blk == 0 && threadIdx.x == 0) scal[(S_HOLD0 + (slot ^ 1)) * cols + c] = 1.0;
    return;
  }
  double rr = 0.0, rzn = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RED_THREADS) {
    const int64_t o = part_at(b, c, nblk, cols, 2, cmajor);
    rr += partial[o];
    rzn += partial[o + 1];
  }
  rr = block_sum(rr, red[0]);
  rzn = block_sum(rzn, red[1]);
  const double rz = scal[(S_RZ0 + slot) * cols + c];
  const double beta = (rz != 0.0) ? rzn / rz : 0.0;
  const int64_t i0 = (int64_t)blk * CHUNK;
  const int64_t i1 = min(n, i0 + CHUNK);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
    const int64_t idx = (int64_t)c * ld + i;
    p[idx] = (VT)(z[idx] + beta * (double)p[idx]);
  }
  if (blk == 0 && threadIdx.x == 0) {
    if (rr > 0.0 && !(rzn > 0.0)) {
      flags[0] = 2;   // breakdown: r^T P r <= 0
      flags[1] = c;
      double *dbg = reinterpret_cast<double *>(flags + 2);
      dbg[0] = rr;
      dbg[1] = rzn;
    }
    scal[(S_RZ0 + (slot ^ 1)) * cols + c] = rzn;
    scal[S_RR * cols + c] = rr;
    scal[S_IT * cols + c] += 1.0;
    const double bn = sqrt(scal[S_BN2 * cols + c]);
    const double lim = kHold * fmax(0.5 * tol * bn, ru * scal[S_RT * cols + c]);
    scal[(S_HOLD0 + (slot ^ 1)) * cols + c] = (sqrt(rr) <= lim) ? 1.0 : 0.0;
  }
}

// ---- device-side control (one wave, thread c = column)

// After the start residual: |b| and |r| per column; a warm start that does
// not lower the energy x.E x / 2 - x.b below that of zero (scal S_EN <= 0:
// its E-norm error, which CG reduces, is not below the zero start's; or not
// finite) is discarded (x = 0, r = b: applied by fallback_kernel); b = 0
// gives q_b = 0. Sets the active flags and clears the status words.
__global__ void ctl_init_kernel(double *__restrict__ scal, int cols, int fc, int x_zero, double tol,
                                int *__restrict__ flags) {
  const int c = threadIdx.x;
  bool act = false, fb_any = false;
  if (c < cols) {
    const double bn = sqrt(scal[S_BN2 * cols + c]);
    double rn = sqrt(scal[S_RR * cols + c]);
    bool fb = false;
    double res = 0.0, init = 0.0;
    if (c < fc) {
      if (bn == 0.0) {
        fb = !x_zero;
        rn = 0.0;
      } else {
        if (!x_zero && !(scal[S_EN * cols + c] > 0.0 && isfinite(rn))) {
          fb = true;
          fb_any = true;
          rn = bn;
        }
        res = rn / bn;
        init = res;
        act = rn > tol * bn;
      }
    }
    if (fb) scal[S_RR * cols + c] = rn * rn;
    scal[S_ACT * cols + c] = act ? 1.0 : 0.0;
    scal[S_FB * cols + c] = fb ? 1.0 : 0.0;
    scal[S_RT * cols + c] = rn;
    scal[S_RES * cols + c] = res;
    scal[S_INIT * cols + c] = init;
    scal[S_IT * cols + c] = 0.0;
    scal[S_HOLD0 * cols + c] = 0.0;
    scal[S_HOLD1 * cols + c] = 0.0;
    scal[S_RST * cols + c] = 0.0;
    scal[S_RPREV * cols + c] = INFINITY;   // no stall test in the first batch
  }
  const bool any = __any(act), anyfb = __any(fb_any);
  if (threadIdx.x == 0) {
    for (int w = 0; w < F_NWORDS; ++w) flags[w] = 0;
    flags[F_ANY] = any ? 1 : 0;
    flags[F_FELLBACK] = anyfb ? 1 : 0;
  }
}

// x = 0, r = b for the columns whose start was discarded
__global__ __launch_bounds__(RED_THREADS) void fallback_kernel(
    double *__restrict__ x, double *__restrict__ r, const double *__restrict__ b,
    const double *__restrict__ scal, int64_t ld, int64_t n, int cols) {
  const int c = blockIdx.y;
  if (scal[S_FB * cols + c] == 0.0) return;
  const int64_t i0 = (int64_t)blockIdx.x * CHUNK;
  const int64_t i1 = min(n, i0 + CHUNK);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RED_THREADS) {
    const int64_t idx = (int64_t)c * ld + i;
    x[idx] = 0.0;
    r[idx] = b[idx];
  }
}

// After a batch of `todo` iterations (it_after in total): decide whether the
// true residual is due — the recursive residual met half the tolerance, fell
// by the reliable-update factor ru below the last true residual (ru = 0:
// never), did not fall at all over the batch (a stalled recursion; not
// tested in the first batch after a start or a true residual, where the
// residual of a restarted recursion may rise for a few steps), or the
// iteration limit is reached.
__global__ void ctl_check_kernel(double *__restrict__ scal, int cols, int it_after, int todo,
                                 int max_iter, double tol, double ru, int *__restrict__ flags) {
  const int c = threadIdx.x;
  bool need = false, bad = false;
  double rel = 0.0;
  if (c < cols && scal[S_ACT * cols + c] != 0.0) {
    const double bn = sqrt(scal[S_BN2 * cols + c]);
    const double rn = sqrt(scal[S_RR * cols + c]);
    if (!isfinite(rn)) bad = true;
    need = rn <= 0.5 * tol * bn || (ru > 0.0 && rn <= ru * scal[S_RT * cols + c]) ||
           rn > scal[S_RPREV * cols + c] || it_after >= max_iter;
    scal[S_RPREV * cols + c] = rn;
    rel = bn > 0.0 ? rn / bn : 0.0;
  }
  const bool any_need = __any(need), any_bad = __any(bad);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rel = fmax(rel, __shfl_xor(rel, off, 64));
  if (threadIdx.x == 0) {
    flags[F_NEED] = any_need ? 1 : 0;
    if (any_bad) flags[F_NONFINITE] = 1;
    *reinterpret_cast<double *>(flags + F_RMAX) = rel;
  }
}

// After a true residual (only when one was due): |r|^2 from the residual
// kernel's partials, record it, retire the columns that meet the tolerance,
// count the update. A column whose true residual exceeds kTrack times the
// recursive one it replaces, or the previous true residual, is marked for a
// restart (p = z at the refresh that follows): its recursion no longer
// tracks the true residual, and the step length rz / p^T E p of a kept
// direction assumes that it does (r orthogonal to the previous directions).
// Left alone, such a column can diverge while its recursive residual stays
// put.
constexpr double kTrack = 4.0;
__global__ void ctl_update_kernel(const double *__restrict__ partial, int nblk,
                                  double *__restrict__ scal, int cols, int fc, double tol,
                                  int *__restrict__ flags) {
  if (flags[F_NEED] == 0) return;
  const int c = threadIdx.x;
  bool act = false;
  double rel = 0.0;
  if (c < cols) {
    double rr = 0.0;
    for (int b = 0; b < nblk; ++b) rr += partial[((int64_t)b * cols + c) * 2];
    const double rec = sqrt(scal[S_RR * cols + c]);   // the recursive residual it replaces
    const double last = scal[S_RT * cols + c];         // the previous true residual
    scal[S_RR * cols + c] = rr;
    scal[S_HOLD0 * cols + c] = 0.0;
    scal[S_HOLD1 * cols + c] = 0.0;
    scal[S_RST * cols + c] = 0.0;
    act = scal[S_ACT * cols + c] != 0.0;
    const double bn = sqrt(scal[S_BN2 * cols + c]);
    if (c < fc && bn != 0.0) {
      const double rn = sqrt(scal[S_RR * cols + c]);
      scal[S_RES * cols + c] = rn / bn;
      if (act) {
        scal[S_RT * cols + c] = rn;
        scal[S_RPREV * cols + c] = INFINITY;   // nor in the first batch after an update
        if (rn <= tol * bn) {
          act = false;
          scal[S_ACT * cols + c] = 0.0;
        } else if (rn > kTrack * rec || rn > last) {
          scal[S_RST * cols + c] = 1.0;
        }
        if (act) rel = rn / bn;
      }
    }
  }
  const bool any = __any(act);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rel = fmax(rel, __shfl_xor(rel, off, 64));
  if (threadIdx.x == 0) {
    flags[F_ANY] = any ? 1 : 0;
    flags[F_UPDATES] += 1;
    // the host's convergence forecast then extrapolates from the true
    // residual of the columns still active, not from the recursive one it
    // replaced (which in FP32 / BF16 runs ahead of it)
    *reinterpret_cast<double *>(flags + F_RMAX) = rel;
  }
}

template <typename VT>
__global__ void sum_slices_kernel(const VT *__restrict__ part, int slices, int64_t stride,
                                  double *__restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = sum_slices(part, slices, stride, i);
}

__global__ void f64_to_f32_kernel(const double *__restrict__ a, float *__restrict__ b,
                                  int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = (float)a[i];
}

__global__ void f32_to_f64_kernel(const float *__restrict__ a, double *__restrict__ b,
                                  int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = (double)a[i];
}

__global__ void zero_kernel(double *__restrict__ a, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = 0.0;
}

// Copy rows of a frame-major (f, n) array into (cols, ld) with zero padding.
__global__ void pack_kernel(const double *__restrict__ src, int64_t n, int64_t f,
                            double *__restrict__ dst, int64_t ld, int64_t cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= ld || c >= cols) return;
  dst[c * ld + i] = (c < f && i < n) ? src[c * n + i] : 0.0;
}

// Two-step neutralisation (Eq. 35): q = x - (sum(x) + Q_sol) d, one block per
// frame. The shift is applied a second time to what rounding left of
// sum(q) + Q_sol (sum(d) = 1 holds only to ~n ulps, and sum(x) + Q_sol can be
// large), which is the same correction along d; reports |sum(q) + Q_sol|.
__global__ __launch_bounds__(RED_THREADS) void project_kernel(
    const double *__restrict__ x, int64_t ld, int64_t n, const double *__restrict__ d,
    const double *__restrict__ qsol, double *__restrict__ q, double *__restrict__ sum_err) {
  __shared__ double red[3][4];
  const int64_t f = blockIdx.x;
  const double *xf = x + f * ld;
  double *qf = q + f * n;
  double s = 0.0;
  // (unrolled so that a thread's loads are in flight together; the order of
  // the additions is unchanged)
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += RED_THREADS) s += xf[i];
  s = block_sum(s, red[0]);
  const double shift = s + qsol[f];
  double t = 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += RED_THREADS) {
    const double qi = xf[i] - shift * d[i];
    qf[i] = qi;
    t += qi;
  }
  t = block_sum(t, red[1]);
  const double shift2 = t + qsol[f];
  double t2 = 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += RED_THREADS) {   // each thread rereads its own q
    const double qi = qf[i] - shift2 * d[i];
    qf[i] = qi;
    t2 += qi;
  }
  t2 = block_sum(t2, red[2]);
  if (threadIdx.x == 0) sum_err[f] = fabs(t2 + qsol[f]);
}

__global__ void diag_inverse_kernel(const double *__restrict__ E, int64_t n, int64_t ld,
                                    double *__restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ld) dinv[i] = (i < n) ? 1.0 / E[i * ld + i] : 0.0;
}

// ------------------------------------------------------------------ host side

dim3 elem_grid(int64_t count) { return dim3((unsigned)((count + 255) / 256)); }

// profiling context of the current call (set by the drivers below)
thread_local Profile *t_prof = nullptr;
thread_local int64_t t_n = 0;

template <typename T> constexpr int prec_of() {
  return sizeof(T) == 8 ? CPM_PREC_F64 : (sizeof(T) == 4 ? CPM_PREC_F32 : CPM_PREC_BF16);
}

// k slices of a wide block product (128-row workgroups, k in steps of 32):
// about 3072 workgroups, several per resident slot (3 workgroups of 4 waves
// per CU): with one per tile (1024 at N = 131072, 768 slots) the last round
// left two thirds of the chip idle, 15.5 -> 11.9 ms for the FP32 product and
// 31.8 -> 24.7 ms for the FP64 one at that size. The slices' partial sums
// (slices x cols x ld of vsize bytes) stay under 1/16 of the bytes of E.
int64_t wide_slices(int64_t ld, int64_t cols, int64_t esize, int64_t vsize, int64_t &kslice) {
  constexpr int64_t kRowsPerWg = 128, kStep = 32, kTargetWgs = 3072;
  static_assert(SP_ROWS == kRowsPerWg && F64_ROWS == kRowsPerWg, "128-row workgroups");
  static_assert(SP_KC == kStep && F64_KC == kStep, "k steps of 32");
  const int64_t tiles = ld / kRowsPerWg;
  const int64_t units = ld / kStep;
  int64_t want = std::max<int64_t>(1, (kTargetWgs + tiles - 1) / tiles);
  want = std::min<int64_t>(want, std::max<int64_t>(1, (ld * esize) / (16 * cols * vsize)));
  want = std::min<int64_t>(want, units);
  kslice = (units + want - 1) / want * kStep;
  return (ld + kslice - 1) / kslice;
}
// the split-bf16 kernel serves FP32 and BF16 E with 32..64 columns
template <typename T> constexpr bool uses_split(int64_t cols) {
  return sizeof(T) <= 4 && cols >= 32;
}

// the streamed-P FP64 kernel serves an FP64 E with 32..64 columns
template <typename T> constexpr bool uses_f64s(int64_t cols) {
  return sizeof(T) == 8 && cols >= 32;
}

int64_t split_slices(int64_t ld, int64_t cols, int64_t esize, int64_t &kslice) {
  return wide_slices(ld, cols, esize, sizeof(float), kslice);
}
int64_t f64s_slices(int64_t ld, int64_t cols, int64_t &kslice) {
  return wide_slices(ld, cols, sizeof(double), sizeof(double), kslice);
}

// k slices of the row-split kernel (16 columns): about 432 workgroups, each
// slice a multiple of the k step and short enough for its P copy in LDS
template <typename T> int64_t rows_slices(int64_t ld, int64_t &kslice) {
  constexpr int64_t kb = 4 * Mv<T>::VEC;
  const int64_t blocks = ld / (16 * MR_WAVES);
  const int64_t want = std::max<int64_t>(1, (432 + blocks - 1) / std::max<int64_t>(1, blocks));
  kslice = (ld / want + kb - 1) / kb * kb;
  kslice = std::min<int64_t>(std::max<int64_t>(kslice, kb), mr_kmax<T>());
  return (ld + kslice - 1) / kslice;
}

// (slice, tile) pairs of the block product for cols columns: entries of p.v
// partials per column
template <typename T> int64_t matvec_npv(int64_t ld, int64_t cols) {
  int64_t k = 0;
  if (uses_split<T>(cols)) return split_slices(ld, cols, sizeof(T), k) * (ld / SP_ROWS);
  if (uses_f64s<T>(cols)) return f64s_slices(ld, cols, k) * (ld / F64_ROWS);
  return rows_slices<T>(ld, k) * (ld / (16 * MR_WAVES));   // 16 columns
}

// slices of the kernel that serves c columns of an E of type T
template <typename T> int64_t slices_for(int64_t ld, int64_t c) {
  int64_t k = 0;
  if (uses_split<T>(c)) return split_slices(ld, c, sizeof(T), k);
  if (uses_f64s<T>(c)) return f64s_slices(ld, c, k);
  return rows_slices<T>(ld, k);   // 16 columns
}

// elements of the partial-product buffer for up to cols columns (slices x
// columns x ld of the widest case) and the most (slice, tile) pairs of p.v
// partials per column
int64_t vpart_elems(int64_t ld, int64_t cols) {
  int64_t e = 0;
  for (int64_t c = kColGroup; c <= cols; c += kColGroup)
    e = std::max({e, c * slices_for<double>(ld, c), c * slices_for<float>(ld, c),
                  c * slices_for<uint16_t>(ld, c)});
  return ld * e;
}
int64_t max_npv(int64_t ld, int64_t cols) {
  int64_t e = 0;
  for (int64_t c = kColGroup; c <= cols; c += kColGroup)
    e = std::max({e, matvec_npv<double>(ld, c), matvec_npv<float>(ld, c),
                  matvec_npv<uint16_t>(ld, c)});
  return e;
}

template <typename T, int NG>
hipError_t launch_matvec_t(hipStream_t st, const T *E, int64_t ld, const typename Mv<T>::VT *P,
                           typename Mv<T>::VT *part, double *pv_part, int &slices,
                           const int *gate) {
  constexpr bool split = uses_split<T>(NG * 16);
  constexpr bool f64s = uses_f64s<T>(NG * 16);
  static_assert(split || f64s || NG == 1, "16 columns or an FP32/BF16/FP64 wide kernel");
  int64_t kslice = 0;
  slices = split ? (int)split_slices(ld, NG * 16, sizeof(T), kslice)
           : f64s ? (int)f64s_slices(ld, NG * 16, kslice)
                  : (int)rows_slices<T>(ld, kslice);
  const int64_t tiles = split ? ld / SP_ROWS : f64s ? ld / F64_ROWS : ld / (16 * MR_WAVES);
  hipEvent_t ea = nullptr, eb = nullptr;
  int *mark = nullptr;
  if (t_prof && t_prof->sample(prec_of<T>())) {
    // algorithmic traffic: E (n x n) once, the n x cols block P read and V written
    const double n = (double)t_n;
    const double work = sizeof(T) * n * n + 2.0 * sizeof(typename Mv<T>::VT) * n * (NG * 16);
    Profile::Rec &r = t_prof->add(prec_of<T>(), work);
    ea = r.a;
    eb = r.b;
    if (gate) mark = t_prof->take_mark(r);
  }
  if constexpr (f64s) {
    hipExtLaunchKernelGGL((block_matvec_f64s_kernel<NG>), dim3((unsigned)tiles, (unsigned)slices),
                          dim3(256), 0, st, ea, eb, 0, reinterpret_cast<const double *>(E), ld,
                          reinterpret_cast<const double *>(P), reinterpret_cast<double *>(part),
                          kslice, (int64_t)(NG * 16) * ld, pv_part, gate, mark);
  } else if constexpr (split) {
    hipExtLaunchKernelGGL((block_matvec_split_kernel<T, NG>),
                          dim3((unsigned)tiles, (unsigned)slices), dim3(256), 0, st, ea, eb, 0, E,
                          ld, P, part, kslice, (int64_t)(NG * 16) * ld, pv_part, gate, mark);
  } else {
    const size_t lds = sizeof(typename Mv<T>::VT) * 16 * (size_t)(kslice + mr_pad<T>());
    hipExtLaunchKernelGGL((block_matvec_rows_kernel<T>), dim3((unsigned)tiles, (unsigned)slices),
                          dim3(64 * MR_WAVES), lds, st, ea, eb, 0, E, ld, P, part, kslice,
                          (int64_t)16 * ld, pv_part, gate, mark);
  }
  return hipGetLastError();
}

// V = E P for cols = 16..64 columns; gate (device int, may be null): the
// launch does nothing when it reads 0
template <typename T>
hipError_t launch_matvec(hipStream_t st, const T *E, int64_t ld, int64_t cols,
                         const typename Mv<T>::VT *P, typename Mv<T>::VT *part, double *pv_part,
                         int &slices, const int *gate = nullptr) {
  switch (cols / 16) {
    case 1: return launch_matvec_t<T, 1>(st, E, ld, P, part, pv_part, slices, gate);
    case 2: return launch_matvec_t<T, 2>(st, E, ld, P, part, pv_part, slices, gate);
    case 3: return launch_matvec_t<T, 3>(st, E, ld, P, part, pv_part, slices, gate);
    case 4: return launch_matvec_t<T, 4>(st, E, ld, P, part, pv_part, slices, gate);
    default: return hipErrorInvalidValue;
  }
}

void free_workspace(Workspace &w) {
  void *ptrs[] = {w.x, w.r, w.rt, w.p, w.z, w.v, w.vpart, w.partial, w.scal, w.red, w.sum_err, w.rsum, w.bx, w.bres, w.flags,
                  w.xf, w.rf, w.pf, w.zf, w.vf, w.bpart};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  if (w.hstat) (void)hipHostFree(w.hstat);
  if (w.hfin) (void)hipHostFree(w.hfin);
  if (w.hfl) (void)hipHostFree(w.hfl);
  for (hipEvent_t e : w.ev)
    if (e) (void)hipEventDestroy(e);
  w = Workspace();
}

cpm_status ensure_workspace(cpm_system *s, int64_t cols) {
  Workspace &w = s->ws;
  if (w.cols >= cols) return CPM_OK;
  s->device_bytes -= (int64_t)w.bytes;
  free_workspace(w);
  const int64_t ld = s->ld;
  const size_t vec = sizeof(double) * (size_t)ld * (size_t)cols;
  const int64_t nblk = (s->n + CHUNK - 1) / CHUNK;
  const int64_t vpe = vpart_elems(ld, cols);
  const int64_t npv = max_npv(ld, cols);   // most p.v partials per column
  size_t total = 0;
  auto alloc = [&](void **p, size_t bytes) -> bool {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    total += bytes;
    return true;
  };
  // x, r, z, b, v (FP64); p (FP64) and pf, vf (FP32) for the mixed modes
  bool ok = alloc(&w.x, vec) && alloc(&w.r, vec) && alloc((void **)&w.rt, vec) &&
            alloc(&w.p, vec) && alloc(&w.z, vec) &&
            alloc(&w.v, sizeof(double) * (size_t)vpe) && alloc((void **)&w.bx, vec) &&
            alloc((void **)&w.bres, vec) &&
            alloc(&w.pf, vec / 2) && alloc(&w.vf, sizeof(float) * (size_t)vpe) &&
            alloc((void **)&w.partial, sizeof(double) * 2 * (size_t)(nblk + npv) * cols) &&
            alloc((void **)&w.scal, sizeof(double) * S_NFIELDS * cols) &&
            alloc((void **)&w.red, sizeof(double) * 3 * MAX_COLS) &&
            alloc((void **)&w.sum_err, sizeof(double) * MAX_COLS) &&
            alloc((void **)&w.rsum, sizeof(double) * MAX_COLS) &&
            alloc((void **)&w.bpart,
                  sizeof(double) * 2 * (size_t)((s->n + PC_ROWS - 1) / PC_ROWS) * cols) &&
            alloc((void **)&w.flags, sizeof(int) * F_NWORDS);
  if (ok && (hipHostMalloc((void **)&w.hstat, sizeof(int) * F_NWORDS * kStatusSlots,
                           hipHostMallocDefault) != hipSuccess ||
             hipHostMalloc((void **)&w.hfin, sizeof(double) * (S_NFIELDS + 1) * MAX_COLS,
                           hipHostMallocDefault) != hipSuccess ||
             hipHostMalloc((void **)&w.hfl, sizeof(int) * F_NWORDS, hipHostMallocDefault) !=
                 hipSuccess)) {
    (void)hipGetLastError();
    ok = false;
  }
  for (hipEvent_t &e : w.ev)
    if (ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
      ok = false;
    }
  if (!ok) {
    free_workspace(w);
    set_error("workspace allocation failed");
    return CPM_ENOMEM;
  }
  if (hipMemset(w.flags, 0, sizeof(int) * F_NWORDS) != hipSuccess ||
      hipMemset(w.scal, 0, sizeof(double) * S_NFIELDS * cols) != hipSuccess) {
    set_error("workspace memset failed");
    return CPM_EDEVICE;
  }
  void *zs[] = {w.x, w.r, w.rt, w.p, w.z, w.bx, w.bres};
  for (void *q : zs)
    if (hipMemset(q, 0, vec) != hipSuccess) {
      set_error("workspace memset failed");
      return CPM_EDEVICE;
    }
  if (hipMemset(w.v, 0, sizeof(double) * (size_t)vpe) != hipSuccess ||
      hipMemset(w.vf, 0, sizeof(float) * (size_t)vpe) != hipSuccess) {
    set_error("workspace memset failed");
    return CPM_EDEVICE;
  }
  void *zf[] = {w.pf};
  for (void *q : zf)
    if (hipMemset(q, 0, vec / 2) != hipSuccess) {
      set_error("workspace memset failed");
      return CPM_EDEVICE;
    }
  w.cols = cols;
  w.bytes = total;
  s->device_bytes += (int64_t)total;
  return CPM_OK;
}

// the local apply z = P r of the sparse P for cols columns of the
// row-interleaved rt; bpart gets one (r.r, r.z) pair per workgroup and
// column; rsum (may be null): the column sums of r for the Eq. 37 fill.
// zt != null: raw output of every column into the row-interleaved zt
// instead of z, p and the dots.
template <typename VT>
void launch_local(hipStream_t st, const cpm_system *s, const Precond &pc, const double *rt,
                  double *z, VT *p, int64_t cols, const double *scal, int slot, double *bpart,
                  bool set_p, const double *rsum, const int *gate, double *zt) {
  const int64_t ld = s->ld, n = s->n;
  if (pc.blk == nullptr) {
    hipLaunchKernelGGL(precond_kernel<VT>,
                       dim3((unsigned)((n + PC_ROWS - 1) / PC_ROWS), (unsigned)(cols / kColGroup)),
                       dim3(PC_THREADS), 0, st, rt, z, p, (const int32_t *)pc.idx,
                       (const double *)pc.val, pc.width, s->atom_order, ld, n, (int)cols, scal,
                       slot, bpart, set_p ? 1 : 0, pc.gap, rsum, gate, zt);
    return;
  }
  const dim3 grid((unsigned)pc.ntiles);
#define CPM_PB(NGV)                                                                            \
  hipLaunchKernelGGL((precond_block_kernel<VT, NGV>), grid, dim3(256), 0, st, rt, z, p,       \
                     (const int64_t *)pc.uoff, (const int32_t *)pc.uidx, (const double *)pc.blk, \
                     s->atom_order, ld, n, (int)cols, scal, slot, bpart, set_p ? 1 : 0, pc.gap,  \
                     rsum, gate, zt)
  switch (cols / kColGroup) {
    case 1: CPM_PB(1); break;
    case 2: CPM_PB(2); break;
    case 3: CPM_PB(3); break;
    default: CPM_PB(4); break;
  }
#undef CPM_PB
}

// the coarse-correction kernels that depend on the number of column groups
template <int NG>
void launch_coarse_ng(hipStream_t st, const cpm_system *s, const double *rt, const int *gate,
                      int stage) {
  const Coarse &cz = s->cz;
  const int64_t ld = s->ld, mp = cz.mp;
  if (stage == 0) {
    hipLaunchKernelGGL(coarse_restrict_kernel<NG>, dim3((unsigned)(mp / 4)), dim3(256), 0, st, rt,
                       ld, (const int32_t *)cz.perm, (const int32_t *)cz.off, mp, cz.c1, gate);
    hipLaunchKernelGGL(coarse_solve_kernel<NG>, dim3((unsigned)(mp / 16)), dim3(256), 0, st,
                       (const double *)cz.eci, mp, (const double *)cz.c1, cz.g1, cz.g1f,
                       (double *)nullptr, 0, gate);
    hipLaunchKernelGGL(coarse_prolong_kernel<NG>, dim3((unsigned)(ld / 64)), dim3(256), 0, st,
                       (const float *)cz.az, (const float *)cz.g1f, mp, rt, ld, cz.ut, gate);
  } else {
    hipLaunchKernelGGL(coarse_gather_kernel<NG>, dim3((unsigned)(mp / kCoarseAlign), (unsigned)cz.ks),
                       dim3(256), 0, st, (const float *)cz.az, (const double *)cz.wt, ld, mp,
                       cz.kslice, NG * 16, cz.c2p, gate);
    const int64_t count = (int64_t)NG * 16 * mp;
    hipLaunchKernelGGL(coarse_sum_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       (const float *)cz.c2p, cz.ks, count, cz.c1, gate);
    hipLaunchKernelGGL(coarse_solve_kernel<NG>, dim3((unsigned)(mp / 16)), dim3(256), 0, st,
                       (const double *)cz.eci, mp, (const double *)cz.c1, cz.g1, (float *)nullptr,
                       cz.dg, 1, gate);
  }
}

// z = P r (PCG-DC, the sparsified inverse, with the Eq. 37 fill and the
// coarse correction where they are on) for cols columns of the
// row-interleaved residual rt; bpart gets one (r.r, r.z) pair per workgroup
// and column. With the Eq. 37 fill, r (column c at r + c * rs, fc columns)
// gives the column sums first.
template <typename VT>
void launch_precond(hipStream_t st, const cpm_system *s, const Precond &pc, const double *rt,
                    const double *r, int64_t rs, int fc, double *z, VT *p, int64_t cols,
                    const double *scal, int slot, double *bpart, bool set_p, const int *gate) {
  const int64_t ld = s->ld, n = s->n;
  if (!s->cz.ready) {
    const double *rsum = nullptr;
    if (pc.gap != 0.0) {
      hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)cols), dim3(RED_THREADS), 0, st, r, rs, n,
                         fc, s->ws.rsum, gate);
      rsum = s->ws.rsum;
    }
    launch_local<VT>(st, s, pc, rt, z, p, cols, scal, slot, bpart, set_p, rsum, gate, nullptr);
    return;
  }
  const Coarse &cz = s->cz;
  auto by_ng = [&](int stage) {
    switch (cols / kColGroup) {
      case 1: launch_coarse_ng<1>(st, s, rt, gate, stage); break;
      case 2: launch_coarse_ng<2>(st, s, rt, gate, stage); break;
      case 3: launch_coarse_ng<3>(st, s, rt, gate, stage); break;
      default: launch_coarse_ng<4>(st, s, rt, gate, stage); break;
    }
  };
  // g1 = E_c^-1 Z^T r, u = r - (E Z) g1
  by_ng(0);
  // w = P u (raw, every column)
  const double *rsum = nullptr;
  if (pc.gap != 0.0) {
    hipLaunchKernelGGL(colsum_rt_kernel, dim3((unsigned)cols), dim3(RED_THREADS), 0, st,
                       (const double *)cz.ut, ld, n, s->ws.rsum, gate);
    rsum = s->ws.rsum;
  }
  launch_local<VT>(st, s, pc, cz.ut, (double *)nullptr, (VT *)nullptr, cols, nullptr, 0, nullptr,
                   false, rsum, gate, cz.wt);
  // dg = g1 - E_c^-1 (E Z)^T w
  by_ng(1);
  // z = w + Z dg, p, dots
  hipLaunchKernelGGL(coarse_finish_kernel<VT>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st,
                     (const double *)cz.wt, (const double *)cz.dg, (const int32_t *)cz.pid, rt, ld,
                     n, (int)cols, cz.mp, z, p, scal, slot, bpart, set_p ? 1 : 0, gate);
}

// The solver over one block of cols columns. VT is the vector type of p and
// v (double for FP64 E, float for FP32 / BF16 E); x, r, z, b are FP64.
template <typename T> struct Solver {
  using VT = typename Mv<T>::VT;
  cpm_system *s;
  hipStream_t st;
  const T *E;
  int64_t n, ld, cols;
  int nblk, npv;
  double *x, *r, *z, *b, *v64, *partial, *pvp, *scal, *rt;
  VT *p, *v;
  int *flags;
  int slot = 0;
  const Precond *pc = nullptr;   // PCG-DC preconditioner (nullptr: Jacobi)
  double tol = 0.0, ru = 0.0;    // tolerance and reliable-update factor (hold test)

  Solver(cpm_system *s_, const T *E_, int64_t cols_, const Precond *pc_)
      : s(s_), st(s_->stream), E(E_), pc(pc_) {
    n = s->n;
    ld = s->ld;
    cols = cols_;
    nblk = (int)((n + CHUNK - 1) / CHUNK);
    npv = (int)matvec_npv<T>(ld, cols);
    Workspace &w = s->ws;
    x = (double *)w.x; r = (double *)w.r; z = (double *)w.z; b = w.bx; v64 = (double *)w.v;
    rt = w.rt;
    partial = w.partial;
    pvp = w.partial + 2 * (int64_t)nblk * cols;
    scal = w.scal;
    flags = w.flags;
    if constexpr (sizeof(VT) == 8) {
      p = (VT *)w.p;
      v = (VT *)w.v;
    } else {
      p = (VT *)w.pf;
      v = (VT *)w.vf;
    }
  }
  dim3 grid() const { return dim3((unsigned)nblk, (unsigned)cols); }
  const int *need() const { return flags + F_NEED; }

  // r = b - E64 x for all columns; scal RR = |r|^2 (gate: skipped when *gate == 0)
  // (sum_rr: also reduce |r|^2 into the scalars; otherwise ctl_update_kernel does)
  hipError_t true_residual(const int *gate, bool sum_rr = true) {
    int sl = 0;
    hipError_t e = launch_matvec<double>(st, s->E64, ld, cols, x, v64, nullptr, sl, gate);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_kernel, grid(), dim3(RED_THREADS), 0, st, v64, sl, ld * cols, b,
                       r, ld, n, (int)cols, partial, gate);
    if (sum_rr)
      hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(MAX_COLS), 0, st, partial, nblk,
                         (int)cols, scal, (int)S_RR, gate);
    return hipGetLastError();
  }

  // partial sums of r.r / r.z per column that the direction and set_scalars
  // kernels add up: one per vector block (Jacobi) or per preconditioner
  // workgroup (DC)
  int npc() const {
    if (s->cz.ready) return (int)((n + 63) / 64);   // coarse_finish_kernel's workgroups
    return pc->blk ? (int)pc->ntiles : (int)((n + PC_ROWS - 1) / PC_ROWS);
  }
  int nred() const { return pc ? npc() : nblk; }
  const double *dots() const { return pc ? s->ws.bpart : partial; }
  int dots_cmajor() const { return pc ? 1 : 0; }

  // z = P r with the DC preconditioner; to_rows: r was written by another
  // kernel than the update, so its row-interleaved copy is made first
  void precondition(bool set_p, const int *gate, bool to_rows) {
    if (to_rows)
      hipLaunchKernelGGL(rows_kernel, dim3((unsigned)(ld / RT_ROWS), (unsigned)(cols / kColGroup)),
                         dim3(RED_THREADS), 0, st, (const double *)r, ld, n, (int)cols, rt, ld,
                         gate);
    launch_precond<VT>(st, s, *pc, rt, r, ld, (int)cols, z, p, cols, scal, slot, s->ws.bpart,
                       set_p, gate);
  }

  // z = M^-1 r (and p = z when restarting); rz into the current slot
  hipError_t refresh(bool set_p, const int *gate) {
    if (pc)
      precondition(set_p, gate, true);
    else
      hipLaunchKernelGGL(cg_refresh_kernel<VT>, grid(), dim3(RED_THREADS), 0, st, r, z, p, s->dinv,
                         ld, n, (int)cols, scal, partial, set_p ? 1 : 0, gate);
    hipLaunchKernelGGL(set_scalars_kernel, dim3((unsigned)cols), dim3(RED_THREADS), 0, st, dots(),
                       nred(), (int)cols, dots_cmajor(), scal, slot, gate);
    return hipGetLastError();
  }

  // one CG iteration of the active columns (nothing once none is active)
  hipError_t iterate() {
    int sl = 0;
    hipError_t e = launch_matvec<T>(st, E, ld, cols, p, v, pvp, sl, flags + F_ANY);
    if (e != hipSuccess) return e;
    // p.v partials: reduced once up front when every update workgroup
    // re-reducing them would read more than kRedLoads values
    const double *pvs = pvp;
    int npvs = npv;
    const int64_t upd_loads = pc ? (int64_t)npv * ld * cols / kColGroup : (int64_t)npv * nblk * cols;
    if (upd_loads > kRedLoads) {
      hipLaunchKernelGGL(sum_cols_kernel, dim3((unsigned)cols), dim3(RED_THREADS), 0, st, pvp, npv,
                         (int)cols, 1, 0, s->ws.red);
      pvs = s->ws.red;
      npvs = 1;
    }
    if (pc) {
      hipLaunchKernelGGL(cg_update_pc_kernel<VT>, dim3((unsigned)(ld / UP_ROWS), (unsigned)(cols / kColGroup)),
                         dim3(RED_THREADS), 0, st, x, r, (const VT *)p, (const VT *)v, sl, ld * cols,
                         ld, n, (int)cols, npvs, pvs, scal, slot, flags, rt);
      precondition(false, flags + F_ANY, false);
    } else {
      hipLaunchKernelGGL(cg_update_kernel<VT>, grid(), dim3(RED_THREADS), 0, st, x, r, z, p,
                         v, sl, ld * cols, s->dinv, ld, n, (int)cols, npvs, pvs, scal, slot, partial,
                         flags);
    }
    const double *ds = dots();
    int nds = nred();
    if (2 * (int64_t)nds * nblk * cols > kRedLoads) {
      hipLaunchKernelGGL(sum_cols_kernel, dim3((unsigned)cols), dim3(RED_THREADS), 0, st, ds, nds,
                         (int)cols, 2, dots_cmajor(), s->ws.red + MAX_COLS);
      ds = s->ws.red + MAX_COLS;
      nds = 1;
    }
    hipLaunchKernelGGL(cg_direction_kernel<VT>, grid(), dim3(RED_THREADS), 0, st, p, z, ld, n,
                       (int)cols, nds, ds, dots_cmajor(), scal, slot, tol, ru, flags);
    slot ^= 1;
    return hipGetLastError();
  }
};

cpm_status breakdown_error(int it_done, const int *fl) {
  double dbg[2];
  std::memcpy(dbg, fl + 2, sizeof(dbg));
  if (fl[F_BREAK] == 2) {
    set_error("PCG breakdown: r^T P r <= 0 (the preconditioner is not positive definite; the "
              "Eq. 37 gap fill can make it indefinite); column " + std::to_string(fl[F_COL]) +
              " within the first " + std::to_string(it_done) + " iterations, r.r=" +
              std::to_string(dbg[0]) + " r.z=" + std::to_string(dbg[1]));
    return CPM_ENOTSPD;
  }
  set_error("CG breakdown: p^T E p <= 0 (E is not positive definite); column " +
            std::to_string(fl[F_COL]) + " within the first " + std::to_string(it_done) +
            " iterations, p.Ep=" + std::to_string(dbg[0]) + " r.z=" + std::to_string(dbg[1]));
  return CPM_ENOTSPD;
}

cpm_status finish_solver(cpm_system *s, int fc, int64_t cols, double tol, cpm_solve_info *info,
                         std::vector<int> &frame_iters, std::vector<double> &frame_res);

// CG with reliable updates on columns [0, fc) of the workspace block: b in
// ws.bx, start in ws.x (x_zero: it is zero; r_given: its residual is already
// in ws.r). On return ws.x holds q_b. Every decision is taken on the device
// (ctl_* kernels); the host enqueues batches of check_every iterations and
// looks at the status words of the batch before the one it has just
// enqueued.
template <typename T>
cpm_status run_solver(cpm_system *s, const T *E, int fc, const cpm_solve_opts &o,
                      cpm_solve_info *info, std::vector<int> &frame_iters,
                      std::vector<double> &frame_res, bool x_zero, bool r_given, bool sync) {
  const int64_t cols = round_up(fc, kColGroup);
  Solver<T> sv(s, E, cols, o.preconditioner == CPM_PRECOND_DC ? &s->pc : nullptr);
  hipStream_t st = s->stream;
  Workspace &w = s->ws;
  const bool f64 = sizeof(T) == 8;
  // reliable-update factor: the recursive residual may fall this far below
  // the last true residual before it is replaced (FP64: only at the end)
  const double ru = f64 ? 0.0 : std::min(0.5, std::max(1e-8, o.inner_tol));
  // FP32 keeps the search direction at a true-residual update (reliable
  // update). BF16: its matrix error (~2^-9 per entry) is too large for the
  // old direction to stay conjugate, so the iteration restarts from the true
  // residual (iterative refinement).
  const bool restart = sizeof(T) == 2;
  const double tol = o.tol;
  sv.tol = tol;
  sv.ru = ru;

  // |b|^2 and the start residual
  hipLaunchKernelGGL(sumsq_kernel, sv.grid(), dim3(RED_THREADS), 0, st, sv.b, sv.ld, sv.n,
                     (int)cols, sv.partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.partial, sv.nblk,
                     (int)cols, sv.scal, (int)S_BN2, nullptr);
  if (x_zero || r_given) {
    // r = b (zero start) or the start's FP64 residual packed by the caller
    if (x_zero)
      CPM_HIP_CHECK(hipMemcpyAsync(sv.r, sv.b, sizeof(double) * sv.ld * cols,
                                   hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(sumsq_kernel, sv.grid(), dim3(RED_THREADS), 0, st, sv.r, sv.ld, sv.n,
                       (int)cols, sv.partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.partial, sv.nblk,
                       (int)cols, sv.scal, (int)S_RR, nullptr);
  } else {
    CPM_HIP_CHECK(sv.true_residual(nullptr));
  }
  if (!x_zero) {
    hipLaunchKernelGGL(start_energy_kernel, sv.grid(), dim3(RED_THREADS), 0, st, sv.x, sv.b, sv.r,
                       sv.ld, sv.n, (int)cols, sv.partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.partial, sv.nblk,
                       (int)cols, sv.scal, (int)S_EN, nullptr);
  }
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.scal, (int)cols, fc,
                     x_zero ? 1 : 0, tol, sv.flags);
  if (!x_zero)
    hipLaunchKernelGGL(fallback_kernel, sv.grid(), dim3(RED_THREADS), 0, st, sv.x, sv.r, sv.b,
                       sv.scal, sv.ld, sv.n, (int)cols);
  sv.slot = 0;
  CPM_HIP_CHECK(sv.refresh(true, nullptr));

  const int check = std::max(1, o.check_every);
  int it = 0, pending = -1, batch = 0;
  auto status_of = [&](int slot) { return w.hstat + slot * F_NWORDS; };
  auto finished = [](const int *fl) { return fl[F_BREAK] || fl[F_NONFINITE] || fl[F_ANY] == 0; };
  auto rmax_of = [](const int *fl) {
    double v;
    std::memcpy(&v, fl + F_RMAX, sizeof(v));
    return v;
  };
  double rhist[2] = {0.0, 0.0};   // largest recursive residual of the last two batches read
  while (it < o.max_iter) {
    const int todo = std::min(check, o.max_iter - it);
    for (int k = 0; k < todo; ++k) CPM_HIP_CHECK(sv.iterate());
    it += todo;
    hipLaunchKernelGGL(ctl_check_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.scal, (int)cols, it,
                       todo, o.max_iter, tol, ru, sv.flags);
    CPM_HIP_CHECK(sv.true_residual(sv.need(), false));
    hipLaunchKernelGGL(ctl_update_kernel, dim3(1), dim3(MAX_COLS), 0, st, sv.partial, sv.nblk,
                       sv.scal, (int)cols, fc,
                       tol, sv.flags);
    CPM_HIP_CHECK(sv.refresh(restart, sv.need()));
    const int slot = batch % kStatusSlots;
    CPM_HIP_CHECK(hipMemcpyAsync(status_of(slot), sv.flags, sizeof(int) * F_NWORDS,
                                 hipMemcpyDeviceToHost, st));
    CPM_HIP_CHECK(hipEventRecord(w.ev[slot], st));
    ++batch;
    // the previous batch's status: stop enqueuing once nothing is active
    if (pending >= 0) {
      CPM_HIP_CHECK(hipEventSynchronize(w.ev[pending]));
      const int *fl = status_of(pending);
      if (finished(fl)) break;
      rhist[0] = rhist[1];
      rhist[1] = rmax_of(fl);
      // when the batch just enqueued is expected to reach the tolerance (its
      // residual extrapolated from the last two), read its status before
      // enqueuing another one, which would only run gated off
      if (rhist[0] > 0.0 && rhist[1] * (rhist[1] / rhist[0]) <= 0.5 * tol) {
        CPM_HIP_CHECK(hipEventSynchronize(w.ev[slot]));
        const int *fl2 = status_of(slot);
        if (finished(fl2)) break;
        rhist[0] = rhist[1];
        rhist[1] = rmax_of(fl2);
        pending = -1;
        continue;
      }
    }
    pending = slot;
  }
  // final state into pinned host memory; the caller may enqueue more work
  // (the projection) before the one synchronisation, then call finish_solver
  CPM_HIP_CHECK(hipMemcpyAsync(w.hfin, sv.scal, sizeof(double) * S_NFIELDS * cols,
                               hipMemcpyDeviceToHost, st));
  CPM_HIP_CHECK(hipMemcpyAsync(w.hfl, sv.flags, sizeof(int) * F_NWORDS, hipMemcpyDeviceToHost, st));
  w.hit = it;
  if (!sync) return CPM_OK;
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  return finish_solver(s, fc, cols, tol, info, frame_iters, frame_res);
}

// The outcome of the last solve from the pinned final state (after the
// stream has been synchronised).
cpm_status finish_solver(cpm_system *s, int fc, int64_t cols, double tol, cpm_solve_info *info,
                         std::vector<int> &frame_iters, std::vector<double> &frame_res) {
  const double *hs = s->ws.hfin;
  const int *fl = s->ws.hfl;
  if (fl[F_BREAK]) return breakdown_error(s->ws.hit, fl);
  if (fl[F_NONFINITE]) {
    set_error("CG produced a non-finite residual");
    return CPM_ENOTSPD;
  }
  int iters = 0;
  double init_res = 0.0;
  for (int c = 0; c < fc; ++c) {
    frame_iters[c] = (int)hs[S_IT * cols + c];
    frame_res[c] = hs[S_RES * cols + c];
    iters = std::max(iters, frame_iters[c]);
    init_res = std::max(init_res, hs[S_INIT * cols + c]);
  }
  if (info) {
    info->initial_rel_resid = std::max(info->initial_rel_resid, init_res);
    if (fl[F_FELLBACK]) info->fell_back = 1;
    info->iterations = std::max(info->iterations, iters);
    info->outer = std::max(info->outer, fl[F_UPDATES]);
    for (int c = 0; c < fc; ++c) info->max_rel_resid = std::max(info->max_rel_resid, frame_res[c]);
  }
  for (int c = 0; c < fc; ++c)
    if (frame_res[c] > tol) {
      set_error("CG did not reach the tolerance within max_iter");
      return CPM_ENOTCONV;
    }
  return CPM_OK;
}

// sync = false: the final state is only enqueued; synchronise the stream,
// then call finish_solver
cpm_status solve_columns(cpm_system *s, int fc, const cpm_solve_opts &o, cpm_solve_info *info,
                         std::vector<int> &frame_iters, std::vector<double> &frame_res,
                         bool x_zero, bool r_given = false, bool sync = true) {
  switch (o.precision) {
    case CPM_PREC_F64:
      return run_solver<double>(s, s->E64, fc, o, info, frame_iters, frame_res, x_zero, r_given,
                                sync);
    case CPM_PREC_F32:
      return run_solver<float>(s, s->E32, fc, o, info, frame_iters, frame_res, x_zero, r_given,
                               sync);
    default:
      return run_solver<uint16_t>(s, s->E16, fc, o, info, frame_iters, frame_res, x_zero,
                                  r_given, sync);
  }
}

}  // namespace

// slices of the Z^T-side coarse product: about 1024 workgroups of
// kCoarseAlign patches, at least 64 atoms and a multiple of 16 per slice
void coarse_slices(int64_t ld, int64_t mp, int &ks, int64_t &kslice) {
  const int64_t pw = std::max<int64_t>(1, mp / kCoarseAlign);
  int64_t want = std::max<int64_t>(1, (1024 + pw - 1) / pw);
  want = std::min<int64_t>(want, std::max<int64_t>(1, ld / 64));
  kslice = round_up((ld + want - 1) / want, 16);
  ks = (int)((ld + kslice - 1) / kslice);
}

void release_workspace(cpm_system *s) {
  s->device_bytes -= (int64_t)s->ws.bytes;
  free_workspace(s->ws);
}

hipError_t launch_diag_inverse(hipStream_t st, const double *E, int64_t n, int64_t ld,
                               double *dinv) {
  hipLaunchKernelGGL(diag_inverse_kernel, elem_grid(ld), dim3(256), 0, st, E, n, ld, dinv);
  return hipGetLastError();
}

cpm_status solve_dprime(cpm_system *s, double tol, int max_iter) {
  t_prof = &s->prof;
  t_n = s->n;
  cpm_status stt = ensure_workspace(s, kColGroup);
  if (stt != CPM_OK) return stt;
  const int64_t ld = s->ld;
  // b = 1 on the n atoms (column 0), zero elsewhere
  std::vector<double> ones(ld * kColGroup, 0.0);
  for (int64_t i = 0; i < s->n; ++i) ones[i] = 1.0;
  CPM_HIP_CHECK(hipMemcpyAsync(s->ws.bx, ones.data(), sizeof(double) * ones.size(),
                               hipMemcpyHostToDevice, s->stream));
  CPM_HIP_CHECK(hipMemsetAsync(s->ws.x, 0, sizeof(double) * ld * kColGroup, s->stream));
  cpm_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  o.tol = tol;
  o.max_iter = max_iter;
  o.precision = CPM_PREC_F64;
  o.check_every = 16;
  o.preconditioner = s->pc.ready ? CPM_PRECOND_DC : CPM_PRECOND_JACOBI;
  std::vector<int> it(kColGroup, 0);
  std::vector<double> res(kColGroup, 0.0);
  stt = solve_columns(s, 1, o, nullptr, it, res, true);
  if (stt != CPM_OK) return stt;
  CPM_HIP_CHECK(hipMemcpyAsync(s->dprime, s->ws.x, sizeof(double) * ld, hipMemcpyDeviceToDevice,
                               s->stream));
  std::vector<double> dp(s->n);
  CPM_HIP_CHECK(hipMemcpyAsync(dp.data(), s->dprime, sizeof(double) * s->n, hipMemcpyDeviceToHost,
                               s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  double c = 0.0;
  for (double v : dp) c += v;
  if (!(c > 0.0) || !std::isfinite(c)) {
    set_error("neutralising vector: 1^T E^-1 1 is not positive");
    return CPM_ENOTSPD;
  }
  s->c_ele = c;
  for (double &v : dp) v /= c;
  dp.resize(ld, 0.0);
  CPM_HIP_CHECK(hipMemcpyAsync(s->dvec, dp.data(), sizeof(double) * ld, hipMemcpyHostToDevice,
                               s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status solve_block(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                       const cpm_solve_opts &o, double *q_out_dev, cpm_solve_info *info,
                       const double *x0_dev, bool project, const double *r0_dev) {
  t_prof = &s->prof;
  t_n = s->n;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t ld = s->ld, n = s->n;
  hipStream_t st = s->stream;
  cpm_status result = CPM_OK;
  for (int64_t f0 = 0; f0 < f; f0 += MAX_COLS) {
    const int fc = (int)std::min<int64_t>(MAX_COLS, f - f0);
    const int64_t cols = round_up(fc, kColGroup);
    cpm_status stt = ensure_workspace(s, cols);
    if (stt != CPM_OK) return stt;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)cols), dim3(256),
                       0, st, b_dev + f0 * n, n, (int64_t)fc, s->ws.bx, ld, cols);
    if (x0_dev) {
      hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)cols),
                         dim3(256), 0, st, x0_dev + f0 * n, n, (int64_t)fc, (double *)s->ws.x, ld,
                         cols);
      if (r0_dev)
        hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)cols),
                           dim3(256), 0, st, r0_dev + f0 * n, n, (int64_t)fc, (double *)s->ws.r,
                           ld, cols);
    } else {
      hipLaunchKernelGGL(zero_kernel, elem_grid(ld * cols), dim3(256), 0, st, (double *)s->ws.x,
                         ld * cols);
    }
    std::vector<int> fit(cols, 0);
    std::vector<double> fres(cols, 0.0);
    // the solve, its final state and the projection are enqueued before
    // the one synchronisation of this block
    stt = solve_columns(s, fc, o, info, fit, fres, x0_dev == nullptr,
                        x0_dev != nullptr && r0_dev != nullptr, false);
    if (stt != CPM_OK) return stt;
    double *sum_err = s->ws.hfin + S_NFIELDS * MAX_COLS;   // pinned
    if (project) {
      hipLaunchKernelGGL(project_kernel, dim3((unsigned)fc), dim3(RED_THREADS), 0, st,
                         (const double *)s->ws.x, ld, n, s->dvec, qsol_dev + f0,
                         q_out_dev + f0 * n, s->ws.sum_err);
      CPM_HIP_CHECK(hipMemcpyAsync(sum_err, s->ws.sum_err, sizeof(double) * fc,
                                   hipMemcpyDeviceToHost, st));
    } else {
      CPM_HIP_CHECK(hipMemcpy2DAsync(q_out_dev + f0 * n, sizeof(double) * n, s->ws.x,
                                     sizeof(double) * ld, sizeof(double) * n, fc,
                                     hipMemcpyDeviceToDevice, st));
    }
    CPM_HIP_CHECK(hipStreamSynchronize(st));
    stt = finish_solver(s, fc, cols, o.tol, info, fit, fres);
    if (stt != CPM_OK && stt != CPM_ENOTCONV) return stt;
    if (stt == CPM_ENOTCONV) result = CPM_ENOTCONV;
    if (info) {
      for (int c = 0; c < fc; ++c) {
        if (project) info->max_abs_sum_q = std::max(info->max_abs_sum_q, sum_err[c]);
        if (info->frame_iters) info->frame_iters[f0 + c] = fit[c];
        if (info->frame_rel_resid) info->frame_rel_resid[f0 + c] = fres[c];
      }
    }
  }
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  if (info)
    info->solve_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return result;
}

cpm_status matvec_cols(cpm_system *s, int precision, const double *p_dev, int64_t f,
                       double *v_dev) {
  return matvec_cols_with(s, precision, nullptr, p_dev, f, v_dev);
}

cpm_status matvec_cols_with(cpm_system *s, int precision, const double *M64, const double *p_dev,
                            int64_t f, double *v_dev) {
  t_prof = &s->prof;
  t_n = s->n;
  if (M64 == nullptr) M64 = s->E64;
  hipStream_t st = s->stream;
  const int64_t ld = s->ld, n = s->n;
  for (int64_t f0 = 0; f0 < f; f0 += MAX_COLS) {
    const int fc = (int)std::min<int64_t>(MAX_COLS, f - f0);
    const int64_t cols = round_up(fc, kColGroup);
    cpm_status stt = ensure_workspace(s, cols);
    if (stt != CPM_OK) return stt;
    double *in = s->ws.bres;   // packed input (double)
    double *out = (double *)s->ws.v;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)cols), dim3(256),
                       0, st, p_dev + f0 * n, n, (int64_t)fc, in, ld, cols);
    int sl = 0;
    double *res = s->ws.bx;   // summed product (double)
    if (precision == CPM_PREC_F64) {
      CPM_HIP_CHECK(launch_matvec<double>(st, M64, ld, cols, in, out, nullptr, sl));
      hipLaunchKernelGGL(sum_slices_kernel<double>, elem_grid(ld * cols), dim3(256), 0, st,
                         (const double *)out, sl, ld * cols, res, ld * cols);
    } else {
      float *pf = (float *)s->ws.pf, *vf = (float *)s->ws.vf;
      hipLaunchKernelGGL(f64_to_f32_kernel, elem_grid(ld * cols), dim3(256), 0, st, in, pf,
                         ld * cols);
      if (precision == CPM_PREC_F32)
        CPM_HIP_CHECK(launch_matvec<float>(st, s->E32, ld, cols, pf, vf, nullptr, sl));
      else
        CPM_HIP_CHECK(launch_matvec<uint16_t>(st, s->E16, ld, cols, pf, vf, nullptr, sl));
      hipLaunchKernelGGL(sum_slices_kernel<float>, elem_grid(ld * cols), dim3(256), 0, st,
                         (const float *)vf, sl, ld * cols, res, ld * cols);
    }
    out = res;
    CPM_HIP_CHECK(hipMemcpy2DAsync(v_dev + f0 * n, sizeof(double) * n, out, sizeof(double) * ld,
                                   sizeof(double) * n, fc, hipMemcpyDeviceToDevice, st));
  }
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

cpm_status precond_cols(cpm_system *s, const double *r_dev, int64_t f, double *z_dev) {
  hipStream_t st = s->stream;
  const int64_t ld = s->ld, n = s->n;
  for (int64_t f0 = 0; f0 < f; f0 += MAX_COLS) {
    const int fc = (int)std::min<int64_t>(MAX_COLS, f - f0);
    const int64_t cols = round_up(fc, kColGroup);
    cpm_status stt = ensure_workspace(s, cols);
    if (stt != CPM_OK) return stt;
    double *in = s->ws.rt, *out = s->ws.bx;
    hipLaunchKernelGGL(rows_kernel, dim3((unsigned)(ld / RT_ROWS), (unsigned)(cols / kColGroup)),
                       dim3(RED_THREADS), 0, st, r_dev + f0 * n, n, n, fc, in, ld,
                       (const int *)nullptr);
    launch_precond<double>(st, s, s->pc, in, r_dev + f0 * n, n, fc, out, (double *)nullptr, cols,
                           nullptr, 0, nullptr, false, nullptr);
    CPM_HIP_CHECK(hipMemcpy2DAsync(z_dev + f0 * n, sizeof(double) * n, out, sizeof(double) * ld,
                                   sizeof(double) * n, fc, hipMemcpyDeviceToDevice, st));
  }
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

}  // namespace cpm
