// Assembly of the Gaussian Ewald matrix E (Sec. II.C, Eq. 22-23).
//
// E = A A^T + R + c0 + diag, where
//   A[i, 2k] = sqrt(w_k) cos(K_k . r_i), A[i, 2k+1] = sqrt(w_k) sin(K_k . r_i)
//   over the half-space k-vectors (w_k already doubled), so that
//   (A A^T)_ij = sum_k w_k cos(K_k . (r_i - r_j)), the reciprocal sum;
//   R_ij = sum over images with d < rcut of [erfc(beta d) - erfc(a_ij d)] / d
//   (n = 0 excluded on the diagonal), c0 = -pi / (V beta^2), and the diagonal
//   adds -2 beta / sqrt(pi) + 2 a_ii / sqrt(pi).
//
// Kernels:
//   phase_matrix_kernel  A for a chunk of k-vectors (FP64, sincospi of the
//                        fractional phase n . (r / L), reduced to [-1/2, 1/2]).
//   syrk_lower_kernel    lower-triangular 128x128 tiles of A A^T with FP64 MFMA
//                        (v_mfma_f64_16x16x4f64), accumulated over k chunks.
//   finalize_kernel      adds R, c0 and the diagonal to the lower triangle,
//                        mirrors it into the upper one; FP32 / BF16 copies.
#include "cpm_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace cpm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SY_TILE = 128;   // output tile edge
constexpr int SY_KB = 16;      // k depth per LDS stage (doubles)
constexpr int SY_LDP = SY_TILE + 16;   // LDS row pitch (doubles)
constexpr int SY_GROUP = 8;    // tiles per super-block edge in the tile order

// A is stored in column blocks of SY_KB: entry (i, k) at
// (k / SY_KB) * (nrows * SY_KB) + i * SY_KB + k % SY_KB, so that one LDS
// stage of a 128-row tile is a contiguous 16 KB piece of memory.
__global__ void phase_matrix_kernel(const double *__restrict__ pos, int64_t n, int64_t nrows,
                                    double inv_lx, double inv_ly, double inv_lz,
                                    const int32_t *__restrict__ kn, const double *__restrict__ kw,
                                    int64_t k0, int64_t kc, int64_t kc_pad,
                                    double *__restrict__ A) {
  const int64_t kk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  if (kk >= kc_pad || i >= nrows) return;
  double c = 0.0, s = 0.0;
  if (i < n && kk < kc) {
    const int64_t k = k0 + kk;
    const double ux = pos[3 * i] * inv_lx, uy = pos[3 * i + 1] * inv_ly,
                 uz = pos[3 * i + 2] * inv_lz;
    double t = (double)kn[3 * k] * ux + (double)kn[3 * k + 1] * uy + (double)kn[3 * k + 2] * uz;
    t -= rint(t);
    const double sw = sqrt(kw[k]);
    sincospi(2.0 * t, &s, &c);
    c *= sw;
    s *= sw;
  }
  double2 v;
  v.x = c;
  v.y = s;
  const int64_t col = 2 * kk;
  *reinterpret_cast<double2 *>(A + (col / SY_KB) * (nrows * SY_KB) + i * SY_KB + col % SY_KB) = v;
}

// Tile index t in [0, T(T+1)/2) -> (ti >= tj).
__device__ inline void tri_index(int64_t t, int64_t &ti, int64_t &tj) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

// Lower-triangular 128x128 tiles of A A^T. 256 threads = 4 waves; wave
// (wr, wc) computes the 64x64 sub-tile rows wr*64.., cols wc*64.. as 4x4
// blocks of 16x16 MFMA outputs. The k loop runs over LDS stages of SY_KB
// columns, double buffered: the global loads of stage s + 1 are in flight
// in registers while stage s is multiplied, so one barrier per stage.
// Tiles come from a host-ordered list (super-blocks of 8x8 tiles) and
// workgroup b takes list entry (b % 8) * per + b / 8: the hardware hands
// workgroups to the 8 XCDs round-robin, so each XCD walks a contiguous run
// of the list and its concurrent tiles share rows of A in its L2.
// The whole tile is written (diagonal tiles included); the upper triangle
// of E is filled from the lower one by finalize_kernel.
__global__ __launch_bounds__(256, 2) void syrk_lower_kernel(const double *__restrict__ A, int64_t nrows,
                                                         int64_t kdim,
                                                         const int32_t *__restrict__ tiles,
                                                         int64_t ntiles, int64_t per,
                                                         double *__restrict__ E, int64_t lde,
                                                         int accumulate) {
  __shared__ double sI[2][SY_KB][SY_LDP];
  __shared__ double sJ[2][SY_KB][SY_LDP];
  const int64_t b = blockIdx.x;
  const int64_t L = (b % 8) * per + b / 8;
  if (L >= ntiles) return;
  const int64_t I0 = (int64_t)tiles[2 * L] * SY_TILE, J0 = (int64_t)tiles[2 * L + 1] * SY_TILE;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};

  // loader: row lrow, k columns kb..kb+7 of the stage; a wave's loads are
  // 4 KB of contiguous memory (column-blocked A)
  const int lrow = tid >> 1, kb = (tid & 1) * 8;
  const int64_t bstride = nrows * SY_KB;
  const double *gI = A + (I0 + lrow) * SY_KB + kb;
  const double *gJ = A + (J0 + lrow) * SY_KB + kb;
  double4 vi0, vi1, vj0, vj1;
  auto gload = [&](int64_t k0) {
    const int64_t o = (k0 / SY_KB) * bstride;
    vi0 = *reinterpret_cast<const double4 *>(gI + o);
    vi1 = *reinterpret_cast<const double4 *>(gI + o + 4);
    vj0 = *reinterpret_cast<const double4 *>(gJ + o);
    vj1 = *reinterpret_cast<const double4 *>(gJ + o + 4);
  };
  auto sstore = [&](int buf) {
    sI[buf][kb + 0][lrow] = vi0.x; sI[buf][kb + 1][lrow] = vi0.y;
    sI[buf][kb + 2][lrow] = vi0.z; sI[buf][kb + 3][lrow] = vi0.w;
    sI[buf][kb + 4][lrow] = vi1.x; sI[buf][kb + 5][lrow] = vi1.y;
    sI[buf][kb + 6][lrow] = vi1.z; sI[buf][kb + 7][lrow] = vi1.w;
    sJ[buf][kb + 0][lrow] = vj0.x; sJ[buf][kb + 1][lrow] = vj0.y;
    sJ[buf][kb + 2][lrow] = vj0.z; sJ[buf][kb + 3][lrow] = vj0.w;
    sJ[buf][kb + 4][lrow] = vj1.x; sJ[buf][kb + 5][lrow] = vj1.y;
    sJ[buf][kb + 6][lrow] = vj1.z; sJ[buf][kb + 7][lrow] = vj1.w;
  };

  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < kdim; k0 += SY_KB) {
    const bool more = k0 + SY_KB < kdim;
    if (more) gload(k0 + SY_KB);
#pragma unroll
    for (int ks = 0; ks < SY_KB / 4; ++ks) {
      double a[4], c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = sI[buf][ks * 4 + lg][wr * 64 + q * 16 + lr];
        c[q] = sJ[buf][ks * 4 + lg][wc * 64 + q * 16 + lr];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], c[y], acc[x][y], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // v_mfma_f64_16x16x4f64 output: D[i][j] lives in lane j + 16 * (i % 4),
  // register i / 4 (row i = 4 * register + lane / 16); each register of a
  // block is 4 rows x 128 contiguous bytes.
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = I0 + wr * 64 + x * 16 + 4 * v + lg;
        const int64_t col = J0 + wc * 64 + y * 16 + lr;
        double *p = E + row * lde + col;
        *p = accumulate ? *p + acc[x][y][v] : acc[x][y][v];
      }
}

__device__ inline uint16_t f64_to_bf16_rne(double x) {
  // Round to float with round-to-odd (keeps a sticky bit), then to bf16 with
  // round-to-nearest-even: equal to a single RNE rounding of x.
  float f = __double2float_rz(x);
  uint32_t u = __float_as_uint(f);
  if ((double)f != x) u |= 1u;
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

__device__ inline int64_t iceil(double x) { return (int64_t)ceil(x); }
__device__ inline int64_t ifloor(double x) { return (int64_t)floor(x); }

// Real-space part of entry (i, j) of Eq. 22 (images with d < rcut; the n = 0
// image excluded for i == j), for the pair in canonical order lo <= hi.
__device__ inline double real_space_entry(const double *__restrict__ pos,
                                          const double *__restrict__ width, int64_t lo,
                                          int64_t hi, double lx, double ly, double lz,
                                          double beta, double rcut) {
  double dx = pos[3 * hi] - pos[3 * lo];
  double dy = pos[3 * hi + 1] - pos[3 * lo + 1];
  double dz = pos[3 * hi + 2] - pos[3 * lo + 2];
  dx -= lx * rint(dx / lx);
  dy -= ly * rint(dy / ly);
  dz -= lz * rint(dz / lz);
  const double wl = width[lo], wh = width[hi];
  const double aij = 1.0 / sqrt(1.0 / (wl * wl) + 1.0 / (wh * wh));
  const double rc2 = rcut * rcut;
  double real = 0.0;
  const int64_t xa = iceil((-rcut - dx) / lx), xb = ifloor((rcut - dx) / lx);
  const int64_t ya = iceil((-rcut - dy) / ly), yb = ifloor((rcut - dy) / ly);
  const int64_t za = iceil((-rcut - dz) / lz), zb = ifloor((rcut - dz) / lz);
  for (int64_t a = xa; a <= xb; ++a) {
    const double ex = dx + (double)a * lx;
    for (int64_t b = ya; b <= yb; ++b) {
      const double ey = dy + (double)b * ly;
      const double exy = ex * ex + ey * ey;
      if (exy >= rc2) continue;
      for (int64_t c = za; c <= zb; ++c) {
        if (lo == hi && a == 0 && b == 0 && c == 0) continue;
        const double ez = dz + (double)c * lz;
        const double d2 = exy + ez * ez;
        if (d2 < rc2) {
          const double d = sqrt(d2);
          real += (erfc(beta * d) - erfc(aij * d)) / d;
        }
      }
    }
  }
  return real;
}

constexpr int FZ_B = 64;   // finalize block edge

// One workgroup per lower 64x64 block (bi >= bj) of the padded ld x ld
// matrix. Each entry of the block's lower part takes the reciprocal sum the
// contraction left there and adds the real-space sum, c0, the Eq. 39 term
// and the diagonal terms; entries outside [0, n)^2 become 0. The block is
// written in place and, through an LDS transpose, to its mirror block
// above the diagonal, so both stores are row-contiguous and E is exactly
// symmetric. FP32 / BF16 copies are the round-to-nearest of the FP64 value.
__global__ __launch_bounds__(256) void finalize_kernel(
    const double *__restrict__ pos, const double *__restrict__ width,
    const double *__restrict__ rs_width, int64_t n, int64_t ld,
    double lx, double ly, double lz, double beta, double rcut, double c0, double slab,
    double *__restrict__ E64, float *__restrict__ E32, uint16_t *__restrict__ E16) {
  __shared__ double tile[FZ_B][FZ_B + 1];
  int64_t bi, bj;
  tri_index(blockIdx.x, bi, bj);
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int64_t j = bj * FZ_B + c;
  for (int r = r0; r < FZ_B; r += 4) {
    const int64_t i = bi * FZ_B + r;
    if (bi == bj && c > r) continue;   // upper half of a diagonal block: mirrored below
    double e = 0.0;
    if (i < n && j < n) {
      const int64_t idx = i * ld + j;
      e = E64[idx] + c0 + real_space_entry(pos, rs_width, j, i, lx, ly, lz, beta, rcut);
      // slab geometry (Eq. 39 in its definite form): (4 pi / V) z_i z_j
      if (slab != 0.0) e += slab * (pos[3 * j + 2] * pos[3 * i + 2]);
      if (i == j) {
        // Gaussian self-energy 2 a_ii / sqrt(pi), a_ii = a_i / sqrt(2) (Eq. 6);
        // a point charge (a_i = inf) has none (end of Sec. II.C); the
        // point-charge simplification keeps it (Sec. III.C)
        const double aii = width[i] * 0.70710678118654752440;
        e -= 2.0 * beta * 0.56418958354775628695;   // 1/sqrt(pi)
        if (isfinite(aii)) e += 2.0 * aii * 0.56418958354775628695;
      }
    }
    const int64_t idx = i * ld + j;
    E64[idx] = e;
    if (E32) E32[idx] = (float)e;
    if (E16) E16[idx] = f64_to_bf16_rne(e);
    tile[r][c] = e;
  }
  __syncthreads();
  // mirror: entry (bj*64 + r, bi*64 + c) = tile[c][r]
  const int64_t jm = bi * FZ_B + c;
  for (int r = r0; r < FZ_B; r += 4) {
    if (bi == bj && c <= r) continue;
    const int64_t idx = (bj * FZ_B + r) * ld + jm;
    const double e = tile[c][r];
    E64[idx] = e;
    if (E32) E32[idx] = (float)e;
    if (E16) E16[idx] = f64_to_bf16_rne(e);
  }
}

}  // namespace

hipError_t launch_phase_matrix(hipStream_t st, const double *pos, int64_t n, int64_t ld,
                               const double box[3], const int32_t *kn, const double *kw,
                               int64_t k0, int64_t kc, int64_t kdim, double *A) {
  // kdim = 2 * (k-vectors per chunk), a multiple of SY_KB; columns of k-vectors
  // beyond kc are zero
  if (kdim % SY_KB != 0 || 2 * kc > kdim) return hipErrorInvalidValue;
  const int64_t kc_pad = kdim / 2;
  dim3 blk(64, 4);
  dim3 grd((unsigned)((kc_pad + 63) / 64), (unsigned)((ld + 3) / 4));
  hipLaunchKernelGGL(phase_matrix_kernel, grd, blk, 0, st, pos, n, ld, 1.0 / box[0], 1.0 / box[1],
                     1.0 / box[2], kn, kw, k0, kc, kc_pad, A);
  return hipGetLastError();
}

std::vector<int32_t> syrk_tile_order(int64_t T) {
  // lower-triangular tiles in super-blocks of SY_GROUP x SY_GROUP tiles
  std::vector<int32_t> t;
  t.reserve((size_t)(T * (T + 1)));
  for (int64_t SI = 0; SI < T; SI += SY_GROUP)
    for (int64_t SJ = 0; SJ <= SI; SJ += SY_GROUP)
      for (int64_t ti = SI; ti < std::min<int64_t>(SI + SY_GROUP, T); ++ti)
        for (int64_t tj = SJ; tj < std::min<int64_t>(SJ + SY_GROUP, T) && tj <= ti; ++tj) {
          t.push_back((int32_t)ti);
          t.push_back((int32_t)tj);
        }
  return t;
}

hipError_t launch_syrk_lower(hipStream_t st, const double *A, int64_t kdim,
                             const int32_t *tiles, int64_t ld, double *E, int64_t lde,
                             bool accumulate, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const int64_t T = ld / SY_TILE;
  const int64_t ntiles = T * (T + 1) / 2;
  const int64_t per = (ntiles + 7) / 8;
  if (kdim % SY_KB != 0 || kdim < SY_KB || ld % SY_TILE != 0) return hipErrorInvalidValue;
  hipExtLaunchKernelGGL(syrk_lower_kernel, dim3((unsigned)(8 * per)), dim3(256), 0, st, ev_start,
                        ev_stop, 0, A, ld, kdim, tiles, ntiles, per, E, lde, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const double *pos, const double *width,
                           const double *rs_width, int64_t n, int64_t ld, const double box[3],
                           double beta, double rcut, bool slab, double *E64, float *E32,
                           uint16_t *E16) {
  const double vol = box[0] * box[1] * box[2];
  const double c0 = -M_PI / (vol * beta * beta);
  const double cs = slab ? 4.0 * M_PI / vol : 0.0;
  if (ld % FZ_B != 0) return hipErrorInvalidValue;
  const int64_t B = ld / FZ_B;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)(B * (B + 1) / 2)), dim3(256), 0, st, pos,
                     width, rs_width, n, ld, box[0], box[1], box[2], beta, rcut, c0, cs, E64,
                     E32, E16);
  return hipGetLastError();
}

}  // namespace cpm
