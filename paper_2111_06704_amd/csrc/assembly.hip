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
//                        (v_mfma_f64_16x16x4f64), mirrored into the upper half.
//   finalize_kernel      adds R, c0 and the diagonal; writes FP32 / BF16 copies.
#include "cpm_internal.h"

#include <cmath>

namespace cpm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SY_TILE = 128;   // output tile edge
constexpr int SY_KB = 16;      // k depth per LDS stage (doubles)

__global__ void phase_matrix_kernel(const double *__restrict__ pos, int64_t n, int64_t nrows,
                                    double inv_lx, double inv_ly, double inv_lz,
                                    const int32_t *__restrict__ kn, const double *__restrict__ kw,
                                    int64_t k0, int64_t kc, int64_t kc_pad, int64_t lda,
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
  *reinterpret_cast<double2 *>(A + i * lda + 2 * kk) = v;
}

// Tile index t in [0, T(T+1)/2) -> (ti >= tj).
__device__ inline void tri_index(int64_t t, int64_t &ti, int64_t &tj) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

// 256 threads = 4 waves; wave (wr, wc) computes the 64x64 sub-tile
// rows wr*64.., cols wc*64.. as 4x4 blocks of 16x16 MFMA outputs.
__global__ __launch_bounds__(256) void syrk_lower_kernel(const double *__restrict__ A, int64_t lda,
                                                         int64_t kdim, double *__restrict__ E,
                                                         int64_t lde, int accumulate) {
  __shared__ double sI[SY_KB][SY_TILE + 2];
  __shared__ double sJ[SY_KB][SY_TILE + 2];
  int64_t ti, tj;
  tri_index(blockIdx.x, ti, tj);
  const int64_t I0 = ti * SY_TILE, J0 = tj * SY_TILE;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const int lrow = tid >> 1, lhalf = tid & 1;   // loader: row, which 8 of 16
  const double *gI = A + (I0 + lrow) * lda + lhalf * 8;
  const double *gJ = A + (J0 + lrow) * lda + lhalf * 8;

  for (int64_t k0 = 0; k0 < kdim; k0 += SY_KB) {
    double4 vi0 = *reinterpret_cast<const double4 *>(gI + k0);
    double4 vi1 = *reinterpret_cast<const double4 *>(gI + k0 + 4);
    double4 vj0 = *reinterpret_cast<const double4 *>(gJ + k0);
    double4 vj1 = *reinterpret_cast<const double4 *>(gJ + k0 + 4);
    const int kb = lhalf * 8;
    sI[kb + 0][lrow] = vi0.x; sI[kb + 1][lrow] = vi0.y; sI[kb + 2][lrow] = vi0.z; sI[kb + 3][lrow] = vi0.w;
    sI[kb + 4][lrow] = vi1.x; sI[kb + 5][lrow] = vi1.y; sI[kb + 6][lrow] = vi1.z; sI[kb + 7][lrow] = vi1.w;
    sJ[kb + 0][lrow] = vj0.x; sJ[kb + 1][lrow] = vj0.y; sJ[kb + 2][lrow] = vj0.z; sJ[kb + 3][lrow] = vj0.w;
    sJ[kb + 4][lrow] = vj1.x; sJ[kb + 5][lrow] = vj1.y; sJ[kb + 6][lrow] = vj1.z; sJ[kb + 7][lrow] = vj1.w;
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < SY_KB / 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = sI[ks * 4 + lg][wr * 64 + q * 16 + lr];
        b[q] = sJ[ks * 4 + lg][wc * 64 + q * 16 + lr];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }

  // v_mfma_f64_16x16x4f64 output: D[i][j] lives in lane j + 16 * (i % 4),
  // register i / 4 (row i = 4 * register + lane / 16).
  const bool diag_tile = (ti == tj);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = I0 + wr * 64 + x * 16 + 4 * v + lg;
        const int64_t col = J0 + wc * 64 + y * 16 + lr;
        const double val = acc[x][y][v];
        if (diag_tile && col > row) continue;
        double *p1 = E + row * lde + col;
        double *p2 = E + col * lde + row;
        if (accumulate) {
          *p1 += val;
          if (row != col) *p2 += val;
        } else {
          *p1 = val;
          if (row != col) *p2 = val;
        }
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

__global__ void finalize_kernel(const double *__restrict__ pos, const double *__restrict__ width,
                                int64_t n, int64_t ld, double lx, double ly, double lz,
                                double beta, double rcut, double c0, double slab,
                                double *__restrict__ E64, float *__restrict__ E32,
                                uint16_t *__restrict__ E16, int64_t jblocks) {
  const int64_t i = (int64_t)blockIdx.x / jblocks;
  const int64_t j = ((int64_t)blockIdx.x % jblocks) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  // canonical order so that (i, j) and (j, i) evaluate identically
  const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
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
        if (i == j && a == 0 && b == 0 && c == 0) continue;
        const double ez = dz + (double)c * lz;
        const double d2 = exy + ez * ez;
        if (d2 < rc2) {
          const double d = sqrt(d2);
          real += (erfc(beta * d) - erfc(aij * d)) / d;
        }
      }
    }
  }
  const int64_t idx = i * ld + j;
  double e = E64[idx] + real + c0;
  // slab geometry (Eq. 39 in its definite form): (4 pi / V) z_i z_j
  if (slab != 0.0) e += slab * (pos[3 * lo + 2] * pos[3 * hi + 2]);
  if (i == j) {
    // Gaussian self-energy 2 a_ii / sqrt(pi), a_ii = a_i / sqrt(2) (Eq. 6);
    // a point charge (a_i = inf) has none (end of Sec. II.C).
    const double aii = wl * 0.70710678118654752440;
    e -= 2.0 * beta * 0.56418958354775628695;   // 1/sqrt(pi)
    if (isfinite(aii)) e += 2.0 * aii * 0.56418958354775628695;
  }
  E64[idx] = e;
  if (E32) E32[idx] = (float)e;
  if (E16) E16[idx] = f64_to_bf16_rne(e);
}

}  // namespace

hipError_t launch_phase_matrix(hipStream_t st, const double *pos, int64_t n, int64_t ld,
                               const double box[3], const int32_t *kn, const double *kw,
                               int64_t k0, int64_t kc, int64_t lda, double *A) {
  const int64_t kc_pad = lda / 2;
  dim3 blk(64, 4);
  dim3 grd((unsigned)((kc_pad + 63) / 64), (unsigned)((ld + 3) / 4));
  hipLaunchKernelGGL(phase_matrix_kernel, grd, blk, 0, st, pos, n, ld, 1.0 / box[0], 1.0 / box[1],
                     1.0 / box[2], kn, kw, k0, kc, kc_pad, lda, A);
  return hipGetLastError();
}

hipError_t launch_syrk_lower(hipStream_t st, const double *A, int64_t lda, int64_t kdim,
                             int64_t ld, double *E, int64_t lde, bool accumulate,
                             hipEvent_t ev_start, hipEvent_t ev_stop) {
  const int64_t T = ld / SY_TILE;
  const int64_t tiles = T * (T + 1) / 2;
  if (kdim % SY_KB != 0 || ld % SY_TILE != 0) return hipErrorInvalidValue;
  hipExtLaunchKernelGGL(syrk_lower_kernel, dim3((unsigned)tiles), dim3(256), 0, st, ev_start,
                        ev_stop, 0, A, lda, kdim, E, lde, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const double *pos, const double *width, int64_t n,
                           int64_t ld, const double box[3], double beta, double rcut, bool slab,
                           double *E64, float *E32, uint16_t *E16) {
  const double vol = box[0] * box[1] * box[2];
  const double c0 = -M_PI / (vol * beta * beta);
  const double cs = slab ? 4.0 * M_PI / vol : 0.0;
  const int64_t jblocks = (n + 255) / 256;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)(jblocks * n)), dim3(256), 0, st, pos, width,
                     n, ld, box[0], box[1], box[2], beta, rcut, c0, cs, E64, E32, E16, jblocks);
  return hipGetLastError();
}

}  // namespace cpm
