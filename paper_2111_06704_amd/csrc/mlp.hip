// Learned CG starting point: a per-atom network 26 -> 64 -> 64 -> 1 (SiLU).
//
// Inputs of atom i in a frame with right-hand side b (Eq. 25):
//   [ (b_i - mean b) / b_scale, layer_i / (n_layers - 1),
//     (b_j - mean b) / b_scale for its 12 nearest electrode neighbours j,
//     r_ij / r_scale for the same neighbours ].
// Output y_i; predicted charge q0_i = q_scale * y_i.
//
// Warm start of the two-step solve (Eq. 29-35): q0 is shifted to
// sum(q0) = -Q_sol; then mu0 = mean(b - E q0) estimates the Lagrange shift
// of Eq. 29, and q_b0 = q0 + mu0 d' (d' = E^-1 1, S9) starts E q_b = b.
// The same construction with q0 = q_chi (the solution without electrolyte)
// is the non-learned warm start.
//
// Training: mean squared error on q / q_scale, gradient by a hand-written
// backward pass (per 64-row tile in LDS), fixed-order reduction over tiles,
// and the Adam update (Kingma & Ba 2015).
#include "cpm_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

namespace cpm {
namespace {

constexpr int NIN = CPM_MLP_IN;
constexpr int NH = CPM_MLP_HIDDEN;
constexpr int NP = CPM_MLP_NPARAM;
constexpr int NNB = 12;
constexpr int TT = 256;         // threads per tile block
// parameter offsets
constexpr int OW1 = 0, OB1 = OW1 + NIN * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH;

__device__ inline float sigm(float a) { return 1.0f / (1.0f + __expf(-a)); }

// per-frame mean of b (fixed-order block reduction)
__global__ __launch_bounds__(256) void frame_mean_kernel(const double *__restrict__ b, int64_t n,
                                                         double *__restrict__ mean) {
  __shared__ double red[256];
  const int64_t f = blockIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) s += b[f * n + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[f] = red[0] / (double)n;
}

// features of rows; row r is (frame, atom) = (id / n, id % n) with id =
// rows_idx ? rows_idx[r] : r0 + r.
__global__ void features_kernel(const double *__restrict__ b, const double *__restrict__ mean,
                                int64_t n, const int32_t *__restrict__ nbr,
                                const float *__restrict__ nbr_r, const int32_t *__restrict__ layer,
                                float inv_layers, float inv_bs, float inv_rs,
                                const int64_t *__restrict__ rows_idx, int64_t r0, int64_t rows,
                                float *__restrict__ feat) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t id = rows_idx ? rows_idx[r] : r0 + r;
  const int64_t f = id / n, i = id % n;
  const double mb = mean[f];
  const double *bf = b + f * n;
  float *o = feat + r * NIN;
  o[0] = (float)((bf[i] - mb) * (double)inv_bs);
  o[1] = (float)layer[i] * inv_layers;
#pragma unroll
  for (int k = 0; k < NNB; ++k) {
    o[2 + k] = (float)((bf[nbr[i * NNB + k]] - mb) * (double)inv_bs);
    o[2 + NNB + k] = nbr_r[i * NNB + k] * inv_rs;
  }
}

// Training gradient on the FP32 matrix cores (v_mfma_f32_16x16x4f32 with
// the operand layout of the inference kernel below: lane (lr, lg) supplies
// A[row lr][k + lg] and B[k + lg][column lr] and receives
// D[row 4 lg + v][column lr]). One workgroup per tile of GR rows; writes
// the tile's gradient (sum over its rows of d/dtheta of (y - t)^2 /
// rows_total) and its loss sum. Products per tile:
//   a1 = X W1 (+ b1), a2 = silu(a1) W2 (+ b2): wave w takes rows 16 w ..;
//   dW2 = silu(a1)^T G2 and dW1 = X^T G1: contractions over the tile's rows;
//   G1 = (G2 W2^T) o silu'(a1): wave w takes rows 16 w ..;
// the output layer (one unit) and the bias sums on the vector units, in a
// fixed order. Rows past the end enter with zero error, so they add nothing.
constexpr int GR = 64;                    // rows per gradient tile (16 per wavefront)
constexpr int NINP = (NIN + 3) / 4 * 4;   // input width padded for the k-steps of 4
constexpr int NHT = NH / 16;              // 16-wide tiles of a hidden layer
static_assert(NH == 64 && NIN <= 32 && TT == 256 && GR == 4 * 16, "gradient tiling");
typedef float mf4 __attribute__((ext_vector_type(4)));
struct GradLds {
  alignas(16) float w1[NINP][NH];
  alignas(16) float w2[NH][NH];
  float b1[NH], b2[NH], w3[NH];
  float x[GR][33];          // inputs, zero beyond NIN (two 16-wide blocks for dW1)
  float h1[GR][NH + 1];     // silu(a1)
  float d1[GR][NH + 1];     // silu'(a1), then G1 = dL/da1
  float g2[GR][NH + 1];     // G2 = dL/da2
  float red[4][NH + 1];     // per-wave sums: dW3, db3
  double lred[4];           // per-wave loss sums
};

__global__ __launch_bounds__(TT) void mlp_grad_kernel(const float *__restrict__ prm,
                                                      const float *__restrict__ feat,
                                                      const float *__restrict__ target,
                                                      int64_t rows, float inv_rows,
                                                      float *__restrict__ gpart,
                                                      double *__restrict__ lpart) {
  __shared__ GradLds L;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int rw = 16 * wave;
  const int64_t r0 = (int64_t)blockIdx.x * GR;
  for (int q = t; q < NINP * NH; q += TT) {
    const int k = q / NH, j = q % NH;
    L.w1[k][j] = k < NIN ? prm[OW1 + k * NH + j] : 0.0f;
  }
  for (int q = t; q < NH * NH; q += TT) L.w2[q / NH][q % NH] = prm[OW2 + q];
  if (t < NH) {
    L.b1[t] = prm[OB1 + t];
    L.b2[t] = prm[OB2 + t];
    L.w3[t] = prm[OW3 + t];
  }
  const float b3 = prm[OB3];
  for (int q = t; q < GR * 32; q += TT) {
    const int r = q / 32, k = q % 32;
    L.x[r][k] = (r0 + r < rows && k < NIN) ? feat[(r0 + r) * NIN + k] : 0.0f;
  }
  __syncthreads();
  // layer 1
  mf4 acc[NHT];
#pragma unroll
  for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < NINP; k += 4) {
    const float a = L.x[rw + lr][k + lg];
#pragma unroll
    for (int u = 0; u < NHT; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.w1[k + lg][16 * u + lr], acc[u], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < NHT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rw + 4 * lg + v, unit = 16 * u + lr;
      const float z = acc[u][v] + L.b1[unit];
      const float sg = sigm(z);
      L.h1[row][unit] = z * sg;
      L.d1[row][unit] = sg * (1.0f + z * (1.0f - sg));
    }
  __syncthreads();
  // layer 2, the output, G2 = dy w3 silu'(a2)
#pragma unroll
  for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
  for (int k = 0; k < NH; k += 4) {
    const float a = L.h1[rw + lr][k + lg];
#pragma unroll
    for (int u = 0; u < NHT; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.w2[k + lg][16 * u + lr], acc[u], 0, 0, 0);
  }
  float dw3[NHT];
#pragma unroll
  for (int u = 0; u < NHT; ++u) dw3[u] = 0.0f;
  float db3 = 0.0f;
  double loss = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = rw + 4 * lg + v;
    float h2[NHT], s2[NHT], sp = 0.0f;
#pragma unroll
    for (int u = 0; u < NHT; ++u) {
      const int unit = 16 * u + lr;
      const float z = acc[u][v] + L.b2[unit];
      const float sg = sigm(z);
      h2[u] = z * sg;
      s2[u] = sg * (1.0f + z * (1.0f - sg));
      sp = fmaf(h2[u], L.w3[unit], sp);
    }
    // every lane of the row group gets the sum over the 64 units
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) sp += __shfl_xor(sp, off, 16);
    const float e = (r0 + row < rows) ? (sp + b3 - target[r0 + row]) : 0.0f;
    const float dy = 2.0f * e * inv_rows;
#pragma unroll
    for (int u = 0; u < NHT; ++u) {
      const int unit = 16 * u + lr;
      L.g2[row][unit] = dy * L.w3[unit] * s2[u];
      dw3[u] = fmaf(h2[u], dy, dw3[u]);
    }
    if (lr == 0) {
      db3 += dy;
      loss += (double)(e * e);
    }
  }
  // over the wave's four row groups (lanes lr, lr + 16, lr + 32, lr + 48)
#pragma unroll
  for (int u = 0; u < NHT; ++u) {
    dw3[u] += __shfl_xor(dw3[u], 16, 64);
    dw3[u] += __shfl_xor(dw3[u], 32, 64);
  }
  db3 += __shfl_xor(db3, 16, 64);
  db3 += __shfl_xor(db3, 32, 64);
  loss += __shfl_xor(loss, 16, 64);
  loss += __shfl_xor(loss, 32, 64);
  if (lg == 0)
#pragma unroll
    for (int u = 0; u < NHT; ++u) L.red[wave][16 * u + lr] = dw3[u];
  if (lane == 0) {
    L.red[wave][NH] = db3;
    L.lred[wave] = loss;
  }
  __syncthreads();
  float *g = gpart + (int64_t)blockIdx.x * NP;
  if (t < NH) g[OW3 + t] = ((L.red[0][t] + L.red[1][t]) + L.red[2][t]) + L.red[3][t];
  if (t == 0) {
    g[OB3] = ((L.red[0][NH] + L.red[1][NH]) + L.red[2][NH]) + L.red[3][NH];
    lpart[blockIdx.x] = ((L.lred[0] + L.lred[1]) + L.lred[2]) + L.lred[3];
  }
  // dW2 = silu(a1)^T G2: wave w takes input units 16 w .., every output block
#pragma unroll
  for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
  for (int k = 0; k < GR; k += 4) {
    const float a = L.h1[k + lg][rw + lr];
#pragma unroll
    for (int u = 0; u < NHT; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.g2[k + lg][16 * u + lr], acc[u], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < NHT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) g[OW2 + (rw + 4 * lg + v) * NH + 16 * u + lr] = acc[u][v];
  // G1 = (G2 W2^T) o silu'(a1): wave w takes rows 16 w .., B = W2^T
#pragma unroll
  for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
  for (int k = 0; k < NH; k += 4) {
    const float a = L.g2[rw + lr][k + lg];
#pragma unroll
    for (int u = 0; u < NHT; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.w2[16 * u + lr][k + lg], acc[u], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < NHT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rw + 4 * lg + v, unit = 16 * u + lr;
      L.d1[row][unit] = acc[u][v] * L.d1[row][unit];
    }
  if (t < NH) {
    float sb = 0.0f;
    for (int r = 0; r < GR; ++r) sb += L.g2[r][t];
    g[OB2 + t] = sb;
  }
  __syncthreads();
  // dW1 = X^T G1: wave w takes inputs 16 (w / 2) .. and output blocks
  // 2 (w % 2), 2 (w % 2) + 1
  {
    const int ib = wave >> 1, ob = 2 * (wave & 1);
    mf4 a2[2] = {mf4{0.0f, 0.0f, 0.0f, 0.0f}, mf4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll 4
    for (int k = 0; k < GR; k += 4) {
      const float a = L.x[k + lg][16 * ib + lr];
#pragma unroll
      for (int q = 0; q < 2; ++q)
        a2[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.d1[k + lg][16 * (ob + q) + lr], a2[q],
                                                     0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int in = 16 * ib + 4 * lg + v;
        if (in < NIN) g[OW1 + in * NH + 16 * (ob + q) + lr] = a2[q][v];
      }
  }
  if (t < NH) {
    float sb = 0.0f;
    for (int r = 0; r < GR; ++r) sb += L.d1[r][t];
    g[OB1 + t] = sb;
  }
}

// grad[p] = sum over tiles (fixed order, FP64 accumulation); loss likewise.
__global__ void grad_reduce_kernel(const float *__restrict__ gpart, int64_t tiles,
                                   float *__restrict__ grad, const double *__restrict__ lpart,
                                   double *__restrict__ loss, double inv_rows) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    double s = 0.0;
    for (int64_t tl = 0; tl < tiles; ++tl) s += (double)gpart[tl * NP + p];
    grad[p] = (float)s;
  }
  if (p == 0) {
    double s = 0.0;
    for (int64_t tl = 0; tl < tiles; ++tl) s += lpart[tl];
    loss[0] = s * inv_rows;
  }
}

__global__ void adam_kernel(float *__restrict__ prm, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.0f - b1) * gi;
  const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / c1, vh = vi / c2;
  prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

// flags[0] = 1 if any row id lies outside [0, total)
__global__ void check_rows_kernel(const int64_t *__restrict__ ids, int64_t count, int64_t total,
                                  int *__restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < count && (ids[r] < 0 || ids[r] >= total)) flag[0] = 1;
}

// gather q / q_scale of rows as float targets
__global__ void targets_kernel(const double *__restrict__ q, const int64_t *__restrict__ rows_idx,
                               int64_t r0, int64_t rows, double inv_qs, float *__restrict__ t) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t id = rows_idx ? rows_idx[r] : r0 + r;
  t[r] = (float)(q[id] * inv_qs);
}

// q0 = q_scale * y, frame-wise shift to sum(q0) = -Q_sol (one block per frame)
__global__ __launch_bounds__(256) void neutral_shift_kernel(const float *__restrict__ y,
                                                            const double *__restrict__ qchi,
                                                            int64_t n, double qs,
                                                            const double *__restrict__ qsol,
                                                            double *__restrict__ q0) {
  __shared__ double red[256];
  const int64_t f = blockIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = y ? qs * (double)y[f * n + i] : qchi[i];
    q0[f * n + i] = v;
    s += v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double shift = (red[0] + qsol[f]) / (double)n;
  __syncthreads();
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) q0[f * n + i] -= shift;
}

// x0 = q0 + mu0 d' with mu0 = mean(b - E q0) (Eq = E q0 given in eq)
// x0 += mu d' with mu = mean(b - E x0) (the Lagrange shift), and when r0 is
// given also the residual of the shifted start, r0 = (b - E x0) - mu 1
// (E d' = 1), so that the solver needs no product of its own for it.
__global__ __launch_bounds__(256) void lagrange_shift_kernel(const double *__restrict__ b,
                                                             const double *__restrict__ eq,
                                                             const double *__restrict__ dprime,
                                                             int64_t n, double *__restrict__ x0,
                                                             double *__restrict__ r0) {
  __shared__ double red[256];
  const int64_t f = blockIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) s += b[f * n + i] - eq[f * n + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double mu = red[0] / (double)n;
  __syncthreads();
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) x0[f * n + i] += mu * dprime[i];
  if (r0 != nullptr)
#pragma unroll 8
    for (int64_t i = threadIdx.x; i < n; i += 256) r0[f * n + i] = (b[f * n + i] - eq[f * n + i]) - mu;
}


// Host 12-neighbour list: order by distance, then azimuth about +z from +x,
// then index; distance and angle compared after rounding to 1e-6.
cpm_status build_neighbours(const cpm_system *s, std::vector<int32_t> &nbr,
                            std::vector<float> &nbr_r) {
  const int64_t n = s->n;
  if (n < NNB + 1) {
    set_error("the warm-start network needs at least 13 electrode atoms");
    return CPM_EINVAL;
  }
  const double *box = s->box;
  nbr.assign(n * NNB, 0);
  nbr_r.assign(n * NNB, 0.0f);
  const double *pos = s->pos_host.data();
  // cell grid
  double reach = 3.0;
  for (;;) {
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = std::max(1, (int)(box[d] / reach));
    std::vector<std::vector<int64_t>> cells((size_t)nc[0] * nc[1] * nc[2]);
    auto cell_of = [&](int64_t i, int d) {
      int c = (int)(pos[3 * i + d] / box[d] * nc[d]);
      return std::min(std::max(c, 0), nc[d] - 1);
    };
    for (int64_t i = 0; i < n; ++i)
      cells[((size_t)cell_of(i, 0) * nc[1] + cell_of(i, 1)) * nc[2] + cell_of(i, 2)].push_back(i);
    bool ok = true;
    struct Cand {
      long long kd, ka;
      int64_t j;
      double d;
    };
    std::vector<Cand> cand;
    for (int64_t i = 0; i < n && ok; ++i) {
      cand.clear();
      const int ci[3] = {cell_of(i, 0), cell_of(i, 1), cell_of(i, 2)};
      int span[3];
      for (int d = 0; d < 3; ++d) span[d] = std::min(1, (nc[d] - 1) / 2 > 0 ? 1 : 0) + 0;
      for (int d = 0; d < 3; ++d) span[d] = nc[d] >= 3 ? 1 : 0;
      std::vector<size_t> seen;
      for (int a = -span[0]; a <= span[0]; ++a)
        for (int bb = -span[1]; bb <= span[1]; ++bb)
          for (int c = -span[2]; c <= span[2]; ++c) {
            const size_t cell = ((size_t)((ci[0] + a + nc[0]) % nc[0]) * nc[1] +
                                 (ci[1] + bb + nc[1]) % nc[1]) * nc[2] + (ci[2] + c + nc[2]) % nc[2];
            if (std::find(seen.begin(), seen.end(), cell) != seen.end()) continue;
            seen.push_back(cell);
            for (int64_t j : cells[cell]) {
              if (j == i) continue;
              double dv[3];
              for (int d = 0; d < 3; ++d) {
                double x = pos[3 * j + d] - pos[3 * i + d];
                x -= box[d] * std::nearbyint(x / box[d]);
                dv[d] = x;
              }
              const double dd = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
              if (dd > reach) continue;
              double az = std::atan2(dv[1], dv[0]);
              if (az < 0) az += 2.0 * M_PI;
              cand.push_back({std::llround(dd * 1e6), std::llround(az * 1e6), j, dd});
            }
          }
      if ((int64_t)cand.size() < NNB) {
        ok = false;
        break;
      }
      std::sort(cand.begin(), cand.end(), [](const Cand &x, const Cand &y) {
        if (x.kd != y.kd) return x.kd < y.kd;
        if (x.ka != y.ka) return x.ka < y.ka;
        return x.j < y.j;
      });
      for (int k = 0; k < NNB; ++k) {
        nbr[i * NNB + k] = (int32_t)cand[k].j;
        nbr_r[i * NNB + k] = (float)cand[k].d;
      }
    }
    if (ok) return CPM_OK;
    reach *= 1.5;
    if (reach > std::max(box[0], std::max(box[1], box[2]))) {
      set_error("could not find 12 neighbours");
      return CPM_EINVAL;
    }
  }
}

}  // namespace

// Inference of many rows: each workgroup copies the parameters into LDS
// once and then runs tiles of IR rows (grid-stride over tiles). The two
// hidden layers are dense products and run on the matrix cores
// (v_mfma_f32_16x16x4f32, FP32 in and out): wavefront w takes rows
// 16 w .. 16 w + 15 of the tile and all NH units as NH / 16 output tiles;
// lane (lr, lg) supplies A = X[row lr][k + lg] and B = W[k + lg][unit lr]
// and receives D[row 4 lg + v][unit lr], v = 0..3. The input width is padded
// with zero columns to a multiple of 4. SiLU is applied once per hidden
// value; the output layer is reduced over the 16 lanes of a row group by
// shuffles in a fixed order. FROM_B: the inputs are formed from b in the
// kernel (same definition as features_kernel), otherwise read from feat.
constexpr int IR = 64;                       // rows per inference tile (16 per wavefront)
static_assert(NH % 16 == 0 && TT == 4 * 64 && IR == 16 * (TT / 64) && TT == 4 * IR &&
                  NNB % 4 == 0 && NIN == 2 + 2 * NNB, "inference tiling");
static_assert(OW1 % 4 == 0 && OB1 % 4 == 0 && OW2 % 4 == 0 && OB2 % 4 == 0 && OW3 % 4 == 0 &&
                  (NH * NH / 4) % TT == 0 && 3 * (NH / 4) <= TT,
              "parameter offsets and sizes in whole float4 pieces");
struct InferLds {
  alignas(16) float w1[NINP][NH];
  alignas(16) float w2[NH][NH];
  alignas(16) float b1[NH];
  alignas(16) float b2[NH];
  alignas(16) float w3[NH];
  float x[IR][NINP + 1];
  float h1[IR][NH + 1];
};

template <bool FROM_B>
__global__ __launch_bounds__(TT) void mlp_infer_kernel(
    const float *__restrict__ prm, const float *__restrict__ feat, const double *__restrict__ b,
    const double *__restrict__ mean, int64_t n, const int32_t *__restrict__ nbr,
    const float *__restrict__ nbr_r, const int32_t *__restrict__ layer, float inv_layers,
    float inv_bs, float inv_rs, int64_t rows, float *__restrict__ y) {
  __shared__ InferLds L;
  const int t = threadIdx.x;
  {
    // parameters into LDS as float4 pieces, every load of a thread issued
    // before its first store (the offsets are multiples of 4 floats)
    constexpr int N1 = NIN * NH / 4, N2 = NH * NH / 4, NV = NH / 4;
    constexpr int L1 = (N1 + TT - 1) / TT, L2 = N2 / TT;
    const float4 *p4 = reinterpret_cast<const float4 *>(prm);
    float4 v1[L1], v2[L2], vb = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < L1; ++u) {
      const int q = t + u * TT;
      if (q < N1) v1[u] = p4[OW1 / 4 + q];
    }
#pragma unroll
    for (int u = 0; u < L2; ++u) v2[u] = p4[OW2 / 4 + t + u * TT];
    if (t < 3 * NV) vb = p4[(t < NV ? OB1 : t < 2 * NV ? OB2 : OW3) / 4 + t % NV];
    float4 *w1 = reinterpret_cast<float4 *>(&L.w1[0][0]);
    float4 *w2 = reinterpret_cast<float4 *>(&L.w2[0][0]);
#pragma unroll
    for (int u = 0; u < L1; ++u) {
      const int q = t + u * TT;
      if (q < N1) w1[q] = v1[u];
    }
    for (int q = N1 + t; q < NINP * NH / 4; q += TT) w1[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < L2; ++u) w2[t + u * TT] = v2[u];
    if (t < 3 * NV) {
      float *dst = t < NV ? L.b1 : t < 2 * NV ? L.b2 : L.w3;
      reinterpret_cast<float4 *>(dst)[t % NV] = vb;
    }
  }
  const float b3 = prm[OB3];
  const int wave = t >> 6, lane = t & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int rw = 16 * wave;   // the wavefront's first row in the tile
  const int64_t tiles = (rows + IR - 1) / IR;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t r0 = tile * IR;
    __syncthreads();   // parameters loaded / previous tile done with x and h1
    if constexpr (FROM_B) {
      // four threads per row, each with a quarter of the neighbours
      constexpr int NQ = NNB / 4;
      const int row = t >> 2, part = t & 3;
      const int64_t r = r0 + row;
      if (r < rows) {
        const int64_t f = r / n, i = r % n;
        const double mb = mean[f];
        const double *bf = b + f * n;
        if (part == 0) {
          L.x[row][0] = (float)((bf[i] - mb) * (double)inv_bs);
          L.x[row][1] = (float)layer[i] * inv_layers;
          for (int k = NIN; k < NINP; ++k) L.x[row][k] = 0.0f;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int k = part * NQ + q;
          L.x[row][2 + k] = (float)((bf[nbr[i * NNB + k]] - mb) * (double)inv_bs);
          L.x[row][2 + NNB + k] = nbr_r[i * NNB + k] * inv_rs;
        }
      } else if (part == 0) {
        for (int k = 0; k < NINP; ++k) L.x[row][k] = 0.0f;
      }
    } else {
      for (int q = t; q < IR * NINP; q += TT) {
        const int r = q / NINP, k = q % NINP;
        L.x[r][k] = (r0 + r < rows && k < NIN) ? feat[(r0 + r) * NIN + k] : 0.0f;
      }
    }
    __syncthreads();
    // layer 1: a1 = X W1, h1 = silu(a1 + b1)
    mf4 acc[NHT];
#pragma unroll
    for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < NINP; k += 4) {
      const float a = L.x[rw + lr][k + lg];
#pragma unroll
      for (int u = 0; u < NHT; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.w1[k + lg][16 * u + lr], acc[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < NHT; ++u) {
      const float bu = L.b1[16 * u + lr];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float z = acc[u][v] + bu;
        L.h1[rw + 4 * lg + v][16 * u + lr] = z * sigm(z);
      }
    }
    __syncthreads();
    // layer 2: a2 = h1 W2
#pragma unroll
    for (int u = 0; u < NHT; ++u) acc[u] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
    for (int k = 0; k < NH; k += 4) {
      const float a = L.h1[rw + lr][k + lg];
#pragma unroll
      for (int u = 0; u < NHT; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L.w2[k + lg][16 * u + lr], acc[u], 0, 0, 0);
    }
    // y = sum_j silu(a2_j + b2_j) w3_j + b3: the lane's NHT units, then the
    // 16 lanes of the row group
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float sp = 0.0f;
#pragma unroll
      for (int u = 0; u < NHT; ++u) {
        const float z = acc[u][v] + L.b2[16 * u + lr];
        sp = fmaf(z * sigm(z), L.w3[16 * u + lr], sp);
      }
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) sp += __shfl_xor(sp, off, 16);
      const int64_t r = r0 + rw + 4 * lg + v;
      if (lr == 0 && r < rows) y[r] = sp + b3;
    }
  }
}

// workgroups of the inference kernel: up to four per CU (three fit its
// LDS at a time), at most one per tile
unsigned infer_blocks(int64_t rows) {
  const int64_t tiles = (rows + IR - 1) / IR;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, 1024));
}

hipError_t launch_mlp_forward(hipStream_t st, const float *params, const float *feat,
                              int64_t rows, float *y) {
  hipLaunchKernelGGL(mlp_infer_kernel<false>, dim3(infer_blocks(rows)), dim3(TT), 0, st, params,
                     feat, (const double *)nullptr, (const double *)nullptr, (int64_t)1,
                     (const int32_t *)nullptr, (const float *)nullptr, (const int32_t *)nullptr,
                     0.0f, 0.0f, 0.0f, rows, y);
  return hipGetLastError();
}

static cpm_status ensure_rows(cpm_system *s, int64_t rows) {
  Mlp &M = s->mlp;
  if (M.feat_rows >= rows) return CPM_OK;
  if (M.feat) (void)hipFree(M.feat);
  if (M.yout) (void)hipFree(M.yout);
  M.feat = nullptr;
  M.yout = nullptr;
  M.feat_rows = 0;
  if (hipMalloc((void **)&M.feat, sizeof(float) * NIN * rows) != hipSuccess ||
      hipMalloc((void **)&M.yout, sizeof(float) * rows) != hipSuccess) {
    (void)hipGetLastError();
    set_error("network scratch allocation failed");
    return CPM_ENOMEM;
  }
  M.feat_rows = rows;
  return CPM_OK;
}

static cpm_status ensure_gpart(cpm_system *s, int64_t tiles) {
  Mlp &M = s->mlp;
  if (M.gpart_tiles >= tiles) return CPM_OK;
  if (M.gpart) (void)hipFree(M.gpart);
  M.gpart = nullptr;
  double *lp = nullptr;
  if (hipMalloc((void **)&M.gpart, sizeof(float) * round_up((int64_t)NP * tiles, 64) +
                                        sizeof(double) * (tiles + 8)) !=
      hipSuccess) {
    (void)hipGetLastError();
    M.gpart_tiles = 0;
    set_error("gradient scratch allocation failed");
    return CPM_ENOMEM;
  }
  (void)lp;
  M.gpart_tiles = tiles;
  return CPM_OK;
}

static double *lpart_of(cpm_system *s) {
  // the loss partials follow the gradient partials at a 256-byte boundary
  return reinterpret_cast<double *>(s->mlp.gpart + round_up((int64_t)NP * s->mlp.gpart_tiles, 64));
}

static cpm_status loss_grad_impl(cpm_system *s, const float *feat, const float *target,
                                 int64_t rows, float *grad_out) {
  const int64_t tiles = (rows + GR - 1) / GR;
  cpm_status rc = ensure_gpart(s, tiles);
  if (rc != CPM_OK) return rc;
  hipStream_t st = s->stream;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)tiles), dim3(TT), 0, st,
                     s->mlp.params, feat, target, rows, (float)(1.0 / (double)rows), s->mlp.gpart,
                     lpart_of(s));
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, s->mlp.gpart,
                     tiles, grad_out, lpart_of(s), s->mlp.loss, 1.0 / (double)rows);
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

static cpm_status adam_impl(cpm_system *s, float lr, float b1, float b2, float eps) {
  Mlp &M = s->mlp;
  M.step += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)M.step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)M.step));
  hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, s->stream, M.params,
                     M.adam_m, M.adam_v, M.grad, lr, b1, b2, eps, c1, c2);
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

static cpm_status features_impl(cpm_system *s, const double *b, int64_t f,
                                const int64_t *rows_idx, int64_t r0, int64_t rows, float *feat,
                                double *mean_buf, bool compute_mean) {
  const Mlp &M = s->mlp;
  hipStream_t st = s->stream;
  if (compute_mean)
    hipLaunchKernelGGL(frame_mean_kernel, dim3((unsigned)f), dim3(256), 0, st, b, s->n, mean_buf);
  const float inv_layers = M.n_layers > 1 ? 1.0f / (float)(M.n_layers - 1) : 0.0f;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, b,
                     mean_buf, s->n, M.nbr, M.nbr_r, M.layer, inv_layers, 1.0f / M.b_scale,
                     1.0f / M.r_scale, rows_idx, r0, rows, feat);
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

// x0 (f, n) for the warm start; mode from the system state: network if its
// parameters are set and requested, else q_chi.
cpm_status warm_start_impl(cpm_system *s, bool use_mlp, const double *b, const double *qsol,
                           int64_t f, double *x0, double *r0) {
  hipStream_t st = s->stream;
  const int64_t n = s->n;
  const float *y = nullptr;
  cpm_status rb = CPM_OK;
  double *mean = (double *)grow_buf(s, s->buf_mean, sizeof(double) * f, &rb);
  if (rb != CPM_OK) return rb;
  // E q0 for the Lagrange shift
  double *eq = (double *)grow_buf(s, s->buf_eq, sizeof(double) * f * n, &rb);
  if (rb != CPM_OK) return rb;
  if (use_mlp) {
    cpm_status rc = ensure_rows(s, f * n);
    if (rc != CPM_OK) return rc;
    const Mlp &M = s->mlp;
    hipLaunchKernelGGL(frame_mean_kernel, dim3((unsigned)f), dim3(256), 0, st, b, n, mean);
    const float inv_layers = M.n_layers > 1 ? 1.0f / (float)(M.n_layers - 1) : 0.0f;
    hipLaunchKernelGGL(mlp_infer_kernel<true>, dim3(infer_blocks(f * n)), dim3(TT), 0, st,
                       (const float *)M.params, (const float *)nullptr, b, (const double *)mean, n,
                       (const int32_t *)M.nbr, (const float *)M.nbr_r, (const int32_t *)M.layer,
                       inv_layers, 1.0f / M.b_scale, 1.0f / M.r_scale, f * n, M.yout);
    y = s->mlp.yout;
  }
  hipLaunchKernelGGL(neutral_shift_kernel, dim3((unsigned)f), dim3(256), 0, st, y, s->qchi, n,
                     (double)s->mlp.q_scale, qsol, x0);
  // E q0 for the Lagrange shift: FP64 when the start's residual r0 is wanted
  // too (it is then the solver's first residual), else the FP32 copy of E
  // when there is one (the shift only sets the start)
  cpm_status rc =
      matvec_cols(s, (r0 == nullptr && s->E32) ? CPM_PREC_F32 : CPM_PREC_F64, x0, f, eq);
  if (rc == CPM_OK)
    hipLaunchKernelGGL(lagrange_shift_kernel, dim3((unsigned)f), dim3(256), 0, st, b, eq,
                       s->dprime, n, x0, r0);
  CPM_HIP_CHECK(hipGetLastError());
  return rc;
}

}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_mlp_init(cpm_system *s, const int32_t *layer_host, int32_t n_layers, float b_scale,
                        float r_scale, float q_scale) {
  if (!s || !layer_host || n_layers < 1 || !(b_scale > 0) || !(r_scale > 0) || !(q_scale > 0)) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  for (int64_t i = 0; i < s->n; ++i)
    if (layer_host[i] < 0 || layer_host[i] >= n_layers) {
      set_error("layer index out of range");
      return CPM_EINVAL;
    }
  std::vector<int32_t> nbr;
  std::vector<float> nbr_r;
  cpm_status rc = build_neighbours(s, nbr, nbr_r);
  if (rc != CPM_OK) return rc;
  Mlp &M = s->mlp;
  auto alloc = [&](void **p, size_t bytes) {
    if (*p) return true;
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  };
  if (!alloc((void **)&M.nbr, sizeof(int32_t) * s->n * NNB) ||
      !alloc((void **)&M.nbr_r, sizeof(float) * s->n * NNB) ||
      !alloc((void **)&M.layer, sizeof(int32_t) * s->n) ||
      !alloc((void **)&M.params, sizeof(float) * NP) ||
      !alloc((void **)&M.adam_m, sizeof(float) * NP) ||
      !alloc((void **)&M.adam_v, sizeof(float) * NP) ||
      !alloc((void **)&M.grad, sizeof(float) * NP) || !alloc((void **)&M.loss, sizeof(double) * 8)) {
    set_error("network allocation failed");
    return CPM_ENOMEM;
  }
  hipStream_t st = s->stream;
  CPM_HIP_CHECK(hipMemcpyAsync(M.nbr, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice, st));
  CPM_HIP_CHECK(hipMemcpyAsync(M.nbr_r, nbr_r.data(), sizeof(float) * nbr_r.size(), hipMemcpyHostToDevice, st));
  CPM_HIP_CHECK(hipMemcpyAsync(M.layer, layer_host, sizeof(int32_t) * s->n, hipMemcpyHostToDevice, st));
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  M.n_layers = n_layers;
  M.b_scale = b_scale;
  M.r_scale = r_scale;
  M.q_scale = q_scale;
  M.ready = true;
  return CPM_OK;
}

cpm_status cpm_mlp_neighbours(const cpm_system *s, int32_t *nbr_host) {
  if (!s || !nbr_host || !s->mlp.ready) {
    set_error("network not initialised");
    return CPM_ESTATE;
  }
  CPM_HIP_CHECK(hipMemcpyAsync(nbr_host, s->mlp.nbr, sizeof(int32_t) * s->n * NNB,
                               hipMemcpyDeviceToHost, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_mlp_set_params(cpm_system *s, const float *params_host) {
  if (!s || !params_host) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.ready) {
    set_error("cpm_mlp_init first");
    return CPM_ESTATE;
  }
  for (int p = 0; p < NP; ++p)
    if (!std::isfinite(params_host[p])) {
      // accepted: a broken network is caught by the residual check of the
      // warm start and the solve falls back to a zero start
      break;
    }
  Mlp &M = s->mlp;
  CPM_HIP_CHECK(hipMemcpyAsync(M.params, params_host, sizeof(float) * NP, hipMemcpyHostToDevice, s->stream));
  CPM_HIP_CHECK(hipMemsetAsync(M.adam_m, 0, sizeof(float) * NP, s->stream));
  CPM_HIP_CHECK(hipMemsetAsync(M.adam_v, 0, sizeof(float) * NP, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  M.step = 0;
  M.params_set = true;
  return CPM_OK;
}

cpm_status cpm_mlp_get_params(const cpm_system *s, float *params_host) {
  if (!s || !params_host || !s->mlp.params_set) {
    set_error("no parameters set");
    return CPM_ESTATE;
  }
  CPM_HIP_CHECK(hipMemcpyAsync(params_host, s->mlp.params, sizeof(float) * NP, hipMemcpyDeviceToHost, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_mlp_features(cpm_system *s, const double *b_dev, int64_t f, float *feat_out_dev) {
  if (!s || !b_dev || !feat_out_dev || f < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.ready) {
    set_error("cpm_mlp_init first");
    return CPM_ESTATE;
  }
  cpm_status rc = CPM_OK;
  double *mean = (double *)grow_buf(s, s->buf_mean, sizeof(double) * f, &rc);
  if (rc != CPM_OK) return rc;
  rc = features_impl(s, b_dev, f, nullptr, 0, f * s->n, feat_out_dev, mean, true);
  if (rc == CPM_OK) CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return rc;
}

cpm_status cpm_mlp_forward(cpm_system *s, const float *feat_dev, int64_t rows, float *y_out_dev) {
  if (!s || !feat_dev || !y_out_dev || rows < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.params_set) {
    set_error("cpm_mlp_set_params first");
    return CPM_ESTATE;
  }
  CPM_HIP_CHECK(launch_mlp_forward(s->stream, s->mlp.params, feat_dev, rows, y_out_dev));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_mlp_loss_grad(cpm_system *s, const float *feat_dev, const float *target_dev,
                             int64_t rows, float *grad_out_dev, double *loss) {
  if (!s || !feat_dev || !target_dev || !grad_out_dev || rows < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.params_set) {
    set_error("cpm_mlp_set_params first");
    return CPM_ESTATE;
  }
  cpm_status rc = loss_grad_impl(s, feat_dev, target_dev, rows, grad_out_dev);
  if (rc != CPM_OK) return rc;
  double l = 0;
  CPM_HIP_CHECK(hipMemcpyAsync(&l, s->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  if (loss) *loss = l;
  return CPM_OK;
}

cpm_status cpm_mlp_train_step(cpm_system *s, const float *feat_dev, const float *target_dev,
                              int64_t rows, float lr, float beta1, float beta2, float eps,
                              double *loss) {
  if (!s || !feat_dev || !target_dev || rows < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.params_set) {
    set_error("cpm_mlp_set_params first");
    return CPM_ESTATE;
  }
  cpm_status rc = loss_grad_impl(s, feat_dev, target_dev, rows, s->mlp.grad);
  if (rc == CPM_OK) rc = adam_impl(s, lr, beta1, beta2, eps);
  if (rc != CPM_OK) return rc;
  double l = 0;
  CPM_HIP_CHECK(hipMemcpyAsync(&l, s->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  if (loss) *loss = l;
  return CPM_OK;
}

cpm_status cpm_mlp_train_epoch(cpm_system *s, const double *b_dev, const double *q_dev, int64_t f,
                               const int64_t *perm_dev, int64_t batch, float lr, float beta1,
                               float beta2, float eps, double *mean_loss) {
  if (!s || !b_dev || !q_dev || !perm_dev || f < 1 || batch < 1 || !(lr > 0)) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->mlp.params_set) {
    set_error("cpm_mlp_set_params first");
    return CPM_ESTATE;
  }
  hipStream_t st = s->stream;
  const int64_t rows_total = f * s->n;
  cpm_status rc = ensure_rows(s, batch);
  if (rc != CPM_OK) return rc;
  const int64_t nb = (rows_total + batch - 1) / batch;
  // buf_aux: the row check's flag, then the loss of each batch
  void *aux = grow_buf(s, s->buf_aux, std::max(sizeof(int), sizeof(double) * (size_t)nb), &rc);
  if (rc != CPM_OK) return rc;
  double *mean = (double *)grow_buf(s, s->buf_mean, sizeof(double) * f, &rc);
  if (rc != CPM_OK) return rc;
  {
    int *flag = (int *)aux, hflag = 0;
    CPM_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(check_rows_kernel, dim3((unsigned)((rows_total + 255) / 256)), dim3(256), 0,
                       st, perm_dev, rows_total, rows_total, flag);
    CPM_HIP_CHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CPM_HIP_CHECK(hipStreamSynchronize(st));
    if (hflag) {
      set_error("perm holds a row id outside [0, f*n)");
      return CPM_EINVAL;
    }
  }
  hipLaunchKernelGGL(frame_mean_kernel, dim3((unsigned)f), dim3(256), 0, st, b_dev, s->n, mean);
  const double inv_qs = 1.0 / (double)s->mlp.q_scale;
  double *lhist = (double *)aux;
  for (int64_t bi = 0; bi < nb; ++bi) {
    const int64_t r0 = bi * batch;
    const int64_t rows = std::min(batch, rows_total - r0);
    rc = features_impl(s, b_dev, f, perm_dev + r0, 0, rows, s->mlp.feat, mean, false);
    if (rc != CPM_OK) break;
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, q_dev,
                       perm_dev + r0, 0, rows, inv_qs, s->mlp.yout);
    rc = loss_grad_impl(s, s->mlp.feat, s->mlp.yout, rows, s->mlp.grad);
    if (rc == CPM_OK) rc = adam_impl(s, lr, beta1, beta2, eps);
    if (rc != CPM_OK) break;
    CPM_HIP_CHECK(hipMemcpyAsync(lhist + bi, s->mlp.loss, sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  std::vector<double> lh(nb);
  if (rc == CPM_OK)
    CPM_HIP_CHECK(hipMemcpyAsync(lh.data(), lhist, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  if (rc != CPM_OK) return rc;
  if (mean_loss) {
    double sum = 0;
    for (double v : lh) sum += v;
    *mean_loss = sum / (double)nb;
  }
  return CPM_OK;
}

cpm_status cpm_set_warm_chi(cpm_system *s, const double *chi_dev, const cpm_solve_opts *opts) {
  if (!s || !chi_dev || !opts) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (!s->dprime_ready) {
    cpm_status rd = solve_dprime(s, 1e-13, 20000);
    if (rd != CPM_OK) return rd;
    s->dprime_ready = true;
  }
  // b = chi / k_e (no electrolyte), Q_sol = 0: q_chi by the two-step solve
  hipStream_t st = s->stream;
  cpm_status rb = CPM_OK;
  double *q0 = (double *)grow_buf(s, s->buf_aux, sizeof(double) * (s->n + 2), &rb);
  if (rb != CPM_OK) return rb;
  double *b = q0 + 2;
  CPM_HIP_CHECK(hipMemsetAsync(q0, 0, sizeof(double) * 2, st));
  cpm_status rc = cpm_rhs(s, nullptr, nullptr, 0, 1, chi_dev, b, q0 + 1);
  if (rc == CPM_OK) {
    cpm_solve_opts o = *opts;
    o.warm_start = CPM_WARM_ZERO;
    rc = solve_block(s, b, q0, 1, o, s->qchi, nullptr, nullptr);
  }
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  if (rc == CPM_OK) s->qchi_ready = true;
  return rc;
}

}  // extern "C"
