// Galvanostatic charge-discharge constraint and the capacitance coefficient
// matrix (Supplementary Note, Eq. S14-S24).
//
// Electrode a carries the prescribed total Q_a; the energy minimum under
// these constraints solves E q = b + Delta u with Delta u_i = Delta mu_a on
// the atoms of a (Eq. S15). cpm_gcd_build solves E a^h = b^h for the M
// indicator vectors b^h with the block (P)CG (Eq. S22-S23), keeps
// A = (a^1 .. a^M) on the device and sums it per electrode into C_E
// (Eq. S24); one workgroup factors C_E (Cholesky, M <= 64) and forms C_E^-1
// and |C_E|. cpm_gcd_solve then takes q_b = E^-1 b from the same solver and
// applies, per frame, Delta mu = C_E^-1 (Q - L q_b) (Eq. S18-S20) and
// q = q_b + A Delta mu (Eq. S17): the per-frame cost beyond the solve is
// one pass over q_b and A.
#include "cpm_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace cpm {
namespace {

constexpr int GT = 256;             // threads of the per-vector kernels (4 waves)
constexpr int kMaxElectrodes = 64;  // one lane per electrode in the factor kernel
constexpr int kGroup = 8;           // electrodes summed per pass over a vector

__device__ inline double wave_total(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[a] = sum of x[i] over the atoms i of electrode a (a < m), in a fixed
// order; kGroup electrodes per pass over x. red holds 4 * kGroup doubles.
// Ends with a barrier, after which every thread may read out.
__device__ void electrode_sums(const double *__restrict__ x, const int32_t *__restrict__ labels,
                               int64_t n, int m, double *out, double *red) {
  const int wave = threadIdx.x >> 6;
  for (int a0 = 0; a0 < m; a0 += kGroup) {
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += GT) {
      const int h = labels[i] - a0;
      const double v = x[i];
#pragma unroll
      for (int g = 0; g < kGroup; ++g) acc[g] += (h == g) ? v : 0.0;
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      const double w = wave_total(acc[g]);
      if ((threadIdx.x & 63) == 0) red[g * 4 + wave] = w;
    }
    __syncthreads();
    const int g = threadIdx.x;
    if (g < kGroup && a0 + g < m)
      out[a0 + g] = (red[g * 4] + red[g * 4 + 1]) + (red[g * 4 + 2] + red[g * 4 + 3]);
    __syncthreads();
  }
}

// b[h * n + i] = 1 if atom i belongs to electrode h, else 0 (Eq. S22)
__global__ void indicator_kernel(const int32_t *__restrict__ labels, int64_t n, int m,
                                 double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int h = blockIdx.y;
  if (i < n && h < m) b[(int64_t)h * n + i] = (labels[i] == h) ? 1.0 : 0.0;
}

// C[a * m + h] = sum over the atoms of a of A[h * n + i] (Eq. S24); one
// workgroup per column h
__global__ __launch_bounds__(GT) void capacitance_kernel(const double *__restrict__ A,
                                                         const int32_t *__restrict__ labels,
                                                         int64_t n, int m, double *__restrict__ C) {
  __shared__ double sums[kMaxElectrodes];
  __shared__ double red[4 * kGroup];
  const int h = blockIdx.x;
  electrode_sums(A + (int64_t)h * n, labels, n, m, sums, red);
  if ((int)threadIdx.x < m) C[threadIdx.x * m + h] = sums[threadIdx.x];
}

// One wave: Csym = (C + C^T) / 2, its Cholesky factor in LDS, |C_E| as the
// product of the squared pivots, and C_E^-1 column by column (lane c solves
// L L^T x = e_c). out = [Csym (m^2) | Cinv (m^2) | det, sum, joint, status];
// status 1 marks a pivot that is not positive and finite (C_E not definite).
__global__ __launch_bounds__(64) void capacitance_factor_kernel(const double *__restrict__ C,
                                                                int m, double *__restrict__ out) {
  __shared__ double L[kMaxElectrodes][kMaxElectrodes + 1];
  const int t = threadIdx.x;
  double *Cs = out;
  double *Ci = out + m * m;
  double *scal = out + 2 * m * m;
  double colsum = 0.0;
  if (t < m) {
    for (int i = 0; i < m; ++i) {
      const double v = 0.5 * (C[i * m + t] + C[t * m + i]);
      L[i][t] = v;
      Cs[i * m + t] = v;
      colsum += v;
    }
  }
  const double total = wave_total(colsum);
  __syncthreads();
  double det = 1.0;
  bool ok = true;
  for (int k = 0; k < m; ++k) {
    const double piv = L[k][k];
    if (!(piv > 0.0) || !isfinite(piv)) {   // the same value on every lane
      ok = false;
      break;
    }
    det *= piv;
    const double lkk = sqrt(piv);
    __syncthreads();
    if (t == k) L[k][k] = lkk;
    if (t > k && t < m) L[t][k] /= lkk;
    __syncthreads();
    if (t > k && t < m)
      for (int j = k + 1; j <= t; ++j) L[t][j] -= L[t][k] * L[j][k];
    __syncthreads();
  }
  if (!ok) {
    if (t == 0) scal[3] = 1.0;
    return;
  }
  if (t < m) {
    // forward: L y = e_t (y_i = 0 for i < t), kept in column t of Ci
    for (int i = 0; i < m; ++i) {
      double s = (i == t) ? 1.0 : 0.0;
      for (int j = t; j < i; ++j) s -= L[i][j] * Ci[j * m + t];
      Ci[i * m + t] = (i < t) ? 0.0 : s / L[i][i];
    }
    // backward: L^T x = y
    for (int i = m - 1; i >= 0; --i) {
      double s = Ci[i * m + t];
      for (int j = i + 1; j < m; ++j) s -= L[j][i] * Ci[j * m + t];
      Ci[i * m + t] = s / L[i][i];
    }
  }
  if (t == 0) {
    scal[0] = det;
    scal[1] = total;
    scal[2] = (m == 2) ? det / total : NAN;
    scal[3] = 0.0;
  }
}

// Per frame f (one workgroup): Delta Q = Q_f - L q_b, Delta mu = C_E^-1
// Delta Q, q = q_b + A Delta mu in place, then err[f] = max over electrodes
// of |sum_a q - Q_a|.
__global__ __launch_bounds__(GT) void gcd_shift_kernel(
    double *__restrict__ q, int64_t n, const int32_t *__restrict__ labels, int m,
    const double *__restrict__ A, const double *__restrict__ Cinv, const double *__restrict__ Q,
    double *__restrict__ dmu_out, double *__restrict__ err) {
  __shared__ double dq[kMaxElectrodes];
  __shared__ double mu[kMaxElectrodes];
  __shared__ double red[4 * kGroup];
  const int64_t f = blockIdx.x;
  double *qf = q + f * n;
  const double *Qf = Q + f * m;
  const int t = threadIdx.x;
  electrode_sums(qf, labels, n, m, dq, red);
  if (t < m) dq[t] = Qf[t] - dq[t];
  __syncthreads();
  if (t < m) {
    double s = 0.0;
    for (int b = 0; b < m; ++b) s += Cinv[t * m + b] * dq[b];
    mu[t] = s;
    if (dmu_out) dmu_out[f * m + t] = s;
  }
  __syncthreads();
  for (int64_t i = t; i < n; i += GT) {
    double s = qf[i];
    for (int b = 0; b < m; ++b) s += A[(int64_t)b * n + i] * mu[b];
    qf[i] = s;
  }
  __syncthreads();
  electrode_sums(qf, labels, n, m, dq, red);
  if (t == 0) {
    double e = 0.0;
    for (int a = 0; a < m; ++a) e = fmax(e, fabs(dq[a] - Qf[a]));
    err[f] = e;
  }
}

void reset_info(cpm_solve_info *info) {
  if (!info) return;
  int *fi = info->frame_iters;
  double *fr = info->frame_rel_resid;
  std::memset(info, 0, sizeof(*info));
  info->frame_iters = fi;
  info->frame_rel_resid = fr;
}

}  // namespace

void free_gcd(Gcd &g) {
  if (g.labels) (void)hipFree(g.labels);
  if (g.A) (void)hipFree(g.A);
  if (g.mats) (void)hipFree(g.mats);
  g = Gcd();
}

}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_gcd_build(cpm_system *s, const int32_t *labels_host, int32_t m,
                         const cpm_solve_opts *opts, double *C_out_host, double *det_out,
                         double *joint_out, cpm_solve_info *info) {
  if (!s || !labels_host || !opts || !C_out_host) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (m < 1 || m > kMaxElectrodes) {
    set_error("need 1 <= m <= 64 electrodes");
    return CPM_EINVAL;
  }
  const int64_t n = s->n;
  std::vector<int64_t> count(m, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t a = labels_host[i];
    if (a < 0 || a >= m) {
      set_error("electrode label out of [0, m)");
      return CPM_EINVAL;
    }
    ++count[a];
  }
  for (int a = 0; a < m; ++a)
    if (count[a] == 0) {
      set_error("electrode " + std::to_string(a) + " has no atoms");
      return CPM_EINVAL;
    }
  cpm_solve_opts o;
  {
    cpm_status ro = check_solve_opts(s, opts, &o);
    if (ro != CPM_OK) return ro;
  }
  o.warm_start = CPM_WARM_ZERO;
  reset_info(info);
  hipStream_t st = s->stream;
  Gcd g;
  g.m = m;
  const int64_t mats = 2 * (int64_t)m * m + 4;
  double *b = nullptr, *craw = nullptr;
  auto fail = [&](cpm_status e) {
    if (b) (void)hipFree(b);
    if (craw) (void)hipFree(craw);
    free_gcd(g);
    return e;
  };
  if (hipMalloc((void **)&g.labels, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc((void **)&g.A, sizeof(double) * m * n) != hipSuccess ||
      hipMalloc((void **)&g.mats, sizeof(double) * mats) != hipSuccess ||
      hipMalloc((void **)&b, sizeof(double) * m * n) != hipSuccess ||
      hipMalloc((void **)&craw, sizeof(double) * m * m) != hipSuccess) {
    (void)hipGetLastError();
    set_error("capacitance allocation failed");
    return fail(CPM_ENOMEM);
  }
  g.bytes = (int64_t)(sizeof(int32_t) * n + sizeof(double) * (m * n + mats));
  if (hipMemcpyAsync(g.labels, labels_host, sizeof(int32_t) * n, hipMemcpyHostToDevice, st) !=
      hipSuccess) {
    set_error("label copy failed");
    return fail(CPM_EDEVICE);
  }
  hipLaunchKernelGGL(indicator_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256),
                     0, st, g.labels, n, (int)m, b);
  cpm_status rc = solve_block(s, b, nullptr, m, o, g.A, info, nullptr, false);
  if (rc != CPM_OK) return fail(rc);
  hipLaunchKernelGGL(capacitance_kernel, dim3((unsigned)m), dim3(GT), 0, st, g.A, g.labels, n,
                     (int)m, craw);
  hipLaunchKernelGGL(capacitance_factor_kernel, dim3(1), dim3(64), 0, st, craw, (int)m, g.mats);
  std::vector<double> host(mats);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(host.data(), g.mats, sizeof(double) * mats, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("capacitance matrix kernels failed");
    return fail(CPM_EDEVICE);
  }
  (void)hipFree(b);
  (void)hipFree(craw);
  b = craw = nullptr;
  const double *scal = host.data() + 2 * m * m;
  if (scal[3] != 0.0) {
    set_error("capacitance matrix is not positive definite");
    free_gcd(g);
    return CPM_ENOTSPD;
  }
  std::memcpy(C_out_host, host.data(), sizeof(double) * m * m);
  if (det_out) *det_out = scal[0];
  if (joint_out) *joint_out = scal[2];
  s->device_bytes -= s->gcd.bytes;
  free_gcd(s->gcd);
  g.ready = true;
  s->gcd = g;
  s->device_bytes += g.bytes;
  return CPM_OK;
}

cpm_status cpm_gcd_solve(cpm_system *s, const double *b_dev, const double *Q_dev, int64_t f,
                         const cpm_solve_opts *opts, double *q_out_dev, double *dmu_out_dev,
                         cpm_solve_info *info) {
  if (!s || !b_dev || !Q_dev || !opts || !q_out_dev) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (f < 1) {
    set_error("need f >= 1");
    return CPM_EINVAL;
  }
  if (!s->gcd.ready) {
    set_error("cpm_gcd_build first");
    return CPM_ESTATE;
  }
  cpm_solve_opts o;
  {
    cpm_status ro = check_solve_opts(s, opts, &o);
    if (ro != CPM_OK) return ro;
  }
  o.warm_start = CPM_WARM_ZERO;
  reset_info(info);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s->stream;
  const Gcd &g = s->gcd;
  cpm_status rc = solve_block(s, b_dev, nullptr, f, o, q_out_dev, info, nullptr, false);
  if (rc != CPM_OK && rc != CPM_ENOTCONV) return rc;
  cpm_status rb = CPM_OK;
  double *err = (double *)grow_buf(s, s->buf_aux, sizeof(double) * f, &rb);
  if (rb != CPM_OK) return rb;
  hipLaunchKernelGGL(gcd_shift_kernel, dim3((unsigned)f), dim3(GT), 0, st, q_out_dev, s->n,
                     g.labels, g.m, g.A, g.mats + g.m * g.m, Q_dev, dmu_out_dev, err);
  std::vector<double> herr(f);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 =
      hipMemcpyAsync(herr.data(), err, sizeof(double) * f, hipMemcpyDeviceToHost, st);
  if (e1 != hipSuccess || e2 != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    set_error("total-charge shift failed");
    return CPM_EDEVICE;
  }
  if (info) {
    for (double v : herr) info->max_abs_sum_q = std::max(info->max_abs_sum_q, v);
    info->solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

}  // extern "C"
