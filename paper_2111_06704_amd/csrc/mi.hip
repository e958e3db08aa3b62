// Matrix-inversion path (Sec. III.B.1, MI; Eq. 33-35).
//
// S = E^-1 (I - 1 d^T) is symmetric, and its column j is exactly the
// two-step charge vector (Eq. 35) of the unit right-hand side e_j with
// Q_sol = 0. cpm_mi_build obtains the columns from the library's own block
// (P)CG, 64 right-hand sides at a time, and keeps S as an ld x ld FP64
// matrix laid out like E (row j = column j, padding zero). Every frame then
// costs one block product: q = S b - Q_sol d (Eq. 33-35).
#include "cpm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace cpm {
namespace {

// b[c][i] = 1 if i == row0 + c else 0 (c < f), row-major (f, n)
__global__ void unit_rhs_kernel(double *__restrict__ b, int64_t n, int64_t row0, int64_t f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < n && c < f) b[c * n + i] = (i == row0 + c) ? 1.0 : 0.0;
}

// q[f][i] -= Q_sol[f] d_i
__global__ void mi_shift_kernel(double *__restrict__ q, const double *__restrict__ qsol,
                                const double *__restrict__ d, int64_t n, int64_t f) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * f) return;
  q[idx] -= qsol[idx / n] * d[idx % n];
}

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_mi_build(cpm_system *s, const cpm_solve_opts *opts) {
  if (!s || !opts) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  const int64_t n = s->n, ld = s->ld;
  hipStream_t st = s->stream;
  double *S = nullptr, *b = nullptr, *q = nullptr, *qs = nullptr;
  const int64_t blk = 64;
  auto cleanup = [&]() {
    if (b) (void)hipFree(b);
    if (q) (void)hipFree(q);
    if (qs) (void)hipFree(qs);
  };
  if (hipMalloc((void **)&S, sizeof(double) * ld * ld) != hipSuccess ||
      hipMalloc((void **)&b, sizeof(double) * blk * n) != hipSuccess ||
      hipMalloc((void **)&q, sizeof(double) * blk * n) != hipSuccess ||
      hipMalloc((void **)&qs, sizeof(double) * blk) != hipSuccess) {
    (void)hipGetLastError();
    if (S) (void)hipFree(S);
    cleanup();
    set_error("MI allocation failed");
    return CPM_ENOMEM;
  }
  auto fail = [&](cpm_status e) {
    (void)hipFree(S);
    cleanup();
    return e;
  };
  if (hipMemsetAsync(S, 0, sizeof(double) * ld * ld, st) != hipSuccess ||
      hipMemsetAsync(qs, 0, sizeof(double) * blk, st) != hipSuccess) {
    set_error("MI memset failed");
    return fail(CPM_EDEVICE);
  }
  cpm_solve_opts o = *opts;
  o.warm_start = CPM_WARM_ZERO;
  for (int64_t row0 = 0; row0 < n; row0 += blk) {
    const int64_t fc = std::min(blk, n - row0);
    hipLaunchKernelGGL(unit_rhs_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)fc), dim3(256),
                       0, st, b, n, row0, fc);
    cpm_status rc = cpm_solve(s, b, qs, fc, &o, q, nullptr);
    if (rc != CPM_OK) return fail(rc);
    if (hipMemcpy2DAsync(S + row0 * ld, sizeof(double) * ld, q, sizeof(double) * n,
                         sizeof(double) * n, fc, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      set_error("MI copy failed");
      return fail(CPM_EDEVICE);
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error("MI build failed");
    return fail(CPM_EDEVICE);
  }
  cleanup();
  if (s->S) {
    (void)hipFree(s->S);
    s->device_bytes -= (int64_t)(sizeof(double) * ld * ld);
  }
  s->S = S;
  s->device_bytes += (int64_t)(sizeof(double) * ld * ld);
  return CPM_OK;
}

cpm_status cpm_mi_solve(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                        double *q_out_dev) {
  if (!s || !b_dev || !qsol_dev || !q_out_dev || f < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->S) {
    set_error("cpm_mi_build first");
    return CPM_ESTATE;
  }
  cpm_status rc = matvec_cols_with(s, CPM_PREC_F64, s->S, b_dev, f, q_out_dev);
  if (rc != CPM_OK) return rc;
  hipLaunchKernelGGL(mi_shift_kernel, dim3((unsigned)((s->n * f + 255) / 256)), dim3(256), 0,
                     s->stream, q_out_dev, qsol_dev, s->dvec, s->n, f);
  CPM_HIP_CHECK(hipGetLastError());
  return CPM_OK;
}

}  // extern "C"
