// Right-hand side b = chi - b_sol for F electrolyte frames (Sec. III.A, Eq. 25).
//
// b_sol,i = sum_I q_I e_iI(a_i) with e_iI the Gaussian Ewald entry (Eq. 22)
// between electrode charge i (inverse width a_i) and point charge I (mixing
// width a_i). Split as in Eq. 20:
//   reciprocal  sum_K w_K [cos(K.r_i) Re S_K + sin(K.r_i) Im S_K],
//               S_K = sum_I q_I exp(i K.r_I)  (ion structure factor)
//   real space  sum_I q_I sum_{images, d < rcut} [erfc(beta d) - erfc(a_i d)] / d
//   background  -pi / (V beta^2) Q_sol,  Q_sol = sum_I q_I.
// Phases are evaluated from the fractional coordinate t = n . (r / L)
// reduced to [-1/2, 1/2] and sincospi(2t), all in FP64; every sum runs in a
// fixed order (no atomics), so results are bitwise reproducible.
#include "cpm_internal.h"

#include <algorithm>
#include <cmath>

namespace cpm {
namespace {

constexpr int RB = 256;       // threads per block
constexpr int KCH = 64;       // k-vectors per LDS chunk in the back-projection
constexpr int FG = 16;        // frames per thread in the back-projection

__global__ __launch_bounds__(RB) void qsum_kernel(const double *__restrict__ q, int64_t m,
                                                  double *__restrict__ qsol) {
  __shared__ double red[RB];
  const int64_t f = blockIdx.x;
  double acc = 0.0;
  for (int64_t I = threadIdx.x; I < m; I += RB) acc += q[f * m + I];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) qsol[f] = red[0];
}

// One thread per k-vector, one grid row per frame; ions stream through LDS.
__global__ __launch_bounds__(RB) void structure_factor_kernel(
    const double *__restrict__ ion_pos, const double *__restrict__ ion_q, int64_t m,
    const int32_t *__restrict__ kn, int64_t nk, double inv_lx, double inv_ly, double inv_lz,
    double *__restrict__ S) {
  __shared__ double su[RB][4];
  const int64_t f = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * RB + threadIdx.x;
  double nx = 0, ny = 0, nz = 0;
  if (k < nk) {
    nx = kn[3 * k];
    ny = kn[3 * k + 1];
    nz = kn[3 * k + 2];
  }
  double sr = 0.0, si = 0.0;
  const double *pf = ion_pos + f * m * 3;
  const double *qf = ion_q + f * m;
  for (int64_t base = 0; base < m; base += RB) {
    const int64_t I = base + threadIdx.x;
    if (I < m) {
      su[threadIdx.x][0] = pf[3 * I] * inv_lx;
      su[threadIdx.x][1] = pf[3 * I + 1] * inv_ly;
      su[threadIdx.x][2] = pf[3 * I + 2] * inv_lz;
      su[threadIdx.x][3] = qf[I];
    }
    __syncthreads();
    const int cnt = (int)((m - base) < RB ? (m - base) : RB);
    for (int j = 0; j < cnt; ++j) {
      double t = nx * su[j][0] + ny * su[j][1] + nz * su[j][2];
      t -= rint(t);
      double s, c;
      sincospi(2.0 * t, &s, &c);
      sr += su[j][3] * c;
      si += su[j][3] * s;
    }
    __syncthreads();
  }
  if (k < nk) {
    S[(f * nk + k) * 2] = sr;
    S[(f * nk + k) * 2 + 1] = si;
  }
}

// Back-projection of the ion structure factors onto the electrode atoms,
// split over k ranges: part[ks][f][i] = sum_{K in range ks} w_K (c_iK Re S_fK
// + s_iK Im S_fK). One thread per atom, FG frames per thread (the phase of
// (i, K) is evaluated once for all FG frames); grid (atom blocks, k splits,
// frame groups).
__global__ __launch_bounds__(RB) void backproject_kernel(
    const double *__restrict__ pos, int64_t n, const int32_t *__restrict__ kn,
    const double *__restrict__ kw, int64_t nk, int64_t kper, double inv_lx, double inv_ly,
    double inv_lz, const double *__restrict__ S, int64_t f_total, double *__restrict__ part) {
  __shared__ double sk[KCH][4];            // nx, ny, nz, w
  __shared__ double ss[FG][KCH][2];        // S for this block's frames
  const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  const int64_t kbeg = (int64_t)blockIdx.y * kper;
  const int64_t kend = min(nk, kbeg + kper);
  const int64_t f0 = (int64_t)blockIdx.z * FG;
  const int nf = (int)((f_total - f0) < FG ? (f_total - f0) : FG);
  double ux = 0, uy = 0, uz = 0;
  if (i < n) {
    ux = pos[3 * i] * inv_lx;
    uy = pos[3 * i + 1] * inv_ly;
    uz = pos[3 * i + 2] * inv_lz;
  }
  double acc[FG];
#pragma unroll
  for (int g = 0; g < FG; ++g) acc[g] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += KCH) {
    const int cnt = (int)((kend - k0) < KCH ? (kend - k0) : KCH);
    for (int t = threadIdx.x; t < KCH; t += RB) {
      if (t < cnt) {
        sk[t][0] = kn[3 * (k0 + t)];
        sk[t][1] = kn[3 * (k0 + t) + 1];
        sk[t][2] = kn[3 * (k0 + t) + 2];
        sk[t][3] = kw[k0 + t];
      }
    }
    for (int t = threadIdx.x; t < FG * KCH; t += RB) {
      const int g = t / KCH, kk = t % KCH;
      double re = 0.0, im = 0.0;
      if (g < nf && kk < cnt) {
        re = S[((f0 + g) * nk + k0 + kk) * 2];
        im = S[((f0 + g) * nk + k0 + kk) * 2 + 1];
      }
      ss[g][kk][0] = re;
      ss[g][kk][1] = im;
    }
    __syncthreads();
    for (int kk = 0; kk < cnt; ++kk) {
      double t = sk[kk][0] * ux + sk[kk][1] * uy + sk[kk][2] * uz;
      t -= rint(t);
      double sn, cs;
      sincospi(2.0 * t, &sn, &cs);
      cs *= sk[kk][3];
      sn *= sk[kk][3];
#pragma unroll
      for (int g = 0; g < FG; ++g) acc[g] += cs * ss[g][kk][0] + sn * ss[g][kk][1];
    }
    __syncthreads();
  }
  if (i < n) {
    for (int g = 0; g < nf; ++g) part[((int64_t)blockIdx.y * f_total + f0 + g) * n + i] = acc[g];
  }
}

// b[f, i] = chi_i / k_e - sum_ks part[ks][f][i] - c0 Q_f (fixed order over ks)
__global__ void assemble_b_kernel(const double *__restrict__ part, int ksplits, int64_t n,
                                  int64_t f_total, const double *__restrict__ chi,
                                  const double *__restrict__ qsol, double c0,
                                  double *__restrict__ b) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * f_total) return;
  const int64_t f = idx / n, i = idx % n;
  double s = 0.0;
  for (int ks = 0; ks < ksplits; ++ks) s += part[((int64_t)ks * f_total + f) * n + i];
  b[idx] = chi[i] * (1.0 / kCoulombVA) - s - c0 * qsol[f];
}

// Images of a displacement d (already reduced to the minimum image) along
// one box edge L with |d + m L| < rcut: m in [lo, hi]. When L >= 2 rcut only
// m = 0 can qualify.
__device__ inline void image_range(double d, double L, double invL, double rcut, bool wide,
                                   int &lo, int &hi) {
  if (wide) {
    lo = 0;
    hi = (fabs(d) < rcut) ? 0 : -1;
  } else {
    lo = (int)ceil((-rcut - d) * invL);
    hi = (int)floor((rcut - d) * invL);
  }
}

// One thread per (electrode atom, frame); ions stream through LDS.
// b[f, i] -= sum_I q_I sum_images [erfc(beta d) - erfc(a_i d)] / d.
__global__ __launch_bounds__(RB) void real_space_ions_kernel(
    const double *__restrict__ pos, const double *__restrict__ width, int64_t n,
    const double *__restrict__ ion_pos, const double *__restrict__ ion_q, int64_t m, double lx,
    double ly, double lz, double beta, double rcut, double *__restrict__ b) {
  __shared__ double si[RB][4];
  const int64_t f = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  double xi = 0, yi = 0, zi = 0, ai = 1.0;
  if (i < n) {
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
    ai = width[i];
  }
  const double ilx = 1.0 / lx, ily = 1.0 / ly, ilz = 1.0 / lz;
  const bool wx = lx >= 2.0 * rcut, wy = ly >= 2.0 * rcut, wz = lz >= 2.0 * rcut;
  const double rc2 = rcut * rcut;
  // limit of [erfc(beta d) - erfc(a d)] / d at d -> 0
  const double lim0 = 2.0 * (ai - beta) * 0.56418958354775628695;
  double acc = 0.0;
  const double *pf = ion_pos + f * m * 3;
  const double *qf = ion_q + f * m;
  for (int64_t base = 0; base < m; base += RB) {
    const int64_t I = base + threadIdx.x;
    if (I < m) {
      si[threadIdx.x][0] = pf[3 * I];
      si[threadIdx.x][1] = pf[3 * I + 1];
      si[threadIdx.x][2] = pf[3 * I + 2];
      si[threadIdx.x][3] = qf[I];
    }
    __syncthreads();
    const int cnt = (int)((m - base) < RB ? (m - base) : RB);
    if (i < n) {
      for (int j = 0; j < cnt; ++j) {
        double dz = zi - si[j][2];
        dz -= lz * rint(dz * ilz);
        int za, zb;
        image_range(dz, lz, ilz, rcut, wz, za, zb);
        if (za > zb) continue;
        double dx = xi - si[j][0];
        double dy = yi - si[j][1];
        dx -= lx * rint(dx * ilx);
        dy -= ly * rint(dy * ily);
        int xa, xb, ya, yb;
        image_range(dx, lx, ilx, rcut, wx, xa, xb);
        image_range(dy, ly, ily, rcut, wy, ya, yb);
        const double q = si[j][3];
        for (int a = xa; a <= xb; ++a) {
          const double ex = dx + (double)a * lx;
          for (int bb = ya; bb <= yb; ++bb) {
            const double ey = dy + (double)bb * ly;
            const double exy = ex * ex + ey * ey;
            if (exy >= rc2) continue;
            for (int c = za; c <= zb; ++c) {
              const double ez = dz + (double)c * lz;
              const double d2 = exy + ez * ez;
              if (d2 < rc2) {
                if (d2 > 0.0) {
                  const double d = sqrt(d2);
                  acc += q * ((erfc(beta * d) - erfc(ai * d)) / d);
                } else {
                  acc += q * lim0;
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (i < n) b[f * n + i] -= acc;
}

}  // namespace

// k splits of the back-projection: enough blocks to fill the chip (~2048),
// at most 64, and a partial buffer of at most ~2^27 doubles.
static int64_t backproject_ksplit(int64_t n, int64_t nk, int64_t f, int64_t &kper) {
  const int64_t iblocks = (n + RB - 1) / RB, fgroups = (f + FG - 1) / FG;
  const int64_t nkk = std::max<int64_t>(nk, 1);
  int64_t ksplit = (2048 + iblocks * fgroups - 1) / (iblocks * fgroups);
  const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 27) / std::max<int64_t>(1, f * n));
  ksplit = std::max<int64_t>(1, std::min<int64_t>({ksplit, 64, nkk, cap}));
  kper = (nkk + ksplit - 1) / ksplit;
  return (nkk + kper - 1) / kper;
}

int64_t rhs_scratch_elems(int64_t n, int64_t nk, int64_t f) {
  // structure factors (2 f nk) + back-projection partials (ksplit f n)
  int64_t kper = 0;
  return 2 * f * std::max<int64_t>(nk, 1) + backproject_ksplit(n, nk, f, kper) * f * n;
}

hipError_t launch_rhs(hipStream_t st, const cpm_system *s, const double *ion_pos,
                      const double *ion_q, int64_t m, int64_t f, const double *chi, double *S,
                      double *b_out, double *qsol_out) {
  const double ilx = 1.0 / s->box[0], ily = 1.0 / s->box[1], ilz = 1.0 / s->box[2];
  const int64_t nk = s->kset.nk, n = s->n;
  const double c0 = -M_PI / (s->vol * s->beta * s->beta);
  if (m > 0) {
    hipLaunchKernelGGL(qsum_kernel, dim3((unsigned)f), dim3(RB), 0, st, ion_q, m, qsol_out);
    hipLaunchKernelGGL(structure_factor_kernel, dim3((unsigned)((nk + RB - 1) / RB), (unsigned)f),
                       dim3(RB), 0, st, ion_pos, ion_q, m, s->kn, nk, ilx, ily, ilz, S);
  } else {
    hipError_t e = hipMemsetAsync(qsol_out, 0, sizeof(double) * f, st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(S, 0, sizeof(double) * 2 * f * std::max<int64_t>(nk, 1), st);
    if (e != hipSuccess) return e;
  }
  const int64_t iblocks = (n + RB - 1) / RB, fgroups = (f + FG - 1) / FG;
  int64_t kper = 0;
  const int64_t ksplit = backproject_ksplit(n, nk, f, kper);
  double *part = S + 2 * f * std::max<int64_t>(nk, 1);
  hipLaunchKernelGGL(backproject_kernel, dim3((unsigned)iblocks, (unsigned)ksplit, (unsigned)fgroups),
                     dim3(RB), 0, st, s->pos, n, s->kn, s->kw, nk, kper, ilx, ily, ilz, S, f, part);
  hipLaunchKernelGGL(assemble_b_kernel, dim3((unsigned)((n * f + 255) / 256)), dim3(256), 0, st,
                     part, (int)ksplit, n, f, chi, qsol_out, c0, b_out);
  if (m > 0) {
    hipLaunchKernelGGL(real_space_ions_kernel, dim3((unsigned)iblocks, (unsigned)f), dim3(RB), 0,
                       st, s->pos, s->width, n, ion_pos, ion_q, m, s->box[0], s->box[1], s->box[2],
                       s->beta, s->rcut, b_out);
  }
  return hipGetLastError();
}

}  // namespace cpm
