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
// reduced to [-1/2, 1/2] and sincospi(2t), all in FP64 (the structure
// factors' (n_x, n_y) phases by a table of 128 roots of unity and a short
// Taylor series, phase_cs); every sum runs in a fixed order (no atomics), so
// results are bitwise reproducible.
#include "cpm_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace cpm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int RB = 256;       // threads per block
constexpr int FG = 16;        // frames per thread in the back-projection
constexpr int BP_AT = 2;      // atoms per thread in the back-projection
constexpr int BP_KCH = 32;    // k-vectors per LDS chunk in the back-projection
constexpr double kErfcZero = 6.5;   // erfc(x) < 4e-20 beyond: below any FP64 sum it enters
static_assert(kErfcIntervals == 8 * 6.5, "erfc table intervals of width 1/8 up to kErfcZero");

// erfc(x) for 0 <= x from the table (0 for x >= kErfcZero): interval j =
// floor(8 x), u = 8 x - (j + 1/2) in [-1/2, 1/2), Horner over the Taylor
// coefficients c_jk = f^(k)(x_j) / (8^k k!). Every lane runs the same
// instructions (no range branches); absolute error below 3e-16.
__device__ inline double erfc_pw(const double *__restrict__ tab, double x) {
  if (!(x < kErfcZero)) return 0.0;
  const double s = 8.0 * x;
  const int j = (int)s;
  const double u = s - ((double)j + 0.5);
  const double *c = tab + j * kErfcTerms;
  double p = c[kErfcTerms - 1];
#pragma unroll
  for (int k = kErfcTerms - 2; k >= 0; --k) p = fma(p, u, c[k]);
  return p;
}

__global__ void fill_zero_kernel(double *__restrict__ v, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) v[i] = 0.0;
}

// Q_sol[f] = sum_I q_I; with m1 != null also M1[f] = sum_I q_I z_I (z in [0, L_z)),
// the ion dipole that the slab correction needs.
__global__ __launch_bounds__(RB) void qsum_kernel(const double *__restrict__ q, int64_t m,
                                                  double *__restrict__ qsol,
                                                  const double *__restrict__ ion_pos, double lz,
                                                  double *__restrict__ m1) {
  __shared__ double red[2][RB];
  const int64_t f = blockIdx.x;
  double acc = 0.0, dip = 0.0;
  for (int64_t I = threadIdx.x; I < m; I += RB) {
    const double qi = q[f * m + I];
    acc += qi;
    if (m1 != nullptr) {
      const double z = ion_pos[(f * m + I) * 3 + 2];
      dip += qi * (z - lz * floor(z / lz));
    }
  }
  red[0][threadIdx.x] = acc;
  red[1][threadIdx.x] = dip;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    qsol[f] = red[0][0];
    if (m1 != nullptr) m1[f] = red[1][0];
  }
}

// Ion structure factors of one group of ions, S_fK = sum_I q_I exp(i K.r_I).
// One thread per (run, frame): a run is up to kRun vectors of one (n_x, n_y)
// column with consecutive n_z. The phase of the run's first vector is
// evaluated directly (sincospi of the fractional phase), the second by one
// complex product with exp(2 pi i z_I / L_z), the following ones by the
// three-term recurrence of the cosine and sine, so kRun vectors cost one
// sincospi and about kRun FMAs per part and ion. Ions stream through LDS.
// Output layout: Sg[((g * nk + k) * f_total + f) * 2 + {0: Re, 1: Im}].
__global__ __launch_bounds__(RB) void structure_factor_kernel(
    const double *__restrict__ ion_pos, const double *__restrict__ ion_q, int64_t m, int64_t ipg,
    const int32_t *__restrict__ kinfo, const int32_t *__restrict__ runs, int64_t nruns,
    int64_t nk, double inv_lx, double inv_ly, double inv_lz, int64_t f_total,
    double *__restrict__ Sg) {
  __shared__ double su[RB][6];   // x/L, y/L, z/L, q, cos and sin of 2 pi z/L
  const int64_t f = blockIdx.y, g = blockIdx.z;
  const int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x;
  int64_t k0 = 0;
  int len = 0;
  double nx = 0, ny = 0, nz = 0;
  if (r < nruns) {
    k0 = runs[2 * r];
    len = runs[2 * r + 1];
    nx = kinfo[4 * k0];
    ny = kinfo[4 * k0 + 1];
    nz = kinfo[4 * k0 + 2];
  }
  double ar[kRun], ai[kRun];
#pragma unroll
  for (int st = 0; st < kRun; ++st) ar[st] = ai[st] = 0.0;
  const double *pf = ion_pos + f * m * 3;
  const double *qf = ion_q + f * m;
  const int64_t i0 = g * ipg, i1 = min(m, i0 + ipg);
  for (int64_t base = i0; base < i1; base += RB) {
    const int64_t I = base + threadIdx.x;
    if (I < i1) {
      const double uz = pf[3 * I + 2] * inv_lz;
      su[threadIdx.x][0] = pf[3 * I] * inv_lx;
      su[threadIdx.x][1] = pf[3 * I + 1] * inv_ly;
      su[threadIdx.x][2] = uz;
      su[threadIdx.x][3] = qf[I];
      double zs, zc;
      sincospi(2.0 * (uz - rint(uz)), &zs, &zc);
      su[threadIdx.x][4] = zc;
      su[threadIdx.x][5] = zs;
    }
    __syncthreads();
    const int cnt = (int)((i1 - base) < RB ? (i1 - base) : RB);
    // two ions per pass: their phase evaluations and recurrences are
    // independent, so each thread keeps four FMA chains in flight; a missing
    // second ion (odd count) enters with q = 0
    for (int j = 0; j < cnt; j += 2) {
      const int j2 = (j + 1 < cnt) ? j + 1 : j;
      const double qb = (j + 1 < cnt) ? su[j2][3] : 0.0;
      double ta = nx * su[j][0] + ny * su[j][1] + nz * su[j][2];
      double tb = nx * su[j2][0] + ny * su[j2][1] + nz * su[j2][2];
      ta -= rint(ta);
      tb -= rint(tb);
      double sna, csa, snb, csb;
      sincospi(2.0 * ta, &sna, &csa);
      sincospi(2.0 * tb, &snb, &csb);
      const double qa = su[j][3];
      const double zca = su[j][4], zsa = su[j][5], zcb = su[j2][4], zsb = su[j2][5];
      // q exp(i (phi + s theta)) for s = 0, 1, ... by the three-term
      // recurrence x_{s+1} = 2 cos(theta) x_s - x_{s-1} (one FMA per part;
      // a rounding error made at step m enters step s with the factor
      // sin((s - m) theta) / sin(theta), at most s - m)
      double c0 = qa * csa, s0 = qa * sna;
      double c1 = c0 * zca - s0 * zsa, s1 = s0 * zca + c0 * zsa;
      double d0 = qb * csb, e0 = qb * snb;
      double d1 = d0 * zcb - e0 * zsb, e1 = e0 * zcb + d0 * zsb;
      const double tza = 2.0 * zca, tzb = 2.0 * zcb;
#pragma unroll
      for (int st = 0; st < kRun; st += 2) {
        ar[st] += c0 + d0;
        ai[st] += s0 + e0;
        ar[st + 1] += c1 + d1;
        ai[st + 1] += s1 + e1;
        c0 = fma(tza, c1, -c0);
        s0 = fma(tza, s1, -s0);
        d0 = fma(tzb, d1, -d0);
        e0 = fma(tzb, e1, -e0);
        c1 = fma(tza, c0, -c1);
        s1 = fma(tza, s0, -s1);
        d1 = fma(tzb, d0, -d1);
        e1 = fma(tzb, e0, -e1);
      }
    }
    __syncthreads();
  }
  if (r < nruns) {
    double *out = Sg + ((g * nk + k0) * f_total + f) * 2;
#pragma unroll
    for (int st = 0; st < kRun; ++st)
      if (st < len) {
        out[st * f_total * 2] = ar[st];
        out[st * f_total * 2 + 1] = ai[st];
      }
  }
}

// Ion structure factors as a product on the FP64 matrix cores. With
// exp(i K.r) = exp(2 pi i (n_x x / L_x + n_y y / L_y)) exp(2 pi i n_z z / L_z)
// = P_c(r) Z_s(r)^(+-1) for the column c = (n_x, n_y) and s = |n_z|,
//   S(c, +s) = sum_I q_I P_c Z_s,   S(c, -s) = sum_I q_I P_c conj(Z_s).
// With q P = a + i b and Z = z + i w these are four real products over the
// ions, AZ = sum a z, BW = sum b w, AW = sum a w, BZ = sum b z:
//   S(c, +s) = (AZ - BW) + i (AW + BZ),  S(c, -s) = (AZ + BW) + i (BZ - AW),
// one pass over the ions for both signs of n_z. A workgroup takes 64
// columns (a wave each 16: the A operand rows) and NSB blocks of 16 s (the
// columns are sorted by their largest |n_z|; the body is compiled for each
// block count), and streams its ion group in chunks of SG_CH ions through
// two LDS buffers:
//   - table phase: the chunk's x / L_x, y / L_y, q and Z_s for s < 16 NSB,
//     eight threads per ion, each a run of 2 NSB consecutive s (Z_s0 by
//     sincospi of the reduced fractional phase, then Z_(s+1) = Z_s Z_1);
//     the raw positions were loaded into registers one chunk ahead;
//   - product phase: per step of 4 ions each lane forms its (column, ion)
//     entry of q P (phase_cs: a table of exp(2 pi i j / 128) and a short
//     Taylor series) and v_mfma_f64_16x16x4f64 accumulates the four
//     products for every s block.
// One barrier per chunk: the table of chunk c + 1 goes to the buffer that
// the product phase of chunk c - 1 read, and every wave has left that phase
// before the barrier of chunk c. Output: Sg as in structure_factor_kernel.
constexpr int SG_CH = 32;      // ions per LDS chunk
constexpr int SG_SB = 3;       // s blocks of 16 at most (|n_z| <= 47)

// LDS of one workgroup: two chunk buffers of Z tables (SG_CH ions x 16 NSB
// s values, sized for the largest NSB) and of x / L_x, y / L_y, q
constexpr int kTw = 128;        // entries of the table of exp(2 pi i j / kTw)
struct SfLds {
  double2 zt[2][SG_CH][16 * SG_SB];
  double su[2][SG_CH][3];
  double2 tw[kTw];
};

// (cos, sin) of 2 pi t without a library sincos: t = j / kTw + d with
// j = rint(kTw t) and |d| <= 1 / (2 kTw), and exp(2 pi i t) = exp(2 pi i j /
// kTw) exp(2 pi i d), the first factor from the table tw, the second from
// the Taylor series of cos(2 pi d) and sin(2 pi d) in d up to d^6 and d^7
// (|2 pi d| <= pi / 128: the first terms left out are below 4e-18). About
// a dozen FP64 operations, against about three times as many for sincospi;
// on this chip the FP64 vector work does not overlap the FP64 matrix-core
// products, so it adds to the kernel's time one for one.
constexpr double kTwoPi = 6.283185307179586;
constexpr double kC1 = -kTwoPi * kTwoPi / 2.0;
constexpr double kC2 = -kC1 * kTwoPi * kTwoPi / 12.0;
constexpr double kC3 = -kC2 * kTwoPi * kTwoPi / 30.0;
constexpr double kS1 = -kTwoPi * kTwoPi * kTwoPi / 6.0;
constexpr double kS2 = -kS1 * kTwoPi * kTwoPi / 20.0;
constexpr double kS3 = -kS2 * kTwoPi * kTwoPi / 42.0;
__device__ __forceinline__ void phase_cs(const double2 *tw, double t, double &c, double &s) {
  const double j = rint(t * kTw);
  const double d = fma(j, -1.0 / kTw, t);
  const double d2 = d * d;
  const double cd = fma(d2, fma(d2, fma(d2, kC3, kC2), kC1), 1.0);
  const double sd = d * fma(d2, fma(d2, fma(d2, kS3, kS2), kS1), kTwoPi);
  const double2 w = tw[(int)(int64_t)j & (kTw - 1)];
  c = fma(w.x, cd, -w.y * sd);
  s = fma(w.y, cd, w.x * sd);
}

template <int NSB>
__device__ __forceinline__ void sf_gemm_body(SfLds &L, const double *__restrict__ ion_pos,
                                             const double *__restrict__ ion_q, int64_t m,
                                             int64_t ipg, const int4 *__restrict__ kcol,
                                             int64_t cbase, int64_t f, int64_t g, double inv_lx,
                                             double inv_ly, double inv_lz, int64_t nk,
                                             int64_t f_total, double *__restrict__ Sg) {
  constexpr int NS = 16 * NSB;        // s values of the tables
  constexpr int PER = NS / 8;         // s values per table thread
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int4 mycol = kcol[cbase + wave * 16 + lr];
  const double cnx = (double)mycol.x, cny = (double)mycol.y;
  d4 acc[NSB][4];
#pragma unroll
  for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[sb][p] = d4{0.0, 0.0, 0.0, 0.0};
  const double *pf = ion_pos + f * m * 3;
  const double *qf = ion_q + f * m;
  const int64_t i0 = g * ipg, i1 = min(m, i0 + ipg);
  const int nchunks = (int)((i1 - i0 + SG_CH - 1) / SG_CH);
  // table thread: ion ti of the chunk, run tj of s values
  const int ti = tid >> 3, tj = tid & 7;
  double rx = 0.0, ry = 0.0, rz = 0.0, rq = 0.0;   // raw data of the next chunk
  auto fetch = [&](int c) {
    const int64_t I = i0 + (int64_t)c * SG_CH + ti;
    rx = ry = rz = rq = 0.0;   // missing ions: q = 0 (and Z = 1)
    if (I < i1) {
      rx = pf[3 * I];
      ry = pf[3 * I + 1];
      rz = pf[3 * I + 2];
      rq = qf[I];
    }
  };
  auto table = [&](int buf) {
    const double uz = rz * inv_lz;
    if (tj == 0) {
      L.su[buf][ti][0] = rx * inv_lx;
      L.su[buf][ti][1] = ry * inv_ly;
      L.su[buf][ti][2] = rq;
    }
    double t = (double)(tj * PER) * uz;
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    L.zt[buf][ti][tj * PER] = make_double2(cs, sn);
    if (PER > 1) {
      double t1 = uz - rint(uz), s1, c1;
      sincospi(2.0 * t1, &s1, &c1);
#pragma unroll
      for (int u = 1; u < PER; ++u) {
        const double c2 = cs * c1 - sn * s1;
        sn = sn * c1 + cs * s1;
        cs = c2;
        L.zt[buf][ti][tj * PER + u] = make_double2(cs, sn);
      }
    }
  };
  // the exp(2 pi i j / kTw) table (read after the first barrier below)
  if (tid < kTw) {
    double sj, cj;
    sincospi(2.0 * (double)tid / kTw, &sj, &cj);
    L.tw[tid] = make_double2(cj, sj);
  }
  if (nchunks > 0) {
    fetch(0);
    table(0);
  }
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    __syncthreads();
    if (c + 1 < nchunks) fetch(c + 1);   // in flight during the products
#pragma unroll 2
    for (int ks = 0; ks < SG_CH / 4; ++ks) {
      const int ion = ks * 4 + lg;
      double2 z[NSB];
#pragma unroll
      for (int sb = 0; sb < NSB; ++sb) z[sb] = L.zt[buf][ion][sb * 16 + lr];
      double sn, cs;
      phase_cs(L.tw, cnx * L.su[buf][ion][0] + cny * L.su[buf][ion][1], cs, sn);
      const double q = L.su[buf][ion][2];
      const double a = q * cs, b = q * sn;
#pragma unroll
      for (int sb = 0; sb < NSB; ++sb) {
        acc[sb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, z[sb].x, acc[sb][0], 0, 0, 0);
        acc[sb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, z[sb].y, acc[sb][1], 0, 0, 0);
        acc[sb][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, z[sb].y, acc[sb][2], 0, 0, 0);
        acc[sb][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, z[sb].x, acc[sb][3], 0, 0, 0);
      }
    }
    if (c + 1 < nchunks) table(buf ^ 1);
  }
  // D[i][j] (column i, s = j of the block) in lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int sb = 0; sb < NSB; ++sb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int4 col = kcol[cbase + wave * 16 + 4 * v + lg];
      const int sv = sb * 16 + lr;
      if (col.z < 0 || sv > col.z) continue;
      const double AZ = acc[sb][0][v], BW = acc[sb][1][v], AW = acc[sb][2][v],
                   BZ = acc[sb][3][v];
      const bool half = col.x == 0 && col.y == 0;   // n_z = 1..m only
      if (!(half && sv == 0)) {
        double *o = Sg + ((g * nk + col.w + sv) * f_total + f) * 2;
        o[0] = AZ - BW;
        o[1] = AW + BZ;
      }
      if (!half && sv > 0) {
        double *o = Sg + ((g * nk + col.w - sv) * f_total + f) * 2;
        o[0] = AZ + BW;
        o[1] = BZ - AW;
      }
    }
  }
}

// One launch for every tile: grid (frames, tiles, ion groups), so that the
// dispatch order runs through the frames of the first tiles (the most s
// blocks, the longest workgroups) first and ends with the tiles of one s
// block; the s-block count of a tile is set by its first column (the
// columns are sorted by their largest |n_z|) and selects the body compiled
// for it.
__global__ __launch_bounds__(256, 2) void sf_gemm_kernel(
    const double *__restrict__ ion_pos, const double *__restrict__ ion_q, int64_t m, int64_t ipg,
    const int4 *__restrict__ kcol, double inv_lx, double inv_ly, double inv_lz, int64_t nk,
    int64_t f_total, double *__restrict__ Sg) {
  __shared__ SfLds L;
  const int64_t f = blockIdx.x, cbase = (int64_t)blockIdx.y * kSfTile, g = blockIdx.z;
  const int nsb = (kcol[cbase].z + 16) / 16;
  if (nsb >= 3)
    sf_gemm_body<3>(L, ion_pos, ion_q, m, ipg, kcol, cbase, f, g, inv_lx, inv_ly, inv_lz, nk,
                    f_total, Sg);
  else if (nsb == 2)
    sf_gemm_body<2>(L, ion_pos, ion_q, m, ipg, kcol, cbase, f, g, inv_lx, inv_ly, inv_lz, nk,
                    f_total, Sg);
  else
    sf_gemm_body<1>(L, ion_pos, ion_q, m, ipg, kcol, cbase, f, g, inv_lx, inv_ly, inv_lz, nk,
                    f_total, Sg);
}

// S[e] = sum_g Sg[g][e] over the ion groups (fixed order)
__global__ void sum_groups_kernel(const double *__restrict__ Sg, int groups, int64_t len,
                                  double *__restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += Sg[(int64_t)g * len + e];
  S[e] = s;
}

// Back-projection of the ion structure factors onto the electrode atoms,
// split over k ranges: part[ks][f][i] = sum_{K in range ks} w_K (c_iK Re S_fK
// + s_iK Im S_fK). Each thread takes AT atoms (i = block base + thread +
// RB a) and FG frames; K data and S_f.K of BP_KCH vectors at a time are
// staged in LDS and read by all lanes at the same address. The phase of
// (i, K) is evaluated directly at the start of every run (and of the range)
// and by the n_z recurrence inside a run. Grid (atom blocks, k splits,
// frame groups).
template <int AT>
__global__ __launch_bounds__(RB) void backproject_kernel(
    const double *__restrict__ pos, int64_t n, const int32_t *__restrict__ kinfo,
    const double *__restrict__ kw, int64_t nk, int64_t kper, double inv_lx, double inv_ly,
    double inv_lz, const double *__restrict__ S, int64_t f_total, double *__restrict__ part) {
  __shared__ int4 sk[BP_KCH];
  __shared__ double sw[BP_KCH];
  __shared__ double2 ss[BP_KCH][FG];
  const int64_t ibase = (int64_t)blockIdx.x * RB * AT + threadIdx.x;
  const int64_t kbeg = (int64_t)blockIdx.y * kper;
  const int64_t kend = min(nk, kbeg + kper);
  const int64_t f0 = (int64_t)blockIdx.z * FG;
  const int nf = (int)((f_total - f0) < FG ? (f_total - f0) : FG);
  double ux[AT], uy[AT], uz[AT], zs[AT], zc[AT], cs[AT], sn[AT];
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    const int64_t i = ibase + RB * a;
    ux[a] = uy[a] = uz[a] = 0.0;
    if (i < n) {
      ux[a] = pos[3 * i] * inv_lx;
      uy[a] = pos[3 * i + 1] * inv_ly;
      uz[a] = pos[3 * i + 2] * inv_lz;
    }
    sincospi(2.0 * (uz[a] - rint(uz[a])), &zs[a], &zc[a]);
    cs[a] = 1.0;
    sn[a] = 0.0;
  }
  double acc[AT][FG];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int g = 0; g < FG; ++g) acc[a][g] = 0.0;
  const int4 *ki4 = reinterpret_cast<const int4 *>(kinfo);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BP_KCH) {
    const int cnt = (int)((kend - k0) < BP_KCH ? (kend - k0) : BP_KCH);
    for (int t = threadIdx.x; t < BP_KCH * FG; t += RB) {
      const int kk = t / FG, g = t % FG;
      double2 v = make_double2(0.0, 0.0);
      if (kk < cnt && g < nf) v = *reinterpret_cast<const double2 *>(S + ((k0 + kk) * f_total + f0 + g) * 2);
      ss[kk][g] = v;
    }
    if (threadIdx.x < cnt) {
      sk[threadIdx.x] = ki4[k0 + threadIdx.x];
      sw[threadIdx.x] = kw[k0 + threadIdx.x];
    }
    __syncthreads();
    for (int kk = 0; kk < cnt; ++kk) {
      const int4 ki = sk[kk];
      const double w = sw[kk];
      if (ki.w != 0 || k0 + kk == kbeg) {
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          double t = (double)ki.x * ux[a] + (double)ki.y * uy[a] + (double)ki.z * uz[a];
          t -= rint(t);
          sincospi(2.0 * t, &sn[a], &cs[a]);
        }
      } else {
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          const double c2 = cs[a] * zc[a] - sn[a] * zs[a];
          sn[a] = cs[a] * zs[a] + sn[a] * zc[a];
          cs[a] = c2;
        }
      }
      double wc[AT], ws[AT];
#pragma unroll
      for (int a = 0; a < AT; ++a) {
        wc[a] = w * cs[a];
        ws[a] = w * sn[a];
      }
#pragma unroll
      for (int g = 0; g < FG; ++g) {
        const double2 sv = ss[kk][g];
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          acc[a][g] = fma(wc[a], sv.x, acc[a][g]);
          acc[a][g] = fma(ws[a], sv.y, acc[a][g]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    const int64_t i = ibase + RB * a;
    if (i < n) {
#pragma unroll
      for (int g = 0; g < FG; ++g)
        if (g < nf) part[((int64_t)blockIdx.y * f_total + f0 + g) * n + i] = acc[a][g];
    }
  }
}

// Factored back-projection for electrode atoms on few z-planes. With
// exp(i K.r) = P_c(x, y) Z_nz(z), P_c = exp(2 pi i (n_x x / L_x + n_y y / L_y)),
// Z_nz = exp(2 pi i n_z z / L_z), for the column c = (n_x, n_y):
//   sum_K w_K Re(exp(-i K.r_i) S_fK) = sum_c Re(conj(P_c(r_i)) T_f(p, c)),
//   T_f(p, c) = sum_nz w_(c, nz) conj(Z_nz(z_p)) S_f(c, nz),
// where z_p is the z shared by every atom of plane p: the n_z sums are
// taken once per (plane, column, frame) instead of once per atom.
//
// plane_table_kernel: T as Re / Im arrays [plane][column][frame] (zero for
// the padding columns). Grid (columns * frames / PT_THREADS, planes); the
// plane's Z_s for s = 0..smax sit in LDS (sincospi of the reduced
// fractional phase), Z_-s = conj(Z_s).
constexpr int PT_THREADS = 256;

__global__ __launch_bounds__(PT_THREADS) void plane_table_kernel(
    const double *__restrict__ plane_uz, const int4 *__restrict__ kcol, int64_t ncols_pad,
    const double *__restrict__ kw, const double *__restrict__ S, int64_t f_total, int smax,
    double *__restrict__ Tre, double *__restrict__ Tim) {
  __shared__ double2 zt[kMaxPlaneS + 1];
  const int p = blockIdx.y;
  const double u = plane_uz[p];
  for (int sv = threadIdx.x; sv <= smax; sv += PT_THREADS) {
    double t = (double)sv * u;
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    zt[sv] = make_double2(cs, sn);
  }
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * PT_THREADS + threadIdx.x;
  if (idx >= ncols_pad * f_total) return;
  const int64_t c = idx / f_total, f = idx - c * f_total;
  const int4 col = kcol[c];
  double re = 0.0, im = 0.0;
  if (col.z >= 0) {
    // (0, 0) holds n_z = 1..m only
    const int lo = (col.x == 0 && col.y == 0) ? 1 : -col.z;
    for (int nz = lo; nz <= col.z; ++nz) {
      const int64_t k = (int64_t)col.w + nz;
      const double2 sv = *reinterpret_cast<const double2 *>(S + (k * f_total + f) * 2);
      const double w = kw[k];
      const double2 z = zt[nz < 0 ? -nz : nz];
      const double zi = nz < 0 ? -z.y : z.y;   // Im Z_nz
      // conj(Z) S = (Re Z Re S + Im Z Im S) + i (Re Z Im S - Im Z Re S)
      re = fma(w, fma(z.x, sv.x, zi * sv.y), re);
      im = fma(w, fma(z.x, sv.y, -zi * sv.x), im);
    }
  }
  const int64_t o = ((int64_t)p * ncols_pad + c) * f_total + f;
  Tre[o] = re;
  Tim[o] = im;
}

// part[f][i] = sum_c cos(theta_ic) Re T_f(p, c) + sin(theta_ic) Im T_f(p, c),
// theta_ic = 2 pi (n_x x_i / L_x + n_y y_i / L_y): the product
// [atoms x (cos, sin) of the columns] . [(Re T, Im T) x frames] on the FP64
// matrix cores. One wave per tile of kPlaneTile atoms of one plane and up to
// 32 frames: per step of 4 columns, lane (r, q) forms the phase of atom r
// and column q once (sincospi of the reduced fractional phase) and gives
// its cosine and sine as the A operand of two v_mfma_f64_16x16x4f64 per 16
// frames, with Re T and Im T of (column q, frame r) as the B operand.
// Grid (tiles / PB_WAVES, frames / 32, column splits): split z takes the
// columns [z cper, (z + 1) cper) and writes part + z f n (summed with the
// other splits when b is assembled).
constexpr int PB_WAVES = 4;

__global__ __launch_bounds__(64 * PB_WAVES) void plane_backproject_kernel(
    const double *__restrict__ pos, int64_t n, const int32_t *__restrict__ tile_plane,
    const int32_t *__restrict__ tile_atom, int64_t ntiles, const int4 *__restrict__ kcol,
    int64_t ncols_pad, int64_t cper, double inv_lx, double inv_ly,
    const double *__restrict__ Tre, const double *__restrict__ Tim, int64_t f_total,
    double *__restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t cbeg = (int64_t)blockIdx.z * cper, cend = min(ncols_pad, cbeg + cper);
  part += (int64_t)blockIdx.z * f_total * n;
  const int64_t t = (int64_t)blockIdx.x * PB_WAVES + wave;
  if (t >= ntiles) return;   // no barriers below: a wave may leave alone
  const int lr = lane & 15, lq = lane >> 4;
  const int p = tile_plane[t];
  const int32_t atom = tile_atom[t * kPlaneTile + lr];
  double ux = 0.0, uy = 0.0;
  if (atom >= 0) {
    ux = pos[3 * (int64_t)atom] * inv_lx;
    uy = pos[3 * (int64_t)atom + 1] * inv_ly;
  }
  const int64_t fa = (int64_t)blockIdx.y * 32 + lr, fb = fa + 16;
  const bool va = fa < f_total, vb = fb < f_total;
  const double *tr = Tre + (int64_t)p * ncols_pad * f_total;
  const double *ti = Tim + (int64_t)p * ncols_pad * f_total;
  d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = cbeg; c0 < cend; c0 += 4) {
    const int64_t c = c0 + lq;
    const int4 col = kcol[c];
    double th = (double)col.x * ux + (double)col.y * uy;
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    const int64_t o = c * f_total;
    const double ra = va ? tr[o + fa] : 0.0, ia = va ? ti[o + fa] : 0.0;
    const double rb = vb ? tr[o + fb] : 0.0, ib = vb ? ti[o + fb] : 0.0;
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(cs, ra, acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, ia, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(cs, rb, acc1, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, ib, acc1, 0, 0, 0);
  }
  // D[i][j] (atom i of the tile, frame j) in lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int32_t a = tile_atom[t * kPlaneTile + 4 * v + lq];
    if (a < 0) continue;
    if (va) part[fa * n + a] = acc0[v];
    if (vb) part[fb * n + a] = acc1[v];
  }
}

// b[f, i] = chi_i / k_e - sum_ks bp[ks][f][i] - sum_g rs[g][f][i] - c0 Q_f
// (fixed order over the k splits and ion groups); slab geometry (Eq. 39 in
// its definite form): - (4 pi / V) M1_f z_i.
__global__ void assemble_b_kernel(const double *__restrict__ bp, int ksplits,
                                  const double *__restrict__ rs, int rgroups, int64_t n,
                                  int64_t f_total, const double *__restrict__ chi,
                                  const double *__restrict__ qsol, double c0,
                                  const double *__restrict__ m1, double cs,
                                  const double *__restrict__ pos, double *__restrict__ b) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * f_total) return;
  const int64_t f = idx / n, i = idx % n;
  const int64_t fn = n * f_total;
  double s = 0.0;
#pragma unroll 8
  for (int ks = 0; ks < ksplits; ++ks) s += bp[ks * fn + idx];
#pragma unroll 8
  for (int g = 0; g < rgroups; ++g) s += rs[g * fn + idx];
  double v = chi[i] * (1.0 / kCoulombVA) - s - c0 * qsol[f];
  if (m1 != nullptr) v -= cs * m1[f] * pos[3 * i + 2];
  b[idx] = v;
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

// One thread per (electrode atom, frame, ion group); ions stream through LDS.
// rs[g][f][i] = sum_{I in group g} q_I sum_images [erfc(beta d) - erfc(a_i d)] / d.
// Thread t takes atom order[t] (compact spatial tiles), so a wavefront's
// atoms are close together and the branch into the erfc terms is taken by
// all lanes or none for most ions.
__global__ __launch_bounds__(RB) void real_space_ions_kernel(
    const double *__restrict__ pos, const double *__restrict__ width,
    const int32_t *__restrict__ order, int64_t n, const double *__restrict__ ion_pos,
    const double *__restrict__ ion_q, int64_t m, int64_t ipg, double lx, double ly, double lz,
    double beta, double rcut, int64_t f_total, const double *__restrict__ etab,
    double *__restrict__ rs) {
  __shared__ double si[RB][4];
  __shared__ double et[kErfcTab];
  for (int q = threadIdx.x; q < kErfcTab; q += RB) et[q] = etab[q];
  __syncthreads();
  const int64_t f = blockIdx.y, g = blockIdx.z;
  const int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x;
  const int64_t i = t < n ? (int64_t)order[t] : -1;
  double xi = 0, yi = 0, zi = 0, ai = 1.0;
  if (i >= 0) {
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
  const int64_t i0 = g * ipg, i1 = min(m, i0 + ipg);
  for (int64_t base = i0; base < i1; base += RB) {
    const int64_t I = base + threadIdx.x;
    if (I < i1) {
      si[threadIdx.x][0] = pf[3 * I];
      si[threadIdx.x][1] = pf[3 * I + 1];
      si[threadIdx.x][2] = pf[3 * I + 2];
      si[threadIdx.x][3] = qf[I];
    }
    __syncthreads();
    const int cnt = (int)((i1 - base) < RB ? (i1 - base) : RB);
    if (i >= 0) {
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
                  acc += q * ((erfc_pw(et, beta * d) - erfc_pw(et, ai * d)) / d);
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
  if (i >= 0) rs[(g * f_total + f) * n + i] = acc;
}

// ---- real space over a cell list of the ions of each frame
//
// The box is cut into ncx x ncy x ncz cells (edges h_d = L_d / nc_d >=
// rcut / 2, at most kMaxCells cells); cell (cx, cy, cz) has index
// (cz ncy + cy) ncx + cx. Every frame's ions are put in cell order, ions of
// one cell in index order (a stable counting sort), in three steps:
//   cell_sort_chunk_kernel  per chunk of kChunk ions: keys (cell << 12 |
//                           local index) sorted in LDS (bitonic; unique keys,
//                           so the order is fixed), the chunk's count per cell
//   cell_scan_kernel        per frame: prefix sums of the counts over the
//                           chunks (per cell) and over the cells
//   cell_scatter_kernel     every ion to cell start + earlier chunks' count +
//                           its rank in its chunk, as (x, y, z, q)
// real_space_cell_kernel then gives each wavefront of 64 spatially compact
// atoms the cells that overlap its bounding box widened by rcut: one
// contiguous range of the sorted ions per (cz, cy) row (two where the x
// range wraps), so the sum runs in a fixed order.
constexpr int kChunk = 4096;            // ions per sorting chunk (12-bit local index)
constexpr int kChunkThreads = 1024;
constexpr int kMaxCells = 8192;         // 13-bit cell index; counts of a chunk fit in LDS

__device__ inline int cell_coord(double x, double L, double invh, int nc) {
  double xw = x - L * floor(x / L);
  int c = (int)(xw * invh);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ __launch_bounds__(kChunkThreads) void cell_sort_chunk_kernel(
    const double *__restrict__ ion_pos, int64_t m, int64_t nchunks, double lx, double ly,
    double lz, double ihx, double ihy, double ihz, int ncx, int ncy, int ncz,
    uint32_t *__restrict__ skeys, int32_t *__restrict__ hist) {
  __shared__ uint32_t keys[kChunk];
  const int64_t chunk = blockIdx.x, f = blockIdx.y;
  const int64_t i0 = chunk * kChunk;
  const int cnt = (int)((m - i0) < kChunk ? (m - i0) : kChunk);
  const double *pf = ion_pos + (f * m + i0) * 3;
  for (int j = threadIdx.x; j < kChunk; j += kChunkThreads) {
    uint32_t key = 0xffffffffu;
    if (j < cnt) {
      const int cx = cell_coord(pf[3 * j], lx, ihx, ncx);
      const int cy = cell_coord(pf[3 * j + 1], ly, ihy, ncy);
      const int cz = cell_coord(pf[3 * j + 2], lz, ihz, ncz);
      key = ((uint32_t)((cz * ncy + cy) * ncx + cx) << 12) | (uint32_t)j;
    }
    keys[j] = key;
  }
  __syncthreads();
  for (int k = 2; k <= kChunk; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = threadIdx.x; i < kChunk; i += kChunkThreads) {
        const int ixj = i ^ jj;
        if (ixj > i) {
          const uint32_t a = keys[i], b = keys[ixj];
          if ((a > b) == ((i & k) == 0)) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < cnt; j += kChunkThreads) skeys[f * m + i0 + j] = keys[j];
  // count of cell c = first position of cell c + 1 - first position of c
  const int ncell = ncx * ncy * ncz;
  int32_t *h = hist + (f * nchunks + chunk) * ncell;
  for (int c = threadIdx.x; c < ncell; c += kChunkThreads) {
    int lo = 0, hi = cnt;
    const uint32_t t0 = (uint32_t)c << 12;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (keys[mid] < t0) lo = mid + 1;
      else hi = mid;
    }
    int lo2 = lo, hi2 = cnt;
    const uint32_t t1 = (uint32_t)(c + 1) << 12;
    while (lo2 < hi2) {
      const int mid = (lo2 + hi2) >> 1;
      if (keys[mid] < t1) lo2 = mid + 1;
      else hi2 = mid;
    }
    h[c] = lo2 - lo;
  }
}

// One workgroup per frame: off[f][chunk][c] = sum of the counts of cell c in
// the earlier chunks; cstart[f][c] = number of ions in cells before c
// (cstart[f][ncell] = m).
__global__ __launch_bounds__(kChunkThreads) void cell_scan_kernel(
    int32_t *__restrict__ hist, int64_t nchunks, int ncell, int64_t m,
    int32_t *__restrict__ cstart) {
  __shared__ int32_t tot[kMaxCells];
  __shared__ int32_t part[kChunkThreads];
  const int64_t f = blockIdx.x;
  int32_t *h = hist + f * nchunks * ncell;
  for (int c = threadIdx.x; c < ncell; c += kChunkThreads) {
    int32_t run = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
      const int32_t v = h[ch * ncell + c];
      h[ch * ncell + c] = run;
      run += v;
    }
    tot[c] = run;
  }
  __syncthreads();
  // exclusive scan of tot over the cells: each thread a contiguous slice
  const int per = (ncell + kChunkThreads - 1) / kChunkThreads;
  const int c0 = threadIdx.x * per, c1 = min(ncell, c0 + per);
  int32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += tot[c];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int t = 0; t < kChunkThreads; ++t) {
      const int32_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t run = part[threadIdx.x];
  int32_t *cs = cstart + f * (ncell + 1);
  for (int c = c0; c < c1; ++c) {
    cs[c] = run;
    run += tot[c];
  }
  if (threadIdx.x == 0) cs[ncell] = (int32_t)m;
}

__global__ __launch_bounds__(kChunkThreads) void cell_scatter_kernel(
    const double *__restrict__ ion_pos, const double *__restrict__ ion_q, int64_t m,
    int64_t nchunks, int ncell, const uint32_t *__restrict__ skeys,
    const int32_t *__restrict__ off, const int32_t *__restrict__ cstart,
    double4 *__restrict__ sorted) {
  __shared__ uint32_t keys[kChunk];
  const int64_t chunk = blockIdx.x, f = blockIdx.y;
  const int64_t i0 = chunk * kChunk;
  const int cnt = (int)((m - i0) < kChunk ? (m - i0) : kChunk);
  for (int j = threadIdx.x; j < cnt; j += kChunkThreads) keys[j] = skeys[f * m + i0 + j];
  __syncthreads();
  const int32_t *o = off + (f * nchunks + chunk) * ncell;
  const int32_t *cs = cstart + f * (ncell + 1);
  const double *pf = ion_pos + f * m * 3;
  const double *qf = ion_q + f * m;
  for (int j = threadIdx.x; j < cnt; j += kChunkThreads) {
    const uint32_t key = keys[j];
    const int c = (int)(key >> 12);
    const int64_t I = i0 + (int64_t)(key & 0xfffu);
    int lo = 0, hi = j;   // first position of cell c in the chunk
    const uint32_t t0 = (uint32_t)c << 12;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (keys[mid] < t0) lo = mid + 1;
      else hi = mid;
    }
    const int64_t dst = (int64_t)cs[c] + o[c] + (j - lo);
    sorted[f * m + dst] = make_double4(pf[3 * I], pf[3 * I + 1], pf[3 * I + 2], qf[I]);
  }
}

// Cells [a, b] (unwrapped, a <= b) along one edge of nc cells: all of them
// once when the range covers the edge.
__device__ inline void cell_span(double lo, double hi, double invh, int nc, int &a, int &b) {
  a = (int)floor(lo * invh);
  b = (int)floor(hi * invh);
  if (b - a + 1 >= nc) {
    a = 0;
    b = nc - 1;
  }
}

__device__ inline int wrap_cell(int c, int nc) {
  c %= nc;
  return c < 0 ? c + nc : c;
}

__global__ __launch_bounds__(64) void real_space_cell_kernel(
    const double *__restrict__ pos, const double *__restrict__ width,
    const int32_t *__restrict__ order, int64_t n, const double4 *__restrict__ sorted,
    const int32_t *__restrict__ cstart, int64_t m, int ncx, int ncy, int ncz, double lx,
    double ly, double lz, double beta, double rcut, int64_t f_total,
    const double *__restrict__ etab, double *__restrict__ rs) {
  __shared__ double4 si[64];
  __shared__ double et[kErfcTab];
  for (int q = threadIdx.x; q < kErfcTab; q += 64) et[q] = etab[q];
  __syncthreads();
  const int64_t f = blockIdx.y;
  const int lane = threadIdx.x;
  const int64_t t = (int64_t)blockIdx.x * 64 + lane;
  const int64_t i = t < n ? (int64_t)order[t] : -1;
  double xi = 0, yi = 0, zi = 0, ai = 1.0;
  if (i >= 0) {
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
    ai = width[i];
  }
  const double ilx = 1.0 / lx, ily = 1.0 / ly, ilz = 1.0 / lz;
  const bool wx = lx >= 2.0 * rcut, wy = ly >= 2.0 * rcut, wz = lz >= 2.0 * rcut;
  // bounding box of the tile about its first atom (lane 0 always holds one)
  const double xr = __shfl(xi, 0, 64), yr = __shfl(yi, 0, 64), zr = __shfl(zi, 0, 64);
  double ex0 = xi - xr, ey0 = yi - yr, ez0 = zi - zr;
  ex0 -= lx * rint(ex0 * ilx);
  ey0 -= ly * rint(ey0 * ily);
  ez0 -= lz * rint(ez0 * ilz);
  if (i < 0) ex0 = ey0 = ez0 = 0.0;
  double xmin = ex0, xmax = ex0, ymin = ey0, ymax = ey0, zmin = ez0, zmax = ez0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    xmin = fmin(xmin, __shfl_xor(xmin, o, 64));
    xmax = fmax(xmax, __shfl_xor(xmax, o, 64));
    ymin = fmin(ymin, __shfl_xor(ymin, o, 64));
    ymax = fmax(ymax, __shfl_xor(ymax, o, 64));
    zmin = fmin(zmin, __shfl_xor(zmin, o, 64));
    zmax = fmax(zmax, __shfl_xor(zmax, o, 64));
  }
  // cells meeting the box widened by rcut (and a hair for rounding at cell
  // edges; the distance test below is exact)
  const double rw = rcut * (1.0 + 1e-9) + 1e-9;
  int xa, xb, ya, yb, za, zb;
  cell_span(xr + xmin - rw, xr + xmax + rw, ncx * ilx, ncx, xa, xb);
  cell_span(yr + ymin - rw, yr + ymax + rw, ncy * ily, ncy, ya, yb);
  cell_span(zr + zmin - rw, zr + zmax + rw, ncz * ilz, ncz, za, zb);
  const int32_t *cs = cstart + f * ((int64_t)ncx * ncy * ncz + 1);
  const double4 *sf = sorted + f * m;
  const double rc2 = rcut * rcut;
  const double lim0 = 2.0 * (ai - beta) * 0.56418958354775628695;
  const int xlen = xb - xa + 1, xw0 = wrap_cell(xa, ncx);
  double acc = 0.0;
  for (int cz = za; cz <= zb; ++cz) {
    const int czw = wrap_cell(cz, ncz);
    for (int cy = ya; cy <= yb; ++cy) {
      const int64_t row = ((int64_t)czw * ncy + wrap_cell(cy, ncy)) * ncx;
      for (int part = 0; part < 2; ++part) {
        int c0, c1;   // cells [c0, c1) of the row
        if (part == 0) {
          c0 = xw0;
          c1 = min(ncx, xw0 + xlen);
        } else {
          c0 = 0;
          c1 = xw0 + xlen - ncx;
          if (c1 <= 0) break;
        }
        const int64_t s0 = cs[row + c0], s1 = cs[row + c1];
        for (int64_t base = s0; base < s1; base += 64) {
          const int64_t q = base + lane;
          if (q < s1) si[lane] = sf[q];
          __syncthreads();
          const int cnt = (int)((s1 - base) < 64 ? (s1 - base) : 64);
          if (i >= 0) {
            for (int j = 0; j < cnt; ++j) {
              const double4 ion = si[j];
              double dz = zi - ion.z;
              dz -= lz * rint(dz * ilz);
              int iza, izb;
              image_range(dz, lz, ilz, rcut, wz, iza, izb);
              if (iza > izb) continue;
              double dx = xi - ion.x;
              double dy = yi - ion.y;
              dx -= lx * rint(dx * ilx);
              dy -= ly * rint(dy * ily);
              int ixa, ixb, iya, iyb;
              image_range(dx, lx, ilx, rcut, wx, ixa, ixb);
              image_range(dy, ly, ily, rcut, wy, iya, iyb);
              const double qv = ion.w;
              for (int a = ixa; a <= ixb; ++a) {
                const double ex = dx + (double)a * lx;
                for (int bb = iya; bb <= iyb; ++bb) {
                  const double ey = dy + (double)bb * ly;
                  const double exy = ex * ex + ey * ey;
                  if (exy >= rc2) continue;
                  for (int c = iza; c <= izb; ++c) {
                    const double ez = dz + (double)c * lz;
                    const double d2 = exy + ez * ez;
                    if (d2 < rc2) {
                      if (d2 > 0.0) {
                        const double d = sqrt(d2);
                        acc += qv * ((erfc_pw(et, beta * d) - erfc_pw(et, ai * d)) / d);
                      } else {
                        acc += qv * lim0;
                      }
                    }
                  }
                }
              }
            }
          }
          __syncthreads();
        }
      }
    }
  }
  if (i >= 0) rs[f * n + i] = acc;
}

}  // namespace

namespace {

// Work split of one cpm_rhs call over f frames of m ions, and the layout of
// its scratch buffer:
//   S   [nk][f][2]             structure factors
//   Sg  [sf_groups][nk][f][2]  per ion group (only when sf_groups > 1)
//   bp  [ksplit][f][n]         back-projection partials
//   T   [2][planes][cols][f]   per-plane n_z sums (factored back-projection)
//   rs  [rs_groups][f][n]      real-space partials
struct RhsPlan {
  int64_t sf_groups = 1, sf_ipg = 0, ksplit = 0, kper = 0, rs_groups = 0, rs_ipg = 0;
  bool sf_gemm = false;         // structure factors on the matrix cores (|n_z| <= 47)
  bool bp_plane = false;        // factored back-projection over the atoms' z-planes
  bool rs_cell = false;         // real space over the cell list of the ions
  int nc[3] = {1, 1, 1};        // cells per box edge
  int64_t nchunks = 0;          // sorting chunks per frame
  int64_t off_sg = 0, off_bp = 0, off_tp = 0, off_rs = 0, off_m1 = 0, off_sorted = 0, off_keys = 0,
          off_hist = 0, off_cstart = 0, total = 0;
};

// below this many ions per frame the cell list costs more than it saves
// (measured: 2000 ions, 4608 atoms: the all-pairs kernel takes 126 us)
constexpr int64_t kCellMinIons = 8192;

// Cells of edge >= rcut / 2 (widened until there are at most kMaxCells).
void cell_grid(const double box[3], double rcut, int nc[3]) {
  double h = 0.5 * rcut;
  for (;;) {
    int64_t tot = 1;
    for (int d = 0; d < 3; ++d) {
      nc[d] = std::max(1, (int)std::floor(box[d] / h));
      tot *= nc[d];
    }
    if (tot <= kMaxCells) return;
    h *= 1.25;
  }
}

constexpr int64_t kTargetBlocks = 2048;          // workgroups that fill the chip several times
constexpr int64_t kPartialCap = (int64_t)1 << 27;  // doubles per partial buffer

// groups of at least RB items each, enough for ~kTargetBlocks workgroups,
// at most 64 and at most cap
int64_t groups_for(int64_t blocks, int64_t items, int64_t cap, int64_t &per) {
  int64_t g = (kTargetBlocks + blocks - 1) / std::max<int64_t>(1, blocks);
  g = std::min<int64_t>({g, std::max<int64_t>(1, items / RB), 64, std::max<int64_t>(1, cap)});
  g = std::max<int64_t>(1, g);
  per = (items + g - 1) / g;
  return per > 0 ? (items + per - 1) / per : 1;
}

// cap_* > 0 bound the ion groups of the structure factor, the k splits of
// the back-projection and the ion groups of the real-space sum (fewer
// partial buffers, less parallelism)
RhsPlan rhs_plan_capped(const cpm_system *s, int64_t m, int64_t f, int64_t cap_sf,
                        int64_t cap_ks, int64_t cap_rs, bool planes) {
  RhsPlan p;
  const int64_t n = s->n, nk = std::max<int64_t>(s->kset.nk, 1);
  const int64_t rblocks = (s->kset.nruns + RB - 1) / RB;
  const int64_t iblocks = (n + RB - 1) / RB, fgroups = (f + FG - 1) / FG;
  const int64_t bblocks = (n + RB * BP_AT - 1) / (RB * BP_AT);
  if (m > 0 && s->kset.nk > 0) {
    p.sf_gemm = s->kset.smax < SG_SB * 16;
    const int64_t sf_blocks = p.sf_gemm ? (s->kset.ncols_pad / kSfTile) * f
                                        : std::max<int64_t>(1, rblocks) * f;
    p.sf_groups = groups_for(sf_blocks, m, std::min(cap_sf, kPartialCap / (2 * nk * f)), p.sf_ipg);
    // k splits of the back-projection: as many as fill every SIMD with three
    // wavefronts (its occupancy) without a fourth on some, at least 32 k each
    const int64_t per = bblocks * fgroups * (RB / 64);
    int64_t ks = std::max<int64_t>(1, (3 * 1024) / per);
    ks = std::min<int64_t>({ks, std::max<int64_t>(1, nk / 32),
                            std::max<int64_t>(1, kPartialCap / (f * n)), cap_ks});
    p.kper = (nk + ks - 1) / ks;
    p.ksplit = (nk + p.kper - 1) / p.kper;
    if (planes && s->nplanes > 0) {
      // column splits (multiples of 64 columns) until about 1024 workgroups
      p.bp_plane = true;
      const int64_t wgs = (s->plane_ntiles + 3) / 4 * ((f + 31) / 32);
      const int64_t units = s->kset.ncols_pad / 64;
      int64_t cs = std::min<int64_t>({std::max<int64_t>(1, (1024 + wgs - 1) / wgs), units,
                                      std::max<int64_t>(1, kPartialCap / (f * n)), cap_ks});
      cs = std::max<int64_t>(1, cs);
      p.kper = (units + cs - 1) / cs * 64;   // columns per split
      p.ksplit = (s->kset.ncols_pad + p.kper - 1) / p.kper;
    }
  }
  if (m >= kCellMinIons) {
    p.rs_cell = true;
    cell_grid(s->box, s->rcut, p.nc);
    p.nchunks = (m + kChunk - 1) / kChunk;
    p.rs_groups = 1;
  } else if (m > 0) {
    p.rs_groups = groups_for(iblocks * f, m, std::min(cap_rs, kPartialCap / (f * n)), p.rs_ipg);
  }
  const int64_t ncell = (int64_t)p.nc[0] * p.nc[1] * p.nc[2];
  p.off_sg = 2 * nk * f;
  p.off_bp = p.off_sg + (p.sf_groups > 1 ? p.sf_groups * 2 * nk * f : 0);
  p.off_tp = p.off_bp + p.ksplit * f * n;
  p.off_rs = p.off_tp + (p.bp_plane ? 2 * (int64_t)s->nplanes * s->kset.ncols_pad * f : 0);
  p.off_m1 = p.off_rs + p.rs_groups * f * n;
  p.off_sorted = (p.off_m1 + f + 3) / 4 * 4;   // 32-byte aligned (double4)
  p.off_keys = p.off_sorted + (p.rs_cell ? 4 * f * m : 0);
  p.off_hist = p.off_keys + (p.rs_cell ? (f * m + 1) / 2 : 0);
  p.off_cstart = p.off_hist + (p.rs_cell ? (f * p.nchunks * ncell + 1) / 2 : 0);
  p.total = p.off_cstart + (p.rs_cell ? (f * (ncell + 1) + 1) / 2 : 0);
  return p;
}

constexpr int64_t kNoCap = (int64_t)1 << 40;

// the default plan, or with limit > 0 the most parallel plan whose scratch
// holds at most limit doubles (halving the largest partial count first)
RhsPlan rhs_plan(const cpm_system *s, int64_t m, int64_t f, int64_t limit = 0) {
  // the factored back-projection first; without it when its per-plane sums
  // do not fit the limit
  for (int planes = 1;; planes = 0) {
    RhsPlan p = rhs_plan_capped(s, m, f, kNoCap, kNoCap, kNoCap, planes != 0);
    int64_t csf = p.sf_groups, cks = std::max<int64_t>(1, p.ksplit), crs = p.rs_groups;
    while (limit > 0 && p.total > limit && (csf > 1 || cks > 1 || crs > 1)) {
      const int64_t nk = std::max<int64_t>(s->kset.nk, 1);
      const int64_t wsf = csf > 1 ? csf * 2 * nk * f : 0, wks = cks > 1 ? cks * f * s->n : 0,
                    wrs = crs > 1 ? crs * f * s->n : 0;
      if (wsf >= wks && wsf >= wrs) csf = std::max<int64_t>(1, csf / 2);
      else if (wks >= wrs) cks = std::max<int64_t>(1, cks / 2);
      else crs = std::max<int64_t>(1, crs / 2);
      p = rhs_plan_capped(s, m, f, csf, cks, crs, planes != 0);
    }
    if (limit <= 0 || p.total <= limit || !p.bp_plane) return p;
  }
}

// ---- cpm_rhs_noalloc: the scratch in a fixed device array
//
// kStaticRhsScratch doubles (32 MiB) per GPU, held by the code object until
// the process ends. Host code takes its device address from
// hipGetSymbolAddress (per device, on first use): the array's name in host
// code is not a device address.
constexpr int64_t kStaticRhsScratch = (int64_t)1 << 22;

}  // namespace

static __device__ __align__(256) double scratch[kStaticRhsScratch];

int64_t rhs_scratch_elems(const cpm_system *s, int64_t m, int64_t f) {
  return rhs_plan(s, m, f).total;
}

int64_t rhs_static_scratch_elems() { return kStaticRhsScratch; }

int64_t rhs_scratch_elems_capped(const cpm_system *s, int64_t m, int64_t f, int64_t limit) {
  return rhs_plan(s, m, f, limit).total;
}

hipError_t rhs_static_scratch(double **ptr) {
  static std::mutex mu;
  static std::vector<double *> per_device;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)per_device.size() <= dev) per_device.resize(dev + 1, nullptr);
  if (!per_device[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[dev] = static_cast<double *>(p);
  }
  *ptr = per_device[dev];
  return hipSuccess;
}

hipError_t launch_rhs(hipStream_t st, const cpm_system *s, const double *ion_pos,
                      const double *ion_q, int64_t m, int64_t f, const double *chi, double *buf,
                      double *b_out, double *qsol_out, int64_t limit) {
  const double ilx = 1.0 / s->box[0], ily = 1.0 / s->box[1], ilz = 1.0 / s->box[2];
  const int64_t nk = s->kset.nk, n = s->n;
  const double c0 = -M_PI / (s->vol * s->beta * s->beta);
  const RhsPlan p = rhs_plan(s, m, f, limit);
  double *S = buf, *bp = buf + p.off_bp, *rs = buf + p.off_rs;
  const int64_t iblocks = (n + RB - 1) / RB, fgroups = (f + FG - 1) / FG;
  double *m1 = s->slab ? buf + p.off_m1 : nullptr;
  if (m > 0) {
    hipLaunchKernelGGL(qsum_kernel, dim3((unsigned)f), dim3(RB), 0, st, ion_q, m, qsol_out, ion_pos,
                       s->box[2], m1);
  } else {
    // zeros by a kernel (no memset node when the caller captures the stream)
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((f + 255) / 256)), dim3(256), 0, st,
                       qsol_out, f);
    if (m1)
      hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((f + 255) / 256)), dim3(256), 0, st,
                         m1, f);
  }
  if (p.ksplit > 0) {
    double *Sg = p.sf_groups > 1 ? buf + p.off_sg : S;
    const int64_t rblocks = (s->kset.nruns + RB - 1) / RB;
    // live timing (cpm_profile_enable): algorithmic flops 4 n_k m f
    hipEvent_t ea = nullptr, eb = nullptr;
    if (s->prof.sample(4)) {
      Profile::Rec &r = s->prof.add(4, 4.0 * (double)nk * (double)m * (double)f);
      ea = r.a;
      eb = r.b;
    }
    if (p.sf_gemm) {
      hipExtLaunchKernelGGL(sf_gemm_kernel,
                            dim3((unsigned)f, (unsigned)(s->kset.ncols_pad / kSfTile),
                                 (unsigned)p.sf_groups),
                            dim3(256), 0, st, ea, eb, 0, ion_pos, ion_q, m, p.sf_ipg,
                            reinterpret_cast<const int4 *>(s->kcol), ilx, ily, ilz, nk, f, Sg);
    } else
      hipExtLaunchKernelGGL(structure_factor_kernel,
                            dim3((unsigned)rblocks, (unsigned)f, (unsigned)p.sf_groups), dim3(RB),
                            0, st, ea, eb, 0, ion_pos, ion_q, m, p.sf_ipg, s->kinfo, s->krun,
                            s->kset.nruns, nk, ilx, ily, ilz, f, Sg);
    if (p.sf_groups > 1) {
      const int64_t len = 2 * nk * f;
      hipLaunchKernelGGL(sum_groups_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st,
                         Sg, (int)p.sf_groups, len, S);
    }
    if (p.bp_plane) {
      const int64_t ncp = s->kset.ncols_pad;
      double *Tre = buf + p.off_tp, *Tim = Tre + (int64_t)s->nplanes * ncp * f;
      hipLaunchKernelGGL(plane_table_kernel,
                         dim3((unsigned)((ncp * f + PT_THREADS - 1) / PT_THREADS),
                              (unsigned)s->nplanes),
                         dim3(PT_THREADS), 0, st, (const double *)s->plane_uz,
                         reinterpret_cast<const int4 *>(s->kcol), ncp, (const double *)s->kw,
                         (const double *)S, f, s->kset.smax, Tre, Tim);
      hipLaunchKernelGGL(plane_backproject_kernel,
                         dim3((unsigned)((s->plane_ntiles + PB_WAVES - 1) / PB_WAVES),
                              (unsigned)((f + 31) / 32), (unsigned)p.ksplit),
                         dim3(64 * PB_WAVES), 0, st, (const double *)s->pos, n,
                         (const int32_t *)s->plane_tile, (const int32_t *)s->plane_atom,
                         s->plane_ntiles, reinterpret_cast<const int4 *>(s->kcol), ncp, p.kper,
                         ilx, ily, (const double *)Tre, (const double *)Tim, f, bp);
    } else {
      const int64_t bblocks = (n + RB * BP_AT - 1) / (RB * BP_AT);
      hipLaunchKernelGGL(backproject_kernel<BP_AT>,
                         dim3((unsigned)bblocks, (unsigned)p.ksplit, (unsigned)fgroups), dim3(RB),
                         0, st, s->pos, n, s->kinfo, s->kw, nk, p.kper, ilx, ily, ilz, S, f, bp);
    }
  }
  if (p.rs_cell) {
    double4 *sorted = reinterpret_cast<double4 *>(buf + p.off_sorted);
    uint32_t *keys = reinterpret_cast<uint32_t *>(buf + p.off_keys);
    int32_t *hist = reinterpret_cast<int32_t *>(buf + p.off_hist);
    int32_t *cstart = reinterpret_cast<int32_t *>(buf + p.off_cstart);
    const int ncell = p.nc[0] * p.nc[1] * p.nc[2];
    hipLaunchKernelGGL(cell_sort_chunk_kernel, dim3((unsigned)p.nchunks, (unsigned)f),
                       dim3(kChunkThreads), 0, st, ion_pos, m, p.nchunks, s->box[0], s->box[1],
                       s->box[2], p.nc[0] * ilx, p.nc[1] * ily, p.nc[2] * ilz, p.nc[0], p.nc[1],
                       p.nc[2], keys, hist);
    hipLaunchKernelGGL(cell_scan_kernel, dim3((unsigned)f), dim3(kChunkThreads), 0, st, hist,
                       p.nchunks, ncell, m, cstart);
    hipLaunchKernelGGL(cell_scatter_kernel, dim3((unsigned)p.nchunks, (unsigned)f),
                       dim3(kChunkThreads), 0, st, ion_pos, ion_q, m, p.nchunks, ncell,
                       (const uint32_t *)keys, (const int32_t *)hist, (const int32_t *)cstart,
                       sorted);
    hipLaunchKernelGGL(real_space_cell_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)f),
                       dim3(64), 0, st, s->pos, s->rs_width, s->atom_order, n,
                       (const double4 *)sorted, (const int32_t *)cstart, m, p.nc[0], p.nc[1],
                       p.nc[2], s->box[0], s->box[1], s->box[2], s->beta, s->rcut, f,
                       (const double *)s->erfc_tab, rs);
  } else if (p.rs_groups > 0) {
    hipLaunchKernelGGL(real_space_ions_kernel, dim3((unsigned)iblocks, (unsigned)f, (unsigned)p.rs_groups),
                       dim3(RB), 0, st, s->pos, s->rs_width, s->atom_order, n, ion_pos, ion_q, m,
                       p.rs_ipg, s->box[0], s->box[1], s->box[2], s->beta, s->rcut, f,
                       (const double *)s->erfc_tab, rs);
  }
  hipLaunchKernelGGL(assemble_b_kernel, dim3((unsigned)((n * f + 255) / 256)), dim3(256), 0, st,
                     bp, (int)p.ksplit, rs, (int)p.rs_groups, n, f, chi, qsol_out, c0,
                     (const double *)m1, 4.0 * M_PI / s->vol, s->pos, b_out);
  return hipGetLastError();
}

// Coefficients of erfc_pw. About x_j = (j + 1/2) / 8: c_j0 = erfc(x_j) and,
// from d^(k+1)/dx^(k+1) erfc(x) = -(2/sqrt(pi)) (-1)^k H_k(x) exp(-x^2) with
// the Hermite recurrence H_(k+1) = 2 x H_k - 2 k H_(k-1), c_j(k+1) = that
// derivative / ((k+1)! 8^(k+1)); long double arithmetic. The truncation
// after degree 11 on |x - x_j| <= 1/16 is below 1e-17.
void erfc_table(double *out) {
  const long double c2 = 2.0L / std::sqrt(3.14159265358979323846264338327950288L);
  for (int j = 0; j < kErfcIntervals; ++j) {
    const long double x = ((long double)j + 0.5L) / 8.0L;
    const long double e = std::exp(-x * x);
    double *c = out + j * kErfcTerms;
    c[0] = std::erfc((double)x);   // x_j is exact in double
    long double hprev = 0.0L, hcur = 1.0L, fact = 1.0L, scale = 1.0L;
    for (int k = 0; k + 1 < kErfcTerms; ++k) {
      const long double sign = (k % 2 == 0) ? -1.0L : 1.0L;
      fact *= (long double)(k + 1);
      scale /= 8.0L;
      c[k + 1] = (double)(sign * c2 * hcur * e * scale / fact);
      const long double hnext = 2.0L * x * hcur - 2.0L * (long double)k * hprev;
      hprev = hcur;
      hcur = hnext;
    }
  }
}

}  // namespace cpm
