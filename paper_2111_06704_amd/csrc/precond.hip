// PCG-DC preconditioner (Sec. III.B.2, Eq. 36): construction.
//
// For every atom tau the local matrix M_tau over tau and its neighbourhood
// (every atom image within rcut) is formed from Eq. 36, factorised
// (Cholesky, FP64), and the column of M_tau^-1 belonging to tau becomes
// column tau of P; entries of different images of one atom add up. CG needs
// a symmetric preconditioner, so it uses (P + P^T) / 2, kept on the host in
// row-major ELL form (entry k of row i at i * width + k, rows padded with
// (i, 0)) and on the device in the form the apply reads: block-dense (tiles
// of 64 atoms over the union of their columns) for large systems, the ELL
// rows for small ones. The construction runs once per system:
// the neighbourhoods on host threads, the local matrices and their batched
// Cholesky factorisations and solves on the device; the apply z = P r of
// every PCG iteration runs on the device (cg.hip). Also here: the
// sparsified inverse of PCG-Normal / Full and the Eq. 37 fill.
#include "cpm_internal.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <string>
#include <thread>

namespace cpm {
namespace {

struct Image {
  int32_t atom;
  int32_t shift;   // packed periodic shift, 0-based per axis
  double x, y, z;
};

// worker threads for the construction: at most 16 (the host share of one
// GPU), fewer if OMP_NUM_THREADS or the hardware says so
int build_threads() {
  int t = (int)std::thread::hardware_concurrency();
  if (t < 1) t = 1;
  if (const char *e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v >= 1) t = std::min(t, v);
  }
  return std::min(t, 16);
}

template <typename F> void parallel_for(int64_t count, F &&body) {
  const int nt = (int)std::min<int64_t>(build_threads(), std::max<int64_t>(1, count));
  std::atomic<int64_t> next{0};
  auto worker = [&](int tid) {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= count) break;
      body(i, tid);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (std::thread &th : pool) th.join();
}

// Neighbourhood of every atom: all images within rc (distance <= rc), the
// atom itself at zero shift excluded, ordered by atom index then shift.
std::vector<std::vector<Image>> neighbourhoods(const std::vector<double> &pos, int64_t n,
                                               const double box[3], double rc) {
  int nr[3];
  for (int d = 0; d < 3; ++d) nr[d] = (int)std::ceil(rc / box[d]) + 1;
  const int w1 = 2 * nr[1] + 1, w2 = 2 * nr[2] + 1;
  const int zero_shift = (nr[0] * w1 + nr[1]) * w2 + nr[2];
  std::vector<Image> imgs;
  for (int a = -nr[0]; a <= nr[0]; ++a)
    for (int b = -nr[1]; b <= nr[1]; ++b)
      for (int c = -nr[2]; c <= nr[2]; ++c)
        for (int64_t i = 0; i < n; ++i) {
          const double x = pos[3 * i] + a * box[0], y = pos[3 * i + 1] + b * box[1],
                       z = pos[3 * i + 2] + c * box[2];
          if (x < -rc || x > box[0] + rc || y < -rc || y > box[1] + rc || z < -rc ||
              z > box[2] + rc)
            continue;
          imgs.push_back({(int32_t)i, (a + nr[0]) * w1 * w2 + (b + nr[1]) * w2 + (c + nr[2]), x, y, z});
        }
  // cells of edge >= rc over (-rc, L + rc)
  int nc[3];
  double cs[3];
  for (int d = 0; d < 3; ++d) {
    const double span = box[d] + 2 * rc;
    nc[d] = std::max(1, std::min(512, (int)(span / rc)));
    cs[d] = span / nc[d];
  }
  auto cell_index = [&](double v, int d) {
    int ci = (int)((v + rc) / cs[d]);
    return std::min(std::max(ci, 0), nc[d] - 1);
  };
  std::vector<int64_t> start((size_t)nc[0] * nc[1] * nc[2] + 1, 0);
  std::vector<int64_t> cell_of(imgs.size());
  for (size_t k = 0; k < imgs.size(); ++k) {
    cell_of[k] = ((int64_t)cell_index(imgs[k].x, 0) * nc[1] + cell_index(imgs[k].y, 1)) * nc[2] +
                 cell_index(imgs[k].z, 2);
    ++start[cell_of[k] + 1];
  }
  for (size_t c = 1; c < start.size(); ++c) start[c] += start[c - 1];
  std::vector<int64_t> fill(start.begin(), start.end() - 1), sorted(imgs.size());
  for (size_t k = 0; k < imgs.size(); ++k) sorted[fill[cell_of[k]]++] = (int64_t)k;

  std::vector<std::vector<Image>> out(n);
  const double rc2 = rc * rc;
  parallel_for(n, [&](int64_t i, int) {
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const int ci[3] = {cell_index(x, 0), cell_index(y, 1), cell_index(z, 2)};
    std::vector<Image> &nb = out[i];
    for (int a = std::max(0, ci[0] - 1); a <= std::min(nc[0] - 1, ci[0] + 1); ++a)
      for (int b = std::max(0, ci[1] - 1); b <= std::min(nc[1] - 1, ci[1] + 1); ++b)
        for (int c = std::max(0, ci[2] - 1); c <= std::min(nc[2] - 1, ci[2] + 1); ++c) {
          const int64_t cell = ((int64_t)a * nc[1] + b) * nc[2] + c;
          for (int64_t s = start[cell]; s < start[cell + 1]; ++s) {
            const Image &im = imgs[sorted[s]];
            if (im.atom == i && im.shift == zero_shift) continue;
            const double dx = im.x - x, dy = im.y - y, dz = im.z - z;
            if (dx * dx + dy * dy + dz * dz <= rc2) nb.push_back(im);
          }
        }
    std::sort(nb.begin(), nb.end(), [](const Image &p, const Image &q) {
      return p.atom != q.atom ? p.atom < q.atom : p.shift < q.shift;
    });
  });
  return out;
}

}  // namespace

void free_precond(Precond &p) {
  void *ptrs[] = {p.idx, p.val, p.uoff, p.uidx, p.blk};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  p = Precond();
}

void free_coarse(Coarse &c) {
  void *ptrs[] = {c.pid, c.perm, c.off, c.az, c.eci, c.ut, c.wt, c.c1, c.g1, c.dg, c.g1f, c.c2p};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  c = Coarse();
}

namespace {

// the tiles' column unions (host): U_t sorted, padded to a multiple of 4
void block_pattern(Precond &p, int64_t n) {
  p.ntiles = (n + kPcTile - 1) / kPcTile;
  std::vector<std::vector<int32_t>> u(p.ntiles);
  parallel_for(p.ntiles, [&](int64_t t, int) {
    std::vector<int32_t> &v = u[t];
    for (int64_t r = t * kPcTile; r < std::min<int64_t>(n, (t + 1) * kPcTile); ++r)
      for (int k = 0; k < p.h_len[r]; ++k) v.push_back(p.h_idx[(size_t)r * p.width + k]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if (v.empty()) v.push_back(0);
    while (v.size() % 4 != 0) v.push_back(v[0]);
  });
  p.h_uoff.assign(p.ntiles + 1, 0);
  for (int64_t t = 0; t < p.ntiles; ++t) p.h_uoff[t + 1] = p.h_uoff[t] + (int64_t)u[t].size();
  p.h_uidx.assign(p.h_uoff[p.ntiles], 0);
  for (int64_t t = 0; t < p.ntiles; ++t)
    std::copy(u[t].begin(), u[t].end(), p.h_uidx.begin() + p.h_uoff[t]);
}

// the dense tile entries (host): P minus gap on its pattern
std::vector<double> block_values(const Precond &p, int64_t n, double gap) {
  std::vector<double> b((size_t)p.h_uoff[p.ntiles] * kPcTile, 0.0);
  parallel_for(p.ntiles, [&](int64_t t, int) {
    const int32_t *u0 = p.h_uidx.data() + p.h_uoff[t];
    int64_t K = p.h_uoff[t + 1] - p.h_uoff[t];
    // the sorted part: the padding repeats U_t[0] after it
    for (int64_t i = 1; i < K; ++i)
      if (u0[i] == u0[0]) {
        K = i;
        break;
      }
    double *bt = b.data() + (size_t)p.h_uoff[t] * kPcTile;
    for (int64_t r = t * kPcTile; r < std::min<int64_t>(n, (t + 1) * kPcTile); ++r)
      for (int k = 0; k < p.h_len[r]; ++k) {
        const int32_t j = p.h_idx[(size_t)r * p.width + k];
        const int64_t kk = std::lower_bound(u0, u0 + K, j) - u0;
        bt[(size_t)kk * kPcTile + (r - t * kPcTile)] += p.h_val[(size_t)r * p.width + k] - gap;
      }
  });
  return b;
}

// p's device form (block-dense from kPcBlockTiles tiles on, else ELL) to
// new device arrays; on success p replaces the system's preconditioner (the
// previous one is freed)
cpm_status install_precond(cpm_system *s, Precond &p) {
  block_pattern(p, s->n);
  // CPM_PRECOND_BLOCK=1 / 0 in the environment forces the form (tests run
  // both at small sizes)
  bool blocks = p.ntiles >= kPcBlockTiles;
  if (const char *e = std::getenv("CPM_PRECOND_BLOCK"))
    if (e[0] == '0' || e[0] == '1') blocks = e[0] == '1';
  std::vector<double> b;
  bool ok = true;
  if (blocks) {
    b = block_values(p, s->n, 0.0);
    ok = hipMalloc((void **)&p.uoff, sizeof(int64_t) * p.h_uoff.size()) == hipSuccess &&
         hipMalloc((void **)&p.uidx, sizeof(int32_t) * p.h_uidx.size()) == hipSuccess &&
         hipMalloc((void **)&p.blk, sizeof(double) * b.size()) == hipSuccess;
  } else {
    ok = hipMalloc((void **)&p.idx, sizeof(int32_t) * p.h_idx.size()) == hipSuccess &&
         hipMalloc((void **)&p.val, sizeof(double) * p.h_val.size()) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_precond(p);
    set_error("preconditioner allocation failed");
    return CPM_ENOMEM;
  }
  if (blocks) {
    CPM_HIP_CHECK(hipMemcpyAsync(p.uoff, p.h_uoff.data(), sizeof(int64_t) * p.h_uoff.size(),
                                 hipMemcpyHostToDevice, s->stream));
    CPM_HIP_CHECK(hipMemcpyAsync(p.uidx, p.h_uidx.data(), sizeof(int32_t) * p.h_uidx.size(),
                                 hipMemcpyHostToDevice, s->stream));
    CPM_HIP_CHECK(hipMemcpyAsync(p.blk, b.data(), sizeof(double) * b.size(),
                                 hipMemcpyHostToDevice, s->stream));
    p.bytes = (int64_t)(sizeof(int64_t) * p.h_uoff.size() + sizeof(int32_t) * p.h_uidx.size() +
                        sizeof(double) * b.size());
  } else {
    CPM_HIP_CHECK(hipMemcpyAsync(p.idx, p.h_idx.data(), sizeof(int32_t) * p.h_idx.size(),
                                 hipMemcpyHostToDevice, s->stream));
    CPM_HIP_CHECK(hipMemcpyAsync(p.val, p.h_val.data(), sizeof(double) * p.h_val.size(),
                                 hipMemcpyHostToDevice, s->stream));
    p.bytes = (int64_t)(sizeof(int32_t) * p.h_idx.size() + sizeof(double) * p.h_val.size());
  }
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  p.sum_p = 0.0;
  for (size_t e = 0; e < p.h_val.size(); ++e) p.sum_p += p.h_val[e];   // padding entries are 0
  s->device_bytes -= s->pc.bytes;
  free_precond(s->pc);
  p.ready = true;
  s->pc = std::move(p);
  s->device_bytes += s->pc.bytes;
  return CPM_OK;
}

std::vector<int32_t> host_atom_order(cpm_system *s) {
  std::vector<int32_t> order(s->n);
  if (hipMemcpyAsync(order.data(), s->atom_order, sizeof(int32_t) * s->n, hipMemcpyDeviceToHost,
                     s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    order.clear();
  return order;
}

// entries of E^-1 = S + d' d'^T / C_ele (S of the matrix-inversion path,
// symmetrised) at the real entries (k < len[t]) of ELL row t (atom order[t]),
// 0 at the padding
__global__ void sparse_inverse_values_kernel(const double *__restrict__ S, int64_t ld,
                                             const double *__restrict__ dprime, double inv_c,
                                             const int32_t *__restrict__ order,
                                             const int32_t *__restrict__ idx,
                                             const int32_t *__restrict__ len, int width, int64_t n,
                                             double *__restrict__ val) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * width) return;
  const int64_t t = e / width;
  const int k = (int)(e - t * width);
  double v = 0.0;
  if (k < len[t]) {
    const int64_t i = order[t], j = idx[e];
    v = 0.5 * (S[i * ld + j] + S[j * ld + i]) + dprime[i] * dprime[j] * inv_c;
  }
  val[e] = v;
}


// Local matrices of Eq. 36 for a batch of atoms, column-major, each padded
// to mm x mm with the identity (which leaves the solution for e_0
// unchanged): img holds, per atom b, its m_b points (tau first, then its
// neighbourhood images) as (x, y, z, a); X gets e_0.
__global__ void dc_local_kernel(const double4 *__restrict__ img, const int32_t *__restrict__ mlen,
                                int mm, double g, double rcut, double erfc_rc,
                                double *__restrict__ A, double *__restrict__ X) {
  const int64_t b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mm * mm) return;
  const int row = (int)(e % mm), col = (int)(e / mm);
  const int m = mlen[b];
  const double4 *p = img + b * mm;
  double v;
  if (row >= m || col >= m) {
    v = (row == col) ? 1.0 : 0.0;
  } else if (row == col) {
    v = sqrt(2.0 / M_PI) * p[row].w;
  } else {
    const double dx = p[row].x - p[col].x, dy = p[row].y - p[col].y, dz = p[row].z - p[col].z;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    v = (r > 0.0 && r < rcut) ? (erfc(g * r) - erfc_rc) / r : 0.0;
  }
  A[b * (int64_t)mm * mm + e] = v;
  if (col == 0) X[b * (int64_t)mm + row] = (row == 0) ? 1.0 : 0.0;
}

// Column tau of P (step 2 of the construction) for every atom: the local
// matrices are formed on the device in batches of atoms with neighbourhoods
// of similar size, factorised and solved for e_0 by the batched Cholesky of
// rocSOLVER (strided, FP64); images of one atom add up on the host.
cpm_status dc_columns_device(cpm_system *s, const std::vector<std::vector<Image>> &nb, double g,
                             double rcut, std::vector<std::vector<std::pair<int32_t, double>>> &col) {
  const int64_t n = s->n;
  hipStream_t st = s->stream;
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return nb[a].size() > nb[b].size(); });
  const int mfirst = (int)nb[order[0]].size() + 1;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  // one batch: at most cap atoms (every per-atom array below holds cap
  // atoms of mfirst points, mfirst being the largest neighbourhood), and
  // local matrices of at most 4 GiB or a quarter of the free memory (at
  // least one matrix); a batch of atoms with mm <= mfirst points takes
  // min(cap, a_elems / mm^2) atoms, so every array bound holds
  const int64_t cap = std::min<int64_t>(n, 16384);
  const size_t budget = std::min<size_t>((size_t)4 << 30, free_b / 4);
  const int64_t a_elems = std::max<int64_t>(
      (int64_t)mfirst * mfirst,
      std::min<int64_t>(cap * mfirst * mfirst, (int64_t)(budget / sizeof(double))));
  double *A = nullptr, *X = nullptr;
  double4 *img = nullptr;
  int32_t *mlen = nullptr, *info = nullptr;
  rocblas_handle h = nullptr;
  auto release = [&]() {
    if (h) (void)rocblas_destroy_handle(h);
    void *ptrs[] = {A, X, img, mlen, info};
    for (void *q : ptrs)
      if (q) (void)hipFree(q);
  };
  if (hipMalloc((void **)&A, sizeof(double) * (size_t)a_elems) != hipSuccess ||
      hipMalloc((void **)&X, sizeof(double) * (size_t)cap * mfirst) != hipSuccess ||
      hipMalloc((void **)&img, sizeof(double4) * (size_t)cap * mfirst) != hipSuccess ||
      hipMalloc((void **)&mlen, sizeof(int32_t) * cap) != hipSuccess ||
      hipMalloc((void **)&info, sizeof(int32_t) * cap) != hipSuccess) {
    (void)hipGetLastError();
    release();
    set_error("PCG-DC: allocation of the local matrices failed");
    return CPM_ENOMEM;
  }
  if (rocblas_create_handle(&h) != rocblas_status_success ||
      rocblas_set_stream(h, st) != rocblas_status_success) {
    release();
    set_error("PCG-DC: rocBLAS handle");
    return CPM_EDEVICE;
  }
  const double erfc_rc = std::erfc(g * rcut);
  std::vector<double4> himg((size_t)cap * mfirst);
  std::vector<int32_t> hlen(cap), hinfo(cap);
  std::vector<double> hx((size_t)cap * mfirst);
  for (int64_t b0 = 0; b0 < n;) {
    const int mm = (int)nb[order[b0]].size() + 1;   // the batch's largest (<= mfirst)
    const int64_t nb_b =
        std::min<int64_t>({n - b0, cap, std::max<int64_t>(1, a_elems / ((int64_t)mm * mm))});
    for (int64_t b = 0; b < nb_b; ++b) {
      const int64_t tau = order[b0 + b];
      const std::vector<Image> &v = nb[tau];
      hlen[b] = (int32_t)v.size() + 1;
      double4 *row = himg.data() + (size_t)b * mm;
      row[0] = make_double4(s->pos_host[3 * tau], s->pos_host[3 * tau + 1], s->pos_host[3 * tau + 2],
                            s->width_host[tau]);
      for (size_t k = 0; k < v.size(); ++k)
        row[k + 1] = make_double4(v[k].x, v[k].y, v[k].z, s->width_host[v[k].atom]);
    }
    hipError_t e = hipMemcpyAsync(img, himg.data(), sizeof(double4) * (size_t)nb_b * mm,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(mlen, hlen.data(), sizeof(int32_t) * nb_b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      const int64_t ent = (int64_t)mm * mm;
      hipLaunchKernelGGL(dc_local_kernel, dim3((unsigned)((ent + 255) / 256), (unsigned)nb_b),
                         dim3(256), 0, st, (const double4 *)img, (const int32_t *)mlen, mm, g, rcut,
                         erfc_rc, A, X);
      e = hipGetLastError();
    }
    const rocblas_stride sa = (rocblas_stride)mm * mm, sx = mm;
    if (e != hipSuccess ||
        rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, mm, A, mm, sa, info,
                                         (rocblas_int)nb_b) != rocblas_status_success ||
        rocsolver_dpotrs_strided_batched(h, rocblas_fill_lower, mm, 1, A, mm, sa, X, mm, sx,
                                         (rocblas_int)nb_b) != rocblas_status_success) {
      release();
      set_error("PCG-DC: batched factorisation failed");
      return CPM_EDEVICE;
    }
    e = hipMemcpyAsync(hx.data(), X, sizeof(double) * (size_t)nb_b * mm, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hinfo.data(), info, sizeof(int32_t) * nb_b, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      release();
      set_error(std::string("PCG-DC: ") + hipGetErrorString(e));
      return CPM_EDEVICE;
    }
    for (int64_t b = 0; b < nb_b; ++b)
      if (hinfo[b] != 0) {
        release();
        set_error("PCG-DC: the local matrix of atom " + std::to_string(order[b0 + b]) +
                  " (Eq. 36) is not positive definite");
        return CPM_ENOTSPD;
      }
    parallel_for(nb_b, [&](int64_t b, int) {
      const int64_t tau = order[b0 + b];
      const std::vector<Image> &v = nb[tau];
      const double *x = hx.data() + (size_t)b * mm;
      std::vector<std::pair<int32_t, double>> &c = col[tau];
      c.push_back({(int32_t)tau, x[0]});
      for (size_t k = 1; k <= v.size(); ++k) {
        const int32_t j = v[k - 1].atom;
        auto it = std::lower_bound(
            c.begin(), c.end(), j,
            [](const std::pair<int32_t, double> &q, int32_t a) { return q.first < a; });
        if (it != c.end() && it->first == j)
          it->second += x[k];
        else
          c.insert(it, {j, x[k]});
      }
    });
    b0 += nb_b;
  }
  release();
  return CPM_OK;
}


// ---- coarse space of the two-level preconditioner

// Patches (host): z-slabs from the sorted z of the atoms (a new slab where
// two consecutive values differ by more than kSlabGap, so a jittered layer
// stays one slab), each split into nx x ny in-plane bins of the box, nx =
// max(1, floor(L_x / edge + 1/2)); empty patches dropped, the rest numbered
// in (slab, x bin, y bin) order. pos: wrapped positions.
std::vector<int32_t> coarse_patch_ids(const std::vector<double> &pos, int64_t n,
                                      const double box[3], double edge, int64_t &m, int &nslab) {
  std::vector<int64_t> by_z(n);
  for (int64_t i = 0; i < n; ++i) by_z[i] = i;
  std::stable_sort(by_z.begin(), by_z.end(),
                   [&](int64_t a, int64_t b) { return pos[3 * a + 2] < pos[3 * b + 2]; });
  std::vector<int64_t> slab(n, 0);
  int64_t sl = 0;
  for (int64_t k = 1; k < n; ++k) {
    if (pos[3 * by_z[k] + 2] - pos[3 * by_z[k - 1] + 2] > kSlabGap) ++sl;
    slab[by_z[k]] = sl;
  }
  nslab = (int)(sl + 1);
  const int64_t nx = std::max<int64_t>(1, (int64_t)std::floor(box[0] / edge + 0.5));
  const int64_t ny = std::max<int64_t>(1, (int64_t)std::floor(box[1] / edge + 0.5));
  std::vector<int64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t bx = std::min<int64_t>(nx - 1, (int64_t)std::floor(pos[3 * i] / box[0] * nx));
    const int64_t by = std::min<int64_t>(ny - 1, (int64_t)std::floor(pos[3 * i + 1] / box[1] * ny));
    key[i] = (slab[i] * nx + bx) * ny + by;
  }
  std::vector<int64_t> keys(key);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  m = (int64_t)keys.size();
  std::vector<int32_t> pid(n);
  for (int64_t i = 0; i < n; ++i)
    pid[i] = (int32_t)(std::lower_bound(keys.begin(), keys.end(), key[i]) - keys.begin());
  return pid;
}

// rows t0 .. t0 + gridDim.y - 1 of (E Z)^T in FP64: out[(t - t0) * ld + i] =
// sum over the atoms j of patch t of E_ij (column j of the symmetric E, read
// coalesced in i); zero for i >= n
__global__ __launch_bounds__(256) void coarse_az_kernel(const double *__restrict__ E, int64_t ld,
                                                        int64_t n, const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ off,
                                                        int64_t t0, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ld) return;
  const int64_t t = t0 + blockIdx.y;
  double v = 0.0;
  if (i < n)
    for (int32_t k = off[t]; k < off[t + 1]; ++k) v += E[(int64_t)perm[k] * ld + i];
  out[(int64_t)blockIdx.y * ld + i] = v;
}

// rows t0 .. of E_c = Z^T E Z: ec[t * mp + u] = sum over the atoms of patch u
// of row t of (E Z)^T (FP64)
__global__ __launch_bounds__(256) void coarse_ec_kernel(const double *__restrict__ az64, int64_t ld,
                                                        const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ off, int64_t m,
                                                        int64_t mp, int64_t t0,
                                                        double *__restrict__ ec) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= m) return;
  const double *row = az64 + (int64_t)blockIdx.y * ld;
  double v = 0.0;
  for (int32_t k = off[u]; k < off[u + 1]; ++k) v += row[perm[k]];
  ec[(t0 + blockIdx.y) * mp + u] = v;
}

__global__ __launch_bounds__(256) void f64_to_f32_rows_kernel(const double *__restrict__ in,
                                                              float *__restrict__ out,
                                                              int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) out[e] = (float)in[e];
}

// E_c (mp x mp, symmetric up to rounding): the mean of (t, u) and (u, t) in
// both, 1 on the diagonal of the padding and 0 elsewhere in it (an SPD
// matrix for the factorisation)
__global__ __launch_bounds__(256) void coarse_ec_sym_kernel(double *__restrict__ ec, int64_t m,
                                                            int64_t mp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= mp * mp) return;
  const int64_t t = e / mp, u = e - t * mp;
  if (t < m && u < m) {
    if (u > t) {
      const double a = 0.5 * (ec[t * mp + u] + ec[u * mp + t]);
      ec[t * mp + u] = a;
      ec[u * mp + t] = a;
    }
  } else {
    ec[e] = (t == u) ? 1.0 : 0.0;
  }
}

// after the inversion (lower triangle of the column-major matrix, i.e.
// ec[t * mp + u] with u >= t): mirror into the other triangle and zero the
// padding, so that E_c^-1 is applied to padded vectors as 0
__global__ __launch_bounds__(256) void coarse_eci_fill_kernel(double *__restrict__ a, int64_t m,
                                                              int64_t mp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= mp * mp) return;
  const int64_t t = e / mp, u = e - t * mp;
  if (t >= m || u >= m)
    a[e] = 0.0;
  else if (u < t)
    a[e] = a[u * mp + t];
}

// temporaries of the coarse-space construction, released on every path
struct CoarseTmp {
  double *az64 = nullptr;
  int32_t *info = nullptr;
  rocblas_handle h = nullptr;
  ~CoarseTmp() {
    if (h) (void)rocblas_destroy_handle(h);
    if (az64) (void)hipFree(az64);
    if (info) (void)hipFree(info);
  }
};

// the coarse space for patches pid (host, n): device arrays, E Z (FP32) and
// E_c^-1; on failure the caller frees c
cpm_status build_coarse(cpm_system *s, const std::vector<int32_t> &pid, int64_t m, Coarse &c) {
  hipStream_t st = s->stream;
  const int64_t n = s->n, ld = s->ld;
  const int64_t mp = (m + kCoarseAlign - 1) / kCoarseAlign * kCoarseAlign;
  c.m = m;
  c.mp = mp;
  // atoms by patch (counting sort: increasing index within a patch)
  std::vector<int32_t> off(mp + 1, 0), perm(n);
  for (int64_t i = 0; i < n; ++i) ++off[pid[i] + 1];
  for (int64_t t = 0; t < mp; ++t) off[t + 1] += off[t];
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) perm[fill[pid[i]]++] = (int32_t)i;
  }
  coarse_slices(ld, mp, c.ks, c.kslice);
  const size_t vec = sizeof(double) * (size_t)ld * kCoarseCols;
  const size_t cv = (size_t)kCoarseCols * mp;
  const int64_t CH = std::min<int64_t>(256, m);   // rows of E Z per pass
  const size_t sizes[] = {sizeof(int32_t) * (size_t)n, sizeof(int32_t) * (size_t)n,
                          sizeof(int32_t) * (size_t)(mp + 1), sizeof(float) * (size_t)mp * ld,
                          sizeof(double) * (size_t)mp * mp, vec, vec, sizeof(double) * cv,
                          sizeof(double) * cv, sizeof(double) * cv, sizeof(float) * cv,
                          sizeof(float) * cv * (size_t)c.ks};
  void **dst[] = {(void **)&c.pid, (void **)&c.perm, (void **)&c.off, (void **)&c.az,
                  (void **)&c.eci, (void **)&c.ut, (void **)&c.wt, (void **)&c.c1,
                  (void **)&c.g1, (void **)&c.dg, (void **)&c.g1f, (void **)&c.c2p};
  CoarseTmp tmp;
  bool ok = true;
  for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
    ok = ok && hipMalloc(dst[k], sizes[k]) == hipSuccess;
    if (ok) c.bytes += (int64_t)sizes[k];
  }
  ok = ok && hipMalloc((void **)&tmp.az64, sizeof(double) * (size_t)CH * ld) == hipSuccess &&
       hipMalloc((void **)&tmp.info, sizeof(int32_t)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    set_error("coarse space: allocation failed");
    return CPM_ENOMEM;
  }
  CPM_HIP_CHECK(hipMemcpyAsync(c.pid, pid.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  CPM_HIP_CHECK(hipMemcpyAsync(c.perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  CPM_HIP_CHECK(hipMemcpyAsync(c.off, off.data(), sizeof(int32_t) * (mp + 1), hipMemcpyHostToDevice,
                               st));
  CPM_HIP_CHECK(hipMemsetAsync(c.az, 0, sizeof(float) * (size_t)mp * ld, st));
  CPM_HIP_CHECK(hipMemsetAsync(c.ut, 0, vec, st));
  CPM_HIP_CHECK(hipMemsetAsync(c.wt, 0, vec, st));
  CPM_HIP_CHECK(hipMemsetAsync(c.eci, 0, sizeof(double) * (size_t)mp * mp, st));
  // E_c is formed and inverted in place in c.eci
  for (int64_t t0 = 0; t0 < m; t0 += CH) {
    const int64_t rows = std::min<int64_t>(CH, m - t0);
    hipLaunchKernelGGL(coarse_az_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)rows),
                       dim3(256), 0, st, (const double *)s->E64, ld, n, (const int32_t *)c.perm,
                       (const int32_t *)c.off, t0, tmp.az64);
    hipLaunchKernelGGL(coarse_ec_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)rows),
                       dim3(256), 0, st, (const double *)tmp.az64, ld, (const int32_t *)c.perm,
                       (const int32_t *)c.off, m, mp, t0, c.eci);
    hipLaunchKernelGGL(f64_to_f32_rows_kernel, dim3((unsigned)((rows * ld + 255) / 256)),
                       dim3(256), 0, st, (const double *)tmp.az64, c.az + t0 * ld, rows * ld);
  }
  const unsigned gm = (unsigned)((mp * mp + 255) / 256);
  hipLaunchKernelGGL(coarse_ec_sym_kernel, dim3(gm), dim3(256), 0, st, c.eci, m, mp);
  CPM_HIP_CHECK(hipGetLastError());
  if (rocblas_create_handle(&tmp.h) != rocblas_status_success ||
      rocblas_set_stream(tmp.h, st) != rocblas_status_success) {
    set_error("coarse space: rocBLAS handle");
    return CPM_EDEVICE;
  }
  int32_t hinfo[2] = {0, 0};
  if (rocsolver_dpotrf(tmp.h, rocblas_fill_lower, (rocblas_int)mp, c.eci, (rocblas_int)mp,
                       tmp.info) != rocblas_status_success ||
      hipMemcpyAsync(hinfo, tmp.info, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("coarse space: factorisation of Z^T E Z failed");
    return CPM_EDEVICE;
  }
  if (hinfo[0] != 0) {
    set_error("coarse space: Z^T E Z is not positive definite");
    return CPM_ENOTSPD;
  }
  if (rocsolver_dpotri(tmp.h, rocblas_fill_lower, (rocblas_int)mp, c.eci, (rocblas_int)mp,
                       tmp.info) != rocblas_status_success ||
      hipMemcpyAsync(hinfo + 1, tmp.info, sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hinfo[1] != 0) {
    set_error("coarse space: inversion of Z^T E Z failed");
    return CPM_EDEVICE;
  }
  hipLaunchKernelGGL(coarse_eci_fill_kernel, dim3(gm), dim3(256), 0, st, c.eci, m, mp);
  CPM_HIP_CHECK(hipGetLastError());
  CPM_HIP_CHECK(hipStreamSynchronize(st));
  return CPM_OK;
}

}  // namespace

}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_precond_dc(cpm_system *s, double g, double rcut) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  if (!(g > 0.0) || !(rcut > 0.0) || !std::isfinite(g) || !std::isfinite(rcut)) {
    set_error("screening g and rcut must be finite and > 0");
    return CPM_EINVAL;
  }
  const int64_t n = s->n;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(s->width_host[i])) {
      set_error("the DC preconditioner needs Gaussian widths (atom " + std::to_string(i) +
                " is a point charge)");
      return CPM_EINVAL;
    }
  const std::vector<std::vector<Image>> nb = neighbourhoods(s->pos_host, n, s->box, rcut);
  int mmax = 1;
  for (const auto &v : nb) mmax = std::max(mmax, (int)v.size() + 1);

  // column tau of P: (atom, value) pairs, images of one atom summed
  std::vector<std::vector<std::pair<int32_t, double>>> col(n);
  cpm_status rcol = dc_columns_device(s, nb, g, rcut, col);
  if (rcol != CPM_OK) return rcol;
  // symmetric part, row by row: P_s[i][j] = (C_i[j] + C_j[i]) / 2
  auto entry = [&](int64_t c, int32_t r) {
    const auto &v = col[c];
    auto it = std::lower_bound(v.begin(), v.end(), r,
                               [](const std::pair<int32_t, double> &e, int32_t a) { return e.first < a; });
    return (it != v.end() && it->first == r) ? it->second : 0.0;
  };
  int width = 1;
  for (const auto &v : col) width = std::max(width, (int)v.size());
  // ELL row t holds the row of atom order[t], the order in which the apply
  // kernel takes the rows
  const std::vector<int32_t> order = host_atom_order(s);
  if ((int64_t)order.size() != n) {
    set_error("reading the atom order failed");
    return CPM_EDEVICE;
  }
  Precond p;
  p.h_idx.assign((size_t)width * n, 0);
  p.h_val.assign((size_t)width * n, 0.0);
  p.h_len.assign(n, 0);
  int64_t nnz = 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = order[t];
    const auto &v = col[i];   // the neighbour relation is symmetric: row i has the atoms of column i
    for (int k = 0; k < width; ++k) {
      if (k < (int)v.size()) {
        p.h_idx[(size_t)t * width + k] = v[k].first;
        p.h_val[(size_t)t * width + k] = 0.5 * (v[k].second + entry(v[k].first, (int32_t)i));
      } else {
        p.h_idx[(size_t)t * width + k] = (int32_t)i;
      }
    }
    p.h_len[t] = (int32_t)v.size();
    nnz += (int64_t)v.size();
  }
  p.kind = 0;
  p.g = g;
  p.rcut = rcut;
  p.width = width;
  p.nnz = nnz;
  p.max_local = mmax;
  return install_precond(s, p);
}

cpm_status cpm_precond_sparse_inverse(cpm_system *s, double rcut) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  if (!(rcut > 0.0) || !std::isfinite(rcut)) {
    set_error("rcut must be finite and > 0");
    return CPM_EINVAL;
  }
  if (!s->S || !s->dprime_ready || !(s->c_ele > 0.0)) {
    set_error("cpm_mi_build first (the sparsified preconditioner takes E^-1 from it)");
    return CPM_ESTATE;
  }
  const int64_t n = s->n;
  // pairs with an image strictly closer than rcut (a neighbourhood lists
  // every image within rcut), the atom itself first
  const std::vector<std::vector<Image>> nb = neighbourhoods(s->pos_host, n, s->box, rcut);
  std::vector<std::vector<int32_t>> row(n);
  parallel_for(n, [&](int64_t i, int) {
    std::vector<int32_t> &r = row[i];
    r.push_back((int32_t)i);
    const double x = s->pos_host[3 * i], y = s->pos_host[3 * i + 1], z = s->pos_host[3 * i + 2];
    for (const Image &im : nb[i]) {
      const double dx = im.x - x, dy = im.y - y, dz = im.z - z;
      if (im.atom != i && dx * dx + dy * dy + dz * dz < rcut * rcut &&
          (r.size() == 1 || r.back() != im.atom))
        r.push_back(im.atom);   // images come ordered by atom: one entry per atom
    }
  });
  int width = 1;
  for (const auto &r : row) width = std::max(width, (int)r.size());
  const std::vector<int32_t> order = host_atom_order(s);
  if ((int64_t)order.size() != n) {
    set_error("reading the atom order failed");
    return CPM_EDEVICE;
  }
  Precond p;
  p.h_idx.assign((size_t)width * n, 0);
  p.h_val.assign((size_t)width * n, 0.0);
  p.h_len.assign(n, 0);
  int64_t nnz = 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = order[t];
    const std::vector<int32_t> &r = row[i];
    for (int k = 0; k < width; ++k)
      p.h_idx[(size_t)t * width + k] = k < (int)r.size() ? r[k] : (int32_t)i;
    p.h_len[t] = (int32_t)r.size();
    nnz += (int64_t)r.size();
  }
  // values on the device from S, then back for the host copy
  int32_t *d_idx = nullptr, *d_len = nullptr, *d_order = nullptr;
  double *d_val = nullptr;
  auto release = [&]() {
    if (d_idx) (void)hipFree(d_idx);
    if (d_len) (void)hipFree(d_len);
    if (d_val) (void)hipFree(d_val);
  };
  if (hipMalloc((void **)&d_idx, sizeof(int32_t) * p.h_idx.size()) != hipSuccess ||
      hipMalloc((void **)&d_len, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc((void **)&d_val, sizeof(double) * p.h_val.size()) != hipSuccess) {
    (void)hipGetLastError();
    release();
    set_error("preconditioner allocation failed");
    return CPM_ENOMEM;
  }
  d_order = s->atom_order;
  hipError_t e = hipMemcpyAsync(d_idx, p.h_idx.data(), sizeof(int32_t) * p.h_idx.size(),
                                hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_len, p.h_len.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) {
    const int64_t tot = (int64_t)width * n;
    hipLaunchKernelGGL(sparse_inverse_values_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256),
                       0, s->stream, (const double *)s->S, s->ld, (const double *)s->dprime,
                       1.0 / s->c_ele, (const int32_t *)d_order, (const int32_t *)d_idx,
                       (const int32_t *)d_len, width, n, d_val);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(p.h_val.data(), d_val, sizeof(double) * p.h_val.size(),
                       hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  release();
  if (e != hipSuccess) {
    set_error(std::string("sparsified inverse: ") + hipGetErrorString(e));
    return CPM_EDEVICE;
  }
  p.kind = 1;
  p.rcut = rcut;
  p.width = width;
  p.nnz = nnz;
  return install_precond(s, p);
}

cpm_status cpm_precond_gap(cpm_system *s, int enable, double *gap_out) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  if (!s->pc.ready) {
    set_error("build a preconditioner first (cpm_precond_dc or cpm_precond_sparse_inverse)");
    return CPM_ESTATE;
  }
  Precond &p = s->pc;
  double gap = 0.0;
  if (enable) {
    if (!s->dprime_ready) {
      cpm_status rd = solve_dprime(s, 1e-13, 20000);
      if (rd != CPM_OK) return rd;
      s->dprime_ready = true;
    }
    const double nn = (double)s->n * (double)s->n;
    const double n_zero = nn - (double)p.nnz;
    // 1^T E^-1 1 = 1^T d' = C_ele
    gap = n_zero > 0.0 ? (s->c_ele - p.sum_p) / n_zero : 0.0;
  }
  if (p.blk != nullptr) {
    const std::vector<double> b = block_values(p, s->n, gap);
    CPM_HIP_CHECK(hipMemcpyAsync(p.blk, b.data(), sizeof(double) * b.size(),
                                 hipMemcpyHostToDevice, s->stream));
  } else {
    std::vector<double> val = p.h_val;
    if (gap != 0.0)
      for (int64_t t = 0; t < s->n; ++t)
        for (int k = 0; k < p.h_len[t]; ++k) val[(size_t)t * p.width + k] -= gap;
    CPM_HIP_CHECK(hipMemcpyAsync(p.val, val.data(), sizeof(double) * val.size(),
                                 hipMemcpyHostToDevice, s->stream));
  }
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  p.gap = gap;
  if (gap_out) *gap_out = gap;
  return CPM_OK;
}

cpm_status cpm_precond_coarse(cpm_system *s, double edge, int64_t *m_out) {
  if (m_out) *m_out = 0;
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  if (!std::isfinite(edge)) {
    set_error("the patch edge must be finite");
    return CPM_EINVAL;
  }
  if (edge <= 0.0) {
    CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
    s->device_bytes -= s->cz.bytes;
    free_coarse(s->cz);
    return CPM_OK;
  }
  if (!s->pc.ready) {
    set_error("build a preconditioner first (cpm_precond_dc or cpm_precond_sparse_inverse)");
    return CPM_ESTATE;
  }
  int64_t m = 0;
  int nslab = 0;
  const std::vector<int32_t> pid = coarse_patch_ids(s->pos_host, s->n, s->box, edge, m, nslab);
  if (m > kMaxCoarse) {
    set_error("coarse space: " + std::to_string(m) + " patches, more than " +
              std::to_string(kMaxCoarse) + " (take a larger patch edge)");
    return CPM_EINVAL;
  }
  // no enqueued solve still reads the previous coarse space
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  s->device_bytes -= s->cz.bytes;
  free_coarse(s->cz);
  Coarse c;
  c.edge = edge;
  c.nslab = nslab;
  const cpm_status rc = build_coarse(s, pid, m, c);
  if (rc != CPM_OK) {
    free_coarse(c);
    return rc;
  }
  c.ready = true;
  s->cz = c;
  s->device_bytes += c.bytes;
  if (m_out) *m_out = m;
  return CPM_OK;
}

cpm_status cpm_precond_apply(cpm_system *s, const double *r_dev, int64_t f, double *z_dev) {
  if (!s || !r_dev || !z_dev || f < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (!s->pc.ready) {
    set_error("cpm_precond_dc first");
    return CPM_ESTATE;
  }
  cpm_status rc = precond_cols(s, r_dev, f, z_dev);
  if (rc == CPM_OK) CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return rc;
}

}  // extern "C"
