// C ABI of libcpm: argument validation, system set-up and orchestration.
#include "cpm_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

namespace cpm {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

Kset make_kset(const double box[3], double beta, double kmax) {
  // K = 2 pi (n_x / L_x, n_y / L_y, n_z / L_z), 0 < |K| <= kmax, one of each
  // +-K pair (n_x > 0, or n_x = 0 and n_y > 0, or n_x = n_y = 0 and n_z > 0);
  // the pair's two terms cos(K.r) = cos(-K.r) are folded into a doubled weight
  // w = 2 (4 pi / V) exp(-K^2 / 4 beta^2) / K^2 (Eq. 13 and 20).
  Kset ks;
  const double vol = box[0] * box[1] * box[2];
  for (int d = 0; d < 3; ++d) ks.nmax[d] = (int)std::floor(kmax * box[d] / (2.0 * M_PI));
  const double k2max = kmax * kmax;
  for (int nx = 0; nx <= ks.nmax[0]; ++nx)
    for (int ny = -ks.nmax[1]; ny <= ks.nmax[1]; ++ny)
      for (int nz = -ks.nmax[2]; nz <= ks.nmax[2]; ++nz) {
        if (nx == 0 && (ny < 0 || (ny == 0 && nz <= 0))) continue;
        const double kx = 2.0 * M_PI * nx / box[0], ky = 2.0 * M_PI * ny / box[1],
                     kz = 2.0 * M_PI * nz / box[2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        if (k2 > k2max) continue;
        ks.n.push_back(nx);
        ks.n.push_back(ny);
        ks.n.push_back(nz);
        ks.w.push_back(2.0 * (4.0 * M_PI / vol) * std::exp(-k2 / (4.0 * beta * beta)) / k2);
      }
  ks.nk = (int64_t)ks.w.size();
  // runs: each (n_x, n_y) column (consecutive n_z) split into nearly equal
  // pieces of at most kRun vectors
  ks.info.assign(4 * ks.nk, 0);
  for (int64_t k = 0; k < ks.nk; ++k) {
    ks.info[4 * k] = ks.n[3 * k];
    ks.info[4 * k + 1] = ks.n[3 * k + 1];
    ks.info[4 * k + 2] = ks.n[3 * k + 2];
  }
  for (int64_t c0 = 0; c0 < ks.nk;) {
    int64_t c1 = c0 + 1;
    while (c1 < ks.nk && ks.n[3 * c1] == ks.n[3 * c0] && ks.n[3 * c1 + 1] == ks.n[3 * c0 + 1]) ++c1;
    const int64_t len = c1 - c0, pieces = (len + kRun - 1) / kRun;
    int64_t k = c0;
    for (int64_t p = 0; p < pieces; ++p) {
      const int64_t l = len / pieces + (p < len % pieces ? 1 : 0);
      ks.runs.push_back((int32_t)k);
      ks.runs.push_back((int32_t)l);
      ks.info[4 * k + 3] = 1;
      k += l;
    }
    c0 = c1;
  }
  ks.nruns = (int64_t)ks.runs.size() / 2;
  // columns: every (n_x, n_y) with n_x > 0 or n_y > 0 holds n_z = -m..m
  // (|K| <= kmax is symmetric in n_z); (0, 0) holds n_z = 1..m
  struct Col { int32_t nx, ny, m, kzero; };
  std::vector<Col> cols;
  for (int64_t c0 = 0; c0 < ks.nk;) {
    int64_t c1 = c0 + 1;
    while (c1 < ks.nk && ks.n[3 * c1] == ks.n[3 * c0] && ks.n[3 * c1 + 1] == ks.n[3 * c0 + 1]) ++c1;
    Col c;
    c.nx = ks.n[3 * c0];
    c.ny = ks.n[3 * c0 + 1];
    c.m = ks.n[3 * (c1 - 1) + 2];
    c.kzero = (int32_t)(c1 - 1 - c.m);
    cols.push_back(c);
    ks.smax = std::max(ks.smax, (int)c.m);
    c0 = c1;
  }
  std::stable_sort(cols.begin(), cols.end(), [](const Col &a, const Col &b) { return a.m > b.m; });
  ks.ncols = (int64_t)cols.size();
  ks.ncols_pad = round_up(std::max<int64_t>(ks.ncols, 1), kSfTile);
  ks.cols.assign(4 * ks.ncols_pad, 0);
  for (int64_t c = 0; c < ks.ncols_pad; ++c) {
    if (c < ks.ncols) {
      ks.cols[4 * c] = cols[c].nx;
      ks.cols[4 * c + 1] = cols[c].ny;
      ks.cols[4 * c + 2] = cols[c].m;
      ks.cols[4 * c + 3] = cols[c].kzero;
    } else {
      ks.cols[4 * c + 2] = -1;
    }
  }
  return ks;
}

// Atoms ordered by cubic tiles of edge 8 A (z, then y, then x tile, then
// index): the 64 atoms of a wavefront sit close together, so a distant
// ion leaves every lane outside the real-space cutoff.
std::vector<int32_t> spatial_order(const std::vector<double> &pos, int64_t n) {
  const double T = 8.0;
  std::vector<int64_t> key(n);
  std::vector<int32_t> idx(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t tx = (int64_t)std::floor(pos[3 * i] / T), ty = (int64_t)std::floor(pos[3 * i + 1] / T),
                  tz = (int64_t)std::floor(pos[3 * i + 2] / T);
    key[i] = (tz * 65536 + ty) * 65536 + tx;
    idx[i] = (int32_t)i;
  }
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  return idx;
}

// Distinct z of the (wrapped) positions, when there are at most kMaxPlanes
// of them: the z / L_z of each plane and tiles of kPlaneTile atoms of one
// plane each (atoms in spatial order within a plane, -1 pads). Empty
// results when the atoms spread over more planes.
void plane_tiles(const std::vector<double> &pos, int64_t n, double lz,
                 const std::vector<int32_t> &order, std::vector<double> &uz,
                 std::vector<int32_t> &tile_plane, std::vector<int32_t> &tile_atom) {
  uz.clear();
  tile_plane.clear();
  tile_atom.clear();
  std::vector<double> zs;
  for (int64_t i = 0; i < n; ++i) {
    const double z = pos[3 * i + 2];
    if (std::find(zs.begin(), zs.end(), z) == zs.end()) {
      if ((int)zs.size() == kMaxPlanes) return;
      zs.push_back(z);
    }
  }
  std::sort(zs.begin(), zs.end());
  std::vector<std::vector<int32_t>> members(zs.size());
  for (int64_t t = 0; t < n; ++t) {
    const int32_t i = order[t];
    const size_t p = std::lower_bound(zs.begin(), zs.end(), pos[3 * i + 2]) - zs.begin();
    members[p].push_back(i);
  }
  for (size_t p = 0; p < zs.size(); ++p) {
    uz.push_back(zs[p] / lz);
    const std::vector<int32_t> &m = members[p];
    for (size_t a = 0; a < m.size(); a += kPlaneTile) {
      tile_plane.push_back((int32_t)p);
      for (int r = 0; r < kPlaneTile; ++r)
        tile_atom.push_back(a + r < m.size() ? m[a + r] : -1);
    }
  }
}

hipEvent_t Profile::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

Profile::Rec &Profile::add(int kind, double work) {
  Rec r;
  r.kind = kind;
  r.work = work;
  r.a = get();
  r.b = get();
  recs.push_back(r);
  return recs.back();
}

void Profile::reset() {
  for (Rec &r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  next_mark = 0;
}

void *grow_buf(cpm_system *s, DevBuf &b, size_t bytes, cpm_status *rc) {
  *rc = CPM_OK;
  if (bytes <= b.bytes) return b.p;
  // at least 1.5x the old size, so that a slowly growing caller reallocates
  // a few times only
  const size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  if (b.p) {
    if (hipStreamSynchronize(s->stream) != hipSuccess) {
      set_error("stream synchronisation before a scratch resize failed");
      *rc = CPM_EDEVICE;
      return nullptr;
    }
    (void)hipFree(b.p);
    s->device_bytes -= (int64_t)b.bytes;
    b = DevBuf();
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b = DevBuf();
    set_error("device allocation of " + std::to_string(want) + " bytes of scratch failed");
    *rc = CPM_ENOMEM;
    return nullptr;
  }
  b.bytes = want;
  s->device_bytes += (int64_t)want;
  return b.p;
}

}  // namespace cpm

using namespace cpm;

namespace {

template <typename T> cpm_status dev_alloc(cpm_system *s, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return CPM_OK;
  if (hipMalloc((void **)p, sizeof(T) * count) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    return CPM_ENOMEM;
  }
  s->device_bytes += (int64_t)(sizeof(T) * count);
  return CPM_OK;
}

void free_system(cpm_system *s) {
  if (!s) return;
  void *ptrs[] = {s->pos, s->width, s->kn, s->kw, s->kinfo, s->krun, s->kcol, s->atom_order,
                  s->plane_uz, s->plane_tile, s->plane_atom, s->E64, s->E32, s->E16, s->dinv, s->dprime,
                  s->dvec, s->qchi, s->erfc_tab, s->rhs_S, s->S, s->mlp.nbr, s->mlp.nbr_r, s->mlp.layer, s->mlp.params,
                  s->mlp.adam_m, s->mlp.adam_v, s->mlp.grad, s->mlp.gpart, s->mlp.loss,
                  s->mlp.feat, s->mlp.yout};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (s->rs_width && s->rs_width != s->width) (void)hipFree(s->rs_width);
  for (DevBuf *b : {&s->buf_warm, &s->buf_eq, &s->buf_mean, &s->buf_aux})
    if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : s->warm_ev)
    if (e) (void)hipEventDestroy(e);
  release_workspace(s);
  free_precond(s->pc);
  free_coarse(s->cz);
  free_gcd(s->gcd);
  s->prof.reset();
  for (hipEvent_t e : s->prof.pool) (void)hipEventDestroy(e);
  if (s->prof.marks) (void)hipFree(s->prof.marks);
  delete s;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace

extern "C" {

const char *cpm_status_str(cpm_status st) {
  switch (st) {
    case CPM_OK: return "CPM_OK";
    case CPM_EINVAL: return "CPM_EINVAL";
    case CPM_ENOMEM: return "CPM_ENOMEM";
    case CPM_EDEVICE: return "CPM_EDEVICE";
    case CPM_ENOTSPD: return "CPM_ENOTSPD";
    case CPM_ENOTCONV: return "CPM_ENOTCONV";
    case CPM_ESTATE: return "CPM_ESTATE";
  }
  return "CPM_UNKNOWN";
}

const char *cpm_last_error(void) { return cpm::last_error(); }

cpm_status cpm_build_E(const double *pos_host, int64_t n, const double *box_host,
                       const cpm_params *params, void *stream, cpm_system **out) {
  if (!out) {
    set_error("out is NULL");
    return CPM_EINVAL;
  }
  *out = nullptr;
  if (!pos_host || !box_host || !params) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (n < 1 || n > (int64_t)1 << 20) {
    set_error("n must be in [1, 2^20]");
    return CPM_EINVAL;
  }
  for (int d = 0; d < 3; ++d)
    if (!(std::isfinite(box_host[d]) && box_host[d] > 0.0)) {
      set_error("box edges must be finite and > 0");
      return CPM_EINVAL;
    }
  const double beta = params->ewald_split;
  if (!(std::isfinite(beta) && beta > 0.0)) {
    set_error("ewald_split must be finite and > 0");
    return CPM_EINVAL;
  }
  if (!(std::isfinite(params->rcut) && params->rcut > 0.0)) {
    set_error("rcut must be finite and > 0");
    return CPM_EINVAL;
  }
  double kmax = params->kmax_override;
  if (!(kmax > 0.0)) {
    const double eps = params->kspace_eps;
    if (!(eps > 0.0 && eps < 1.0)) {
      set_error("kspace_eps must be in (0, 1) when kmax_override <= 0");
      return CPM_EINVAL;
    }
    kmax = 2.0 * beta * std::sqrt(std::log(1.0 / eps));
  }
  if (!std::isfinite(kmax)) {
    set_error("kmax must be finite");
    return CPM_EINVAL;
  }
  if (params->store_mask & ~(unsigned)(CPM_STORE_F32 | CPM_STORE_BF16 | CPM_PROFILE_BUILD)) {
    set_error("unknown bits in store_mask");
    return CPM_EINVAL;
  }
  std::vector<double> width(n);
  const bool point_self = params->point_charge_self != 0;
  for (int64_t i = 0; i < n; ++i) {
    const double a = params->gauss_inv_width_per_atom ? params->gauss_inv_width_per_atom[i]
                                                      : params->gauss_inv_width;
    if (!(a > 0.0) || std::isnan(a)) {   // +inf is a point charge
      set_error("Gaussian inverse widths must be > 0 (inf = point charge)");
      return CPM_EINVAL;
    }
    if (point_self && !std::isfinite(a)) {
      set_error("point_charge_self needs finite widths (they set the self-energy)");
      return CPM_EINVAL;
    }
    width[i] = a;
  }
  std::vector<double> pos(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    if (!finite3(pos_host + 3 * i)) {
      set_error("non-finite position at atom " + std::to_string(i));
      return CPM_EINVAL;
    }
    for (int d = 0; d < 3; ++d) {
      double x = std::fmod(pos_host[3 * i + d], box_host[d]);
      if (x < 0) x += box_host[d];
      if (x >= box_host[d]) x -= box_host[d];
      pos[3 * i + d] = x;
    }
  }
  // coincident atoms (minimum image), via a uniform cell grid
  {
    const double tol2 = 1e-12;   // (1e-6 A)^2
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = std::max(1, std::min(256, (int)(box_host[d] / 2.0)));
    std::vector<std::vector<int64_t>> cells((size_t)nc[0] * nc[1] * nc[2]);
    auto cell_of = [&](int64_t i, int d) {
      int c = (int)(pos[3 * i + d] / box_host[d] * nc[d]);
      return std::min(std::max(c, 0), nc[d] - 1);
    };
    for (int64_t i = 0; i < n; ++i)
      cells[((size_t)cell_of(i, 0) * nc[1] + cell_of(i, 1)) * nc[2] + cell_of(i, 2)].push_back(i);
    for (int64_t i = 0; i < n; ++i) {
      const int ci[3] = {cell_of(i, 0), cell_of(i, 1), cell_of(i, 2)};
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            const int cx = (ci[0] + a + nc[0]) % nc[0], cy = (ci[1] + b + nc[1]) % nc[1],
                      cz = (ci[2] + c + nc[2]) % nc[2];
            for (int64_t j : cells[((size_t)cx * nc[1] + cy) * nc[2] + cz]) {
              if (j <= i) continue;
              double d2 = 0;
              for (int d = 0; d < 3; ++d) {
                double dx = pos[3 * j + d] - pos[3 * i + d];
                dx -= box_host[d] * std::nearbyint(dx / box_host[d]);
                d2 += dx * dx;
              }
              if (d2 < tol2) {
                set_error("atoms " + std::to_string(i) + " and " + std::to_string(j) +
                          " coincide (distance < 1e-6 A)");
                return CPM_EINVAL;
              }
            }
          }
    }
  }

  cpm_system *s = new (std::nothrow) cpm_system();
  if (!s) {
    set_error("host allocation failed");
    return CPM_ENOMEM;
  }
  s->stream = (hipStream_t)stream;
  (void)hipGetDevice(&s->device);
  s->n = n;
  s->ld = round_up(n, 128);
  for (int d = 0; d < 3; ++d) s->box[d] = box_host[d];
  s->vol = box_host[0] * box_host[1] * box_host[2];
  s->beta = beta;
  s->rcut = params->rcut;
  s->kmax = kmax;
  s->kset = make_kset(box_host, beta, kmax);
  s->slab = params->slab_correction != 0;
  s->point_self = point_self;
  s->prof.enabled = (params->store_mask & CPM_PROFILE_BUILD) != 0;
  s->pos_host = pos;
  s->width_host = width;
  const int64_t ld = s->ld, nk = s->kset.nk;
  hipStream_t st = s->stream;

  cpm_status rc = CPM_OK;
  auto fail = [&](cpm_status e) {
    free_system(s);
    return e;
  };
  if ((rc = dev_alloc(s, &s->pos, 3 * n)) || (rc = dev_alloc(s, &s->width, n)) ||
      (rc = dev_alloc(s, &s->kn, 3 * std::max<int64_t>(nk, 1))) ||
      (rc = dev_alloc(s, &s->kw, std::max<int64_t>(nk, 1))) ||
      (rc = dev_alloc(s, &s->kinfo, 4 * std::max<int64_t>(nk, 1))) ||
      (rc = dev_alloc(s, &s->krun, 2 * std::max<int64_t>(s->kset.nruns, 1))) ||
      (rc = dev_alloc(s, &s->kcol, 4 * s->kset.ncols_pad)) ||
      (rc = dev_alloc(s, &s->atom_order, n)) ||
      (rc = dev_alloc(s, &s->E64, (size_t)ld * ld)) || (rc = dev_alloc(s, &s->dinv, ld)) ||
      (rc = dev_alloc(s, &s->dprime, ld)) || (rc = dev_alloc(s, &s->dvec, ld)) ||
      (rc = dev_alloc(s, &s->qchi, ld)) || (rc = dev_alloc(s, &s->erfc_tab, kErfcTab)))
    return fail(rc);
  if (point_self) {
    if ((rc = dev_alloc(s, &s->rs_width, n))) return fail(rc);
  } else {
    s->rs_width = s->width;
  }
  if ((params->store_mask & CPM_STORE_F32) && (rc = dev_alloc(s, &s->E32, (size_t)ld * ld)))
    return fail(rc);
  if ((params->store_mask & CPM_STORE_BF16) && (rc = dev_alloc(s, &s->E16, (size_t)ld * ld)))
    return fail(rc);

#define BUILD_CHECK(expr)                                                  \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));        \
      return fail(CPM_EDEVICE);                                            \
    }                                                                      \
  } while (0)

  std::vector<double> etab(kErfcTab);
  erfc_table(etab.data());
  BUILD_CHECK(hipMemcpyAsync(s->erfc_tab, etab.data(), sizeof(double) * kErfcTab,
                             hipMemcpyHostToDevice, st));
  BUILD_CHECK(hipMemcpyAsync(s->pos, pos.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
  BUILD_CHECK(hipMemcpyAsync(s->width, width.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  if (point_self) {
    const std::vector<double> unscreened(n, INFINITY);
    BUILD_CHECK(hipMemcpyAsync(s->rs_width, unscreened.data(), sizeof(double) * n,
                               hipMemcpyHostToDevice, st));
  }
  if (nk > 0) {
    BUILD_CHECK(hipMemcpyAsync(s->kn, s->kset.n.data(), sizeof(int32_t) * 3 * nk,
                               hipMemcpyHostToDevice, st));
    BUILD_CHECK(hipMemcpyAsync(s->kw, s->kset.w.data(), sizeof(double) * nk, hipMemcpyHostToDevice,
                               st));
    BUILD_CHECK(hipMemcpyAsync(s->kinfo, s->kset.info.data(), sizeof(int32_t) * 4 * nk,
                               hipMemcpyHostToDevice, st));
    BUILD_CHECK(hipMemcpyAsync(s->kcol, s->kset.cols.data(), sizeof(int32_t) * 4 * s->kset.ncols_pad,
                               hipMemcpyHostToDevice, st));
    BUILD_CHECK(hipMemcpyAsync(s->krun, s->kset.runs.data(), sizeof(int32_t) * 2 * s->kset.nruns,
                               hipMemcpyHostToDevice, st));
  }
  const std::vector<int32_t> order = spatial_order(pos, n);
  BUILD_CHECK(hipMemcpyAsync(s->atom_order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice,
                             st));
  if (nk > 0 && s->kset.smax <= kMaxPlaneS) {
    std::vector<double> uz;
    std::vector<int32_t> tp, ta;
    plane_tiles(pos, n, box_host[2], order, uz, tp, ta);
    if (!uz.empty()) {
      s->nplanes = (int)uz.size();
      s->plane_ntiles = (int64_t)tp.size();
      if ((rc = dev_alloc(s, &s->plane_uz, uz.size())) ||
          (rc = dev_alloc(s, &s->plane_tile, tp.size())) ||
          (rc = dev_alloc(s, &s->plane_atom, ta.size())))
        return fail(rc);
      BUILD_CHECK(hipMemcpyAsync(s->plane_uz, uz.data(), sizeof(double) * uz.size(),
                                 hipMemcpyHostToDevice, st));
      BUILD_CHECK(hipMemcpyAsync(s->plane_tile, tp.data(), sizeof(int32_t) * tp.size(),
                                 hipMemcpyHostToDevice, st));
      BUILD_CHECK(hipMemcpyAsync(s->plane_atom, ta.data(), sizeof(int32_t) * ta.size(),
                                 hipMemcpyHostToDevice, st));
      // the host vectors go out of scope: wait for the copies
      BUILD_CHECK(hipStreamSynchronize(st));
    }
  }
  BUILD_CHECK(hipMemsetAsync(s->qchi, 0, sizeof(double) * ld, st));

  // Reciprocal part A A^T in chunks of k-vectors whose phase matrix stays
  // under 24 GiB (or a third of the free memory): every chunk but the first
  // adds to the lower tiles of E, so larger chunks re-read E less often.
  // finalize_kernel writes every entry of E (padding included), so E needs
  // no clearing.
  if (nk > 0) {
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    size_t budget = std::min<size_t>((size_t)24 << 30, free_b / 3);
    int64_t kc = (int64_t)(budget / (sizeof(double) * 2 * (size_t)ld));
    kc = std::max<int64_t>(8, kc / 8 * 8);
    // equal chunks (the last one is not padded with zero columns)
    const int64_t nchunks = (nk + kc - 1) / kc;
    kc = round_up((nk + nchunks - 1) / nchunks, 8);
    const int64_t lda = 2 * kc;
    double *A = nullptr;
    int32_t *tiles = nullptr;
    const std::vector<int32_t> order_t = syrk_tile_order(ld / 128);
    if ((int64_t)order_t.size() != (ld / 128) * (ld / 128 + 1)) {
      set_error("internal: tile list size");
      return fail(CPM_EDEVICE);
    }
    // CPM_PROGRESS=1 in the environment: one line on stderr per finished
    // chunk (long assemblies)
    const char *prog_env = std::getenv("CPM_PROGRESS");
    const bool progress = prog_env && prog_env[0] == '1';
    const auto t_asm = std::chrono::steady_clock::now();
    if (hipMalloc((void **)&A, sizeof(double) * (size_t)ld * lda) != hipSuccess ||
        hipMalloc((void **)&tiles, sizeof(int32_t) * order_t.size()) != hipSuccess) {
      (void)hipGetLastError();
      if (A) (void)hipFree(A);
      set_error("phase matrix allocation failed");
      return fail(CPM_ENOMEM);
    }
    auto release = [&]() {
      (void)hipFree(A);
      (void)hipFree(tiles);
    };
    hipError_t e = hipMemcpyAsync(tiles, order_t.data(), sizeof(int32_t) * order_t.size(),
                                  hipMemcpyHostToDevice, st);
    for (int64_t k0 = 0; k0 < nk && e == hipSuccess; k0 += kc) {
      const int64_t kcur = std::min(kc, nk - k0);
      e = launch_phase_matrix(st, s->pos, n, ld, s->box, s->kn, s->kw, k0, kcur,
                              round_up(2 * kcur, 16), A);
      // algorithmic flops of the contraction: 2 products (cos, sin) per
      // k-vector for each unique pair i <= j, 2 flops each
      hipEvent_t ea = nullptr, eb = nullptr;
      if (s->prof.enabled) {
        Profile::Rec &r = s->prof.add(3, 4.0 * (double)kcur * (double)n * (double)(n + 1) / 2.0);
        ea = r.a;
        eb = r.b;
      }
      if (e == hipSuccess)
        e = launch_syrk_lower(st, A, round_up(2 * kcur, 16), tiles, ld, s->E64, ld, k0 > 0, ea,
                              eb);
      if (progress && e == hipSuccess) {
        e = hipStreamSynchronize(st);
        std::fprintf(stderr, "cpm_build_E: k-vectors %lld of %lld done (%.1f s)\n",
                     (long long)(k0 + kcur), (long long)nk,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t_asm).count());
        std::fflush(stderr);
      }
    }
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      release();
      set_error(std::string("E assembly launch failed: ") + hipGetErrorString(e));
      return fail(CPM_EDEVICE);
    }
    BUILD_CHECK(hipStreamSynchronize(st));
    release();
  } else {
    BUILD_CHECK(hipMemsetAsync(s->E64, 0, sizeof(double) * ld * ld, st));
  }
  BUILD_CHECK(launch_finalize(st, s->pos, s->width, s->rs_width, n, ld, s->box, beta, s->rcut,
                              s->slab, s->E64, s->E32, s->E16));
  BUILD_CHECK(launch_diag_inverse(st, s->E64, n, ld, s->dinv));
  BUILD_CHECK(hipStreamSynchronize(st));
#undef BUILD_CHECK

  // d' = E^-1 1 is solved on first use (cpm_solve, cpm_get_dprime, ...):
  // E of point charges alone need not be positive definite, and its entries
  // are still useful.
  *out = s;
  return CPM_OK;
}

void cpm_free(cpm_system *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_system(s);
}

cpm_status cpm_set_stream(cpm_system *s, void *stream) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  s->stream = (hipStream_t)stream;
  return CPM_OK;
}

cpm_status cpm_describe(const cpm_system *s, int64_t *n, int64_t *n_kvec, double *kmax,
                        int64_t *device_bytes) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  if (n) *n = s->n;
  if (n_kvec) *n_kvec = s->kset.nk;
  if (kmax) *kmax = s->kmax;
  if (device_bytes) *device_bytes = s->device_bytes;
  return CPM_OK;
}

cpm_status cpm_rhs(cpm_system *s, const double *ion_pos_dev, const double *ion_q_dev, int64_t m,
                   int64_t f, const double *chi_dev, double *b_out_dev, double *qsol_out_dev) {
  if (!s || !chi_dev || !b_out_dev || !qsol_out_dev || (m > 0 && (!ion_pos_dev || !ion_q_dev))) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (f < 1 || m < 0) {
    set_error("need f >= 1 and m >= 0");
    return CPM_EINVAL;
  }
  const int64_t fchunk = 1024;
  // scratch for the largest of the chunk sizes used (full chunks and the tail)
  int64_t need = rhs_scratch_elems(s, m, std::min(f, fchunk));
  if (f > fchunk && f % fchunk) need = std::max(need, rhs_scratch_elems(s, m, f % fchunk));
  if (s->rhs_S_elems < need) {
    if (s->rhs_S) {
      (void)hipFree(s->rhs_S);
      s->device_bytes -= (int64_t)(sizeof(double) * s->rhs_S_elems);
      s->rhs_S = nullptr;
      s->rhs_S_elems = 0;
    }
    cpm_status rc = dev_alloc(s, &s->rhs_S, need);
    if (rc != CPM_OK) return rc;
    s->rhs_S_elems = need;
  }
  for (int64_t f0 = 0; f0 < f; f0 += fchunk) {
    const int64_t fc = std::min(fchunk, f - f0);
    CPM_HIP_CHECK(launch_rhs(s->stream, s, m > 0 ? ion_pos_dev + f0 * m * 3 : nullptr,
                             m > 0 ? ion_q_dev + f0 * m : nullptr, m, fc, chi_dev, s->rhs_S,
                             b_out_dev + f0 * s->n, qsol_out_dev + f0));
  }
  return CPM_OK;
}

cpm_status cpm_rhs_noalloc(cpm_system *s, const double *ion_pos_dev, const double *ion_q_dev,
                           int64_t m, int64_t f, const double *chi_dev, double *b_out_dev,
                           double *qsol_out_dev) {
  if (!s || !chi_dev || !b_out_dev || !qsol_out_dev || (m > 0 && (!ion_pos_dev || !ion_q_dev))) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (f < 1 || m < 0) {
    set_error("need f >= 1 and m >= 0");
    return CPM_EINVAL;
  }
  const int64_t cap = rhs_static_scratch_elems();
  const int64_t fchunk = 1024;
  int64_t need = rhs_scratch_elems_capped(s, m, std::min(f, fchunk), cap);
  if (f > fchunk && f % fchunk)
    need = std::max(need, rhs_scratch_elems_capped(s, m, f % fchunk, cap));
  if (need > cap) {
    set_error("cpm_rhs_noalloc: " + std::to_string(m) + " ions x " + std::to_string(std::min(f, fchunk)) +
              " frames need " + std::to_string(need) + " doubles of scratch; the static buffer holds " +
              std::to_string(cap) + " (use cpm_rhs)");
    return CPM_EINVAL;
  }
  double *buf = nullptr;
  CPM_HIP_CHECK(rhs_static_scratch(&buf));
  for (int64_t f0 = 0; f0 < f; f0 += fchunk) {
    const int64_t fc = std::min(fchunk, f - f0);
    CPM_HIP_CHECK(launch_rhs(s->stream, s, m > 0 ? ion_pos_dev + f0 * m * 3 : nullptr,
                             m > 0 ? ion_q_dev + f0 * m : nullptr, m, fc, chi_dev, buf,
                             b_out_dev + f0 * s->n, qsol_out_dev + f0, cap));
  }
  return CPM_OK;
}

}  // extern "C"

cpm_status cpm::check_solve_opts(const cpm_system *s, const cpm_solve_opts *opts,
                                  cpm_solve_opts *out) {
  cpm_solve_opts o = *opts;
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) {
    set_error("tol must be finite and > 0");
    return CPM_EINVAL;
  }
  if (o.max_iter < 1) {
    set_error("max_iter must be >= 1");
    return CPM_EINVAL;
  }
  if (o.preconditioner != CPM_PRECOND_JACOBI && o.preconditioner != CPM_PRECOND_DC) {
    set_error("unknown preconditioner");
    return CPM_EINVAL;
  }
  if (o.preconditioner == CPM_PRECOND_DC && !s->pc.ready) {
    set_error("CPM_PRECOND_DC: call cpm_precond_dc first");
    return CPM_ESTATE;
  }
  if (o.precision == CPM_PREC_F32 && !s->E32) {
    set_error("FP32 copy of E not stored (store_mask)");
    return CPM_EINVAL;
  }
  if (o.precision == CPM_PREC_BF16 && !s->E16) {
    set_error("BF16 copy of E not stored (store_mask)");
    return CPM_EINVAL;
  }
  if (o.precision < CPM_PREC_F64 || o.precision > CPM_PREC_BF16) {
    set_error("unknown precision");
    return CPM_EINVAL;
  }
  if (o.precision != CPM_PREC_F64 && !(o.inner_tol > 0.0 && o.inner_tol < 1.0)) o.inner_tol = 1e-3;
  if (o.check_every < 1) o.check_every = 8;
  *out = o;
  return CPM_OK;
}

extern "C" {

namespace {
cpm_status ensure_dprime(cpm_system *s) {
  if (s->dprime_ready) return CPM_OK;
  cpm_status rc = solve_dprime(s, 1e-13, 20000);
  if (rc == CPM_OK) s->dprime_ready = true;
  return rc;
}
}  // namespace

cpm_status cpm_solve(cpm_system *s, const double *b_dev, const double *qsol_dev, int64_t f,
                     const cpm_solve_opts *opts, double *q_out_dev, cpm_solve_info *info) {
  if (!s || !b_dev || !qsol_dev || !opts || !q_out_dev) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  {
    cpm_status rd = ensure_dprime(s);
    if (rd != CPM_OK) return rd;
  }
  if (f < 1) {
    set_error("need f >= 1");
    return CPM_EINVAL;
  }
  cpm_solve_opts o;
  {
    cpm_status ro = check_solve_opts(s, opts, &o);
    if (ro != CPM_OK) return ro;
  }
  if (info) {
    int *fi = info->frame_iters;
    double *fr = info->frame_rel_resid;
    std::memset(info, 0, sizeof(*info));
    info->frame_iters = fi;
    info->frame_rel_resid = fr;
  }
  const auto t_call = std::chrono::steady_clock::now();
  const double *x0 = nullptr, *r0 = nullptr;
  double *x0_buf = nullptr;
  if (o.warm_start == CPM_WARM_CHI || o.warm_start == CPM_WARM_MLP) {
    if (o.warm_start == CPM_WARM_MLP && !(s->mlp.ready && s->mlp.params_set)) {
      set_error("CPM_WARM_MLP needs cpm_mlp_init and cpm_mlp_set_params first");
      return CPM_ESTATE;
    }
    if (o.warm_start == CPM_WARM_CHI && !s->qchi_ready) {
      set_error("CPM_WARM_CHI needs cpm_set_warm_chi first");
      return CPM_ESTATE;
    }
    if (!s->warm_ev[0]) {
      CPM_HIP_CHECK(hipEventCreate(&s->warm_ev[0]));
      CPM_HIP_CHECK(hipEventCreate(&s->warm_ev[1]));
    }
    // the start and its FP64 residual (the solver's first residual)
    cpm_status rb = CPM_OK;
    x0_buf = (double *)grow_buf(s, s->buf_warm, sizeof(double) * 2 * f * s->n, &rb);
    if (rb != CPM_OK) return rb;
    CPM_HIP_CHECK(hipEventRecord(s->warm_ev[0], s->stream));
    cpm_status rc = warm_start_impl(s, o.warm_start == CPM_WARM_MLP, b_dev, qsol_dev, f, x0_buf,
                                    x0_buf + f * s->n);
    if (rc != CPM_OK) return rc;
    CPM_HIP_CHECK(hipEventRecord(s->warm_ev[1], s->stream));
    x0 = x0_buf;
    r0 = x0_buf + f * s->n;
  } else if (o.warm_start != CPM_WARM_ZERO) {
    set_error("unknown warm_start");
    return CPM_EINVAL;
  }
  cpm_status rc = solve_block(s, b_dev, qsol_dev, f, o, q_out_dev, info, x0, true, r0);
  if (info) {
    // the solve has synchronised the stream: the warm start's time from its
    // events, the call's from the host clock
    float ms = 0.0f;
    if (x0_buf && hipEventElapsedTime(&ms, s->warm_ev[0], s->warm_ev[1]) == hipSuccess)
      info->warm_ms = ms;
    info->solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
  }
  return rc;
}

cpm_status cpm_warm_start(cpm_system *s, int warm_start, const double *b_dev,
                          const double *qsol_dev, int64_t f, double *x0_out_dev,
                          double *r0_out_dev) {
  if (!s || !b_dev || !qsol_dev || !x0_out_dev || !r0_out_dev || f < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if (warm_start != CPM_WARM_CHI && warm_start != CPM_WARM_MLP) {
    set_error("warm_start must be CPM_WARM_CHI or CPM_WARM_MLP");
    return CPM_EINVAL;
  }
  if (warm_start == CPM_WARM_MLP && !(s->mlp.ready && s->mlp.params_set)) {
    set_error("CPM_WARM_MLP needs cpm_mlp_init and cpm_mlp_set_params first");
    return CPM_ESTATE;
  }
  if (warm_start == CPM_WARM_CHI && !s->qchi_ready) {
    set_error("CPM_WARM_CHI needs cpm_set_warm_chi first");
    return CPM_ESTATE;
  }
  {
    cpm_status rd = ensure_dprime(s);
    if (rd != CPM_OK) return rd;
  }
  cpm_status rc = warm_start_impl(s, warm_start == CPM_WARM_MLP, b_dev, qsol_dev, f, x0_out_dev,
                                  r0_out_dev);
  if (rc != CPM_OK) return rc;
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_get_E(const cpm_system *s, int precision, void *dst_dev, int64_t ld) {
  if (!s || !dst_dev) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (ld < s->n) {
    set_error("ld must be >= n");
    return CPM_EINVAL;
  }
  const void *src = nullptr;
  size_t es = 0;
  if (precision == CPM_PREC_F64) { src = s->E64; es = 8; }
  else if (precision == CPM_PREC_F32) { src = s->E32; es = 4; }
  else if (precision == CPM_PREC_BF16) { src = s->E16; es = 2; }
  if (!src) {
    set_error("requested precision of E is not stored");
    return CPM_EINVAL;
  }
  CPM_HIP_CHECK(hipMemcpy2DAsync(dst_dev, es * ld, src, es * s->ld, es * s->n, s->n,
                                 hipMemcpyDeviceToDevice, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_get_E_block(const cpm_system *s, int precision, int64_t row0, int64_t col0,
                           int64_t rows, int64_t cols, void *dst_dev, int64_t ld) {
  if (!s || !dst_dev) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  if (row0 < 0 || col0 < 0 || rows < 1 || cols < 1 || row0 + rows > s->n || col0 + cols > s->n ||
      ld < cols) {
    set_error("block outside E or ld < cols");
    return CPM_EINVAL;
  }
  const void *src = nullptr;
  size_t es = 0;
  if (precision == CPM_PREC_F64) { src = s->E64; es = 8; }
  else if (precision == CPM_PREC_F32) { src = s->E32; es = 4; }
  else if (precision == CPM_PREC_BF16) { src = s->E16; es = 2; }
  if (!src) {
    set_error("requested precision of E is not stored");
    return CPM_EINVAL;
  }
  const char *base = static_cast<const char *>(src) + es * ((size_t)row0 * s->ld + col0);
  CPM_HIP_CHECK(hipMemcpy2DAsync(dst_dev, es * ld, base, es * s->ld, es * cols, rows,
                                 hipMemcpyDeviceToDevice, s->stream));
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_get_dprime(cpm_system *s, double *dst_dev, double *c_ele) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  {
    cpm_status rd = ensure_dprime(s);
    if (rd != CPM_OK) return rd;
  }
  if (dst_dev)
    CPM_HIP_CHECK(hipMemcpyAsync(dst_dev, s->dprime, sizeof(double) * s->n, hipMemcpyDeviceToDevice,
                                 s->stream));
  if (c_ele) *c_ele = s->c_ele;
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return CPM_OK;
}

cpm_status cpm_profile_enable(cpm_system *s, int on) {
  if (!s) {
    set_error("NULL system");
    return CPM_EINVAL;
  }
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  s->prof.reset();
  if (on && !s->prof.marks) {
    if (hipMalloc((void **)&s->prof.marks, sizeof(int) * Profile::kMarks) != hipSuccess) {
      (void)hipGetLastError();
      s->prof.marks = nullptr;   // gated launches are then all counted
    }
  }
  s->prof.enabled = on != 0;
  s->prof.stride = on > 1 ? on : 1;
  for (int64_t &c : s->prof.seen) c = 0;
  return CPM_OK;
}

cpm_status cpm_profile_read(cpm_system *s, cpm_profile_info *out) {
  if (!s || !out) {
    set_error("NULL argument");
    return CPM_EINVAL;
  }
  CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  std::memset(out, 0, sizeof(*out));
  std::vector<int> marks(s->prof.next_mark, 1);
  if (s->prof.next_mark > 0)
    CPM_HIP_CHECK(hipMemcpy(marks.data(), s->prof.marks, sizeof(int) * s->prof.next_mark,
                            hipMemcpyDeviceToHost));
  for (const Profile::Rec &r : s->prof.recs) {
    if (r.mark >= 0 && marks[r.mark] == 0) continue;   // gated off: no product computed
    float ms = 0.f;
    CPM_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    out->launches[r.kind] += 1;
    out->ms[r.kind] += ms;
    out->work[r.kind] += r.work;
  }
  return CPM_OK;
}

cpm_status cpm_matvec(cpm_system *s, int precision, const double *p_dev, int64_t f,
                      double *v_dev) {
  if (!s || !p_dev || !v_dev || f < 1) {
    set_error("invalid argument");
    return CPM_EINVAL;
  }
  if ((precision == CPM_PREC_F32 && !s->E32) || (precision == CPM_PREC_BF16 && !s->E16) ||
      precision < 0 || precision > 2) {
    set_error("requested precision of E is not stored");
    return CPM_EINVAL;
  }
  cpm_status rc = matvec_cols(s, precision, p_dev, f, v_dev);
  if (rc == CPM_OK) CPM_HIP_CHECK(hipStreamSynchronize(s->stream));
  return rc;
}

}  // extern "C"
