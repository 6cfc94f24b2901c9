// Plan, scheduling and C ABI of the multipole estimator (include/pkm.h).
//
// One plan = one mesh size, box, observer, window and precision.  pkm_paint runs
//   catalog sums -> zero meshes -> paint (data, then -alpha x randoms) -> forward z of D1, D2
//   -> forward y -> x pass with interlace combine + compensation (writes C and G = x-inverse
//   of C) -> inverse y of G,
// leaving C (the combined field, F_0 of eq. Pell-ours) and G (D_c, transformed along z only)
// resident.  pkm_compute_multipoles then runs, per group of (l, m) fields,
//   zpre (inverse z of G = D_c, Y_lm(xhat) weighting, forward z per field) -> column pass
//   per field (y for FP32, x for FP64) -> xpost (the remaining axis, sum_m Y_lm(khat) B_lm,
//   product with C, binning)
// and one fixed-order reduction per group.  The l = 0 bin (|C|^2) and the mode counts are
// taken in the first xpost pass.  pkm_prepare / pkm_enqueue / pkm_finish issue the same
// work asynchronously; runtime.hip builds batches and the serving loop on them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/pkm.h"
#include "kernels.hpp"
#include "device_common.hpp"
#include "internal.hpp"

using namespace pkm;

// One field group of a multipole request: field-table offsets, reduce map, histogram shape.
struct GroupCfg {
  int nf = 0, fofs = 0, pofs = 0, mofs = 0, nv = 0, nslots = 0, copies = 1;
};
struct ComputeCfg {
  int ell_max = -1;
  // 0: spherical harmonics, even l (Sec. 2.1); 1: Cartesian monomials, even l; 2: spherical
  // harmonics, every l (odd l binned as Im[C conj A_l]: pkm_compute_multipoles_all)
  int basis = 0;
  std::vector<double> edges;
  int nb = 0, total_vals = 0, nfields_total = 0;
  std::vector<GroupCfg> groups;
};

struct pkm_plan {
  pkm_params p{};
  pkm_device dev{};
  hipStream_t stream = nullptr;
  bool fp64 = false;
  size_t es = 4;        // real element bytes
  size_t mesh_bytes = 0;
  FftShape fs{};
  Frame frame{};        // harmonic frame (mean line of sight -> (1,1,1)/sqrt 3)
  // resident buffers
  void* d1 = nullptr;
  void* d2 = nullptr;
  void* s1 = nullptr;
  void* s2 = nullptr;
  void* c = nullptr;
  void* g = nullptr;
  std::vector<void*> fields;
  void** ptrs_dev = nullptr;  // device array of buffer pointers (fields, then scratch slots)
  int ptr_cap = 0;
  void** paint_ptrs = nullptr;  // device array {s1, s2, g} for the paint passes
  ComputeCfg cc;              // tables of the last prepared multipole request
  // asynchronous estimate (pkm_prepare / pkm_enqueue / pkm_finish)
  int prep_ell = -1;          // the request of the last pkm_prepare (spherical basis)
  std::vector<double> prep_edges;
  double* slot = nullptr;     // pinned host staging, slot_cap doubles
  size_t slot_cap = 0;
  hipEvent_t done = nullptr;
  int64_t pend_nd = 0, pend_nr = 0;
  bool pending_async = false;
  int* ftab_dev = nullptr;    // (l, m, slot) per field, all groups
  int ftab_cap = 0;
  int* map_dev = nullptr;     // reduce map per value
  int map_cap = 0;
  void* tw = nullptr;
  void* ytab = nullptr;
  void* invw = nullptr;
  void* phase = nullptr;
  long long* thr_dev = nullptr;
  int thr_cap = 0;
  double* partial = nullptr;
  size_t partial_cap = 0;  // doubles
  double* out_dev = nullptr;
  size_t out_cap = 0;
  double* sums_dev = nullptr;  // 4 sums, the 2 catalogs' max |w|, 3 x SUM_BLOCKS partials
  unsigned long long* det_acc = nullptr;  // deterministic mode: 64-bit paint accumulators
  double* det_scale = nullptr;            // deterministic mode: the shared fixed-point scale
  double* cat_dev = nullptr;   // staging for host catalogs
  size_t cat_cap = 0;          // doubles
  // tile sort of the particles
  int ts = 16;                 // painting tile side
  int ntiles = 0;
  int* tile_count = nullptr;   // ntiles + 1
  int* tile_off = nullptr;     // ntiles + 1
  int* tile_of = nullptr;      // per particle
  int* tile_rank = nullptr;
  void* payload = nullptr;     // 32 bytes per particle, tile order
  int* scan_sums = nullptr;    // block sums of the tile scan
  size_t sort_cap = 0;         // particles
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // state
  bool painted = false;
  double alpha = 0, norm_I = 0, shot = 0;
  int n_transforms = 0;
  std::string err;
  pkm_stats_t stats{};
  int64_t bytes = 0;
  std::unordered_map<void*, size_t> sizes;
  // bumped whenever a device buffer is allocated or freed or the request tables are rebuilt:
  // an issued or captured batch item is only valid for the generation it was added at
  uint64_t gen = 1;
  // per-launch stage timing
  bool stage_timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  size_t ev_used = 0;
};

namespace {

constexpr int SUM_BLOCKS = 1024;

struct Fail {
  pkm_status st;
};

bool is_smooth(int n) {
  if (n < 16 || n > 1024 || n % 4) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Radix schedule for length L with E elements per thread; radices must divide E.
bool make_sched(int L, int E, uint32_t* sched, int* nst) {
  static const int rad[] = {8, 6, 4, 3, 2};
  int rem = L, k = 0;
  uint32_t s = 0;
  while (rem > 1) {
    bool found = false;
    for (int r : rad) {
      if (E % r == 0 && rem % r == 0) {
        s |= (uint32_t)r << (4 * k);
        ++k;
        rem /= r;
        found = true;
        break;
      }
    }
    if (!found || k > 8) return false;
  }
  *sched = s;
  *nst = k;
  return L % E == 0;
}

int pick_e(int L) {
  if ((L & (L - 1)) == 0) return L >= 256 ? 16 : (L >= 8 ? 8 : 4);
  if (L % 12 == 0) return 12;
  if (L % 6 == 0) return 6;
  return 0;
}

void check_hip(pkm_plan* pl, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (pl) pl->err = std::string(what) + " failed: " + hipGetErrorString(e);
    throw Fail{e == hipErrorOutOfMemory ? PKM_ENOMEM : PKM_EDEVICE};
  }
}

// Stage timing: events bracket each launch when enabled; resolved after the stream syncs.
struct StageScope {
  pkm_plan* pl;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take() {
    if (pl->ev_used == pl->ev_pool.size()) {
      hipEvent_t e;
      check_hip(pl, hipEventCreate(&e), "event");
      pl->ev_pool.push_back(e);
    }
    return pl->ev_pool[pl->ev_used++];
  }
  StageScope(pkm_plan* p, int s) : pl(p), stage(s) {
    if (!pl->stage_timing) return;
    a = take();
    b = take();
    check_hip(pl, hipEventRecord(a, pl->stream), "event");
  }
  ~StageScope() {
    if (!a) return;
    if (hipEventRecord(b, pl->stream) == hipSuccess) pl->pending.push_back({stage, {a, b}});
  }
};

void resolve_stages(pkm_plan* pl) {
  for (auto& pe : pl->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      pl->stats.stage_ms[pe.first] += ms;
      pl->stats.stage_launches[pe.first] += 1;
    }
  }
  pl->pending.clear();
  pl->ev_used = 0;
}

void* dalloc(pkm_plan* pl, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* ptr = nullptr;
  if (pl->dev.alloc) {
    ptr = pl->dev.alloc(bytes, pl->dev.hip_stream, pl->dev.alloc_ctx);
    if (!ptr) {
      pl->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
      throw Fail{PKM_ENOMEM};
    }
  } else {
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      pl->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
      throw Fail{PKM_ENOMEM};
    }
  }
  pl->bytes += (int64_t)bytes;
  pl->sizes[ptr] = bytes;
  ++pl->gen;
  return ptr;
}

void dfree(pkm_plan* pl, void* ptr) {
  if (!ptr) return;
  auto it = pl->sizes.find(ptr);
  if (it != pl->sizes.end()) {
    pl->bytes -= (int64_t)it->second;
    pl->sizes.erase(it);
  }
  ++pl->gen;
  if (pl->dev.free) pl->dev.free(ptr, pl->dev.hip_stream, pl->dev.alloc_ctx);
  else (void)hipFree(ptr);
}

template <typename T> void upload_tables(pkm_plan* pl) {
  const int n = pl->p.nmesh;
  std::vector<T> tw(2 * (size_t)n), invw(n), ph(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)n;
    tw[2 * j] = (T)std::cos(a);
    tw[2 * j + 1] = (T)(-std::sin(a));
    const int f = j < n / 2 ? j : j - n;
    const double x = M_PI * (double)f / (double)n;
    double wc;
    if (pl->p.interlaced) {
      const double sinc = f == 0 ? 1.0 : std::sin(x) / x;
      wc = std::pow(sinc, pl->p.window);
    } else {
      const double s2 = std::sin(x) * std::sin(x);
      const double al = pl->p.window == 1 ? 1.0 : pl->p.window == 2 ? 1.0 - 2.0 / 3.0 * s2 : 1.0 - s2 + 2.0 / 15.0 * s2 * s2;
      wc = std::sqrt(al);
    }
    invw[j] = (T)(1.0 / wc);
    ph[2 * j] = (T)std::cos(x);
    ph[2 * j + 1] = (T)std::sin(x);
  }
  // real-harmonic recurrence coefficients, per |m|
  std::vector<T> yt((size_t)(YLM_LMAX + 1) * YLM_STRIDE, (T)0);
  for (int m = 0; m <= YLM_LMAX; ++m) {
    double q = 1.0;
    for (int j = 1; j <= m; ++j) q *= (2.0 * j - 1.0) / (2.0 * j);
    const double cmm = m == 0 ? std::sqrt(1.0 / (4.0 * M_PI)) : std::sqrt((2.0 * m + 1.0) / (2.0 * M_PI) * q);
    T* c = yt.data() + (size_t)m * YLM_STRIDE;
    c[0] = (T)cmm;
    for (int l = m + 1; l <= YLM_LMAX; ++l) {
      const int j = l - m;
      const double l2 = (double)l * l, m2 = (double)m * m;
      c[2 * j - 1] = (T)std::sqrt((4.0 * l2 - 1.0) / (l2 - m2));
      c[2 * j] = (T)(j >= 2 ? std::sqrt(((l - 1.0) * (l - 1.0) - m2) * (2.0 * l + 1.0) / ((2.0 * l - 3.0) * (l2 - m2)))
                            : 0.0);
    }
  }
  check_hip(pl, hipMemcpy(pl->tw, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice), "upload twiddles");
  check_hip(pl, hipMemcpy(pl->invw, invw.data(), invw.size() * sizeof(T), hipMemcpyHostToDevice), "upload window");
  check_hip(pl, hipMemcpy(pl->phase, ph.data(), ph.size() * sizeof(T), hipMemcpyHostToDevice), "upload phase");
  check_hip(pl, hipMemcpy(pl->ytab, yt.data(), yt.size() * sizeof(T), hipMemcpyHostToDevice), "upload ylm table");
}

// The Householder reflection that takes the mean line of sight (observer to box centre) to
// (1,1,1)/sqrt(3); the identity when they already agree or the observer is at the centre.
Frame harmonic_frame(const pkm_params& p) {
  Frame f{};
  double l[3], nl = 0.0;
  for (int a = 0; a < 3; ++a) {
    l[a] = p.box_origin[a] + 0.5 * p.box_len - p.observer[a];
    nl += l[a] * l[a];
  }
  for (int a = 0; a < 9; ++a) f.r[a] = (a % 4 == 0) ? 1.0 : 0.0;
  for (int a = 0; a < 9; ++a) f.f[a] = (float)f.r[a];
  nl = std::sqrt(nl);
  if (!(nl > 0.0)) return f;
  const double b = 1.0 / std::sqrt(3.0);
  double w[3], nw = 0.0;
  for (int a = 0; a < 3; ++a) {
    w[a] = l[a] / nl - b;
    nw += w[a] * w[a];
  }
  if (nw >= 1e-24)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) f.r[3 * i + j] -= 2.0 * w[i] * w[j] / nw;
  for (int a = 0; a < 9; ++a) f.f[a] = (float)f.r[a];
  return f;
}

// Weighted fields of a request: 2l+1 per even l >= 2 (spherical), or (p+1)(p+2)/2 monomials
// per even degree p >= 2 (Cartesian); the l = 0 / p = 0 field is C itself.
// Request kinds of ComputeCfg::basis.
constexpr int BASIS_ALL_ELL = 2;
int ell_step(int basis) { return basis == BASIS_ALL_ELL ? 1 : 2; }
// Multipole rows of a result: every l, or the even ones.
int ell_rows(int ell_max, int basis) { return basis == BASIS_ALL_ELL ? ell_max + 1 : ell_max / 2 + 1; }

int fields_for(int ell_max, int basis = 0) {
  int f = 0;
  for (int l = ell_step(basis); l <= ell_max; l += ell_step(basis)) f += basis == 1 ? (l + 1) * (l + 2) / 2 : 2 * l + 1;
  return f;
}

// Coefficients of the Legendre polynomial L_l in powers of mu: L_l = sum_p c[p] mu^p (FP64,
// exact: the denominators are powers of two), by Bonnet's recurrence.
std::vector<double> legendre_coeffs(int l) {
  std::vector<double> a(l + 1, 0.0), b(l + 1, 0.0), c(l + 1, 0.0);
  a[0] = 1.0;
  if (l == 0) return a;
  b[1] = 1.0;
  for (int k = 1; k < l; ++k) {  // (k+1) L_{k+1} = (2k+1) mu L_k - k L_{k-1}
    std::fill(c.begin(), c.end(), 0.0);
    for (int p = 0; p < l; ++p) c[p + 1] += (2.0 * k + 1.0) * b[p];
    for (int p = 0; p <= l; ++p) c[p] = (c[p] - k * a[p]) / (k + 1.0);
    a = b;
    b = c;
  }
  return b;
}

// Bytes of one kz-major field buffer [kz][x][y]: n/2 kz planes of n n + fpad complex values.
size_t field_bytes(const pkm_plan* pl) {
  return pl->mesh_bytes + (size_t)(pl->p.nmesh / 2) * pl->fs.fpad * 2 * pl->es;
}

void ensure_fields(pkm_plan* pl, int want) {
  while ((int)pl->fields.size() < want) pl->fields.push_back(dalloc(pl, field_bytes(pl)));
  const int need_ptr = (int)pl->fields.size() + 8;
  if (pl->ptr_cap < need_ptr) {
    dfree(pl, pl->ptrs_dev);
    pl->ptrs_dev = (void**)dalloc(pl, sizeof(void*) * need_ptr);
    pl->ptr_cap = need_ptr;
  }
  std::vector<void*> host(pl->ptr_cap, nullptr);
  for (size_t i = 0; i < pl->fields.size(); ++i) host[i] = pl->fields[i];
  check_hip(pl, hipMemcpy(pl->ptrs_dev, host.data(), sizeof(void*) * pl->ptr_cap, hipMemcpyHostToDevice),
            "upload field pointers");
}

// Device array [ptr_cap-8 .. ) holds ad-hoc pointers for single-buffer passes.
void** scratch_ptrs(pkm_plan* pl, std::initializer_list<void*> ps) {
  std::vector<void*> host(ps);
  void** dst = pl->ptrs_dev + (pl->ptr_cap - 8);
  check_hip(pl, hipMemcpy(dst, host.data(), sizeof(void*) * host.size(), hipMemcpyHostToDevice), "upload pointers");
  return dst;
}

// ------------------------------------------------------------------------------------------
// Estimate, split into a host-side preparation and a device-only enqueue.  The enqueue
// functions allocate nothing and never wait on the device, so they may be recorded into a
// HIP graph or overlap with other plans' work on other streams.
// ------------------------------------------------------------------------------------------

// Device catalog pointers and counts of one estimate.
struct DevCats {
  const double *dp = nullptr, *dw = nullptr, *dn = nullptr;
  const double *rp = nullptr, *rw = nullptr, *rn = nullptr;
  int64_t nd = 0, nr = 0;
};

// Copy host catalogs into the plan's staging buffer (device catalogs pass through).
DevCats stage_catalogs(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* rand) {
  hipStream_t s = pl->stream;
  size_t need = 0;
  for (const pkm_catalog* cat : {data, rand})
    if (cat && !cat->on_device) need += (size_t)cat->n * 3 + (cat->w ? cat->n : 0) + (cat->nbar ? cat->n : 0);
  if (need > pl->cat_cap) {
    dfree(pl, pl->cat_dev);
    pl->cat_dev = nullptr;
    pl->cat_cap = 0;
    pl->cat_dev = (double*)dalloc(pl, need * sizeof(double));
    pl->cat_cap = need;
  }
  size_t offset = 0;
  auto one = [&](const pkm_catalog* cat, const double** pos, const double** w, const double** nbar) {
    if (cat->on_device) {
      *pos = cat->pos;
      *w = cat->w;
      *nbar = cat->nbar;
      return;
    }
    const size_t nn = (size_t)cat->n;
    auto up = [&](const double* src, size_t count, const char* what) {
      double* dst = pl->cat_dev + offset;
      check_hip(pl, hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyHostToDevice, s), what);
      offset += count;
      return (const double*)dst;
    };
    *pos = up(cat->pos, nn * 3, "upload pos");
    *w = cat->w ? up(cat->w, nn, "upload w") : nullptr;
    *nbar = cat->nbar ? up(cat->nbar, nn, "upload nbar") : nullptr;
  };
  DevCats dc;
  one(data, &dc.dp, &dc.dw, &dc.dn);
  dc.nd = data->n;
  if (rand) {
    one(rand, &dc.rp, &dc.rw, &dc.rn);
    dc.nr = rand->n;
  }
  return dc;
}

void reserve_particles(pkm_plan* pl, int64_t ntot) {
  if ((size_t)ntot <= pl->sort_cap) return;
  for (int** b : {&pl->tile_of, &pl->tile_rank}) {
    dfree(pl, *b);
    *b = nullptr;
  }
  dfree(pl, pl->payload);
  pl->payload = nullptr;
  pl->sort_cap = 0;
  pl->tile_of = (int*)dalloc(pl, sizeof(int) * ntot);
  pl->tile_rank = (int*)dalloc(pl, sizeof(int) * ntot);
  pl->payload = dalloc(pl, 32 * (size_t)ntot);
  pl->sort_cap = (size_t)ntot;
}

// alpha = N_d / N_r (unweighted counts); 0 for a periodic box.
double alpha_of(int64_t nd, int64_t nr) { return nr > 0 ? (double)nd / (double)nr : 0.0; }

// I and S from the catalog sums {sum_d w^2, -, sum_r w^2, sum_r w^2 nbar}.
void scalars_of(const pkm_plan* pl, const double* sums, int64_t nd, int64_t nr, double* alpha, double* norm_I,
                double* shot) {
  const double sd2 = sums[0];
  *alpha = alpha_of(nd, nr);
  if (nr > 0) {
    *norm_I = *alpha * sums[3];
    *shot = (sd2 + *alpha * *alpha * sums[2]) / *norm_I;
  } else {
    const double L = pl->p.box_len;
    const double nbar = (double)nd / (L * L * L);
    *norm_I = nbar * sd2;
    *shot = sd2 / *norm_I;
  }
}

// The estimator divides by I (Sec. 2.1, eq. FKP-density): it has no value when I is not positive, as when every
// random weight (or n-bar), or in a periodic box every data weight, is zero.
bool norm_ok(double norm_I) { return norm_I > 0.0 && std::isfinite(norm_I); }
const char* const ZERO_NORM = "normalisation I is not positive (the weights or n-bar of the randoms, or the "
                              "weights of the data in a periodic box, sum to zero)";

// Catalog sums, painting, forward transforms, combine and inverse of the combined field.
// Leaves the sums in sums_dev[0..3], C and G resident.  Needs sort capacity >= nd + nr.
template <typename T> void enqueue_paint(pkm_plan* pl, const DevCats& dc) {
  hipStream_t s = pl->stream;
  const int n = pl->p.nmesh;
  const size_t cells = (size_t)n * n * n;
  const bool has_r = dc.nr > 0;
  {
    StageScope ss(pl, PKM_STAGE_SUMS);
    // sums_dev: [0..3] the sums of both catalogs, [4], [5] their largest |w|, then partials
    check_hip(pl, launch_catalog_sums(dc.dw, nullptr, dc.nd, pl->sums_dev + 6, SUM_BLOCKS, pl->sums_dev,
                                      pl->sums_dev + 4, s),
              "sums");
    if (has_r)
      check_hip(pl, launch_catalog_sums(dc.rw, dc.rn, dc.nr, pl->sums_dev + 6, SUM_BLOCKS, pl->sums_dev + 2,
                                        pl->sums_dev + 5, s),
                "sums");
  }
  T* d1 = (T*)pl->d1;
  T* d2 = pl->p.interlaced ? (T*)pl->d2 : nullptr;
  const double scale = (double)n / pl->p.box_len;
  const int64_t ntot = dc.nd + dc.nr;
  if ((size_t)ntot > pl->sort_cap) {
    pl->err = "particle count above the plan's reserved capacity";
    throw Fail{PKM_EINVAL};
  }
  const double alpha = alpha_of(dc.nd, dc.nr);
  const bool det = pl->p.deterministic != 0;
  {
    StageScope ss(pl, PKM_STAGE_FILL);
    check_hip(pl, launch_fill<int>(pl->tile_count, (size_t)TILE_COUNT_COPIES * (pl->ntiles + 1), 0, s), "fill");
    if (det) {
      check_hip(pl, launch_fill<unsigned long long>(pl->det_acc, cells * (d2 ? 2 : 1), 0ull, s), "fill");
    } else {
      check_hip(pl, launch_fill<T>(d1, cells, T(0), s), "fill");
      if (d2) check_hip(pl, launch_fill<T>(d2, cells, T(0), s), "fill");
    }
  }
  {
    StageScope ss(pl, PKM_STAGE_PAINT);
    check_hip(pl, launch_tile_sort(dc.dp, dc.nd, 0, pl->p.box_origin, scale, n, pl->ts, pl->tile_count, pl->tile_of,
                                   pl->tile_rank, s),
              "tile sort");
    if (has_r)
      check_hip(pl, launch_tile_sort(dc.rp, dc.nr, dc.nd, pl->p.box_origin, scale, n, pl->ts, pl->tile_count,
                                     pl->tile_of, pl->tile_rank, s),
                "tile sort");
    check_hip(pl, launch_tile_offsets(pl->tile_count, pl->ntiles, pl->tile_off, pl->tile_of, pl->tile_rank, dc.nd,
                                      ntot, dc.dp, dc.dw, dc.rp, dc.rw, alpha, pl->payload, pl->scan_sums, s),
              "tile offsets");
    check_hip(pl, launch_paint_tiles<T>(pl->tile_off, pl->payload, pl->ntiles, pl->p.box_origin, scale, n,
                                        pl->p.window, pl->ts, d1, d2, pl->sums_dev + 4,
                                        has_r ? pl->sums_dev + 5 : nullptr, alpha, s,
                                        det ? pl->det_acc : nullptr, det ? pl->det_scale : nullptr),
              "paint");
    if (det) check_hip(pl, launch_det_convert<T>(pl->det_acc, d1, d2, n, pl->det_scale, s), "paint convert");
  }
  const int nbuf = d2 ? 2 : 1;
  void** sp = pl->paint_ptrs;  // {s1, s2, g}
  {
    StageScope ss(pl, PKM_STAGE_ZFWD);
    check_hip(pl, launch_zfwd<T>(pl->fs, d1, d2, pl->s1, pl->s2, nbuf, pl->tw, s), "zfwd");
  }
  {
    StageScope ss(pl, PKM_STAGE_YCOL);
    check_hip(pl, launch_col<T>(pl->fs, sp, nbuf, 1, false, pl->tw, s), "y pass");
  }
  const bool need_dc = pl->p.interlaced || pl->p.compensated;
  {
    StageScope ss(pl, PKM_STAGE_XCOMBINE);
    check_hip(pl, launch_xcombine<T>(pl->fs, pl->s1, pl->s2, pl->c, need_dc ? pl->g : nullptr, pl->p.interlaced,
                                     pl->p.compensated, pl->invw, pl->phase, pl->tw, s),
              "x combine");
  }
  if (need_dc) {
    StageScope ss(pl, PKM_STAGE_IYCOL);
    check_hip(pl, launch_col<T>(pl->fs, sp + 2, 1, 1, true, pl->tw, s), "inverse y pass");
  }
}

template <typename T> void run_paint(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* rand) {
  hipStream_t s = pl->stream;
  DevCats dc = stage_catalogs(pl, data, rand);
  reserve_particles(pl, dc.nd + dc.nr);
  check_hip(pl, hipEventRecord(pl->ev0, s), "event");
  enqueue_paint<T>(pl, dc);
  double sums[4] = {0, 0, 0, 0};
  check_hip(pl, hipMemcpyAsync(sums, pl->sums_dev, sizeof sums, hipMemcpyDeviceToHost, s), "download sums");
  check_hip(pl, hipEventRecord(pl->ev1, s), "event");
  check_hip(pl, hipStreamSynchronize(s), "sync");
  scalars_of(pl, sums, dc.nd, dc.nr, &pl->alpha, &pl->norm_I, &pl->shot);
  if (!norm_ok(pl->norm_I)) {
    pl->err = ZERO_NORM;
    throw Fail{PKM_EINVAL};
  }
  resolve_stages(pl);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, pl->ev0, pl->ev1);
  pl->stats.ms_paint = ms;
  const double R = (double)pl->mesh_bytes;
  const int nbuf = pl->p.interlaced ? 2 : 1;
  const bool need_dc = pl->p.interlaced || pl->p.compensated;
  const double cat_bytes = 40.0 * (double)(dc.nd + dc.nr);
  pl->stats.model_bytes_paint = cat_bytes + nbuf * (2 * R) /*zero + scatter*/ + nbuf * (2 * R) /*z*/ +
                                nbuf * (2 * R) /*y*/ + nbuf * R + 2 * R /*x combine*/ + (need_dc ? 2 * R : 0);
  pl->painted = true;
}

// Host tables of a multipole request (thresholds, field groups, reduce maps, partial sums),
// cached until ell_max or the edges change.
template <typename T>
void prepare_compute(pkm_plan* pl, int ell_max, const double* k_edges, int n_edges, int basis = 0) {
  ComputeCfg& cc = pl->cc;
  if (cc.ell_max == ell_max && cc.basis == basis && cc.edges.size() == (size_t)n_edges &&
      std::equal(cc.edges.begin(), cc.edges.end(), k_edges))
    return;
  cc = ComputeCfg{};
  ++pl->gen;
  const int n = pl->p.nmesh;
  const int nb = n_edges - 1;
  {
    const int need = fields_for(ell_max, basis);
    if ((int)pl->fields.size() < need && (pl->p.max_group <= 0 || (int)pl->fields.size() < pl->p.max_group))
      ensure_fields(pl, pl->p.max_group > 0 ? std::min(need, pl->p.max_group) : need);
  }
  // integer thresholds T_i = ceil(((e_i * L) / (2 pi))^2)
  std::vector<long long> thr(n_edges);
  const double twopi = 2.0 * M_PI;
  for (int i = 0; i < n_edges; ++i) {
    const double t = (k_edges[i] * pl->p.box_len) / twopi;
    const double t2 = t * t;
    thr[i] = t2 >= 9.0e18 ? (long long)9.0e18 : (long long)std::ceil(t2);
  }
  if (pl->thr_cap < n_edges) {
    dfree(pl, pl->thr_dev);
    pl->thr_dev = (long long*)dalloc(pl, sizeof(long long) * n_edges);
    pl->thr_cap = n_edges;
  }
  check_hip(pl, hipMemcpy(pl->thr_dev, thr.data(), sizeof(long long) * n_edges, hipMemcpyHostToDevice), "thr");
  // fields and groups
  struct F { int l, m, slot; };
  std::vector<std::vector<F>> groups;
  const int fmax = (int)pl->fields.size();
  {
    // fields ordered by l (or degree p); a group holds at most fmax fields (any number of
    // multipoles).  Cartesian fields carry (p, 32 i + j) for the monomial x^i y^j z^(p-i-j).
    std::vector<F> cur;
    int nl = 0, last_l = -1;
    auto add = [&](int l, int m) {
      if ((int)cur.size() == fmax) {
        groups.push_back(cur);
        cur.clear();
        nl = 0;
        last_l = -1;
      }
      if (l != last_l) { ++nl; last_l = l; }
      cur.push_back({l, m, nl - 1});
    };
    for (int l = ell_step(basis); l <= ell_max; l += ell_step(basis)) {
      if (basis == 1) {
        for (int i = 0; i <= l; ++i)
          for (int j = 0; i + j <= l; ++j) add(l, 32 * i + j);
      } else {
        for (int m = -l; m <= l; ++m) add(l, m);
      }
    }
    if (!cur.empty()) groups.push_back(cur);
    if (groups.empty()) groups.push_back({});  // l = 0 only
  }
  const int rows = 2 + ell_rows(ell_max, basis);  // count, ksum, Q0, then Q2, Q4, ... (or Q1, Q2, ...)
  const size_t col_lds = xpost_base_bytes(pl->fs, sizeof(T) == 8) + sizeof(long long) * (size_t)n_edges;
  if (col_lds + sizeof(double) * 5 * (size_t)nb > 160 * 1024) {
    pl->err = "too many k bins for one pass";
    throw Fail{PKM_EINVAL};
  }
  const int total_vals = rows * nb;
  if (pl->out_cap < (size_t)total_vals) {
    dfree(pl, pl->out_dev);
    pl->out_dev = (double*)dalloc(pl, sizeof(double) * total_vals);
    pl->out_cap = total_vals;
  }
  // Per group two field tables of (buffer, l, m, slot): the pre-pass walks the fields
  // |m|-major (|m| ascending, then l, +m before -m) so the harmonic recurrence of one field
  // continues from the previous one; the post-pass walks them l-major (slots contiguous),
  // |m| ascending with +m before -m.  Buffer b of a group holds its b-th field (l-major).
  std::vector<int> ftab, maps;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const auto& g = groups[gi];
    std::vector<int> idx(g.size());
    for (size_t i = 0; i < g.size(); ++i) idx[i] = (int)i;
    auto key_pre = [&](int i) {
      return basis == 1 ? std::make_tuple(g[i].l, g[i].m, false) : std::make_tuple(std::abs(g[i].m), g[i].l, g[i].m < 0);
    };
    auto key_post = [&](int i) { return std::make_tuple(g[i].slot, std::abs(g[i].m), g[i].m < 0); };
    std::vector<int> pre = idx, post = idx;
    std::stable_sort(pre.begin(), pre.end(), [&](int a, int b) { return key_pre(a) < key_pre(b); });
    std::stable_sort(post.begin(), post.end(), [&](int a, int b) { return key_post(a) < key_post(b); });
    GroupCfg gc;
    gc.nf = (int)g.size();
    gc.fofs = (int)ftab.size() / 4;
    for (int i : pre) { ftab.push_back(i); ftab.push_back(g[i].l); ftab.push_back(g[i].m); ftab.push_back(g[i].slot); }
    gc.pofs = (int)ftab.size() / 4;
    for (int i : post) { ftab.push_back(i); ftab.push_back(g[i].l); ftab.push_back(g[i].m); ftab.push_back(g[i].slot); }
    std::vector<int> slot_l;
    for (auto& f : g) if ((int)slot_l.size() <= f.slot) slot_l.push_back(f.l);
    const bool first = gi == 0;
    gc.mofs = (int)maps.size();
    int nv = 0;
    if (first) for (int r = 0; r < 3; ++r) for (int b = 0; b < nb; ++b) { maps.push_back(r * nb + b); ++nv; }
    for (size_t si = 0; si < slot_l.size(); ++si)
      for (int b = 0; b < nb; ++b) { maps.push_back((2 + slot_l[si] / ell_step(basis)) * nb + b); ++nv; }
    gc.nv = nv;
    gc.nslots = (int)slot_l.size();
    cc.groups.push_back(gc);
    cc.nfields_total += gc.nf;
  }
  if (pl->ftab_cap < (int)ftab.size() + 4) {
    dfree(pl, pl->ftab_dev);
    pl->ftab_dev = (int*)dalloc(pl, sizeof(int) * (ftab.size() + 4));
    pl->ftab_cap = (int)ftab.size() + 4;
  }
  if (!ftab.empty())
    check_hip(pl, hipMemcpy(pl->ftab_dev, ftab.data(), sizeof(int) * ftab.size(), hipMemcpyHostToDevice), "ftab");
  if (pl->map_cap < (int)maps.size()) {
    dfree(pl, pl->map_dev);
    pl->map_dev = (int*)dalloc(pl, sizeof(int) * maps.size());
    pl->map_cap = (int)maps.size();
  }
  check_hip(pl, hipMemcpy(pl->map_dev, maps.data(), sizeof(int) * maps.size(), hipMemcpyHostToDevice), "maps");
  const int nblk = post_blocks(pl->fs);
  int max_nv = 0;
  for (auto& gc : cc.groups) max_nv = std::max(max_nv, gc.nv);
  if (pl->partial_cap < (size_t)nblk * max_nv) {
    dfree(pl, pl->partial);
    pl->partial = (double*)dalloc(pl, sizeof(double) * (size_t)nblk * max_nv);
    pl->partial_cap = (size_t)nblk * max_nv;
  }
  // histogram copies per block: one per wave when the LDS budget of two post-pass blocks per
  // CU allows (the register budget allows no more than two)
  // (deterministic mode: one per wave always, within the LDS of one block per CU, so that no
  // two waves add to the same bin)
  const int waves = ((n / pl->fs.e_post) * pl->fs.tile_post + 63) / 64;
  const size_t lds_cap = pl->p.deterministic ? 150 * 1024 : 80 * 1024;
  const size_t budget = col_lds + 1024 < lds_cap ? lds_cap - col_lds - 1024 : 0;
  for (auto& gc : cc.groups) {
    const int copies = (int)std::min<size_t>((size_t)waves, budget / (sizeof(double) * (size_t)std::max(1, gc.nv)));
    gc.copies = std::max(1, copies);
    if (pl->p.deterministic && gc.copies < waves) {
      pl->err = "deterministic mode: one post-pass histogram per wavefront does not fit LDS for these bins";
      throw Fail{PKM_ENOMEM};
    }
  }
  cc.ell_max = ell_max;
  cc.basis = basis;
  cc.nb = nb;
  cc.total_vals = total_vals;
  cc.edges.assign(k_edges, k_edges + n_edges);
}

// Every group's pre-pass, y pass, post-pass and reduction into out_dev (zeroed first).
template <typename T> void enqueue_compute(pkm_plan* pl) {
  hipStream_t s = pl->stream;
  const ComputeCfg& cc = pl->cc;
  const int n = pl->p.nmesh;
  check_hip(pl, launch_fill<double>(pl->out_dev, cc.total_vals, 0.0, s), "zero out");
  const bool dc_real = !(pl->p.interlaced || pl->p.compensated);
  const double off[3] = {pl->p.box_origin[0] - pl->p.observer[0], pl->p.box_origin[1] - pl->p.observer[1],
                         pl->p.box_origin[2] - pl->p.observer[2]};
  const double h = pl->p.box_len / n;
  const double dc_scale = 2.0 / ((double)n * n * n);
  for (size_t gi = 0; gi < cc.groups.size(); ++gi) {
    const GroupCfg& gc = cc.groups[gi];
    const int* ft = pl->ftab_dev + 4 * gc.fofs;
    const int* ftp = pl->ftab_dev + 4 * gc.pofs;
    if (gc.nf > 0) {
      {
        StageScope ss(pl, PKM_STAGE_ZPRE);
        check_hip(pl, launch_zpre<T>(pl->fs, pl->g, dc_real ? (const T*)pl->d1 : nullptr, nullptr, pl->ptrs_dev,
                                     gc.nf, ft, dc_scale, off, h, pl->ytab, pl->tw, pl->frame, cc.basis, s),
                  "zpre");
      }
      // kz-major fields: the column pass runs along x within each kz plane, the post-pass
      // along the contiguous y lines
      StageScope ss(pl, PKM_STAGE_YCOL);
      check_hip(pl, launch_col<T>(pl->fs, pl->ptrs_dev, gc.nf, 0, false, pl->tw, s, true), "field column pass");
    }
    int nblocks = 0;
    {
      StageScope ss(pl, PKM_STAGE_XPOST);
      check_hip(pl, launch_xpost<T>(pl->fs, pl->ptrs_dev, gc.nf, ftp, gc.nslots, gi == 0 ? 1 : 0, pl->c, pl->ytab,
                                    BinSpec{pl->thr_dev, cc.nb, gc.copies}, (double)(2.0 * M_PI / pl->p.box_len),
                                    pl->partial, &nblocks, pl->tw, pl->frame, cc.basis, s),
                "post-pass");
    }
    StageScope ss(pl, PKM_STAGE_REDUCE);
    check_hip(pl, launch_reduce(pl->partial, nblocks, gc.nv, pl->out_dev, pl->map_dev + gc.mofs, 1, s), "reduce");
  }
}

// P_l, k_mean and mode counts from the reduced bin sums (FP64, host).
void normalize(const pkm_plan* pl, const double* res, double norm_I, double shot, pkm_result* out) {
  const ComputeCfg& cc = pl->cc;
  const int nb = cc.nb;
  for (int b = 0; b < nb; ++b) {
    const double cnt = res[b];
    if (out->n_modes) out->n_modes[b] = (int64_t)llround(cnt);
    if (out->k_mean) out->k_mean[b] = cnt > 0 ? res[nb + b] / cnt : NAN;
    if (out->poles) {
      for (int il = 0; il < ell_rows(cc.ell_max, cc.basis); ++il) {
        double q = res[(2 + il) * nb + b];
        if (cc.basis == 1) {
          // Cartesian rows hold R_p = sum Re[C conj M_p], M_p the transform of D_c (khat.xhat)^p
          // (R_0 = sum |C|^2); P_l takes (2l+1) sum_p c_lp R_p with L_l = sum_p c_lp mu^p
          const std::vector<double> c = legendre_coeffs(2 * il);
          q = 0.0;
          for (int p = 0; p <= 2 * il; p += 2) q += c[p] * res[(2 + p / 2) * nb + b];
          q *= 4.0 * il + 1.0;
        }
        double v = cnt > 0 ? q / (norm_I * cnt) : NAN;
        if (il == 0) v -= shot;
        out->poles[(size_t)il * nb + b] = v;
      }
    }
  }
  const int n_fwd = pl->p.interlaced ? 2 : 1;
  const int n_inv = (pl->p.interlaced || pl->p.compensated) ? 1 : 0;
  out->n_transforms = cc.nfields_total + n_fwd + n_inv;
}

template <typename T>
void run_compute(pkm_plan* pl, int ell_max, const double* k_edges, int n_edges, int basis, pkm_result* out) {
  hipStream_t s = pl->stream;
  prepare_compute<T>(pl, ell_max, k_edges, n_edges, basis);
  const ComputeCfg& cc = pl->cc;
  check_hip(pl, hipEventRecord(pl->ev0, s), "event");
  enqueue_compute<T>(pl);
  check_hip(pl, hipEventRecord(pl->ev1, s), "event");
  std::vector<double> res(cc.total_vals);
  check_hip(pl, hipMemcpyAsync(res.data(), pl->out_dev, sizeof(double) * cc.total_vals, hipMemcpyDeviceToHost, s),
            "download");
  check_hip(pl, hipStreamSynchronize(s), "sync");
  resolve_stages(pl);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, pl->ev0, pl->ev1);
  pl->stats.ms_compute = ms;
  pl->stats.n_groups = (int)cc.groups.size();
  const double X = (double)pl->mesh_bytes;
  pl->stats.model_bytes_compute = 0;
  for (const GroupCfg& gc : cc.groups) {
    const double nf = (double)gc.nf;
    pl->stats.model_bytes_compute += (nf > 0 ? X + nf * X : 0) + 2 * nf * X + nf * X + X;
  }
  normalize(pl, res.data(), pl->norm_I, pl->shot, out);
  out->alpha = pl->alpha;
  out->norm_I = pl->norm_I;
  out->shot_noise = pl->shot;
  pl->n_transforms = out->n_transforms;
  pl->stats.n_transforms = pl->n_transforms;
}

// Whole estimate (paint + multipoles) on device catalogs, results copied to a pinned host
// slot of (4 + total_vals) doubles: the catalog sums, then the reduced bin sums.  Requires
// prepare_compute and reserve_particles beforehand; allocates nothing and does not wait.
template <typename T> void enqueue_estimate(pkm_plan* pl, const DevCats& dc, double* slot) {
  hipStream_t s = pl->stream;
  enqueue_paint<T>(pl, dc);
  enqueue_compute<T>(pl);
  check_hip(pl, hipMemcpyAsync(slot, pl->sums_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "download sums");
  check_hip(pl, hipMemcpyAsync(slot + 4, pl->out_dev, sizeof(double) * pl->cc.total_vals, hipMemcpyDeviceToHost, s),
            "download bins");
}

// Multipoles of the painted field the plan already holds (its last paint or estimate), for the
// prepared request, with that paint's catalog sums copied again: the same slot layout as
// enqueue_estimate.  Allocates nothing and does not wait.
template <typename T> void enqueue_compute_copy(pkm_plan* pl, double* slot) {
  hipStream_t s = pl->stream;
  enqueue_compute<T>(pl);
  check_hip(pl, hipMemcpyAsync(slot, pl->sums_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "download sums");
  check_hip(pl, hipMemcpyAsync(slot + 4, pl->out_dev, sizeof(double) * pl->cc.total_vals, hipMemcpyDeviceToHost, s),
            "download bins");
}

// PKM_EINVAL, with `out` untouched, when the normalisation has no value.
pkm_status finish_from_slot(const pkm_plan* pl, const double* slot, int64_t nd, int64_t nr, pkm_result* out) {
  double alpha, norm_I, shot;
  scalars_of(pl, slot, nd, nr, &alpha, &norm_I, &shot);
  if (!norm_ok(norm_I)) return PKM_EINVAL;
  normalize(pl, slot + 4, norm_I, shot, out);
  out->alpha = alpha;
  out->norm_I = norm_I;
  out->shot_noise = shot;
  return PKM_OK;
}

// (k, mu) cells of one request: (n_k_edges - 1) (n_mu_edges - 1) <= this, the limit of the
// binning kernel's LDS histogram (two doubles per cell in 48 KB)
constexpr int KMU_MAX_CELLS = 3072;

template <typename T>
void run_kmu(pkm_plan* pl, const double* k_edges, int nke, const double* mu_edges, int nme, double* pk, int64_t* nm) {
  hipStream_t s = pl->stream;
  const int nb = nke - 1, nmu = nme - 1;
  std::vector<long long> thr(nke);
  for (int i = 0; i < nke; ++i) {
    const double t = (k_edges[i] * pl->p.box_len) / (2.0 * M_PI);
    const double t2 = t * t;
    thr[i] = t2 >= 9.0e18 ? (long long)9.0e18 : (long long)std::ceil(t2);
  }
  const int nvals = 2 * nb * nmu;
  const int nblk = 1024;
  long long* thr_d = (long long*)dalloc(pl, sizeof(long long) * nke);
  double* mue_d = (double*)dalloc(pl, sizeof(double) * nme);
  double* part = (double*)dalloc(pl, sizeof(double) * (size_t)nblk * nvals);
  double* outd = (double*)dalloc(pl, sizeof(double) * nvals);
  try {
    check_hip(pl, hipMemcpy(thr_d, thr.data(), sizeof(long long) * nke, hipMemcpyHostToDevice), "thr");
    check_hip(pl, hipMemcpy(mue_d, mu_edges, sizeof(double) * nme, hipMemcpyHostToDevice), "mu edges");
    double l[3] = {pl->p.los[0], pl->p.los[1], pl->p.los[2]};
    const double ln = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    for (double& v : l) v /= ln;
    check_hip(pl, launch_kmu<T>(pl->fs, pl->c, l, BinSpec{thr_d, nb, 1}, mue_d, nmu, part, nblk, s), "kmu");
    check_hip(pl, launch_reduce(part, nblk, nvals, outd, nullptr, 0, s), "reduce");
    std::vector<double> res(nvals);
    check_hip(pl, hipMemcpy(res.data(), outd, sizeof(double) * nvals, hipMemcpyDeviceToHost), "download");
    for (int i = 0; i < nb * nmu; ++i) {
      const double cnt = res[2 * i];
      if (nm) nm[i] = (int64_t)llround(cnt);
      if (pk) pk[i] = cnt > 0 ? res[2 * i + 1] / (pl->norm_I * cnt) - pl->shot : NAN;
    }
  } catch (...) {
    dfree(pl, thr_d); dfree(pl, mue_d); dfree(pl, part); dfree(pl, outd);
    throw;
  }
  dfree(pl, thr_d); dfree(pl, mue_d); dfree(pl, part); dfree(pl, outd);
}

// ------------------------------------------------------------------------------------------
// Allocation-free (k, mu) binning.  Its thresholds, mu edges, per-block partial sums, reduced
// sums and normalised outputs live in one file-scope device array, `scratch`, sized for the
// largest request the (k, mu) kernel takes (KMU_MAX_CELLS cells, the limit of its LDS
// histogram).  Each device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for the current device.
// ------------------------------------------------------------------------------------------
constexpr int KMU_NOALLOC_BLOCKS = 256;    // k_kmu grid of the allocation-free path
constexpr size_t kmu_align(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t KMU_OFF_THR = 0;
constexpr size_t KMU_OFF_MU = KMU_OFF_THR + kmu_align(sizeof(long long) * (KMU_MAX_CELLS + 1));
constexpr size_t KMU_OFF_PART = KMU_OFF_MU + kmu_align(sizeof(double) * (KMU_MAX_CELLS + 1));
constexpr size_t KMU_OFF_SUMS = KMU_OFF_PART + kmu_align(sizeof(double) * 2 * (size_t)KMU_MAX_CELLS * KMU_NOALLOC_BLOCKS);
constexpr size_t KMU_OFF_PK = KMU_OFF_SUMS + kmu_align(sizeof(double) * 2 * KMU_MAX_CELLS);
constexpr size_t KMU_OFF_NM = KMU_OFF_PK + kmu_align(sizeof(double) * KMU_MAX_CELLS);
constexpr size_t KMU_SCRATCH_BYTES = KMU_OFF_NM + kmu_align(sizeof(long long) * KMU_MAX_CELLS);  // 12.7 MB

static __device__ __align__(256) unsigned char scratch[KMU_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the plan's device (current: the entry point set it), looked
// up once per device.
unsigned char* scratch_of(pkm_plan* pl) {
  const int dev = pl->dev.device_id;
  if (dev < 0 || dev >= MAX_DEVICES) {
    pl->err = "device id out of range";
    throw Fail{PKM_EINVAL};
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      pl->err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      throw Fail{PKM_EDEVICE};
    }
    g_scratch_ptr[dev] = (unsigned char*)ptr;
  }
  return g_scratch_ptr[dev];
}

template <typename T>
void run_kmu_noalloc(pkm_plan* pl, const double* k_edges, int nke, const double* mu_edges, int nme, double* pk,
                     int64_t* nm) {
  hipStream_t s = pl->stream;
  const int nb = nke - 1, nmu = nme - 1, ncells = nb * nmu;
  unsigned char* base = scratch_of(pl);
  long long* thr_d = (long long*)(base + KMU_OFF_THR);
  double* mue_d = (double*)(base + KMU_OFF_MU);
  double* part = (double*)(base + KMU_OFF_PART);
  double* sums = (double*)(base + KMU_OFF_SUMS);
  double* pk_d = (double*)(base + KMU_OFF_PK);
  long long* nm_d = (long long*)(base + KMU_OFF_NM);
  long long thr[KMU_MAX_CELLS + 1];  // host stack: the same thresholds as the allocating path
  for (int i = 0; i < nke; ++i) {
    const double t = (k_edges[i] * pl->p.box_len) / (2.0 * M_PI);
    const double t2 = t * t;
    thr[i] = t2 >= 9.0e18 ? (long long)9.0e18 : (long long)std::ceil(t2);
  }
  check_hip(pl, hipMemcpyAsync(thr_d, thr, sizeof(long long) * nke, hipMemcpyHostToDevice, s), "thr");
  check_hip(pl, hipMemcpyAsync(mue_d, mu_edges, sizeof(double) * nme, hipMemcpyHostToDevice, s), "mu edges");
  double l[3] = {pl->p.los[0], pl->p.los[1], pl->p.los[2]};
  const double ln = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
  for (double& v : l) v /= ln;
  // every block writes all 2 ncells of its partial row, the reduction and the normalisation
  // write every cell: nothing of an earlier call is read
  check_hip(pl, launch_kmu<T>(pl->fs, pl->c, l, BinSpec{thr_d, nb, 1}, mue_d, nmu, part, KMU_NOALLOC_BLOCKS, s),
            "kmu");
  check_hip(pl, launch_reduce(part, KMU_NOALLOC_BLOCKS, 2 * ncells, sums, nullptr, 0, s), "reduce");
  check_hip(pl, launch_kmu_finish(sums, ncells, pl->norm_I, pl->shot, pk_d, nm_d, s), "kmu finish");
  if (pk) check_hip(pl, hipMemcpyAsync(pk, pk_d, sizeof(double) * ncells, hipMemcpyDeviceToHost, s), "download");
  if (nm) check_hip(pl, hipMemcpyAsync(nm, nm_d, sizeof(long long) * ncells, hipMemcpyDeviceToHost, s), "download");
  check_hip(pl, hipStreamSynchronize(s), "sync");
}

template <typename T> void run_fft_forward(pkm_plan* pl, const void* in, void* out) {
  hipStream_t s = pl->stream;
  check_hip(pl, launch_zfwd<T>(pl->fs, (const T*)in, nullptr, out, nullptr, 1, pl->tw, s), "zfwd");
  void** sp = scratch_ptrs(pl, {out});
  check_hip(pl, launch_col<T>(pl->fs, sp, 1, 1, false, pl->tw, s), "y pass");
  check_hip(pl, launch_col<T>(pl->fs, sp, 1, 0, false, pl->tw, s), "x pass");
  check_hip(pl, hipStreamSynchronize(s), "sync");
}

template <typename T> void run_fft_inverse(pkm_plan* pl, void* in, void* out) {
  hipStream_t s = pl->stream;
  void** sp = scratch_ptrs(pl, {in});
  check_hip(pl, launch_col<T>(pl->fs, sp, 1, 0, true, pl->tw, s), "x pass");
  check_hip(pl, launch_col<T>(pl->fs, sp, 1, 1, true, pl->tw, s), "y pass");
  const double off[3] = {0, 0, 0};
  const int n = pl->p.nmesh;
  check_hip(pl, launch_zpre<T>(pl->fs, in, nullptr, (T*)out, pl->ptrs_dev, 0, pl->ftab_dev, 2.0 / ((double)n * n * n),
                               off, 1.0, pl->ytab, pl->tw, pl->frame, 0, s),
            "z inverse");
  check_hip(pl, hipStreamSynchronize(s), "sync");
}

template <typename T> void read_dc(pkm_plan* pl, void* host, size_t bytes) {
  hipStream_t s = pl->stream;
  if (!(pl->p.interlaced || pl->p.compensated)) {
    check_hip(pl, hipMemcpy(host, pl->d1, bytes, hipMemcpyDeviceToHost), "read d1");
    return;
  }
  void* tmp = dalloc(pl, pl->mesh_bytes);
  const double off[3] = {0, 0, 0};
  const int n = pl->p.nmesh;
  hipError_t e = launch_zpre<T>(pl->fs, pl->g, nullptr, (T*)tmp, pl->ptrs_dev, 0, pl->ftab_dev,
                                2.0 / ((double)n * n * n), off, 1.0, pl->ytab, pl->tw, pl->frame, 0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(host, tmp, bytes, hipMemcpyDeviceToHost);
  dfree(pl, tmp);
  check_hip(pl, e, "read D_c");
}

// Launch shape of the transform passes for one mesh size and precision.
// Field buffers are kz-major, [kz][x][y], with kz planes of n n complex values plus 256
// bytes (32 FP32 or 16 FP64 values): the column pass steps from row to row within a plane and
// the pre-pass writes across planes; a plain power-of-two plane stride puts those accesses on
// few HBM channels.
int field_pad(bool fp64) { return fp64 ? 16 : 32; }

bool make_shape(const pkm_params& p, FftShape* out) {
  FftShape fs{};
  const int n = p.nmesh;
  const bool fp64 = p.precision == PKM_FP64;
  fs.n = n;
  fs.e_col = pick_e(n);
  fs.e_z = pick_e(n / 2);
  // register budget: FP64 column passes of the generic kernels use at most 8 elements per
  // thread (12 / 6 for lengths with a factor 3); the compile-time FP64 column kernels for
  // 256..1024 take 16 (the autotuner's pick at 512^3)
  const bool pow2_table = n >= 256 && n <= 1024 && (n & (n - 1)) == 0;
  if (fp64 && fs.e_col == 16 && !pow2_table) fs.e_col = 8;
  // z lines: 2E nodes per thread carry the harmonic recurrence in the pre-pass, which spills
  // at 12 (radix-3 lengths) as it would at 16
  if (fs.e_z == 16) fs.e_z = 8;
  if (fs.e_z == 12) fs.e_z = 6;
  // FP64 at 512: 4 elements per thread keep the pre-pass at 228 VGPRs and two waves per SIMD
  // (8 need 256 VGPRs and 149 AGPRs: one wave); measured 7% faster, the z pass 8% slower
  if (fp64 && n == 512) fs.e_z = 4;
  if (!fs.e_col || !fs.e_z || !make_sched(n, fs.e_col, &fs.sched_col, &fs.nst_col) ||
      !make_sched(n / 2, fs.e_z, &fs.sched_z, &fs.nst_z)) {
    return false;
  }
  // tile columns: 16 (128-byte rows in FP32, 256 in FP64: the autotuner's pick for FP64 at
  // 512^3), at most 512 threads and the LDS of one compute unit per column-pass block
  fs.tile = 16;
  const int pt_col = n / fs.e_col;
  while (fs.tile > 1 && (pt_col * fs.tile > 512 || (n / 2) % fs.tile || colpass_smem_bytes(fs, fp64) > 160 * 1024))
    fs.tile /= 2;
  // post-pass: at most 8 elements per thread (register budget of the fused recurrence), 6 for
  // lengths with a factor 3, except FP64 at 384 and 768: there 12 (one wave per line and two
  // fewer radix stages) measured 22% (384) and 39% (768) faster than 6, where in FP32 the
  // two took the same time
  fs.e_post = fs.e_col > 8 && fs.e_col % 8 == 0 ? 8 : fs.e_col;
  if (fs.e_post == 12 && !(fp64 && (n == 384 || n == 768))) fs.e_post = 6;
  if (!make_sched(n, fs.e_post, &fs.sched_post, &fs.nst_post)) {
    return false;
  }
  // 256-thread post-pass blocks (several resident per CU); narrow tiles share 128-byte rows
  // through L2 because consecutive tiles run on the same XCD
  {
    const int pt_post = n / fs.e_post;
    int tp = std::max(1, 256 / pt_post);
    tp = std::min(tp, 16);
    while (tp > 1 && (n / 2) % tp) tp /= 2;
    // a line wider than a wavefront synchronises its whole block at every radix stage: one
    // line per block (with more blocks per CU) measured 8-16% faster at 768 and 1024
    if (pt_post > 64) tp = 1;
    fs.tile_post = tp;
  }
  // z lines per block: a power of two dividing n (a block's lines share one x plane, and the
  // pre-pass writes them as runs of consecutive y into the kz-major field buffers)
  const int pt_z = (n / 2) / fs.e_z;
  // At most 256 threads per block, or 512 for FP32 from N = 512 up (16 lines of 512: the
  // pre-pass then writes 128-byte runs, measured faster than the 64-byte runs of 8 lines).
  const int zmax = (fp64 || n < 512) ? 256 : 512;
  fs.zlines = 1;
  for (;;) {
    FftShape next = fs;
    next.zlines = fs.zlines * 2;
    if (next.zlines * pt_z > zmax || n % next.zlines || zpass_smem_bytes(next, fp64) > 160 * 1024) break;
    fs = next;
  }
  fs.fpad = field_pad(fp64);
  *out = fs;
  return true;
}

bool is_elem(int e) { return e == 4 || e == 6 || e == 8 || e == 12 || e == 16; }

// Override the built-in shape with the non-zero fields of `sh`, checking every kernel limit.
bool apply_shape(const pkm_params& p, const pkm_shape& sh, FftShape* fs, int* ts, std::string* why) {
  const int n = p.nmesh, nh = n / 2;
  const bool fp64 = p.precision == PKM_FP64;
  FftShape f = *fs;
  auto fail = [&](const char* m) { *why = m; return false; };
  if (sh.e_col) {
    if (!is_elem(sh.e_col) || !make_sched(n, sh.e_col, &f.sched_col, &f.nst_col)) return fail("bad e_col");
    f.e_col = sh.e_col;
  }
  if (sh.tile) f.tile = sh.tile;
  if (f.tile < 1 || nh % f.tile || (n / f.e_col) * f.tile > 512 || colpass_smem_bytes(f, fp64) > 160 * 1024)
    return fail("column-pass tile breaks a kernel limit");
  if (sh.e_z) {
    if (!is_elem(sh.e_z) || !make_sched(nh, sh.e_z, &f.sched_z, &f.nst_z)) return fail("bad e_z");
    f.e_z = sh.e_z;
  }
  if (sh.zlines) f.zlines = sh.zlines;
  if (f.zlines < 1 || n % f.zlines || (nh / f.e_z) * f.zlines > (fp64 ? 256 : 512) ||
      zpass_smem_bytes(f, fp64) > 160 * 1024)
    return fail("z-pass lines break a kernel limit");
  if (sh.e_post) {
    if (!is_elem(sh.e_post) || !make_sched(n, sh.e_post, &f.sched_post, &f.nst_post)) return fail("bad e_post");
    f.e_post = sh.e_post;
  }
  if (sh.tile_post) f.tile_post = sh.tile_post;
  if (f.tile_post < 1 || nh % f.tile_post || (n / f.e_post) * f.tile_post > 256 ||
      xpost_base_bytes(f, fp64) > 150 * 1024)
    return fail("post-pass tile breaks a kernel limit");
  if (sh.post_axis && sh.post_axis != 2)
    return fail("post_axis must be 0 or 2: the post-pass runs along y over kz-major field buffers");
  if (sh.paint_tile) {
    if ((sh.paint_tile != 4 && sh.paint_tile != 8 && sh.paint_tile != 16) || n % sh.paint_tile)
      return fail("paint_tile must be 4, 8 or 16 and divide nmesh");
    *ts = sh.paint_tile;
  }
  *fs = f;
  return true;
}

pkm_shape shape_of(const FftShape& fs, int ts) {
  pkm_shape sh{};
  sh.e_col = fs.e_col;
  sh.tile = fs.tile;
  sh.e_z = fs.e_z;
  sh.zlines = fs.zlines;
  sh.e_post = fs.e_post;
  sh.tile_post = fs.tile_post;
  sh.paint_tile = ts;
  sh.post_axis = 2;  // y
  return sh;
}

pkm_status validate_params(const pkm_params* p, std::string* why) {
  if (!p) { *why = "params is NULL"; return PKM_EINVAL; }
  if (!is_smooth(p->nmesh)) { *why = "nmesh must be 2^a 3^b with a >= 2 and 16 <= N <= 1024"; return PKM_EINVAL; }
  if (!(p->box_len > 0) || !std::isfinite(p->box_len)) { *why = "box_len must be positive"; return PKM_EINVAL; }
  if (p->window < 1 || p->window > 3) { *why = "window must be 1 (NGP), 2 (CIC) or 3 (TSC)"; return PKM_EINVAL; }
  if (p->precision != PKM_FP32 && p->precision != PKM_FP64) { *why = "precision must be FP32 or FP64"; return PKM_EINVAL; }
  if (p->ell_max_hint < 0 || p->ell_max_hint > 16 || p->ell_max_hint % 2) {
    *why = "ell_max_hint must be even and in 0..16";
    return PKM_EINVAL;
  }
  if (p->deterministic != 0 && p->deterministic != 1) { *why = "deterministic must be 0 or 1"; return PKM_EINVAL; }
  if (p->los_mode == PKM_LOS_GLOBAL) {
    const double l2 = p->los[0] * p->los[0] + p->los[1] * p->los[1] + p->los[2] * p->los[2];
    if (!(l2 > 0)) { *why = "los must be a nonzero vector"; return PKM_EINVAL; }
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->box_origin[a]) || !std::isfinite(p->observer[a])) {
      *why = "box_origin and observer must be finite";
      return PKM_EINVAL;
    }
  return PKM_OK;
}

pkm_status validate_catalog(const pkm_catalog* c, bool need_nbar, std::string* why) {
  if (!c) { *why = "catalog is NULL"; return PKM_EINVAL; }
  if (c->n < 0) { *why = "catalog size must be >= 0"; return PKM_EINVAL; }
  if (c->n > PKM_MAX_PARTICLES) { *why = "catalog larger than PKM_MAX_PARTICLES"; return PKM_EINVAL; }
  if (c->n > 0 && !c->pos) { *why = "catalog positions are NULL"; return PKM_EINVAL; }
  if (need_nbar && c->n > 0 && !c->nbar) { *why = "randoms need nbar"; return PKM_EINVAL; }
  return PKM_OK;
}

template <typename F> pkm_status guarded(pkm_plan* pl, F&& f) {
  try {
    f();
    return PKM_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    if (pl) pl->err = "host allocation failed";
    return PKM_ENOMEM;
  } catch (...) {
    if (pl) pl->err = "unexpected host exception";
    return PKM_EDEVICE;
  }
}

void free_all(pkm_plan* pl) {
  for (void* f : pl->fields) dfree(pl, f);
  pl->fields.clear();
  for (void* ptr : {pl->d1, pl->d2, pl->s1, pl->s2, pl->c, pl->g, (void*)pl->ptrs_dev, (void*)pl->ftab_dev,
                    (void*)pl->map_dev, pl->tw, pl->ytab, pl->invw, pl->phase, (void*)pl->thr_dev, (void*)pl->partial,
                    (void*)pl->out_dev, (void*)pl->sums_dev, (void*)pl->cat_dev, (void*)pl->tile_count,
                    (void*)pl->tile_off, (void*)pl->tile_of, (void*)pl->tile_rank, pl->payload,
                    (void*)pl->scan_sums, (void*)pl->paint_ptrs, (void*)pl->det_acc, (void*)pl->det_scale})
    dfree(pl, ptr);
  if (pl->slot) (void)hipHostFree(pl->slot);
  if (pl->done) (void)hipEventDestroy(pl->done);
  for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
  if (pl->ev0) (void)hipEventDestroy(pl->ev0);
  if (pl->ev1) (void)hipEventDestroy(pl->ev1);
}

pkm_status validate_request(pkm_plan* pl, int ell_max, const double* k_edges, int n_edges, bool all_ell = false) {
  if (!k_edges || n_edges < 2) { pl->err = "need k_edges (n_edges >= 2)"; return PKM_EINVAL; }
  if (all_ell) {
    if (ell_max < 0 || ell_max > 16) { pl->err = "ell_max must be in 0..16"; return PKM_EINVAL; }
  } else if (ell_max < 0 || ell_max > 16 || ell_max % 2) {
    pl->err = "ell_max must be even and in 0..16";
    return PKM_EINVAL;
  }
  for (int i = 0; i < n_edges; ++i) {
    if (!(k_edges[i] >= 0.0) || !std::isfinite(k_edges[i])) { pl->err = "k edges must be finite and >= 0"; return PKM_EINVAL; }
    if (i > 0 && !(k_edges[i] > k_edges[i - 1])) { pl->err = "k edges must be strictly increasing"; return PKM_EINVAL; }
  }
  return PKM_OK;
}

// Host-only checks of a data/randoms pair (no device access).
pkm_status check_pair(const pkm_catalog* data, const pkm_catalog* randoms, std::string* why) {
  if (validate_catalog(data, false, why) != PKM_OK || (randoms && validate_catalog(randoms, true, why) != PKM_OK))
    return PKM_EINVAL;
  if (data->n == 0) { *why = "data catalog is empty"; return PKM_EINVAL; }
  if (randoms && randoms->n == 0) { *why = "random catalog is empty (pass NULL for a periodic box)"; return PKM_EINVAL; }
  // the painting sort keeps per-tile counts and offsets in 32-bit integers
  if (data->n + (randoms ? randoms->n : 0) > PKM_MAX_PARTICLES) {
    *why = "data + random objects above PKM_MAX_PARTICLES";
    return PKM_EINVAL;
  }
  return PKM_OK;
}

pkm_status validate_pair(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* randoms) {
  std::string why;
  if (check_pair(data, randoms, &why) != PKM_OK) {
    pl->err = why;
    return PKM_EINVAL;
  }
  return PKM_OK;
}

}  // namespace

// Internal entry points shared with the batch and serving runtime (runtime.hip).
namespace pkm_internal {

pkm_status prepare(pkm_plan* pl, int ell_max, const double* k_edges, int n_edges, int64_t max_particles) {
  if (validate_request(pl, ell_max, k_edges, n_edges) != PKM_OK) return PKM_EINVAL;
  if (max_particles < 1 || max_particles > PKM_MAX_PARTICLES) {
    pl->err = "max_particles must be in 1..PKM_MAX_PARTICLES";
    return PKM_EINVAL;
  }
  if (pl->pending_async) { pl->err = "an enqueued estimate has not been finished"; return PKM_EBUSY; }
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) prepare_compute<double>(pl, ell_max, k_edges, n_edges);
    else prepare_compute<float>(pl, ell_max, k_edges, n_edges);
    reserve_particles(pl, max_particles);
    pl->prep_ell = ell_max;
    pl->prep_edges.assign(k_edges, k_edges + n_edges);
    const size_t want = 4 + (size_t)pl->cc.total_vals;
    if (pl->slot_cap < want) {
      if (pl->slot) check_hip(pl, hipHostFree(pl->slot), "hipHostFree");
      pl->slot = nullptr;
      pl->slot_cap = 0;
      check_hip(pl, hipHostMalloc((void**)&pl->slot, want * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
      pl->slot_cap = want;
    }
    pl->stats.device_bytes = pl->bytes;
  });
}

// Doubles of a result slot (catalog sums + bin sums) of the prepared request.
size_t slot_doubles(const pkm_plan* pl) { return 4 + (size_t)pl->cc.total_vals; }
// The request tables are shared with the synchronous calls: a pkm_compute_multipoles with
// other settings replaces them, and then the prepared request (and the size of its result
// slot) no longer holds until pkm_prepare is called again.
bool prepared(const pkm_plan* pl) {
  return pl->prep_ell >= 0 && pl->sort_cap > 0 && pl->cc.ell_max == pl->prep_ell && pl->cc.basis == 0 &&
         pl->cc.edges == pl->prep_edges;
}
hipStream_t stream_of(const pkm_plan* pl) { return pl->stream; }
int device_of(const pkm_plan* pl) { return pl->dev.device_id; }
int64_t device_bytes(const pkm_plan* pl) { return pl->bytes; }
uint64_t generation(const pkm_plan* pl) { return pl->gen; }
std::string& error_of(pkm_plan* pl) { return pl->err; }

// Enqueue one estimate of device catalogs with its results copied to `slot` (pinned host,
// slot_doubles(pl) doubles).  No allocation, no host wait: safe inside stream capture.
pkm_status enqueue(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* randoms, double* slot, bool timed) {
  if (validate_pair(pl, data, randoms) != PKM_OK) return PKM_EINVAL;
  if (!data->on_device || (randoms && !randoms->on_device)) {
    pl->err = "asynchronous estimates take device-resident catalogs";
    return PKM_EINVAL;
  }
  if (!prepared(pl)) {
    pl->err = "plan not prepared for this request (pkm_prepare, again after a synchronous call with other settings)";
    return PKM_EORDER;
  }
  if ((size_t)(data->n + (randoms ? randoms->n : 0)) > pl->sort_cap) {
    pl->err = "particle count above the prepared capacity";
    return PKM_EINVAL;
  }
  // per-launch timing events only when asked for and not recorded into a graph
  const bool timing = pl->stage_timing;
  pl->stage_timing = timing && timed;
  pkm_status st = guarded(pl, [&] {
    DevCats dc;
    dc.dp = data->pos; dc.dw = data->w; dc.dn = data->nbar; dc.nd = data->n;
    if (randoms) { dc.rp = randoms->pos; dc.rw = randoms->w; dc.rn = randoms->nbar; dc.nr = randoms->n; }
    if (pl->fp64) enqueue_estimate<double>(pl, dc, slot); else enqueue_estimate<float>(pl, dc, slot);
  });
  pl->stage_timing = timing;
  if (st == PKM_OK) pl->painted = false;  // the resident fields now belong to the enqueued estimate
  return st;
}

pkm_status enqueue_compute_only(pkm_plan* pl, double* slot) {
  if (!prepared(pl)) {
    pl->err = "plan not prepared for this request";
    return PKM_EORDER;
  }
  const bool timing = pl->stage_timing;
  pl->stage_timing = false;
  pkm_status st = guarded(pl, [&] {
    if (pl->fp64) enqueue_compute_copy<double>(pl, slot); else enqueue_compute_copy<float>(pl, slot);
  });
  pl->stage_timing = timing;
  return st;
}

pkm_status finish(pkm_plan* pl, const double* slot, int64_t nd, int64_t nr, pkm_result* out, std::string* why) {
  const pkm_status st = finish_from_slot(pl, slot, nd, nr, out);
  if (st != PKM_OK) *why = ZERO_NORM;
  return st;
}

int64_t footprint(const pkm_params* p, int ell_max, int n_edges, int64_t n_particles) {
  FftShape fs{};
  if (!make_shape(*p, &fs)) return -1;
  const int64_t n = p->nmesh;
  const int64_t mesh = (p->precision == PKM_FP64 ? 8 : 4) * n * n * n;
  int nf = fields_for(std::max(ell_max, p->ell_max_hint == 0 ? 4 : p->ell_max_hint));
  if (p->max_group > 0) nf = std::min(nf, p->max_group);
  nf = std::max(nf, 1);
  const int64_t meshes = (p->interlaced ? 6 : 4) + nf;
  const int64_t pads = (int64_t)nf * (n / 2) * fs.fpad * 2 * (p->precision == PKM_FP64 ? 8 : 4);
  const int64_t nb = std::max(1, n_edges - 1);
  const int64_t partial = (int64_t)post_blocks(fs) * (3 + ell_max / 2) * nb * 8;
  const int64_t ts = 8;
  const int64_t ntiles = (n / ts) * (n / ts) * (n / ts);
  const int64_t det = p->deterministic ? 8 * n * n * n * (p->interlaced ? 2 : 1) : 0;
  return meshes * mesh + pads + 80 * n_particles + partial + 8 * ntiles + det + (4 << 20);
}

}  // namespace pkm_internal

// -------------------------------------------------------------------------------------------
// C ABI
// -------------------------------------------------------------------------------------------
namespace {
// why the calling thread's last pkm_plan_create failed (pkm_plan_last_error(NULL))
thread_local std::string g_create_err = "no plan";
}  // namespace

extern "C" {

int pkm_abi_version(void) { return PKM_ABI_VERSION; }

int64_t pkm_plan_footprint(const pkm_params* p, int32_t ell_max, int32_t n_edges, int64_t n_particles) {
  if (!p || ell_max < 0 || ell_max > 16 || n_edges < 2 || n_particles < 0) return -1;
  std::string why;
  if (validate_params(p, &why) != PKM_OK) return -1;
  return pkm_internal::footprint(p, ell_max, n_edges, n_particles);
}

pkm_status pkm_check_catalogs(const pkm_catalog* data, const pkm_catalog* randoms) {
  std::string why;
  return check_pair(data, randoms, &why);
}

const char* pkm_status_str(pkm_status s) {
  switch (s) {
    case PKM_OK: return "ok";
    case PKM_EINVAL: return "invalid argument";
    case PKM_EORDER: return "compute before paint";
    case PKM_ENOMEM: return "out of memory / over budget";
    case PKM_EDEVICE: return "device error";
    case PKM_EBUSY: return "busy";
    case PKM_ECANCELLED: return "cancelled";
  }
  return "unknown status";
}

pkm_status pkm_plan_create(const pkm_params* p, const pkm_device* dev, pkm_plan** out) {
  return pkm_plan_create_shaped(p, dev, nullptr, out);
}

pkm_status pkm_plan_create_shaped(const pkm_params* p, const pkm_device* dev, const pkm_shape* shape,
                                  pkm_plan** out) {
  g_create_err = "no plan";
  if (!out) return PKM_EINVAL;
  std::string why;
  pkm_status st = validate_params(p, &why);
  if (st != PKM_OK) { g_create_err = why; return st; }
  FftShape fs0{};
  int ts0 = 8;
  if (!make_shape(*p, &fs0)) { g_create_err = "no launch shape for these parameters"; return PKM_EINVAL; }
  while (p->nmesh % ts0) ts0 /= 2;
  if (shape && !apply_shape(*p, *shape, &fs0, &ts0, &why)) { g_create_err = why; return PKM_EINVAL; }
  pkm_plan* pl = new (std::nothrow) pkm_plan();
  if (!pl) { g_create_err = "host allocation failed"; return PKM_ENOMEM; }
  pl->p = *p;
  if (const char* env = std::getenv("PKM_DETERMINISTIC"))
    if (env[0] == '1') pl->p.deterministic = 1;
  pl->frame = harmonic_frame(pl->p);
  if (pl->p.ell_max_hint == 0) pl->p.ell_max_hint = 4;
  if (dev) pl->dev = *dev;
  pl->stream = (hipStream_t)pl->dev.hip_stream;
  pl->fp64 = p->precision == PKM_FP64;
  pl->es = pl->fp64 ? 8 : 4;
  const int n = p->nmesh;
  pl->mesh_bytes = pl->es * (size_t)n * n * n;
  pl->fs = fs0;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->dev.device_id) == hipSuccess)
      pl->fs.cus = cus;
  }
  st = guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    check_hip(pl, hipEventCreate(&pl->ev0), "event");
    check_hip(pl, hipEventCreate(&pl->ev1), "event");
    pl->d1 = dalloc(pl, pl->mesh_bytes);
    if (p->interlaced) pl->d2 = dalloc(pl, pl->mesh_bytes);
    pl->s1 = dalloc(pl, pl->mesh_bytes);
    if (p->interlaced) pl->s2 = dalloc(pl, pl->mesh_bytes);
    pl->c = dalloc(pl, pl->mesh_bytes);
    pl->g = dalloc(pl, pl->mesh_bytes);
    pl->tw = dalloc(pl, 2 * pl->es * n);
    pl->invw = dalloc(pl, pl->es * n);
    pl->phase = dalloc(pl, 2 * pl->es * n);
    pl->ytab = dalloc(pl, pl->es * (YLM_LMAX + 1) * YLM_STRIDE);
    pl->sums_dev = (double*)dalloc(pl, sizeof(double) * (6 + 3 * SUM_BLOCKS));
    if (pl->p.deterministic) {
      pl->det_acc = (unsigned long long*)dalloc(pl, sizeof(unsigned long long) * (size_t)n * n * n *
                                                        (p->interlaced ? 2 : 1));
      pl->det_scale = (double*)dalloc(pl, sizeof(double));
    }
    pl->ts = ts0;
    pl->ntiles = (n / pl->ts) * (n / pl->ts) * (n / pl->ts);
    pl->tile_count = (int*)dalloc(pl, sizeof(int) * (size_t)TILE_COUNT_COPIES * (pl->ntiles + 1));
    pl->tile_off = (int*)dalloc(pl, sizeof(int) * (pl->ntiles + 1));
    pl->scan_sums = (int*)dalloc(pl, sizeof(int) * tile_scan_scratch(pl->ntiles));
    int want = fields_for(pl->p.ell_max_hint);
    if (p->max_group > 0) want = std::min(want, p->max_group);
    ensure_fields(pl, std::max(want, 1));
    pl->ftab_dev = (int*)dalloc(pl, sizeof(int) * 4 * 64);
    pl->ftab_cap = 4 * 64;
    pl->paint_ptrs = (void**)dalloc(pl, sizeof(void*) * 3);
    void* pp[3] = {pl->s1, pl->s2, pl->g};
    check_hip(pl, hipMemcpy(pl->paint_ptrs, pp, sizeof pp, hipMemcpyHostToDevice), "upload paint pointers");
    check_hip(pl, hipEventCreateWithFlags(&pl->done, hipEventDisableTiming), "event");
    if (pl->fp64) upload_tables<double>(pl); else upload_tables<float>(pl);
  });
  if (st != PKM_OK) {
    g_create_err = pl->err;
    free_all(pl);
    delete pl;
    return st;
  }
  pl->stats.device_bytes = pl->bytes;
  *out = pl;
  return PKM_OK;
}

pkm_status pkm_paint(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* randoms) {
  if (!pl) return PKM_EINVAL;
  if (validate_pair(pl, data, randoms) != PKM_OK) return PKM_EINVAL;
  if (pl->pending_async) { pl->err = "an enqueued estimate has not been finished"; return PKM_EBUSY; }
  pl->painted = false;
  pkm_status st = guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_paint<double>(pl, data, randoms); else run_paint<float>(pl, data, randoms);
  });
  pl->stats.device_bytes = pl->bytes;
  return st;
}

pkm_status pkm_compute_multipoles_basis(pkm_plan* pl, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                        int32_t basis, pkm_result* out) {
  if (!pl) return PKM_EINVAL;
  if (!out) { pl->err = "need a result"; return PKM_EINVAL; }
  if (basis != PKM_BASIS_SPHERICAL && basis != PKM_BASIS_CARTESIAN) {
    pl->err = "basis must be PKM_BASIS_SPHERICAL or PKM_BASIS_CARTESIAN";
    return PKM_EINVAL;
  }
  if (validate_request(pl, ell_max, k_edges, n_edges) != PKM_OK) return PKM_EINVAL;
  if (pl->pending_async) { pl->err = "an enqueued estimate has not been finished"; return PKM_EBUSY; }
  if (!pl->painted) { pl->err = "pkm_paint must succeed before pkm_compute_multipoles"; return PKM_EORDER; }
  pkm_status st = guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_compute<double>(pl, ell_max, k_edges, n_edges, basis, out);
    else run_compute<float>(pl, ell_max, k_edges, n_edges, basis, out);
  });
  pl->stats.device_bytes = pl->bytes;
  return st;
}

pkm_status pkm_compute_multipoles(pkm_plan* pl, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                  pkm_result* out) {
  return pkm_compute_multipoles_basis(pl, ell_max, k_edges, n_edges, PKM_BASIS_SPHERICAL, out);
}

pkm_status pkm_compute_multipoles_all(pkm_plan* pl, int32_t ell_max, const double* k_edges, int32_t n_edges,
                                      pkm_result* out) {
  if (!pl) return PKM_EINVAL;
  if (!out) { pl->err = "need a result"; return PKM_EINVAL; }
  if (validate_request(pl, ell_max, k_edges, n_edges, true) != PKM_OK) return PKM_EINVAL;
  if (pl->pending_async) { pl->err = "an enqueued estimate has not been finished"; return PKM_EBUSY; }
  if (!pl->painted) { pl->err = "pkm_paint must succeed before pkm_compute_multipoles_all"; return PKM_EORDER; }
  pkm_status st = guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_compute<double>(pl, ell_max, k_edges, n_edges, BASIS_ALL_ELL, out);
    else run_compute<float>(pl, ell_max, k_edges, n_edges, BASIS_ALL_ELL, out);
  });
  pl->stats.device_bytes = pl->bytes;
  return st;
}

// Arguments of the (k, mu) calls; PKM_OK when the request can run.
pkm_status validate_kmu(pkm_plan* pl, const double* k_edges, int32_t n_k_edges, const double* mu_edges,
                        int32_t n_mu_edges) {
  if (!k_edges || !mu_edges || n_k_edges < 2 || n_mu_edges < 2) { pl->err = "need k and mu edges"; return PKM_EINVAL; }
  for (int i = 0; i < n_k_edges; ++i)
    if (!(k_edges[i] >= 0) || (i > 0 && !(k_edges[i] > k_edges[i - 1]))) { pl->err = "bad k edges"; return PKM_EINVAL; }
  for (int i = 0; i < n_mu_edges; ++i)
    if (!(mu_edges[i] >= 0 && mu_edges[i] <= 1) || (i > 0 && !(mu_edges[i] > mu_edges[i - 1]))) {
      pl->err = "mu edges must increase within [0, 1]";
      return PKM_EINVAL;
    }
  if ((int64_t)(n_k_edges - 1) * (n_mu_edges - 1) > KMU_MAX_CELLS) {
    pl->err = "too many (k, mu) cells for one pass (limit 3072)";
    return PKM_EINVAL;
  }
  if (pl->p.los_mode != PKM_LOS_GLOBAL) { pl->err = "plan was not created with los_mode = GLOBAL"; return PKM_EINVAL; }
  if (pl->pending_async) { pl->err = "an enqueued estimate has not been finished"; return PKM_EBUSY; }
  if (!pl->painted) { pl->err = "pkm_paint must succeed first"; return PKM_EORDER; }
  return PKM_OK;
}

pkm_status pkm_kmu_global(pkm_plan* pl, const double* k_edges, int32_t n_k_edges, const double* mu_edges,
                          int32_t n_mu_edges, double* pkmu_out, int64_t* nmodes_out) {
  if (!pl) return PKM_EINVAL;
  const pkm_status v = validate_kmu(pl, k_edges, n_k_edges, mu_edges, n_mu_edges);
  if (v != PKM_OK) return v;
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_kmu<double>(pl, k_edges, n_k_edges, mu_edges, n_mu_edges, pkmu_out, nmodes_out);
    else run_kmu<float>(pl, k_edges, n_k_edges, mu_edges, n_mu_edges, pkmu_out, nmodes_out);
  });
}

pkm_status pkm_kmu_global_noalloc(pkm_plan* pl, const double* k_edges, int32_t n_k_edges, const double* mu_edges,
                                  int32_t n_mu_edges, double* pkmu_out, int64_t* nmodes_out) {
  if (!pl) return PKM_EINVAL;
  const pkm_status v = validate_kmu(pl, k_edges, n_k_edges, mu_edges, n_mu_edges);
  if (v != PKM_OK) return v;
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_kmu_noalloc<double>(pl, k_edges, n_k_edges, mu_edges, n_mu_edges, pkmu_out, nmodes_out);
    else run_kmu_noalloc<float>(pl, k_edges, n_k_edges, mu_edges, n_mu_edges, pkmu_out, nmodes_out);
  });
}

pkm_status pkm_stats(const pkm_plan* pl, pkm_stats_t* out) {
  if (!pl || !out) return PKM_EINVAL;
  *out = pl->stats;
  out->device_bytes = pl->bytes;
  return PKM_OK;
}

pkm_status pkm_set_stage_timing(pkm_plan* pl, int32_t enable) {
  if (!pl) return PKM_EINVAL;
  pl->stage_timing = enable != 0;
  return PKM_OK;
}

pkm_status pkm_reset_stats(pkm_plan* pl) {
  if (!pl) return PKM_EINVAL;
  for (int i = 0; i < PKM_NSTAGES; ++i) {
    pl->stats.stage_ms[i] = 0.0;
    pl->stats.stage_launches[i] = 0;
  }
  return PKM_OK;
}

const char* pkm_plan_last_error(const pkm_plan* pl) { return pl ? pl->err.c_str() : g_create_err.c_str(); }

void pkm_plan_destroy(pkm_plan* pl) {
  if (!pl) return;
  (void)hipSetDevice(pl->dev.device_id);
  if (pl->stream) (void)hipStreamSynchronize(pl->stream); else (void)hipDeviceSynchronize();
  free_all(pl);
  delete pl;
}

pkm_status pkm_fft3d_forward(pkm_plan* pl, const void* in, void* out) {
  if (!pl || !in || !out) return PKM_EINVAL;
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_fft_forward<double>(pl, in, out); else run_fft_forward<float>(pl, in, out);
  });
}

pkm_status pkm_fft3d_inverse(pkm_plan* pl, void* in, void* out) {
  if (!pl || !in || !out) return PKM_EINVAL;
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    if (pl->fp64) run_fft_inverse<double>(pl, in, out); else run_fft_inverse<float>(pl, in, out);
  });
}

pkm_status pkm_plan_read_buffer(pkm_plan* pl, int32_t which, void* host, size_t bytes) {
  if (!pl || !host) return PKM_EINVAL;
  if (which < 0 || which > 3) { pl->err = "which must be 0..3"; return PKM_EINVAL; }
  if (bytes != pl->mesh_bytes) { pl->err = "bytes must equal the mesh buffer size"; return PKM_EINVAL; }
  if (!pl->painted) { pl->err = "nothing painted"; return PKM_EORDER; }
  if (which == 1 && !pl->p.interlaced) { pl->err = "plan is not interlaced"; return PKM_EINVAL; }
  return guarded(pl, [&] {
    check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice");
    check_hip(pl, hipStreamSynchronize(pl->stream), "sync");
    if (which == 0) check_hip(pl, hipMemcpy(host, pl->d1, bytes, hipMemcpyDeviceToHost), "read");
    else if (which == 1) check_hip(pl, hipMemcpy(host, pl->d2, bytes, hipMemcpyDeviceToHost), "read");
    else if (which == 2) check_hip(pl, hipMemcpy(host, pl->c, bytes, hipMemcpyDeviceToHost), "read");
    else if (pl->fp64) read_dc<double>(pl, host, bytes);
    else read_dc<float>(pl, host, bytes);
  });
}

pkm_status pkm_plan_shape(const pkm_plan* pl, pkm_shape* out) {
  if (!pl || !out) return PKM_EINVAL;
  *out = shape_of(pl->fs, pl->ts);
  return PKM_OK;
}

pkm_status pkm_autotune(const pkm_params* p, const pkm_device* dev, int32_t ell_max, int64_t n_particles,
                        int32_t reps, pkm_shape* best, double* best_ms, double* default_ms) {
  std::string why;
  if (validate_params(p, &why) != PKM_OK) return PKM_EINVAL;
  if (ell_max < 0 || ell_max > 16 || ell_max % 2 || n_particles < 22 || reps < 1) return PKM_EINVAL;
  const int n = p->nmesh, nh = n / 2;
  const double L = p->box_len;
  pkm_device d{};
  if (dev) d = *dev;
  if (hipSetDevice(d.device_id) != hipSuccess) return PKM_EDEVICE;
  // synthetic catalog: uniform in the box, 1/21 data and 20/21 randoms (seeded)
  const int64_t nd = std::max<int64_t>(1, n_particles / 21), nr = n_particles - nd;
  std::vector<double> hpos(3 * (size_t)n_particles), hw((size_t)n_particles, 1.0),
      hn((size_t)n_particles, (double)nd / (L * L * L));
  uint64_t state = 0x9E3779B97F4A7C15ull;
  for (double& v : hpos) {  // splitmix64 -> uniform [0, 1)
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  }
  for (int64_t i = 0; i < n_particles; ++i)
    for (int a = 0; a < 3; ++a) hpos[3 * i + a] = p->box_origin[a] + hpos[3 * i + a] * L;
  pkm_catalog dc{hpos.data(), hw.data(), hn.data(), nd, 0};
  pkm_catalog rc{hpos.data() + 3 * nd, hw.data() + nd, hn.data() + nd, nr, 0};
  std::vector<double> edges;
  const double kf = 2.0 * M_PI / L;
  for (double k = 0.0; k < M_PI * n / L; k += 4.0 * kf) edges.push_back(k);
  if (edges.size() < 2) edges.push_back(M_PI * n / L);
  const int nb = (int)edges.size() - 1;
  std::vector<double> poles((size_t)(ell_max / 2 + 1) * nb), kmean(nb);
  std::vector<int64_t> nmodes(nb);
  // device ms per stage of one estimate with a shape (negative: shape rejected or failed)
  auto time_shape = [&](const pkm_shape& sh, double* stage_ms) -> double {
    pkm_plan* pl = nullptr;
    pkm_params pp = *p;
    if (pp.ell_max_hint < ell_max) pp.ell_max_hint = ell_max;
    if (pkm_plan_create_shaped(&pp, &d, &sh, &pl) != PKM_OK) return -1.0;
    pkm_result r{poles.data(), kmean.data(), nmodes.data(), 0, 0, 0, 0};
    double total = -1.0;
    if (pkm_paint(pl, &dc, &rc) == PKM_OK && pkm_compute_multipoles(pl, ell_max, edges.data(), nb + 1, &r) == PKM_OK) {
      pkm_set_stage_timing(pl, 1);
      pkm_reset_stats(pl);
      bool ok = true;
      for (int k = 0; k < reps && ok; ++k)
        ok = pkm_paint(pl, &dc, &rc) == PKM_OK && pkm_compute_multipoles(pl, ell_max, edges.data(), nb + 1, &r) == PKM_OK;
      if (ok) {
        total = 0.0;
        for (int st = 0; st < PKM_NSTAGES; ++st) {
          stage_ms[st] = pl->stats.stage_ms[st] / reps;
          total += stage_ms[st];
        }
      }
    }
    pkm_plan_destroy(pl);
    return total;
  };
  double ms[PKM_NSTAGES];
  pkm_shape cur{};
  const double base = time_shape(cur, ms);
  if (base < 0) return PKM_EDEVICE;
  auto group_ms = [&](const double* m, std::initializer_list<int> st) {
    double t = 0;
    for (int i : st) t += m[i];
    return t;
  };
  // one group at a time: keep the candidate with the smallest time over the group's stages
  auto tune = [&](std::vector<pkm_shape> cands, std::initializer_list<int> stages) {
    double best_t = -1.0;
    pkm_shape keep = cur;
    for (const pkm_shape& c : cands) {
      double m[PKM_NSTAGES];
      if (time_shape(c, m) < 0) continue;
      const double t = group_ms(m, stages);
      if (best_t < 0 || t < best_t) { best_t = t; keep = c; }
    }
    cur = keep;
  };
  {
    std::vector<pkm_shape> c;
    for (int ts : {4, 8, 16}) { pkm_shape s2 = cur; s2.paint_tile = ts; c.push_back(s2); }
    tune(c, {PKM_STAGE_PAINT});
  }
  {
    std::vector<pkm_shape> c;
    for (int e : {4, 8, 16})
      for (int zl = 1; zl <= 64; zl *= 2) {
        if ((nh / e) * zl > (p->precision == PKM_FP64 ? 256 : 512) || (nh / e) * zl < 64) continue;
        pkm_shape s2 = cur; s2.e_z = e; s2.zlines = zl; c.push_back(s2);
      }
    tune(c, {PKM_STAGE_ZFWD, PKM_STAGE_ZPRE});
  }
  {
    std::vector<pkm_shape> c;
    for (int e : {4, 8, 16})
      for (int tl : {4, 8, 16}) {
        if ((n / e) * tl > 512 || (n / e) * tl < 64) continue;
        pkm_shape s2 = cur; s2.e_col = e; s2.tile = tl; c.push_back(s2);
      }
    tune(c, {PKM_STAGE_YCOL, PKM_STAGE_XCOMBINE, PKM_STAGE_IYCOL});
  }
  {
    std::vector<pkm_shape> c;
    for (int e : {4, 8})
      for (int tl : {1, 2, 4, 8, 16}) {
        if ((n / e) * tl > 256 || (n / e) * tl < 64) continue;
        pkm_shape s2 = cur; s2.e_post = e; s2.tile_post = tl; c.push_back(s2);
      }
    tune(c, {PKM_STAGE_YCOL, PKM_STAGE_XPOST});
  }
  double m[PKM_NSTAGES];
  double tuned = time_shape(cur, m);
  if (tuned < 0 || tuned > base) {  // no gain over the built-in shape
    cur = pkm_shape{};
    tuned = base;
  }
  // report the full shape the choice resolves to
  {
    FftShape fs{};
    int ts = 8;
    make_shape(*p, &fs);
    while (n % ts) ts /= 2;
    apply_shape(*p, cur, &fs, &ts, &why);
    if (best) *best = shape_of(fs, ts);
  }
  if (best_ms) *best_ms = tuned;
  if (default_ms) *default_ms = base;
  return PKM_OK;
}

pkm_status pkm_prepare(pkm_plan* pl, int32_t ell_max, const double* k_edges, int32_t n_edges,
                       int64_t max_particles) {
  if (!pl) return PKM_EINVAL;
  return pkm_internal::prepare(pl, ell_max, k_edges, n_edges, max_particles);
}

pkm_status pkm_enqueue(pkm_plan* pl, const pkm_catalog* data, const pkm_catalog* randoms) {
  if (!pl) return PKM_EINVAL;
  if (pl->pending_async) { pl->err = "the previous enqueued estimate has not been finished"; return PKM_EBUSY; }
  if (!data) { pl->err = "data catalog is NULL"; return PKM_EINVAL; }
  pkm_status st = guarded(pl, [&] { check_hip(pl, hipSetDevice(pl->dev.device_id), "hipSetDevice"); });
  if (st != PKM_OK) return st;
  st = pkm_internal::enqueue(pl, data, randoms, pl->slot, true);
  if (st != PKM_OK) return st;
  st = guarded(pl, [&] { check_hip(pl, hipEventRecord(pl->done, pl->stream), "event"); });
  if (st != PKM_OK) return st;
  pl->pend_nd = data->n;
  pl->pend_nr = randoms ? randoms->n : 0;
  pl->pending_async = true;
  return PKM_OK;
}

pkm_status pkm_query(pkm_plan* pl) {
  if (!pl) return PKM_EINVAL;
  if (!pl->pending_async) { pl->err = "nothing enqueued"; return PKM_EORDER; }
  const hipError_t e = hipEventQuery(pl->done);
  if (e == hipSuccess) return PKM_OK;
  if (e == hipErrorNotReady) return PKM_EBUSY;
  pl->err = std::string("event query failed: ") + hipGetErrorString(e);
  return PKM_EDEVICE;
}

pkm_status pkm_finish(pkm_plan* pl, pkm_result* out) {
  if (!pl) return PKM_EINVAL;
  if (!out) { pl->err = "need a result"; return PKM_EINVAL; }
  if (!pl->pending_async) { pl->err = "nothing enqueued"; return PKM_EORDER; }
  pkm_status st = guarded(pl, [&] { check_hip(pl, hipEventSynchronize(pl->done), "event synchronize"); });
  pl->pending_async = false;
  if (st != PKM_OK) return st;
  resolve_stages(pl);
  if (finish_from_slot(pl, pl->slot, pl->pend_nd, pl->pend_nr, out) != PKM_OK) {
    pl->err = ZERO_NORM;  // the plan stays unpainted
    return PKM_EINVAL;
  }
  pl->alpha = out->alpha;
  pl->norm_I = out->norm_I;
  pl->shot = out->shot_noise;
  pl->n_transforms = out->n_transforms;
  pl->painted = true;
  return PKM_OK;
}

}  // extern "C"
