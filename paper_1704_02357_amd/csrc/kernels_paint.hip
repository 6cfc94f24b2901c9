// Catalog reductions and mass assignment (Sec. 2.1 FKP field, Sec. 2.3 TSC painting with
// interlacing).  Mesh coordinates are computed in FP64 with explicitly rounded operations
// (u = (x - o) * (N / L); no fused multiply-add) so that node indices and fractions match
// any other IEEE implementation of the same formula bit for bit.
#include <algorithm>

#include "kernels.hpp"
#include "device_common.hpp"

namespace pkm {

namespace {

constexpr int SUM_THREADS = 256;

__global__ void __launch_bounds__(SUM_THREADS) k_catalog_sums(const double* __restrict__ w,
                                                              const double* __restrict__ nbar, int64_t n,
                                                              double* __restrict__ partial) {
  __shared__ double s0[SUM_THREADS], s1[SUM_THREADS], s2[SUM_THREADS];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double wi = w ? w[i] : 1.0;
    const double w2 = wi * wi;
    a0 += w2;
    a1 += w2 * (nbar ? nbar[i] : 1.0);
    a2 = fmax(a2, fabs(wi));
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int h = SUM_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = s0[0];
    partial[3 * blockIdx.x + 1] = s1[0];
    partial[3 * blockIdx.x + 2] = s2[0];
  }
}

__global__ void __launch_bounds__(SUM_THREADS) k_sum_partials2(const double* __restrict__ partial, int nblk,
                                                               double* __restrict__ out2, double* __restrict__ wmax) {
  __shared__ double s0[SUM_THREADS], s1[SUM_THREADS], s2[SUM_THREADS];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += SUM_THREADS) {
    a0 += partial[3 * b];
    a1 += partial[3 * b + 1];
    a2 = fmax(a2, partial[3 * b + 2]);
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int h = SUM_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = s0[0];
    out2[1] = s1[0];
    *wmax = s2[0];
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__device__ __forceinline__ int wrap(long long c, int n) {
  long long r = c % n;
  return (int)(r < 0 ? r + n : r);
}

// ---------------------------------------------------------------------------------------
// Tile-sorted painting.  Particles are counting-sorted by the tile (TS^3 nodes) holding
// their base node floor(u); each workgroup accumulates one tile plus the halo its window
// reaches, one LDS region per mesh (for TSC (TS + 3)^3 nodes from t0 - 1 on the plain mesh and
// (TS + 2)^3 from t0 on the +1/2 interlaced one; PaintReach), then adds the non-zero region
// cells to the global meshes with atomics.  A tap that falls outside its region (only possible
// through FP64 rounding at a cell face) goes straight to a global atomic.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void mesh_u(const double* __restrict__ pos, int64_t i, double o0, double o1, double o2,
                                       double scale, double* u) {
  u[0] = __dmul_rn(__dsub_rn(pos[3 * i + 0], o0), scale);
  u[1] = __dmul_rn(__dsub_rn(pos[3 * i + 1], o1), scale);
  u[2] = __dmul_rn(__dsub_rn(pos[3 * i + 2], o2), scale);
}

// Tile counters come in NCOPY copies of ntiles + 1: a block counts into copy blockIdx mod
// NCOPY.  Workgroups are dispatched round-robin over the 8 XCDs, so each copy is then updated
// from one XCD only and its cache lines stay in that XCD's L2 instead of moving between XCDs
// on every atomic.  (Any copy assignment is correct; this one is only faster.)  The rank
// returned carries the copy in its top bits.
constexpr int NCOPY = TILE_COUNT_COPIES;
constexpr int RANK_BITS = 28;

// Each thread takes CPT particles per round (blockDim apart) and issues their counter atomics
// back to back, so CPT atomics per thread are in flight at once: the pass is bound by the
// latency of returning atomics, not by their number.
constexpr int CPT = 4;
__global__ void k_tile_count(const double* __restrict__ pos, int64_t n, int64_t base, double o0, double o1,
                             double o2, double scale, int nmesh, int ts, int ntiles, int* __restrict__ count,
                             int* __restrict__ tile_of, int* __restrict__ rank) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * CPT;
  const int tpa = nmesh / ts;
  const int copy = blockIdx.x % NCOPY;
  int* cnt = count + (size_t)copy * (ntiles + 1);
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * CPT + threadIdx.x; i0 < n; i0 += stride) {
    int tile[CPT], r[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t i = i0 + (int64_t)j * blockDim.x;
      tile[j] = -1;
      if (i < n) {
        double u[3];
        mesh_u(pos, i, o0, o1, o2, scale, u);
        int tc[3];
        for (int a = 0; a < 3; ++a) tc[a] = wrap((long long)floor(u[a]), nmesh) / ts;
        tile[j] = (tc[0] * tpa + tc[1]) * tpa + tc[2];
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (tile[j] >= 0) r[j] = atomicAdd(&cnt[tile[j]], 1);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t i = i0 + (int64_t)j * blockDim.x;
      if (tile[j] >= 0) {
        tile_of[base + i] = tile[j];
        rank[base + i] = r[j] | (copy << RANK_BITS);
      }
    }
  }
}

constexpr int SCAN_THREADS = 1024;
// Exclusive scan in three launches: per-block scans (block sums out), one-block scan of
// the block sums, and the addition of the scanned sums.  Coalesced throughout.
__device__ __forceinline__ int block_scan_excl(int v, int* part) {
  part[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < SCAN_THREADS; d <<= 1) {
    const int add = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  return part[threadIdx.x] - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_blocks(const int* __restrict__ count, int n,
                                                              int* __restrict__ off, int* __restrict__ bsum) {
  __shared__ int part[SCAN_THREADS];
  const int i = blockIdx.x * SCAN_THREADS + threadIdx.x;
  int v = 0;
  if (i < n)
    for (int c = 0; c < NCOPY; ++c) v += count[(size_t)c * (n + 1) + i];
  const int ex = block_scan_excl(v, part);
  if (i < n) off[i] = ex;
  if (threadIdx.x == SCAN_THREADS - 1) bsum[blockIdx.x] = ex + v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(int* __restrict__ bsum, int nb, int* __restrict__ off,
                                                            int n) {
  __shared__ int part[SCAN_THREADS];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += SCAN_THREADS) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    const int ex = block_scan_excl(v, part);
    if (i < nb) bsum[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == SCAN_THREADS - 1) carry += ex + v;
    __syncthreads();
  }
  if (threadIdx.x == 0) off[n] = carry;
}

// Final tile offsets, and the counters turned in place into per-copy start offsets:
// count[c][i] <- off[i] + sum over c' < c of count[c'][i].
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_add(const int* __restrict__ bsum, int n,
                                                           int* __restrict__ off, int* __restrict__ count) {
  const int i = blockIdx.x * SCAN_THREADS + threadIdx.x;
  if (i >= n) return;
  int start = off[i] + bsum[blockIdx.x];
  off[i] = start;
  for (int c = 0; c < NCOPY; ++c) {
    int* p = count + (size_t)c * (n + 1) + i;
    const int v = *p;
    *p = start;
    start += v;
  }
}

// Scatter each particle's payload (x, y, z, signed weight) to its slot in tile order.
__global__ void k_tile_scatter(const int* __restrict__ tile_of, const int* __restrict__ rank, int64_t nd, int64_t n,
                               int ntiles, const int* __restrict__ start, const double* __restrict__ dpos,
                               const double* __restrict__ dw, const double* __restrict__ rpos,
                               const double* __restrict__ rw, double alpha, double4* __restrict__ payload) {
  // CPT particles per thread and round, loads first: several offset lookups in flight at once
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * CPT;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * CPT + threadIdx.x; i0 < n; i0 += stride) {
    int dst[CPT];
    double4 p[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t i = i0 + (int64_t)j * blockDim.x;
      dst[j] = -1;
      if (i < n) {
        const bool isd = i < nd;
        const int64_t k = isd ? i : i - nd;
        const double* pos = isd ? dpos : rpos;
        const double* wp = isd ? dw : rw;
        p[j].x = pos[3 * k];
        p[j].y = pos[3 * k + 1];
        p[j].z = pos[3 * k + 2];
        p[j].w = (wp ? wp[k] : 1.0) * (isd ? 1.0 : -alpha);
        const int r = rank[i];
        const int copy = (int)((unsigned)r >> RANK_BITS);
        dst[j] = start[(size_t)copy * (ntiles + 1) + tile_of[i]] + (r & ((1 << RANK_BITS) - 1));
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (dst[j] >= 0) payload[dst[j]] = p[j];
  }
}

// Unwrapped taps of the window at u: nodes c0 + j (j < W) with weights wt[j].
template <int W>
__device__ __forceinline__ void taps_unwrapped(double u, long long* c0, double* wt) {
  if constexpr (W == 1) {
    *c0 = (long long)floor(__dadd_rn(u, 0.5));
    wt[0] = 1.0;
  } else if constexpr (W == 2) {
    const double c = floor(u);
    const double d = __dsub_rn(u, c);
    *c0 = (long long)c;
    wt[0] = 1.0 - d;
    wt[1] = d;
  } else {
    const double c = floor(__dadd_rn(u, 0.5));
    const double d = __dsub_rn(u, c);
    *c0 = (long long)c - 1;
    const double a = 0.5 - d, b = 0.5 + d;
    wt[0] = 0.5 * a * a;
    wt[1] = 0.75 - d * d;
    wt[2] = 0.5 * b * b;
  }
}

// One tap into the LDS region: FP64 atomic add (FP64 meshes), or, for FP32 meshes, an
// integer add of the tap rounded to a multiple of 1/sc (fixed point; 64-bit integer LDS atomics
// are faster than FP64 ones on gfx950, and FP32 LDS atomics far slower).
// Deterministic mode (FIXED for FP64 too): every tap is rounded to a multiple of 1/sc of one
// scale shared by all tiles, so integer sums of the taps are exact in any order.
template <typename T, bool DET>
__device__ __forceinline__ void region_add(double* __restrict__ reg, int i, double v, double sc) {
  if constexpr (sizeof(T) == 4 || DET)
    lds_atomic_add<unsigned long long>(reinterpret_cast<unsigned long long*>(reg) + i,
                                       (unsigned long long)__double2ll_rn(v * sc));
  else
    lds_atomic_add<double>(reg + i, v);
}

template <typename T, int W, bool DET>
__device__ __forceinline__ void tile_scatter(double* __restrict__ reg, T* __restrict__ mesh,
                                             unsigned long long* __restrict__ acc, const double* u, double wgt,
                                             int nmesh, const long long* r0, int rsz, double sc) {
  long long c0[3];
  double w[3][W];
  taps_unwrapped<W>(u[0], &c0[0], w[0]);
  taps_unwrapped<W>(u[1], &c0[1], w[1]);
  taps_unwrapped<W>(u[2], &c0[2], w[2]);
  const int ra0 = (int)(c0[0] - r0[0]), rb0 = (int)(c0[1] - r0[1]), rc0 = (int)(c0[2] - r0[2]);
  const bool inside = ra0 >= 0 && ra0 + W <= rsz && rb0 >= 0 && rb0 + W <= rsz && rc0 >= 0 && rc0 + W <= rsz;
  if (inside) {
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const double wa = wgt * w[0][a];
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const double wab = wa * w[1][b];
        const int row = ((ra0 + a) * rsz + (rb0 + b)) * rsz + rc0;
#pragma unroll
        for (int c = 0; c < W; ++c) region_add<T, DET>(reg, row + c, wab * w[2][c], sc);
      }
    }
    return;
  }
  // a tap outside the LDS region (FP64 rounding at a cell face): straight to the mesh
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const double wa = wgt * w[0][a];
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const double wab = wa * w[1][b];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const size_t g = ((size_t)wrap(c0[0] + a, nmesh) * nmesh + wrap(c0[1] + b, nmesh)) * nmesh +
                         wrap(c0[2] + c, nmesh);
        if constexpr (DET)
          atomicAdd(&acc[g], (unsigned long long)__double2ll_rn(wab * w[2][c] * sc));
        else
          unsafeAtomicAdd(&mesh[g], (T)(wab * w[2][c]));
      }
    }
  }
}

// Per-axis reach of a window from a particle's base node b = floor(u): the plain mesh's taps
// lie on nodes b + LO1 .. b + LO1 + EXT1 - 1 + (0 .. ts - 1 over the tile's base nodes), the
// interlaced mesh's (taps of u + 1/2) on b + LO2 ..; so the LDS region of a tile of ts base
// nodes per axis is ts + EXT nodes wide from t0 + LO.  NGP: one tap at floor(u + 1/2), in
// {b, b + 1} (plain) and b + 1 (interlaced).  CIC: b, b + 1 (plain) and floor(u + 1/2) + {0, 1}
// within b .. b + 2.  TSC: floor(u + 1/2) + {-1, 0, 1} within b - 1 .. b + 2 (plain) and
// b + 1 + {-1, 0, 1} (interlaced).  A tap that FP64 rounding of u + 1/2 at a cell face moves
// outside goes to the mesh directly (tile_scatter).
template <int W> struct PaintReach;
template <> struct PaintReach<1> { static constexpr int LO1 = 0, EXT1 = 1, LO2 = 1, EXT2 = 0; };
template <> struct PaintReach<2> { static constexpr int LO1 = 0, EXT1 = 1, LO2 = 0, EXT2 = 2; };
template <> struct PaintReach<3> { static constexpr int LO1 = -1, EXT1 = 3, LO2 = 0, EXT2 = 2; };

// Add the non-zero cells of one LDS region (side N, origin t0 + LO) to the mesh with global
// atomics (or, DET, the integer sums to the 64-bit accumulators).
template <typename T, bool DET, int N, int LO>
__device__ __forceinline__ void flush_region(const double* __restrict__ reg, T* __restrict__ mesh,
                                             unsigned long long* __restrict__ acc, const int* t0, int nmesh,
                                             double isc) {
  for (int i = threadIdx.x; i < N * N * N; i += blockDim.x) {
    const long long q = reinterpret_cast<const long long*>(reg)[i];
    T v;
    if constexpr (sizeof(T) == 4 && !DET)
      v = (T)((double)q * isc);
    else
      v = (T)reg[i];
    if (DET ? q == 0 : v == T(0)) continue;
    // region node (ra, rb, rc) is mesh node t0 + LO + (ra, rb, rc), wrapped once at most
    const int rc = i % N, rb = (i / N) % N, ra = i / (N * N);
    int gx = t0[0] + LO + ra, gy = t0[1] + LO + rb, gz = t0[2] + LO + rc;
    gx += gx < 0 ? nmesh : (gx >= nmesh ? -nmesh : 0);
    gy += gy < 0 ? nmesh : (gy >= nmesh ? -nmesh : 0);
    gz += gz < 0 ? nmesh : (gz >= nmesh ? -nmesh : 0);
    const size_t g = ((size_t)gx * nmesh + gy) * nmesh + gz;
    if constexpr (DET)
      atomicAdd(&acc[g], (unsigned long long)q);
    else
      unsafeAtomicAdd(&mesh[g], v);
  }
}

// DET: the tiles' integer sums go to the 64-bit accumulators acc1 / acc2 (one per mesh) with
// integer atomics at the shared scale *gsc, instead of floating-point atomics to d1 / d2.
template <typename T, int W, int TS, bool DET>
__global__ void __launch_bounds__(256) k_paint_tiles(const int* __restrict__ off, const double4* __restrict__ payload,
                                                     double o0, double o1, double o2, double scale, int nmesh,
                                                     T* __restrict__ d1, T* __restrict__ d2,
                                                     const double* __restrict__ wmax_d,
                                                     const double* __restrict__ wmax_r, double alpha,
                                                     unsigned long long* __restrict__ acc1,
                                                     unsigned long long* __restrict__ acc2,
                                                     const double* __restrict__ gsc) {
  constexpr int ts = TS;
  using R = PaintReach<W>;
  constexpr int n1 = ts + R::EXT1, n2 = ts + R::EXT2;  // region sides of the two meshes
  extern __shared__ __align__(16) unsigned char smem[];
  // natural tile order: consecutive tiles land on different XCDs, which spreads the dense
  // survey region evenly (measured faster than XCD-local orders that keep halos in one L2)
  const int tile = blockIdx.x;
  const int start = off[tile], end = off[tile + 1];
  if (start == end) return;
  double* r1 = reinterpret_cast<double*>(smem);   // FP64 accumulation for both precisions
  double* r2 = r1 + n1 * n1 * n1;
  const bool two = d2 != nullptr;
  const int ncells = n1 * n1 * n1 + (two ? n2 * n2 * n2 : 0);
  for (int i = threadIdx.x; i < ncells; i += blockDim.x) r1[i] = 0.0;
  const int tpa = nmesh / ts;
  const int tz = tile % tpa, ty = (tile / tpa) % tpa, tx = tile / (tpa * tpa);
  const int t0[3] = {tx * ts, ty * ts, tz * ts};
  // fixed-point scale (FP32 meshes): no region cell can exceed B = (particles of the tile) x
  // (largest |payload weight|), since a particle's taps sum to its weight; B sc <= 2^61
  double sc = 1.0;
  if constexpr (DET) {
    sc = *gsc;
  } else if constexpr (sizeof(T) == 4) {
    const double wm = fmax(*wmax_d, wmax_r ? alpha * *wmax_r : 0.0);
    const double bound = (double)(end - start) * wm;
    int e = 0;
    if (bound > 0.0) (void)frexp(bound, &e);  // bound < 2^e
    sc = ldexp(1.0, 61 - e);
  }
  __syncthreads();
  for (int j = start + threadIdx.x; j < end; j += blockDim.x) {
    const double4 p = payload[j];
    const double wgt = p.w;
    double u[3];
    u[0] = __dmul_rn(__dsub_rn(p.x, o0), scale);
    u[1] = __dmul_rn(__dsub_rn(p.y, o1), scale);
    u[2] = __dmul_rn(__dsub_rn(p.z, o2), scale);
    // region origins (unwrapped, in this particle's frame): the tile origin t0 plus LO
    long long r01[3], r02[3];
    for (int a = 0; a < 3; ++a) {
      const long long cu = (long long)floor(u[a]);
      const long long base = cu - (wrap(cu, nmesh) - t0[a]);
      r01[a] = base + R::LO1;
      r02[a] = base + R::LO2;
    }
    tile_scatter<T, W, DET>(r1, d1, acc1, u, wgt, nmesh, r01, n1, sc);
    if (two) {
      u[0] = __dadd_rn(u[0], 0.5);
      u[1] = __dadd_rn(u[1], 0.5);
      u[2] = __dadd_rn(u[2], 0.5);
      tile_scatter<T, W, DET>(r2, d2, acc2, u, wgt, nmesh, r02, n2, sc);
    }
  }
  __syncthreads();
  const double isc = 1.0 / sc;  // a power of two: exact
  flush_region<T, DET, n1, R::LO1>(r1, d1, acc1, t0, nmesh, isc);
  if (two) flush_region<T, DET, n2, R::LO2>(r2, d2, acc2, t0, nmesh, isc);
}

// Deterministic mode: the shared fixed-point scale.  A node's value is a sum of taps of the
// particles whose base node lies within one window width of it, which belong to at most 8
// tiles (2 per axis for tiles of at least 3 nodes), so |value| <= B = 8 (largest tile count)
// (largest |payload weight|); sc = 2^(60 - e) with B < 2^e keeps every partial and total sum
// below 2^60 in magnitude.
__global__ void k_det_scale(const int* __restrict__ off, int ntiles, const double* __restrict__ wmax_d,
                            const double* __restrict__ wmax_r, double alpha, double* __restrict__ gsc) {
  __shared__ int s[256];
  int m = 0;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) m = max(m, off[t + 1] - off[t]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double wm = fmax(*wmax_d, wmax_r ? alpha * *wmax_r : 0.0);
    const double bound = 8.0 * (double)s[0] * wm;
    int e = 0;
    if (bound > 0.0) (void)frexp(bound, &e);
    *gsc = ldexp(1.0, 60 - e);
  }
}

// Deterministic mode: mesh value = accumulated integer / sc.
template <typename T>
__global__ void k_det_convert(const unsigned long long* __restrict__ acc, T* __restrict__ d, size_t n,
                              const double* __restrict__ gsc) {
  const double isc = 1.0 / *gsc;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    d[i] = (T)((double)(long long)acc[i] * isc);
}

}  // namespace

hipError_t launch_catalog_sums(const double* w, const double* nbar, int64_t n, double* partial, int nblk,
                               double* out2, double* wmax, hipStream_t s) {
  k_catalog_sums<<<nblk, SUM_THREADS, 0, s>>>(w, nbar, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials2<<<1, SUM_THREADS, 0, s>>>(partial, nblk, out2, wmax);
  return hipGetLastError();
}

template <typename T> hipError_t launch_fill(T* p, size_t n, T v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill<T><<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_tile_sort(const double* pos, int64_t n, int64_t base, const double* origin, double scale,
                            int nmesh, int ts, int* count, int* tile_of, int* rank, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 256 * CPT - 1) / (256 * CPT);
  if (blocks > 16384) blocks = 16384;
  const int tpa = nmesh / ts;
  k_tile_count<<<(unsigned)blocks, 256, 0, s>>>(pos, n, base, origin[0], origin[1], origin[2], scale, nmesh, ts,
                                                tpa * tpa * tpa, count, tile_of, rank);
  return hipGetLastError();
}

hipError_t launch_tile_offsets(int* count, int ntiles, int* off, const int* tile_of, const int* rank,
                               int64_t nd, int64_t ntot, const double* dpos, const double* dw, const double* rpos,
                               const double* rw, double alpha, void* payload, int* bsum, hipStream_t s) {
  const int nblk = (ntiles + SCAN_THREADS - 1) / SCAN_THREADS;
  k_scan_blocks<<<nblk, SCAN_THREADS, 0, s>>>(count, ntiles, off, bsum);
  k_scan_sums<<<1, SCAN_THREADS, 0, s>>>(bsum, nblk, off, ntiles);
  k_scan_add<<<nblk, SCAN_THREADS, 0, s>>>(bsum, ntiles, off, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ntot == 0) return e;
  int64_t blocks = (ntot + 256 * CPT - 1) / (256 * CPT);
  if (blocks > 16384) blocks = 16384;
  k_tile_scatter<<<(unsigned)blocks, 256, 0, s>>>(tile_of, rank, nd, ntot, ntiles, count, dpos, dw, rpos, rw,
                                                  alpha, (double4*)payload);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_paint_tiles(const int* off, const void* payload, int ntiles, const double* origin, double scale,
                              int nmesh, int window, int ts, T* d1, T* d2, const double* wmax_d,
                              const double* wmax_r, double alpha, hipStream_t s, unsigned long long* acc,
                              double* gsc) {
  const bool two = d2 != nullptr;
  int e1 = 0, e2 = 0;  // region sides ts + e1 (plain mesh) and ts + e2 (interlaced mesh)
  if (window == 1) { e1 = PaintReach<1>::EXT1; e2 = PaintReach<1>::EXT2; }
  else if (window == 2) { e1 = PaintReach<2>::EXT1; e2 = PaintReach<2>::EXT2; }
  else { e1 = PaintReach<3>::EXT1; e2 = PaintReach<3>::EXT2; }
  const size_t c1 = (size_t)(ts + e1) * (ts + e1) * (ts + e1), c2 = (size_t)(ts + e2) * (ts + e2) * (ts + e2);
  const size_t sm = sizeof(double) * (c1 + (two ? c2 : 0));
  const double4* pl = (const double4*)payload;
  unsigned long long* acc2 = (acc && two) ? acc + (size_t)nmesh * nmesh * nmesh : nullptr;
  if (acc) {
    k_det_scale<<<1, 256, 0, s>>>(off, ntiles, wmax_d, wmax_r, alpha, gsc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#define PKM_PAINT(WV, TV)                                                                                      \
  if (window == WV && ts == TV) {                                                                              \
    if (acc)                                                                                                   \
      k_paint_tiles<T, WV, TV, true><<<ntiles, 256, sm, s>>>(off, pl, origin[0], origin[1], origin[2], scale,  \
                                                             nmesh, d1, d2, wmax_d, wmax_r, alpha, acc, acc2,  \
                                                             gsc);                                            \
    else                                                                                                       \
      k_paint_tiles<T, WV, TV, false><<<ntiles, 256, sm, s>>>(off, pl, origin[0], origin[1], origin[2], scale, \
                                                              nmesh, d1, d2, wmax_d, wmax_r, alpha, nullptr,   \
                                                              nullptr, nullptr);                              \
    return hipGetLastError();                                                                                  \
  }
  PKM_PAINT(1, 4) PKM_PAINT(2, 4) PKM_PAINT(3, 4)
  PKM_PAINT(1, 8) PKM_PAINT(2, 8) PKM_PAINT(3, 8)
  PKM_PAINT(1, 16) PKM_PAINT(2, 16) PKM_PAINT(3, 16)
#undef PKM_PAINT
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_det_convert(const unsigned long long* acc, T* d1, T* d2, int nmesh, const double* gsc,
                              hipStream_t s) {
  const size_t n = (size_t)nmesh * nmesh * nmesh;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  k_det_convert<T><<<blocks, 256, 0, s>>>(acc, d1, n, gsc);
  if (d2) k_det_convert<T><<<blocks, 256, 0, s>>>(acc + n, d2, n, gsc);
  return hipGetLastError();
}

template hipError_t launch_paint_tiles<float>(const int*, const void*, int, const double*, double, int, int, int,
                                              float*, float*, const double*, const double*, double, hipStream_t,
                                              unsigned long long*, double*);
template hipError_t launch_paint_tiles<double>(const int*, const void*, int, const double*, double, int, int, int,
                                               double*, double*, const double*, const double*, double, hipStream_t,
                                               unsigned long long*, double*);
template hipError_t launch_det_convert<float>(const unsigned long long*, float*, float*, int, const double*,
                                              hipStream_t);
template hipError_t launch_det_convert<double>(const unsigned long long*, double*, double*, int, const double*,
                                               hipStream_t);
template hipError_t launch_fill<unsigned long long>(unsigned long long*, size_t, unsigned long long, hipStream_t);
template hipError_t launch_fill<float>(float*, size_t, float, hipStream_t);
template hipError_t launch_fill<int>(int*, size_t, int, hipStream_t);
template hipError_t launch_fill<double>(double*, size_t, double, hipStream_t);

}  // namespace pkm
