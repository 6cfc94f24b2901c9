// Transform passes of the multipole estimator (Sec. 2.1 eq. Pell-ours / eq. Fell, Sec. 2.3).
//
// Data layout.  A real mesh is R[x][y][z] (z contiguous).  A half spectrum is
// H[x][y][kz] with kz in [0, N/2) contiguous: the kz = N/2 plane is never stored because
// the combined field is zero on every Nyquist plane and those modes belong to no k bin.
// x and y indices are frequencies in FFT order (j < N/2 -> j, else j - N).
//
// Passes (each one read and one write of every element, tiles staged through LDS):
//   z pass   : real lines -> half-complex lines (length-N/2 complex FFT + split), optional
//              pre-pass: inverse z of G to the real field D_c, then Y_lm(xhat) weighting
//              and forward z for every field of a group.
//   column   : length-N transforms along y or x over tiles of `tile` adjacent kz columns.
//   xcombine : forward x of both painted meshes + interlace combine + compensation +
//              Nyquist zero, then inverse x of C.
//   xpost    : last transform of every field of a group (along y), sum_m Y_lm(khat) B_lm,
//              product with C, and binning into per-block partial sums.
// The weighted fields are kz-major, [kz][x][y] (kz planes of n n + fpad elements): the
// pre-pass writes them transposed, the field column pass runs along x within each kz plane,
// and the post-pass reads whole contiguous y lines.
// Both harmonic passes evaluate Y_lm for the direction turned by the plan's Frame (any
// orthogonal frame gives the same sums over m), or, with the CART flag, the monomials of
// the Cartesian decomposition.
//
// Every kernel takes two extra template constants: NC (mesh side) and TC (tile width, or
// lines per block for the z passes).  For the built-in shapes of the power-of-two meshes and
// of 384 and 768 (radix-3 schedules) the launchers instantiate them with the plan's values, so
// all index arithmetic and the radix schedule fold to constants; NC = TC = 0 selects the
// runtime-generic path used for the other sizes and shapes.
#include <algorithm>

#include "kernels.hpp"
#include "device_common.hpp"

namespace pkm {

namespace {

constexpr double FOUR_PI = 12.566370614359172953850573533118;
constexpr int ZPAD = 3;  // z-line LDS layout: one spare slot per 8 complex
__host__ __device__ constexpr int zpitch(int nh) { return nh + (nh >> ZPAD) + 1; }
constexpr int XPAD = 3;  // post-pass line exchange: one spare slot per 8 elements
__host__ __device__ constexpr int xrows(int n) { return n + (n >> XPAD) + 1; }
// z-pass blocks: up to 512 threads in FP32 (16 lines of 512: the pre-pass then writes
// 128-byte runs of y), 256 in FP64, whose pre-pass needs more than 256 registers per thread
// and so cannot hold two waves per SIMD
template <typename T> __host__ __device__ constexpr int zmax_threads() { return sizeof(T) == 4 ? 512 : 256; }
constexpr int XMAX_THREADS = 512;
constexpr int XPOST_THREADS = 256;

// Global-memory accesses through address-space-1 pointers (buffer pointers read from a
// device array would otherwise be generic and compile to flat instructions).
#define PKM_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ cx<T> gload(const cx<T>* p, size_t i) {
  const PKM_GLOBAL T* q = (const PKM_GLOBAL T*)(const void*)p;
  return mk<T>(q[2 * i], q[2 * i + 1]);
}
template <typename T> __device__ __forceinline__ void gstore(cx<T>* p, size_t i, cx<T> v) {
  PKM_GLOBAL T* q = (PKM_GLOBAL T*)(void*)p;
  q[2 * i] = v.x;
  q[2 * i + 1] = v.y;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Remap so
// that consecutive logical tiles (which share 128-byte rows when a tile is narrower than
// that, and neighbouring rows otherwise) run on the same XCD one after the other.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  if (nblk % 8) return b;
  return (b % 8) * (nblk / 8) + b / 8;
}

// Copy the twiddle table into LDS (n entries); returns the LDS copy.
template <typename T>
__device__ __forceinline__ cx<T>* stage_twiddles(cx<T>* dst, const cx<T>* __restrict__ tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = tw[i];
  return dst;
}

__device__ __forceinline__ int tdiv(int i, int tile) { return (tile & (tile - 1)) == 0 ? i >> (__ffs(tile) - 1) : i / tile; }
__device__ __forceinline__ int tmod(int i, int tile) { return (tile & (tile - 1)) == 0 ? i & (tile - 1) : i % tile; }

// Tile of `tile` adjacent kz columns x n rows: element i = tid + j*bs (j < E) of the tile is
// row i / tile, column i % tile.  All E loads are issued before any is consumed.  With
// RPAD > 0 the LDS row index is padded (one spare row per 2^RPAD rows).
template <typename T, int E>
__device__ __forceinline__ void tile_load(cx<T>* v, const cx<T>* __restrict__ g, size_t base, size_t rs, int tile,
                                          int bs) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = threadIdx.x + j * bs;
    v[j] = gload<T>(g, base + (size_t)tdiv(i, tile) * rs + tmod(i, tile));
  }
}
template <typename T, int E, int RPAD>
__device__ __forceinline__ void tile_to_lds(cx<T>* lds, const cx<T>* v, int tile, int pitch, int bs) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = threadIdx.x + j * bs;
    lds[padi<RPAD>(tdiv(i, tile)) * pitch + tmod(i, tile)] = v[j];
  }
}
// G contiguous lines of nh complex: element i = tid + j*bs is line i / nh, entry i % nh.
template <typename T, int E>
__device__ __forceinline__ void lines_to_lds(cx<T>* lds, const cx<T>* __restrict__ src, int nh, int lp, int bs) {
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = gload<T>(src, threadIdx.x + j * bs);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = threadIdx.x + j * bs;
    lds[tdiv(i, nh) * lp + padi<ZPAD>(tmod(i, nh))] = v[j];
  }
}

// Runtime description of one line transform (generic path).
struct LineRt {
  int L;           // line length
  uint32_t sched;  // radix schedule
  int nst;
  int pt;          // threads per line
  int ntw;         // entries of the W_ntw^j table
};

// Line transform with the line in registers on entry and exit (element e = position
// t + pt*e).  LC > 0: compile-time schedule (WAVE = the line lies inside one wavefront);
// LC = 0: generic schedule through the LDS line, block-wide barriers.
template <typename T, int E, bool INV, int PAD, int LC, bool WAVE>
__device__ __forceinline__ void xf_regs(cx<T>* lds, int off, int es, const LineRt& rt, int t, cx<T>* u,
                                        const cx<T>* twst, const cx<T>* __restrict__ twl) {
  if constexpr (LC > 0) {
    ct_fft_regs<T, E, INV, PAD, LC, WAVE>(lds, off, es, t, u, twst);
  } else {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) lds[off + padi<PAD>(t + rt.pt * e) * es] = u[e];
    __syncthreads();
    lds_fft<T, E, INV, PAD>(lds, off, es, rt.L, rt.sched, rt.nst, t, rt.pt, twl, rt.ntw);
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = lds[off + padi<PAD>(t + rt.pt * e) * es];
  }
}
// Same with the input line already in LDS (filled, and a block barrier since).
template <typename T, int E, bool INV, int PAD, int LC, bool WAVE>
__device__ __forceinline__ void xf_lds_in(cx<T>* lds, int off, int es, const LineRt& rt, int t, cx<T>* u,
                                          const cx<T>* twst, const cx<T>* __restrict__ twl) {
  if constexpr (LC > 0) {
    ct_fft_lds_in<T, E, INV, PAD, LC, WAVE>(lds, off, es, t, u, twst);
  } else {
    lds_fft<T, E, INV, PAD>(lds, off, es, rt.L, rt.sched, rt.nst, t, rt.pt, twl, rt.ntw);
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = lds[off + padi<PAD>(t + rt.pt * e) * es];
  }
}
// LDS entries of the per-stage twiddle table (compile-time path only).
template <int E, int LC> __host__ __device__ constexpr int twst_size() { return LC > 0 ? ct_tw_total(E, LC) : 0; }

// Forward split of a packed half-length transform: X_k = E_k + W_N^k O_k.
template <typename T>
__device__ __forceinline__ cx<T> r2c_split(const cx<T>* line, int k, int nh, const cx<T>* __restrict__ tw) {
  const cx<T> zk = line[padi<ZPAD>(k)];
  const cx<T> zm = cconj<T>(line[padi<ZPAD>(k == 0 ? 0 : nh - k)]);
  const cx<T> e = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y));
  const cx<T> d = mk<T>(T(0.5) * (zk.x - zm.x), T(0.5) * (zk.y - zm.y));
  const cx<T> o = mk<T>(d.y, -d.x);  // d / i
  return cadd<T>(e, cmul<T>(tw[k], o));
}

// Inverse split: Z_k = E_k + i O_k with E_k = (X_k + conj X_{nh-k})/2,
// O_k = (X_k - conj X_{nh-k}) conj(W_N^k) / 2; X_{nh} = 0 and X_0 taken real.
template <typename T>
__device__ __forceinline__ cx<T> c2r_split(const cx<T>* line, int k, int nh, const cx<T>* __restrict__ tw) {
  cx<T> xk = line[padi<ZPAD>(k)];
  cx<T> xp;
  if (k == 0) {
    xk.y = T(0);
    xp = mk<T>(T(0), T(0));
  } else {
    xp = cconj<T>(line[padi<ZPAD>(nh - k)]);
  }
  const cx<T> e = mk<T>(T(0.5) * (xk.x + xp.x), T(0.5) * (xk.y + xp.y));
  const cx<T> d = mk<T>(T(0.5) * (xk.x - xp.x), T(0.5) * (xk.y - xp.y));
  const cx<T> o = cmul<T>(d, cconj<T>(tw[k]));
  return mk<T>(e.x - o.y, e.y + o.x);  // e + i o
}

__device__ __forceinline__ int sfreq(int j, int n) { return j < (n >> 1) ? j : j - n; }

// Histogram in LDS: `copies` copies of nvals doubles; wave w uses copy w % copies.
__device__ __forceinline__ void hist_zero(double* h, int total) {
  for (int i = threadIdx.x; i < total; i += blockDim.x) h[i] = 0.0;
}
__device__ __forceinline__ void hist_flush(const double* h, int copies, int nvals, double* out) {
  for (int v = threadIdx.x; v < nvals; v += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < copies; ++c) s += h[c * nvals + v];
    out[v] = s;
  }
}

// ------------------------------------------------------------------------------------------
// z pass, forward (real -> half complex)
// ------------------------------------------------------------------------------------------
// LDS of the z passes: G padded lines, the W_N^j table (N entries; the splits read the
// first N/2), and on the compile-time path the per-stage table of the length-N/2 transform.
template <typename T, int E, int NC, int TC>
__global__ void __launch_bounds__(zmax_threads<T>()) k_zfwd(int n_rt, int g_rt, uint32_t sched, int nst,
                                                        const T* __restrict__ in0, const T* __restrict__ in1,
                                                        void* __restrict__ out0, void* __restrict__ out1,
                                                        const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int n = NC > 0 ? NC : n_rt;
  const int G = TC > 0 ? TC : g_rt;
  const int nh = n >> 1;
  const int lp = zpitch(nh);
  const int pt = nh / E;
  const int bs = pt * G;
  constexpr bool WAVE = NC > 0 && NC / 2 / E <= 64;
  const T* in = blockIdx.y ? in1 : in0;
  void* out = blockIdx.y ? out1 : out0;
  const size_t line0 = (size_t)blockIdx.x * G;
  const int tid = threadIdx.x;
  cx<T>* twl = stage_twiddles<T>(lds + (size_t)G * lp, tw, n);
  cx<T>* twst = twl + n;
  if constexpr (NC > 0) ct_twiddles<T, E, NC / 2, NC>(twst, tw);
  lines_to_lds<T, E>(lds, reinterpret_cast<const cx<T>*>(in) + line0 * nh, nh, lp, bs);
  __syncthreads();
  const int t = tid % pt, g = tid / pt;
  cx<T>* line = lds + g * lp;
  if constexpr (NC > 0) {
    cx<T> u[E];
    ct_fft_lds_in<T, E, false, ZPAD, NC / 2, WAVE>(lds, g * lp, 1, t, u, twst);
#pragma unroll
    for (int e = 0; e < E; ++e) line[padi<ZPAD>(t + pt * e)] = u[e];
    ct_sync<WAVE>();
  } else {
    lds_fft<T, E, false, ZPAD>(lds, g * lp, 1, nh, sched, nst, t, pt, twl, n);
  }
  const size_t ob = (line0 + g) * nh;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + pt * e;
    gstore<T>((cx<T>*)out, ob + k, r2c_split<T>(line, k, nh, twl));
  }
}

// ------------------------------------------------------------------------------------------
// column pass (length N along y or x), in place.  Lane c = tid % tile, t = tid / tile: the
// tile load leaves rows t + pt*e of column c in the thread's registers, which is the
// transform's own register layout, so LDS is used only between radix stages.  Tiles run over
// the contiguous axis (clen elements: N/2 kz of a half spectrum, N y of a kz-major field
// buffer) within each outer plane.
// ------------------------------------------------------------------------------------------
template <typename T, int E, bool INV, int NC, int TC>
__global__ void __launch_bounds__(XMAX_THREADS) k_col(int n_rt, int tile_rt, uint32_t sched, int nst,
                                                       void* const* __restrict__ bufs, size_t row_stride,
                                                       size_t outer_stride, int clen, const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int n = NC > 0 ? NC : n_rt;
  const int tile = TC > 0 ? TC : tile_rt;
  const int pt = n / E;
  const int bs = pt * tile;
  const int tiles = clen / tile;
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int outer = blk / tiles;
  const int c0 = (blk % tiles) * tile;
  cx<T>* buf = reinterpret_cast<cx<T>*>(bufs[blockIdx.y]);
  const size_t base = (size_t)outer * outer_stride + c0;
  const int pitch = tile + 1;
  const int tid = threadIdx.x;
  const int c = tid % tile, t = tid / tile;
  cx<T> u[E];
  tile_load<T, E>(u, buf, base, row_stride, tile, bs);
  // generic path: the W_N^j table; compile-time path: the per-stage table only
  cx<T>* twl = lds + (size_t)n * pitch;
  cx<T>* twst = twl;
  if constexpr (NC > 0) ct_twiddles<T, E, NC, NC>(twst, tw); else stage_twiddles<T>(twl, tw, n);
  const LineRt rt{n, sched, nst, pt, n};
  xf_regs<T, E, INV, 0, NC, false>(lds, c, pitch, rt, t, u, twst, twl);
#pragma unroll
  for (int e = 0; e < E; ++e) gstore<T>(buf, base + (size_t)(t + pt * e) * row_stride + c, u[e]);
}

// ------------------------------------------------------------------------------------------
// x pass of the painted meshes + combine + inverse x of C (same lane layout as k_col)
// ------------------------------------------------------------------------------------------
template <typename T, int E, int NC, int TC>
__global__ void __launch_bounds__(XMAX_THREADS) k_xcombine(int n_rt, int tile_rt, uint32_t sched, int nst,
                                                            const cx<T>* __restrict__ s1, const cx<T>* __restrict__ s2,
                                                            cx<T>* __restrict__ cout, cx<T>* __restrict__ gout,
                                                            int interlaced, int compensated,
                                                            const T* __restrict__ invw,
                                                            const cx<T>* __restrict__ phase,
                                                            const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = NC > 0 ? NC : n_rt;
  const int tile = TC > 0 ? TC : tile_rt;
  const int nh = n >> 1;
  const int pitch = tile + 1;
  const int pt = n / E;
  const int bs = pt * tile;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int tiles = nh / tile;
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int y = blk / tiles;
  const int kz0 = (blk % tiles) * tile;
  const size_t rs = (size_t)n * nh;
  const size_t base = (size_t)y * nh + kz0;
  const int tid = threadIdx.x;
  const int c = tid % tile, t = tid / tile;
  const int kz = kz0 + c;
  cx<T> a1[E];
  cx<T> a2[E];
  tile_load<T, E>(a1, s1, base, rs, tile, bs);
  if (interlaced) tile_load<T, E>(a2, s2, base, rs, tile, bs);
  // generic path: the W_N^j table; compile-time path: the per-stage table only
  cx<T>* twl = lds + (size_t)n * pitch;
  cx<T>* twst = twl;
  if constexpr (NC > 0) ct_twiddles<T, E, NC, NC>(twst, tw); else stage_twiddles<T>(twl, tw, n);
  const LineRt rt{n, sched, nst, pt, n};
  xf_regs<T, E, false, 0, NC, false>(lds, c, pitch, rt, t, a1, twst, twl);
  if (interlaced) {
    xf_regs<T, E, false, 0, NC, false>(lds, c, pitch, rt, t, a2, twst, twl);
    const cx<T> pyz = cmul<T>(phase[y], phase[kz]);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + pt * e;
      const cx<T> b = cmul<T>(a2[e], cmul<T>(phase[x], pyz));
      a1[e] = mk<T>(T(0.5) * (a1[e].x + b.x), T(0.5) * (a1[e].y + b.y));
    }
  }
  const bool ynyq = (y == nh);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = t + pt * e;
    cx<T> v = a1[e];
    if (compensated) v = cscale<T>(v, invw[x] * invw[y] * invw[kz]);
    if (ynyq || x == nh) v = mk<T>(T(0), T(0));
    a1[e] = v;
    gstore<T>(cout, base + c + (size_t)x * rs, v);
  }
  if (gout == nullptr) return;
  xf_regs<T, E, true, 0, NC, false>(lds, c, pitch, rt, t, a1, twst, twl);
#pragma unroll
  for (int e = 0; e < E; ++e) gstore<T>(gout, base + (size_t)(t + pt * e) * rs + c, a1[e]);
}

// ------------------------------------------------------------------------------------------
// z pre-pass: D_c from G (inverse z), then weighted forward z for every field of the group.
// Fields come |m|-major (the table order) so the harmonic recurrence continues across them.
// Each line is transformed by the threads of one wavefront (compile-time path).  A block holds
// G lines of one x plane (consecutive y); the finished lines of a field are parked in a second
// LDS region and written transposed into the kz-major field buffer [kz][x][y], G consecutive
// y per piece (the post-pass then reads whole y lines).
// ------------------------------------------------------------------------------------------
template <typename T, int E, int NC, int TC, bool CART = false>
__global__ void __launch_bounds__(zmax_threads<T>()) k_zpre(int n_rt, int g_rt, uint32_t sched, int nst,
                                                        const cx<T>* __restrict__ gin, const T* __restrict__ real_in,
                                                        T* __restrict__ real_out, void* const* __restrict__ bufs,
                                                        int nf, const int* __restrict__ fields, T scale, double off0,
                                                        double off1, double off2, double h,
                                                        const T* __restrict__ ytab, const cx<T>* __restrict__ tw,
                                                        Frame fr, int fpad) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int n = NC > 0 ? NC : n_rt;
  const int G = TC > 0 ? TC : g_rt;
  const int nh = n >> 1;
  const int lp = zpitch(nh);
  const int pt = nh / E;
  const int bs = pt * G;
  constexpr bool WAVE = NC > 0 && NC / 2 / E <= 64;
  const size_t line0 = (size_t)blockIdx.x * G;
  const int tid = threadIdx.x;
  const int t = tid % pt, g = tid / pt;
  const size_t lineg = line0 + g;
  cx<T>* line = lds + g * lp;
  // two line regions alternate between fields: field f is transformed and parked in region
  // f mod 2 while the transposed writes of field f - 1 may still read the other one
  const size_t region = (size_t)G * lp;
  cx<T>* twl = stage_twiddles<T>(lds + 2 * region, tw, n);
  cx<T>* twst = twl + n;
  if constexpr (NC > 0) ct_twiddles<T, E, NC / 2, NC>(twst, tw);
  const LineRt rt{nh, sched, nst, pt, n};
  T r[2 * E];
  if (real_in) {
    const cx<T>* src = reinterpret_cast<const cx<T>*>(real_in) + lineg * nh;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<T> v = gload<T>(src, t + pt * e);
      r[2 * e] = v.x;
      r[2 * e + 1] = v.y;
    }
    __syncthreads();
  } else {
    lines_to_lds<T, E>(lds, gin + line0 * nh, nh, lp, bs);
    __syncthreads();
    cx<T> z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = c2r_split<T>(line, t + pt * e, nh, twl);
    xf_regs<T, E, true, ZPAD, NC / 2, WAVE>(lds, g * lp, 1, rt, t, z, twst, twl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      r[2 * e] = z[e].x * scale;
      r[2 * e + 1] = z[e].y * scale;
    }
    if (real_out) {
      cx<T>* dst = reinterpret_cast<cx<T>*>(real_out) + lineg * nh;
#pragma unroll
      for (int e = 0; e < E; ++e) gstore<T>(dst, t + pt * e, mk<T>(r[2 * e], r[2 * e + 1]));
    }
  }
  if (nf == 0) return;
  // unit vectors from the observer to this thread's nodes (x, y fixed by the line), formed
  // in FP64 and rounded once: in FP32 the distance to a far observer rounds the same way for
  // whole planes of nodes, and the slope of high-degree harmonics near the pole would turn
  // that common bias into a systematic error of the multipoles
  const int ix = (int)(lineg / n), iy = (int)(lineg % n);
  const double px = off0 + ix * h, py = off1 + iy * h;
  const double pxy2 = px * px + py * py;
  // a node at the observer has no direction: its weighted value is zero for every field
  T ux[2 * E], uy[2 * E], uz[2 * E];
#pragma unroll
  for (int q = 0; q < 2 * E; ++q) {
    const double pz = off2 + (2 * (t + pt * (q >> 1)) + (q & 1)) * h;
    const double rr = sqrt(pxy2 + pz * pz);
    const bool zero = !(rr > 0.0);
    const double inv = zero ? 0.0 : 1.0 / rr;
    const double vx = px * inv, vy = py * inv, vz = pz * inv;
    ux[q] = (T)(fr.r[0] * vx + fr.r[1] * vy + fr.r[2] * vz);
    uy[q] = (T)(fr.r[3] * vx + fr.r[4] * vy + fr.r[5] * vz);
    uz[q] = (T)(fr.r[6] * vx + fr.r[7] * vy + fr.r[8] * vz);
    if (zero) r[q] = T(0);
  }
  // the block's lines: x plane bx, y = by0 .. by0 + G - 1 (G divides n)
  const int bx = (int)(line0 / n), by0 = (int)(line0 % n);
  const size_t fplane = (size_t)n * n + fpad;
  const size_t fo = (size_t)bx * n + by0;
  YRun<T, 2 * E> yr;
  yrun_init(yr);
  for (int f = 0; f < nf; ++f) {
    T yv[2 * E];
    if constexpr (CART)
      monomial_eval<T, 2 * E>(fields[4 * f + 1], fields[4 * f + 2], T(1), ux, uy, uz, yv);
    else
      yrun_eval<T, 2 * E>(yr, fields[4 * f + 1], fields[4 * f + 2], ux, uy, uz, yv, ytab);
    cx<T> u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = mk<T>(r[2 * e] * yv[2 * e], r[2 * e + 1] * yv[2 * e + 1]);
    cx<T>* park = lds + (f & 1) * region;
    xf_regs<T, E, false, ZPAD, NC / 2, WAVE>(park, g * lp, 1, rt, t, u, twst, twl);
    // park the line where its transform ran (the threads of the line have finished reading
    // those slots), then every thread writes G consecutive y of one kz: the split needs X_k
    // and X_{nh-k} of a line.  The barrier also orders the last reads of this region by the
    // transposed writes of field f - 2 before this field's transform reused it.
    if constexpr (WAVE) ct_sync<true>(); else __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) park[g * lp + padi<ZPAD>(t + pt * e)] = u[e];
    __syncthreads();
    cx<T>* out = reinterpret_cast<cx<T>*>(bufs[fields[4 * f]]);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int o = tid + e * bs;
      const int gg = tmod(o, G), k = tdiv(o, G);
      gstore<T>(out, (size_t)k * fplane + fo + gg, r2c_split<T>(park + gg * lp, k, nh, twl));
    }
  }
}

// ------------------------------------------------------------------------------------------
// post-pass: the last transform of every field, along y (kz-major field buffers hold whole y
// lines), sum_m Y_lm(khat) B, product with C, binning.  A tile is TP lines of one x plane,
// kz = kz0 .. kz0 + TP - 1; thread (t, c) transforms line c and holds y = t + pt e, the
// transform's own register layout, so each line is loaded straight into registers (whole
// contiguous lines, the next field prefetched during the current one) and LDS carries only the
// stage exchanges (within one wavefront on the compile-time path), the tile's C and the
// histograms.  Fields come l-major (slots contiguous): one complex accumulator per element holds
// sum_m Y_lm(khat) B_lm of the current slot and is folded against C into the FP64 bins at the
// slot's last field.
// ------------------------------------------------------------------------------------------
// LDS entries (complex) before the histograms: exchanges, the tile's C, twiddles.
template <typename T, int E, int NC>
__host__ __device__ constexpr size_t xpost_elems(int n, int tp) {
  return (size_t)tp * xrows(n) + (size_t)tp * n + (NC > 0 ? twst_size<E, NC>() : n);
}

// Tiles of a persistent post-pass block.  When the tile count and the grid are multiples of
// 8, block b (dispatched to XCD b mod 8) walks a contiguous eighth of the tiles, so the
// blocks of one XCD work on neighbouring tiles (which share 128-byte rows) at the same time.
struct TileWalk {
  int ntiles, first, step, end, chunk0;
  __device__ TileWalk(int nt) : ntiles(nt) {
    const int G = gridDim.x, b = blockIdx.x;
    if (nt % 8 == 0 && G % 8 == 0 && G <= nt) {
      const int per = nt / 8;
      chunk0 = (b % 8) * per;
      first = b / 8;
      step = G / 8;
      end = per;
    } else {
      chunk0 = 0;
      first = b;
      step = G;
      end = nt;
    }
  }
  __device__ int tile(int j) const { return chunk0 + j; }
};

// k bins of E elements at once from thresholds in LDS: all searches step together, so the
// LDS reads of the E elements overlap.  -1 for modes outside [thr[0], thr[nb]) or excluded.
template <int E>
__device__ __forceinline__ void kbins_lds(const long long* thr, int nb, const int* n2, const bool* excl, int* bin) {
  int lo[E], hi[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    lo[e] = 0;
    hi[e] = nb;
  }
  for (int w = nb; w > 1; w = (w + 1) >> 1) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int mid = (lo[e] + hi[e]) >> 1;
      if (hi[e] - lo[e] > 1) {
        if (thr[mid] <= (long long)n2[e]) lo[e] = mid;
        else hi[e] = mid;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool in = !excl[e] && (long long)n2[e] >= thr[0] && (long long)n2[e] < thr[nb];
    bin[e] = in ? lo[e] : -1;
  }
}

template <typename T, int E, int NC, int TC, bool CART = false>
__global__ void __launch_bounds__(XPOST_THREADS) k_xpost(int n_rt, int tp_rt, uint32_t sched, int nst,
                                                          void* const* __restrict__ bufs, int nf,
                                                          const int* __restrict__ fields, int nslots, int with_l0,
                                                          double kf, const cx<T>* __restrict__ cin,
                                                          const T* __restrict__ ytab,
                                                          const long long* __restrict__ thr, int nb, int copies,
                                                          double* __restrict__ partial,
                                                          const cx<T>* __restrict__ tw, Frame frm, int fpad) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = NC > 0 ? NC : n_rt;
  const int TP = TC > 0 ? TC : tp_rt;
  const int nh = n >> 1;
  const int pt = n / E;
  const int bs = pt * TP;
  constexpr bool WAVE = NC > 0 && NC / E <= 64;
  const int lx = xrows(n);  // padded length of a line's exchange region
  cx<T>* exch = reinterpret_cast<cx<T>*>(smem);
  cx<T>* cst = exch + (size_t)TP * lx;  // C of the tile, [line][y]
  cx<T>* twl = cst + (size_t)TP * n;
  cx<T>* twst = twl;
  double* hist = reinterpret_cast<double*>(smem + sizeof(cx<T>) * xpost_elems<T, E, NC>(n, TP));
  const int l0rows = with_l0 ? 3 : 0;
  const int nvals = (l0rows + nslots) * nb;
  long long* thr_l = reinterpret_cast<long long*>(hist + (size_t)copies * nvals);
  hist_zero(hist, copies * nvals);
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) thr_l[i] = thr[i];
  if constexpr (NC > 0) ct_twiddles<T, E, NC, NC>(twst, tw); else stage_twiddles<T>(twl, tw, n);
  const int kgroups = nh / TP;
  const size_t fplane = (size_t)n * n + fpad;   // kz plane of a field buffer
  const size_t cplane = (size_t)n * nh;         // x plane of C
  const int tid = threadIdx.x;
  // rows fastest across the lanes of a wave: a line's transform stays inside one wave
  const int t = tid % pt, c = tid / pt;
  double* h = hist + ((tid >> 6) % copies) * nvals;
  const LineRt rt{n, sched, nst, pt, n};
  const TileWalk walk(n * kgroups);
  // first element of this thread's line in a field buffer: kz = kz0 + c of x plane x
  auto fline = [&](int tl) {
    return (size_t)((tl % kgroups) * TP + c) * fplane + (size_t)(tl / kgroups) * n + t;
  };
  cx<T> nxt[E];
  int j = walk.first;
  if (j < walk.end && nf > 0) {
    const cx<T>* b0 = reinterpret_cast<const cx<T>*>(bufs[fields[0]]);
    const size_t fb0 = fline(walk.tile(j));
#pragma unroll
    for (int e = 0; e < E; ++e) nxt[e] = gload<T>(b0, fb0 + pt * e);
  }
  for (; j < walk.end; j += walk.step) {
    const int tl = walk.tile(j);
    const int x = tl / kgroups, kz0 = (tl % kgroups) * TP;
    const int kz = kz0 + c;
    const size_t fb = fline(tl);
    // C of the tile: TP consecutive kz per y row (coalesced), kept in LDS for the whole tile
    __syncthreads();  // previous tile's reads of cst done; first tile: histograms, thresholds, twiddles staged
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int i = tid + q * bs;
      const int y = tdiv(i, TP), cc = tmod(i, TP);
      cst[cc * n + y] = gload<T>(cin, (size_t)x * cplane + (size_t)y * nh + kz0 + cc);
    }
    __syncthreads();
    const int fx = sfreq(x, n);
    const bool xnyq = (x == nh);
    // Hermitian weight; the spherical sum also carries the 4 pi of the addition theorem
    const double w4pi = ((kz == 0) ? 1.0 : 2.0) * (CART ? 1.0 : FOUR_PI);
    // per element: k bin (-1 when the mode is excluded) and unit wave vector
    int bin[E];
    T ux[E], uy[E], uz[E];
    {
      int n2[E];
      bool excl[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int y = t + pt * e;
        const int fy = sfreq(y, n);
        n2[e] = fx * fx + fy * fy + kz * kz;
        excl[e] = xnyq || y == nh || n2[e] == 0;
        // wave vectors cover every direction, so their rounding is not correlated: the
        // rotation runs in the working precision
        const T ki = n2[e] > 0 ? T(1) / sqrt((T)n2[e]) : T(0);
        const T vx = (T)fx * ki, vy = (T)fy * ki, vz = (T)kz * ki;
        ux[e] = frm.at<T>(0) * vx + frm.at<T>(1) * vy + frm.at<T>(2) * vz;
        uy[e] = frm.at<T>(3) * vx + frm.at<T>(4) * vy + frm.at<T>(5) * vz;
        uz[e] = frm.at<T>(6) * vx + frm.at<T>(7) * vy + frm.at<T>(8) * vz;
      }
      kbins_lds<E>(thr_l, nb, n2, excl, bin);
    }
    cx<T> acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = mk<T>(T(0), T(0));
    YRun<T, E> yr;
    yrun_init(yr);
    for (int f = 0; f < nf; ++f) {
      cx<T> u[E];
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = nxt[e];
      // prefetch the next field's line (or the next tile's first field) during this one
      if (f + 1 < nf) {
        const cx<T>* bn = reinterpret_cast<const cx<T>*>(bufs[fields[4 * (f + 1)]]);
#pragma unroll
        for (int e = 0; e < E; ++e) nxt[e] = gload<T>(bn, fb + pt * e);
      } else if (j + walk.step < walk.end) {
        const cx<T>* bn = reinterpret_cast<const cx<T>*>(bufs[fields[0]]);
        const size_t fbn = fline(walk.tile(j + walk.step));
#pragma unroll
        for (int e = 0; e < E; ++e) nxt[e] = gload<T>(bn, fbn + pt * e);
      }
      xf_regs<T, E, false, XPAD, NC, WAVE>(exch, c * lx, 1, rt, t, u, twst, twl);
      const int slot = fields[4 * f + 3];
      {
        T yv[E];
        if constexpr (CART)
          monomial_eval<T, E>(fields[4 * f + 1], fields[4 * f + 2], (T)multinomial(fields[4 * f + 1], fields[4 * f + 2]),
                              ux, uy, uz, yv);
        else
          yrun_eval<T, E, false>(yr, fields[4 * f + 1], fields[4 * f + 2], ux, uy, uz, yv, ytab);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = mk<T>(acc[e].x + yv[e] * u[e].x, acc[e].y + yv[e] * u[e].y);
      }
      if (f + 1 == nf || fields[4 * (f + 1) + 3] != slot) {
        double* hs = h + (l0rows + slot) * nb;
        // even l: Re[C conj acc]; odd l (spherical basis only): Im[C conj acc], the part of
        // the shell average that survives when a mode and its mirror are summed
        const bool odd = !CART && (fields[4 * f + 1] & 1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (bin[e] >= 0) {
            const cx<T> cv = cst[c * n + t + pt * e];
            const double q = odd ? (double)cv.y * (double)acc[e].x - (double)cv.x * (double)acc[e].y
                                 : (double)cv.x * (double)acc[e].x + (double)cv.y * (double)acc[e].y;
            lds_atomic_add<double>(&hs[bin[e]], w4pi * q);
          }
          acc[e] = mk<T>(T(0), T(0));
        }
      }
    }
    if (with_l0) {
      const double w = (kz == 0) ? 1.0 : 2.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (bin[e] < 0) continue;
        const int y = t + pt * e;
        const int fy = sfreq(y, n);
        const int n2 = fx * fx + fy * fy + kz * kz;
        const cx<T> cv = cst[c * n + y];
        lds_atomic_add<double>(&h[bin[e]], w);
        lds_atomic_add<double>(&h[nb + bin[e]], w * kf * sqrt((double)n2));
        lds_atomic_add<double>(&h[2 * nb + bin[e]], w * ((double)cv.x * (double)cv.x + (double)cv.y * (double)cv.y));
      }
    }
  }
  __syncthreads();
  hist_flush(hist, copies, nvals, partial + (size_t)blockIdx.x * nvals);
}

// ------------------------------------------------------------------------------------------
// fixed-order reduction of per-block partial sums
// ------------------------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
__global__ void __launch_bounds__(RED_THREADS) k_reduce(const double* __restrict__ partial, int nblocks, int nvals,
                                                        double* __restrict__ out, const int* __restrict__ map,
                                                        int accumulate) {
  __shared__ double s[RED_THREADS];
  const int v = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) a += partial[(size_t)b * nvals + v];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int hh = RED_THREADS / 2; hh > 0; hh >>= 1) {
    if ((int)threadIdx.x < hh) s[threadIdx.x] += s[threadIdx.x + hh];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int o = map ? map[v] : v;
    out[o] = accumulate ? out[o] + s[0] : s[0];
  }
}

// ------------------------------------------------------------------------------------------
// global line of sight (k, mu) binning of |C|^2
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_kmu(int n, const cx<T>* __restrict__ cin, double l0, double l1, double l2,
                      const long long* __restrict__ thr, int nb, const double* __restrict__ mue, int nmu,
                      double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* hist = reinterpret_cast<double*>(smem);
  const int nvals = 2 * nb * nmu;
  hist_zero(hist, nvals);
  __syncthreads();
  const int nh = n >> 1;
  const size_t total = (size_t)n * n * nh;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int kz = (int)(i % nh);
    const size_t xy = i / nh;
    const int y = (int)(xy % n), x = (int)(xy / n);
    if (x == nh || y == nh) continue;
    const int fx = sfreq(x, n), fy = sfreq(y, n);
    const long long n2 = (long long)fx * fx + (long long)fy * fy + (long long)kz * kz;
    if (n2 == 0) continue;
    const int kb = kbin_of(n2, thr, nb);
    if (kb < 0) continue;
    const double dot = __dadd_rn(__dadd_rn(__dmul_rn((double)fx, l0), __dmul_rn((double)fy, l1)),
                                 __dmul_rn((double)kz, l2));
    const double mu = __ddiv_rn(fabs(dot), __dsqrt_rn((double)n2));
    // mu bin: last edge <= mu -> last bin; else largest j with mue[j] <= mu
    int mb;
    if (mu >= mue[nmu]) mb = nmu - 1;
    else if (mu < mue[0]) mb = -1;
    else {
      int lo = 0, hi = nmu;
      while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (mue[mid] <= mu) lo = mid; else hi = mid; }
      mb = lo;
    }
    if (mb < 0) continue;
    const cx<T> v = cin[i];
    const double p2 = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    const double omega = (kz == 0) ? 1.0 : 2.0;
    const int cell = kb * nmu + mb;
    lds_atomic_add<double>(&hist[2 * cell], omega);
    lds_atomic_add<double>(&hist[2 * cell + 1], omega * p2);
  }
  __syncthreads();
  hist_flush(hist, 1, nvals, partial + (size_t)blockIdx.x * nvals);
}

// Normalisation of reduced (k, mu) sums on the device, FP64 with explicitly rounded
// operations (the host form of the same formula gives identical bits):
// pk[i] = sum_i / (I cnt_i) - S (NaN for an empty cell), nm[i] = cnt_i.
__global__ void k_kmu_finish(const double* __restrict__ sums, int ncells, double norm_I, double shot,
                             double* __restrict__ pk, long long* __restrict__ nm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncells) return;
  const double cnt = sums[2 * i];
  nm[i] = __double2ll_rn(cnt);
  pk[i] = cnt > 0.0 ? __dsub_rn(__ddiv_rn(sums[2 * i + 1], __dmul_rn(norm_I, cnt)), shot)
                    : __longlong_as_double(0x7ff8000000000000LL);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static int zthreads(const FftShape& fs) { return (fs.n / 2 / fs.e_z) * fs.zlines; }
// LDS sizes.  Twiddles: the generic path stages the W_N^j table (N entries); the per-stage
// table of the compile-time path has fewer than L entries for a length-L transform.
static size_t zsmem(const FftShape& fs, size_t cs) {
  return cs * ((size_t)fs.zlines * zpitch(fs.n / 2) + fs.n + fs.n / 2);
}
// the pre-pass keeps a second line region for the finished lines of a field
static size_t zpresmem(const FftShape& fs, size_t cs) {
  return cs * (2 * (size_t)fs.zlines * zpitch(fs.n / 2) + fs.n + fs.n / 2);
}
int xpass_threads(const FftShape& fs) { return (fs.n / fs.e_col) * fs.tile; }
int xpass_blocks(const FftShape& fs) { return fs.n * ((fs.n / 2) / fs.tile); }
// Persistent post-pass grid: two blocks of 256 threads per compute unit (the register budget
// allows no more), or as many smaller blocks as hold the same threads, at most one per tile.
int post_blocks(const FftShape& fs) {
  const int tiles = fs.n * ((fs.n / 2) / fs.tile_post);
  const int cus = fs.cus > 0 ? fs.cus : 256;
  const int nthr = (fs.n / fs.e_post) * fs.tile_post;
  return std::min(tiles, std::max(2, 512 / nthr) * cus);
}
static size_t colsmem(const FftShape& fs, size_t cs) { return cs * ((size_t)fs.n * (fs.tile + 1) + fs.n); }
size_t zpass_smem_bytes(const FftShape& fs, bool fp64) {
  return zpresmem(fs, fp64 ? sizeof(double2) : sizeof(float2));
}
size_t colpass_smem_bytes(const FftShape& fs, bool fp64) {
  return colsmem(fs, fp64 ? sizeof(double2) : sizeof(float2));
}
size_t xpost_base_bytes(const FftShape& fs, bool fp64) {
  const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
  return cs * ((size_t)fs.tile_post * xrows(fs.n) + (size_t)fs.tile_post * fs.n + fs.n);
}

#define PKM_DISPATCH_E(EVAL, CALL)                  \
  switch (EVAL) {                                   \
    case 4: { constexpr int E = 4; CALL; break; }   \
    case 6: { constexpr int E = 6; CALL; break; }   \
    case 8: { constexpr int E = 8; CALL; break; }   \
    case 12: { constexpr int E = 12; CALL; break; } \
    case 16: { constexpr int E = 16; CALL; break; } \
    default: return hipErrorInvalidValue;           \
  }

// Compile-time instantiations: (N, E, TC) triples matching the plan's shape rules for FP32
// and FP64 at the power-of-two sizes and at 384 and 768; anything else runs the generic
// kernels.
#define PKM_TRY(NV, EV, TV, EARG, TARG, CALL)      \
  if (fs.n == NV && (EARG) == EV && (TARG) == TV) { \
    constexpr int NC = NV, E = EV, TC = TV;         \
    CALL;                                           \
    return hipGetLastError();                       \
  }

#define PKM_TRY_Z(CALL)                        \
  PKM_TRY(64, 8, 64, fs.e_z, fs.zlines, CALL)  \
  PKM_TRY(128, 8, 32, fs.e_z, fs.zlines, CALL) \
  PKM_TRY(256, 8, 16, fs.e_z, fs.zlines, CALL) \
  PKM_TRY(512, 8, 16, fs.e_z, fs.zlines, CALL) \
  PKM_TRY(512, 8, 8, fs.e_z, fs.zlines, CALL)  \
  PKM_TRY(1024, 8, 8, fs.e_z, fs.zlines, CALL) \
  PKM_TRY(1024, 8, 4, fs.e_z, fs.zlines, CALL) \
  PKM_TRY(384, 6, 8, fs.e_z, fs.zlines, CALL)  \
  PKM_TRY(768, 6, 8, fs.e_z, fs.zlines, CALL)  \
  PKM_TRY(768, 6, 4, fs.e_z, fs.zlines, CALL)  \
  PKM_TRY(512, 4, 4, fs.e_z, fs.zlines, CALL)

#define PKM_TRY_COL(CALL)                         \
  PKM_TRY(64, 8, 16, fs.e_col, fs.tile, CALL)     \
  PKM_TRY(128, 8, 16, fs.e_col, fs.tile, CALL)    \
  PKM_TRY(256, 16, 16, fs.e_col, fs.tile, CALL)   \
  PKM_TRY(512, 16, 16, fs.e_col, fs.tile, CALL)   \
  PKM_TRY(1024, 16, 8, fs.e_col, fs.tile, CALL)   \
  PKM_TRY(64, 8, 8, fs.e_col, fs.tile, CALL)      \
  PKM_TRY(128, 8, 8, fs.e_col, fs.tile, CALL)     \
  PKM_TRY(256, 8, 8, fs.e_col, fs.tile, CALL)     \
  PKM_TRY(512, 8, 8, fs.e_col, fs.tile, CALL)     \
  PKM_TRY(1024, 8, 4, fs.e_col, fs.tile, CALL)     \
  PKM_TRY(384, 12, 16, fs.e_col, fs.tile, CALL)    \
  PKM_TRY(768, 12, 8, fs.e_col, fs.tile, CALL)

#define PKM_TRY_POST(CALL)                           \
  PKM_TRY(64, 8, 16, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(128, 8, 16, fs.e_post, fs.tile_post, CALL) \
  PKM_TRY(256, 8, 8, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(512, 8, 4, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(1024, 8, 2, fs.e_post, fs.tile_post, CALL) \
  PKM_TRY(1024, 8, 1, fs.e_post, fs.tile_post, CALL) \
  PKM_TRY(384, 6, 4, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(768, 6, 2, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(768, 6, 1, fs.e_post, fs.tile_post, CALL)  \
  PKM_TRY(384, 12, 8, fs.e_post, fs.tile_post, CALL) \
  PKM_TRY(768, 12, 4, fs.e_post, fs.tile_post, CALL)

template <typename T>
hipError_t launch_zfwd(const FftShape& fs, const T* in0, const T* in1, void* out0, void* out1, int nbuf,
                       const void* tw, hipStream_t s) {
  const int lines = fs.n * fs.n;
  dim3 grid(lines / fs.zlines, nbuf);
  const size_t sm = zsmem(fs, sizeof(cx<T>));
  PKM_TRY_Z((k_zfwd<T, E, NC, TC><<<grid, zthreads(fs), sm, s>>>(fs.n, fs.zlines, fs.sched_z, fs.nst_z, in0, in1,
                                                                   out0, out1, (const cx<T>*)tw)));
  PKM_DISPATCH_E(fs.e_z, (k_zfwd<T, E, 0, 0><<<grid, zthreads(fs), sm, s>>>(fs.n, fs.zlines, fs.sched_z, fs.nst_z, in0,
                                                                          in1, out0, out1, (const cx<T>*)tw)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col(const FftShape& fs, void* const* bufs_dev, int nbuf, int axis, bool inverse, const void* tw,
                      hipStream_t s, bool fields) {
  const size_t n = fs.n, nh = fs.n / 2;
  // half spectra [x][y][kz]: rows along y (axis 1) or x (axis 0), tiles over kz;
  // kz-major field buffers [kz][x][y]: rows along x within a kz plane, tiles over y
  size_t row_stride, outer_stride;
  int clen;
  if (fields) {
    row_stride = n;
    outer_stride = n * n + fs.fpad;
    clen = fs.n;
  } else {
    const size_t plane = n * nh;
    row_stride = axis == 1 ? nh : plane;
    outer_stride = axis == 1 ? plane : nh;
    clen = fs.n / 2;
  }
  dim3 grid(xpass_blocks(fs), nbuf);
  const size_t sm = colsmem(fs, sizeof(cx<T>));
  if (inverse) {
    PKM_TRY_COL((k_col<T, E, true, NC, TC><<<grid, xpass_threads(fs), sm, s>>>(
        fs.n, fs.tile, fs.sched_col, fs.nst_col, bufs_dev, row_stride, outer_stride, clen, (const cx<T>*)tw)));
    PKM_DISPATCH_E(fs.e_col, (k_col<T, E, true, 0, 0><<<grid, xpass_threads(fs), sm, s>>>(
                                  fs.n, fs.tile, fs.sched_col, fs.nst_col, bufs_dev, row_stride, outer_stride, clen,
                                  (const cx<T>*)tw)));
  } else {
    PKM_TRY_COL((k_col<T, E, false, NC, TC><<<grid, xpass_threads(fs), sm, s>>>(
        fs.n, fs.tile, fs.sched_col, fs.nst_col, bufs_dev, row_stride, outer_stride, clen, (const cx<T>*)tw)));
    PKM_DISPATCH_E(fs.e_col, (k_col<T, E, false, 0, 0><<<grid, xpass_threads(fs), sm, s>>>(
                                  fs.n, fs.tile, fs.sched_col, fs.nst_col, bufs_dev, row_stride, outer_stride, clen,
                                  (const cx<T>*)tw)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xcombine(const FftShape& fs, void* s1, void* s2, void* c_out, void* g_out, int interlaced,
                           int compensated, const void* invw, const void* phase, const void* tw, hipStream_t s) {
  const size_t sm = colsmem(fs, sizeof(cx<T>));
  PKM_TRY_COL((k_xcombine<T, E, NC, TC><<<xpass_blocks(fs), xpass_threads(fs), sm, s>>>(
      fs.n, fs.tile, fs.sched_col, fs.nst_col, (const cx<T>*)s1, (const cx<T>*)s2, (cx<T>*)c_out, (cx<T>*)g_out,
      interlaced, compensated, (const T*)invw, (const cx<T>*)phase, (const cx<T>*)tw)));
  PKM_DISPATCH_E(fs.e_col, (k_xcombine<T, E, 0, 0><<<xpass_blocks(fs), xpass_threads(fs), sm, s>>>(
                               fs.n, fs.tile, fs.sched_col, fs.nst_col, (const cx<T>*)s1, (const cx<T>*)s2,
                               (cx<T>*)c_out, (cx<T>*)g_out, interlaced, compensated, (const T*)invw,
                               (const cx<T>*)phase, (const cx<T>*)tw)));
  return hipGetLastError();
}

template <typename T, bool CART>
hipError_t launch_zpre_basis(const FftShape& fs, const void* g_in, const T* real_in, T* real_out,
                             void* const* bufs_dev, int nf, const int* fields_dev, double scale, const double* off,
                             double h, const void* ytab, const void* tw, const Frame& frame, hipStream_t s) {
  const int lines = fs.n * fs.n;
  const size_t sm = zpresmem(fs, sizeof(cx<T>));
  PKM_TRY_Z((k_zpre<T, E, NC, TC, CART><<<lines / fs.zlines, zthreads(fs), sm, s>>>(
      fs.n, fs.zlines, fs.sched_z, fs.nst_z, (const cx<T>*)g_in, real_in, real_out, bufs_dev, nf, fields_dev,
      (T)scale, off[0], off[1], off[2], h, (const T*)ytab, (const cx<T>*)tw, frame, fs.fpad)));
  PKM_DISPATCH_E(fs.e_z, (k_zpre<T, E, 0, 0, CART><<<lines / fs.zlines, zthreads(fs), sm, s>>>(
                             fs.n, fs.zlines, fs.sched_z, fs.nst_z, (const cx<T>*)g_in, real_in, real_out, bufs_dev,
                             nf, fields_dev, (T)scale, off[0], off[1], off[2], h, (const T*)ytab,
                             (const cx<T>*)tw, frame, fs.fpad)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zpre(const FftShape& fs, const void* g_in, const T* real_in, T* real_out, void* const* bufs_dev,
                       int nf, const int* fields_dev, double scale, const double* off, double h, const void* ytab,
                       const void* tw, const Frame& frame, int basis, hipStream_t s) {
  if (basis == 1)
    return launch_zpre_basis<T, true>(fs, g_in, real_in, real_out, bufs_dev, nf, fields_dev, scale, off, h, ytab, tw,
                                      frame, s);
  return launch_zpre_basis<T, false>(fs, g_in, real_in, real_out, bufs_dev, nf, fields_dev, scale, off, h, ytab, tw,
                                     frame, s);
}

template <typename T, bool CART>
hipError_t launch_xpost_basis(const FftShape& fs, void* const* bufs_dev, int nf, const int* fields_dev, int nslots,
                              int with_l0, const void* c_in, const void* ytab, const BinSpec& bs, double kf,
                              double* partial, int* nblocks_out, const void* tw, const Frame& frame, hipStream_t s) {
  if (nslots < 0) return hipErrorInvalidValue;
  const int rows = (with_l0 ? 3 : 0) + nslots;
  const size_t sm = xpost_base_bytes(fs, sizeof(T) == 8) + sizeof(double) * (size_t)bs.hist_copies * rows * bs.nb +
                    sizeof(long long) * (size_t)(bs.nb + 1);
  const int nblk = post_blocks(fs);
  const int nthr = (fs.n / fs.e_post) * fs.tile_post;
  if (nthr > XPOST_THREADS) return hipErrorInvalidValue;
  *nblocks_out = nblk;
  PKM_TRY_POST((k_xpost<T, E, NC, TC, CART><<<nblk, nthr, sm, s>>>(
      fs.n, fs.tile_post, fs.sched_post, fs.nst_post, bufs_dev, nf, fields_dev, nslots, with_l0, kf,
      (const cx<T>*)c_in, (const T*)ytab, bs.thr, bs.nb, bs.hist_copies, partial, (const cx<T>*)tw, frame,
      fs.fpad)));
  PKM_DISPATCH_E(fs.e_post, (k_xpost<T, E, 0, 0, CART><<<nblk, nthr, sm, s>>>(
                                fs.n, fs.tile_post, fs.sched_post, fs.nst_post, bufs_dev, nf, fields_dev, nslots,
                                with_l0, kf, (const cx<T>*)c_in, (const T*)ytab, bs.thr, bs.nb, bs.hist_copies,
                                partial, (const cx<T>*)tw, frame, fs.fpad)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xpost(const FftShape& fs, void* const* bufs_dev, int nf, const int* fields_dev, int nslots,
                        int with_l0, const void* c_in, const void* ytab, const BinSpec& bs, double kf,
                        double* partial, int* nblocks_out, const void* tw, const Frame& frame, int basis,
                        hipStream_t s) {
  if (basis == 1)
    return launch_xpost_basis<T, true>(fs, bufs_dev, nf, fields_dev, nslots, with_l0, c_in, ytab, bs, kf, partial,
                                       nblocks_out, tw, frame, s);
  return launch_xpost_basis<T, false>(fs, bufs_dev, nf, fields_dev, nslots, with_l0, c_in, ytab, bs, kf, partial,
                                      nblocks_out, tw, frame, s);
}

hipError_t launch_reduce(const double* partial, int nblocks, int nvals, double* out, const int* map, int accumulate,
                         hipStream_t s) {
  if (nvals <= 0) return hipSuccess;
  k_reduce<<<nvals, RED_THREADS, 0, s>>>(partial, nblocks, nvals, out, map, accumulate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_kmu(const FftShape& fs, const void* c_in, const double* los, const BinSpec& bs,
                      const double* mu_edges, int nmu, double* partial, int nblk, hipStream_t s) {
  const size_t sm = sizeof(double) * 2 * (size_t)bs.nb * nmu;
  k_kmu<T><<<nblk, 256, sm, s>>>(fs.n, (const cx<T>*)c_in, los[0], los[1], los[2], bs.thr, bs.nb, mu_edges, nmu,
                                 partial);
  return hipGetLastError();
}

hipError_t launch_kmu_finish(const double* sums, int ncells, double norm_I, double shot, double* pk, long long* nm,
                             hipStream_t s) {
  if (ncells <= 0) return hipSuccess;
  k_kmu_finish<<<(ncells + 255) / 256, 256, 0, s>>>(sums, ncells, norm_I, shot, pk, nm);
  return hipGetLastError();
}

#define PKM_INST(T)                                                                                           \
  template hipError_t launch_zfwd<T>(const FftShape&, const T*, const T*, void*, void*, int, const void*,         \
                                     hipStream_t);                                                                \
  template hipError_t launch_col<T>(const FftShape&, void* const*, int, int, bool, const void*, hipStream_t,     \
                                     bool);                                                                        \
  template hipError_t launch_xcombine<T>(const FftShape&, void*, void*, void*, void*, int, int, const void*,     \
                                         const void*, const void*, hipStream_t);                                 \
  template hipError_t launch_zpre<T>(const FftShape&, const void*, const T*, T*, void* const*, int, const int*,   \
                                     double, const double*, double, const void*, const void*, const Frame&, int,   \
                                     hipStream_t);                                                                 \
  template hipError_t launch_xpost<T>(const FftShape&, void* const*, int, const int*, int, int, const void*,     \
                                      const void*, const BinSpec&, double, double*, int*, const void*,           \
                                      const Frame&, int, hipStream_t);                                           \
  template hipError_t launch_kmu<T>(const FftShape&, const void*, const double*, const BinSpec&, const double*,   \
                                    int, double*, int, hipStream_t);
PKM_INST(float)
PKM_INST(double)

}  // namespace pkm
