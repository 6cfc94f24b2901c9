// Launch wrappers for the estimator's HIP kernels (definitions in kernels_*.hip).
// Every wrapper enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkm {

struct FftShape {
  int n;            // mesh side N
  int e_col;        // elements per thread for the length-N column transforms
  int e_z;          // elements per thread for the length-N/2 line transforms
  uint32_t sched_col;  // radix schedule (4 bits per stage) for length N
  int nst_col;
  uint32_t sched_z;    // radix schedule for length N/2
  int nst_z;
  int tile;         // columns per column-pass tile
  int zlines;       // lines per z-pass block
  int e_post;       // elements per thread in the post-pass (last transform + binning)
  uint32_t sched_post;
  int nst_post;
  int tile_post;    // columns per post-pass tile
  int cus;          // compute units of the device (0: unknown)
  int fpad;         // extra elements per kz plane of a field buffer [kz][x][y]: the plane
                    // stride n n + fpad is then not a power of two
};

// Bytes of LDS of the z-pass and column-pass blocks of a shape.
size_t zpass_smem_bytes(const FftShape& fs, bool fp64);
size_t colpass_smem_bytes(const FftShape& fs, bool fp64);

// LDS bytes of a post-pass block without its histograms.
size_t xpost_base_bytes(const FftShape& fs, bool fp64);

// Orthogonal matrix (rows r[0..2], r[3..5], r[6..8]) applied to every unit vector, node
// direction and wave vector alike, before harmonics or monomials are evaluated.  The sums
// over m (or over the monomials of one degree) depend on k.x only, so any orthogonal matrix
// gives the same multipoles; the plan picks one that turns the mean line of sight to
// (1,1,1)/sqrt(3), away from the coordinate poles where FP32 rounding of a direction
// cosine becomes a large, and across the survey correlated, angle error.
struct Frame {
  double r[9];
  float f[9];  // the same, rounded (FP32 passes)
  template <typename T> __host__ __device__ T at(int i) const {
    if constexpr (sizeof(T) == 4) return f[i]; else return (T)r[i];
  }
};

struct BinSpec {
  const long long* thr;  // device, nb+1 integer thresholds on |n|^2
  int nb;
  int hist_copies;       // per-block histogram copies (1 .. number of waves)
};

// Catalog sums: out2[0] = sum w^2, out2[1] = sum w^2 nbar, *wmax = max |w| (w, nbar may be
// null => 1).  partial holds 3 nblk doubles.
hipError_t launch_catalog_sums(const double* w, const double* nbar, int64_t n, double* partial, int nblk,
                               double* out2, double* wmax, hipStream_t s);

template <typename T> hipError_t launch_fill(T* p, size_t n, T v, hipStream_t s);

// Counting sort of particles by tile of their base node (tile side ts): per particle the
// tile id and its rank within the tile (atomic counter), for catalog entries [base, base+n).
// `count` holds TILE_COUNT_COPIES zeroed copies of ntiles + 1 counters (a block uses one copy);
// launch_tile_offsets turns them in place into per-copy start offsets.
hipError_t launch_tile_sort(const double* pos, int64_t n, int64_t base, const double* origin, double scale,
                            int nmesh, int ts, int* count, int* tile_of, int* rank, hipStream_t s);
// Exclusive scan of the tile counts (off has ntiles + 1 entries), then the particle payload
// (x, y, z, w for data / -alpha w for randoms; 32 bytes each) written in tile order.
hipError_t launch_tile_offsets(int* count, int ntiles, int* off, const int* tile_of, const int* rank,
                               int64_t nd, int64_t ntot, const double* dpos, const double* dw, const double* rpos,
                               const double* rw, double alpha, void* payload, int* bsum, hipStream_t s);
constexpr int TILE_COUNT_COPIES = 8;
// Scratch entries needed by the tile scan (block sums).
inline int tile_scan_scratch(int ntiles) { return (ntiles + 1023) / 1024 + 1; }
// Tile-wise painting from the sorted payload.
template <typename T>
// wmax_d / wmax_r: device pointers to the largest |w| of each catalog (wmax_r null without
// randoms); they bound the per-tile fixed-point accumulation of FP32 meshes.
// acc (deterministic mode, else null): 64-bit accumulators, n^3 per mesh (two meshes when d2 is
// set), zeroed by the caller; the paint then leaves d1 / d2 untouched and writes the shared
// fixed-point scale to *gsc, and launch_det_convert turns the accumulators into the meshes.
hipError_t launch_paint_tiles(const int* off, const void* payload, int ntiles, const double* origin, double scale,
                              int nmesh, int window, int ts, T* d1, T* d2, const double* wmax_d,
                              const double* wmax_r, double alpha, hipStream_t s, unsigned long long* acc = nullptr,
                              double* gsc = nullptr);
template <typename T>
hipError_t launch_det_convert(const unsigned long long* acc, T* d1, T* d2, int nmesh, const double* gsc,
                              hipStream_t s);

// Forward real-to-half-complex transform along z of nbuf real meshes (nbuf <= 2).
template <typename T>
hipError_t launch_zfwd(const FftShape& fs, const T* in0, const T* in1, void* out0, void* out1, int nbuf,
                       const void* tw, hipStream_t s);

// Column transform of nbuf buffers in place: half spectra [x][y][kz] along y (axis = 1) or x
// (axis = 0); fields = true: kz-major field buffers [kz][x][y] (kz planes of n n + fs.fpad
// elements) along x.
template <typename T>
hipError_t launch_col(const FftShape& fs, void* const* bufs_dev, int nbuf, int axis, bool inverse,
                      const void* tw, hipStream_t s, bool fields = false);

// x-pass of the forward transforms of the two painted meshes, interlace combine,
// compensation and Nyquist zeroing; writes C and, when g_out != null, G = C inverse-
// transformed along x.
template <typename T>
hipError_t launch_xcombine(const FftShape& fs, void* s1, void* s2, void* c_out, void* g_out, int interlaced,
                           int compensated, const void* invw, const void* phase, const void* tw, hipStream_t s);

// Inverse z (half-complex to real) of G, scaled to D_c, then for every field f in the group
// the Y_lm(xhat)-weighted forward transform along z into the kz-major field buffer bufs[f]
// ([kz][x][y], kz planes of n n + fs.fpad elements).  Needs fs.zlines to divide n.  If real_in != null the
// field D_c is read directly from that real mesh instead.  If real_out != null D_c is also
// written there.  basis 1 (Cartesian decomposition): field f is weighted by the monomial
// xhat^a of degree fields[4f+1] and index code fields[4f+2] instead of Y_lm(xhat).
template <typename T>
hipError_t launch_zpre(const FftShape& fs, const void* g_in, const T* real_in, T* real_out, void* const* bufs_dev,
                       int nf, const int* fields_dev, double scale, const double* off, double h, const void* ytab,
                       const void* tw, const Frame& frame, int basis, hipStream_t s);

// Last transform pass of every field of the group (along y over the kz-major field buffers),
// sum over m of Y_lm(khat) B_lm per multipole slot, product with C and binning.  Odd l
// (spherical basis) are binned as Im[C conj (sum)] instead of Re.  Per block the partial sums are rows of nb bins:
// [count, sum |k|, sum |C|^2] when with_l0, then one row of sum 4 pi Y Re[C conj B] per slot.
// basis 1: the slot sums (p!/a!) khat^a B_a over the monomials a of one degree p, and its row
// holds sum Re[C conj (that sum)] without the 4 pi.
template <typename T>
hipError_t launch_xpost(const FftShape& fs, void* const* bufs_dev, int nf, const int* fields_dev, int nslots,
                        int with_l0, const void* c_in, const void* ytab, const BinSpec& bs, double kf,
                        double* partial, int* nblocks_out, const void* tw, const Frame& frame, int basis,
                        hipStream_t s);

// out[map[v]] (+)= sum_b partial[b*nvals + v] (map null -> identity), fixed order.
hipError_t launch_reduce(const double* partial, int nblocks, int nvals, double* out, const int* map, int accumulate,
                         hipStream_t s);

// Global line of sight: (k, mu) cells; partial[block][cell*2 + {0: sum w, 1: sum w |C|^2}].
template <typename T>
hipError_t launch_kmu(const FftShape& fs, const void* c_in, const double* los, const BinSpec& bs,
                      const double* mu_edges, int nmu, double* partial, int nblk, hipStream_t s);

// Device-side normalisation of reduced (k, mu) sums {count, sum |C|^2} per cell into
// P = sum / (I count) - S (NaN when empty) and the integer counts.
hipError_t launch_kmu_finish(const double* sums, int ncells, double norm_I, double shot, double* pk, long long* nm,
                             hipStream_t s);

int xpass_blocks(const FftShape& fs);
int xpass_threads(const FftShape& fs);
int post_blocks(const FftShape& fs);

}  // namespace pkm
