// Catalog reductions and mass assignment (Sec. 2.1 FKP field, Sec. 2.3 TSC painting with
// interlacing).  Mesh coordinates are computed in FP64 with explicitly rounded operations
// (u = (x - o) * (N / L); no fused multiply-add) so that node indices and fractions match
// any other IEEE implementation of the same formula bit for bit.
#include "kernels.hpp"
#include "device_common.hpp"

namespace pkm {

namespace {

constexpr int SUM_THREADS = 256;

__global__ void __launch_bounds__(SUM_THREADS) k_catalog_sums(const double* __restrict__ w,
                                                              const double* __restrict__ nbar, int64_t n,
                                                              double* __restrict__ partial) {
  __shared__ double s0[SUM_THREADS], s1[SUM_THREADS];
  double a0 = 0.0, a1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double wi = w ? w[i] : 1.0;
    const double w2 = wi * wi;
    a0 += w2;
    a1 += w2 * (nbar ? nbar[i] : 1.0);
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int h = SUM_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0[0];
    partial[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ void __launch_bounds__(SUM_THREADS) k_sum_partials2(const double* __restrict__ partial, int nblk,
                                                               double* __restrict__ out2) {
  __shared__ double s0[SUM_THREADS], s1[SUM_THREADS];
  double a0 = 0.0, a1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += SUM_THREADS) {
    a0 += partial[2 * b];
    a1 += partial[2 * b + 1];
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int h = SUM_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = s0[0];
    out2[1] = s1[0];
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

// Per-axis taps of the assignment window at mesh coordinate u: nodes idx[0..nt) and weights.
__device__ __forceinline__ int axis_taps(double u, int window, int nmesh, int* idx, double* wt) {
  if (window == 1) {
    const double c = floor(__dadd_rn(u, 0.5));
    idx[0] = wrap((long long)c, nmesh);
    wt[0] = 1.0;
    return 1;
  }
  if (window == 2) {
    const double c = floor(u);
    const double d = __dsub_rn(u, c);
    const long long ci = (long long)c;
    idx[0] = wrap(ci, nmesh);
    idx[1] = wrap(ci + 1, nmesh);
    wt[0] = 1.0 - d;
    wt[1] = d;
    return 2;
  }
  const double c = floor(__dadd_rn(u, 0.5));
  const double d = __dsub_rn(u, c);
  const long long ci = (long long)c;
  idx[0] = wrap(ci - 1, nmesh);
  idx[1] = wrap(ci, nmesh);
  idx[2] = wrap(ci + 1, nmesh);
  const double a = 0.5 - d, b = 0.5 + d;
  wt[0] = 0.5 * a * a;
  wt[1] = 0.75 - d * d;
  wt[2] = 0.5 * b * b;
  return 3;
}

template <typename T>
__device__ __forceinline__ void scatter(T* __restrict__ mesh, const double* u, double wgt, int window, int nmesh) {
  int ix[3], iy[3], iz[3];
  double wx[3], wy[3], wz[3];
  const int nt = axis_taps(u[0], window, nmesh, ix, wx);
  axis_taps(u[1], window, nmesh, iy, wy);
  axis_taps(u[2], window, nmesh, iz, wz);
  for (int a = 0; a < nt; ++a) {
    const double wa = wgt * wx[a];
    const size_t ba = (size_t)ix[a] * nmesh;
    for (int b = 0; b < nt; ++b) {
      const double wab = wa * wy[b];
      const size_t bb = (ba + iy[b]) * nmesh;
      for (int c = 0; c < nt; ++c) {
        unsafeAtomicAdd(&mesh[bb + iz[c]], (T)(wab * wz[c]));
      }
    }
  }
}

template <typename T>
__global__ void k_paint(const double* __restrict__ pos, const double* __restrict__ w, int64_t n, double wscale,
                        double o0, double o1, double o2, double scale, int nmesh, int window, T* __restrict__ d1,
                        T* __restrict__ d2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double u[3];
    u[0] = __dmul_rn(__dsub_rn(pos[3 * i + 0], o0), scale);
    u[1] = __dmul_rn(__dsub_rn(pos[3 * i + 1], o1), scale);
    u[2] = __dmul_rn(__dsub_rn(pos[3 * i + 2], o2), scale);
    const double wgt = (w ? w[i] : 1.0) * wscale;
    scatter<T>(d1, u, wgt, window, nmesh);
    if (d2) {
      u[0] = __dadd_rn(u[0], 0.5);
      u[1] = __dadd_rn(u[1], 0.5);
      u[2] = __dadd_rn(u[2], 0.5);
      scatter<T>(d2, u, wgt, window, nmesh);
    }
  }
}

}  // namespace

hipError_t launch_catalog_sums(const double* w, const double* nbar, int64_t n, double* partial, int nblk,
                               double* out2, hipStream_t s) {
  k_catalog_sums<<<nblk, SUM_THREADS, 0, s>>>(w, nbar, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials2<<<1, SUM_THREADS, 0, s>>>(partial, nblk, out2);
  return hipGetLastError();
}

template <typename T> hipError_t launch_fill(T* p, size_t n, T v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill<T><<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_paint(const double* pos, const double* w, int64_t n, double wscale, const double* origin,
                        double scale, int nmesh, int window, T* d1, T* d2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  k_paint<T><<<(unsigned)blocks, 256, 0, s>>>(pos, w, n, wscale, origin[0], origin[1], origin[2], scale, nmesh,
                                             window, d1, d2);
  return hipGetLastError();
}

template hipError_t launch_fill<float>(float*, size_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, size_t, double, hipStream_t);
template hipError_t launch_paint<float>(const double*, const double*, int64_t, double, const double*, double, int,
                                        int, float*, float*, hipStream_t);
template hipError_t launch_paint<double>(const double*, const double*, int64_t, double, const double*, double, int,
                                         int, double*, double*, hipStream_t);

}  // namespace pkm
