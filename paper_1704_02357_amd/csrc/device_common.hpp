// Device-side building blocks shared by the estimator's kernels (gfx950, wave64):
// complex arithmetic, small-radix DFTs, an LDS-resident Stockham FFT over a batch of
// lines, the real/complex packing of a real-input transform, the real spherical-harmonic
// recurrence and the integer k-bin search.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkm {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using cx = typename vec2<T>::type;

template <typename T> __device__ __forceinline__ cx<T> mk(T re, T im) { cx<T> r; r.x = re; r.y = im; return r; }
template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cx<T> rot_mi(cx<T> a) {
  return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ---------------------------------------------------------------------------------------
// Radix-R DFT on registers: y_s = sum_t x_t exp(-+2 pi i s t / R), R in {2,3,4,6,8}.
// ---------------------------------------------------------------------------------------
template <typename T, bool INV> __device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd<T>(a, b);
  v[1] = csub<T>(a, b);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a0 = cadd<T>(v[0], v[2]), b0 = csub<T>(v[0], v[2]);
  cx<T> a1 = cadd<T>(v[1], v[3]), b1 = rot_mi<T, INV>(csub<T>(v[1], v[3]));
  v[0] = cadd<T>(a0, a1);
  v[2] = csub<T>(a0, a1);
  v[1] = cadd<T>(b0, b1);
  v[3] = csub<T>(b0, b1);
}

template <typename T, bool INV> __device__ __forceinline__ void dft3(cx<T>* v) {
  const T h = T(0.5);
  const T s3 = INV ? T(-0.86602540378443864676) : T(0.86602540378443864676);
  cx<T> t1 = cadd<T>(v[1], v[2]);
  cx<T> t2 = csub<T>(v[1], v[2]);
  cx<T> m = mk<T>(v[0].x - h * t1.x, v[0].y - h * t1.y);
  // forward: y1 = m - i s3 t2, y2 = m + i s3 t2
  cx<T> it = mk<T>(s3 * t2.y, -s3 * t2.x);  // -i * s3 * t2
  v[0] = cadd<T>(v[0], t1);
  v[1] = cadd<T>(m, it);
  v[2] = csub<T>(m, it);
}

template <typename T, bool INV> __device__ __forceinline__ void dft6(cx<T>* v) {
  // split t -> (t, t+3): a_t = x_t + x_{t+3}, b_t = (x_t - x_{t+3}) W6^t
  cx<T> a[3], b[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    a[t] = cadd<T>(v[t], v[t + 3]);
    b[t] = csub<T>(v[t], v[t + 3]);
  }
  const T c1 = T(0.5), s1 = INV ? T(0.86602540378443864676) : T(-0.86602540378443864676);
  b[1] = cmul<T>(b[1], mk<T>(c1, s1));    // W6^1
  b[2] = cmul<T>(b[2], mk<T>(-c1, s1));   // W6^2
  dft3<T, INV>(a);
  dft3<T, INV>(b);
  v[0] = a[0]; v[2] = a[1]; v[4] = a[2];
  v[1] = b[0]; v[3] = b[1]; v[5] = b[2];
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> a[4], b[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    a[t] = cadd<T>(v[t], v[t + 4]);
    b[t] = csub<T>(v[t], v[t + 4]);
  }
  const T r = T(0.70710678118654752440);
  // b_t *= W8^t
  b[1] = INV ? mk<T>(r * (b[1].x - b[1].y), r * (b[1].x + b[1].y))
             : mk<T>(r * (b[1].x + b[1].y), r * (b[1].y - b[1].x));
  b[2] = rot_mi<T, INV>(b[2]);
  b[3] = INV ? mk<T>(-r * (b[3].x + b[3].y), r * (b[3].x - b[3].y))
             : mk<T>(r * (b[3].y - b[3].x), -r * (b[3].x + b[3].y));
  dft4<T, INV>(a);
  dft4<T, INV>(b);
  v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
  v[1] = b[0]; v[3] = b[1]; v[5] = b[2]; v[7] = b[3];
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft_r(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 6) dft6<T, INV>(v);
  else dft8<T, INV>(v);
}

// ---------------------------------------------------------------------------------------
// Stockham (decimation-in-time, autosorting) FFT of a batch of lines resident in LDS.
// Element i of a line sits at lds[off + i*es].  Each line is processed by Pt = L/E threads;
// this thread is number t of its line.  At a stage of radix R and span m, butterfly b
// (b = t + q*Pt, q < E/R) reads x_s = in[b + s L/R], multiplies by W_{mR}^{s k} (k = b mod m),
// applies the radix-R DFT and writes y_s to out[(b/m) m R + k + s m].  The stage runs in
// place: all reads finish at a barrier before any write.  Twiddles come from
// tw[j] = exp(-2 pi i j / Ntw); W_{mR}^{q} = tw[q * Ntw/(mR)].  The caller must hold a
// barrier between filling the lines and calling this; it returns after a barrier.
// ---------------------------------------------------------------------------------------
// Physical LDS slot of element i: with PAD > 0 one spare slot follows every 2^PAD elements,
// which breaks the power-of-two strides of the first Stockham stages across LDS banks.
template <int PAD> __device__ __forceinline__ int padi(int i) { return PAD > 0 ? i + (i >> PAD) : i; }

template <typename T, int E, int R, bool INV, int PAD>
__device__ __forceinline__ void stockham_stage(cx<T>* lds, int off, int es, int L, int m, int t, int Pt,
                                               const cx<T>* __restrict__ tw, int Ntw) {
  constexpr int NB = E / R;
  cx<T> v[E];
  const int Lr = L / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int b = t + q * Pt;
#pragma unroll
    for (int s = 0; s < R; ++s) v[q * R + s] = lds[off + padi<PAD>(b + s * Lr) * es];
  }
  __syncthreads();
  const int step = Ntw / (m * R);
  const bool pow2 = (m & (m - 1)) == 0;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int b = t + q * Pt;
    const int k = pow2 ? (b & (m - 1)) : b % m;
    const int base = (b - k) * R + k;  // (b/m) m R + k
    if (k != 0) {
#pragma unroll
      for (int s = 1; s < R; ++s) {
        cx<T> w = tw[s * k * step];
        if (INV) w.y = -w.y;
        v[q * R + s] = cmul<T>(v[q * R + s], w);
      }
    }
    dft_r<T, R, INV>(&v[q * R]);
#pragma unroll
    for (int s = 0; s < R; ++s) lds[off + padi<PAD>(base + s * m) * es] = v[q * R + s];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Compile-time Stockham FFT for L = 2^a 3^b with the line held in registers on entry and
// exit.  At each stage the first of the radices 8, 6, 4, 3, 2 that divides both E and the
// remaining length (the order the host's schedules use); spans, strides and twiddle offsets
// are constants.  Element e of the register array u is position t + PT*e of the line (PT = L/E
// threads per line, this thread number t).  The first stage reads its inputs straight from
// u and the last stage's outputs are exactly the positions t + PT*e again, so only the
// exchanges between stages go through LDS (at lds[off + padi<PAD>(i)*es]).
//
// Twiddles come from a per-stage table (ct_twiddles): the stage of span M and radix R keeps
// W_{MR}^{sk} at offset ct_tw_off(M) + k(R-1) + (s-1), so lanes with consecutive k read
// consecutive entries instead of the strided, bank-conflicting reads of a W_N^j table.
//
// WAVE = true when every line lies inside one wavefront: the stage exchanges then need only
// a wavefront-level ordering (LDS operations of one wave complete in issue order).
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int ct_radix(int e, int rem) {
  return (e % 8 == 0 && rem % 8 == 0)   ? 8
         : (e % 6 == 0 && rem % 6 == 0) ? 6
         : (e % 4 == 0 && rem % 4 == 0) ? 4
         : (e % 3 == 0 && rem % 3 == 0) ? 3
                                        : 2;
}
// Offset of the twiddles of the stage with span mstage (all stages with span < mstage).
__host__ __device__ constexpr int ct_tw_off(int e, int L, int mstage) {
  int m = 1, sz = 0;
  while (m < mstage && m < L) {
    const int r = ct_radix(e, L / m);
    if (m > 1) sz += m * (r - 1);
    m *= r;
  }
  return sz;
}
__host__ __device__ constexpr int ct_tw_total(int e, int L) { return ct_tw_off(e, L, L); }
__host__ __device__ constexpr int ct_last_radix(int e, int L) {
  int m = 1, r = 2;
  while (m < L) {
    r = ct_radix(e, L / m);
    m *= r;
  }
  return r;
}

// Fill the per-stage table from tw[j] = exp(-2 pi i j / NTW) (NTW a multiple of L).
template <typename T, int E, int L, int NTW>
__device__ __forceinline__ void ct_twiddles(cx<T>* dst, const cx<T>* __restrict__ tw) {
  constexpr int total = ct_tw_total(E, L);
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    int m = 1, off = 0;
    for (;;) {
      const int r = ct_radix(E, L / m);
      if (m > 1) {
        const int sz = m * (r - 1);
        if (i < off + sz) {
          const int j = i - off;
          const int k = j / (r - 1), s = j % (r - 1) + 1;
          dst[i] = tw[s * k * (NTW / (m * r))];
          break;
        }
        off += sz;
      }
      m *= r;
    }
  }
}

// Ordering of LDS accesses between the threads that share a line.
template <bool WAVE> __device__ __forceinline__ void ct_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Stage of span M: inputs v[q*R + s] = x[b + s*L/R], b = t + q*PT.
template <typename T, int E, int PAD, int L, int M>
__device__ __forceinline__ void ct_gather(const cx<T>* lds, int off, int es, int t, cx<T>* v) {
  constexpr int R = ct_radix(E, L / M), PT = L / E, NB = E / R, LR = L / R;
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int s = 0; s < R; ++s) v[q * R + s] = lds[off + padi<PAD>(t + q * PT + s * LR) * es];
}
template <typename T, int E, bool INV, int L, int M>
__device__ __forceinline__ void ct_butterflies(int t, cx<T>* v, const cx<T>* twst) {
  constexpr int R = ct_radix(E, L / M), PT = L / E, NB = E / R, OFF = ct_tw_off(E, L, M);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if constexpr (M > 1) {
      const int k = (t + q * PT) % M;  // a mask when M is a power of two
#pragma unroll
      for (int s = 1; s < R; ++s) {
        cx<T> w = twst[OFF + k * (R - 1) + (s - 1)];
        if (INV) w.y = -w.y;
        v[q * R + s] = cmul<T>(v[q * R + s], w);
      }
    }
    dft_r<T, R, INV>(&v[q * R]);
  }
}
// Outputs y_s of butterfly b go to (b/M) M R + (b mod M) + s M.
template <typename T, int E, int PAD, int L, int M>
__device__ __forceinline__ void ct_scatter(cx<T>* lds, int off, int es, int t, const cx<T>* v) {
  constexpr int R = ct_radix(E, L / M), PT = L / E, NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int b = t + q * PT;
    const int k = b % M;
    const int base = (b - k) * R + k;
#pragma unroll
    for (int s = 0; s < R; ++s) lds[off + padi<PAD>(base + s * M) * es] = v[q * R + s];
  }
}
template <typename T, int E, bool INV, int PAD, int L, bool WAVE, int M>
__device__ __forceinline__ void ct_rest(cx<T>* lds, int off, int es, int t, cx<T>* v, const cx<T>* twst) {
  ct_butterflies<T, E, INV, L, M>(t, v, twst);
  constexpr int R = ct_radix(E, L / M);
  if constexpr (M * R < L) {
    ct_sync<WAVE>();
    ct_scatter<T, E, PAD, L, M>(lds, off, es, t, v);
    ct_sync<WAVE>();
    ct_gather<T, E, PAD, L, M * R>(lds, off, es, t, v);
    ct_rest<T, E, INV, PAD, L, WAVE, M * R>(lds, off, es, t, v, twst);
  }
}

// Transform of u in place (registers).  The caller must have finished every read of the
// line's LDS slots by the threads of the line (ct_sync<WAVE> or stronger) and the twiddle
// table must be visible.  On return the LDS slots hold intermediate data.
template <typename T, int E, bool INV, int PAD, int L, bool WAVE>
__device__ __forceinline__ void ct_fft_regs(cx<T>* lds, int off, int es, int t, cx<T>* u, const cx<T>* twst) {
  constexpr int R0 = ct_radix(E, L), NB0 = E / R0;
  constexpr int RL = ct_last_radix(E, L), NBL = E / RL;
  cx<T> v[E];
#pragma unroll
  for (int q = 0; q < NB0; ++q)
#pragma unroll
    for (int s = 0; s < R0; ++s) v[q * R0 + s] = u[q + s * NB0];
  ct_rest<T, E, INV, PAD, L, WAVE, 1>(lds, off, es, t, v, twst);
#pragma unroll
  for (int q = 0; q < NBL; ++q)
#pragma unroll
    for (int s = 0; s < RL; ++s) u[q + s * NBL] = v[q * RL + s];
}

// Same with the input line already in LDS (filled and made visible by the caller).
template <typename T, int E, bool INV, int PAD, int L, bool WAVE>
__device__ __forceinline__ void ct_fft_lds_in(cx<T>* lds, int off, int es, int t, cx<T>* u, const cx<T>* twst) {
  constexpr int RL = ct_last_radix(E, L), NBL = E / RL;
  cx<T> v[E];
  ct_gather<T, E, PAD, L, 1>(lds, off, es, t, v);
  ct_rest<T, E, INV, PAD, L, WAVE, 1>(lds, off, es, t, v, twst);
#pragma unroll
  for (int q = 0; q < NBL; ++q)
#pragma unroll
    for (int s = 0; s < RL; ++s) u[q + s * NBL] = v[q * RL + s];
}

// Radix schedule packed 4 bits per stage (stage 0 in the low bits), nst stages.
template <typename T, int E, bool INV, int PAD = 0>
__device__ __forceinline__ void lds_fft(cx<T>* lds, int off, int es, int L, uint32_t sched, int nst, int t, int Pt,
                                        const cx<T>* __restrict__ tw, int Ntw) {
  int m = 1;
  for (int st = 0; st < nst; ++st) {
    const int r = (sched >> (4 * st)) & 15;
    if constexpr (E % 8 == 0) {
      if (r == 8) { stockham_stage<T, E, 8, INV, PAD>(lds, off, es, L, m, t, Pt, tw, Ntw); m *= 8; continue; }
    }
    if constexpr (E % 6 == 0) {
      if (r == 6) { stockham_stage<T, E, 6, INV, PAD>(lds, off, es, L, m, t, Pt, tw, Ntw); m *= 6; continue; }
    }
    if constexpr (E % 4 == 0) {
      if (r == 4) { stockham_stage<T, E, 4, INV, PAD>(lds, off, es, L, m, t, Pt, tw, Ntw); m *= 4; continue; }
    }
    if constexpr (E % 3 == 0) {
      if (r == 3) { stockham_stage<T, E, 3, INV, PAD>(lds, off, es, L, m, t, Pt, tw, Ntw); m *= 3; continue; }
    }
    if constexpr (E % 2 == 0) {
      if (r == 2) { stockham_stage<T, E, 2, INV, PAD>(lds, off, es, L, m, t, Pt, tw, Ntw); m *= 2; continue; }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Real spherical harmonics in Cartesian form, no trigonometry:
//   Y_lm(u) = q_l^{|m|}(u_z) * Re/Im[(u_x + i u_y)^{|m|}]   (Re for m >= 0, Im for m < 0)
// where q_l^m = N_lm P_l^m(t) / (1 - t^2)^{m/2} obeys
//   q_m^m = c_m,  q_{m+1}^m = a_{m+1,m} t q_m^m,  q_l^m = a_lm t q_{l-1}^m - b_lm q_{l-2}^m.
// The coefficient table (built in FP64 on the host, rounded to T) is laid out per |m|:
// tab[m*STRIDE + 0] = c_m, tab[m*STRIDE + 2*(l-m)-1] = a_lm, tab[m*STRIDE + 2*(l-m)] = b_lm.
// ---------------------------------------------------------------------------------------
constexpr int YLM_LMAX = 16;
constexpr int YLM_STRIDE = 2 * YLM_LMAX + 2;

// Running evaluation of real Y_lm at NV points over a sequence of fields.  The state keeps
// (ux + i uy)^am and the recurrence pair (q_{l-1}^am, q_l^am) of the last field, so a field
// with the same |m| and a larger l continues the recurrence, the -m partner of a field costs
// nothing, and a field with |m| one larger costs one complex multiply plus a restart of the
// recurrence.  Fields in any other order restart from scratch (still correct).  Control flow
// depends only on (l, m), which are wave-uniform.
// Cartesian decomposition (Sec. 2.1, the monomial form the spherical-harmonic expansion
// replaces): a field of degree p is weighted by the monomial u_x^i u_y^j u_z^(p-i-j), its
// index packed as code = 32 i + j.  out = coef * monomial for NV directions.
__host__ __device__ constexpr int cart_code(int i, int j) { return 32 * i + j; }

template <typename T, int NV>
__device__ __forceinline__ void monomial_eval(int p, int code, T coef, const T* ux, const T* uy, const T* uz,
                                              T* out) {
  const int i = code >> 5, j = code & 31, k = p - i - j;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = coef;
  for (int q = 0; q < i; ++q) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] *= ux[v];
  }
  for (int q = 0; q < j; ++q) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] *= uy[v];
  }
  for (int q = 0; q < k; ++q) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] *= uz[v];
  }
}

// p! / (i! j! (p-i-j)!), exact in integers for p <= 16 (at most 2018016)
__device__ __forceinline__ int multinomial(int p, int code) {
  const int i = code >> 5, j = code & 31;
  long long c = 1;
  for (int q = 1; q <= i; ++q) c = c * (p - i + q) / q;          // binom(p, i)
  for (int q = 1; q <= j; ++q) c = c * (p - i - j + q) / q;      // binom(p - i, j)
  return (int)c;
}

template <typename T, int NV> struct YRun {
  T cr[NV], ci[NV], q0[NV], q1[NV];
  int am, l;
};

template <typename T, int NV> __device__ __forceinline__ void yrun_init(YRun<T, NV>& s) {
  s.am = -1;
  s.l = -1;
}

// PAIRS: advance the recurrence two degrees per iteration (fewer register copies, more
// registers live); off for register-bound callers.
template <typename T, int NV, bool PAIRS = true>
__device__ __forceinline__ void yrun_eval(YRun<T, NV>& s, int ell, int m, const T* ux, const T* uy, const T* uz,
                                          T* out, const T* __restrict__ tab) {
  const int am = m < 0 ? -m : m;
  if (am != s.am || ell < s.l) {
    if (s.am < 0 || am < s.am) {
#pragma unroll
      for (int v = 0; v < NV; ++v) { s.cr[v] = T(1); s.ci[v] = T(0); }
      s.am = 0;
    }
    for (int j = s.am; j < am; ++j) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T nr = s.cr[v] * ux[v] - s.ci[v] * uy[v];
        s.ci[v] = s.cr[v] * uy[v] + s.ci[v] * ux[v];
        s.cr[v] = nr;
      }
    }
    s.am = am;
    const T c0 = tab[am * YLM_STRIDE];
#pragma unroll
    for (int v = 0; v < NV; ++v) { s.q1[v] = c0; s.q0[v] = T(0); }
    s.l = am;
  }
  const T* c = tab + am * YLM_STRIDE;
  int l = s.l + 1;
  // two degrees per iteration with the pair's roles swapped in between (no register copies)
  for (; PAIRS && l + 1 <= ell; l += 2) {
    const int j = l - am;
    const T a1 = c[2 * j - 1], b1 = c[2 * j];  // b = 0 for j = 1
    const T a2 = c[2 * j + 1], b2 = c[2 * j + 2];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      s.q0[v] = a1 * uz[v] * s.q1[v] - b1 * s.q0[v];  // q_l
      s.q1[v] = a2 * uz[v] * s.q0[v] - b2 * s.q1[v];  // q_{l+1}
    }
  }
  for (; l <= ell; ++l) {
    const int j = l - am;
    const T a = c[2 * j - 1], b = c[2 * j];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T q2 = a * uz[v] * s.q1[v] - b * s.q0[v];
      s.q0[v] = s.q1[v];
      s.q1[v] = q2;
    }
  }
  s.l = ell;
  if (m < 0) {  // m is the same for the whole wave
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = s.q1[v] * s.ci[v];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = s.q1[v] * s.cr[v];
  }
}

// Atomic add to an LDS location (native ds_add_f32 / ds_add_f64; a plain atomicAdd through a
// generic pointer may compile to a flat atomic).
template <typename T> __device__ __forceinline__ void lds_atomic_add(T* p, T v) {
  typedef __attribute__((address_space(3))) T LT;
  __hip_atomic_fetch_add((LT*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bin index of an integer squared wavenumber: largest i with thr[i] <= n2, if i < nb; else -1.
__device__ __forceinline__ int kbin_of(long long n2, const long long* __restrict__ thr, int nb) {
  if (n2 < thr[0] || n2 >= thr[nb]) return -1;
  int lo = 0, hi = nb;  // thr[lo] <= n2 < thr[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (thr[mid] <= n2) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace pkm
