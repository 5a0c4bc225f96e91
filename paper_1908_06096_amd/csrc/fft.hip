// Longitude transforms of every ring in one launch (report section 4.2.5
// runs one FFT library call per latitude because the lengths differ; here a
// work list of (ring, field chunk) items covers all rings and fields).
//
// A ring of n = 2h points is transformed as a complex DFT of length h of
// z_t = g_{2t} + i g_{2t+1} plus an O(h) pre/post step.  The complex DFT is
// an in-LDS Stockham autosort FFT with radices 2, 3, 4, 5 when h is
// 5-smooth; otherwise it is the chirp-z (Bluestein) identity
//   X_q = c_q sum_t (z_t c_t) conj(c_{q-t}),  c_t = exp(-i pi t^2 / h),
// evaluated as a cyclic convolution of 5-smooth length L >= 2h - 1 with two
// more FFTs.  Inverse DFTs use conj(DFT(conj(x))).
#include "sht_internal.h"

namespace shtmi {

template <typename T>
struct V2T;
template <>
struct V2T<float> {
  typedef float2 type;
};
template <>
struct V2T<double> {
  typedef double2 type;
};

template <typename C>
__device__ inline C cadd(C a, C b) {
  return C{a.x + b.x, a.y + b.y};
}
template <typename C>
__device__ inline C csub(C a, C b) {
  return C{a.x - b.x, a.y - b.y};
}
template <typename C>
__device__ inline C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C>
__device__ inline C cconj(C a) {
  return C{a.x, -a.y};
}
template <typename C>
__device__ inline C cmul_negi(C a) {  // -i a
  return C{a.y, -a.x};
}
template <typename C, typename T>
__device__ inline C cscale(C a, T s) {
  return C{a.x * s, a.y * s};
}

// Forward DFT of R points in registers.
template <typename T, int R>
__device__ inline void butterfly(typename V2T<T>::type* v) {
  typedef typename V2T<T>::type C;
  if constexpr (R == 2) {
    const C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T s3 = (T)0.86602540378443864676;  // sin(2 pi / 3)
    const C t1 = cadd(v[1], v[2]);
    const C t2 = C{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
    const C d = cscale(csub(v[1], v[2]), s3);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, cmul_negi(d));
    v[2] = csub(t2, cmul_negi(d));
  } else if constexpr (R == 4) {
    const C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const C c = cadd(v[1], v[3]), d = cmul_negi(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  } else if constexpr (R == 5) {
    const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5)
    const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
    const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
    const C p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    const C p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    const C x0 = v[0];
    const C a1 = C{x0.x + c1 * p1.x + c2 * p2.x, x0.y + c1 * p1.y + c2 * p2.y};
    const C a2 = C{x0.x + c2 * p1.x + c1 * p2.x, x0.y + c2 * p1.y + c1 * p2.y};
    const C b1 = C{s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y};
    const C b2 = C{s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y};
    v[0] = C{x0.x + p1.x + p2.x, x0.y + p1.y + p2.y};
    v[1] = cadd(a1, cmul_negi(b1));
    v[4] = csub(a1, cmul_negi(b1));
    v[2] = cadd(a2, cmul_negi(b2));
    v[3] = csub(a2, cmul_negi(b2));
  }
}

// One Stockham pass of radix R over L points in LDS, after Ns points have
// been combined: butterfly b reads buf[b + r L/R] (twiddled by
// exp(-2 pi i r (b mod Ns) / (Ns R))) and writes buf[(b / Ns) Ns R + b mod Ns
// + r Ns].  All reads of the pass land in registers before the barrier, so
// one buffer suffices.
template <typename T, int R>
__device__ inline void stockham_pass(typename V2T<T>::type* buf, int L, int Ns,
                                     const typename V2T<T>::type* roots) {
  typedef typename V2T<T>::type C;
  constexpr int MAXB = FFT_REGS / R;
  const int nb = L / R;
  const int tw = L / (Ns * R);
  C v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * FFT_THREADS;
    if (b < nb) {
      const int k = b % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[b + r * nb];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], roots[r * k * tw]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * FFT_THREADS;
    if (b < nb) {
      butterfly<T, R>(v[i]);
      const int k = b % Ns;
      const int d = (b / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[d + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// Forward DFT of L points held in LDS (result in natural order, in place).
template <typename T>
__device__ void fft_lds(typename V2T<T>::type* buf, const FftClass& c, const int32_t* rad,
                        const typename V2T<T>::type* roots) {
  int Ns = 1;
  for (int q = 0; q < c.nrad; ++q) {
    const int R = rad[q];
    if (R == 4) stockham_pass<T, 4>(buf, c.L, Ns, roots);
    else if (R == 2) stockham_pass<T, 2>(buf, c.L, Ns, roots);
    else if (R == 3) stockham_pass<T, 3>(buf, c.L, Ns, roots);
    else stockham_pass<T, 5>(buf, c.L, Ns, roots);
    Ns *= R;
  }
}

// Forward complex DFT of length h of buf[0..h); the result is left in
// buf[0..h).  For chirp-z classes buf must hold L entries.
template <typename T>
__device__ void dft_h(typename V2T<T>::type* buf, const FftClass& c, const int32_t* rad,
                      const typename V2T<T>::type* tabs) {
  typedef typename V2T<T>::type C;
  const C* roots = tabs + c.root_off;
  if (!c.bluestein) {
    fft_lds<T>(buf, c, rad, roots);
    return;
  }
  const C* chirp = tabs + c.chirp_off;
  const C* khat = tabs + c.khat_off;
  for (int t = threadIdx.x; t < c.L; t += FFT_THREADS) buf[t] = (t < c.h) ? cmul(buf[t], chirp[t]) : C{0, 0};
  __syncthreads();
  fft_lds<T>(buf, c, rad, roots);
  for (int u = threadIdx.x; u < c.L; u += FFT_THREADS) buf[u] = cconj(cmul(buf[u], khat[u]));
  __syncthreads();
  fft_lds<T>(buf, c, rad, roots);
  for (int q = threadIdx.x; q < c.h; q += FFT_THREADS) buf[q] = cmul(chirp[q], cconj(buf[q]));
  __syncthreads();
}

constexpr int FFT_FCHUNK = 16;

// ---------------------------------------------------------------------------
// Synthesis: ring j, fields [f0, f0 + FFT_FCHUNK).
//   X_m = c_m for m <= mmax_j (Im c_0 dropped), 0 above, Nyquist 0;
//   Z_q = (X_q + conj X_{h-q}) + i w^q (X_q - conj X_{h-q}),  w = exp(2 pi i / n);
//   z = inverse DFT_h(Z) (no 1/h);  g_{2t} = Re z_t,  g_{2t+1} = Im z_t.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void fourier_synthesis_kernel(DevPlan p, const int2* items,
                                                                        const T* __restrict__ four,
                                                                        T* __restrict__ grid) {
  typedef typename V2T<T>::type C;
  extern __shared__ __align__(16) unsigned char smem[];
  C* buf = (C*)smem;
  const int2 it = items[blockIdx.x];
  const RingInfo ri = p.rings[it.x];
  const FftClass cl = p.classes[ri.cls];
  const C* tabs = (const C*)p.fft;
  const C* post = tabs + cl.post_off;
  const C* fc = (const C*)four;
  const int h = cl.h, mmax = ri.mmax;
  const int fend = min(it.y + FFT_FCHUNK, p.F);
  for (int f = it.y; f < fend; ++f) {
    const C* cf = fc + ri.frow * (int64_t)p.Fp + f;
    for (int q = threadIdx.x; q < h; q += FFT_THREADS) {
      C xq = (q <= mmax) ? cf[(int64_t)q * p.Fp] : C{0, 0};
      if (q == 0) xq.y = 0;
      const int q2 = h - q;
      const C xr = (q >= 1 && q2 <= mmax) ? cconj(cf[(int64_t)q2 * p.Fp]) : C{0, 0};
      const C s = cadd(xq, xr);
      const C d = csub(xq, xr);
      const C om = cconj(post[q]);
      const C t = cmul(om, d);
      const C z = C{s.x - t.y, s.y + t.x};  // s + i t
      buf[q] = cconj(z);
    }
    __syncthreads();
    dft_h<T>(buf, cl, p.classes[ri.cls].rad, tabs);
    T* g = grid + (int64_t)f * p.npts + ri.goff;
    for (int t = threadIdx.x; t < h; t += FFT_THREADS) {
      const C r = buf[t];
      g[2 * t] = r.x;
      g[2 * t + 1] = -r.y;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Analysis: north ring j and its mirror, fields [f0, f0 + FFT_FCHUNK).
//   Z = DFT_h(z),  X_m = (Z_m + conj Z_{h-m})/2 - (i/2) w^{-m} (Z_m - conj Z_{h-m}),
//   chat_m = X_m / n;  S = w_j (chat_N + chat_S),  A = w_j (chat_N - chat_S).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void fourier_analysis_kernel(DevPlan p, const int2* items,
                                                                       const T* __restrict__ grid,
                                                                       T* __restrict__ four) {
  typedef typename V2T<T>::type C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 it = items[blockIdx.x];
  const RingInfo rn = p.rings[it.x];
  const RingInfo rs = p.rings[rn.mirror];
  const FftClass cl = p.classes[rn.cls];
  C* buf = (C*)smem;
  C* keep = buf + cl.L;
  const C* tabs = (const C*)p.fft;
  const C* post = tabs + cl.post_off;
  C* fc = (C*)four;
  const int h = cl.h, mmax = rn.mmax;
  const T scale = (T)(p.w[it.x] / (double)rn.nlon);
  const int fend = min(it.y + FFT_FCHUNK, p.F);
  for (int f = it.y; f < fend; ++f) {
    for (int side = 0; side < 2; ++side) {
      const T* g = grid + (int64_t)f * p.npts + (side ? rs.goff : rn.goff);
      for (int t = threadIdx.x; t < h; t += FFT_THREADS) buf[t] = C{g[2 * t], g[2 * t + 1]};
      __syncthreads();
      dft_h<T>(buf, cl, p.classes[rn.cls].rad, tabs);
      for (int m = threadIdx.x; m <= mmax; m += FFT_THREADS) {
        const C zm = buf[m];
        const C zr = cconj(buf[m == 0 ? 0 : h - m]);
        const C s = cadd(zm, zr);
        const C d = csub(zm, zr);
        const C t = cmul(post[m], d);
        // X = s/2 - (i/2) t
        C x = C{(T)0.5 * (s.x + t.y), (T)0.5 * (s.y - t.x)};
        if (m == 0) x = C{zm.x + zm.y, 0};
        x = cscale(x, scale);
        if (side == 0) {
          keep[m] = x;
        } else {
          const C xn = keep[m];
          C* row = fc + ((rn.frow + m) * 2) * (int64_t)p.Fp + f;
          row[0] = cadd(xn, x);
          row[p.Fp] = csub(xn, x);
        }
      }
      __syncthreads();
    }
  }
}

size_t fft_lds_bytes(int prec, int L, int mmax) {
  const size_t c = (prec == SHT_FP64) ? 16 : 8;
  return c * ((size_t)L + (size_t)mmax + 1);
}

hipError_t launch_fourier_synthesis(const DevPlan& p, int prec, const int2* items, int nitems, size_t lds,
                                    const void* four, void* grid, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(fourier_synthesis_kernel<double>, dim3(nitems), dim3(FFT_THREADS), lds, s, p, items,
                       (const double*)four, (double*)grid);
  else
    hipLaunchKernelGGL(fourier_synthesis_kernel<float>, dim3(nitems), dim3(FFT_THREADS), lds, s, p, items,
                       (const float*)four, (float*)grid);
  return hipGetLastError();
}

hipError_t launch_fourier_analysis(const DevPlan& p, int prec, const int2* items, int nitems, size_t lds,
                                   const void* grid, void* four, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(fourier_analysis_kernel<double>, dim3(nitems), dim3(FFT_THREADS), lds, s, p, items,
                       (const double*)grid, (double*)four);
  else
    hipLaunchKernelGGL(fourier_analysis_kernel<float>, dim3(nitems), dim3(FFT_THREADS), lds, s, p, items,
                       (const float*)grid, (float*)four);
  return hipGetLastError();
}

hipError_t fft_set_max_lds(size_t bytes) {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)fourier_synthesis_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)fourier_synthesis_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)fourier_analysis_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)fourier_analysis_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace shtmi
