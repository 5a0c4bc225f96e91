// Plan-time kernels: Gaussian latitudes and weights, normalised associated
// Legendre tables, and the twiddle / chirp tables of the ring FFTs.  All
// arithmetic is float64; values are rounded once to the table type.
#include "sht_internal.h"

#include <cmath>

namespace shtmi {

// ---------------------------------------------------------------------------
// Gaussian latitudes: roots of the Legendre polynomial P_nlat by Newton
// iteration, one thread per root of the north half.  P_n and P_{n-1} come
// from the three-term recurrence k P_k = (2k-1) mu P_{k-1} - (k-1) P_{k-2};
// the derivative is P'_n = n (P_{n-1} - mu P_n) / (1 - mu^2) and the weight
// 2 / ((1 - mu^2) P'_n^2).  1 - mu^2 is formed as (1 - mu)(1 + mu) so that it
// keeps its relative accuracy at the rings nearest the poles.
// ---------------------------------------------------------------------------

__device__ static void legendre_pair(int n, double x, double* pn, double* pn1) {
  double pm = 1.0, p = x;
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p - (k - 1.0) * pm) / k;
    pm = p;
    p = pk;
  }
  *pn = p;
  *pn1 = pm;
}

__global__ void gauss_kernel(int nlat, double* mu, double* w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int nh = nlat / 2;
  if (j >= nh) return;
  double x = cos(M_PI * ((j + 1) - 0.25) / (nlat + 0.5));
  double p, pm;
  for (int it = 0; it < 100; ++it) {
    legendre_pair(nlat, x, &p, &pm);
    const double one_m = (1.0 - x) * (1.0 + x);
    const double dp = nlat * (pm - x * p) / one_m;
    const double step = p / dp;
    x -= step;
    if (fabs(step) < 1e-15) break;
  }
  legendre_pair(nlat, x, &p, &pm);
  const double one_m = (1.0 - x) * (1.0 + x);
  const double dp = nlat * (pm - x * p) / one_m;
  const double wt = 2.0 / (one_m * dp * dp);
  mu[j] = x;
  mu[nlat - 1 - j] = -x;
  w[j] = wt;
  w[nlat - 1 - j] = wt;
}

hipError_t launch_gauss(int nlat, double* mu, double* w, hipStream_t s) {
  const int nh = nlat / 2;
  hipLaunchKernelGGL(gauss_kernel, dim3((nh + 63) / 64), dim3(64), 0, s, nlat, mu, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pbar_n^m tables.  Thread (m, r) evaluates the column n = m..D (D the
// table degree) at the r-th north ring carrying m:
//   Pbar_0^0 = 1/sqrt(2),  Pbar_k^k = f_k sin(theta) Pbar_{k-1}^{k-1},  f_k = sqrt((2k+1)/(2k)),
//   Pbar_n^m = a_n (mu Pbar_{n-1}^m - b_n Pbar_{n-2}^m)   (n > m, Pbar_{m-1}^m = 0),
//   a_n = sqrt((4n^2-1)/(n^2-m^2)),  b_n = e_{n-1},  e_n = sqrt((n^2-m^2)/(4n^2-1)),  e_m = 0
// (at n = m + 1, a_n = sqrt(2m+3)).  The factors f_k and the pairs
// (a_n, e_n) per (m, n) are computed once, in float64, by pbar_coef_kernel;
// in pbar_kernel they are the same for every lane (scalar loads), so no
// thread takes a square root per n.
// Even and odd n - m go to separate tables (parity 0 and 1); within a table
// element (row r, k) with n = m + parity + 2k sits in chunk k / KCH at
// [r][k % KCH].  The thread walks n - m in blocks of 2 KCH = 16: a block
// fills exactly one chunk row of each parity (even and odd n - m), so the
// values stay in registers (static indices) and leave as two 8-value
// stores; lanes of consecutive rings write consecutive chunk rows.  Past
// n = D the coefficients are zero, so the recurrence yields zeros there,
// and rows past L start from zero: padding rows and columns are written as
// zeros by the same code.
// ---------------------------------------------------------------------------

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

struct TabStore {
  int prec;
  void* tab;
  int64_t total;  // elements per plane (bf16 split: hi plane then lo plane)
  // KCH consecutive elements from e (a multiple of KCH), rounded once each
  __device__ void put8(int64_t e, const double* v) const {
    static_assert(KCH == 8, "chunk rows of 8");
    if (prec == SHT_FP64) {
      double2* d = (double2*)((double*)tab + e);
#pragma unroll
      for (int i = 0; i < 4; ++i) gstore(d + i, make_double2(v[2 * i], v[2 * i + 1]));
    } else if (prec == SHT_FP32) {
      float4* d = (float4*)((float*)tab + e);
      gstore(d, make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]));
      gstore(d + 1, make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]));
    } else {
      uint32_t h[4], l[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float x0 = (float)v[2 * i], x1 = (float)v[2 * i + 1];
        const uint16_t h0 = bf16_rne(x0), h1 = bf16_rne(x1);
        const uint16_t l0 = bf16_rne(x0 - bf16_to_float(h0)), l1 = bf16_rne(x1 - bf16_to_float(h1));
        h[i] = (uint32_t)h0 | ((uint32_t)h1 << 16);
        l[i] = (uint32_t)l0 | ((uint32_t)l1 << 16);
      }
      gstore((uint4*)((uint16_t*)tab + e), make_uint4(h[0], h[1], h[2], h[3]));
      gstore((uint4*)((uint16_t*)tab + total + e), make_uint4(l[0], l[1], l[2], l[3]));
    }
  }
};

__device__ inline int64_t tab_index(const MInfo& mi, int par, int r, int k) {
  return mi.toff[par] + (int64_t)(k / KCH) * mi.Lp * KCH + (int64_t)r * KCH + (k % KCH);
}

// Coefficients: f_k (k = 0..D; f_0 unused) and, per m, (a_n, e_n) at
// coef[coff(m) + n - m] for n - m = 0..pbar_coef_count(D, m) - 1, zero
// where n - m = 0 (a_m and e_m) or n > D.
__global__ void pbar_coef_kernel(int D, const MInfo* ms, int nm, double* sect, double2* coef) {
  const int m = blockIdx.y;
  if (m >= nm) return;
  const MInfo mi = ms[m];
  const int cnt = pbar_coef_count(D, mi.m);
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < cnt; d += gridDim.x * blockDim.x) {
    const int n = mi.m + d;
    const double nn = (double)n * n, mm = (double)mi.m * mi.m;
    const bool live = d >= 1 && n <= D;
    const double a = live ? sqrt((4.0 * nn - 1.0) / (nn - mm)) : 0.0;
    const double e = live ? sqrt((nn - mm) / (4.0 * nn - 1.0)) : 0.0;
    coef[mi.coff + d] = make_double2(a, e);
  }
  if (m == 0)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= D; k += gridDim.x * blockDim.x)
      sect[k] = k >= 1 ? sqrt((2.0 * k + 1.0) / (2.0 * k)) : 0.0;
}

// Vector plans also store H_k^m = (1 - mu^2) dPbar_k^m/dmu for k = m..Nh
// (Nh = N, one below the Pbar degree), from the derivative identity
//   H_k = (k + 1) e_k Pbar_{k-1} - k e_{k+1} Pbar_{k+1}   (e_m = 0),
// formed in the same blocks of 16 from the Pbar values around k.  H has the
// opposite parity in mu to Pbar (H_k(-mu) = -(-1)^{k-m} H_k(mu)), so its
// table puts odd k - m in plane 0 (paired, like Pbar's plane 0, with the
// symmetric part of the data) and even k - m in plane 1; `hms` describes
// that layout (K[0] = number of odd k - m, K[1] = number of even).
__global__ void pbar_kernel(DevPlan p, const MInfo* ms, TabStore st, const MInfo* hms, TabStore hst, int Nh,
                            const double* sect, const double2* coef) {
  constexpr int B = 2 * KCH;
  const MInfo mi = ms[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mi.Lp) return;
  const int m = mi.m;
  const int D = p.N;
  const bool with_h = (hms != nullptr);
  MInfo hi{};
  if (with_h) hi = hms[blockIdx.y];
  double x = 0.0, pmm = 0.0;  // rows past L: every value is zero
  if (r < mi.L) {
    x = p.mu[mi.first_ring + r];
    const double s = sqrt((1.0 - x) * (1.0 + x));
    pmm = 1.0 / sqrt(2.0);
    for (int k = 1; k <= m; ++k) pmm = sect[k] * s * pmm;
  }
  const double2* cf = coef + mi.coff;
  const int nb = (D - m + B) / B;  // blocks covering n - m = 0..D - m
  double prev = 0.0, cur = pmm;   // Pbar at n - m = B c - 1 and B c
  for (int c = 0; c < nb; ++c) {
    const double2* q = cf + B * c;
    double v[B + 1];  // Pbar at n - m = B c + j
    v[0] = cur;
    double p2 = prev, p1 = cur;
#pragma unroll
    for (int j = 1; j <= B; ++j) {
      const double pn = q[j].x * __fma_rn(x, p1, -(q[j - 1].y * p2));
      v[j] = pn;
      p2 = p1;
      p1 = pn;
    }
    double ev[KCH], od[KCH];
#pragma unroll
    for (int i = 0; i < KCH; ++i) {
      ev[i] = v[2 * i];
      od[i] = v[2 * i + 1];
    }
    st.put8(tab_index(mi, 0, r, KCH * c), ev);
    if (KCH * c < mi.Kp[1]) st.put8(tab_index(mi, 1, r, KCH * c), od);
    if (with_h) {
      double hv[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int d = B * c + j, k = m + d;
        const double below = j == 0 ? prev : v[j - 1];
        const double h = (k + 1.0) * q[j].y * below - (double)k * q[j + 1].y * v[j + 1];
        hv[j] = k <= Nh ? h : 0.0;
      }
      double hodd[KCH], hev[KCH];
#pragma unroll
      for (int i = 0; i < KCH; ++i) {
        hev[i] = hv[2 * i];
        hodd[i] = hv[2 * i + 1];
      }
      if (KCH * c < hi.Kp[0]) hst.put8(tab_index(hi, 0, r, KCH * c), hodd);
      if (KCH * c < hi.Kp[1]) hst.put8(tab_index(hi, 1, r, KCH * c), hev);
    }
    prev = v[B - 1];
    cur = v[B];
  }
}

hipError_t launch_pbar_planes(const DevPlan& p, int prec, const MInfo* d_ms, int nm, int max_Lp,
                              void* tab, int64_t plane_elems, const MInfo* d_hms, void* htab, int64_t hplane_elems,
                              int Nh, const double* sect, const double2* coef, hipStream_t s) {
  TabStore st{prec, tab, plane_elems};
  TabStore hst{prec, htab, hplane_elems};
  const int bs = 64;
  hipLaunchKernelGGL(pbar_kernel, dim3((max_Lp + bs - 1) / bs, nm), dim3(bs), 0, s, p, d_ms, st, d_hms, hst, Nh,
                     sect, coef);
  return hipGetLastError();
}

hipError_t launch_pbar_coef(int D, const MInfo* d_ms, int nm, double* sect, double2* coef, hipStream_t s) {
  hipLaunchKernelGGL(pbar_coef_kernel, dim3(4, nm), dim3(256), 0, s, D, d_ms, nm, sect, coef);
  return hipGetLastError();
}

// Copy one wavenumber's table back as float64 [L][N-m+1] (tests).
__global__ void table_export_kernel(MInfo mi, int N, int prec, const void* tab, int64_t plane,
                                    double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ncol = N - mi.m + 1;
  if (idx >= (int64_t)mi.L * ncol) return;
  const int r = (int)(idx / ncol);
  const int d = (int)(idx % ncol);
  const int64_t e = tab_index(mi, d & 1, r, d >> 1);
  double v;
  if (prec == SHT_FP64) v = ((const double*)tab)[e];
  else if (prec == SHT_FP32) v = ((const float*)tab)[e];
  else v = (double)bf16_to_float(((const uint16_t*)tab)[e]) + (double)bf16_to_float(((const uint16_t*)tab)[plane + e]);
  out[idx] = v;
}

hipError_t launch_table_export_planes(const DevPlan& p, int prec, const MInfo& mi, int64_t plane,
                                      double* out, hipStream_t s) {
  const int64_t n = (int64_t)mi.L * (p.N - mi.m + 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(table_export_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mi, p.N, prec,
                     p.tab, plane, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FFT tables.  fft_tables_kernel, one work group per class, reduces each
// angle exactly in integer arithmetic before one float64 sincospi call:
//   twiddles, pass after pass (radix R after Ns points are combined):
//          exp(-2 pi i r k / (Ns R))             k < Ns, 1 <= r < R
//   post   exp(-2 pi i q / (2h))                   q < h
//   chirp  exp(-i pi (t^2 mod 2h) / h)             t < h
// khat_kernel makes the chirp-z (Bluestein) convolution kernel, the
// length-L DFT of the conjugate chirp wrapped around zero with the 1/L of
// the inverse DFT folded in:
//   khat_u = (1/L) sum_{|t| < h} c_t exp(-2 pi i u t / L),  c_t = exp(i pi t^2 / h).
// c_t is even in t, so the terms t and -t pair into a real cosine:
//   khat_u = (1/L) (1 + 2 sum_{t=1}^{h-1} c_t cos(2 pi j / L)),  j = u t mod L,
// with j advanced by u per term and cos(2 pi j / L) = Re(W_hi[j >> 8] W_lo[j & 255])
// from two float64 tables of unit roots exp(-2 pi i j / L) in LDS; c_t comes
// in chunks of KH_CHUNK from sincospi of (t^2 mod 2h) / h.  Every value is
// formed in float64 (about three roundings per term against one for a
// sincospi per term, which cost an int64 remainder each and made the kernel
// 40 to 80 times slower).
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline void put_c(T* base, int64_t i, double re, double im) {
  base[2 * i] = (T)re;
  base[2 * i + 1] = (T)im;
}

template <typename T>
__global__ void fft_tables_kernel(const FftClass* cls, T* fft) {
  const FftClass c = cls[blockIdx.x];
  const int L = c.L, h = c.h;
  int64_t off = c.root_off;
  int Ns = 1;
  for (int pass = 0; pass < c.nrad; ++pass) {
    const int R = c.rad[pass];
    const int NR = Ns * R;
    for (int e = threadIdx.x; e < Ns * (R - 1); e += blockDim.x) {
      const int k = e / (R - 1);
      const int r = e % (R - 1) + 1;
      double sn, cs;
      sincospi(-2.0 * (double)((r * k) % NR) / (double)NR, &sn, &cs);
      put_c(fft, off + e, cs, sn);
    }
    off += Ns * (R - 1);
    Ns = NR;
  }
  for (int q = threadIdx.x; q < h; q += blockDim.x) {
    double sn, cs;
    sincospi(-(double)q / (double)h, &sn, &cs);
    put_c(fft, c.post_off + q, cs, sn);
  }
  if (!c.bluestein) return;
  for (int t = threadIdx.x; t < h; t += blockDim.x) {
    const int64_t r = ((int64_t)t * t) % (2 * (int64_t)h);
    double sn, cs;
    sincospi(-(double)r / (double)h, &sn, &cs);
    put_c(fft, c.chirp_off + t, cs, sn);
  }
}

constexpr int KH_THREADS = 256, KH_LO = 256, KH_HI = 512, KH_CHUNK = 512;
// lengths the two root tables cover
constexpr int64_t KH_MAX_L = (int64_t)KH_LO * KH_HI;

// block (x, class): u = x KH_THREADS + thread
template <typename T>
__global__ void khat_kernel(const FftClass* cls, T* fft) {
  const FftClass c = cls[blockIdx.y];
  if (!c.bluestein) return;
  const int L = c.L, h = c.h;
  const int u0 = blockIdx.x * KH_THREADS;
  if (u0 >= L) return;
  __shared__ double2 wlo[KH_LO], whi[KH_HI], ct[KH_CHUNK];
  const int nhi = (L + KH_LO - 1) / KH_LO;
  for (int j = threadIdx.x; j < KH_LO; j += KH_THREADS) {
    double sn, cs;
    sincospi(-2.0 * (double)j / (double)L, &sn, &cs);
    wlo[j] = make_double2(cs, sn);
  }
  for (int j = threadIdx.x; j < nhi; j += KH_THREADS) {
    double sn, cs;
    sincospi(-2.0 * (double)(((int64_t)j * KH_LO) % L) / (double)L, &sn, &cs);
    whi[j] = make_double2(cs, sn);
  }
  const int u = u0 + threadIdx.x;
  double re = 0.0, im = 0.0;
  int j = 0;  // u t mod L
  for (int t0 = 1; t0 < h; t0 += KH_CHUNK) {
    const int n = min(KH_CHUNK, h - t0);
    __syncthreads();  // the previous chunk is consumed (and the root tables are written)
    for (int i = threadIdx.x; i < n; i += KH_THREADS) {
      const int64_t t = t0 + i;
      double sn, cs;
      sincospi((double)((t * t) % (2 * (int64_t)h)) / (double)h, &sn, &cs);
      ct[i] = make_double2(cs, sn);
    }
    __syncthreads();
    if (u < L) {
      for (int i = 0; i < n; ++i) {
        j += u;
        if (j >= L) j -= L;
        const double2 a = whi[j >> 8], b = wlo[j & (KH_LO - 1)];
        const double w = a.x * b.x - a.y * b.y;  // cos(2 pi j / L)
        const double2 cv = ct[i];
        re = fma(cv.x, w, re);
        im = fma(cv.y, w, im);
      }
    }
  }
  if (u < L) put_c(fft, c.khat_off + u, (1.0 + 2.0 * re) / L, (2.0 * im) / L);
}

hipError_t launch_fft_tables(const DevPlan& p, int prec, const FftClass* d_cls, int ncls,
                             const FftClass* h_cls, void* fft, hipStream_t s) {
  (void)p;
  if (ncls == 0) return hipSuccess;
  int maxL = 0;
  for (int i = 0; i < ncls; ++i)
    if (h_cls[i].bluestein) {
      if ((int64_t)h_cls[i].L > KH_MAX_L) return hipErrorInvalidValue;
      maxL = std::max(maxL, h_cls[i].L);
    }
  const dim3 kg((unsigned)std::max(1, (maxL + KH_THREADS - 1) / KH_THREADS), (unsigned)ncls);
  if (prec == SHT_FP64) {
    hipLaunchKernelGGL(fft_tables_kernel<double>, dim3(ncls), dim3(256), 0, s, d_cls, (double*)fft);
    if (maxL > 0) hipLaunchKernelGGL(khat_kernel<double>, kg, dim3(KH_THREADS), 0, s, d_cls, (double*)fft);
  } else {
    hipLaunchKernelGGL(fft_tables_kernel<float>, dim3(ncls), dim3(256), 0, s, d_cls, (float*)fft);
    if (maxL > 0) hipLaunchKernelGGL(khat_kernel<float>, kg, dim3(KH_THREADS), 0, s, d_cls, (float*)fft);
  }
  return hipGetLastError();
}

}  // namespace shtmi
