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
// Pbar_n^m tables.  Thread (m, r) evaluates the column n = m..N at the r-th
// north ring carrying m:
//   Pbar_0^0 = 1/sqrt(2),  Pbar_k^k = sqrt((2k+1)/(2k)) sin(theta) Pbar_{k-1}^{k-1},
//   Pbar_{m+1}^m = sqrt(2m+3) mu Pbar_m^m,
//   Pbar_n^m = a (mu Pbar_{n-1}^m - b Pbar_{n-2}^m),
//   a = sqrt((4n^2-1)/(n^2-m^2)),  b = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)).
// Even and odd n - m go to separate tables (parity 0 and 1); within a table
// element (row r, k) with n = m + parity + 2k sits in chunk k / KCH at
// [r][k % KCH].  Padding rows and columns are written as zeros.
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
  __device__ void put(int64_t e, double v) const {
    if (prec == SHT_FP64) {
      ((double*)tab)[e] = v;
    } else if (prec == SHT_FP32) {
      ((float*)tab)[e] = (float)v;
    } else {
      const float x = (float)v;
      const uint16_t hi = bf16_rne(x);
      const uint16_t lo = bf16_rne(x - bf16_to_float(hi));
      ((uint16_t*)tab)[e] = hi;
      ((uint16_t*)tab)[total + e] = lo;
    }
  }
};

__device__ inline int64_t tab_index(const MInfo& mi, int par, int r, int k) {
  return mi.toff[par] + (int64_t)(k / KCH) * mi.Lp * KCH + (int64_t)r * KCH + (k % KCH);
}

// Vector plans also store H_k^m = (1 - mu^2) dPbar_k^m/dmu for k = m..Nh
// (Nh = N, one below the Pbar degree), from the derivative identity
//   H_k = (k + 1) e_k Pbar_{k-1} - k e_{k+1} Pbar_{k+1},
//   e_k = sqrt((k^2 - m^2) / (4 k^2 - 1))   (e_m = 0),
// evaluated as soon as the recurrence has produced Pbar_{k+1}.  H has the
// opposite parity in mu to Pbar (H_k(-mu) = -(-1)^{k-m} H_k(mu)), so its
// table puts odd k - m in plane 0 (paired, like Pbar's plane 0, with the
// symmetric part of the data) and even k - m in plane 1; `hms` describes
// that layout (K[0] = number of odd k - m, K[1] = number of even).
__device__ inline double eps_nm(int k, int m) {
  if (k <= m) return 0.0;
  return sqrt(((double)k * k - (double)m * m) / (4.0 * (double)k * k - 1.0));
}

__global__ void pbar_kernel(DevPlan p, const MInfo* ms, TabStore st, const MInfo* hms, TabStore hst, int Nh) {
  const MInfo mi = ms[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mi.Lp) return;
  const int m = mi.m;
  const int N = p.N;
  const bool with_h = (hms != nullptr);
  MInfo hi{};
  if (with_h) hi = hms[blockIdx.y];
  if (r >= mi.L) {
    for (int par = 0; par < 2; ++par)
      for (int k = 0; k < mi.Kp[par]; ++k) st.put(tab_index(mi, par, r, k), 0.0);
    if (with_h)
      for (int par = 0; par < 2; ++par)
        for (int k = 0; k < hi.Kp[par]; ++k) hst.put(tab_index(hi, par, r, k), 0.0);
    return;
  }
  const double x = p.mu[mi.first_ring + r];
  const double s = sqrt((1.0 - x) * (1.0 + x));
  // H_k once Pbar_{k-1} (pkm1) and Pbar_{k+1} (pkp1) are known
  auto put_h = [&](int k, double pkm1, double pkp1) {
    if (!with_h || k > Nh) return;
    const double h = (k + 1.0) * eps_nm(k, m) * pkm1 - (double)k * eps_nm(k + 1, m) * pkp1;
    const int d = k - m;
    hst.put(tab_index(hi, (d & 1) ? 0 : 1, r, d >> 1), h);
  };
  double pmm = 1.0 / sqrt(2.0);
  for (int k = 1; k <= m; ++k) pmm = sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * pmm;
  st.put(tab_index(mi, 0, r, 0), pmm);
  if (N > m) {
    double p2 = pmm;
    double p1 = sqrt(2.0 * m + 3.0) * x * pmm;
    st.put(tab_index(mi, 1, r, 0), p1);
    put_h(m, 0.0, p1);
    for (int n = m + 2; n <= N; ++n) {
      const double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      const double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
      const double pn = a * (x * p1 - b * p2);
      st.put(tab_index(mi, (n - m) & 1, r, (n - m) >> 1), pn);
      put_h(n - 1, p2, pn);
      p2 = p1;
      p1 = pn;
    }
  }
  for (int par = 0; par < 2; ++par)
    for (int k = mi.K[par]; k < mi.Kp[par]; ++k) st.put(tab_index(mi, par, r, k), 0.0);
  if (with_h)
    for (int par = 0; par < 2; ++par)
      for (int k = hi.K[par]; k < hi.Kp[par]; ++k) hst.put(tab_index(hi, par, r, k), 0.0);
}

hipError_t launch_pbar_planes(const DevPlan& p, int prec, const MInfo* d_ms, int nm, int max_Lp,
                              void* tab, int64_t plane_elems, const MInfo* d_hms, void* htab, int64_t hplane_elems,
                              int Nh, hipStream_t s) {
  TabStore st{prec, tab, plane_elems};
  TabStore hst{prec, htab, hplane_elems};
  const int bs = 64;
  hipLaunchKernelGGL(pbar_kernel, dim3((max_Lp + bs - 1) / bs, nm), dim3(bs), 0, s, p, d_ms, st, d_hms, hst, Nh);
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
// FFT tables, one work group per class.  Angles are reduced exactly in
// integer arithmetic before one float64 sincospi call:
//   twiddles, pass after pass (radix R after Ns points are combined):
//          exp(-2 pi i r k / (Ns R))             k < Ns, 1 <= r < R
//   post   exp(-2 pi i q / (2h))                   q < h
//   chirp  exp(-i pi (t^2 mod 2h) / h)             t < h
//   khat_u = (1/L) sum_{|t| < h} exp(+i pi t^2/h) exp(-2 pi i u t / L)
// khat is the length-L DFT of the conjugate chirp wrapped around zero, i.e.
// the kernel of the chirp-z (Bluestein) convolution, with the 1/L of the
// inverse DFT folded in.
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
  // khat: phase of term t is pi (t^2 L - 2 u t h) / (h L), reduced mod 2 h L
  const int64_t hl = (int64_t)h * L;
  for (int u = threadIdx.x; u < L; u += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int t = -(h - 1); t <= h - 1; ++t) {
      int64_t num = ((int64_t)t * t) * L - 2 * (int64_t)u * t * h;
      num %= 2 * hl;
      if (num < 0) num += 2 * hl;
      double sn, cs;
      sincospi((double)num / (double)hl, &sn, &cs);
      re += cs;
      im += sn;
    }
    put_c(fft, c.khat_off + u, re / L, im / L);
  }
}

hipError_t launch_fft_tables(const DevPlan& p, int prec, const FftClass* d_cls, int ncls,
                             const FftClass* h_cls, void* fft, hipStream_t s) {
  (void)p;
  (void)h_cls;
  if (ncls == 0) return hipSuccess;
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(fft_tables_kernel<double>, dim3(ncls), dim3(256), 0, s, d_cls, (double*)fft);
  else
    hipLaunchKernelGGL(fft_tables_kernel<float>, dim3(ncls), dim3(256), 0, s, d_cls, (float*)fft);
  return hipGetLastError();
}

}  // namespace shtmi
