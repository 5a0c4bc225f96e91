// Spectral-space kernels of the derivative and vector (wind) transforms.
//
// The report's reason for the spectral method is that derivatives become
// pointwise operations on the coefficients (section 4.4.1).  On the unit
// sphere, with mu = sin(latitude):
//   d/dlambda of a_n^m Pbar_n^m e^{i m lambda}  ->  i m a_n^m;
//   the horizontal Laplacian                     ->  -n (n + 1) a_n^m;
//   (1 - mu^2) dPbar_n^m/dmu = (n + 1) e_n Pbar_{n-1}^m - n e_{n+1} Pbar_{n+1}^m,
//   e_n = e_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)),
// the last being the derivative identity of the normalised associated
// Legendre functions combined with their three-term recurrence.
//
// Winds U = u cos(lat), V = v cos(lat) from vorticity zeta and divergence D
// (zeta = Lap psi, D = Lap chi):
//   U = dchi/dlambda - (1 - mu^2) dpsi/dmu,   V = dpsi/dlambda + (1 - mu^2) dchi/dmu.
// With the identity above, the mu derivative moves into spectral space as a
// two-term combination of neighbouring degrees, so U and V are scalar
// syntheses of degree up to N + 1:
//   U_k = i m chi_k + (k - 1) e_k psi_{k-1} - (k + 2) e_{k+1} psi_{k+1}
//   V_k = i m psi_k - (k - 1) e_k chi_{k-1} + (k + 2) e_{k+1} chi_{k+1}
// for k = m .. N + 1 (psi, chi zero above N): the synthesis needs only the
// Pbar table, extended by one degree.
//
// The inverse relations, integrated by parts over mu and evaluated by the
// same Gaussian quadrature with q_j = w_j / (1 - mu_j^2):
//   zeta_n = sum_j q_j [i m V_{j,m} Pbar_n(mu_j) + U_{j,m} H_n(mu_j)]
//   D_n    = sum_j q_j [i m U_{j,m} Pbar_n(mu_j) - V_{j,m} H_n(mu_j)]
// with H_n = (1 - mu^2) dPbar_n/dmu.  The same identity would turn the H
// sums into -n e_{n+1} Uh_{n+1} + (n + 1) e_n Uh_{n-1} of the Pbar analyses
// Uh of U / (1 - mu^2), but that difference of two large neighbours cancels
// (Uh decays slowly: U / (1 - mu^2) is not smooth at the poles) and
// multiplies the rounding of the products by up to ~N; the analysis
// therefore takes H from a table of its own (computed in float64 with the
// Pbar table) and forms the two projections PU, PV (Pbar) and HU, HV (H) as
// matrix products, combined here.
//
// All arithmetic here is float64; values are rounded once to the data type
// on store.  Im of every m = 0 coefficient is ignored on input and written
// as 0.
#include "sht_internal.h"

namespace shtmi {
namespace {

template <typename T>
struct Cx {
  double re, im;
};

// complex index of (m, n) in the m-major triangular layout of degree D
__device__ __forceinline__ int64_t slot(int D, int m, int n) { return (int64_t)m * (2 * D + 3 - m) / 2 + (n - m); }

__device__ __forceinline__ double eps(int n, int m) {
  const double a = (double)n * n - (double)m * m;
  return sqrt(a / (4.0 * (double)n * n - 1.0));
}

template <typename T>
__device__ __forceinline__ Cx<T> load(const T* base, int64_t c, bool real_only) {
  const T* q = base + 2 * c;
  return Cx<T>{(double)q[0], real_only ? 0.0 : (double)q[1]};
}

template <typename T>
__device__ __forceinline__ void store(T* base, int64_t c, double re, double im) {
  T* q = base + 2 * c;
  q[0] = (T)re;
  q[1] = (T)im;
}

// U, V spectral coefficients (degree N + 1, rows f and F + f of `uv`) of
// vector field f, from vorticity / divergence (rows f and F + f of `in`,
// degree N) or, with `gradient`, from one scalar field (row f of `in`: chi =
// the field, psi = 0).  Block (x, m, z): k = m + x * blockDim + thread.
template <typename T>
__global__ void uv_from_potentials_kernel(int N, int F, bool gradient, const T* __restrict__ in, T* __restrict__ uv) {
  const int m = blockIdx.y;
  const int k = m + blockIdx.x * blockDim.x + threadIdx.x;
  const int D = N + 1;
  if (k > D) return;
  const int64_t nsN = (int64_t)(N + 1) * (N + 2) / 2;
  const int64_t nsD = (int64_t)(D + 1) * (D + 2) / 2;
  const bool m0 = (m == 0);
  for (int f = blockIdx.z; f < F; f += gridDim.z) {
    // psi_n and chi_n for n in {k-1, k, k+1} (zero outside m..N)
    double pr[3] = {0, 0, 0}, pi[3] = {0, 0, 0}, cr[3] = {0, 0, 0}, ci[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
      const int n = k - 1 + d;
      if (n < m || n > N || n == 0) continue;
      const double il = -1.0 / ((double)n * (n + 1));
      if (gradient) {
        const Cx<T> a = load(in + (int64_t)f * 2 * nsN, slot(N, m, n), m0);
        cr[d] = a.re;
        ci[d] = a.im;
      } else {
        const Cx<T> z = load(in + (int64_t)f * 2 * nsN, slot(N, m, n), m0);
        const Cx<T> dv = load(in + (int64_t)(F + f) * 2 * nsN, slot(N, m, n), m0);
        pr[d] = il * z.re;
        pi[d] = il * z.im;
        cr[d] = il * dv.re;
        ci[d] = il * dv.im;
      }
    }
    const double em = (double)m;
    const double lo = (k > m) ? (k - 1.0) * eps(k, m) : 0.0;  // (k - 1) e_k
    const double hi = (k + 2.0) * eps(k + 1, m);               // (k + 2) e_{k+1}
    // i m x = (-m x.im, m x.re)
    const double ur = -em * ci[1] + lo * pr[0] - hi * pr[2];
    const double ui = em * cr[1] + lo * pi[0] - hi * pi[2];
    const double vr = -em * pi[1] - lo * cr[0] + hi * cr[2];
    const double vi = em * pr[1] - lo * ci[0] + hi * ci[2];
    store(uv + (int64_t)f * 2 * nsD, slot(D, m, k), ur, m0 ? 0.0 : ui);
    store(uv + (int64_t)(F + f) * 2 * nsD, slot(D, m, k), vr, m0 ? 0.0 : vi);
  }
}

// Vorticity and divergence (degree N, rows f and F + f of `out`) from the
// projections of q U and q V on Pbar (`pw`, rows f and F + f, degree N + 1
// layout) and on H (`hw`, same rows and layout; the H table's planes hold odd
// n - m in plane 0 and even n - m in plane 1, so the value of degree n sits
// at n + 1 when n - m is even and at n - 1 when it is odd).
template <typename T>
__global__ void vortdiv_from_projections_kernel(int N, int F, const T* __restrict__ pw, const T* __restrict__ hw,
                                                T* __restrict__ out) {
  const int m = blockIdx.y;
  const int n = m + blockIdx.x * blockDim.x + threadIdx.x;
  if (n > N) return;
  const int D = N + 1;
  const int64_t nsN = (int64_t)(N + 1) * (N + 2) / 2;
  const int64_t nsD = (int64_t)(D + 1) * (D + 2) / 2;
  const bool m0 = (m == 0);
  const double em = (double)m;
  const int nh = ((n - m) & 1) ? n - 1 : n + 1;
  for (int f = blockIdx.z; f < F; f += gridDim.z) {
    const Cx<T> pu = load(pw + (int64_t)f * 2 * nsD, slot(D, m, n), m0);
    const Cx<T> pv = load(pw + (int64_t)(F + f) * 2 * nsD, slot(D, m, n), m0);
    const Cx<T> hu = load(hw + (int64_t)f * 2 * nsD, slot(D, m, nh), m0);
    const Cx<T> hv = load(hw + (int64_t)(F + f) * 2 * nsD, slot(D, m, nh), m0);
    const double zr = -em * pv.im + hu.re;
    const double zi = em * pv.re + hu.im;
    const double dr = -em * pu.im - hv.re;
    const double di = em * pu.re - hv.im;
    const bool mean = (n == 0);  // zeta_0^0 = D_0^0 = 0
    store(out + (int64_t)f * 2 * nsN, slot(N, m, n), mean ? 0.0 : zr, m0 ? 0.0 : zi);
    store(out + (int64_t)(F + f) * 2 * nsN, slot(N, m, n), mean ? 0.0 : dr, m0 ? 0.0 : di);
  }
}

// Pointwise spectral operators on `count` fields of degree N (in place
// allowed).
template <typename T>
__global__ void spectral_op_kernel(int N, int count, int op, const T* in, T* out) {
  const int m = blockIdx.y;
  const int n = m + blockIdx.x * blockDim.x + threadIdx.x;
  if (n > N) return;
  const int64_t ns = (int64_t)(N + 1) * (N + 2) / 2;
  const bool m0 = (m == 0);
  double fr = 0.0, fi = 0.0;  // out = (fr + i fi) * in
  if (op == SHT_OP_DLAMBDA) {
    fi = (double)m;
  } else if (op == SHT_OP_LAPLACIAN) {
    fr = -(double)n * (n + 1);
  } else if (n > 0) {
    fr = -1.0 / ((double)n * (n + 1));
  }
  for (int f = blockIdx.z; f < count; f += gridDim.z) {
    const Cx<T> a = load(in + (int64_t)f * 2 * ns, slot(N, m, n), m0);
    const double re = fr * a.re - fi * a.im;
    const double im = fr * a.im + fi * a.re;
    store(out + (int64_t)f * 2 * ns, slot(N, m, n), re, m0 ? 0.0 : im);
  }
}

__global__ void analysis_weight_kernel(int nlat, const double* mu, const double* w, double* wa) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlat) return;
  const double x = mu[j];
  wa[j] = w[j] / ((1.0 - x) * (1.0 + x));
}

constexpr int kThreads = 128;

dim3 spectral_grid(int kmax_plus1, int nm, int fields) {
  return dim3((unsigned)((kmax_plus1 + kThreads - 1) / kThreads), (unsigned)nm,
              (unsigned)std::min(std::max(fields, 1), 1024));
}

}  // namespace

hipError_t launch_uv_from_potentials(int N, int F, bool gradient, int prec, const void* in, void* uv, hipStream_t s) {
  const dim3 g = spectral_grid(N + 2, N + 1, F);
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(uv_from_potentials_kernel<double>, g, dim3(kThreads), 0, s, N, F, gradient,
                       (const double*)in, (double*)uv);
  else
    hipLaunchKernelGGL(uv_from_potentials_kernel<float>, g, dim3(kThreads), 0, s, N, F, gradient,
                       (const float*)in, (float*)uv);
  return hipGetLastError();
}

hipError_t launch_vortdiv_from_projections(int N, int F, int prec, const void* pw, const void* hw, void* out,
                                           hipStream_t s) {
  const dim3 g = spectral_grid(N + 1, N + 1, F);
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(vortdiv_from_projections_kernel<double>, g, dim3(kThreads), 0, s, N, F, (const double*)pw,
                       (const double*)hw, (double*)out);
  else
    hipLaunchKernelGGL(vortdiv_from_projections_kernel<float>, g, dim3(kThreads), 0, s, N, F, (const float*)pw,
                       (const float*)hw, (float*)out);
  return hipGetLastError();
}

hipError_t launch_spectral_op(int N, int count, int op, int prec, const void* in, void* out, hipStream_t s) {
  const dim3 g = spectral_grid(N + 1, N + 1, count);
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(spectral_op_kernel<double>, g, dim3(kThreads), 0, s, N, count, op, (const double*)in,
                       (double*)out);
  else
    hipLaunchKernelGGL(spectral_op_kernel<float>, g, dim3(kThreads), 0, s, N, count, op, (const float*)in,
                       (float*)out);
  return hipGetLastError();
}

hipError_t launch_analysis_weight(int nlat, const double* mu, const double* w, double* wa, hipStream_t s) {
  hipLaunchKernelGGL(analysis_weight_kernel, dim3((nlat + 63) / 64), dim3(64), 0, s, nlat, mu, w, wa);
  return hipGetLastError();
}

}  // namespace shtmi
