// Kernels of the time-stepping workload: the transform pair with one
// grid-point operation between synthesis and analysis and one spectral
// operation after it, as a spectral model's time step runs (report sections
// 4.2.2-4.2.3: the loop over time steps of synthesis, grid-point
// computations and analysis, with all arrays allocated outside it).
//
// The step is semi-implicit Euler for the reaction-diffusion equation
//   du/dt = nu Lap u + r u (1 - u)
// on the unit sphere: the logistic reaction term is explicit on the grid,
//   g <- g + dt r g (1 - g),
// and the diffusion implicit in spectral space (Lap -> -n (n + 1)):
//   a_n^m <- a_n^m / (1 + dt nu n (n + 1)).
#include "sht_internal.h"

namespace shtmi {
namespace {

// g <- g + a g (1 - g) with a = dt r, 16 bytes per thread and iteration
// (the grid is 16-byte aligned); the last n % V elements one by one.
template <typename T>
__global__ void logistic_kernel(int64_t n, T a, T* __restrict__ g) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  const int64_t nv = n / V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    vec x = ((const vec*)g)[i];
    x = x + a * x * (T(1) - x);
    ((vec*)g)[i] = x;
  }
  for (int64_t i = nv * V + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T x = g[i];
    g[i] = x + a * x * (T(1) - x);
  }
}

template <typename T>
__global__ void implicit_diffusion_kernel(int N, int F, double c, T* __restrict__ spec) {
  // c = dt * nu; block (x, m, z): n = m + x * blockDim + thread
  const int m = blockIdx.y;
  const int n = m + blockIdx.x * blockDim.x + threadIdx.x;
  if (n > N) return;
  const int64_t ns = (int64_t)(N + 1) * (N + 2) / 2;
  const int64_t s = (int64_t)m * (2 * N + 3 - m) / 2 + (n - m);
  const T f = (T)(1.0 / (1.0 + c * (double)n * (n + 1)));
  for (int k = blockIdx.z; k < F; k += gridDim.z) {
    T* q = spec + 2 * ((int64_t)k * ns + s);
    q[0] *= f;
    q[1] = (m == 0) ? T(0) : q[1] * f;
  }
}

}  // namespace

hipError_t launch_logistic(int prec, int64_t n, double a, void* grid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int threads = 256;
  const int64_t per_block = (int64_t)threads * (prec == SHT_FP64 ? 2 : 4);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, 1 << 20));
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(logistic_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, s, n, a, (double*)grid);
  else
    hipLaunchKernelGGL(logistic_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, s, n, (float)a,
                       (float*)grid);
  return hipGetLastError();
}

hipError_t launch_implicit_diffusion(int prec, int N, int F, double c, void* spec, hipStream_t s) {
  const int threads = 128;
  const dim3 g((unsigned)((N + 1 + threads - 1) / threads), (unsigned)(N + 1), (unsigned)std::min(F, 1024));
  if (prec == SHT_FP64)
    hipLaunchKernelGGL(implicit_diffusion_kernel<double>, g, dim3(threads), 0, s, N, F, c, (double*)spec);
  else
    hipLaunchKernelGGL(implicit_diffusion_kernel<float>, g, dim3(threads), 0, s, N, F, c, (float*)spec);
  return hipGetLastError();
}

}  // namespace shtmi
