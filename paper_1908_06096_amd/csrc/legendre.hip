// Legendre transform as one matrix product per zonal wavenumber m, split into
// the symmetric and antisymmetric halves (even and odd n - m), on gfx950
// MFMA.  The report (section 4.2.4) runs these products as zero-padded,
// uniform-size batched DGEMMs; here a flat work list covers every
// (m, row tile, column tile) of every product at its own size, so no
// padding flops are issued beyond the last partial tile of each m.
//
// Operand layouts (k indexes n = m + parity + 2k):
//   tables   per (m, parity): chunks of KCH k, each [rows][KCH]
//   spectral [F][nspec] complex; column c = 2 f + (0: re, 1: im)
//   Fourier  synthesis form  row (four_row[j] + m), 2 Fp reals per row
//            analysis form   row ((four_row[j] + m) * 2 + parity)
//
// MFMA 16x16x4 (f32 and f64) operand placement, lane l of a wave:
//   A[row l % 16][k l / 16], B[k l / 16][col l % 16];
//   accumulator element i holds D[row][col l % 16] with
//   row = 4 (l / 16) + i for f32 and row = 4 i + l / 16 for f64.
#include "sht_internal.h"

namespace shtmi {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<float> {
  typedef f32x4 type;
};
template <>
struct Acc<double> {
  typedef f64x4 type;
};

__device__ inline f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16 x 16 output block held in accumulator element e of a lane.
template <typename T>
__device__ inline int acc_row(int lane, int e) {
  return sizeof(T) == 8 ? 4 * e + (lane >> 4) : 4 * (lane >> 4) + e;
}

// ---------------------------------------------------------------------------
// Synthesis: for m and the tile of north-ring rows [t0, t0 + BM) and real
// columns [c0, c0 + BN):
//   S[r][c] = sum_k T0[r][k] a[m + 2k][c],   A[r][c] = sum_k T1[r][k] a[m + 2k + 1][c]
//   c(ring)        = S + A
//   c(mirror ring) = S - A
// Four waves in a 2 x 2 arrangement, each owning a (BM/2) x (BN/2) block of
// both accumulators.  One iteration consumes KCH k of each parity
// (2 KCH consecutive n).
// ---------------------------------------------------------------------------

template <typename T, int BM, int BN>
__global__ __launch_bounds__(256) void legendre_inverse_kernel(DevPlan p, const WorkItem* items,
                                                               const T* __restrict__ spec,
                                                               T* __restrict__ four) {
  typedef typename Acc<T>::type acc_t;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int IM = WM / 16, IN = WN / 16;
  constexpr int KI = KCH;
  __shared__ T As[2][KI][BM];
  __shared__ T Bs[2][KI][BN];

  const WorkItem it = items[blockIdx.x];
  const MInfo mi = p.ms[it.m];
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const T* tab = (const T*)p.tab;
  const int twoF = 2 * p.F;
  const int nk = (mi.Kp[0] > mi.Kp[1] ? mi.Kp[0] : mi.Kp[1]) / KI;

  acc_t acc[2][IM][IN];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < IN; ++j) acc[q][i][j] = acc_t{0, 0, 0, 0};

  for (int kc = 0; kc < nk; ++kc) {
    // table chunk kc of both parities, rows [t0, t0 + BM) -> As[par][kk][r]
    for (int idx = tid; idx < 2 * BM * KI; idx += 256) {
      const int par = idx / (BM * KI);
      const int rem = idx - par * (BM * KI);
      const int r = rem / KI;
      const int kk = rem - r * KI;
      const int row = it.t0 + r;
      const int64_t toff = par ? mi.toff[1] : mi.toff[0];
      const int kp = par ? mi.Kp[1] : mi.Kp[0];
      T v = 0;
      if (row < mi.Lp && kc * KI < kp) v = tab[toff + (int64_t)kc * mi.Lp * KI + (int64_t)row * KI + kk];
      As[par][kk][r] = v;
    }
    // spectral n = m + 2 KI kc + i (i < 2 KI), fields [c0/2, c0/2 + BN/2) -> Bs[i&1][i>>1][c]
    for (int idx = tid; idx < (BN / 2) * 2 * KI; idx += 256) {
      const int fi = idx / (2 * KI);
      const int i = idx - fi * (2 * KI);
      const int f = it.c0 / 2 + fi;
      const int n = m + 2 * KI * kc + i;
      T re = 0, im = 0;
      if (n <= p.N && f < p.F) {
        const int64_t e = ((int64_t)f * p.nspec + mi.spec_off + (n - m)) * 2;
        re = spec[e];
        im = (m == 0) ? (T)0 : spec[e + 1];
      }
      Bs[i & 1][i >> 1][2 * fi] = re;
      Bs[i & 1][i >> 1][2 * fi + 1] = im;
    }
    __syncthreads();
#pragma unroll
    for (int par = 0; par < 2; ++par) {
#pragma unroll
      for (int ks = 0; ks < KI / 4; ++ks) {
        T a[IM], b[IN];
#pragma unroll
        for (int i = 0; i < IM; ++i) a[i] = As[par][ks * 4 + (lane >> 4)][wr * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < IN; ++j) b[j] = Bs[par][ks * 4 + (lane >> 4)][wc * WN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < IN; ++j) acc[par][i][j] = mfma16x16x4(a[i], b[j], acc[par][i][j]);
      }
    }
    __syncthreads();
  }

  const int64_t rowlen = 2 * (int64_t)p.Fp;
#pragma unroll
  for (int i = 0; i < IM; ++i) {
#pragma unroll
    for (int j = 0; j < IN; ++j) {
      const int col = it.c0 + wc * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = it.t0 + wr * WM + i * 16 + acc_row<T>(lane, e);
        if (row < mi.L && col < twoF) {
          const RingInfo rn = p.rings[mi.first_ring + row];
          const RingInfo rs = p.rings[rn.mirror];
          const T S = acc[0][i][j][e];
          const T A = acc[1][i][j][e];
          four[(rn.frow + m) * rowlen + col] = S + A;
          four[(rs.frow + m) * rowlen + col] = S - A;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Analysis: for m, output k tile [t0, t0 + BK) and real columns [c0, c0 + BC):
//   a[m + 2k + par][c] = sum_r T_par[r][k] X_par[r][c],  X_0 = S, X_1 = A,
// computed transposed (rows c, columns k) so that each lane holds the real
// and imaginary part of one coefficient.  The sum runs over the north rings
// carrying m, KJ rings per iteration.
// ---------------------------------------------------------------------------

template <typename T, int BC, int BK>
__global__ __launch_bounds__(256) void legendre_direct_kernel(DevPlan p, const WorkItem* items,
                                                              const T* __restrict__ four,
                                                              T* __restrict__ spec) {
  typedef typename Acc<T>::type acc_t;
  constexpr int WC = BC / 2, WK = BK / 2;
  constexpr int IC = WC / 16, IK = WK / 16;
  constexpr int KJ = 16;
  __shared__ T Xs[2][KJ][BC];
  __shared__ T Ts[2][KJ][BK];

  const WorkItem it = items[blockIdx.x];
  const MInfo mi = p.ms[it.m];
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const T* tab = (const T*)p.tab;
  const int twoF = 2 * p.F;
  const int64_t rowlen = 2 * (int64_t)p.Fp;

  acc_t acc[2][IC][IK];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < IC; ++i)
#pragma unroll
      for (int j = 0; j < IK; ++j) acc[q][i][j] = acc_t{0, 0, 0, 0};

  for (int r0 = 0; r0 < mi.L; r0 += KJ) {
    for (int idx = tid; idx < 2 * KJ * BC; idx += 256) {
      const int par = idx / (KJ * BC);
      const int rem = idx - par * (KJ * BC);
      const int rr = rem / BC;
      const int cc = rem - rr * BC;
      const int r = r0 + rr;
      const int c = it.c0 + cc;
      T v = 0;
      if (r < mi.L && c < twoF) {
        const RingInfo rg = p.rings[mi.first_ring + r];
        v = four[((rg.frow + m) * 2 + par) * rowlen + c];
      }
      Xs[par][rr][cc] = v;
    }
    for (int idx = tid; idx < 2 * KJ * BK; idx += 256) {
      const int par = idx / (KJ * BK);
      const int rem = idx - par * (KJ * BK);
      const int kb = rem / (KJ * KCH);
      const int rem2 = rem - kb * (KJ * KCH);
      const int rr = rem2 / KCH;
      const int kk = rem2 - rr * KCH;
      const int k = it.t0 + kb * KCH + kk;
      const int64_t toff = par ? mi.toff[1] : mi.toff[0];
      const int kp = par ? mi.Kp[1] : mi.Kp[0];
      T v = 0;
      if (k < kp) v = tab[toff + (int64_t)(k / KCH) * mi.Lp * KCH + (int64_t)(r0 + rr) * KCH + (k % KCH)];
      Ts[par][rr][kb * KCH + kk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int par = 0; par < 2; ++par) {
#pragma unroll
      for (int ks = 0; ks < KJ / 4; ++ks) {
        T a[IC], b[IK];
#pragma unroll
        for (int i = 0; i < IC; ++i) a[i] = Xs[par][ks * 4 + (lane >> 4)][wr * WC + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < IK; ++j) b[j] = Ts[par][ks * 4 + (lane >> 4)][wc * WK + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < IC; ++i)
#pragma unroll
          for (int j = 0; j < IK; ++j) acc[par][i][j] = mfma16x16x4(a[i], b[j], acc[par][i][j]);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int par = 0; par < 2; ++par) {
#pragma unroll
    for (int i = 0; i < IC; ++i) {
#pragma unroll
      for (int j = 0; j < IK; ++j) {
        const int k = it.t0 + wc * WK + j * 16 + (lane & 15);
        if (k >= mi.K[par]) continue;
        const int n = m + 2 * k + par;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = it.c0 + wr * WC + i * 16 + acc_row<T>(lane, e);
          if (c < twoF) {
            const int f = c >> 1;
            T v = acc[par][i][j][e];
            if (m == 0 && (c & 1)) v = 0;
            spec[((int64_t)f * p.nspec + mi.spec_off + (n - m)) * 2 + (c & 1)] = v;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Tile shapes and launchers
// ---------------------------------------------------------------------------

constexpr int INV64_BM = 64, INV64_BN = 64, DIR64_BC = 64, DIR64_BK = 64;
constexpr int INV32_BM = 128, INV32_BN = 128, DIR32_BC = 128, DIR32_BK = 64;

void legendre_tiles(int prec, int* inv_rows, int* inv_cols, int* dir_rows, int* dir_cols) {
  if (prec == SHT_FP64) {
    *inv_rows = INV64_BM;
    *inv_cols = INV64_BN;
    *dir_rows = DIR64_BK;
    *dir_cols = DIR64_BC;
  } else {
    *inv_rows = INV32_BM;
    *inv_cols = INV32_BN;
    *dir_rows = DIR32_BK;
    *dir_cols = DIR32_BC;
  }
}

hipError_t launch_legendre_inverse(const DevPlan& p, int prec, const WorkItem* items, int nitems,
                                   const void* spec, void* four, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (prec == SHT_FP64)
    hipLaunchKernelGGL((legendre_inverse_kernel<double, INV64_BM, INV64_BN>), dim3(nitems), dim3(256), 0, s, p,
                       items, (const double*)spec, (double*)four);
  else if (prec == SHT_FP32)
    hipLaunchKernelGGL((legendre_inverse_kernel<float, INV32_BM, INV32_BN>), dim3(nitems), dim3(256), 0, s, p,
                       items, (const float*)spec, (float*)four);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
}

hipError_t launch_legendre_direct(const DevPlan& p, int prec, const WorkItem* items, int nitems,
                                  const void* four, void* spec, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (prec == SHT_FP64)
    hipLaunchKernelGGL((legendre_direct_kernel<double, DIR64_BC, DIR64_BK>), dim3(nitems), dim3(256), 0, s, p,
                       items, (const double*)four, (double*)spec);
  else if (prec == SHT_FP32)
    hipLaunchKernelGGL((legendre_direct_kernel<float, DIR32_BC, DIR32_BK>), dim3(nitems), dim3(256), 0, s, p,
                       items, (const float*)four, (float*)spec);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
}

}  // namespace shtmi
