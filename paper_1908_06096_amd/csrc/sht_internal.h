// Internal plan layout shared by the host runtime and the HIP kernels.
//
// Nothing here is part of the public ABI (include/sht.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/sht.h"

namespace shtmi {

// ---------------------------------------------------------------------------
// Constants of the layouts
// ---------------------------------------------------------------------------

// Legendre tables are stored per (m, parity) as chunks of KCH consecutive
// k (n = m + parity + 2k); each chunk is [rows][KCH], rows padded with zeros
// to ROWPAD, a multiple of every product's ring step (the BF16 analysis
// reads rings 32 at a time, unguarded).
constexpr int KCH = 8;
constexpr int ROWPAD = 32;
// Field stride of the Fourier workspace (complex elements) is F rounded up.
constexpr int FPAD = 16;

// FFT: threads per work group and complex values each thread may hold in
// registers during one pass (or one butterfly of a prime radix above it);
// together they bound the transform length.
// Transforms run in work groups of FFT_THREADS_SMALL threads (even tiers)
// where that many threads per field cover every pass with the fewest
// passes, else of FFT_THREADS (odd tiers): smaller groups wait at smaller
// barriers and more of them share a CU.  Tiers 2 and 3 are the kernels that
// also hold the passes of the prime radices above FFT_BIG_PRIME, for the
// classes that need them (those butterflies take every register a pass has,
// and in the other kernels they would make the code around the passes
// spill).  A work group transforms up to G fields of one ring side by side;
// work is listed in chunks of FFT_FCHUNK fields.
constexpr int FFT_THREADS = 512;
constexpr int FFT_THREADS_SMALL = 256;
constexpr int FFT_TIERS = 4;
constexpr int FFT_BIG_PRIME = 23;
// The largest prime radix in FP32.  41, 43 and 47 were radices too, but their
// passes saved and reloaded ~48 callee-saved registers per call and spilled
// (their rings moved ~4.7x their algorithmic bytes); as chirp-z classes the
// stages measured the same or faster.
constexpr int FFT_MAX_PRIME = 37;
__host__ __device__ constexpr int fft_tier_threads(int tier) { return (tier & 1) ? FFT_THREADS : FFT_THREADS_SMALL; }
constexpr int FFT_REGS = 20;
constexpr int FFT_MAX_RADICES = 20;
constexpr int FFT_FCHUNK = 16;
constexpr int FFT_MAX_G = 8;

// Device-memory accesses through address-space-1 pointers.  Pointers read
// out of plan structures are generic, and generic (FLAT) accesses count
// against the LDS wait counter as well as the memory one, so every wait for
// an LDS read would also wait for loads still in flight; these helpers make
// the compiler emit global_load / global_store instead.
// HIP's float2 / double2 are classes whose copy constructor takes a generic
// reference, which would drop the address space again, so 8- and 16-byte
// values move as native clang vectors of 32-bit words.
#define SHT_GLOBAL __attribute__((address_space(1)))
typedef uint32_t gword2 __attribute__((ext_vector_type(2)));
typedef uint32_t gword4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  if constexpr (sizeof(T) == 8 && alignof(T) >= 8) {
    const gword2 w = *(const SHT_GLOBAL gword2*)p;
    return __builtin_bit_cast(T, w);
  } else if constexpr (sizeof(T) == 16 && alignof(T) >= 16) {
    const gword4 w = *(const SHT_GLOBAL gword4*)p;
    return __builtin_bit_cast(T, w);
  } else if constexpr (!__is_arithmetic(T) && sizeof(T) % 4 == 0) {
    // metadata structures: word by word (uniform addresses become scalar loads)
    struct Words {
      uint32_t w[sizeof(T) / 4];
    } u;
    const SHT_GLOBAL uint32_t* q = (const SHT_GLOBAL uint32_t*)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = q[i];
    return __builtin_bit_cast(T, u);
  } else {
    return *(const SHT_GLOBAL T*)p;
  }
}
// The same for LDS (address space 3), for pointers the compiler cannot
// trace to a __shared__ object (arguments of non-inlined functions), which
// would otherwise become FLAT accesses.
#define SHT_LDS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ T lload(const T* p) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte values");
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, *(const SHT_LDS gword2*)p);
  } else {
    return __builtin_bit_cast(T, *(const SHT_LDS gword4*)p);
  }
}
template <typename T>
__device__ __forceinline__ void lstore(T* p, const T& v) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte values");
  if constexpr (sizeof(T) == 8) {
    *(SHT_LDS gword2*)p = __builtin_bit_cast(gword2, v);
  } else {
    *(SHT_LDS gword4*)p = __builtin_bit_cast(gword4, v);
  }
}

template <typename T>
__device__ __forceinline__ void gstore(T* p, const T& v) {
  if constexpr (sizeof(T) == 8 && alignof(T) >= 8) {
    *(SHT_GLOBAL gword2*)p = __builtin_bit_cast(gword2, v);
  } else if constexpr (sizeof(T) == 16 && alignof(T) >= 16) {
    *(SHT_GLOBAL gword4*)p = __builtin_bit_cast(gword4, v);
  } else {
    *(SHT_GLOBAL T*)p = v;
  }
}

// A store marked non-temporal (streaming): for outputs written once and not
// read again by the kernel, so that they leave the L2 before the inputs
// still being read.  Only where each store instruction covers whole
// 128-byte lines: partial lines written this way lose the L2's merging
// (measured up to 3x slower).
template <typename T>
__device__ __forceinline__ void gstore_nt(T* p, const T& v) {
  static_assert(__is_arithmetic(T) || sizeof(T) == 8 || sizeof(T) == 16, "scalars, 8- or 16-byte values");
  if constexpr (__is_arithmetic(T))
    __builtin_nontemporal_store(v, (SHT_GLOBAL T*)p);
  else if constexpr (sizeof(T) == 8)
    __builtin_nontemporal_store(__builtin_bit_cast(gword2, v), (SHT_GLOBAL gword2*)p);
  else
    __builtin_nontemporal_store(__builtin_bit_cast(gword4, v), (SHT_GLOBAL gword4*)p);
}

// ---------------------------------------------------------------------------
// Device metadata
// ---------------------------------------------------------------------------

struct RingInfo {
  int32_t nlon;   // points on the ring
  int32_t mmax;   // highest wavenumber carried
  int32_t cls;    // FFT class (index into FftClass)
  int32_t mirror; // index of the mirror ring
  int64_t goff;   // grid offset of the ring (elements)
  int64_t frow;   // first Fourier workspace row of the ring
};

// One FFT class per distinct half length h = nlon / 2.  The real DFT of
// length 2h is carried out as a complex DFT of length h; when h has a prime
// factor above the largest prime radix (37 in FP32, 23 in FP64) that DFT is
// a chirp-z convolution of length L (5-smooth, L >= 2h - 1), otherwise
// L = h.
struct FftClass {
  int32_t h;
  int32_t L;
  int32_t bluestein;
  int32_t nrad;
  int32_t rad[FFT_MAX_RADICES];
  int32_t G;          // fields transformed side by side per work group (power of two)
  int32_t gshift;     // log2 G; each field gets fft_tier_threads(tier) / G threads
  int32_t tier;       // launch: work-group size fft_tier_threads(tier), prime radices above
                      // FFT_BIG_PRIME when tier >= 2
  int64_t root_off;   // L - 1 twiddles, pass after pass: exp(-2 pi i r k / (Ns R)) at
                      // k (R - 1) + r - 1 of the pass table (k < Ns, 1 <= r < R)
  int64_t post_off;   // h complex values exp(-2 pi i q / (2h))
  int64_t chirp_off;  // h complex values exp(-i pi t^2 / h)      (bluestein)
  int64_t khat_off;   // L complex: DFT_L of the conjugate chirp / L (bluestein)
  uint64_t radpack;   // rad[0..nrad) at 6 bits each (radix q in bits 6q..6q+5), so that
                      // the passes take their radix from a register, not a memory load
};
constexpr int FFT_PACK_RADICES = 10;  // radices radpack holds
__host__ __device__ constexpr int packed_radix(uint64_t pack, int q) { return (int)((pack >> (6 * q)) & 63u); }

struct MInfo {
  int32_t m;
  int32_t first_ring; // first north ring with mmax >= m
  int32_t L;          // north rings carrying m
  int32_t Lp;         // L padded to ROWPAD
  int32_t K[2];       // number of n of each parity (n - m even / odd)
  int32_t Kp[2];      // padded to KCH
  int64_t toff[2];    // element offset of each parity table
  int64_t spec_off;   // index(m, m) in the spectral layout
  int64_t coff;       // first (a_n, e_n) of m in the recurrence coefficients
};

// A Legendre work item: wavenumber, tile along the table rows or columns,
// tile along the field columns, and the plan (index into the launch's plan
// array) it belongs to; m < 0 marks an empty slot of the work list.
struct WorkItem {
  int32_t m;
  int32_t t0;  // first row (synthesis: ring row; analysis: k index)
  int32_t c0;  // first real column (2 f + re/im)
  int32_t plan;
};

// An FFT work item: a ring (a north ring for analysis) and the fields
// [f0, fend) transformed side by side (at most the class's G); ring < 0
// marks an empty slot of the work list.
struct FftItem {
  int32_t ring;
  int32_t f0;
  int32_t plan;
  int32_t fend;
  int32_t cls;  // the ring's FFT class (read with the ring, not after it)
};

// Device buffers of one transform: spectral [F][nspec] complex, grid
// [F][npts] real, Fourier workspace.
struct IoBind {
  void* spec;
  void* grid;
  void* ws;
  void* pad;  // Legendre tables to use instead of the plan's (table-free plans), or null
  // pointwise steps fused into the stores of a time step (0: none):
  double grid_a;  // synthesis grid values g <- g + a g (1 - g)
  double spec_c;  // analysis coefficients a_n^m <- a_n^m / (1 + c n (n + 1))
};

// The two pointwise steps of the reaction-diffusion time step, with one
// rounding order wherever they are applied.
template <typename T>
__device__ __forceinline__ T logistic_step(T g, T a) {
  return __builtin_fma(a * g, T(1) - g, g);
}
template <typename T>
__device__ __forceinline__ T diffusion_factor(int n, double c) {
  return (T)(1.0 / (1.0 + c * (double)n * (double)(n + 1)));
}

// Column-tile variants of the Legendre products (2F real columns per m):
// 128, 64 or 32 columns per tile.  Narrow tiles keep small field counts
// from wasting most of each MFMA.
enum TileVariant { TILE_C128 = 0, TILE_C64 = 1, TILE_C32 = 2, NUM_TILE_VARIANTS = 3 };

// Device-side view of a plan passed to kernels by value.
struct DevPlan {
  int32_t N, nlat, nh, F, Fp;
  int64_t npts, nspec;
  const RingInfo* rings;
  const FftClass* classes;
  const MInfo* ms;
  const double* mu;
  const double* w;
  const double* wa;     // analysis weight per ring: w (scalar plans), w / (1 - mu^2) (vector plans)
  const void* tab;      // Pbar tables (double, float, or bf16 hi/lo pairs)
  const void* fft;      // complex FFT tables in the data type
  int64_t tab_plane;    // element offset of the lo plane of a BF16 split table
};

// Records a failed HIP call as the calling thread's last HIP error (see
// sht_last_hip_error) and returns SHT_EHIP (capi.hip).
int hip_status(hipError_t e);

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// tables.hip
hipError_t launch_gauss(int nlat, double* mu, double* w, hipStream_t s);
// Pbar tables (and, when d_hms is not null, the H = (1 - mu^2) dPbar/dmu
// tables of degree <= Nh in the layout d_hms describes).
hipError_t launch_pbar_planes(const DevPlan& p, int prec, const MInfo* d_ms, int nm, int max_Lp,
                              void* tab, int64_t plane_elems, const MInfo* d_hms, void* htab, int64_t hplane_elems,
                              int Nh, const double* sect, const double2* coef, hipStream_t s);
// The recurrence's coefficients: sect[k] (k = 0..D) and, per m, coef[coff(m)
// + n - m] = (a_n, e_n) for n = m..D.
hipError_t launch_pbar_coef(int D, const MInfo* d_ms, int nm, double* sect, double2* coef, hipStream_t s);
// Recurrence coefficients per m for table degree D: n - m = 0 .. 16 b, with
// b the number of 16-degree blocks covering n = m..D.
__host__ __device__ inline int pbar_coef_count(int D, int m) { return 16 * ((D - m + 16) / 16) + 1; }
hipError_t launch_fft_tables(const DevPlan& p, int prec, const FftClass* d_cls, int ncls,
                             const FftClass* h_cls, void* fft, hipStream_t s);
hipError_t launch_table_export_planes(const DevPlan& p, int prec, const MInfo& mi, int64_t plane,
                                      double* out, hipStream_t s);

// legendre.hip.  One launch covers `nitems` items of the plans in `plans`;
// `grid_blocks` work groups loop over the items (grid stride).  Buffers come
// from io[item.plan] when io is not null, else from io0.
hipError_t launch_legendre_inverse(const DevPlan* plans, int prec, int variant, const WorkItem* items, int nitems,
                                   const IoBind* io, IoBind io0, int grid_blocks, hipStream_t s);
hipError_t launch_legendre_direct(const DevPlan* plans, int prec, int variant, const WorkItem* items, int nitems,
                                  const IoBind* io, IoBind io0, int grid_blocks, hipStream_t s);
// tile shape of a variant: rows (synthesis) / k (analysis) and columns
void legendre_tiles(int prec, int variant, int* inv_rows, int* inv_cols, int* dir_rows, int* dir_cols);
bool legendre_variant_supported(int prec, int variant);
// work groups per CU the kernel of a variant can keep resident
int legendre_blocks_per_cu(int prec, int variant, bool inverse);

// vector.hip: spectral-space kernels of the derivative and vector
// transforms (degree N inputs and outputs, degree N + 1 wind coefficients).
hipError_t launch_uv_from_potentials(int N, int F, bool gradient, int prec, const void* in, void* uv, hipStream_t s);
hipError_t launch_vortdiv_from_projections(int N, int F, int prec, const void* pw, const void* hw, void* out,
                                           hipStream_t s);
hipError_t launch_spectral_op(int N, int count, int op, int prec, const void* in, void* out, hipStream_t s);
hipError_t launch_analysis_weight(int nlat, const double* mu, const double* w, double* wa, hipStream_t s);

// stepper.hip: the grid-point and spectral operations of the time step.

// fft.hip.  Same launch model, one launch per tier: the items of one launch
// all belong to classes of that tier.
hipError_t launch_fourier_synthesis(const DevPlan* plans, int prec, int tier, const FftItem* items, int nitems,
                                    const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s);
hipError_t launch_fourier_analysis(const DevPlan* plans, int prec, int tier, const FftItem* items, int nitems,
                                   const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s);
hipError_t fft_set_max_lds(size_t bytes);
// LDS of a work group of G transforms of length L
size_t fft_lds_bytes(int prec, int L, int G);
size_t fft_grid_blocks(int nitems);
int fft_blocks_per_cu(int prec, int tier, size_t lds);

}  // namespace shtmi
