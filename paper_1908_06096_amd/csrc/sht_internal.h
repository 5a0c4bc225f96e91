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
// k (n = m + parity + 2k); each chunk is [rows][KCH], rows padded to ROWPAD.
constexpr int KCH = 8;
constexpr int ROWPAD = 16;
// Field stride of the Fourier workspace (complex elements) is F rounded up.
constexpr int FPAD = 16;

// FFT: threads per work group and complex values each thread may hold in
// registers during one pass; together they bound the transform length.
constexpr int FFT_THREADS = 256;
constexpr int FFT_REGS = 32;
constexpr int FFT_MAX_RADICES = 20;

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
// factor above 5 that DFT is a chirp-z convolution of length L (5-smooth,
// L >= 2h - 1), otherwise L = h.
struct FftClass {
  int32_t h;
  int32_t L;
  int32_t bluestein;
  int32_t nrad;
  int32_t rad[FFT_MAX_RADICES];
  int64_t root_off;   // L - 1 twiddles, pass after pass: exp(-2 pi i r k / (Ns R)) at
                      // k (R - 1) + r - 1 of the pass table (k < Ns, 1 <= r < R)
  int64_t post_off;   // h complex values exp(-2 pi i q / (2h))
  int64_t chirp_off;  // h complex values exp(-i pi t^2 / h)      (bluestein)
  int64_t khat_off;   // L complex: DFT_L of the conjugate chirp / L (bluestein)
};

struct MInfo {
  int32_t m;
  int32_t first_ring; // first north ring with mmax >= m
  int32_t L;          // north rings carrying m
  int32_t Lp;         // L padded to ROWPAD
  int32_t K[2];       // number of n of each parity (n - m even / odd)
  int32_t Kp[2];      // padded to KCH
  int64_t toff[2];    // element offset of each parity table
  int64_t spec_off;   // index(m, m) in the spectral layout
};

// A Legendre work item: wavenumber, tile along the table rows or columns,
// tile along the field columns.
struct WorkItem {
  int32_t m;
  int32_t t0;  // first row (synthesis: ring row; analysis: k index)
  int32_t c0;  // first real column (2 f + re/im)
  int32_t pad;
};

// Device-side view of a plan passed to kernels by value.
struct DevPlan {
  int32_t N, nlat, nh, F, Fp;
  int64_t npts, nspec;
  const RingInfo* rings;
  const FftClass* classes;
  const MInfo* ms;
  const double* mu;
  const double* w;
  const void* tab;      // Pbar tables (double, float, or bf16 hi/lo pairs)
  const void* fft;      // complex FFT tables in the data type
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// tables.hip
hipError_t launch_gauss(int nlat, double* mu, double* w, hipStream_t s);
hipError_t launch_pbar_planes(const DevPlan& p, int prec, const MInfo* d_ms, int nm, int max_Lp,
                              void* tab, int64_t plane_elems, hipStream_t s);
hipError_t launch_fft_tables(const DevPlan& p, int prec, const FftClass* d_cls, int ncls,
                             const FftClass* h_cls, void* fft, hipStream_t s);
hipError_t launch_table_export_planes(const DevPlan& p, int prec, const MInfo& mi, int64_t plane,
                                      double* out, hipStream_t s);

// legendre.hip
// plane: element offset of the lo plane of a BF16 split table (unused otherwise)
hipError_t launch_legendre_inverse(const DevPlan& p, int prec, const WorkItem* items, int nitems, int64_t plane,
                                   const void* spec, void* four, hipStream_t s);
hipError_t launch_legendre_direct(const DevPlan& p, int prec, const WorkItem* items, int nitems, int64_t plane,
                                  const void* four, void* spec, hipStream_t s);
// tile shapes the work lists are built for
void legendre_tiles(int prec, int* inv_rows, int* inv_cols, int* dir_rows, int* dir_cols);

// fft.hip
hipError_t launch_fourier_synthesis(const DevPlan& p, int prec, const int2* items, int nitems, size_t lds,
                                    const void* four, void* grid, hipStream_t s);
hipError_t launch_fourier_analysis(const DevPlan& p, int prec, const int2* items, int nitems, size_t lds,
                                   const void* grid, void* four, hipStream_t s);
hipError_t fft_set_max_lds(size_t bytes);
size_t fft_lds_bytes(int prec, int L, int mmax);

}  // namespace shtmi
