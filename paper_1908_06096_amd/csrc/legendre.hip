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

// Raw buffer descriptor over `bytes` bytes from `base` (no stride; loads
// past the range return zero), and 8- / 16-byte loads through one with a
// lane offset and a uniform offset (bytes).  The range field is 32 bits:
// longer arrays get the largest range, which is exact wherever a read can
// pass the end (offsets are kept within 4 GB of the base by the callers).
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint64_t bytes) {
  const uint32_t n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, 0x00020000);
}
// The same over a base and range that are the same on every lane, read
// from the first lane so that the descriptor provably sits in scalar
// registers (instructions that need it there otherwise loop over lanes).
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc_uniform(const void* base, uint64_t bytes) {
  const uint64_t a = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const uint32_t n = __builtin_amdgcn_readfirstlane(bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes);
  return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0, (int)n, 0x00020000);
}
template <typename V>
__device__ __forceinline__ V rsrc_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(V) == 8 || sizeof(V) == 16, "8- or 16-byte values");
  if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

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

// 16-byte vectors and complex pairs of the element type.
template <typename T>
struct Vec;
template <>
struct Vec<float> {
  typedef float4 type;
  typedef float2 pair;
  static constexpr int n = 4;
};
template <>
struct Vec<double> {
  typedef double2 type;
  typedef double2 pair;
  static constexpr int n = 2;
};

// LDS rows are padded by 16 elements: consecutive rows then start 16 banks
// apart, so the 64 lanes of an MFMA operand read (4 rows x 16 columns) hit
// distinct banks.
constexpr int LDS_PAD = 16;

// ---------------------------------------------------------------------------
// Synthesis: for m and the tile of north-ring rows [t0, t0 + BM) and real
// columns [c0, c0 + BN):
//   S[r][c] = sum_k T0[r][k] a[m + 2k][c],   A[r][c] = sum_k T1[r][k] a[m + 2k + 1][c]
//   c(ring)        = S + A
//   c(mirror ring) = S - A
// Four waves in a 2 x 2 arrangement, each owning a (BM/2) x (BN/2) block of
// both accumulators.  One iteration consumes KI k of each parity (2 KI
// consecutive n); the next iteration's operands are fetched into registers
// while the current one is multiplied out of LDS.
// ---------------------------------------------------------------------------

template <typename T, int BM, int BN, int KI, int WCOL>
__device__ __forceinline__ void inverse_tile(const DevPlan& p, const WorkItem it, const T* __restrict__ spec,
                                             T* __restrict__ four) {
  typedef typename Acc<T>::type acc_t;
  typedef typename Vec<T>::type V;
  typedef typename Vec<T>::pair C2;
  constexpr int VN = Vec<T>::n;
  constexpr int WROW = 4 / WCOL;           // waves along rows x along columns
  constexpr int WM = BM / WROW, WN = BN / WCOL;
  constexpr int IM = WM / 16, IN = WN / 16;
  constexpr int NC = KI / KCH;             // table chunks per parity per iteration
  constexpr int AUNITS = 2 * NC * BM;      // (parity, chunk, row) units of KCH elements
  constexpr int AU = AUNITS / 256;
  constexpr int FT = BN / 2;               // fields per tile
  constexpr int TPF = 256 / FT;            // threads per field
  constexpr int NB = 2 * KI / TPF;         // complex values per thread per iteration
  static_assert(AUNITS % 256 == 0 && 256 % FT == 0 && (2 * KI) % TPF == 0 && TPF % 2 == 0, "tile shape");
  __shared__ T As[2][KI][BM + LDS_PAD];
  __shared__ T Bs[2][KI][BN + LDS_PAD];
  // FP32: spectral row k of parity p has its column index XORed with
  // 4 (2 p + (k / 2) mod 2).  The parities' planes and every other row share
  // banks, so the staging writes (lanes of two fields over 8 (parity, k)
  // pairs) would meet on 4 bank groups; permuted they use all 16.  FP64:
  // rows are 640 bytes apart, so the 16-byte stores of one field's 8 lanes
  // (4 k x 2 parities, 16 bytes each) all met on one bank group; the column
  // is XORed with 2 (2 (k mod 4) + p), which gives the 8 lanes 8 different
  // 16-byte slots of 128 bytes.  Both permutations stay within 16-column
  // blocks and are the same for a lane across the step's operand reads
  // (k = 4 ks + lane / 16), which stay conflict-free.
  auto bcol = [](int par, int k, int col) {
    return sizeof(T) == 4 ? col ^ (4 * (2 * par + ((k >> 1) & 1))) : col ^ (2 * (2 * (k & 3) + par));
  };

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WCOL, wc = wave % WCOL;
  const T* tab = (const T*)p.tab;
  const int twoF = 2 * p.F;
  const int kpmax = mi.Kp[0] > mi.Kp[1] ? mi.Kp[0] : mi.Kp[1];
  const int nk = (kpmax + KI - 1) / KI;

  // Table and spectral loads go through buffer descriptors: reads past a
  // parity table's padded k range return zero, so spectral values read past
  // n = N (another wavenumber's, finite) meet zero table entries; rows past
  // the table and fields past F only feed outputs that are never stored.
  // Unit a = tid + 256 a: parity and chunk are the same across a wave (its
  // descriptor is uniform), the row is the lane's.
  uint32_t a_off[AU];
  int a_par[AU], a_ch[AU], a_row[AU];
#pragma unroll
  for (int a = 0; a < AU; ++a) {
    const int u = tid + 256 * a;
    a_par[a] = __builtin_amdgcn_readfirstlane(u / (NC * BM));
    a_ch[a] = __builtin_amdgcn_readfirstlane((u / BM) % NC);
    a_row[a] = u % BM;
    a_off[a] = ((uint32_t)a_ch[a] * mi.Lp + (uint32_t)(it.t0 + a_row[a])) * (KCH * (uint32_t)sizeof(T));
  }
  const __amdgpu_buffer_rsrc_t t_rs0 = buffer_rsrc(tab + mi.toff[0], (uint32_t)mi.Kp[0] * mi.Lp * (uint32_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t t_rs1 = buffer_rsrc(tab + mi.toff[1], (uint32_t)mi.Kp[1] * mi.Lp * (uint32_t)sizeof(T));
  const uint32_t a_step = (uint32_t)NC * mi.Lp * KCH * (uint32_t)sizeof(T);  // bytes per iteration
  // spectral values owned by this thread: field fi, n offsets q + TPF j;
  // the descriptor starts at the tile's first field
  const int fi = tid / TPF;
  const int q = tid % TPF;
  const int f0 = it.c0 / 2;
  const int f = f0 + fi;
  const uint32_t fl = (uint32_t)((f < p.F ? f : p.F - 1) - f0);
  const int64_t sbase = (int64_t)f0 * p.nspec + mi.spec_off;
  const __amdgpu_buffer_rsrc_t b_rs =
      buffer_rsrc((const C2*)spec + sbase, (uint64_t)((int64_t)p.F * p.nspec - sbase) * sizeof(C2));
  const uint32_t b_off = (fl * (uint32_t)p.nspec + (uint32_t)q) * (uint32_t)sizeof(C2);
  const bool m0 = m == 0;
  const int b_par = q & 1;

  V ra[AU][KCH / VN];
  C2 rb[NB];
  auto fetch = [&](int kc) {
    const uint32_t sa = (uint32_t)kc * a_step;
#pragma unroll
    for (int a = 0; a < AU; ++a) {
#pragma unroll
      for (int v = 0; v < KCH / VN; ++v) ra[a][v] = rsrc_load<V>(a_par[a] ? t_rs1 : t_rs0, a_off[a] + v * sizeof(V), sa);
    }
    // raw loads only: anything computed from them here would wait for them
    const uint32_t sb = (uint32_t)kc * (2 * KI) * (uint32_t)sizeof(C2);
#pragma unroll
    for (int j = 0; j < NB; ++j) rb[j] = rsrc_load<C2>(b_rs, b_off + TPF * j * (uint32_t)sizeof(C2), sb);
  };

  acc_t acc[2][IM][IN];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < IN; ++j) acc[par][i][j] = acc_t{0, 0, 0, 0};

  fetch(0);
  for (int kc = 0; kc < nk; ++kc) {
#pragma unroll
    for (int a = 0; a < AU; ++a) {
      const T* e = (const T*)ra[a];
#pragma unroll
      for (int kk = 0; kk < KCH; ++kk) As[a_par[a]][a_ch[a] * KCH + kk][a_row[a]] = e[kk];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = (q >> 1) + (TPF / 2) * j;
      const int bc = bcol(b_par, k, 2 * fi);
      *(C2*)&Bs[b_par][k][bc] = rb[j];
      // Im a_n^0 is dropped: a constant store, so that nothing is computed
      // from the prefetched registers before this step (the compiler would
      // compute it right after the loads and wait for them there)
      if (m0) Bs[b_par][k][bc + 1] = 0;
    }
    __syncthreads();
    if (kc + 1 < nk) fetch(kc + 1);
#pragma unroll
    for (int par = 0; par < 2; ++par) {
#pragma unroll
      for (int ks = 0; ks < KI / 4; ++ks) {
        T av[IM], bv[IN];
#pragma unroll
        for (int i = 0; i < IM; ++i) av[i] = As[par][ks * 4 + (lane >> 4)][wr * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < IN; ++j) {
          const int k = ks * 4 + (lane >> 4);
          bv[j] = Bs[par][k][bcol(par, k, wc * WN + j * 16 + (lane & 15))];
        }
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < IN; ++j) acc[par][i][j] = mfma16x16x4(av[i], bv[j], acc[par][i][j]);
      }
    }
    __syncthreads();
  }

  const int64_t rowlen = 2 * (int64_t)p.Fp;
#pragma unroll
  for (int i = 0; i < IM; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = it.t0 + wr * WM + i * 16 + acc_row<T>(lane, e);
      if (row >= mi.L) continue;
      const RingInfo rn = gload(p.rings + mi.first_ring + row);
      T* dn = four + (rn.frow + m) * rowlen;
      T* ds = four + (gload(p.rings + rn.mirror).frow + m) * rowlen;
#pragma unroll
      for (int j = 0; j < IN; ++j) {
        const int col = it.c0 + wc * WN + j * 16 + (lane & 15);
        if (col < twoF) {
          const T S = acc[0][i][j][e];
          const T A = acc[1][i][j][e];
          if constexpr (sizeof(T) == 8) {
            // 16 lanes write 128 contiguous bytes of a row (whole lines when
            // the workspace is 128-byte aligned): streaming stores (26.6 ->
            // 26.3 ms at TCo1279; the FP32 half lines measured slower)
            gstore_nt(dn + col, S + A);
            gstore_nt(ds + col, S - A);
          } else {
            gstore(dn + col, S + A);
            gstore(ds + col, S - A);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Analysis: for m, output k tile [t0, t0 + BK) and real columns [c0, c0 + BC):
//   a[m + 2k + par][c] = sum_r T_par[r][k] X_par[r][c],  X_0 = S, X_1 = A,
// where S = N + S' and A = N - S' are formed as the operand is staged from
// the two Fourier rows of north ring r: N (the ring's w chat) and S' (its
// mirror's),
// computed transposed (rows c, columns k) so that, in f32, each lane holds
// the real and imaginary part of one coefficient.  The sum runs over the
// north rings carrying m, KJ rings per iteration, with the next rings'
// operands fetched into registers during the multiply.
// ---------------------------------------------------------------------------

template <typename T, int BC, int BK, int KJ, int WKW>
__device__ __forceinline__ void direct_tile(const DevPlan& p, const WorkItem it, const T* __restrict__ four,
                                            T* __restrict__ spec, double sc) {
  typedef typename Acc<T>::type acc_t;
  typedef typename Vec<T>::type V;
  typedef typename Vec<T>::pair C2;
  constexpr int VN = Vec<T>::n;
  constexpr int WCW = 4 / WKW;             // waves along columns c x along k
  constexpr int WC = BC / WCW, WK = BK / WKW;
  constexpr int IC = WC / 16, IK = WK / 16;
  constexpr int CS = BC / VN;                 // vectors per X row segment
  constexpr int XUNITS = KJ * CS;             // (ring row, vector): both Fourier rows each
  constexpr int XU = (XUNITS + 255) / 256;
  constexpr int NCH = BK / KCH;               // table chunks per parity
  constexpr int TUNITS = 2 * NCH * KJ;        // (parity, chunk, ring) units of KCH elements
  constexpr int TU = TUNITS / 256;
  static_assert((XUNITS % 256 == 0 || XUNITS < 256) && TUNITS % 256 == 0 && KJ % 4 == 0, "tile shape");
  __shared__ T Xs[2][KJ][BC + LDS_PAD];
  __shared__ T Ts[2][KJ][BK + LDS_PAD];
  // FP32: in the table rows of rings 2 and 3 mod 4 the 16-byte column units
  // swap in pairs (unit ^ 1).  Rows are 16 banks apart, so without it the
  // staging writes (lanes of consecutive rings, one unit each) of rings r
  // and r + 2 meet on the same banks; with it four consecutive rings use
  // four bank groups.  The operand reads (rings 4s + lane / 16) take a
  // permutation that is the same for a lane across the whole step and stays
  // within 16-column blocks, so they remain conflict-free.
  // FP64: rows are 640 bytes apart, so the 16-byte stores of 8 consecutive
  // rings all met on one bank group; the 16-byte unit is XORed with the ring
  // mod 8, which spreads them over 8 slots (the operand reads then take one
  // of two permutations per lane, by ks mod 2).
  auto tcol = [](int ring, int col) {
    return sizeof(T) == 4 ? col ^ (VN * ((ring >> 1) & 1)) : col ^ (VN * (ring & 7));
  };

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WKW, wc = wave % WKW;
  const T* tab = (const T*)p.tab;
  const int twoF = 2 * p.F;
  const int64_t rowlen = 2 * (int64_t)p.Fp;
  const int nj = (mi.L + KJ - 1) / KJ;

  // X unit: (ring row, column vector), loading the N and S' rows.  Rings
  // past L read ring L - 1 (their table rows are the zero padding: steps of
  // KJ rings never pass L rounded up to ROWPAD), columns past the row
  // (outputs never stored) are clamped into it, and the Fourier row offsets
  // of the next step's rings are looked up one step ahead.  With fewer
  // units than threads the upper threads load nothing.
  int x_rr[XU], x_c[XU], x_cg[XU];
  bool x_on[XU];
#pragma unroll
  for (int a = 0; a < XU; ++a) {
    const int u = tid + 256 * a;
    x_on[a] = u < XUNITS;
    x_c[a] = (u % CS) * VN;
    x_cg[a] = min(it.c0 + x_c[a], 2 * p.Fp - VN);
    x_rr[a] = (u / CS) % KJ;
  }
  // table unit: (parity, chunk, ring row) through one descriptor per parity
  // (the parity is the same across a wave); chunks past the table read zero
  int t_par[TU], t_ch[TU], t_rr[TU];
  uint32_t t_off[TU];
#pragma unroll
  for (int a = 0; a < TU; ++a) {
    const int u = tid + 256 * a;
    t_par[a] = __builtin_amdgcn_readfirstlane(u / (KJ * NCH));
    t_ch[a] = (u / KJ) % NCH;
    t_rr[a] = u % KJ;
    t_off[a] = ((uint32_t)(it.t0 / KCH + t_ch[a]) * mi.Lp + (uint32_t)t_rr[a]) * (KCH * (uint32_t)sizeof(T));
  }
  const __amdgpu_buffer_rsrc_t t_rs0 = buffer_rsrc(tab + mi.toff[0], (uint32_t)mi.Kp[0] * mi.Lp * (uint32_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t t_rs1 = buffer_rsrc(tab + mi.toff[1], (uint32_t)mi.Kp[1] * mi.Lp * (uint32_t)sizeof(T));

  int64_t fr[XU], fr_next[XU];
  auto fetch_rows = [&](int jc, int64_t* dst) {
#pragma unroll
    for (int a = 0; a < XU; ++a) dst[a] = gload(&p.rings[mi.first_ring + min(jc * KJ + x_rr[a], mi.L - 1)].frow);
  };
  V rx[XU][2];
  V rt[TU][KCH / VN];
  auto fetch = [&](int jc) {
#pragma unroll
    for (int a = 0; a < XU; ++a) {
      if (!x_on[a]) continue;
      const T* row = four + ((fr[a] + m) * 2) * rowlen + x_cg[a];
      rx[a][0] = gload((const V*)row);
      rx[a][1] = gload((const V*)(row + rowlen));
    }
    const uint32_t so = (uint32_t)jc * KJ * KCH * (uint32_t)sizeof(T);
#pragma unroll
    for (int a = 0; a < TU; ++a) {
#pragma unroll
      for (int v = 0; v < KCH / VN; ++v) rt[a][v] = rsrc_load<V>(t_par[a] ? t_rs1 : t_rs0, t_off[a] + v * sizeof(V), so);
    }
  };

  acc_t acc[2][IC][IK];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int i = 0; i < IC; ++i)
#pragma unroll
      for (int j = 0; j < IK; ++j) acc[par][i][j] = acc_t{0, 0, 0, 0};

  fetch_rows(0, fr);
  fetch(0);
  if (nj > 1) fetch_rows(1, fr_next);
  for (int jc = 0; jc < nj; ++jc) {
#pragma unroll
    for (int a = 0; a < XU; ++a) {
      if (!x_on[a]) continue;
      *(V*)&Xs[0][x_rr[a]][x_c[a]] = rx[a][0] + rx[a][1];  // S = N + S'
      *(V*)&Xs[1][x_rr[a]][x_c[a]] = rx[a][0] - rx[a][1];  // A = N - S'
    }
#pragma unroll
    for (int a = 0; a < TU; ++a)
#pragma unroll
      for (int v = 0; v < KCH / VN; ++v)
        *(V*)&Ts[t_par[a]][t_rr[a]][tcol(t_rr[a], t_ch[a] * KCH + v * VN)] = rt[a][v];
    __syncthreads();
    if (jc + 1 < nj) {
#pragma unroll
      for (int a = 0; a < XU; ++a) fr[a] = fr_next[a];
      fetch(jc + 1);
      if (jc + 2 < nj) fetch_rows(jc + 2, fr_next);
    }
#pragma unroll
    for (int par = 0; par < 2; ++par) {
#pragma unroll
      for (int ks = 0; ks < KJ / 4; ++ks) {
        T av[IC], bv[IK];
#pragma unroll
        for (int i = 0; i < IC; ++i) av[i] = Xs[par][ks * 4 + (lane >> 4)][wr * WC + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < IK; ++j) {
          const int ring = ks * 4 + (lane >> 4);
          bv[j] = Ts[par][ring][tcol(ring, wc * WK + j * 16 + (lane & 15))];
        }
#pragma unroll
        for (int i = 0; i < IC; ++i)
#pragma unroll
          for (int j = 0; j < IK; ++j) acc[par][i][j] = mfma16x16x4(av[i], bv[j], acc[par][i][j]);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int par = 0; par < 2; ++par) {
    const int K = par ? mi.K[1] : mi.K[0];
#pragma unroll
    for (int j = 0; j < IK; ++j) {
      const int k = it.t0 + wc * WK + j * 16 + (lane & 15);
      if (k >= K) continue;
      C2* dst = (C2*)spec + (mi.spec_off + 2 * k + par);
      // fused implicit diffusion of a time step (sc != 0)
      const T fd = sc != 0.0 ? diffusion_factor<T>(m + 2 * k + par, sc) : T(1);
#pragma unroll
      for (int i = 0; i < IC; ++i) {
        if constexpr (sizeof(T) == 4) {
          // rows 4 (l/16) + e: e = 0, 1 and e = 2, 3 are (re, im) of two fields
#pragma unroll
          for (int e = 0; e < 4; e += 2) {
            const int c = it.c0 + wr * WC + i * 16 + 4 * (lane >> 4) + e;
            if (c < twoF) {
              C2 v = C2{acc[par][i][j][e], acc[par][i][j][e + 1]};
              if (m == 0) v.y = 0;
              if (sc != 0.0) v = C2{v.x * fd, v.y * fd};
              gstore(dst + (int64_t)(c >> 1) * p.nspec, v);
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = it.c0 + wr * WC + i * 16 + acc_row<T>(lane, e);
            if (c < twoF) {
              T v = acc[par][i][j][e];
              if (m == 0 && (c & 1)) v = 0;
              if (sc != 0.0) v *= fd;
              gstore((T*)(dst + (int64_t)(c >> 1) * p.nspec) + (c & 1), v);
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 split precision.  Every operand x (float32) is split into
// hi = bf16_rne(x) and lo = bf16_rne(x - hi); a product is accumulated in
// float32 as lo*hi + hi*lo + hi*hi (the lo*lo term, below float32 rounding of
// the result, is dropped).  MFMA 16x16x32 bf16: lane l holds 8 consecutive K
// of row l % 16 of A (and of column l % 16 of B) starting at K = 8 (l / 16);
// the output placement is that of the f32 16x16x4 instruction.  LDS rows
// are K-contiguous so a lane's operand is one 16-byte read; rows are padded
// by 8 elements so that 16 lanes reading 16 rows hit distinct banks.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16;

__device__ inline f32x4 mfma_bf16(const uint4& a, const uint4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// Split of two floats a, b: words holding (hi_a, hi_b) and (lo_a, lo_b),
// element a in the low half.  The conversions round to nearest even (one
// v_cvt_pk_bf16_f32 each); hi is widened back exactly by a shift.
__device__ inline void split2_bf16(float a, float b, uint32_t* hi, uint32_t* lo) {
  const f32x2v x = {a, b};
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2v));
  const float ha = __uint_as_float(h << 16), hb = __uint_as_float(h & 0xffff0000u);
  const f32x2v r = {a - ha, b - hb};
  *hi = h;
  *lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2v));
}

constexpr int BPAD = 8;



// Synthesis in BF16 split precision on a tile of 128 rings x 64 real
// columns, both parities.  Wave w computes parity w >> 1 on the rows
// [64 (w & 1), +64): a 64 x 64 block of 4 x 4 MFMA blocks, so that each
// 16-byte operand read from LDS feeds four MFMAs per split term and the
// four waves of a SIMD's work groups stay within the LDS rate.  The two
// parities meet in the epilogue through LDS (the N/S fold needs S and A of
// the same element).
//
// LDS operand layout [parity][plane][k chunk of 8][row or column] x 8 k:
// a lane's operand (8 consecutive k of one row or column) is one 16-byte
// read, and 8 lanes reading 8 consecutive rows touch distinct banks.
// The table stages are copied into LDS one step ahead (two stage buffers);
// the spectral values are loaded into registers one step ahead (clamped
// field index, zeros selected) and split into the one spectral stage.
constexpr int BF_BM = 128, BF_BN = 64, BF_KI = 32;

// Spectral-stage slot of column c in k chunk ch: the column XOR the chunk,
// which stays within c's aligned group of 16 columns (so 16 lanes reading
// 16 consecutive columns of one chunk still cover all banks) and spreads
// the chunks of one column over different banks.
__device__ __forceinline__ int bsw(int c, int ch) { return c ^ ch; }

__device__ __forceinline__ void inverse_bf16x3_tile(const DevPlan& p, const WorkItem it, const float* __restrict__ spec,
                                                    float* __restrict__ four) {
  constexpr int BM = BF_BM, BN = BF_BN, KI = BF_KI;
  constexpr int NCK = KI / KCH;         // k chunks per parity per step
  constexpr int AS = 2 * 2 * NCK * BM;  // 16-byte units of one table stage
  constexpr int BS = 2 * 2 * NCK * BN;  // 16-byte units of the spectral stage
  constexpr int FROW = BN + 4;          // epilogue exchange row (floats)
  static_assert(BM == 128 && BN == 64 && BM * FROW * 4 <= 2 * AS * 16, "tile shape");
  // two table stages [par][plane][chunk][BM], then the spectral stage
  // [par][plane][chunk][BN]; 80 KB, two work groups per CU
  __shared__ __align__(16) uint4 smem[2 * AS + BS];
  uint4* Bs = smem + 2 * AS;
  float* Xs = (float*)smem;  // epilogue: A parity [BM][FROW]

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int par = wave >> 1, rh = wave & 1;
  const int kpmax = mi.Kp[0] > mi.Kp[1] ? mi.Kp[0] : mi.Kp[1];
  const int nk = (kpmax + KI - 1) / KI;

  // Loads go through buffer descriptors, one per (parity, plane) table and
  // one for the spectral array from index(m, m) on: reads past a table's
  // padded k range return zero, so spectral values read past n = N (the
  // next wavenumber's, or zeros past the end) meet zero table entries, and
  // rows past the table or fields past F only feed outputs never stored.
  const u16* tab = (const u16*)p.tab;
  const uint32_t a_step = __builtin_amdgcn_readfirstlane((uint32_t)NCK * mi.Lp * KCH * 2);  // bytes per step
  // Table stages are copied from memory straight into LDS, 16 bytes a lane:
  // one copy fills 1 KB at a wave-uniform LDS address with 64 consecutive
  // table units (8 k of 64 consecutive rings, contiguous in the table's
  // chunk-major layout).  Wave w copies parity w / 2, plane w % 2: NCK
  // chunks times two 64-row halves per step.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int cpar = wv >> 1, cpl = wv & 1;
  const __amdgpu_buffer_rsrc_t tr = buffer_rsrc_uniform(tab + (cpl ? p.tab_plane : 0) + mi.toff[cpar],
                                                        (uint64_t)mi.Kp[cpar] * mi.Lp * 2);
  const uint32_t t_lane = (uint32_t)(it.t0 + lane) * KCH * 2;
  auto fetch_table = [&](int kc, int stage) {
    const uint32_t sa = (uint32_t)kc * a_step;
#pragma unroll
    for (int ch = 0; ch < NCK; ++ch) {
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        SHT_LDS void* dst = (SHT_LDS void*)(smem + stage * AS + ((cpar * 2 + cpl) * NCK + ch) * BM + 64 * hf);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(tr, dst, 16, t_lane + (uint32_t)(ch * mi.Lp + 64 * hf) * KCH * 2,
                                                 sa, 0, 0);
      }
    }
  };
  // spectral values: thread (fi, sg) loads segment sg (8 consecutive n - m,
  // both parities: 64 contiguous bytes) of field fi within the step.  The
  // segment is the fastest index, so one load instruction touches 8 fields'
  // rows rather than 32 (the L1's tag lookups, not the bytes, bounded the
  // gather).  The descriptor starts at the tile's first field, so offsets
  // stay small.
  const int fi = tid >> 3, sg = tid & 7;
  const int f0 = it.c0 / 2;
  const int f = f0 + fi;
  const uint32_t fl = (uint32_t)((f < p.F ? f : p.F - 1) - f0);
  const int64_t sbase = (int64_t)f0 * p.nspec + mi.spec_off;
  const __amdgpu_buffer_rsrc_t sr =
      buffer_rsrc_uniform((const float2*)spec + sbase, (uint64_t)((int64_t)p.F * p.nspec - sbase) * 8u);
  const uint32_t b_off = (fl * (uint32_t)p.nspec + 8u * sg) * 8u;
  const bool m0 = m == 0;

  // (raw loads only: anything computed from them here would wait for them)
  float4 rv[4];
  auto fetch_spec = [&](int kc) {
    const uint32_t sb = (uint32_t)kc * (2 * KI * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      rv[q] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(sr, b_off + 16 * q, sb, 0));
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  fetch_table(0, 0);
  fetch_spec(0);
  for (int kc = 0; kc < nk; ++kc) {
    // element i of the segment: parity i & 1, k = 4 sg + i / 2 within the step
    // (chunk sg / 2, offset 4 (sg & 1)); columns 2 fi (re) and 2 fi + 1 (im);
    // Im a_n^0 is dropped
    float2 rb[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      rb[2 * q] = make_float2(rv[q].x, m0 ? 0.f : rv[q].y);
      rb[2 * q + 1] = make_float2(rv[q].z, m0 ? 0.f : rv[q].w);
    }
#pragma unroll
    for (int pa = 0; pa < 2; ++pa) {
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        uint32_t h[2], l[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float2 u = rb[4 * e + pa], w = rb[4 * e + 2 + pa];
          split2_bf16(comp ? u.y : u.x, comp ? w.y : w.x, &h[e], &l[e]);
        }
        // column swizzled by the chunk (see bsw): the 8 lanes of a field
        // write 4 chunks 1 KB apart, which would share banks
        const int slot = ((pa * 2) * NCK + (sg >> 1)) * BN + bsw(2 * fi + comp, sg >> 1);
        uint2* dh = (uint2*)(Bs + slot) + (sg & 1);
        uint2* dl = (uint2*)(Bs + slot + NCK * BN) + (sg & 1);
        *dh = make_uint2(h[0], h[1]);
        *dl = make_uint2(l[0], l[1]);
      }
    }
    // this wave's table copies for step kc have landed; after the barrier
    // every wave's have
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (kc + 1 < nk) {
      fetch_table(kc + 1, (kc + 1) & 1);
      fetch_spec(kc + 1);
    }
    const uint4* As = smem + (kc & 1) * AS;
    uint4 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = bsw(16 * j + (lane & 15), lane >> 4);
      bh[j] = Bs[((par * 2 + 0) * NCK + (lane >> 4)) * BN + c];
      bl[j] = Bs[((par * 2 + 1) * NCK + (lane >> 4)) * BN + c];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 64 * rh + 16 * i + (lane & 15);
      const uint4 ah = As[((par * 2 + 0) * NCK + (lane >> 4)) * BM + r];
      const uint4 al = As[((par * 2 + 1) * NCK + (lane >> 4)) * BM + r];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = mfma_bf16(al, bh[j], acc[i][j]);
        acc[i][j] = mfma_bf16(ah, bl[j], acc[i][j]);
        acc[i][j] = mfma_bf16(ah, bh[j], acc[i][j]);
      }
    }
    // every wave's LDS reads of this step are done before the next step
    // overwrites the spectral stage (and, a step later, this table stage);
    // the table copies in flight are waited for where they are used, not
    // here (a __syncthreads would wait for them too)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  }
  __syncthreads();

  // epilogue: the parity-1 waves hand A to the parity-0 waves through LDS;
  // element (i, j, e): row 64 rh + 16 i + 4 (lane / 16) + e, column 16 j + lane % 16
  if (par == 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          Xs[(64 * rh + 16 * i + 4 * (lane >> 4) + e) * FROW + 16 * j + (lane & 15)] = acc[i][j][e];
  }
  __syncthreads();
  if (par == 0) {
    const int64_t rowlen = 2 * (int64_t)p.Fp;
    const int twoF = 2 * p.F;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rl = 64 * rh + 16 * i + 4 * (lane >> 4) + e;
        const int row = it.t0 + rl;
        if (row >= mi.L) continue;
        const RingInfo rn = gload(p.rings + mi.first_ring + row);
        float* dn = four + (rn.frow + m) * rowlen;
        float* ds = four + (gload(p.rings + rn.mirror).frow + m) * rowlen;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int cl = 16 * j + (lane & 15);
          const int col = it.c0 + cl;
          if (col < twoF) {
            const float S = acc[i][j][e];
            const float A = Xs[rl * FROW + cl];
            gstore(dn + col, S + A);
            gstore(ds + col, S - A);
          }
        }
      }
    }
  }
  __syncthreads();
}

// Synthesis in BF16 split precision on a wide tile: 32 NW rings x 128 real
// columns, both parities, NW waves, MFMA 32x32x16 (NW = 4: 128-ring tiles,
// two work groups per CU; NW = 8: 256-ring tiles, one).  A step takes 16 k
// of each parity (32 consecutive n): 4 NW KB of table and 16 KB of
// spectral operand move into LDS for 24 NW MFMAs, and both
// stages are double buffered (64 or 96 KB), so one barrier per step
// separates the copies of step k + 1 from the products of step k.  Wave w
// owns rows 64 (w >> 1) and columns 64 (w & 1) of both parities (2 x 2
// blocks of 32 x 32 each), so the N/S fold (S + A, S - A) happens in its
// registers.
//
// MFMA 32x32x16 bf16 operand placement, lane l: A[row l % 32][k 8 (l / 32)
// + i], B[k 8 (l / 32) + i][col l % 32] (i < 8, one 16-byte operand);
// accumulator element e holds D[8 (e / 4) + 4 (l / 32) + e % 4][l % 32].
//
// LDS stage layout, 16-byte units of 8 consecutive k:
//   table     [parity][plane][k chunk (2)][row (32 NW)]
//   spectral  [parity][plane][k chunk (2)][column (128) ^ chunk]
// (the spectral column is XORed with the chunk so that the two chunks'
// staging writes, which the lanes of one field make 4 bytes apart, fall on
// different banks; the operand reads keep 32 consecutive units per chunk).
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline f32x16 mfma32_bf16(const uint4& a, const uint4& b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

constexpr int BW_BN = 128, BW_KI = 16;
// waves of the wide synthesis work group: four (two work groups per CU)
// measured 6.68 ms at TCo1279 x 411, eight (one per CU) 6.93 ms
constexpr int BW_WAVES = 4;

template <int NW>
__device__ __forceinline__ void inverse_bf16x3_wide_tile(const DevPlan& p, const WorkItem it,
                                                         const float* __restrict__ spec, float* __restrict__ four) {
  constexpr int BM = 32 * NW, BN = BW_BN, KI = BW_KI;
  constexpr int NT = 64 * NW;
  constexpr int NCK = KI / KCH;         // k chunks per parity per step (2)
  constexpr int AS = 2 * 2 * NCK * BM;  // 16-byte units of one table stage
  constexpr int BS = 2 * 2 * NCK * BN;  // 16-byte units of one spectral stage
  static_assert(NCK == 2 && (NW == 4 || NW == 8) && BN == 128, "tile shape");
  __shared__ __align__(16) uint4 smem[2 * AS + 2 * BS];  // 64 KB (4 waves) or 96 KB (8 waves)

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int rq = wave >> 1, cq = wave & 1;
  const int kpmax = mi.Kp[0] > mi.Kp[1] ? mi.Kp[0] : mi.Kp[1];
  const int nk = (kpmax + KI - 1) / KI;

  // Table copies: a stage is 8 (parity, plane, chunk) slices of BM rows, in
  // 64-row groups of 1 KB (64 lanes x 16 bytes, contiguous in the
  // chunk-major table); each wave copies four groups, of 8 / NW slices that
  // share a parity and plane.  Reads past the table's padded k range return
  // zero; rows past Lp read the next chunk's rows and only feed rows past L,
  // whose outputs are never stored.
  constexpr int RG = BM / 64, CPW = 8 / NW;  // row groups per slice, slices per wave
  const u16* tab = (const u16*)p.tab;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int cpar = (wv * CPW) >> 2, cpl = ((wv * CPW) >> 1) & 1;
  // (selects rather than indexing mi.toff / mi.Kp with a variable, which
  // would put a copy of mi in memory)
  const int64_t ctoff = cpar ? mi.toff[1] : mi.toff[0];
  const int ckp = cpar ? mi.Kp[1] : mi.Kp[0];
  const __amdgpu_buffer_rsrc_t tr =
      buffer_rsrc_uniform(tab + (cpl ? p.tab_plane : 0) + ctoff, (uint64_t)ckp * mi.Lp * 2);
  const uint32_t a_step = __builtin_amdgcn_readfirstlane((uint32_t)NCK * mi.Lp * KCH * 2);
  auto fetch_table = [&](int kc, int stage) {
    const uint32_t sa = (uint32_t)kc * a_step;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int slice = wv * CPW + g / RG, rg = g % RG, cch = slice & 1;
      SHT_LDS void* dst = (SHT_LDS void*)(smem + stage * AS + slice * BM + 64 * rg);
      const uint32_t t_lane = ((uint32_t)(it.t0 + 64 * rg + lane) + (uint32_t)cch * mi.Lp) * KCH * 2;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(tr, dst, 16, t_lane, sa, 0, 0);
    }
  };
  // Spectral values: thread (fi, sg) loads n - m = 32 kc + 4 (U sg + u) .. + 3
  // (u < U) of field f0 + fi (16 bytes each); the field index is clamped to
  // F - 1 (fields past F only feed outputs never stored) and values read
  // past n = N meet zero table entries.
  constexpr int SGN = NT / 64, U = 8 / SGN;  // segments per field, 4-n units per thread
  const int fi = tid / SGN, sg = tid % SGN;
  const int f0 = it.c0 / 2;
  const int f = f0 + fi;
  const uint32_t fl = (uint32_t)((f < p.F ? f : p.F - 1) - f0);
  const int64_t sbase = (int64_t)f0 * p.nspec + mi.spec_off;
  const __amdgpu_buffer_rsrc_t sr =
      buffer_rsrc_uniform((const float2*)spec + sbase, (uint64_t)((int64_t)p.F * p.nspec - sbase) * 8u);
  const uint32_t b_off = (fl * (uint32_t)p.nspec + 4u * U * sg) * 8u;
  const bool m0 = m == 0;
  float4 rv[2 * U];
  auto fetch_spec = [&](int kc) {
    const uint32_t sb = (uint32_t)kc * (2 * KI * 8);
#pragma unroll
    for (int i = 0; i < 2 * U; ++i)
      rv[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(sr, b_off + 16 * i, sb, 0));
  };

  f32x16 acc[2][2][2];
#pragma unroll
  for (int pa = 0; pa < 2; ++pa)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[pa][i][j] = f32x16{};

  fetch_table(0, 0);
  fetch_spec(0);
  for (int kc = 0; kc < nk; ++kc) {
    const int st = kc & 1;
    uint4* Bs = smem + 2 * AS + st * BS;
    // n - m = 4 s + q (q < 4, s = U sg + u): parity q & 1, k = 2 s + (q >> 1)
    // within the step, i.e. chunk s >> 2, bytes 4 (s & 3) of the unit; Im a_n^0
    // dropped
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int su = U * sg + u;
      const int ch = su >> 2;
      const float4 r0 = rv[2 * u], r1 = rv[2 * u + 1];
#pragma unroll
      for (int pa = 0; pa < 2; ++pa) {
#pragma unroll
        for (int comp = 0; comp < 2; ++comp) {
          const float x0 = pa ? (comp ? r0.w : r0.z) : (comp ? r0.y : r0.x);
          const float x1 = pa ? (comp ? r1.w : r1.z) : (comp ? r1.y : r1.x);
          uint32_t h, l;
          split2_bf16((comp && m0) ? 0.f : x0, (comp && m0) ? 0.f : x1, &h, &l);
          const int col = (2 * fi + comp) ^ ch;
          uint32_t* dh = (uint32_t*)(Bs + ((pa * 2 + 0) * NCK + ch) * BN + col) + (su & 3);
          uint32_t* dl = (uint32_t*)(Bs + ((pa * 2 + 1) * NCK + ch) * BN + col) + (su & 3);
          *dh = h;
          *dl = l;
        }
      }
    }
    // this step's table copies (issued a step ago) have landed in every wave,
    // and every wave's spectral staging is visible
    __syncthreads();
    if (kc + 1 < nk) {
      fetch_table(kc + 1, st ^ 1);
      fetch_spec(kc + 1);
    }
    const uint4* As = smem + st * AS;
    const int ch = lane >> 5;
#pragma unroll
    for (int pa = 0; pa < 2; ++pa) {
      uint4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = 64 * rq + 32 * i + (lane & 31);
        ah[i] = As[((pa * 2 + 0) * NCK + ch) * BM + r];
        al[i] = As[((pa * 2 + 1) * NCK + ch) * BM + r];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = (64 * cq + 32 * j + (lane & 31)) ^ ch;
        bh[j] = Bs[((pa * 2 + 0) * NCK + ch) * BN + c];
        bl[j] = Bs[((pa * 2 + 1) * NCK + ch) * BN + c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[pa][i][j] = mfma32_bf16(al[i], bh[j], acc[pa][i][j]);
          acc[pa][i][j] = mfma32_bf16(ah[i], bl[j], acc[pa][i][j]);
          acc[pa][i][j] = mfma32_bf16(ah[i], bh[j], acc[pa][i][j]);
        }
    }
  }
  __syncthreads();

  // epilogue: Fourier row offsets of the tile's rings and their mirrors
  // through LDS, then north = S + A and south = S - A from the registers
  int64_t* roff = (int64_t*)smem;  // [BM][2]
  const int64_t rowlen = 2 * (int64_t)p.Fp;
  if (tid < BM) {
    const int row = it.t0 + tid;
    int64_t on = 0, os = 0;
    if (row < mi.L) {
      const RingInfo rn = gload(p.rings + mi.first_ring + row);
      on = (rn.frow + m) * rowlen;
      os = (gload(p.rings + rn.mirror).frow + m) * rowlen;
    }
    roff[2 * tid] = on;
    roff[2 * tid + 1] = os;
  }
  __syncthreads();
  const int twoF = 2 * p.F;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = 64 * rq + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      if (it.t0 + rl >= mi.L) continue;
      float* dn = four + roff[2 * rl];
      float* ds = four + roff[2 * rl + 1];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = it.c0 + 64 * cq + 32 * j + (lane & 31);
        if (col < twoF) {
          const float S = acc[0][i][j][e];
          const float A = acc[1][i][j][e];
          // 32 lanes write 128 contiguous bytes of a row (whole lines when
          // the workspace is 128-byte aligned): streaming stores (6.73 ->
          // 6.43 ms at TCo1279)
          gstore_nt(dn + col, S + A);
          gstore_nt(ds + col, S - A);
        }
      }
    }
  }
  __syncthreads();
}

// Analysis in BF16 split precision: out^T[c][k] = sum_j X^T[c][j] T[j][k]
// with K = rings.  Both operands need the rings contiguous per lane, so the
// Fourier rows are gathered 8 rings at a time per column and the table
// chunks ([ring][8 k]) are transposed 8 x 8 in registers.  The K loop runs
// without guards (see the unit comments below); ring row offsets are
// looked up a step ahead of the rows' loads.
template <int BC, int BK>
__device__ __forceinline__ void direct_bf16x3_tile(const DevPlan& p, const WorkItem it,
                                                   const float* __restrict__ four, float* __restrict__ spec,
                                                   double sc) {
  const int64_t plane = p.tab_plane;
  constexpr int KJ = 32;
  constexpr int WC = BC / 2, WK = BK / 2;
  constexpr int IC = WC / 16, IK = WK / 16;
  constexpr int NCH = BK / KCH;
  static_assert((BC / 4) * (KJ / 4) == 256, "X units");
  constexpr int TUNITS = 2 * NCH * (KJ / 8) * 2;  // (plane, parity, chunk, ring octet)
  static_assert(TUNITS <= 256, "table units");
  __shared__ __align__(16) u16 Xs[2][2][BC][KJ + BPAD];  // [plane][parity][col c][ring]
  __shared__ __align__(16) u16 Ts[2][2][BK][KJ + BPAD];  // [plane][parity][k][ring]

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const u16* tab = (const u16*)p.tab;
  const int twoF = 2 * p.F;
  const int64_t rowlen = 2 * (int64_t)p.Fp;
  const int nj = (mi.L + KJ - 1) / KJ;

  // X unit: (ring quad, column quad), the column quad fastest, so a load
  // instruction covers two 512-byte row segments (with four rings' 256-byte
  // segments per instruction the L1's tag lookups made the gather 30%
  // slower).  A thread loads the N and S' rows of its 4 rings and forms
  // S = N + S' and A = N - S'.  Rings past L are read at ring L - 1 (their
  // table rows are zero or past the table), and columns past the row end
  // (outputs never stored) are clamped into the row.
  static_assert(BC / 4 == 32, "X units: 32 column quads");
  const int x_cq = tid & 31;
  const int x_q = tid >> 5;
  const int x_c = min(it.c0 + 4 * x_cq, 2 * p.Fp - 4);
  // table unit: (plane, parity, chunk, ring octet), read through one buffer
  // descriptor per (parity, plane): chunks past the table return zero
  const int t_oct = tid % (KJ / 8);
  const int t_ch = (tid / (KJ / 8)) % NCH;
  const int t_par = (tid / ((KJ / 8) * NCH)) % 2;
  const int t_pl = tid / ((KJ / 8) * NCH * 2);
  const bool t_on = tid < TUNITS;  // whole waves
  const __amdgpu_buffer_rsrc_t trs =
      buffer_rsrc(tab + (t_pl ? plane : 0) + (t_par ? mi.toff[1] : mi.toff[0]),
                  (uint32_t)(t_par ? mi.Kp[1] : mi.Kp[0]) * mi.Lp * 2);
  const uint32_t t_off = ((uint32_t)(it.t0 / KCH + t_ch) * mi.Lp + 8u * t_oct) * (KCH * 2);

  // the Fourier rows of the rings of step jc + 1 are looked up one step ahead
  int64_t fr[4], fr_next[4];
  auto fetch_rows = [&](int jc, int64_t* dst) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = min(jc * KJ + 4 * x_q + e, mi.L - 1);
      dst[e] = gload(&p.rings[mi.first_ring + r].frow);
    }
  };
  float4 rx[4][2];  // [ring][N, S']
  uint4 rt[8];
  auto fetch = [&](int jc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float* row = four + ((fr[e] + m) * 2) * rowlen + x_c;
      rx[e][0] = gload((const float4*)row);
      rx[e][1] = gload((const float4*)(row + rowlen));
    }
    if (t_on) {
      const uint32_t so = (uint32_t)jc * KJ * (KCH * 2);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        rt[e] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(trs, t_off + e * (KCH * 2), so, 0));
    }
  };

  f32x4 acc[2][IC][IK];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int i = 0; i < IC; ++i)
#pragma unroll
      for (int j = 0; j < IK; ++j) acc[par][i][j] = f32x4{0, 0, 0, 0};

  fetch_rows(0, fr);
  fetch(0);
  if (nj > 1) fetch_rows(1, fr_next);
  for (int jc = 0; jc < nj; ++jc) {
    // X: 4 columns x 4 rings of S = N + S' and A = N - S' -> per column and
    // parity 4 rings of hi and lo (half of an 8-ring operand unit)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      float4 x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float4 n = rx[e][0], s = rx[e][1];
        x[e] = par ? make_float4(n.x - s.x, n.y - s.y, n.z - s.z, n.w - s.w)
                   : make_float4(n.x + s.x, n.y + s.y, n.z + s.z, n.w + s.w);
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        uint32_t h[2], l[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float4 u = x[2 * e], w = x[2 * e + 1];
          const float a = cc == 0 ? u.x : cc == 1 ? u.y : cc == 2 ? u.z : u.w;
          const float b = cc == 0 ? w.x : cc == 1 ? w.y : cc == 2 ? w.z : w.w;
          split2_bf16(a, b, &h[e], &l[e]);
        }
        *(uint2*)&Xs[0][par][4 * x_cq + cc][4 * x_q] = make_uint2(h[0], h[1]);
        *(uint2*)&Xs[1][par][4 * x_cq + cc][4 * x_q] = make_uint2(l[0], l[1]);
      }
    }
    // table: 8 rings x 8 k (16-bit) -> 8 k x 8 rings
    {
      const uint32_t* w = (const uint32_t*)rt;  // w[4 e + d] holds k = 2d, 2d + 1 of ring e
#pragma unroll
      for (int kk = 0; kk < KCH; ++kk) {
        uint32_t o[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint32_t a = w[4 * (2 * d) + (kk >> 1)];
          const uint32_t b = w[4 * (2 * d + 1) + (kk >> 1)];
          o[d] = (kk & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
        }
        if (t_on) *(uint4*)&Ts[t_pl][t_par][t_ch * KCH + kk][8 * t_oct] = make_uint4(o[0], o[1], o[2], o[3]);
      }
    }
    __syncthreads();
    if (jc + 1 < nj) {
#pragma unroll
      for (int e = 0; e < 4; ++e) fr[e] = fr_next[e];
      fetch(jc + 1);
      if (jc + 2 < nj) fetch_rows(jc + 2, fr_next);
    }
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      uint4 ah[IC], al[IC], bh[IK], bl[IK];
      const int jq = 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < IC; ++i) {
        const int c = wr * WC + i * 16 + (lane & 15);
        ah[i] = *(const uint4*)&Xs[0][par][c][jq];
        al[i] = *(const uint4*)&Xs[1][par][c][jq];
      }
#pragma unroll
      for (int j = 0; j < IK; ++j) {
        const int k = wc * WK + j * 16 + (lane & 15);
        bh[j] = *(const uint4*)&Ts[0][par][k][jq];
        bl[j] = *(const uint4*)&Ts[1][par][k][jq];
      }
#pragma unroll
      for (int i = 0; i < IC; ++i)
#pragma unroll
        for (int j = 0; j < IK; ++j) {
          acc[par][i][j] = mfma_bf16(al[i], bh[j], acc[par][i][j]);
          acc[par][i][j] = mfma_bf16(ah[i], bl[j], acc[par][i][j]);
          acc[par][i][j] = mfma_bf16(ah[i], bh[j], acc[par][i][j]);
        }
    }
    __syncthreads();
  }

#pragma unroll
  for (int par = 0; par < 2; ++par) {
    const int K = par ? mi.K[1] : mi.K[0];
#pragma unroll
    for (int j = 0; j < IK; ++j) {
      const int k = it.t0 + wc * WK + j * 16 + (lane & 15);
      if (k >= K) continue;
      float2* dst = (float2*)spec + (mi.spec_off + 2 * k + par);
      const float fd = sc != 0.0 ? diffusion_factor<float>(m + 2 * k + par, sc) : 1.f;
#pragma unroll
      for (int i = 0; i < IC; ++i) {
#pragma unroll
        for (int e = 0; e < 4; e += 2) {
          const int c = it.c0 + wr * WC + i * 16 + 4 * (lane >> 4) + e;
          if (c < twoF) {
            float2 v = make_float2(acc[par][i][j][e], acc[par][i][j][e + 1]);
            if (m == 0) v.y = 0.f;
            if (sc != 0.0) v = make_float2(v.x * fd, v.y * fd);
            gstore(dst + (int64_t)(c >> 1) * p.nspec, v);
          }
        }
      }
    }
  }
}

// Analysis in BF16 split precision on a tile of 128 k x 128 real columns,
// both parities, eight waves, MFMA 32x32x16: out^T[c][k] = sum_j X^T[c][j]
// T[j][k] over the rings j, 32 rings per step.  Both operands stay in LDS in
// the order they have in memory -- the table as its chunks ([ring][8 k]),
// the Fourier data as ring rows of columns -- and are read into the MFMA
// operand form (8 consecutive rings per lane) with the transposing LDS
// reads of gfx950 (ds_read_b64_tr_b16: within each group of 16 lanes, lane
// i receives element i % 4 of the 8-byte reads addressed by lanes
// 4 t + i / 4, t = 0..3, which was checked on the device).  So the table
// stage is a straight buffer-to-LDS copy, and the Fourier stage is written
// row-contiguous after the S/A fold and the split.
//
// Wave w computes parity w >> 2 on k half (w >> 1) & 1 and column half
// w & 1: 2 x 2 blocks of 32 x 32.  Waves whose k half lies past K skip
// their products.  Both stages are double buffered (136 KB), so one barrier
// per step separates the stores of step j + 1 from the products of step j.
constexpr int DW_BK = 128, DW_BC = 128, DW_KJ = 32;
// LDS banks (measured with the bank-conflict counter): the transposing reads
// of lanes 0..31 (and of 32..63) are served together from 256 bytes (64
// banks of 4 bytes), 8-byte stores 16 lanes at a time from 128 bytes.
// Fourier stage row: 128 columns + 16 (288 bytes), with the 16-column
// blocks b stored at 32 ((b & 1) 4 + b / 2) bytes: a transposing read takes
// 4 rings of blocks b and b + 1 (b even), which then fall on 8 different
// 32-byte bank groups (the rings 32 bytes apart, the blocks 128 apart).
constexpr int DW_XROW = DW_BC + 16;

typedef short i16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint2 lds_read_tr16(const SHT_LDS void* a) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_ds_read_tr16_b64_v4i16((SHT_LDS i16x4*)a));
}

__device__ __forceinline__ void direct_bf16x3_wide_tile(const DevPlan& p, const WorkItem it,
                                                        const float* __restrict__ four, float* __restrict__ spec,
                                                        double sc) {
  constexpr int BK = DW_BK, BC = DW_BC, KJ = DW_KJ, XROW = DW_XROW;
  constexpr int NCH = BK / KCH;                 // table chunks per parity (16)
  constexpr int TS = 2 * 2 * NCH * KJ;          // 16-byte units of a table stage
  constexpr int XS = 2 * 2 * KJ * XROW / 8;     // 16-byte units of a Fourier stage
  static_assert(KJ == 32 && NCH == 16 && BC == 128, "tile shape");
  __shared__ __align__(16) uint4 smem[2 * TS + 2 * XS];  // 136 KB

  const MInfo mi = gload(p.ms + it.m);
  const int m = mi.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nj = (mi.L + KJ - 1) / KJ;

  // Table copies: wave w fills (parity, plane) = w >> 1, chunk pairs
  // 4 (w & 1) .. + 3 of a stage, one 1 KB instruction per pair (64 lanes x
  // 16 bytes: 2 chunks x 32 rings).  In the stage, ring r of chunk c sits at
  // position r ^ (4 (c & 1)) ^ (8 ((c >> 1) & 1)) (chosen through the source
  // address), so that the transposing reads of 32 lanes, which take 4 rings
  // of four consecutive chunks, cover all banks.  Reads past the padded k range return zero; steps
  // never pass Lp (a multiple of the step), and rows in [L, Lp) are zero.
  const u16* tab = (const u16*)p.tab;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int cpar = wv >> 2, cpl = (wv >> 1) & 1;
  const int64_t ctoff = cpar ? mi.toff[1] : mi.toff[0];
  const int ckp = cpar ? mi.Kp[1] : mi.Kp[0];
  const __amdgpu_buffer_rsrc_t trs =
      buffer_rsrc_uniform(tab + (cpl ? p.tab_plane : 0) + ctoff, (uint64_t)ckp * mi.Lp * 2);
  const int lc = lane >> 5;                       // chunk of the pair
  uint32_t t_lane[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int cc = 2 * (4 * (wv & 1) + g) + lc;   // chunk within the tile
    const int lring = (lane & 31) ^ (4 * lc) ^ (8 * (g & 1));  // ring stored at this lane's position
    t_lane[g] = ((uint32_t)(it.t0 / KCH + cc) * mi.Lp + (uint32_t)lring) * (KCH * 2);
  }
  auto fetch_table = [&](int jc, int stage) {
    const uint32_t so = __builtin_amdgcn_readfirstlane((uint32_t)jc * KJ * (KCH * 2));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int pr = 4 * (wv & 1) + g;
      SHT_LDS void* dst = (SHT_LDS void*)(smem + stage * TS + ((cpar * 2 + cpl) * NCH + 2 * pr) * KJ);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(trs, dst, 16, t_lane[g], so, 0, 0);
    }
  };

  // Fourier rows: thread (rp, pos) loads the N and S' rows of rings 2 rp and
  // 2 rp + 1 of the step at the column quad cq whose stage place is 4 pos
  // (columns 4 cq .. + 3 are stored at 4 pos .. + 3 of the row), so that the
  // stores of consecutive lanes are contiguous; a load instruction still
  // covers two 512-byte row segments.  Rings past L are read at ring L - 1
  // (their table rows are zero); columns past the row end (outputs never
  // stored) are clamped into the row.
  const int64_t rowlen = 2 * (int64_t)p.Fp;
  const int x_pos = tid & 31, x_rp = tid >> 5;
  const int x_bp = x_pos >> 2;
  const int x_cq = 4 * (x_bp < 4 ? 2 * x_bp : 2 * x_bp - 7) + (x_pos & 3);
  const int x_c = min(it.c0 + 4 * x_cq, 2 * p.Fp - 4);
  int64_t fr[2], fr_next[2];
  auto fetch_rows = [&](int jc, int64_t* dst) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int r = min(jc * KJ + 2 * x_rp + e, mi.L - 1);
      dst[e] = gload(&p.rings[mi.first_ring + r].frow);
    }
  };
  float4 rx[2][2];  // [ring][N, S']
  auto fetch_x = [&]() {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float* row = four + ((fr[e] + m) * 2) * rowlen + x_c;
      rx[e][0] = gload((const float4*)row);
      rx[e][1] = gload((const float4*)(row + rowlen));
    }
  };

  // operand reads.  Table (B operand, column k): lane (g = lane / 16,
  // i = lane % 16) addresses ring 8 (g >> 1) + 4 h + t of chunk
  // 2 (g & 1) + (q >> 1), at position ring ^ 4 (q >> 1) ^ 8 (g & 1), bytes
  // 8 (q & 1) of the unit, with t = i / 4, q = i % 4, for the two reads
  // h = 0, 1 of a fragment (rings 0..3 and 4..7 of the lane's 8).  Fourier
  // (A operand, column c): ring 8 (g >> 1) + 4 h + t, column
  // 64 chh + 32 i + 16 (g & 1) + 4 q, whose 16-column block 4 chh + 2 i +
  // (g & 1) sits at 32 (4 (g & 1) + 2 chh + i) bytes of the row.
  const int par = wave >> 2, kh = (wave >> 1) & 1, chh = wave & 1;
  const int g = lane >> 4, li = lane & 15, lt = li >> 2, lq = li & 3;
  uint32_t tb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    tb[h] = (uint32_t)(((2 * (g & 1) + (lq >> 1)) * KJ +
                        ((8 * (g >> 1) + 4 * h + lt) ^ (4 * (lq >> 1)) ^ (8 * (g & 1)))) * 16 +
                       8 * (lq & 1));
  const uint32_t xb = (uint32_t)(((8 * (g >> 1) + lt) * XROW + 64 * (g & 1) + 4 * lq) * 2);
  const bool live = it.t0 + 64 * kh < (par ? mi.K[1] : mi.K[0]);

  f32x16 acc[2][2];  // [column block][k block]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};

  fetch_rows(0, fr);
  fetch_table(0, 0);
  fetch_x();
  if (nj > 1) fetch_rows(1, fr_next);
  for (int jc = 0; jc < nj; ++jc) {
    const int st = jc & 1;
    // S = N + S', A = N - S' for 2 rings x 4 columns, split, one 8-byte
    // store per (ring, S/A, plane)
    {
      u16* Xs = (u16*)(smem + 2 * TS + st * XS);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float4 n = rx[e][0], q = rx[e][1];
#pragma unroll
        for (int sa = 0; sa < 2; ++sa) {
          const float4 x = sa ? make_float4(n.x - q.x, n.y - q.y, n.z - q.z, n.w - q.w)
                              : make_float4(n.x + q.x, n.y + q.y, n.z + q.z, n.w + q.w);
          uint32_t h0, l0, h1, l1;
          split2_bf16(x.x, x.y, &h0, &l0);
          split2_bf16(x.z, x.w, &h1, &l1);
          const int row = 2 * x_rp + e;
          lstore((uint2*)(Xs + ((sa * 2 + 0) * KJ + row) * XROW + 4 * x_pos), make_uint2(h0, h1));
          lstore((uint2*)(Xs + ((sa * 2 + 1) * KJ + row) * XROW + 4 * x_pos), make_uint2(l0, l1));
        }
      }
    }
    // this step's table copies (issued a step ago) have landed in every
    // wave, and every wave's Fourier stores are visible
    __syncthreads();
    if (jc + 1 < nj) {
      fr[0] = fr_next[0];
      fr[1] = fr_next[1];
      fetch_table(jc + 1, st ^ 1);
      fetch_x();
      if (jc + 2 < nj) fetch_rows(jc + 2, fr_next);
    }
    if (live) {
      const char* Tb = (const char*)(smem + st * TS) + (size_t)((par * 2) * NCH + 8 * kh) * KJ * 16;
      const char* Xb = (const char*)(smem + 2 * TS + st * XS) + (size_t)(par * 2) * KJ * XROW * 2 + 2 * 16 * 2 * chh;
#pragma unroll
      for (int s = 0; s < 2; ++s) {  // 16 rings per MFMA
        uint4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
          for (int pl = 0; pl < 2; ++pl) {
            const char* base = Xb + pl * KJ * XROW * 2 + 16 * s * XROW * 2 + 16 * i * 2 + xb;
            const uint2 lo = lds_read_tr16((const SHT_LDS void*)base);
            const uint2 hi = lds_read_tr16((const SHT_LDS void*)(base + 4 * XROW * 2));
            (pl ? al[i] : ah[i]) = make_uint4(lo.x, lo.y, hi.x, hi.y);
          }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int pl = 0; pl < 2; ++pl) {
            const char* base = Tb + (size_t)(pl * NCH + 4 * j) * KJ * 16 + 16 * s * 16;
            const uint2 lo = lds_read_tr16((const SHT_LDS void*)(base + tb[0]));
            const uint2 hi = lds_read_tr16((const SHT_LDS void*)(base + tb[1]));
            (pl ? bl[j] : bh[j]) = make_uint4(lo.x, lo.y, hi.x, hi.y);
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = mfma32_bf16(al[i], bh[j], acc[i][j]);
            acc[i][j] = mfma32_bf16(ah[i], bl[j], acc[i][j]);
            acc[i][j] = mfma32_bf16(ah[i], bh[j], acc[i][j]);
          }
      }
    }
  }
  __syncthreads();

  // accumulator element e of lane l: column c = 8 (e / 4) + 4 (l / 32) + e % 4
  // of the block, k = l % 32: (re, im) pairs in elements (0, 1) and (2, 3)
  if (!live) return;
  const int K = par ? mi.K[1] : mi.K[0];
  const int twoF = 2 * p.F;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = it.t0 + 64 * kh + 32 * j + (lane & 31);
    if (k >= K) continue;
    float2* dst = (float2*)spec + (mi.spec_off + 2 * k + par);
    const float fd = sc != 0.0 ? diffusion_factor<float>(m + 2 * k + par, sc) : 1.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        const int c = it.c0 + 64 * chh + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (c < twoF) {
          float2 v = make_float2(acc[i][j][e], acc[i][j][e + 1]);
          if (m == 0) v.y = 0.f;
          if (sc != 0.0) v = make_float2(v.x * fd, v.y * fd);
          gstore(dst + (int64_t)(c >> 1) * p.nspec, v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernels: work groups loop over the items (grid stride), each item with its
// own plan and buffers.
// ---------------------------------------------------------------------------

template <typename T, int BM, int BN, int KI, int WCOL>
__global__ __launch_bounds__(256, 2) void legendre_inverse_kernel(const DevPlan* __restrict__ plans,
                                                               const WorkItem* __restrict__ items, int nitems,
                                                               const IoBind* __restrict__ io, IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    inverse_tile<T, BM, BN, KI, WCOL>(p, it, (const T*)b.spec, (T*)b.ws);
  }
}

template <typename T, int BC, int BK, int KJ, int WKW>
__global__ __launch_bounds__(256, 2) void legendre_direct_kernel(const DevPlan* __restrict__ plans,
                                                              const WorkItem* __restrict__ items, int nitems,
                                                              const IoBind* __restrict__ io, IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    direct_tile<T, BC, BK, KJ, WKW>(p, it, (const T*)b.ws, (T*)b.spec, b.spec_c);
  }
}

__global__ __launch_bounds__(256, 2) void legendre_inverse_bf16x3_kernel(const DevPlan* __restrict__ plans,
                                                                      const WorkItem* __restrict__ items, int nitems,
                                                                      const IoBind* __restrict__ io, IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    inverse_bf16x3_tile(p, it, (const float*)b.spec, (float*)b.ws);
  }
}

__global__ __launch_bounds__(64 * BW_WAVES, BW_WAVES == 4 ? 2 : 1) void legendre_inverse_bf16x3_wide_kernel(
    const DevPlan* __restrict__ plans, const WorkItem* __restrict__ items, int nitems, const IoBind* __restrict__ io,
    IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    inverse_bf16x3_wide_tile<BW_WAVES>(p, it, (const float*)b.spec, (float*)b.ws);
  }
}

template <int BC, int BK>
__global__ __launch_bounds__(256, 2) void legendre_direct_bf16x3_kernel(const DevPlan* __restrict__ plans,
                                                                     const WorkItem* __restrict__ items, int nitems,
                                                                     const IoBind* __restrict__ io, IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    direct_bf16x3_tile<BC, BK>(p, it, (const float*)b.ws, (float*)b.spec, b.spec_c);
  }
}

__global__ __launch_bounds__(512, 1) void legendre_direct_bf16x3_wide_kernel(const DevPlan* __restrict__ plans,
                                                                          const WorkItem* __restrict__ items,
                                                                          int nitems, const IoBind* __restrict__ io,
                                                                          IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const WorkItem it = gload(items + w);
    if (it.m < 0) continue;  // empty slot of the work list
    DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    if (b.pad) p.tab = b.pad;  // tables made for this call (table-free plans)
    direct_bf16x3_wide_tile(p, it, (const float*)b.ws, (float*)b.spec, b.spec_c);
  }
}

// ---------------------------------------------------------------------------
// Variants: (synthesis rows BM, columns BN, waves along columns) and
// (analysis columns BC, k tile BK, waves along k).
// ---------------------------------------------------------------------------

#define INV_F64_C64 legendre_inverse_kernel<double, 64, 64, 16, 2>
#define INV_F64_C32 legendre_inverse_kernel<double, 64, 32, 16, 1>
#define INV_F32_C128 legendre_inverse_kernel<float, 128, 128, 16, 2>
#define INV_F32_C64 legendre_inverse_kernel<float, 128, 64, 16, 2>
#define INV_F32_C32 legendre_inverse_kernel<float, 128, 32, 16, 1>
#define INV_BF16 legendre_inverse_bf16x3_kernel
#define INV_BF16_WIDE legendre_inverse_bf16x3_wide_kernel
#define DIR_F64_C64 legendre_direct_kernel<double, 64, 64, 16, 2>
#define DIR_F64_C32 legendre_direct_kernel<double, 32, 64, 16, 4>
#define DIR_F32_C128 legendre_direct_kernel<float, 128, 64, 16, 2>
#define DIR_F32_C64 legendre_direct_kernel<float, 64, 64, 16, 2>
#define DIR_F32_C32 legendre_direct_kernel<float, 32, 64, 16, 4>
#define DIR_BF16 legendre_direct_bf16x3_kernel<128, 64>
#define DIR_BF16_WIDE legendre_direct_bf16x3_wide_kernel

bool legendre_variant_supported(int prec, int variant) {
  if (prec == SHT_FP64) return variant == TILE_C64 || variant == TILE_C32;
  if (prec == SHT_FP32) return variant >= 0 && variant < NUM_TILE_VARIANTS;
  // bf16x3: synthesis 128 x 64 (C64) or 128 x 128 (C128); analysis 64 k x
  // 128 columns (C64) or 128 k x 128 columns (C128)
  return variant == TILE_C64 || variant == TILE_C128;
}

void legendre_tiles(int prec, int variant, int* inv_rows, int* inv_cols, int* dir_rows, int* dir_cols) {
  const int cols = variant == TILE_C128 ? 128 : variant == TILE_C64 ? 64 : 32;
  *inv_rows = (prec == SHT_FP64) ? 64 : 128;
  *inv_cols = cols;
  if (prec == SHT_BF16X3 && variant == TILE_C128) *inv_rows = 32 * BW_WAVES;
  *dir_rows = (prec == SHT_BF16X3 && variant == TILE_C128) ? 128 : 64;
  *dir_cols = (prec == SHT_BF16X3) ? 128 : cols;
}

template <typename K>
static const void* fn(K k) {
  return (const void*)k;
}

static const void* inverse_fn(int prec, int variant) {
  if (prec == SHT_FP64) return variant == TILE_C32 ? fn(INV_F64_C32) : fn(INV_F64_C64);
  if (prec == SHT_FP32)
    return variant == TILE_C128 ? fn(INV_F32_C128) : variant == TILE_C64 ? fn(INV_F32_C64) : fn(INV_F32_C32);
  return variant == TILE_C128 ? fn(INV_BF16_WIDE) : fn(INV_BF16);
}

static int inverse_threads(int prec, int variant) {
  return (prec == SHT_BF16X3 && variant == TILE_C128) ? 64 * BW_WAVES : 256;
}
static int direct_threads(int prec, int variant) { return (prec == SHT_BF16X3 && variant == TILE_C128) ? 512 : 256; }

static const void* direct_fn(int prec, int variant) {
  if (prec == SHT_FP64) return variant == TILE_C32 ? fn(DIR_F64_C32) : fn(DIR_F64_C64);
  if (prec == SHT_FP32)
    return variant == TILE_C128 ? fn(DIR_F32_C128) : variant == TILE_C64 ? fn(DIR_F32_C64) : fn(DIR_F32_C32);
  return variant == TILE_C128 ? fn(DIR_BF16_WIDE) : fn(DIR_BF16);
}

int legendre_blocks_per_cu(int prec, int variant, bool inverse) {
  int n = 0;
  const void* f = inverse ? inverse_fn(prec, variant) : direct_fn(prec, variant);
  const int threads = inverse ? inverse_threads(prec, variant) : direct_threads(prec, variant);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, threads, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

static hipError_t launch(const void* f, int threads, int grid_blocks, hipStream_t s, const DevPlan* plans,
                         const WorkItem* items, int nitems, const IoBind* io, IoBind io0) {
  void* args[] = {(void*)&plans, (void*)&items, (void*)&nitems, (void*)&io, (void*)&io0};
  return hipLaunchKernel(f, dim3(grid_blocks), dim3(threads), args, 0, s);
}

hipError_t launch_legendre_inverse(const DevPlan* plans, int prec, int variant, const WorkItem* items, int nitems,
                                   const IoBind* io, IoBind io0, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (!legendre_variant_supported(prec, variant)) return hipErrorInvalidValue;
  return launch(inverse_fn(prec, variant), inverse_threads(prec, variant), grid_blocks, s, plans, items, nitems, io,
                io0);
}

hipError_t launch_legendre_direct(const DevPlan* plans, int prec, int variant, const WorkItem* items, int nitems,
                                  const IoBind* io, IoBind io0, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (!legendre_variant_supported(prec, variant)) return hipErrorInvalidValue;
  return launch(direct_fn(prec, variant), direct_threads(prec, variant), grid_blocks, s, plans, items, nitems, io,
                io0);
}

}  // namespace shtmi
