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

// LDS index of FFT element i.  Kept unpadded: then the R reads and the R
// writes of a butterfly sit at constant strides from one base address and
// need no per-element address arithmetic (padding against bank conflicts
// was measured and bought nothing, while costing that arithmetic).
__device__ inline int lds_ix(int i) { return i; }

// Forward DFT of R points in registers.  Radices 8, 9 and 16 are built from
// smaller ones by one Cooley-Tukey step (even/odd halves for 8 and 16,
// 3 x 3 for 9).
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
  } else if constexpr (R == 8 || R == 16) {
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    butterfly<T, H>(e);
    butterfly<T, H>(o);
    // o[k] *= exp(-2 pi i k / R)
    constexpr double c16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                               0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    constexpr double s16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                               1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
#pragma unroll
    for (int k = 1; k < H; ++k) {
      const int q = k * (16 / R);
      o[k] = cmul(o[k], C{(T)c16[q], (T)-s16[q]});
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + H] = csub(e[k], o[k]);
    }
  } else if constexpr (R == 9) {
    // X[k1 + 3 k2] = sum_n2 w9^(n2 k1) w3^(n2 k2) DFT3_n1(v[3 n1 + n2])[k1]
    const T c1 = (T)0.76604444311897803520, s1 = (T)0.64278760968653932632;  // 2 pi / 9
    const T c2 = (T)0.17364817766693034885, s2 = (T)0.98480775301220805936;  // 4 pi / 9
    const T c4 = (T)-0.93969262078590838405, s4 = (T)0.34202014332566873304; // 8 pi / 9
    C y[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      C t[3] = {v[n2], v[3 + n2], v[6 + n2]};
      butterfly<T, 3>(t);
      y[n2][0] = t[0];
      y[n2][1] = t[1];
      y[n2][2] = t[2];
    }
    y[1][1] = cmul(y[1][1], C{c1, -s1});
    y[1][2] = cmul(y[1][2], C{c2, -s2});
    y[2][1] = cmul(y[2][1], C{c2, -s2});
    y[2][2] = cmul(y[2][2], C{c4, -s4});
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      C t[3] = {y[0][k1], y[1][k1], y[2][k1]};
      butterfly<T, 3>(t);
      v[k1] = t[0];
      v[k1 + 3] = t[1];
      v[k1 + 6] = t[2];
    }
  }
}

// What the last pass of a transform does with its outputs.
enum PassOut { OUT_PLAIN = 0, OUT_KHAT = 1, OUT_CHIRP = 2 };

// One Stockham pass of radix R over L points in LDS, after Ns points have
// been combined: butterfly b reads x[b + r L/R], twiddles input r by
// exp(-2 pi i r (b mod Ns) / (Ns R)) (the pass's table holds these at
// (b mod Ns)(R - 1) + r - 1, so lanes with consecutive b read consecutive
// entries) and writes y[(b / Ns) Ns R + b mod Ns + r Ns].  All reads of the pass land in registers before the barrier, so
// one LDS buffer suffices.  OUT_KHAT stores conj(y khat) and OUT_CHIRP
// stores c_q conj(y_q) for q < h (the element-wise steps of the chirp-z
// convolution).  Each instantiation is its own non-inlined function so that
// its registers are allocated for it alone.
template <typename T, int R, int MODE>
__device__ __noinline__ void stockham_pass(typename V2T<T>::type* buf, int L, int Ns,
                                           const typename V2T<T>::type* tw, const typename V2T<T>::type* aux,
                                           int h) {
  typedef typename V2T<T>::type C;
  constexpr int MAXB = FFT_REGS / R;
  const int nb = L / R;
  // b mod Ns by multiply-high: for b < 2^14 and 1 < Ns <= 2^13,
  // floor(b / Ns) = umulhi(b, ceil(2^32 / Ns)) exactly
  const uint32_t magic = Ns > 1 ? 0xFFFFFFFFu / (uint32_t)Ns + 1u : 0u;
  C v[MAXB][R];
  int kk[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * FFT_THREADS;
    kk[i] = Ns > 1 ? b - (int)__umulhi((uint32_t)b, magic) * Ns : 0;
    if (b < nb) {
      const C* src = buf + b;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * nb];
      if (Ns > 1) {
        const C* t = tw + kk[i] * (R - 1) - 1;
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], t[r]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * FFT_THREADS;
    if (b < nb) {
      butterfly<T, R>(v[i]);
      const int k = kk[i];
      const int d = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int o = d + r * Ns;
        if constexpr (MODE == OUT_PLAIN) {
          buf[o] = v[i][r];
        } else if constexpr (MODE == OUT_KHAT) {
          buf[o] = cconj(cmul(v[i][r], aux[o]));
        } else {
          if (o < h) buf[o] = cmul(aux[o], cconj(v[i][r]));
        }
      }
    }
  }
  __syncthreads();
}

template <typename T, int MODE>
__device__ inline void pass_dispatch(int R, typename V2T<T>::type* buf, int L, int Ns,
                                     const typename V2T<T>::type* tw, const typename V2T<T>::type* aux, int h) {
  switch (R) {
    case 16: stockham_pass<T, 16, MODE>(buf, L, Ns, tw, aux, h); break;
    case 9: stockham_pass<T, 9, MODE>(buf, L, Ns, tw, aux, h); break;
    case 8: stockham_pass<T, 8, MODE>(buf, L, Ns, tw, aux, h); break;
    case 5: stockham_pass<T, 5, MODE>(buf, L, Ns, tw, aux, h); break;
    case 4: stockham_pass<T, 4, MODE>(buf, L, Ns, tw, aux, h); break;
    case 3: stockham_pass<T, 3, MODE>(buf, L, Ns, tw, aux, h); break;
    default: stockham_pass<T, 2, MODE>(buf, L, Ns, tw, aux, h); break;
  }
}

// Forward DFT of L points held in LDS (natural order in and out); the last
// pass applies MODE.
template <typename T, int MODE>
__device__ void fft_lds(typename V2T<T>::type* buf, int L, int nrad, const int32_t* rad,
                        const typename V2T<T>::type* tw, const typename V2T<T>::type* aux, int h) {
  int Ns = 1;
  for (int q = 0; q < nrad; ++q) {
    const int R = rad[q];
    if (q == nrad - 1) pass_dispatch<T, MODE>(R, buf, L, Ns, tw, aux, h);
    else pass_dispatch<T, OUT_PLAIN>(R, buf, L, Ns, tw, aux, h);
    tw += Ns * (R - 1);
    Ns *= R;
  }
}

// Forward complex DFT of length h.  On entry buf[t] holds z_t, t < h,
// already multiplied by the chirp c_t for chirp-z classes, whose entries
// h <= t < L must be zero.  On exit buf[q], q < h, holds Z_q.  Chirp-z:
// A = DFT_L(a), B = conj(A khat), Z_q = c_q conj(DFT_L(B))_q.
template <typename T>
__device__ void dft_h(typename V2T<T>::type* buf, const FftClass& c, const int32_t* rad,
                      const typename V2T<T>::type* tabs) {
  const typename V2T<T>::type* tw = tabs + c.root_off;
  if (!c.bluestein) {
    fft_lds<T, OUT_PLAIN>(buf, c.L, c.nrad, rad, tw, nullptr, c.h);
    return;
  }
  fft_lds<T, OUT_KHAT>(buf, c.L, c.nrad, rad, tw, tabs + c.khat_off, c.h);
  fft_lds<T, OUT_CHIRP>(buf, c.L, c.nrad, rad, tw, tabs + c.chirp_off, c.h);
}

constexpr int FFT_FCHUNK = 16;
constexpr int NUM_XCD = 8;

// Work-group -> (work item, field).  One work item is a ring (pair) and a
// chunk of FFT_FCHUNK fields that share cache lines of the Fourier buffer
// (fields are its innermost index).  Work groups are handed to the XCDs
// round-robin by id, so the FFT_FCHUNK fields of an item get ids that are
// congruent modulo NUM_XCD and adjacent in dispatch order: they run on one
// XCD at the same time and their strided accesses meet in that XCD's L2.
__device__ inline bool decode_block(int bid, int nitems, int* item, int* slot) {
  const int grp = bid / (NUM_XCD * FFT_FCHUNK);
  const int r = bid - grp * (NUM_XCD * FFT_FCHUNK);
  *item = grp * NUM_XCD + r % NUM_XCD;
  *slot = r / NUM_XCD;
  return *item < nitems;
}

__host__ __device__ inline size_t fft_grid_blocks_dev(int nitems) {
  return (size_t)((nitems + NUM_XCD - 1) / NUM_XCD) * NUM_XCD * FFT_FCHUNK;
}

size_t fft_grid_blocks(int nitems) { return fft_grid_blocks_dev(nitems); }

// ---------------------------------------------------------------------------
// Synthesis: ring j, one field of the chunk [f0, f0 + FFT_FCHUNK).
//   X_m = c_m for m <= mmax_j (Im c_0 dropped), 0 above, Nyquist 0;
//   Z_q = (X_q + conj X_{h-q}) + i w^q (X_q - conj X_{h-q}),  w = exp(2 pi i / n);
//   z = inverse DFT_h(Z) = conj(DFT_h(conj Z));  g_{2t} = Re z_t,  g_{2t+1} = Im z_t.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void synthesis_field(const DevPlan& p, int ring, int f, const T* __restrict__ four,
                                                T* __restrict__ grid) {
  typedef typename V2T<T>::type C;
  extern __shared__ __align__(16) unsigned char smem[];
  const RingInfo ri = p.rings[ring];
  const FftClass cl = p.classes[ri.cls];
  const int32_t* rad = p.classes[ri.cls].rad;
  const C* tabs = (const C*)p.fft;
  C* buf = (C*)smem;
  const C* post = tabs + cl.post_off;
  const C* chirp = tabs + cl.chirp_off;
  const C* fc = (const C*)four;
  const int h = cl.h, mmax = ri.mmax, L = cl.L;
  const bool blue = cl.bluestein;
  const int64_t Fp = p.Fp;
  {
    const C* cf = fc + ri.frow * Fp + f;
    for (int q = threadIdx.x; q < (blue ? L : h); q += FFT_THREADS) {
      C y = C{0, 0};
      if (q < h) {
        C xq = (q <= mmax) ? cf[q * Fp] : C{0, 0};
        if (q == 0) xq.y = 0;
        const int q2 = h - q;
        const C xr = (q >= 1 && q2 <= mmax) ? cconj(cf[q2 * Fp]) : C{0, 0};
        const C s = cadd(xq, xr);
        const C t = cmul(cconj(post[q]), csub(xq, xr));
        y = C{s.x - t.y, -(s.y + t.x)};  // conj(s + i t)
        if (blue) y = cmul(y, chirp[q]);
      }
      buf[lds_ix(q)] = y;
    }
    __syncthreads();
    dft_h<T>(buf, cl, rad, tabs);
    T* g = grid + (int64_t)f * p.npts + ri.goff;
    for (int t = threadIdx.x; t < h; t += FFT_THREADS) {
      const C y = buf[lds_ix(t)];
      g[2 * t] = y.x;
      g[2 * t + 1] = -y.y;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Analysis: north ring j and its mirror, one field of the chunk [f0, f0 + FFT_FCHUNK).
//   Z = DFT_h(z),  X_m = (Z_m + conj Z_{h-m})/2 - (i/2) w^{-m} (Z_m - conj Z_{h-m}),
//   chat_m = X_m / n;  S = w_j (chat_N + chat_S),  A = w_j (chat_N - chat_S).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void analysis_field(const DevPlan& p, int ring, int f, const T* __restrict__ grid,
                                               T* __restrict__ four) {
  typedef typename V2T<T>::type C;
  extern __shared__ __align__(16) unsigned char smem[];
  const RingInfo rn = p.rings[ring];
  const RingInfo rs = p.rings[rn.mirror];
  const FftClass cl = p.classes[rn.cls];
  const int32_t* rad = p.classes[rn.cls].rad;
  const C* tabs = (const C*)p.fft;
  C* buf = (C*)smem;
  C* keep = buf + lds_ix(cl.L) + 1;
  const C* post = tabs + cl.post_off;
  const C* chirp = tabs + cl.chirp_off;
  C* fc = (C*)four;
  const int h = cl.h, mmax = rn.mmax, L = cl.L;
  const bool blue = cl.bluestein;
  const T scale = (T)(p.w[ring] / (double)rn.nlon);
  {
    for (int side = 0; side < 2; ++side) {
      const T* g = grid + (int64_t)f * p.npts + (side ? rs.goff : rn.goff);
      for (int t = threadIdx.x; t < (blue ? L : h); t += FFT_THREADS) {
        C z = C{0, 0};
        if (t < h) {
          z = C{g[2 * t], g[2 * t + 1]};
          if (blue) z = cmul(z, chirp[t]);
        }
        buf[lds_ix(t)] = z;
      }
      __syncthreads();
      dft_h<T>(buf, cl, rad, tabs);
      for (int m = threadIdx.x; m <= mmax; m += FFT_THREADS) {
        const C zm = buf[lds_ix(m)];
        const C zr = cconj(buf[lds_ix(m == 0 ? 0 : h - m)]);
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
  const size_t padded = (size_t)L + 1;
  return c * (padded + (mmax >= 0 ? (size_t)mmax + 1 : 0));
}

// Kernels: work groups loop over virtual block ids (grid stride) so that a
// launch of any size keeps the XCD grouping of decode_block.
template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void fourier_synthesis_kernel(const DevPlan* __restrict__ plans,
                                                                        const FftItem* __restrict__ items, int nitems,
                                                                        const IoBind* __restrict__ io, IoBind io0) {
  const int nvirt = (int)fft_grid_blocks_dev(nitems);
  for (int v = blockIdx.x; v < nvirt; v += gridDim.x) {
    int item, slot;
    if (!decode_block(v, nitems, &item, &slot)) continue;
    const FftItem it = items[item];
    const DevPlan p = plans[it.plan];
    const int f = it.f0 + slot;
    if (f >= p.F) continue;
    const IoBind b = io ? io[it.plan] : io0;
    synthesis_field<T>(p, it.ring, f, (const T*)b.ws, (T*)b.grid);
  }
}

template <typename T>
__global__ __launch_bounds__(FFT_THREADS) void fourier_analysis_kernel(const DevPlan* __restrict__ plans,
                                                                       const FftItem* __restrict__ items, int nitems,
                                                                       const IoBind* __restrict__ io, IoBind io0) {
  const int nvirt = (int)fft_grid_blocks_dev(nitems);
  for (int v = blockIdx.x; v < nvirt; v += gridDim.x) {
    int item, slot;
    if (!decode_block(v, nitems, &item, &slot)) continue;
    const FftItem it = items[item];
    const DevPlan p = plans[it.plan];
    const int f = it.f0 + slot;
    if (f >= p.F) continue;
    const IoBind b = io ? io[it.plan] : io0;
    analysis_field<T>(p, it.ring, f, (const T*)b.grid, (T*)b.ws);
  }
}

static hipError_t launch_fft(const void* f, int grid_blocks, size_t lds, hipStream_t s, const DevPlan* plans,
                             const FftItem* items, int nitems, const IoBind* io, IoBind io0) {
  void* args[] = {(void*)&plans, (void*)&items, (void*)&nitems, (void*)&io, (void*)&io0};
  return hipLaunchKernel(f, dim3(grid_blocks), dim3(FFT_THREADS), args, lds, s);
}

hipError_t launch_fourier_synthesis(const DevPlan* plans, int prec, const FftItem* items, int nitems,
                                    const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  const void* f = prec == SHT_FP64 ? (const void*)fourier_synthesis_kernel<double>
                                   : (const void*)fourier_synthesis_kernel<float>;
  return launch_fft(f, grid_blocks, lds, s, plans, items, nitems, io, io0);
}

hipError_t launch_fourier_analysis(const DevPlan* plans, int prec, const FftItem* items, int nitems,
                                   const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  const void* f = prec == SHT_FP64 ? (const void*)fourier_analysis_kernel<double>
                                   : (const void*)fourier_analysis_kernel<float>;
  return launch_fft(f, grid_blocks, lds, s, plans, items, nitems, io, io0);
}

int fft_blocks_per_cu(int prec, size_t lds) {
  int n = 0;
  const void* f = prec == SHT_FP64 ? (const void*)fourier_synthesis_kernel<double>
                                   : (const void*)fourier_synthesis_kernel<float>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, FFT_THREADS, lds) != hipSuccess || n < 1) n = 1;
  return n;
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
