// Longitude transforms of every ring in one launch (report section 4.2.5
// runs one FFT library call per latitude because the lengths differ; here a
// work list of (ring, field chunk) items covers all rings and fields).
//
// A ring of n = 2h points is transformed as a complex DFT of length h of
// z_t = g_{2t} + i g_{2t+1} plus an O(h) pre/post step.  The complex DFT is
// an in-LDS Stockham autosort FFT when h has no prime factor above the
// largest prime radix (37 in FP32, 23 in FP64); otherwise it is the chirp-z (Bluestein) identity
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

// LDS layout of the transforms.  The FFT kernels have no LDS but their
// dynamic buffer, which therefore starts at LDS address 0 (checked on the
// host).  Element y of that buffer, counted over the whole work group,
// sits in slot y + (y >> S): one spare slot after every 2^S elements.  The
// early Stockham passes write with a lane stride of R elements (R Ns with
// Ns < 64), which unpadded would put most lanes of a wave on the same
// banks; the spare slots spread them.  S is 3 for 8-byte elements (FP32
// complex) and 5 for 16-byte ones (FP64): measured over the TCo1279 stages,
// FP32 spacings of 8, 16 and 32 elements took 16.6, 17.6 and 17.2 ms per
// synthesis (4: 17.6), FP64 spacings of 8, 16 and 32 took 39.5, 40.2 and
// 39.3 ms.  Field s of a work group owns the elements [s fs, s fs + L),
// fs = lds_stride(L) a multiple of 32, so the byte address of any element
// is (y + (y >> S)) * sizeof(C), two instructions from its index.
__host__ __device__ constexpr int fft_pad_shift(size_t elem) { return elem == 8 ? 3 : 5; }
__host__ __device__ constexpr uint32_t lds_stride(int L) { return ((uint32_t)L + 31u) & ~31u; }
// slots that hold the elements [0, n)
__host__ __device__ constexpr size_t lds_slots(size_t n, size_t elem) { return n + (n >> fft_pad_shift(elem)) + 1; }
template <typename C>
__device__ __forceinline__ SHT_LDS C* lds_elem(uint32_t y) {
  return (SHT_LDS C*)((y + (y >> fft_pad_shift(sizeof(C)))) * (uint32_t)sizeof(C));
}

// 8- and 16-byte values in LDS through an address-space-3 pointer (32-bit
// addresses), and from a table through a raw buffer descriptor whose range
// is not checked (every offset used is inside the table).
template <typename C>
__device__ __forceinline__ C lds_load(const SHT_LDS C* p) {
  if constexpr (sizeof(C) == 8) return __builtin_bit_cast(C, *(const SHT_LDS gword2*)p);
  else return __builtin_bit_cast(C, *(const SHT_LDS gword4*)p);
}
template <typename C>
__device__ __forceinline__ void lds_store(SHT_LDS C* p, const C& v) {
  if constexpr (sizeof(C) == 8) *(SHT_LDS gword2*)p = __builtin_bit_cast(gword2, v);
  else *(SHT_LDS gword4*)p = __builtin_bit_cast(gword4, v);
}
// The base is the same on every lane (a table of the transform's class);
// reading it from the first lane tells the compiler so, which keeps the
// descriptor in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base) {
  const uint64_t a = (uint64_t)base;
  const uint64_t u = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
  return __builtin_amdgcn_make_buffer_rsrc((void*)u, (short)0, (int)0x7fffffff, 0x00020000);
}
template <typename C>
__device__ __forceinline__ C buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  if constexpr (sizeof(C) == 8) return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
  else return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0));
}
// The same over `bytes` bytes from a base that is the same on every lane:
// loads past the range return zero and stores past it are dropped, which
// the sweeps use in place of per-element guards (offsets stay below 2^31:
// the host refuses plans whose ring blocks would not).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc_range(const void* base, uint32_t bytes) {
  const uint64_t a = (uint64_t)base;
  const uint64_t u = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
  return __builtin_amdgcn_make_buffer_rsrc((void*)u, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
template <typename C>
__device__ __forceinline__ void buffer_store(const C& v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  if constexpr (sizeof(C) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(gword2, v), r, byte_off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(gword4, v), r, byte_off, 0, 0);
}

// exp(-2 pi i j / R) at compile time: the angle is reduced exactly to
// |r| <= pi/4 from the nearest quarter turn (4j - qR is an integer), then
// sine and cosine of r are summed as Taylor series to double precision.
struct UnitRoot {
  double c, s;  // cos and sin of 2 pi j / R; the root is c - i s
};
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr UnitRoot unit_root(int j, int R) {
  j = ((j % R) + R) % R;
  const int q = (8 * j + R) / (2 * R);  // nearest integer to 4 j / R
  const double r = (kPi / 2) * (double)(4 * j - q * R) / (double)R;
  const double c = taylor_cos(r), sn = taylor_sin(r);
  switch (q & 3) {
    case 0: return UnitRoot{c, sn};
    case 1: return UnitRoot{-sn, c};
    case 2: return UnitRoot{-c, -sn};
    default: return UnitRoot{sn, -c};
  }
}

template <typename T, int R>
__device__ inline void butterfly(typename V2T<T>::type* v);

// One Cooley-Tukey step for R = R1 R2 in registers: with n = R2 n1 + n2 and
// k = k1 + R1 k2,
//   X[k] = sum_n2 W_R2^(n2 k2) W_R^(n2 k1) sum_n1 x[n] W_R1^(n1 k1),
// i.e. R2 DFTs of length R1, twiddles W_R^(n2 k1), R1 DFTs of length R2.
template <typename T, int R1, int R2>
__device__ inline void butterfly_ct(typename V2T<T>::type* v) {
  typedef typename V2T<T>::type C;
  constexpr int R = R1 * R2;
  C y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[R2 * n1 + n2];
    butterfly<T, R1>(y[n2]);
  }
#pragma unroll
  for (int n2 = 1; n2 < R2; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      const UnitRoot w = unit_root(n2 * k1, R);
      y[n2][k1] = cmul(y[n2][k1], C{(T)w.c, (T)-w.s});
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    C t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
    butterfly<T, R2>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
  }
}

// cos and sin of 2 pi j / P for j < P, evaluated by the front end (a
// constexpr object), so that the unrolled butterflies below index constants
// rather than expanding unit_root's series P^2 / 4 times.
template <int P>
struct RootTable {
  double c[P], s[P];
  constexpr RootTable() : c(), s() {
    for (int j = 0; j < P; ++j) {
      const UnitRoot r = unit_root(j, P);
      c[j] = r.c;
      s[j] = r.s;
    }
  }
};

// DFT of an odd prime number P of points.  With the pairs
// u_j = x_j + x_{P-j} and v_j = x_j - x_{P-j} (1 <= j <= H = (P - 1) / 2),
//   X_0 = x_0 + sum_j u_j,
//   X_k = a_k - i b_k and X_{P-k} = a_k + i b_k (1 <= k <= H), where
//   a_k = x_0 + sum_j cos(2 pi j k / P) u_j and b_k = sum_j sin(2 pi j k / P) v_j:
// 4 H^2 real multiply-adds, with the cosines and sines folded to immediates.
// Each output pair goes to emit(k, X_k) as soon as it is formed, so a pass
// can store it at once and hold only the pairs and two outputs (about P
// complex values) rather than all P outputs beside the pairs.
template <typename T, int P, typename E>
__device__ inline void butterfly_odd_emit(const typename V2T<T>::type* v, E&& emit) {
  typedef typename V2T<T>::type C;
  constexpr int H = (P - 1) / 2;
  constexpr RootTable<P> rt{};
  C u[H], w[H];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    u[j - 1] = cadd(v[j], v[P - j]);
    w[j - 1] = csub(v[j], v[P - j]);
  }
  const C x0 = v[0];
  C s0 = x0;
#pragma unroll
  for (int j = 0; j < H; ++j) s0 = cadd(s0, u[j]);
  emit(0, s0);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    C a = x0, b = C{0, 0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const T cjk = (T)rt.c[(j * k) % P], sjk = (T)rt.s[(j * k) % P];
      a.x += cjk * u[j - 1].x;
      a.y += cjk * u[j - 1].y;
      b.x += sjk * w[j - 1].x;
      b.y += sjk * w[j - 1].y;
    }
    emit(k, cadd(a, cmul_negi(b)));
    emit(P - k, csub(a, cmul_negi(b)));
  }
}

template <typename T, int P>
__device__ inline void butterfly_odd(typename V2T<T>::type* v) {
  typedef typename V2T<T>::type C;
  butterfly_odd_emit<T, P>(v, [&](int r, const C& y) { v[r] = y; });
}

__host__ __device__ constexpr bool odd_prime_radix(int R) {
  return R == 7 || R == 11 || R == 13 || R == 17 || R == 19 || R == 23 || R == 29 || R == 31 || R == 37;
}

// Forward DFT of R points in registers.  Radices 2, 3, 4 and 5 are written
// out; 8 and 16 take one even/odd step, 9 a 3 x 3 step, the odd primes
// from 7 to 37 the pair form above, and the composite radices 6, 10, 12,
// 14, 15, 18 and 20 the generic step above.
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
  } else if constexpr (odd_prime_radix(R)) {
    butterfly_odd<T, R>(v);
  } else if constexpr (R == 6) {
    butterfly_ct<T, 3, 2>(v);
  } else if constexpr (R == 10) {
    butterfly_ct<T, 5, 2>(v);
  } else if constexpr (R == 12) {
    butterfly_ct<T, 4, 3>(v);
  } else if constexpr (R == 14) {
    butterfly_ct<T, 7, 2>(v);
  } else if constexpr (R == 15) {
    butterfly_ct<T, 5, 3>(v);
  } else if constexpr (R == 18) {
    butterfly_ct<T, 9, 2>(v);
  } else if constexpr (R == 20) {
    butterfly_ct<T, 5, 4>(v);
  } else {
    static_assert(R == 0, "unsupported radix");
  }
}

// What the last pass of a transform does with its outputs.
enum PassOut { OUT_PLAIN = 0, OUT_HEAD = 1, OUT_GRID = 2, OUT_GRID_CHIRP = 3, OUT_GRID_LOG = 4, OUT_GRID_CHIRP_LOG = 5 };

// One Stockham pass of radix R over L points in LDS, after Ns points have
// been combined, carried out by the nt threads (thread lt) that own this
// transform: butterfly b reads x[b + r L/R], twiddles input r by
// exp(-2 pi i r (b mod Ns) / (Ns R)) (the pass's table holds these at
// (b mod Ns)(R - 1) + r - 1, so lanes with consecutive b read consecutive
// entries) and writes y[(b / Ns) Ns R + b mod Ns + r Ns].  All reads of the
// pass land in registers before the barrier, so one LDS buffer suffices.
//   OUT_HEAD stores y_q for q < h only (the analysis applies the chirp-z
//     convolution's last element-wise step, c_q conj(y_q), to the values it
//     reads afterwards);
//   OUT_GRID writes conj(y_q) and OUT_GRID_CHIRP writes conj(c_q) y_q, the
//     conjugates of y_q and of c_q conj(y_q), for q < h to io in device
//     memory (nothing when io is null), as non-temporal stores (2% faster
//     at TCo1279: the grid streams past the Fourier rows still being read
//     from L2); OUT_GRID_LOG and OUT_GRID_CHIRP_LOG
//     write each real value g of those as g + ga g (1 - g) (the grid-point
//     step of a time step), in instantiations of their own so that the plain
//     transforms' stores carry no test of ga.
// Each instantiation is its own non-inlined function so that its registers
// are allocated for it alone.  Every thread of the work group calls it (the
// barriers).
template <typename T, int R, int MODE>
__device__ __noinline__ void stockham_pass(uint32_t e0, int L, int Ns,
                                           const typename V2T<T>::type* tw, const typename V2T<T>::type* aux,
                                           typename V2T<T>::type* io, int h, int lt, int nt, T ga) {
  typedef typename V2T<T>::type C;
  // a radix above FFT_REGS (a prime) runs as the first pass only (the plan
  // sees to it): Ns = 1, no twiddles, one butterfly per thread
  constexpr bool FIRST = R > FFT_REGS;
  constexpr int MAXB = FIRST ? 1 : FFT_REGS / R;
  // the lengths are the same on every lane; arguments arrive in vector
  // registers, and read from the first lane the divisions below are scalar
  L = __builtin_amdgcn_readfirstlane(L);
  Ns = __builtin_amdgcn_readfirstlane(Ns);
  nt = __builtin_amdgcn_readfirstlane(nt);
  h = __builtin_amdgcn_readfirstlane(h);
  if constexpr (FIRST) Ns = 1;
  const int nb = L / R;
  // b mod Ns by multiply-high: for b < 2^14 and 1 < Ns <= 2^13,
  // floor(b / Ns) = umulhi(b, ceil(2^32 / Ns)) exactly
  const uint32_t magic = Ns > 1 ? 0xFFFFFFFFu / (uint32_t)Ns + 1u : 0u;
  // twiddles and the chirp-z factors through buffer descriptors: 32-bit
  // offsets, the per-r displacement in the instruction's immediate
  const __amdgpu_buffer_rsrc_t trs = buffer_rsrc(tw);
  const __amdgpu_buffer_rsrc_t ars = buffer_rsrc(aux);
  C v[MAXB][R];
  int kk[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = lt + i * nt;
    kk[i] = Ns > 1 ? b - (int)__umulhi((uint32_t)b, magic) * Ns : 0;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds_load(lds_elem<C>(e0 + (uint32_t)(b + r * nb)));
      if (!FIRST && Ns > 1) {
        const uint32_t t = (uint32_t)(kk[i] * (R - 1)) * (uint32_t)sizeof(C);
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], buffer_load<C>(trs, t + (r - 1) * sizeof(C)));
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = lt + i * nt;
    if (b < nb) {
      const int k = kk[i];
      const int d = (b - k) * R + k;
      auto emit = [&](int r, const C& y) {
        const int o = d + r * Ns;
        const uint32_t ao = (uint32_t)o * (uint32_t)sizeof(C);
        if constexpr (MODE == OUT_PLAIN) {
          lds_store(lds_elem<C>(e0 + (uint32_t)o), y);
        } else if constexpr (MODE == OUT_HEAD) {
          if (o < h) lds_store(lds_elem<C>(e0 + (uint32_t)o), y);
        } else if constexpr (MODE == OUT_GRID || MODE == OUT_GRID_LOG) {
          // plain transforms have L = h, so o < h always
          if (io) {
            C g = cconj(y);
            if constexpr (MODE == OUT_GRID_LOG) g = C{logistic_step(g.x, ga), logistic_step(g.y, ga)};
            gstore_nt(io + o, g);
          }
        } else {
          if (io && o < h) {
            C g = cmul(cconj(buffer_load<C>(ars, ao)), y);
            if constexpr (MODE == OUT_GRID_CHIRP_LOG) g = C{logistic_step(g.x, ga), logistic_step(g.y, ga)};
            gstore_nt(io + o, g);
          }
        }
      };
      if constexpr (odd_prime_radix(R)) {
        butterfly_odd_emit<T, R>(v[i], emit);
      } else {
        butterfly<T, R>(v[i]);
#pragma unroll
        for (int r = 0; r < R; ++r) emit(r, v[i][r]);
      }
    }
  }
  __syncthreads();
}

template <typename T, int MODE, bool BIG>
__device__ __forceinline__ void pass_dispatch(int R, uint32_t e0, int L, int Ns,
                                     const typename V2T<T>::type* tw, const typename V2T<T>::type* aux,
                                     typename V2T<T>::type* io, int h, int lt, int nt, T ga = T(0)) {
#define SHT_PASS(RR) stockham_pass<T, RR, MODE>(e0, L, Ns, tw, aux, io, h, lt, nt, ga)
  // radices with a factor above 5 occur only in plain transforms of length h
  // (the chirp-z lengths are 5-smooth); the primes above FFT_BIG_PRIME only
  // in the BIG kernels, and only in FP32
  constexpr bool PLAIN_LEN = MODE == OUT_PLAIN || MODE == OUT_GRID || MODE == OUT_GRID_LOG;
  if constexpr (PLAIN_LEN && BIG && sizeof(T) == 4) {
    switch (R) {
      case 37: SHT_PASS(37); return;
      case 31: SHT_PASS(31); return;
      case 29: SHT_PASS(29); return;
      default: break;
    }
  }
  if constexpr (PLAIN_LEN) {
    switch (R) {
      case 23: SHT_PASS(23); return;
      case 19: SHT_PASS(19); return;
      case 17: SHT_PASS(17); return;
      case 14: SHT_PASS(14); return;
      case 13: SHT_PASS(13); return;
      case 11: SHT_PASS(11); return;
      case 7: SHT_PASS(7); return;
      default: break;
    }
  }
  switch (R) {
    case 20: SHT_PASS(20); break;
    case 18: SHT_PASS(18); break;
    case 16: SHT_PASS(16); break;
    case 15: SHT_PASS(15); break;
    case 12: SHT_PASS(12); break;
    case 10: SHT_PASS(10); break;
    case 9: SHT_PASS(9); break;
    case 8: SHT_PASS(8); break;
    case 6: SHT_PASS(6); break;
    case 5: SHT_PASS(5); break;
    case 4: SHT_PASS(4); break;
    case 3: SHT_PASS(3); break;
    default: SHT_PASS(2); break;
  }
#undef SHT_PASS
}

// Passes q0 <= q < q1 of a forward DFT of L points held in LDS (radices
// packed in rp), starting after Ns points have been combined with tw at pass
// q0's table; the last of them applies MODE with aux and io.  All passes
// from Ns = 1: natural order in and out.
template <typename T, int MODE, bool BIG>
__device__ __forceinline__ void fft_passes(uint32_t e0, int L, uint64_t rp, int q0, int q1, int Ns,
                                           const typename V2T<T>::type* tw, const typename V2T<T>::type* aux,
                                           typename V2T<T>::type* io, int h, int lt, int nt, T ga = T(0)) {
  for (int q = q0; q < q1; ++q) {
    const int R = packed_radix(rp, q);
    if (q == q1 - 1) pass_dispatch<T, MODE, BIG>(R, e0, L, Ns, tw, aux, io, h, lt, nt, ga);
    else pass_dispatch<T, OUT_PLAIN, BIG>(R, e0, L, Ns, tw, nullptr, nullptr, h, lt, nt);
    tw += Ns * (R - 1);
    Ns *= R;
  }
}

// The middle of the chirp-z convolution: the last pass of the forward
// transform (radix R, after Ns = L / R points), the element-wise step
// B = conj(A khat), and the first pass of the second transform, which runs
// the same radix sequence, whose first radix is also R (the plan gives
// chirp-z classes palindromic sequences), at Ns = 1.
// Butterfly b of both passes covers the elements b + r L/R (r < R): the
// first pass writes them and the second reads them, so one thread takes
// both in registers, with no LDS round trip or barrier in between, and
// writes y[b R + r].  The twiddles exp(-2 pi i r b / L) are the first
// pass's (b < Ns).
template <typename T, int R>
__device__ __noinline__ void chirp_middle_pass(uint32_t e0, int L, const typename V2T<T>::type* tw,
                                               const typename V2T<T>::type* khat, int lt, int nt) {
  typedef typename V2T<T>::type C;
  constexpr int MAXB = FFT_REGS / R;
  L = __builtin_amdgcn_readfirstlane(L);  // uniform: a scalar division
  nt = __builtin_amdgcn_readfirstlane(nt);
  const int nb = L / R;
  const __amdgpu_buffer_rsrc_t trs = buffer_rsrc(tw);
  const __amdgpu_buffer_rsrc_t krs = buffer_rsrc(khat);
  C v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = lt + i * nt;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds_load(lds_elem<C>(e0 + (uint32_t)(b + r * nb)));
      const uint32_t t = (uint32_t)(b * (R - 1)) * (uint32_t)sizeof(C);
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], buffer_load<C>(trs, t + (r - 1) * sizeof(C)));
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = lt + i * nt;
    if (b < nb) {
      butterfly<T, R>(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[i][r] = cconj(cmul(v[i][r], buffer_load<C>(krs, (uint32_t)(b + r * nb) * (uint32_t)sizeof(C))));
      butterfly<T, R>(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) lds_store(lds_elem<C>(e0 + (uint32_t)(b * R + r)), v[i][r]);
    }
  }
  __syncthreads();
}

// The chirp-z lengths are 5-smooth.
template <typename T>
__device__ __forceinline__ void middle_dispatch(int R, uint32_t e0, int L, const typename V2T<T>::type* tw,
                                                const typename V2T<T>::type* khat, int lt, int nt) {
#define SHT_MID(RR) chirp_middle_pass<T, RR>(e0, L, tw, khat, lt, nt)
  switch (R) {
    case 20: SHT_MID(20); break;
    case 18: SHT_MID(18); break;
    case 16: SHT_MID(16); break;
    case 15: SHT_MID(15); break;
    case 12: SHT_MID(12); break;
    case 10: SHT_MID(10); break;
    case 9: SHT_MID(9); break;
    case 8: SHT_MID(8); break;
    case 6: SHT_MID(6); break;
    case 5: SHT_MID(5); break;
    case 4: SHT_MID(4); break;
    case 3: SHT_MID(3); break;
    default: SHT_MID(2); break;
  }
#undef SHT_MID
}

// Forward complex DFT of length h.  Input: z_t, t < h, in LDS at
// element e0 + t, multiplied by the chirp c_t for chirp-z classes, whose
// entries h <= t < L must be zero.  Output: Z_q, q < h, in LDS at element
// e0 + q, or with GRID_OUT its conjugate written to io (nothing when io is
// null).  Chirp-z: A = DFT_L(a), B = conj(A khat), y = DFT_L(B) and
// Z_q = c_q conj(y_q); without GRID_OUT the LDS holds y_q, and the caller
// forms Z_q for the q it reads.  The radix sequence begins and ends with the
// same radix, so the second DFT's first pass fuses with the first DFT's
// last (a chirp-z length exceeds the largest radix, so each DFT has at
// least two passes).
template <typename T, bool GRID_OUT, bool BIG, bool LOG = false>
__device__ __forceinline__ void dft_h(uint32_t e0, const FftClass& c,
                      const typename V2T<T>::type* tabs, typename V2T<T>::type* io, int lt, int nt, T ga = T(0)) {
  const typename V2T<T>::type* tw = tabs + c.root_off;
  const int p = c.nrad;
  // the packed radices are the same on every lane: in scalar registers they
  // stay out of the vector registers the code around the pass calls holds
  // (as a vector value the analysis kernel spilled, 2 ms slower at TCo1279)
  const uint64_t rp = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(c.radpack >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)c.radpack);
  constexpr int GRID_MODE = LOG ? OUT_GRID_LOG : OUT_GRID;
  constexpr int CHIRP_MODE = LOG ? OUT_GRID_CHIRP_LOG : OUT_GRID_CHIRP;
  if (!c.bluestein) {
    fft_passes<T, GRID_OUT ? GRID_MODE : OUT_PLAIN, BIG>(e0, c.L, rp, 0, p, 1, tw, nullptr, io, c.h, lt, nt, ga);
    return;
  }
  const int R = packed_radix(rp, 0);
  fft_passes<T, OUT_PLAIN, false>(e0, c.L, rp, 0, p - 1, 1, tw, nullptr, nullptr, c.h, lt, nt);
  middle_dispatch<T>(R, e0, c.L, tw + (c.L / R - 1), tabs + c.khat_off, lt, nt);
  fft_passes<T, GRID_OUT ? CHIRP_MODE : OUT_HEAD, false>(e0, c.L, rp, 1, p, R, tw + (R - 1), tabs + c.chirp_off,
                                                         io, c.h, lt, nt, ga);
}

// Sweeps over a ring (gathers, scatters) issue the global loads of
// FFT_SWEEP iterations before using any of them.
constexpr int FFT_SWEEP = 4;

// Launch size: one work group per item.
size_t fft_grid_blocks(int nitems) { return (size_t)nitems; }

// ---------------------------------------------------------------------------
// Synthesis: ring j, the fields [f0, fend) side by side (fend - f0 <= G).
//   X_m = c_m for m <= mmax_j (Im c_0 dropped), 0 above, Nyquist 0;
//   Z_q = (X_q + conj X_{h-q}) + i w^q (X_q - conj X_{h-q}),  w = exp(2 pi i / n);
//   z = inverse DFT_h(Z) = conj(DFT_h(conj Z));  g_{2t} = Re z_t,  g_{2t+1} = Im z_t.
// Field f0 + s owns the LDS elements [s fs, s fs + L), fs = lds_stride(L), and threads
// [s nt, (s + 1) nt).
// The gather of X reads element e as (q = e / G, s = e mod G), so that
// neighbouring lanes read neighbouring fields of one Fourier row.
// ---------------------------------------------------------------------------

template <typename T, int NT, bool BIG>
__device__ __forceinline__ void synthesis_group(const DevPlan& p, int ring, int cls, int fb, int fend,
                                                const T* __restrict__ four, T* __restrict__ grid, T ga) {
  typedef typename V2T<T>::type C;
  const RingInfo ri = gload(p.rings + ring);
  const FftClass cl = gload(p.classes + cls);
  const C* tabs = (const C*)p.fft;
  const C* post = tabs + cl.post_off;
  const C* chirp = tabs + cl.chirp_off;
  const C* fc = (const C*)four;
  const int h = cl.h, mmax = ri.mmax, L = cl.L;
  const bool blue = cl.bluestein;
  const int64_t Fp = p.Fp;
  const int gs = cl.gshift, G = 1 << gs;
  const int nt = NT >> gs;
  const int sub = threadIdx.x / nt, lt = threadIdx.x - sub * nt;
  const uint32_t fs = lds_stride(L);
  {
    // Z_q and Z_{h-q} are built from the same two coefficients X_q and
    // X_{h-q}, so pair p = q (0 <= q <= h/2) loads them once and writes both.
    // The loads go through descriptors: the group's Fourier rows 0..mmax of
    // the ring (X_q = 0 above mmax, and X_h, read for q = 0, is past them as
    // mmax < h), and the post and chirp tables (h entries each).  Fields past
    // F read the row's padding columns; their transforms are never stored.
    const __amdgpu_buffer_rsrc_t xr =
        buffer_rsrc_range(fc + ri.frow * Fp + fb, (uint32_t)((mmax + 1) * Fp * (int64_t)sizeof(C)));
    const __amdgpu_buffer_rsrc_t pr = buffer_rsrc_range(post, (uint32_t)(h * sizeof(C)));
    const __amdgpu_buffer_rsrc_t cr = buffer_rsrc_range(chirp, blue ? (uint32_t)(h * sizeof(C)) : 0u);
    const uint32_t rowb = (uint32_t)(Fp * sizeof(C));
    const int np = (h / 2 + 1) << gs;
    for (int e0 = threadIdx.x; e0 < np; e0 += FFT_SWEEP * NT) {
      // the factors of h - q follow from those of q: w^{-(h-q)} = -conj(w^{-q})
      // and c_{h-q} = (-1)^h c_q ((h - q)^2 = q^2 mod 2h for even h)
      C xa[FFT_SWEEP], xb[FFT_SWEEP], pa[FFT_SWEEP], ca[FFT_SWEEP];
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int e = e0 + u * NT;
        const uint32_t s = (uint32_t)(e & (G - 1)), q = (uint32_t)(e >> gs), q2 = (uint32_t)h - q;
        xa[u] = xb[u] = pa[u] = ca[u] = C{0, 0};
        // lanes past the pairs (most of a small ring's) skip the loads, whole
        // waves at a time
        if (e < np) {
          xa[u] = buffer_load<C>(xr, q * rowb + s * (uint32_t)sizeof(C));
          xb[u] = buffer_load<C>(xr, q2 * rowb + s * (uint32_t)sizeof(C));
          pa[u] = buffer_load<C>(pr, q * (uint32_t)sizeof(C));
          if (blue) ca[u] = buffer_load<C>(cr, q * (uint32_t)sizeof(C));
        }
      }
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int e = e0 + u * NT;
        if (e < np) {
          const int s = e & (G - 1), q = e >> gs, q2 = h - q;
          C A = xa[u];
          if (q == 0) A.y = 0;  // Im c_0 is dropped
          const C B = xb[u];
          {
            // Z_q from X_q = A and conj X_{h-q} = conj B; zero where nothing was loaded
            const C xr = cconj(B);
            const C sm = cadd(A, xr);
            const C t = cmul(cconj(pa[u]), csub(A, xr));
            C y = C{sm.x - t.y, -(sm.y + t.x)};  // conj(sm + i t)
            if (blue) y = cmul(y, ca[u]);
            lds_store(lds_elem<C>(s * fs + q), y);
          }
          if (q >= 1 && q2 != q) {
            // Z_{h-q} from X_{h-q} = B and conj X_q = conj A; conj(w^{-(h-q)}) = -w^{-q}
            const C xr = cconj(A);
            const C sm = cadd(B, xr);
            const C t = cmul(pa[u], csub(xr, B));
            C y = C{sm.x - t.y, -(sm.y + t.x)};
            if (blue) y = cmul(y, (h & 1) ? C{-ca[u].x, -ca[u].y} : ca[u]);
            lds_store(lds_elem<C>(s * fs + q2), y);
          }
        }
      }
    }
    // chirp-z classes: zero padding h <= t < L
    if (blue) {
      const int nz = (L - h) << gs;
      for (int e = threadIdx.x; e < nz; e += NT) {
        const int s = e & (G - 1), t = h + (e >> gs);
        lds_store(lds_elem<C>(s * fs + t), C{0, 0});
      }
    }
    __syncthreads();
    // ring offsets and lengths are even, so (g_{2t}, g_{2t+1}) is one aligned pair
    const int f = fb + sub;
    C* g = f < fend ? (C*)(grid + (int64_t)f * p.npts + ri.goff) : nullptr;
    // the last pass writes the grid (the conjugate of the inverse transform)
    // the time step's grid-point operation has stores of its own (the
    // choice is uniform across the work group)
    if (ga != T(0)) dft_h<T, true, BIG, true>(sub * fs, cl, tabs, g, lt, nt, ga);
    else dft_h<T, true, BIG>(sub * fs, cl, tabs, g, lt, nt);
  }
}

// ---------------------------------------------------------------------------
// Analysis: north ring j and its mirror, one after the other, the fields
// [f0, fend) side by side.
//   Z = DFT_h(z),  X_m = (Z_m + conj Z_{h-m})/2 - (i/2) w^{-m} (Z_m - conj Z_{h-m}),
//   chat_m = X_m / n, written as w_j chat_m to the north ring's Fourier
//   row: slot 0 for the ring, slot 1 for its mirror (the Legendre analysis
//   forms S = N + S' and A = N - S' as it stages them, so neither ring
//   waits in LDS for the other; one work item still takes both, which
//   measured faster than one ring per item).  An item of at most G/2 fields
//   (the few fields of a small transform) transforms both rings at once:
//   the mirror's fields take the upper half of the G field slots.  The
//   halves meet at thread NT/2, a wave boundary, so every wave's ring is
//   uniform.  Otherwise the rings go one after the other.  The output step
//   writes element e as (m = e / G, slot s = e mod G) so that neighbouring
//   lanes write neighbouring fields of one Fourier row.
// ---------------------------------------------------------------------------

template <typename T, int NT, bool BIG>
__device__ __forceinline__ void analysis_group(const DevPlan& p, int ring, int cls, int fb, int fend,
                                               const T* __restrict__ grid, T* __restrict__ four) {
  typedef typename V2T<T>::type C;
  // the mirror of north ring j is ring nlat - 1 - j
  const RingInfo rn = gload(p.rings + ring);
  const RingInfo rs = gload(p.rings + (p.nlat - 1 - ring));
  const FftClass cl = gload(p.classes + cls);
  const C* tabs = (const C*)p.fft;
  const int h = cl.h, mmax = rn.mmax, L = cl.L;
  const int gs = cl.gshift, G = 1 << gs;
  const uint32_t fs = lds_stride(L);
  const C* post = tabs + cl.post_off;
  const C* chirp = tabs + cl.chirp_off;
  C* fc = (C*)four;
  const bool blue = cl.bluestein;
  const T scale = (T)(gload(p.wa + ring) / (double)rn.nlon);
  const int nt = NT >> gs;
  const int sub = threadIdx.x / nt, lt = threadIdx.x - sub * nt;
  const int Q = blue ? L : h;
  const int M = mmax + 1;
  const int half = G >> 1;
  const bool both = fend - fb <= half;
  const int my_side = both && sub >= half ? 1 : 0;
  const int f = fb + sub - my_side * half;
  const uint32_t dst = sub * fs;
  // Grid loads through a descriptor from field fb's ring (the same on every
  // lane) that ends after the h points of field fend - 1: fields past fend
  // read zero; t >= h is selected to zero (other fields' rows follow).
  // Chirp factors through one of h entries.  Fourier stores through a
  // descriptor from field fb of the north ring's first row to the end of
  // its rows 0..mmax (both slots): wavenumbers past mmax start past it and
  // are dropped, and fields past F (zero transforms) write zeros into the
  // rows' padding columns.
  const __amdgpu_buffer_rsrc_t cr = buffer_rsrc_range(chirp, blue ? (uint32_t)(h * sizeof(C)) : 0u);
  const uint32_t fo = (uint32_t)(f - fb) * (uint32_t)p.npts * (uint32_t)sizeof(T);
  const uint32_t grange = (uint32_t)(((int64_t)(fend - 1 - fb) * p.npts + 2 * (int64_t)h) * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t orr = buffer_rsrc_range(
      fc + (rn.frow * 2) * (int64_t)p.Fp + fb, (uint32_t)(2 * ((int64_t)mmax + 1) * p.Fp * (int64_t)sizeof(C)));
  for (int pass = 0; pass < (both ? 1 : 2); ++pass) {
    const int side = both ? my_side : pass;
    const __amdgpu_buffer_rsrc_t gr =
        buffer_rsrc_range(grid + (int64_t)fb * p.npts + (side ? rs.goff : rn.goff), grange);
    for (int t0 = lt; t0 < Q; t0 += FFT_SWEEP * nt) {
      C z[FFT_SWEEP], c[FFT_SWEEP];
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int t = t0 + u * nt;
        z[u] = C{0, 0};
        c[u] = C{1, 0};
        // the chirp-z padding (t >= h, more than half of those rings) loads
        // nothing
        if (t < h) {
          z[u] = buffer_load<C>(gr, fo + (uint32_t)t * (uint32_t)sizeof(C));
          if (blue) c[u] = buffer_load<C>(cr, (uint32_t)t * (uint32_t)sizeof(C));
        }
      }
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int t = t0 + u * nt;
        if (t < Q) lds_store(lds_elem<C>(dst + t), blue ? cmul(z[u], c[u]) : z[u]);
      }
    }
    __syncthreads();
    dft_h<T, false, BIG>(dst, cl, tabs, nullptr, lt, nt);
    // chirp-z classes hold y_q: Z_m = c_m conj(y_m), and
    // conj Z_{h-m} = conj(c_{h-m}) y_{h-m} with c_{h-m} = (-1)^h c_m
    const int nm = M << gs;
    const __amdgpu_buffer_rsrc_t pr = buffer_rsrc_range(post, (uint32_t)(h * sizeof(C)));
    for (int e0 = threadIdx.x; e0 < nm; e0 += FFT_SWEEP * NT) {
      C pm[FFT_SWEEP], cm[FFT_SWEEP];
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int e = e0 + u * NT;
        const uint32_t m = (uint32_t)(e >> gs);
        pm[u] = C{0, 0};
        cm[u] = C{1, 0};
        if (e < nm) {
          pm[u] = buffer_load<C>(pr, m * (uint32_t)sizeof(C));
          if (blue) cm[u] = buffer_load<C>(cr, m * (uint32_t)sizeof(C));
        }
      }
#pragma unroll
      for (int u = 0; u < FFT_SWEEP; ++u) {
        const int e = e0 + u * NT;
        if (e >= nm) continue;
        const int s = e & (G - 1), m = e >> gs;
        const int es = both ? (s >= half ? 1 : 0) : side;  // the ring of slot s
        C zm = lds_load(lds_elem<C>(s * fs + m));
        C zr = lds_load(lds_elem<C>(s * fs + (m == 0 ? 0 : h - m)));
        if (blue) {
          const C cr = (m > 0 && (h & 1)) ? C{-cm[u].x, -cm[u].y} : cm[u];
          zm = cmul(cm[u], cconj(zm));
          zr = cmul(cconj(cr), zr);
        } else {
          zr = cconj(zr);
        }
        const C sm = cadd(zm, zr);
        const C d = csub(zm, zr);
        const C t = cmul(pm[u], d);
        // X = sm/2 - (i/2) t
        C x = C{(T)0.5 * (sm.x + t.y), (T)0.5 * (sm.y - t.x)};
        if (m == 0) x = C{zm.x + zm.y, 0};
        buffer_store(cscale(x, scale), orr,
                     (((uint32_t)m * 2u + (uint32_t)es) * (uint32_t)p.Fp + (uint32_t)(s - es * half * both)) *
                         (uint32_t)sizeof(C));
      }
    }
    // the next transform's input sweep overwrites this one
    __syncthreads();
  }
}

size_t fft_lds_bytes(int prec, int L, int G) {
  const size_t c = (prec == SHT_FP64) ? 16 : 8;
  return c * lds_slots((size_t)G * lds_stride(L), c);
}

// Kernels: work groups loop over the items (grid stride), one kernel per
// work-group size NT.  FP32 kernels are held to 128 VGPRs (4 waves per SIMD:
// four 256-thread or two 512-thread work groups per CU); FP64 ones need twice
// the registers and get 2 waves per SIMD.
template <typename T>
struct FftWaves {
  static constexpr int value = sizeof(T) == 4 ? 4 : 2;
};

template <typename T, int NT, bool BIG>
__global__ __launch_bounds__(NT, FftWaves<T>::value) void fourier_synthesis_kernel(const DevPlan* __restrict__ plans,
                                                                                  const FftItem* __restrict__ items,
                                                                                  int nitems,
                                                                                  const IoBind* __restrict__ io,
                                                                                  IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const FftItem it = gload(items + w);
    if (it.ring < 0) continue;
    const DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    synthesis_group<T, NT, BIG>(p, it.ring, it.cls, it.f0, it.fend, (const T*)b.ws, (T*)b.grid, (T)b.grid_a);
  }
}

template <typename T, int NT, bool BIG>
__global__ __launch_bounds__(NT, FftWaves<T>::value) void fourier_analysis_kernel(const DevPlan* __restrict__ plans,
                                                                                 const FftItem* __restrict__ items,
                                                                                 int nitems,
                                                                                 const IoBind* __restrict__ io,
                                                                                 IoBind io0) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const FftItem it = gload(items + w);
    if (it.ring < 0) continue;
    const DevPlan p = gload(plans + it.plan);
    const IoBind b = io ? gload(io + it.plan) : io0;
    analysis_group<T, NT, BIG>(p, it.ring, it.cls, it.f0, it.fend, (const T*)b.grid, (T*)b.ws);
  }
}

// The kernel of a precision, direction and tier (FP64 classes never take
// the prime radices above FFT_BIG_PRIME, so its tiers 2 and 3 are 0 and 1).
template <typename T, bool BIG>
static const void* fft_kernel_of(bool synthesis, bool large) {
  if (synthesis)
    return large ? (const void*)fourier_synthesis_kernel<T, FFT_THREADS, BIG>
                 : (const void*)fourier_synthesis_kernel<T, FFT_THREADS_SMALL, BIG>;
  return large ? (const void*)fourier_analysis_kernel<T, FFT_THREADS, BIG>
               : (const void*)fourier_analysis_kernel<T, FFT_THREADS_SMALL, BIG>;
}

static const void* fft_kernel(int prec, bool synthesis, int tier) {
  const bool large = (tier & 1) != 0;
  if (prec == SHT_FP64) return fft_kernel_of<double, false>(synthesis, large);
  return tier >= 2 ? fft_kernel_of<float, true>(synthesis, large) : fft_kernel_of<float, false>(synthesis, large);
}

static hipError_t launch_fft(const void* f, int threads, int grid_blocks, size_t lds, hipStream_t s,
                             const DevPlan* plans, const FftItem* items, int nitems, const IoBind* io, IoBind io0) {
  void* args[] = {(void*)&plans, (void*)&items, (void*)&nitems, (void*)&io, (void*)&io0};
  return hipLaunchKernel(f, dim3(grid_blocks), dim3(threads), args, lds, s);
}

hipError_t launch_fourier_synthesis(const DevPlan* plans, int prec, int tier, const FftItem* items, int nitems,
                                    const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  return launch_fft(fft_kernel(prec, true, tier), fft_tier_threads(tier), grid_blocks, lds, s, plans, items, nitems,
                    io, io0);
}

hipError_t launch_fourier_analysis(const DevPlan* plans, int prec, int tier, const FftItem* items, int nitems,
                                   const IoBind* io, IoBind io0, size_t lds, int grid_blocks, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  return launch_fft(fft_kernel(prec, false, tier), fft_tier_threads(tier), grid_blocks, lds, s, plans, items, nitems,
                    io, io0);
}

int fft_blocks_per_cu(int prec, int tier, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fft_kernel(prec, true, tier), fft_tier_threads(tier), lds) !=
          hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

// Every FFT kernel addresses its dynamic LDS buffer from LDS address 0,
// which holds only while the kernels declare no LDS of their own.
hipError_t fft_set_max_lds(size_t bytes) {
  for (int prec : {SHT_FP64, SHT_FP32})
    for (int syn = 0; syn < 2; ++syn)
      for (int tier = 0; tier < FFT_TIERS; ++tier) {
        const void* f = fft_kernel(prec, syn != 0, tier);
        hipFuncAttributes a;
        hipError_t e = hipFuncGetAttributes(&a, f);
        if (e != hipSuccess) return e;
        if (a.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

}  // namespace shtmi
