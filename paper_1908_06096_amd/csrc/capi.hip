// Host runtime and C ABI: plan construction (geometry, FFT classes, table
// layout, work lists), one device arena per plan, the stream-ordered entry
// points, and batches of plans run in shared launches.  Following the
// report's restructured time step (section 4.2.3), everything that allocates
// or copies metadata happens once at plan (or batch) creation; the transform
// calls only enqueue kernels.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "sht_internal.h"

using namespace shtmi;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return SHT_EHIP;
}

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool five_smooth(int64_t x) {
  if (x < 1) return false;
  for (int p : {2, 3, 5})
    while (x % p == 0) x /= p;
  return x == 1;
}

// A length the passes of a precision can factor: no prime factor above its
// largest prime radix, FFT_MAX_PRIME in FP32 (the primes above FFT_BIG_PRIME
// run in kernels of their own) and FFT_BIG_PRIME in FP64 (where those
// butterflies spill).
bool radix_smooth(int64_t x, int prec) {
  if (x < 1) return false;
  const int maxp = prec == SHT_FP64 ? FFT_BIG_PRIME : FFT_MAX_PRIME;
  for (int p : {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37})
    if (p <= maxp)
      while (x % p == 0) x /= p;
  return x == 1;
}

// Radices the passes can use (each has a register butterfly), larger first.
constexpr int kRadices[] = {37, 31, 29, 23, 20, 19, 18, 17, 16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2};

// A pass of radix R over L points fits `threads` threads when its L / R
// butterflies fit the FFT_REGS / R butterflies each thread holds (one for
// the prime radices above FFT_REGS).
bool radix_fits(int L, int R, int threads) {
  return (int64_t)(L / R) <= (int64_t)std::max(1, FFT_REGS / R) * threads;
}

// Fewest passes for the cofactor x of L (memoised), and the first radix.
// Radices above FFT_REGS are taken for the first pass only (x = L).
int fewest_passes(int L, int x, int threads, std::map<int, std::pair<int, int>>* memo) {
  if (x == 1) return 0;
  auto it = memo->find(x);
  if (it != memo->end()) return it->second.first;
  int bp = 1 << 20, br = 0;
  for (int R : kRadices)
    if (x % R == 0 && (R <= FFT_REGS || x == L) && radix_fits(L, R, threads)) {
      const int c = 1 + fewest_passes(L, x / R, threads, memo);
      if (c < bp) {
        bp = c;
        br = R;
      }
    }
  (*memo)[x] = {bp, br};
  return bp;
}

// Radix sequence for a length without prime factors above FFT_MAX_PRIME (the chirp-z
// lengths are 5-smooth): the fewest passes that all fit
// `threads` threads, the larger radix first among equally short sequences.
// Each pass is one LDS round trip and two barriers, which is what the
// transforms' time goes to.  Empty when no sequence fits.
// With `palindrome` the first and last radices are equal: a chirp-z class
// runs the sequence twice and fuses the last pass of the first transform
// with the first pass of the second.
std::vector<int> radices(int L, int threads = FFT_THREADS, bool palindrome = false) {
  std::map<int, std::pair<int, int>> memo;
  std::vector<int> r;
  if (!palindrome) {
    if (fewest_passes(L, L, threads, &memo) >= (1 << 20)) return r;
    for (int x = L; x > 1; x /= memo[x].second) r.push_back(memo[x].second);
    return r;
  }
  int best = 1 << 20, ba = 0;
  for (int a : kRadices) {
    if (a > FFT_REGS || L % (a * a) != 0 || !radix_fits(L, a, threads)) continue;
    const int n = 2 + fewest_passes(L, L / (a * a), threads, &memo);
    if (n < best) {
      best = n;
      ba = a;
    }
  }
  if (ba == 0) return r;
  r.push_back(ba);
  for (int x = L / (ba * ba); x > 1; x /= memo[x].second) r.push_back(memo[x].second);
  r.push_back(ba);
  return r;
}

// Chirp-z length for half length h: among the 5-smooth L >= 2h - 1 (up to a
// quarter above) with a palindromic radix sequence of p passes, the one with
// the least L (2p - 1), the LDS traffic of the two transforms with their
// middle passes fused.  0 when none fits.
int bluestein_length(int h) {
  const int64_t lo = 2 * (int64_t)h - 1;
  const int64_t hi = lo + std::max<int64_t>(64, lo / 4);
  int best = 0;
  double best_cost = 0;
  for (int64_t L = lo; L <= hi && L < (1 << 14); ++L) {
    if (!five_smooth(L)) continue;
    const std::vector<int> r = radices((int)L, FFT_THREADS, true);
    if (r.empty()) continue;
    const double cost = (double)L * (double)(2 * r.size() - 1);
    if (best == 0 || cost < best_cost) {
      best = (int)L;
      best_cost = cost;
    }
  }
  return best;
}

// The dynamic-LDS limit is a property of the kernel functions: raise it to
// the largest any plan needs.
std::mutex g_lds_mu;
size_t g_lds_max = 0;

hipError_t ensure_lds(size_t bytes) {
  std::lock_guard<std::mutex> lk(g_lds_mu);
  if (bytes <= g_lds_max) return hipSuccess;
  hipError_t e = fft_set_max_lds(bytes);
  if (e == hipSuccess) g_lds_max = bytes;
  return e;
}

int cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) return 256;
  return n;
}

// Default column-tile variant for 2F real columns: 32 columns when they
// cover them, else 64.  The 128-column FP32 tiles hold twice the
// accumulators (two work groups per CU instead of three) and pad 2F further;
// at TCo1279 x 411 they measured 8% (synthesis) and 22% (analysis) slower.
// sht_plan_set_tile and the batch autotuner can still choose them.
int default_variant(int prec, int F) {
  const int cols = 2 * F;
  if (prec == SHT_BF16X3) return TILE_C128;  // wide tiles: 6.7 / 6.9 against 9.6 / 10.8 ms at TCo1279 x 411
  if (cols <= 32) return TILE_C32;
  return TILE_C64;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Tables of one chunk of wavenumbers in a table-free plan (bytes).
constexpr int64_t kChunkTableBytes = (int64_t)256 << 20;

}  // namespace

int shtmi::hip_status(hipError_t e) {
  (void)hipGetLastError();
  return hip_fail(e);
}

// Device tables of a (truncation, grid, precision): geometry metadata,
// latitudes and weights, Pbar tables, FFT tables.  Shared by every plan made
// from the same base plan; freed with the last of them.
// The arenas are stream-ordered allocations (hipMallocAsync on the creating
// stream), so that they can also be released in stream order
// (sht_plan_destroy_async) without waiting for the whole device.
struct SharedTables {
  void* arena = nullptr;
  size_t bytes = 0;
  bool async = false;         // release in stream order on `release`
  hipStream_t release = nullptr;
  ~SharedTables() {
    if (!arena) return;
    if (async) {
      (void)hipFreeAsync(arena, release);
    } else {
      (void)hipDeviceSynchronize();
      (void)hipFreeAsync(arena, nullptr);
      (void)hipStreamSynchronize(nullptr);
    }
  }
};

struct sht_plan_s {
  // N: truncation (fixes the grid and the per-ring Fourier truncation).
  // ndeg: highest degree of the tables and of the internal spectral layout
  // (N, or N + 1 for vector plans, whose wind coefficients reach N + 1).
  // F: fields the kernels transform (2 Fv components for vector plans).
  int N = 0, grid = 0, F = 0, prec = 0, nlat = 0, nh = 0, Fp = 0;
  int vec = 0, ndeg = 0, Fv = 0;
  int64_t npts = 0, nspec = 0, nfour = 0;
  int64_t nspec_d = 0;  // internal spectral layout (degree ndeg)
  int elem = 8;
  int variant = TILE_C128;
  std::vector<RingInfo> rings;
  std::vector<FftClass> classes;
  std::vector<MInfo> ms;
  std::vector<int64_t> ring_off, four_row;
  std::vector<WorkItem> inv_items, dir_items;
  std::vector<FftItem> syn_items, ana_items;  // work groups, tier by tier
  int syn_off[FFT_TIERS + 1] = {}, ana_off[FFT_TIERS + 1] = {};  // first work group of each tier
  int64_t tab_plane = 0;
  size_t tab_bytes = 0, fft_bytes = 0;
  size_t inv_cap = 0, dir_cap = 0;  // work items the arena holds
  int64_t ncoef = 0;                 // (a_n, e_n) pairs of the recurrence
  // table-free plans: no resident Pbar tables; the wavenumbers are cut into
  // chunks [chunk_m[c], chunk_m[c + 1]) whose tables (at most chunk_bytes,
  // offsets relative to the chunk) are made in the workspace right before
  // each chunk's product; inv_off / dir_off index each chunk's work items
  int notab = 0;
  int64_t chunk_limit = 0;  // requested bytes per chunk
  std::vector<int> chunk_m;
  std::vector<int> inv_off, dir_off;
  size_t chunk_bytes = 0;
  double* d_sect = nullptr;
  double2* d_coef = nullptr;
  size_t lds_syn = 0, lds_ana = 0;            // largest of the tiers'
  size_t lds_syn_t[FFT_TIERS] = {}, lds_ana_t[FFT_TIERS] = {};
  int max_Lp = 0;
  // device: shared tables, and this plan's own arena (descriptor, work lists)
  std::shared_ptr<SharedTables> tables;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  DevPlan dp{};
  DevPlan* d_self = nullptr;
  WorkItem* d_inv = nullptr;
  WorkItem* d_dir = nullptr;
  FftItem* d_syn = nullptr;
  FftItem* d_ana = nullptr;
  MInfo* d_ms = nullptr;
  FftClass* d_cls = nullptr;
  // vector plans: the H = (1 - mu^2) dPbar/dmu table of degree <= N (planes
  // by the parity of H: odd n - m in plane 0), its per-m layout, and the
  // descriptor the analysis product takes to run over it
  std::vector<MInfo> hms;
  int64_t htab_plane = 0;
  size_t htab_bytes = 0;
  MInfo* d_hms = nullptr;
  DevPlan dph{};
  DevPlan* d_self_h = nullptr;
};

namespace {

// Legendre work items of one plan for a tile variant, tagged with `plan`.
void legendre_items_raw(const sht_plan_s* p, int variant, int plan, std::vector<WorkItem>* inv,
                        std::vector<WorkItem>* dir) {
  int ir, ic, dr, dc;
  legendre_tiles(p->prec, variant, &ir, &ic, &dr, &dc);
  const int twoF = 2 * p->F;
  const size_t ncol_i = (size_t)(twoF + ic - 1) / ic, ncol_d = (size_t)(twoF + dc - 1) / dc;
  size_t ni = 0, nd = 0;
  for (const MInfo& mi : p->ms) {
    if (mi.L == 0) continue;
    ni += (size_t)(mi.L + ir - 1) / ir * ncol_i;
    nd += (size_t)(std::max(mi.K[0], mi.K[1]) + dr - 1) / dr * ncol_d;
  }
  inv->reserve(inv->size() + ni);
  dir->reserve(dir->size() + nd);
  for (const MInfo& mi : p->ms) {
    if (mi.L == 0) continue;
    for (int t0 = 0; t0 < mi.L; t0 += ir)
      for (int c0 = 0; c0 < twoF; c0 += ic) inv->push_back(WorkItem{mi.m, t0, c0, plan});
    const int kmax = std::max(mi.K[0], mi.K[1]);
    for (int t0 = 0; t0 < kmax; t0 += dr)
      for (int c0 = 0; c0 < twoF; c0 += dc) dir->push_back(WorkItem{mi.m, t0, c0, plan});
  }
}

// Work groups go to the XCDs round-robin by id.
constexpr int NUM_XCD = 8;

// A work list with every tile of a wavenumber on one XCD: each operand
// slice of (plan, m) (table rows or columns, spectral or Fourier columns)
// is shared by the tiles of the other dimension, and with all of them on
// one XCD both slices come through its L2 once (spreading them over the
// XCDs read the spectral and Fourier slices from memory once per tile of
// the other dimension).  Wavenumbers go to the XCD with the least work so
// far (items arrive costliest first; the work of an item is `steps(item)`),
// and the XCD queues are interleaved by id, with empty slots (m = -1) where
// a queue has run out.  Input: the items of one (plan, m) consecutive.
template <typename Steps>
void legendre_arrange(std::vector<WorkItem>* items, Steps steps) {
  std::vector<WorkItem> in;
  in.swap(*items);
  std::vector<WorkItem> q[NUM_XCD];
  for (auto& v : q) v.reserve(in.size() / NUM_XCD + 64);
  double load[NUM_XCD] = {0};
  size_t i = 0;
  while (i < in.size()) {
    size_t j = i;
    while (j < in.size() && in[j].m == in[i].m && in[j].plan == in[i].plan) ++j;
    const int x = (int)(std::min_element(load, load + NUM_XCD) - load);
    load[x] += (double)(j - i) * steps(in[i]);
    q[x].insert(q[x].end(), in.begin() + i, in.begin() + j);
    i = j;
  }
  size_t most = 0;
  for (const auto& v : q) most = std::max(most, v.size());
  items->reserve(most * NUM_XCD);
  for (size_t r = 0; r < most; ++r)
    for (int x = 0; x < NUM_XCD; ++x) items->push_back(r < q[x].size() ? q[x][r] : WorkItem{-1, 0, 0, 0});
}

// Arranged work lists of one plan.  For a table-free plan the lists are the
// chunks' lists back to back; inv_off / dir_off (if given) receive where
// each chunk's items start (nchunks + 1 entries).
void legendre_items(const sht_plan_s* p, int variant, int plan, std::vector<WorkItem>* inv,
                    std::vector<WorkItem>* dir, std::vector<int>* inv_off = nullptr,
                    std::vector<int>* dir_off = nullptr) {
  auto steps_inv = [&](const WorkItem& w) { return (double)std::max(p->ms[w.m].Kp[0], p->ms[w.m].Kp[1]) + 8.0; };
  auto steps_dir = [&](const WorkItem& w) { return (double)p->ms[w.m].Lp + 8.0; };
  if (!p->notab) {
    legendre_items_raw(p, variant, plan, inv, dir);
    // synthesis tiles step through k, analysis tiles through the rings
    legendre_arrange(inv, steps_inv);
    legendre_arrange(dir, steps_dir);
    return;
  }
  if (inv_off) inv_off->assign(1, 0);
  if (dir_off) dir_off->assign(1, 0);
  for (size_t c = 0; c + 1 < p->chunk_m.size(); ++c) {
    sht_plan_s part;  // the chunk's wavenumbers
    part.prec = p->prec;
    part.F = p->F;
    part.ms.assign(p->ms.begin() + p->chunk_m[c], p->ms.begin() + p->chunk_m[c + 1]);
    std::vector<WorkItem> a, b;
    legendre_items_raw(&part, variant, plan, &a, &b);
    legendre_arrange(&a, steps_inv);
    legendre_arrange(&b, steps_dir);
    inv->insert(inv->end(), a.begin(), a.end());
    dir->insert(dir->end(), b.begin(), b.end());
    if (inv_off) inv_off->push_back((int)inv->size());
    if (dir_off) dir_off->push_back((int)dir->size());
  }
}

// FFT work items (chunks of up to FFT_FCHUNK fields) of one plan, longest
// transforms first, into the lists of their classes' tiers.
void fft_items(const sht_plan_s* p, int plan, std::vector<FftItem>* syn, std::vector<FftItem>* ana) {
  std::vector<int> order(p->nlat);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return p->classes[p->rings[a].cls].L > p->classes[p->rings[b].cls].L;
  });
  for (int j : order)
    for (int f0 = 0; f0 < p->F; f0 += FFT_FCHUNK) {
      const int fend = std::min(f0 + FFT_FCHUNK, p->F);
      const int t = p->classes[p->rings[j].cls].tier;
      syn[t].push_back(FftItem{j, f0, plan, fend, p->rings[j].cls});
      if (j < p->nh) ana[t].push_back(FftItem{j, f0, plan, fend, p->rings[j].cls});
    }
}

// Work-group list from a list of chunks (items of up to FFT_FCHUNK fields,
// in launch order): a chunk of a class with G fields per work group becomes
// ceil(n / G) work groups.  Work groups go to the XCDs round-robin by id, so
// the groups of one chunk are given ids congruent modulo NUM_XCD, 8 chunks
// side by side (empty slots where a chunk has fewer groups than the others
// of its eight): they run on one XCD at the same time, and their strided
// reads and writes of the chunk's Fourier rows (fields are the innermost
// index) meet in that XCD's L2.  The groups are appended to *items.
void fft_arrange(const sht_plan_t* plans, const std::vector<FftItem>& chunks, std::vector<FftItem>* items) {
  // work groups per chunk, and the list's length (8 chunks side by side,
  // each group of them as long as its longest)
  std::vector<int> ng(chunks.size());
  size_t total = 0;
  for (size_t c0 = 0; c0 < chunks.size(); c0 += NUM_XCD) {
    int most = 0;
    for (size_t k = c0; k < std::min(chunks.size(), c0 + NUM_XCD); ++k) {
      const FftItem& c = chunks[k];
      const int G = plans[c.plan]->classes[c.cls].G;
      ng[k] = (c.fend - c.f0 + G - 1) / G;
      most = std::max(most, ng[k]);
    }
    total += (size_t)most * NUM_XCD;
  }
  items->reserve(items->size() + total);
  for (size_t c0 = 0; c0 < chunks.size(); c0 += NUM_XCD) {
    const int nc = (int)std::min<size_t>(NUM_XCD, chunks.size() - c0);
    int most = 0;
    for (int k = 0; k < nc; ++k) most = std::max(most, ng[c0 + k]);
    for (int j = 0; j < most; ++j)
      for (int k = 0; k < NUM_XCD; ++k) {
        if (k < nc && j < ng[c0 + k]) {
          const FftItem& c = chunks[c0 + k];
          const int G = plans[c.plan]->classes[c.cls].G;
          const int f0 = c.f0 + j * G;
          items->push_back(FftItem{c.ring, f0, c.plan, std::min(f0 + G, c.fend), c.cls});
        } else {
          items->push_back(FftItem{-1, 0, 0, 0, 0});
        }
      }
  }
}

// Work-group size and fields per work group of each FFT class.  An even
// tier (FFT_THREADS_SMALL threads) where that many threads per field reach
// the pass count FFT_THREADS threads do, and one field's LDS leaves the small
// groups' occupancy at what their registers allow (a launch's LDS per group
// is its largest item's); tiers 2 and 3 for the classes whose first radix is
// a prime above FFT_BIG_PRIME.  G: the most fields (up to
// FFT_MAX_G) whose threads per field (the tier's work-group size / G) still
// hold every pass with the same pass count and whose LDS fits the tier's
// budget, the most LDS that keeps the occupancy the tier's longest class has
// with G = 1, and whose fields' rings lie within 2^31 bytes of the first
// one's (the analysis reads them through one descriptor with 32-bit
// offsets: (G - 1) npts + 2h grid values).  The classes come in with the
// radices for FFT_THREADS threads per field.
void choose_groups(int prec, int64_t npts, std::vector<FftClass>* cls) {
  auto lds = [&](const FftClass& c, int G) { return fft_lds_bytes(prec, c.L, G); };
  for (FftClass& c : *cls) {
    // a prime radix above FFT_BIG_PRIME is always the first pass
    const int big = c.rad[0] > FFT_BIG_PRIME ? 2 : 0;
    const int full = fft_blocks_per_cu(prec, big, 0);
    const std::vector<int> rs = radices(c.L, FFT_THREADS_SMALL, c.bluestein);
    const bool small = !rs.empty() && (int)rs.size() == c.nrad && fft_blocks_per_cu(prec, big, lds(c, 1)) >= full;
    c.tier = big + (small ? 0 : 1);
    if (small)
      for (size_t q = 0; q < rs.size(); ++q) c.rad[q] = rs[q];
  }
  size_t budget[FFT_TIERS];
  for (int t = 0; t < FFT_TIERS; ++t) {
    size_t need1 = 0;
    for (const FftClass& c : *cls)
      if (c.tier == t) need1 = std::max(need1, lds(c, 1));
    budget[t] = need1;
    if (need1 == 0) continue;
    const int occ = fft_blocks_per_cu(prec, t, need1);
    for (size_t b = need1 + 1024; b <= 160 * 1024; b += 1024) {
      if (fft_blocks_per_cu(prec, t, b) < occ) break;
      budget[t] = b;
    }
  }
  for (FftClass& c : *cls) {
    const int threads = fft_tier_threads(c.tier);
    int gs = 0;
    std::vector<int> best(c.rad, c.rad + c.nrad);
    for (int s = 0; (2 << s) <= FFT_MAX_G; ++s) {
      const int G = 2 << s;
      const std::vector<int> rad = radices(c.L, threads / G, c.bluestein);
      if (rad.empty() || rad.size() > (size_t)c.nrad) break;
      if (lds(c, G) > budget[c.tier]) break;
      const int64_t elem = prec == SHT_FP64 ? 8 : 4;
      if (((int64_t)(G - 1) * npts + 2 * (int64_t)c.h) * elem >= ((int64_t)1 << 31)) break;
      gs = s + 1;
      best = rad;
    }
    c.G = 1 << gs;
    c.gshift = gs;
    for (size_t q = 0; q < best.size(); ++q) c.rad[q] = best[q];
  }
}

// The launches of an FFT stage, one per tier, over a work list whose
// work groups off[t] <= i < off[t + 1] belong to tier t, one work group per
// list entry (a launch with none is skipped).
hipError_t fft_launch_tiers(bool synthesis, const DevPlan* plans, int prec, const FftItem* items, const int* off,
                            const IoBind* io, IoBind io0, const size_t* lds, hipStream_t s) {
  for (int t = 0; t < FFT_TIERS; ++t) {
    const int first = off[t], count = off[t + 1] - off[t];
    const hipError_t e =
        synthesis ? launch_fourier_synthesis(plans, prec, t, items + first, count, io, io0, lds[t],
                                             (int)fft_grid_blocks(count), s)
                  : launch_fourier_analysis(plans, prec, t, items + first, count, io, io0, lds[t],
                                            (int)fft_grid_blocks(count), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One launch list from per-tier chunk lists (each in launch order): each
// tier's chunks become its work groups, tier by tier; off[t] is the first
// work group of tier t, off[FFT_TIERS] the total.
void fft_join(const sht_plan_t* plans, std::vector<FftItem>* tiers, std::vector<FftItem>* out, int* off) {
  out->clear();
  for (int t = 0; t < FFT_TIERS; ++t) {
    off[t] = (int)out->size();
    fft_arrange(plans, tiers[t], out);
  }
  off[FFT_TIERS] = (int)out->size();
}

// The FFT sweeps address one ring's Fourier rows (both analysis slots, all
// fields of the row) with 32-bit byte offsets.
bool fourier_offsets_fit(const sht_plan_s* p) {
  const int64_t csize = (p->prec == SHT_FP64) ? 16 : 8;
  int mm = 0;
  for (const RingInfo& r : p->rings) mm = std::max(mm, r.mmax);
  return 2 * ((int64_t)mm + 1) * p->Fp * csize < ((int64_t)1 << 31);
}

// The FFT classes of the distinct half lengths hs (sorted) of a grid with
// npts points: transform length and radix plan, table offsets, tier, fields
// per work group and packed radices; *fft_bytes receives the size of their
// tables.
int make_fft_classes(int prec, int64_t npts, const std::vector<int>& hs, std::vector<FftClass>* classes,
                     size_t* fft_bytes) {
  const int csize = (prec == SHT_FP64) ? 16 : 8;
  classes->clear();
  int64_t off = 0;
  for (int h : hs) {
    FftClass c{};
    c.h = h;
    if (radix_smooth(h, prec) && !radices(h).empty()) {
      c.L = h;
      c.bluestein = 0;
    } else {
      c.L = bluestein_length(h);
      c.bluestein = 1;
    }
    std::vector<int> rad = c.L > 0 ? radices(c.L, FFT_THREADS, c.bluestein) : std::vector<int>();
    // a chirp-z transform fuses its middle passes, which takes two passes
    if (rad.empty() || (int)rad.size() > FFT_MAX_RADICES || (c.bluestein && rad.size() < 2)) return SHT_EUNSUPPORTED;
    c.nrad = (int)rad.size();
    for (size_t q = 0; q < rad.size(); ++q) c.rad[q] = rad[q];
    c.root_off = off;
    off += c.L;
    c.post_off = off;
    off += h;
    if (c.bluestein) {
      c.chirp_off = off;
      off += h;
      c.khat_off = off;
      off += c.L;
    }
    classes->push_back(c);
  }
  *fft_bytes = (size_t)off * csize;
  choose_groups(prec, npts, classes);
  for (FftClass& c : *classes) {
    if (c.nrad > FFT_PACK_RADICES) return SHT_EUNSUPPORTED;
    c.radpack = 0;
    for (int q = 0; q < c.nrad; ++q) c.radpack |= (uint64_t)c.rad[q] << (6 * q);
  }
  return SHT_OK;
}

// Class lists by (device, grid, truncation, precision), kept for the life of
// the process: the chirp-z length search, the radix plans and the group
// choice take ~16 ms of host time at TCo1279, and a served truncation's
// tables are made again after every eviction.
std::mutex g_cls_mu;
std::map<std::array<int, 4>, std::pair<std::vector<FftClass>, size_t>> g_cls_cache;

int build_host(sht_plan_s* p) {
  const int N = p->N;
  // ---- geometry ----
  std::vector<int> nlon;
  if (p->grid == SHT_GRID_FULL) {
    if (N % 2 == 0) return SHT_EUNSUPPORTED;  // odd nlat: no mirror for the equator ring
    p->nlat = N + 1;
    nlon.assign(p->nlat, 2 * N + 2);
  } else {
    p->nlat = 2 * (N + 1);
    nlon.resize(p->nlat);
    for (int i = 0; i <= N; ++i) nlon[i] = nlon[p->nlat - 1 - i] = 20 + 4 * i;
  }
  p->nh = p->nlat / 2;
  p->Fp = (int)round_up(p->F, FPAD);
  const int D = p->ndeg;
  p->nspec = (int64_t)(N + 1) * (N + 2) / 2;
  p->nspec_d = (int64_t)(D + 1) * (D + 2) / 2;
  p->rings.resize(p->nlat);
  p->ring_off.assign(p->nlat + 1, 0);
  p->four_row.assign(p->nlat + 1, 0);
  for (int j = 0; j < p->nlat; ++j) {
    RingInfo& r = p->rings[j];
    r.nlon = nlon[j];
    r.mmax = std::min(N, (nlon[j] - 1) / 2);
    r.mirror = p->nlat - 1 - j;
    r.goff = p->ring_off[j];
    r.frow = p->four_row[j];
    p->ring_off[j + 1] = p->ring_off[j] + r.nlon;
    p->four_row[j + 1] = p->four_row[j] + r.mmax + 1;
  }
  p->npts = p->ring_off[p->nlat];
  p->nfour = p->four_row[p->nlat];
  if (!fourier_offsets_fit(p)) return SHT_EUNSUPPORTED;

  // ---- FFT classes (one per distinct half length) ----
  std::vector<int> hs;
  for (auto& r : p->rings) hs.push_back(r.nlon / 2);
  std::sort(hs.begin(), hs.end());
  hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    // bf16x3 plans transform in FP32: the same classes as FP32 plans
    const std::array<int, 4> key{dev, p->grid, N, p->prec == SHT_FP64 ? SHT_FP64 : SHT_FP32};
    bool hit = false;
    {
      std::lock_guard<std::mutex> lk(g_cls_mu);
      auto it = g_cls_cache.find(key);
      if (it != g_cls_cache.end()) {
        p->classes = it->second.first;
        p->fft_bytes = it->second.second;
        hit = true;
      }
    }
    if (!hit) {
      const int rc = make_fft_classes(p->prec, p->npts, hs, &p->classes, &p->fft_bytes);
      if (rc != SHT_OK) return rc;
      std::lock_guard<std::mutex> lk(g_cls_mu);
      g_cls_cache.emplace(key, std::make_pair(p->classes, p->fft_bytes));
    }
  }
  for (auto& r : p->rings) {
    const int h = r.nlon / 2;
    r.cls = (int)(std::lower_bound(hs.begin(), hs.end(), h) - hs.begin());
    const FftClass& c = p->classes[r.cls];
    size_t& ls = p->lds_syn_t[c.tier];
    size_t& la = p->lds_ana_t[c.tier];
    ls = std::max(ls, fft_lds_bytes(p->prec, c.L, c.G));
    la = std::max(la, fft_lds_bytes(p->prec, c.L, c.G));
    p->lds_syn = std::max(p->lds_syn, ls);
    p->lds_ana = std::max(p->lds_ana, la);
  }
  if (p->lds_ana > 160 * 1024) return SHT_EUNSUPPORTED;

  // ---- Legendre tables: per m, rings carrying m and the two parity tables ----
  int64_t toff = 0;
  for (int m = 0; m <= N; ++m) {
    MInfo mi{};
    mi.m = m;
    int first = p->nh;
    for (int j = 0; j < p->nh; ++j)
      if (p->rings[j].mmax >= m) {
        first = j;
        break;
      }
    for (int j = first; j < p->nh; ++j)
      if (p->rings[j].mmax < m) return SHT_EUNSUPPORTED;  // rings carrying m must be contiguous
    mi.first_ring = first;
    mi.L = p->nh - first;
    mi.Lp = (int)round_up(mi.L, ROWPAD);
    mi.K[0] = (D - m) / 2 + 1;
    mi.K[1] = (D - m + 1) / 2;
    mi.Kp[0] = (int)round_up(mi.K[0], KCH);
    mi.Kp[1] = (int)round_up(mi.K[1], KCH);
    mi.toff[0] = toff;
    mi.toff[1] = toff + (int64_t)mi.Kp[0] * mi.Lp;
    toff = mi.toff[1] + (int64_t)mi.Kp[1] * mi.Lp;
    mi.spec_off = (int64_t)m * (2 * D + 3 - m) / 2;
    mi.coff = p->ncoef;
    p->ncoef += pbar_coef_count(D, m);
    p->max_Lp = std::max(p->max_Lp, mi.Lp);
    p->ms.push_back(mi);
  }
  p->tab_plane = toff;
  const int tab_elem = (p->prec == SHT_FP64) ? 8 : 4;  // BF16 split: two 2-byte planes
  p->tab_bytes = (size_t)toff * tab_elem;
  if (p->notab) {
    // chunks of consecutive wavenumbers whose tables fit kChunkTableBytes
    // (or one wavenumber, if a single one is larger), offsets per chunk
    p->chunk_m.assign(1, 0);
    int64_t used = 0, most = 0;
    for (MInfo& mi : p->ms) {
      const int64_t need = ((int64_t)mi.Kp[0] + mi.Kp[1]) * mi.Lp;
      if (used > 0 && (used + need) * tab_elem > p->chunk_limit) {
        p->chunk_m.push_back(mi.m);
        used = 0;
      }
      mi.toff[0] = used;
      mi.toff[1] = used + (int64_t)mi.Kp[0] * mi.Lp;
      used += need;
      most = std::max(most, used);
    }
    p->chunk_m.push_back(N + 1);
    p->tab_plane = most;  // the BF16 lo plane starts here in the chunk scratch
    p->chunk_bytes = (size_t)most * tab_elem;
    p->tab_bytes = 0;
  }
  if (p->vec) {
    // H table: degrees m..N; plane 0 odd n - m, plane 1 even n - m.  Its
    // products write degree n at spec_off + parity + 2k of the wind layout
    // (degree N + 1), i.e. n - 1 (odd) or n + 1 (even), inside m's block.
    int64_t hoff = 0;
    for (const MInfo& mi : p->ms) {
      MInfo hi = mi;
      hi.K[0] = (N - mi.m + 1) / 2;
      hi.K[1] = (N - mi.m) / 2 + 1;
      hi.Kp[0] = (int)round_up(hi.K[0], KCH);
      hi.Kp[1] = (int)round_up(hi.K[1], KCH);
      hi.toff[0] = hoff;
      hi.toff[1] = hoff + (int64_t)hi.Kp[0] * hi.Lp;
      hoff = hi.toff[1] + (int64_t)hi.Kp[1] * hi.Lp;
      p->hms.push_back(hi);
    }
    p->htab_plane = hoff;
    p->htab_bytes = (size_t)hoff * tab_elem;
  }

  // ---- work lists (m ascending = cost descending for both products) ----
  p->variant = default_variant(p->prec, p->F);
  legendre_items(p, p->variant, 0, &p->inv_items, &p->dir_items, &p->inv_off, &p->dir_off);
  {
    std::vector<FftItem> st[FFT_TIERS], at[FFT_TIERS];
    fft_items(p, 0, st, at);
    fft_join(&p, st, &p->syn_items, p->syn_off);
    fft_join(&p, at, &p->ana_items, p->ana_off);
  }
  return SHT_OK;
}

// The plan's own arena: its descriptor and work lists (tables already set).
// The Legendre lists get room for the variant in use; sht_plan_set_tile
// makes a new arena when another variant needs more.
int build_own(sht_plan_s* p, hipStream_t s) {
  const size_t inv_cap = p->inv_items.size(), dir_cap = p->dir_items.size();
  p->inv_cap = inv_cap;
  p->dir_cap = dir_cap;
  const size_t parts[6] = {sizeof(DevPlan), sizeof(WorkItem) * inv_cap, sizeof(WorkItem) * dir_cap,
                           sizeof(FftItem) * p->syn_items.size(), sizeof(FftItem) * p->ana_items.size(),
                           p->vec ? sizeof(DevPlan) : 0};
  size_t total = 0;
  for (size_t q : parts) total += align256(q);
  if (hipMallocAsync(&p->arena, total, s) != hipSuccess) {
    (void)hipGetLastError();
    p->arena = nullptr;
    return SHT_ENOMEM;
  }
  p->arena_bytes = total;
  char* o = (char*)p->arena;
  void* ptr[6];
  for (int i = 0; i < 6; ++i) {
    ptr[i] = o;
    o += align256(parts[i]);
  }
  p->d_self = (DevPlan*)ptr[0];
  p->d_inv = (WorkItem*)ptr[1];
  p->d_dir = (WorkItem*)ptr[2];
  p->d_syn = (FftItem*)ptr[3];
  p->d_ana = (FftItem*)ptr[4];
  p->d_self_h = p->vec ? (DevPlan*)ptr[5] : nullptr;
  HIP_TRY(hipMemcpyAsync(p->d_self, &p->dp, sizeof(DevPlan), hipMemcpyHostToDevice, s));
  if (p->vec) HIP_TRY(hipMemcpyAsync(p->d_self_h, &p->dph, sizeof(DevPlan), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_inv, p->inv_items.data(), sizeof(WorkItem) * p->inv_items.size(), hipMemcpyHostToDevice,
                         s));
  HIP_TRY(hipMemcpyAsync(p->d_dir, p->dir_items.data(), sizeof(WorkItem) * p->dir_items.size(), hipMemcpyHostToDevice,
                         s));
  HIP_TRY(hipMemcpyAsync(p->d_syn, p->syn_items.data(), parts[3], hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_ana, p->ana_items.data(), parts[4], hipMemcpyHostToDevice, s));
  return SHT_OK;
}

int build_device(sht_plan_s* p, hipStream_t s) {
  void *v_rings, *v_cls, *v_ms, *v_mu, *v_w, *v_tab, *v_fft, *v_wa, *v_hms, *v_htab, *v_sect, *v_coef;
  struct Part {
    void** dst;
    size_t bytes;
  };
  const Part parts[] = {
      {&v_rings, sizeof(RingInfo) * p->rings.size()},
      {&v_cls, sizeof(FftClass) * p->classes.size()},
      {&v_ms, sizeof(MInfo) * p->ms.size()},
      {&v_mu, sizeof(double) * p->nlat},
      {&v_w, sizeof(double) * p->nlat},
      {&v_tab, p->tab_bytes},
      {&v_fft, p->fft_bytes},
      {&v_wa, p->vec ? sizeof(double) * p->nlat : 0},
      {&v_hms, sizeof(MInfo) * p->hms.size()},
      {&v_htab, p->htab_bytes},
      {&v_sect, sizeof(double) * (p->ndeg + 1)},
      {&v_coef, sizeof(double2) * p->ncoef},
  };
  size_t total = 0;
  for (const Part& q : parts) total += align256(q.bytes);
  p->tables = std::make_shared<SharedTables>();
  if (hipMallocAsync(&p->tables->arena, total, s) != hipSuccess) {
    (void)hipGetLastError();
    p->tables->arena = nullptr;
    return SHT_ENOMEM;
  }
  p->tables->bytes = total;
  size_t o = 0;
  for (const Part& q : parts) {
    *q.dst = (char*)p->tables->arena + o;
    o += align256(q.bytes);
  }
  DevPlan& d = p->dp;
  d.N = p->ndeg;
  d.nlat = p->nlat;
  d.nh = p->nh;
  d.F = p->F;
  d.Fp = p->Fp;
  d.npts = p->npts;
  d.nspec = p->nspec_d;
  d.rings = (const RingInfo*)v_rings;
  d.classes = (const FftClass*)v_cls;
  d.ms = (const MInfo*)v_ms;
  d.mu = (const double*)v_mu;
  d.w = (const double*)v_w;
  d.wa = p->vec ? (const double*)v_wa : (const double*)v_w;
  d.tab = v_tab;
  d.fft = v_fft;
  d.tab_plane = p->tab_plane;
  p->d_ms = (MInfo*)v_ms;
  p->d_cls = (FftClass*)v_cls;
  if (p->vec) {
    p->d_hms = (MInfo*)v_hms;
    p->dph = d;
    p->dph.ms = (const MInfo*)v_hms;
    p->dph.tab = v_htab;
    p->dph.tab_plane = p->htab_plane;
  }

  HIP_TRY(hipMemcpyAsync(v_rings, p->rings.data(), parts[0].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_cls, p->classes.data(), parts[1].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_ms, p->ms.data(), parts[2].bytes, hipMemcpyHostToDevice, s));
  if (p->vec) HIP_TRY(hipMemcpyAsync(v_hms, p->hms.data(), sizeof(MInfo) * p->hms.size(), hipMemcpyHostToDevice, s));
  int rc = build_own(p, s);
  if (rc != SHT_OK) return rc;

  HIP_TRY(launch_gauss(p->nlat, (double*)v_mu, (double*)v_w, s));
  if (p->vec) HIP_TRY(launch_analysis_weight(p->nlat, (const double*)v_mu, (const double*)v_w, (double*)v_wa, s));
  p->d_sect = (double*)v_sect;
  p->d_coef = (double2*)v_coef;
  HIP_TRY(launch_pbar_coef(p->ndeg, p->d_ms, (int)p->ms.size(), (double*)v_sect, (double2*)v_coef, s));
  if (!p->notab)
    HIP_TRY(launch_pbar_planes(d, p->prec, p->d_ms, (int)p->ms.size(), p->max_Lp, v_tab, p->tab_plane,
                               p->vec ? p->d_hms : nullptr, v_htab, p->htab_plane, p->N, (const double*)v_sect,
                               (const double2*)v_coef, s));
  HIP_TRY(launch_fft_tables(d, p->prec, p->d_cls, (int)p->classes.size(), p->classes.data(), v_fft, s));
  HIP_TRY(ensure_lds(std::max(p->lds_syn, p->lds_ana)));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  return SHT_OK;
}

IoBind bind_of(const void* spec, const void* grid, const void* ws) {
  return IoBind{const_cast<void*>(spec), const_cast<void*>(grid), const_cast<void*>(ws), nullptr};
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

struct sht_batch_s {
  int n = 0, prec = 0, flags = 0;
  std::vector<sht_plan_t> plans;
  std::vector<int> variant;
  std::vector<WorkItem> inv[NUM_TILE_VARIANTS], dir[NUM_TILE_VARIANTS];
  std::vector<FftItem> syn, ana;  // work groups, tier by tier
  int syn_off[FFT_TIERS + 1] = {}, ana_off[FFT_TIERS + 1] = {};
  std::vector<size_t> ws_off;
  size_t ws_bytes = 0;
  size_t lds_syn = 0, lds_ana = 0;
  size_t lds_syn_t[FFT_TIERS] = {}, lds_ana_t[FFT_TIERS] = {};
  std::vector<IoBind> io_host;
  bool bound = false;
  // device
  void* arena = nullptr;
  DevPlan* d_plans = nullptr;
  IoBind* d_io = nullptr;
  WorkItem* d_inv[NUM_TILE_VARIANTS] = {};
  WorkItem* d_dir[NUM_TILE_VARIANTS] = {};
  FftItem* d_syn = nullptr;
  FftItem* d_ana = nullptr;
  int grid_inv[NUM_TILE_VARIANTS] = {}, grid_dir[NUM_TILE_VARIANTS] = {};
  hipGraphExec_t g_inv = nullptr, g_dir = nullptr;
};

namespace {

// Cost model used to order a batch's items (largest first, so that the
// grid-stride assignment ends with short items): K chunks of a synthesis
// tile, rings of an analysis tile, transform length of an FFT item.
int64_t inv_cost(const sht_batch_s* b, const WorkItem& w) {
  const MInfo& mi = b->plans[w.plan]->ms[w.m];
  return (int64_t)std::max(mi.Kp[0], mi.Kp[1]);
}

int64_t dir_cost(const sht_batch_s* b, const WorkItem& w) { return (int64_t)b->plans[w.plan]->ms[w.m].L; }

int64_t fft_cost(const sht_batch_s* b, const FftItem& w) {
  const sht_plan_s* p = b->plans[w.plan];
  return (int64_t)p->classes[p->rings[w.ring].cls].L;
}

// The bound buffers reach the device table through kernel arguments: the
// write is ordered on the caller's stream after the runs enqueued before
// it (a run still in flight keeps the buffers it started with), and no host
// staging buffer has to outlive the call.
constexpr int BIND_CHUNK = 32;
struct BindChunk {
  IoBind io[BIND_CHUNK];
};

__global__ void write_binds_kernel(IoBind* dst, BindChunk c, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = c.io[i];
}

hipError_t write_binds(IoBind* dst, const std::vector<IoBind>& io, hipStream_t s) {
  for (size_t i0 = 0; i0 < io.size(); i0 += BIND_CHUNK) {
    BindChunk c{};
    const int n = (int)std::min<size_t>(BIND_CHUNK, io.size() - i0);
    for (int k = 0; k < n; ++k) c.io[k] = io[i0 + k];
    hipLaunchKernelGGL(write_binds_kernel, dim3(1), dim3(BIND_CHUNK), 0, s, dst + i0, c, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void destroy_graphs(sht_batch_s* b) {
  if (b->g_inv) (void)hipGraphExecDestroy(b->g_inv);
  if (b->g_dir) (void)hipGraphExecDestroy(b->g_dir);
  b->g_inv = b->g_dir = nullptr;
}

// (Re)build the batch's work lists from the per-plan variants and upload them.
int batch_upload(sht_batch_s* b, hipStream_t s) {
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v) {
    b->inv[v].clear();
    b->dir[v].clear();
  }
  std::vector<FftItem> st[FFT_TIERS], at[FFT_TIERS];
  for (int i = 0; i < b->n; ++i) {
    legendre_items_raw(b->plans[i], b->variant[i], i, &b->inv[b->variant[i]], &b->dir[b->variant[i]]);
    fft_items(b->plans[i], i, st, at);
  }
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v) {
    std::stable_sort(b->inv[v].begin(), b->inv[v].end(),
                     [&](const WorkItem& x, const WorkItem& y) { return inv_cost(b, x) > inv_cost(b, y); });
    std::stable_sort(b->dir[v].begin(), b->dir[v].end(),
                     [&](const WorkItem& x, const WorkItem& y) { return dir_cost(b, x) > dir_cost(b, y); });
    legendre_arrange(&b->inv[v], [&](const WorkItem& w) { return (double)inv_cost(b, w) + 8.0; });
    legendre_arrange(&b->dir[v], [&](const WorkItem& w) {
      return (double)b->plans[w.plan]->ms[w.m].Lp + 8.0;
    });
  }
  for (int t = 0; t < FFT_TIERS; ++t) {
    std::stable_sort(st[t].begin(), st[t].end(),
                     [&](const FftItem& x, const FftItem& y) { return fft_cost(b, x) > fft_cost(b, y); });
    std::stable_sort(at[t].begin(), at[t].end(),
                     [&](const FftItem& x, const FftItem& y) { return fft_cost(b, x) > fft_cost(b, y); });
  }
  fft_join(b->plans.data(), st, &b->syn, b->syn_off);
  fft_join(b->plans.data(), at, &b->ana, b->ana_off);

  destroy_graphs(b);
  if (b->arena) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(b->arena));
    b->arena = nullptr;
  }
  size_t total = align256(sizeof(DevPlan) * b->n) + align256(sizeof(IoBind) * b->n);
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v)
    total += align256(sizeof(WorkItem) * b->inv[v].size()) + align256(sizeof(WorkItem) * b->dir[v].size());
  total += align256(sizeof(FftItem) * b->syn.size()) + align256(sizeof(FftItem) * b->ana.size());
  if (hipMalloc(&b->arena, total) != hipSuccess) {
    (void)hipGetLastError();
    b->arena = nullptr;
    return SHT_ENOMEM;
  }
  char* o = (char*)b->arena;
  auto take = [&](size_t bytes) {
    char* r = o;
    o += align256(bytes);
    return (void*)r;
  };
  b->d_plans = (DevPlan*)take(sizeof(DevPlan) * b->n);
  b->d_io = (IoBind*)take(sizeof(IoBind) * b->n);
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v) {
    b->d_inv[v] = (WorkItem*)take(sizeof(WorkItem) * b->inv[v].size());
    b->d_dir[v] = (WorkItem*)take(sizeof(WorkItem) * b->dir[v].size());
  }
  b->d_syn = (FftItem*)take(sizeof(FftItem) * b->syn.size());
  b->d_ana = (FftItem*)take(sizeof(FftItem) * b->ana.size());

  std::vector<DevPlan> dps(b->n);
  for (int i = 0; i < b->n; ++i) dps[i] = b->plans[i]->dp;
  HIP_TRY(hipMemcpy(b->d_plans, dps.data(), sizeof(DevPlan) * b->n, hipMemcpyHostToDevice));
  if (b->bound) {
    HIP_TRY(write_binds(b->d_io, b->io_host, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v) {
    if (!b->inv[v].empty())
      HIP_TRY(hipMemcpy(b->d_inv[v], b->inv[v].data(), sizeof(WorkItem) * b->inv[v].size(), hipMemcpyHostToDevice));
    if (!b->dir[v].empty())
      HIP_TRY(hipMemcpy(b->d_dir[v], b->dir[v].data(), sizeof(WorkItem) * b->dir[v].size(), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(b->d_syn, b->syn.data(), sizeof(FftItem) * b->syn.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_ana, b->ana.data(), sizeof(FftItem) * b->ana.size(), hipMemcpyHostToDevice));

  // grid sizes: persistent = as many work groups as can be resident
  const bool persistent = b->flags & SHT_BATCH_PERSISTENT;
  const int cus = cu_count();
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v) {
    const int ni = (int)b->inv[v].size(), nd = (int)b->dir[v].size();
    b->grid_inv[v] = ni;
    b->grid_dir[v] = nd;
    if (persistent && ni) b->grid_inv[v] = std::min(ni, cus * legendre_blocks_per_cu(b->prec, v, true));
    if (persistent && nd) b->grid_dir[v] = std::min(nd, cus * legendre_blocks_per_cu(b->prec, v, false));
  }
  // FFT launches keep one work group per item (fft_launch_tiers): measured
  // on uneven batches, letting the hardware hand out work groups balanced the
  // rings' very different lengths better than a resident grid looping over
  // them.
  return SHT_OK;
}

int batch_enqueue_inverse(sht_batch_s* b, hipStream_t s) {
  const IoBind none{};
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v)
    HIP_TRY(launch_legendre_inverse(b->d_plans, b->prec, v, b->d_inv[v], (int)b->inv[v].size(), b->d_io, none,
                                    b->grid_inv[v], s));
  HIP_TRY(fft_launch_tiers(true, b->d_plans, b->prec, b->d_syn, b->syn_off, b->d_io, none,
                           b->lds_syn_t, s));
  return SHT_OK;
}

int batch_enqueue_direct(sht_batch_s* b, hipStream_t s) {
  const IoBind none{};
  HIP_TRY(fft_launch_tiers(false, b->d_plans, b->prec, b->d_ana, b->ana_off, b->d_io, none,
                           b->lds_ana_t, s));
  for (int v = 0; v < NUM_TILE_VARIANTS; ++v)
    HIP_TRY(launch_legendre_direct(b->d_plans, b->prec, v, b->d_dir[v], (int)b->dir[v].size(), b->d_io, none,
                                   b->grid_dir[v], s));
  return SHT_OK;
}

// Run through a captured graph when the batch asks for one (not on the
// legacy default stream, which cannot be captured).
int batch_run(sht_batch_s* b, hipStream_t s, bool inverse) {
  if (!b->bound) return SHT_EINVAL;
  hipGraphExec_t* exec = inverse ? &b->g_inv : &b->g_dir;
  if (!(b->flags & SHT_BATCH_GRAPH) || s == nullptr)
    return inverse ? batch_enqueue_inverse(b, s) : batch_enqueue_direct(b, s);
  if (!*exec) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = inverse ? batch_enqueue_inverse(b, s) : batch_enqueue_direct(b, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != SHT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e);
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *exec = nullptr;
      return hip_fail(e);
    }
  }
  HIP_TRY(hipGraphLaunch(*exec, s));
  return SHT_OK;
}

}  // namespace

namespace {

// Free a plan's own arena after a failed creation (nothing of it is in use).
void release_own(sht_plan_s* p) {
  if (!p->arena) return;
  (void)hipDeviceSynchronize();
  (void)hipFreeAsync(p->arena, nullptr);
  (void)hipStreamSynchronize(nullptr);
  p->arena = nullptr;
}

int plan_create(sht_plan_t* out, int truncation, int grid, int nfields, int precision, bool vec, void* hip_stream,
                bool notab = false, int64_t chunk_limit = 0) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (vec && notab) return SHT_EUNSUPPORTED;
  if (truncation < 1 || nfields < 1 || nfields > (vec ? (1 << 29) : (1 << 30))) return SHT_EINVAL;
  if (grid != SHT_GRID_FULL && grid != SHT_GRID_OCTAHEDRAL) return SHT_EINVAL;
  if (precision != SHT_FP64 && precision != SHT_FP32 && precision != SHT_BF16X3) return SHT_EINVAL;
  sht_plan_s* p = new (std::nothrow) sht_plan_s();
  if (!p) return SHT_ENOMEM;
  p->N = truncation;
  p->grid = grid;
  p->vec = vec ? 1 : 0;
  p->notab = notab ? 1 : 0;
  p->chunk_limit = chunk_limit > 0 ? chunk_limit : kChunkTableBytes;
  p->ndeg = truncation + (vec ? 1 : 0);
  p->Fv = nfields;
  p->F = vec ? 2 * nfields : nfields;
  p->prec = precision;
  p->elem = (precision == SHT_FP64) ? 8 : 4;
  int rc = build_host(p);
  if (rc == SHT_OK) rc = build_device(p, (hipStream_t)hip_stream);
  if (rc != SHT_OK) {
    release_own(p);
    delete p;  // releases the tables
    return rc;
  }
  *out = p;
  return SHT_OK;
}

}  // namespace

extern "C" {

int sht_plan_create(sht_plan_t* out, int truncation, int grid, int nfields, int precision, void* hip_stream) {
  return plan_create(out, truncation, grid, nfields, precision, false, hip_stream);
}

int sht_plan_create_vector(sht_plan_t* out, int truncation, int grid, int nfields, int precision, void* hip_stream) {
  return plan_create(out, truncation, grid, nfields, precision, true, hip_stream);
}

int sht_plan_create_table_free(sht_plan_t* out, int truncation, int grid, int nfields, int precision,
                               size_t chunk_bytes, void* hip_stream) {
  if (chunk_bytes > ((size_t)1 << 40)) return SHT_EINVAL;
  return plan_create(out, truncation, grid, nfields, precision, false, hip_stream, true, (int64_t)chunk_bytes);
}

int sht_plan_create_like(sht_plan_t* out, sht_plan_t base, int nfields, void* hip_stream) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (!base || nfields < 1) return SHT_EINVAL;
  sht_plan_s* p = new (std::nothrow) sht_plan_s();
  if (!p) return SHT_ENOMEM;
  p->N = base->N;
  p->grid = base->grid;
  p->prec = base->prec;
  p->vec = base->vec;
  p->ndeg = base->ndeg;
  p->nspec_d = base->nspec_d;
  p->hms = base->hms;
  p->notab = base->notab;
  p->chunk_limit = base->chunk_limit;
  p->chunk_m = base->chunk_m;
  p->chunk_bytes = base->chunk_bytes;
  p->d_sect = base->d_sect;
  p->d_coef = base->d_coef;
  p->htab_plane = base->htab_plane;
  p->htab_bytes = base->htab_bytes;
  p->d_hms = base->d_hms;
  p->elem = base->elem;
  p->nlat = base->nlat;
  p->nh = base->nh;
  p->npts = base->npts;
  p->nspec = base->nspec;
  p->nfour = base->nfour;
  p->rings = base->rings;
  p->classes = base->classes;
  p->ms = base->ms;
  p->ring_off = base->ring_off;
  p->four_row = base->four_row;
  p->tab_plane = base->tab_plane;
  p->tab_bytes = base->tab_bytes;
  p->fft_bytes = base->fft_bytes;
  p->lds_syn = base->lds_syn;
  p->lds_ana = base->lds_ana;
  for (int t = 0; t < FFT_TIERS; ++t) {
    p->lds_syn_t[t] = base->lds_syn_t[t];
    p->lds_ana_t[t] = base->lds_ana_t[t];
  }
  p->max_Lp = base->max_Lp;
  p->tables = base->tables;
  p->d_ms = base->d_ms;
  p->d_cls = base->d_cls;
  p->Fv = nfields;
  p->F = p->vec ? 2 * nfields : nfields;
  p->Fp = (int)round_up(p->F, FPAD);
  if (!fourier_offsets_fit(p)) {
    delete p;
    return SHT_EUNSUPPORTED;
  }
  p->dp = base->dp;
  p->dp.F = p->F;
  p->dp.Fp = p->Fp;
  p->dph = base->dph;
  p->dph.F = p->F;
  p->dph.Fp = p->Fp;
  p->variant = default_variant(p->prec, p->F);
  legendre_items(p, p->variant, 0, &p->inv_items, &p->dir_items, &p->inv_off, &p->dir_off);
  {
    std::vector<FftItem> st[FFT_TIERS], at[FFT_TIERS];
    fft_items(p, 0, st, at);
    fft_join(&p, st, &p->syn_items, p->syn_off);
    fft_join(&p, at, &p->ana_items, p->ana_off);
  }
  int rc = build_own(p, (hipStream_t)hip_stream);
  if (rc == SHT_OK) {
    hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  if (rc != SHT_OK) {
    release_own(p);
    delete p;
    return rc;
  }
  *out = p;
  return SHT_OK;
}

int sht_plan_destroy(sht_plan_t p) {
  if (!p) return SHT_EINVAL;
  int rc = SHT_OK;
  if (p->arena) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFreeAsync(p->arena, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  delete p;  // the tables go with the last plan that shares them
  return rc;
}

int sht_plan_destroy_async(sht_plan_t p, void* hip_stream) {
  if (!p) return SHT_EINVAL;
  int rc = SHT_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  if (p->arena) {
    const hipError_t e = hipFreeAsync(p->arena, s);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  if (p->tables) {
    // if this plan holds the last reference, the tables go in stream order too
    p->tables->async = true;
    p->tables->release = s;
  }
  delete p;
  return rc;
}

int sht_plan_info(sht_plan_t p, sht_info* out) {
  if (!p || !out) return SHT_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->truncation = p->N;
  out->grid = p->grid;
  out->nfields = p->Fv;
  out->precision = p->prec;
  out->nlat = p->nlat;
  out->fpad = p->Fp;
  out->npts = p->npts;
  out->nspec = p->nspec;
  out->nfour = p->nfour;
  out->workspace_bytes = (int64_t)sht_workspace_size(p);
  out->table_bytes = (int64_t)(p->tab_bytes + p->htab_bytes);
  out->plan_bytes = (int64_t)p->arena_bytes + (p->tables ? (int64_t)p->tables->bytes : 0);
  out->own_bytes = (int64_t)p->arena_bytes;
  out->elem_bytes = p->elem;
  out->tile = p->variant;
  out->vector = p->vec;
  out->degree = p->ndeg;
  out->table_free = p->notab;
  out->chunk_table_bytes = (int64_t)p->chunk_bytes;
  return SHT_OK;
}

int sht_plan_geometry(sht_plan_t p, double* mu, double* w, int32_t* nlon, int32_t* mmax, int64_t* ring_offset,
                      int64_t* four_row) {
  if (!p) return SHT_EINVAL;
  if (mu) HIP_TRY(hipMemcpy(mu, p->dp.mu, sizeof(double) * p->nlat, hipMemcpyDeviceToHost));
  if (w) HIP_TRY(hipMemcpy(w, p->dp.w, sizeof(double) * p->nlat, hipMemcpyDeviceToHost));
  for (int j = 0; j < p->nlat; ++j) {
    if (nlon) nlon[j] = p->rings[j].nlon;
    if (mmax) mmax[j] = p->rings[j].mmax;
  }
  if (ring_offset) std::copy(p->ring_off.begin(), p->ring_off.end(), ring_offset);
  if (four_row) std::copy(p->four_row.begin(), p->four_row.end(), four_row);
  return SHT_OK;
}

int sht_plan_legendre_table(sht_plan_t p, int m, double* out, int32_t* first_ring) {
  if (!p || m < 0 || m > p->N || p->notab) return SHT_EINVAL;
  const MInfo& mi = p->ms[m];
  if (first_ring) *first_ring = mi.first_ring;
  if (!out) return SHT_OK;
  const size_t n = (size_t)mi.L * (p->ndeg - m + 1);
  if (n == 0) return SHT_OK;
  double* tmp = nullptr;
  HIP_TRY(hipMalloc(&tmp, n * sizeof(double)));
  hipError_t e = launch_table_export_planes(p->dp, p->prec, mi, p->tab_plane, tmp, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, tmp, n * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e);
  return SHT_OK;
}

int sht_plan_set_tile(sht_plan_t p, int tile, void* stream) {
  if (!p || !legendre_variant_supported(p->prec, tile)) return SHT_EINVAL;
  std::vector<WorkItem> inv, dir;
  std::vector<int> inv_off, dir_off;
  legendre_items(p, tile, 0, &inv, &dir, &inv_off, &dir_off);
  const hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s));
  if (inv.size() > p->inv_cap || dir.size() > p->dir_cap) {
    // a new arena with room for these lists (the plan may have run on other
    // streams: wait for the device before the old one goes)
    HIP_TRY(hipDeviceSynchronize());
    sht_plan_s keep;  // what to restore if the new arena cannot be made
    keep.arena = p->arena;
    keep.inv_items.swap(p->inv_items);
    keep.dir_items.swap(p->dir_items);
    keep.variant = p->variant;
    keep.inv_cap = p->inv_cap;
    keep.dir_cap = p->dir_cap;
    keep.d_self = p->d_self;
    keep.d_inv = p->d_inv;
    keep.d_dir = p->d_dir;
    keep.d_syn = p->d_syn;
    keep.d_ana = p->d_ana;
    keep.d_self_h = p->d_self_h;
    void* old = p->arena;
    p->arena = nullptr;
    p->inv_items = inv;
    p->dir_items = dir;
    p->variant = tile;
    std::vector<int> keep_io = p->inv_off, keep_do = p->dir_off;
    p->inv_off = inv_off;
    p->dir_off = dir_off;
    const int rc = build_own(p, s);
    if (rc != SHT_OK) {
      if (p->arena) {
        (void)hipStreamSynchronize(s);
        (void)hipFreeAsync(p->arena, s);
        (void)hipStreamSynchronize(s);
      }
      p->arena = keep.arena;
      p->inv_items.swap(keep.inv_items);
      p->dir_items.swap(keep.dir_items);
      p->variant = keep.variant;
      p->inv_off = keep_io;
      p->dir_off = keep_do;
      p->inv_cap = keep.inv_cap;
      p->dir_cap = keep.dir_cap;
      p->d_self = keep.d_self;
      p->d_inv = keep.d_inv;
      p->d_dir = keep.d_dir;
      p->d_syn = keep.d_syn;
      p->d_ana = keep.d_ana;
      p->d_self_h = keep.d_self_h;
      keep.arena = nullptr;
      return rc;
    }
    keep.arena = nullptr;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFreeAsync(old, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SHT_OK;
  }
  HIP_TRY(hipMemcpy(p->d_inv, inv.data(), sizeof(WorkItem) * inv.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_dir, dir.data(), sizeof(WorkItem) * dir.size(), hipMemcpyHostToDevice));
  p->inv_items = inv;
  p->dir_items = dir;
  p->inv_off = inv_off;
  p->dir_off = dir_off;
  p->variant = tile;
  return SHT_OK;
}

size_t sht_workspace_size(sht_plan_t p) {
  if (!p) return 0;
  const size_t four = (size_t)p->nfour * p->Fp * 2 * p->elem;
  if (p->notab) return align256(four) + p->chunk_bytes;  // the Fourier buffer, then one chunk's tables
  if (!p->vec) return four;
  // vector plans: the Fourier buffer, then two arrays of wind coefficients
  // of degree N + 1 (synthesis input / Pbar projections, and H projections)
  return align256(four) + 2 * align256((size_t)p->F * p->nspec_d * 2 * p->elem);
}

}  // extern "C"

namespace {

// The stages on a plan's internal layouts (degree ndeg, F fields or
// components); the public stage calls add the checks of the scalar layout.
// Table-free plans: each chunk of wavenumbers has its tables made in the
// workspace (after the Fourier buffer), then its product runs on them.
void* chunk_tables(sht_plan_t p, void* ws) { return (char*)ws + align256((size_t)p->nfour * p->Fp * 2 * p->elem); }

hipError_t make_chunk_tables(sht_plan_t p, int c, void* tab, hipStream_t s) {
  const int m0 = p->chunk_m[c], nm = p->chunk_m[c + 1] - m0;
  return launch_pbar_planes(p->dp, p->prec, p->d_ms + m0, nm, p->max_Lp, tab, p->tab_plane, nullptr, nullptr, 0,
                            p->N, p->d_sect, p->d_coef, s);
}

int stage_legendre_inverse(sht_plan_t p, const void* spec, void* four, void* stream) {
  const hipStream_t s = (hipStream_t)stream;
  if (p->notab) {
    void* tab = chunk_tables(p, four);
    IoBind io = bind_of(spec, nullptr, four);
    io.pad = tab;
    for (size_t c = 0; c + 1 < p->chunk_m.size(); ++c) {
      HIP_TRY(make_chunk_tables(p, (int)c, tab, s));
      const int n = p->inv_off[c + 1] - p->inv_off[c];
      HIP_TRY(launch_legendre_inverse(p->d_self, p->prec, p->variant, p->d_inv + p->inv_off[c], n, nullptr, io, n,
                                      s));
    }
    return SHT_OK;
  }
  HIP_TRY(launch_legendre_inverse(p->d_self, p->prec, p->variant, p->d_inv, (int)p->inv_items.size(), nullptr,
                                  bind_of(spec, nullptr, four), (int)p->inv_items.size(), s));
  return SHT_OK;
}

// grid_a != 0: each grid value g is stored as g + grid_a g (1 - g) (the
// grid-point step of a time step, fused into the last pass's stores)
int stage_fourier_synthesis(sht_plan_t p, const void* four, void* grid, void* stream, double grid_a = 0.0) {
  IoBind io = bind_of(nullptr, grid, four);
  io.grid_a = grid_a;
  HIP_TRY(fft_launch_tiers(true, p->d_self, p->prec, p->d_syn, p->syn_off, nullptr, io, p->lds_syn_t,
                           (hipStream_t)stream));
  return SHT_OK;
}

int stage_fourier_analysis(sht_plan_t p, const void* grid, void* four, void* stream) {
  HIP_TRY(fft_launch_tiers(false, p->d_self, p->prec, p->d_ana, p->ana_off, nullptr,
                           bind_of(nullptr, grid, four), p->lds_ana_t, (hipStream_t)stream));
  return SHT_OK;
}

// spec_c != 0: each coefficient is stored divided by 1 + spec_c n (n + 1)
// (the implicit diffusion of a time step, fused into the products' stores)
int stage_legendre_direct(sht_plan_t p, const void* four, void* spec, void* stream, double spec_c = 0.0) {
  const hipStream_t s = (hipStream_t)stream;
  if (p->notab) {
    void* tab = chunk_tables(p, const_cast<void*>(four));
    IoBind io = bind_of(spec, nullptr, four);
    io.pad = tab;
    io.spec_c = spec_c;
    for (size_t c = 0; c + 1 < p->chunk_m.size(); ++c) {
      HIP_TRY(make_chunk_tables(p, (int)c, tab, s));
      const int n = p->dir_off[c + 1] - p->dir_off[c];
      HIP_TRY(launch_legendre_direct(p->d_self, p->prec, p->variant, p->d_dir + p->dir_off[c], n, nullptr, io, n, s));
    }
    return SHT_OK;
  }
  IoBind io = bind_of(spec, nullptr, four);
  io.spec_c = spec_c;
  HIP_TRY(launch_legendre_direct(p->d_self, p->prec, p->variant, p->d_dir, (int)p->dir_items.size(), nullptr, io,
                                 (int)p->dir_items.size(), s));
  return SHT_OK;
}

bool scalar_plan(sht_plan_t p) { return p && !p->vec; }
bool vector_plan(sht_plan_t p) { return p && p->vec; }

// The wind-coefficient arrays of a vector plan's workspace (after the
// Fourier buffer): 0 = synthesis input / Pbar projections, 1 = H projections.
void* wind_spec(sht_plan_t p, void* ws, int which = 0) {
  return (char*)ws + align256((size_t)p->nfour * p->Fp * 2 * p->elem) +
         which * align256((size_t)p->F * p->nspec_d * 2 * p->elem);
}

}  // namespace

extern "C" {

int sht_legendre_inverse(sht_plan_t p, const void* spec, void* four, void* stream) {
  if (!scalar_plan(p) || !spec || !four) return SHT_EINVAL;
  return stage_legendre_inverse(p, spec, four, stream);
}

int sht_fourier_synthesis(sht_plan_t p, const void* four, void* grid, void* stream) {
  if (!scalar_plan(p) || !four || !grid) return SHT_EINVAL;
  return stage_fourier_synthesis(p, four, grid, stream);
}

int sht_fourier_analysis(sht_plan_t p, const void* grid, void* four, void* stream) {
  if (!scalar_plan(p) || !four || !grid) return SHT_EINVAL;
  return stage_fourier_analysis(p, grid, four, stream);
}

int sht_legendre_direct(sht_plan_t p, const void* four, void* spec, void* stream) {
  if (!scalar_plan(p) || !spec || !four) return SHT_EINVAL;
  return stage_legendre_direct(p, four, spec, stream);
}

int sht_inverse(sht_plan_t p, const void* spec, void* grid, void* ws, void* stream) {
  if (!scalar_plan(p) || !spec || !grid || !ws) return SHT_EINVAL;
  int rc = stage_legendre_inverse(p, spec, ws, stream);
  if (rc != SHT_OK) return rc;
  return stage_fourier_synthesis(p, ws, grid, stream);
}

int sht_direct(sht_plan_t p, const void* grid, void* spec, void* ws, void* stream) {
  if (!scalar_plan(p) || !spec || !grid || !ws) return SHT_EINVAL;
  int rc = stage_fourier_analysis(p, grid, ws, stream);
  if (rc != SHT_OK) return rc;
  return stage_legendre_direct(p, ws, spec, stream);
}

int sht_vector_inverse(sht_plan_t p, const void* vortdiv, void* uv, void* ws, void* stream) {
  if (!vector_plan(p) || !vortdiv || !uv || !ws) return SHT_EINVAL;
  void* wind = wind_spec(p, ws);
  HIP_TRY(launch_uv_from_potentials(p->N, p->Fv, false, p->prec, vortdiv, wind, (hipStream_t)stream));
  int rc = stage_legendre_inverse(p, wind, ws, stream);
  if (rc != SHT_OK) return rc;
  return stage_fourier_synthesis(p, ws, uv, stream);
}

int sht_gradient(sht_plan_t p, const void* spec, void* uv, void* ws, void* stream) {
  if (!vector_plan(p) || !spec || !uv || !ws) return SHT_EINVAL;
  void* wind = wind_spec(p, ws);
  HIP_TRY(launch_uv_from_potentials(p->N, p->Fv, true, p->prec, spec, wind, (hipStream_t)stream));
  int rc = stage_legendre_inverse(p, wind, ws, stream);
  if (rc != SHT_OK) return rc;
  return stage_fourier_synthesis(p, ws, uv, stream);
}

int sht_vector_direct(sht_plan_t p, const void* uv, void* vortdiv, void* ws, void* stream) {
  if (!vector_plan(p) || !vortdiv || !uv || !ws) return SHT_EINVAL;
  void* pw = wind_spec(p, ws, 0);
  void* hw = wind_spec(p, ws, 1);
  int rc = stage_fourier_analysis(p, uv, ws, stream);
  if (rc != SHT_OK) return rc;
  rc = stage_legendre_direct(p, ws, pw, stream);
  if (rc != SHT_OK) return rc;
  // the same product over the H table
  HIP_TRY(launch_legendre_direct(p->d_self_h, p->prec, p->variant, p->d_dir, (int)p->dir_items.size(), nullptr,
                                 bind_of(hw, nullptr, ws), (int)p->dir_items.size(), (hipStream_t)stream));
  HIP_TRY(launch_vortdiv_from_projections(p->N, p->Fv, p->prec, pw, hw, vortdiv, (hipStream_t)stream));
  return SHT_OK;
}

int sht_spectral_op(sht_plan_t p, int op, int count, const void* in, void* out, void* stream) {
  if (!p || !in || !out || count < 0) return SHT_EINVAL;
  if (op != SHT_OP_DLAMBDA && op != SHT_OP_LAPLACIAN && op != SHT_OP_INV_LAPLACIAN) return SHT_EINVAL;
  if (count == 0) return SHT_OK;
  HIP_TRY(launch_spectral_op(p->N, count, op, p->prec, in, out, (hipStream_t)stream));
  return SHT_OK;
}

int sht_batch_create(sht_batch_t* out, const sht_plan_t* plans, int n, int flags, void* stream) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (!plans || n < 1 || (flags & ~(SHT_BATCH_PERSISTENT | SHT_BATCH_GRAPH))) return SHT_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!scalar_plan(plans[i]) || plans[i]->notab || plans[i]->prec != plans[0]->prec) return SHT_EINVAL;
  sht_batch_s* b = new (std::nothrow) sht_batch_s();
  if (!b) return SHT_ENOMEM;
  b->n = n;
  b->prec = plans[0]->prec;
  b->flags = flags;
  b->plans.assign(plans, plans + n);
  b->variant.resize(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    b->variant[i] = plans[i]->variant;
    b->ws_off.push_back(off);
    off += align256(sht_workspace_size(plans[i]));
    b->lds_syn = std::max(b->lds_syn, plans[i]->lds_syn);
    b->lds_ana = std::max(b->lds_ana, plans[i]->lds_ana);
    for (int t = 0; t < FFT_TIERS; ++t) {
      b->lds_syn_t[t] = std::max(b->lds_syn_t[t], plans[i]->lds_syn_t[t]);
      b->lds_ana_t[t] = std::max(b->lds_ana_t[t], plans[i]->lds_ana_t[t]);
    }
  }
  b->ws_bytes = off;
  const int rc = batch_upload(b, (hipStream_t)stream);
  if (rc != SHT_OK) {
    if (b->arena) (void)hipFree(b->arena);
    delete b;
    return rc;
  }
  *out = b;
  return SHT_OK;
}

size_t sht_batch_workspace_size(sht_batch_t b) { return b ? b->ws_bytes : 0; }

int sht_batch_bind(sht_batch_t b, void* const* spec, void* const* grid, void* workspace, void* stream) {
  if (!b || !spec || !grid || !workspace) return SHT_EINVAL;
  std::vector<IoBind> io(b->n);
  for (int i = 0; i < b->n; ++i) {
    if (!spec[i] || !grid[i]) return SHT_EINVAL;
    io[i] = IoBind{spec[i], grid[i], (char*)workspace + b->ws_off[i], nullptr};
  }
  HIP_TRY(write_binds(b->d_io, io, (hipStream_t)stream));
  b->io_host = io;
  b->bound = true;
  return SHT_OK;
}

int sht_batch_inverse(sht_batch_t b, void* stream) {
  if (!b) return SHT_EINVAL;
  return batch_run(b, (hipStream_t)stream, true);
}

int sht_batch_direct(sht_batch_t b, void* stream) {
  if (!b) return SHT_EINVAL;
  return batch_run(b, (hipStream_t)stream, false);
}

int sht_batch_tune(sht_batch_t b, void* stream) {
  if (!b || !b->bound) return SHT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SHT_EHIP;
  }
  // one measurement per distinct (truncation, grid, fields) in the batch:
  // the plan's two Legendre products with each supported tile variant (the
  // second of two runs counts).  Synthesis reads the bound spectral input and
  // writes the plan's workspace; analysis writes a temporary spectral array,
  // so the caller's buffers keep their contents.
  std::map<std::vector<int>, int> chosen;
  int rc = SHT_OK;
  for (int i = 0; i < b->n && rc == SHT_OK; ++i) {
    sht_plan_s* p = b->plans[i];
    const std::vector<int> key{p->N, p->grid, p->F};
    auto hit = chosen.find(key);
    if (hit != chosen.end()) {
      b->variant[i] = hit->second;
      continue;
    }
    int best = b->variant[i];
    float best_ms = 1e30f;
    for (int v = 0; v < NUM_TILE_VARIANTS && rc == SHT_OK; ++v) {
      if (!legendre_variant_supported(b->prec, v)) continue;
      std::vector<WorkItem> items, dir;
      legendre_items(p, v, 0, &items, &dir);
      const int ni = (int)items.size(), nd = (int)dir.size();
      items.insert(items.end(), dir.begin(), dir.end());
      WorkItem* d_items = nullptr;
      void* d_spec = nullptr;
      const size_t spec_bytes = (size_t)p->F * p->nspec * 2 * p->elem;
      if (hipMalloc(&d_items, sizeof(WorkItem) * items.size()) != hipSuccess ||
          hipMalloc(&d_spec, spec_bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (d_items) (void)hipFree(d_items);
        rc = SHT_ENOMEM;
        break;
      }
      hipError_t e = hipMemcpy(d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice);
      const IoBind io = b->io_host[i];
      const IoBind io_dir{d_spec, io.grid, io.ws, nullptr};
      float ms = 0.f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_legendre_inverse(p->d_self, p->prec, v, d_items, ni, nullptr, io, ni, s);
        if (e == hipSuccess)
          e = launch_legendre_direct(p->d_self, p->prec, v, d_items + ni, nd, nullptr, io_dir, nd, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      (void)hipFree(d_items);
      (void)hipFree(d_spec);
      if (e != hipSuccess) {
        rc = hip_fail(e);
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    chosen[key] = best;
    b->variant[i] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SHT_OK) return rc;
  return batch_upload(b, s);
}

int sht_batch_set_tiles(sht_batch_t b, const int32_t* tiles, void* stream) {
  if (!b || !tiles) return SHT_EINVAL;
  for (int i = 0; i < b->n; ++i)
    if (!legendre_variant_supported(b->prec, tiles[i])) return SHT_EINVAL;
  for (int i = 0; i < b->n; ++i) b->variant[i] = tiles[i];
  return batch_upload(b, (hipStream_t)stream);
}

int sht_batch_tiles(sht_batch_t b, int32_t* out) {
  if (!b || !out) return SHT_EINVAL;
  for (int i = 0; i < b->n; ++i) out[i] = b->variant[i];
  return SHT_OK;
}

int sht_batch_destroy(sht_batch_t b) {
  if (!b) return SHT_EINVAL;
  int rc = SHT_OK;
  destroy_graphs(b);
  if (b->arena) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(b->arena);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  delete b;
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Time stepping
// ---------------------------------------------------------------------------

struct sht_stepper_s {
  sht_plan_t plan = nullptr;
  void* spec = nullptr;
  void* grid = nullptr;
  void* ws = nullptr;
  double dt = 0, rate = 0, nu = 0;
  int graph_steps = 1;  // steps captured in one graph
  hipGraphExec_t exec = nullptr;
};

namespace {

// One time step on the stepper's buffers, for the reaction-diffusion
// equation du/dt = nu Lap u + r u (1 - u) on the unit sphere (report
// sections 4.2.2-4.2.3: the loop over time steps of synthesis, grid-point
// computations and analysis, on arrays allocated outside it): semi-implicit
// Euler, the logistic term explicit on the grid, g <- g + dt r g (1 - g),
// fused into the synthesis' grid stores, and the diffusion implicit in
// spectral space (Lap -> -n (n + 1)), a_n^m <- a_n^m / (1 + dt nu n (n + 1)),
// fused into the analysis' coefficient stores: four stages, no pass of its
// own over the grid or the coefficients.
int enqueue_step(const sht_stepper_s* st, hipStream_t s) {
  sht_plan_t p = st->plan;
  int rc = stage_legendre_inverse(p, st->spec, st->ws, s);
  if (rc == SHT_OK) rc = stage_fourier_synthesis(p, st->ws, st->grid, s, st->dt * st->rate);
  if (rc == SHT_OK) rc = stage_fourier_analysis(p, st->grid, st->ws, s);
  if (rc == SHT_OK) rc = stage_legendre_direct(p, st->ws, st->spec, s, st->dt * st->nu);
  return rc;
}

// Capture graph_steps steps into one graph on stream `s` (which must not be
// the null stream).
int capture_step(sht_stepper_s* st, hipStream_t s) {
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = SHT_OK;
  for (int i = 0; i < st->graph_steps && rc == SHT_OK; ++i) rc = enqueue_step(st, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != SHT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e);
  const hipError_t ei = hipGraphInstantiate(&st->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    st->exec = nullptr;
    return hip_fail(ei);
  }
  return SHT_OK;
}

}  // namespace

extern "C" {

int sht_stepper_create(sht_stepper_t* out, sht_plan_t plan, double dt, double rate, double nu, void* spec,
                       void* grid, void* workspace, int flags, int graph_steps, void* hip_stream) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (!scalar_plan(plan) || !spec || !grid || !workspace || (flags & ~SHT_STEP_GRAPH)) return SHT_EINVAL;
  if (graph_steps < 1 || graph_steps > 4096) return SHT_EINVAL;
  if (!(dt >= 0.0) || !(nu >= 0.0) || !std::isfinite(rate) || !std::isfinite(dt) || !std::isfinite(nu))
    return SHT_EINVAL;
  if ((flags & SHT_STEP_GRAPH) && !hip_stream) return SHT_EINVAL;  // the null stream cannot be captured
  sht_stepper_s* st = new (std::nothrow) sht_stepper_s();
  if (!st) return SHT_ENOMEM;
  st->plan = plan;
  st->spec = spec;
  st->grid = grid;
  st->ws = workspace;
  st->dt = dt;
  st->rate = rate;
  st->nu = nu;
  st->graph_steps = (flags & SHT_STEP_GRAPH) ? graph_steps : 1;
  if (flags & SHT_STEP_GRAPH) {
    const int rc = capture_step(st, (hipStream_t)hip_stream);
    if (rc != SHT_OK) {
      delete st;
      return rc;
    }
  }
  *out = st;
  return SHT_OK;
}

int sht_stepper_run(sht_stepper_t st, int nsteps, void* hip_stream) {
  if (!st || nsteps < 0) return SHT_EINVAL;
  const hipStream_t s = (hipStream_t)hip_stream;
  int left = nsteps;
  if (st->exec)
    for (; left >= st->graph_steps; left -= st->graph_steps) HIP_TRY(hipGraphLaunch(st->exec, s));
  for (; left > 0; --left) {
    const int rc = enqueue_step(st, s);
    if (rc != SHT_OK) return rc;
  }
  return SHT_OK;
}

int sht_stepper_destroy(sht_stepper_t st) {
  if (!st) return SHT_EINVAL;
  int rc = SHT_OK;
  if (st->exec) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGraphExecDestroy(st->exec);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  delete st;
  return rc;
}

const char* sht_strerror(int status) {
  switch (status) {
    case SHT_OK: return "success";
    case SHT_EINVAL: return "invalid argument";
    case SHT_EUNSUPPORTED: return "unsupported truncation, grid or precision";
    case SHT_ENOMEM: return "device allocation failed";
    case SHT_EHIP: return "HIP runtime error";
    case SHT_ESCRATCH: return "workspace larger than the library's static scratch";
    default: return "unknown status";
  }
}

int sht_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
