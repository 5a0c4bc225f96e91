// Host runtime and C ABI: plan construction (geometry, FFT classes, table
// layout, work lists), one device arena per plan, and the stream-ordered
// entry points.  Following the report's restructured time step (section
// 4.2.3), everything that allocates or copies metadata happens once at plan
// creation; the transform calls only enqueue kernels.
#include <algorithm>
#include <cstring>
#include <new>
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

// Radix sequence for a 5-smooth length, fewest passes first: the power of
// two as 16s plus one 2, 4 or 8; the power of three as 9s plus one 3; 5s.
std::vector<int> radices(int L) {
  std::vector<int> r;
  int x = L, e2 = 0;
  while (x % 2 == 0) {
    x /= 2;
    ++e2;
  }
  for (; e2 >= 4; e2 -= 4) r.push_back(16);
  if (e2 > 0) r.push_back(1 << e2);
  while (x % 9 == 0) {
    r.push_back(9);
    x /= 9;
  }
  if (x % 3 == 0) {
    r.push_back(3);
    x /= 3;
  }
  while (x % 5 == 0) {
    r.push_back(5);
    x /= 5;
  }
  return r;
}

// Every Stockham pass must fit FFT_REGS complex values per thread.
bool fits_registers(int L, const std::vector<int>& rad) {
  for (int R : rad)
    if ((int64_t)(L / R) > (int64_t)(FFT_REGS / R) * FFT_THREADS) return false;
  return true;
}

}  // namespace

struct sht_plan_s {
  int N = 0, grid = 0, F = 0, prec = 0, nlat = 0, nh = 0, Fp = 0;
  int64_t npts = 0, nspec = 0, nfour = 0;
  int elem = 8;
  std::vector<RingInfo> rings;
  std::vector<FftClass> classes;
  std::vector<MInfo> ms;
  std::vector<int64_t> ring_off, four_row;
  std::vector<WorkItem> inv_items, dir_items;
  std::vector<int2> syn_items, ana_items;
  int64_t tab_plane = 0;
  size_t tab_bytes = 0, fft_bytes = 0;
  size_t lds_syn = 0, lds_ana = 0;
  int max_Lp = 0;
  // device
  void* arena = nullptr;
  size_t arena_bytes = 0;
  DevPlan dp{};
  WorkItem* d_inv = nullptr;
  WorkItem* d_dir = nullptr;
  int2* d_syn = nullptr;
  int2* d_ana = nullptr;
  MInfo* d_ms = nullptr;
  FftClass* d_cls = nullptr;
};

namespace {

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
  p->nspec = (int64_t)(N + 1) * (N + 2) / 2;
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

  // ---- FFT classes (one per distinct half length) ----
  const int csize = (p->prec == SHT_FP64) ? 16 : 8;
  std::vector<int> hs;
  for (auto& r : p->rings) hs.push_back(r.nlon / 2);
  std::sort(hs.begin(), hs.end());
  hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
  int64_t off = 0;
  for (int h : hs) {
    FftClass c{};
    c.h = h;
    if (five_smooth(h)) {
      c.L = h;
      c.bluestein = 0;
    } else {
      int64_t L = 2 * (int64_t)h - 1;
      while (!five_smooth(L)) ++L;
      c.L = (int)L;
      c.bluestein = 1;
    }
    std::vector<int> rad = radices(c.L);
    if ((int)rad.size() > FFT_MAX_RADICES || !fits_registers(c.L, rad)) return SHT_EUNSUPPORTED;
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
    p->classes.push_back(c);
  }
  p->fft_bytes = (size_t)off * csize;
  for (auto& r : p->rings) {
    const int h = r.nlon / 2;
    r.cls = (int)(std::lower_bound(hs.begin(), hs.end(), h) - hs.begin());
    const FftClass& c = p->classes[r.cls];
    p->lds_syn = std::max(p->lds_syn, fft_lds_bytes(p->prec, c.L, -1));
    p->lds_ana = std::max(p->lds_ana, fft_lds_bytes(p->prec, c.L, r.mmax));
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
    mi.K[0] = (N - m) / 2 + 1;
    mi.K[1] = (N - m + 1) / 2;
    mi.Kp[0] = (int)round_up(mi.K[0], KCH);
    mi.Kp[1] = (int)round_up(mi.K[1], KCH);
    mi.toff[0] = toff;
    mi.toff[1] = toff + (int64_t)mi.Kp[0] * mi.Lp;
    toff = mi.toff[1] + (int64_t)mi.Kp[1] * mi.Lp;
    mi.spec_off = (int64_t)m * (2 * N + 3 - m) / 2;
    p->max_Lp = std::max(p->max_Lp, mi.Lp);
    p->ms.push_back(mi);
  }
  p->tab_plane = toff;
  const int tab_elem = (p->prec == SHT_FP64) ? 8 : (p->prec == SHT_FP32 ? 4 : 4);
  p->tab_bytes = (size_t)toff * tab_elem;

  // ---- work lists (m ascending = cost descending for both products) ----
  int ir, ic, dr, dc;
  legendre_tiles(p->prec, &ir, &ic, &dr, &dc);
  const int twoF = 2 * p->F;
  for (const MInfo& mi : p->ms) {
    if (mi.L == 0) continue;
    for (int t0 = 0; t0 < mi.L; t0 += ir)
      for (int c0 = 0; c0 < twoF; c0 += ic) p->inv_items.push_back(WorkItem{mi.m, t0, c0, 0});
    const int kmax = std::max(mi.K[0], mi.K[1]);
    for (int t0 = 0; t0 < kmax; t0 += dr)
      for (int c0 = 0; c0 < twoF; c0 += dc) p->dir_items.push_back(WorkItem{mi.m, t0, c0, 0});
  }
  // FFT items, longest transforms first
  std::vector<int> order(p->nlat);
  for (int j = 0; j < p->nlat; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return p->classes[p->rings[a].cls].L > p->classes[p->rings[b].cls].L;
  });
  const int fchunk = 16;
  for (int j : order)
    for (int f0 = 0; f0 < p->F; f0 += fchunk) {
      p->syn_items.push_back(int2{j, f0});
      if (j < p->nh) p->ana_items.push_back(int2{j, f0});
    }
  return SHT_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int build_device(sht_plan_s* p, hipStream_t s) {
  struct Part {
    void** dst;
    size_t bytes;
  };
  void *v_rings, *v_cls, *v_ms, *v_mu, *v_w, *v_tab, *v_fft, *v_inv, *v_dir, *v_syn, *v_ana;
  const Part parts[] = {
      {&v_rings, sizeof(RingInfo) * p->rings.size()},
      {&v_cls, sizeof(FftClass) * p->classes.size()},
      {&v_ms, sizeof(MInfo) * p->ms.size()},
      {&v_mu, sizeof(double) * p->nlat},
      {&v_w, sizeof(double) * p->nlat},
      {&v_tab, p->tab_bytes},
      {&v_fft, p->fft_bytes},
      {&v_inv, sizeof(WorkItem) * p->inv_items.size()},
      {&v_dir, sizeof(WorkItem) * p->dir_items.size()},
      {&v_syn, sizeof(int2) * p->syn_items.size()},
      {&v_ana, sizeof(int2) * p->ana_items.size()},
  };
  size_t total = 0;
  for (const Part& q : parts) total += align256(q.bytes);
  if (hipMalloc(&p->arena, total) != hipSuccess) {
    (void)hipGetLastError();
    p->arena = nullptr;
    return SHT_ENOMEM;
  }
  p->arena_bytes = total;
  size_t o = 0;
  for (const Part& q : parts) {
    *q.dst = (char*)p->arena + o;
    o += align256(q.bytes);
  }
  HIP_TRY(hipMemcpyAsync(v_rings, p->rings.data(), parts[0].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_cls, p->classes.data(), parts[1].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_ms, p->ms.data(), parts[2].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_inv, p->inv_items.data(), parts[7].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_dir, p->dir_items.data(), parts[8].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_syn, p->syn_items.data(), parts[9].bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v_ana, p->ana_items.data(), parts[10].bytes, hipMemcpyHostToDevice, s));

  DevPlan& d = p->dp;
  d.N = p->N;
  d.nlat = p->nlat;
  d.nh = p->nh;
  d.F = p->F;
  d.Fp = p->Fp;
  d.npts = p->npts;
  d.nspec = p->nspec;
  d.rings = (const RingInfo*)v_rings;
  d.classes = (const FftClass*)v_cls;
  d.ms = (const MInfo*)v_ms;
  d.mu = (const double*)v_mu;
  d.w = (const double*)v_w;
  d.tab = v_tab;
  d.fft = v_fft;
  p->d_inv = (WorkItem*)v_inv;
  p->d_dir = (WorkItem*)v_dir;
  p->d_syn = (int2*)v_syn;
  p->d_ana = (int2*)v_ana;
  p->d_ms = (MInfo*)v_ms;
  p->d_cls = (FftClass*)v_cls;

  HIP_TRY(launch_gauss(p->nlat, (double*)v_mu, (double*)v_w, s));
  HIP_TRY(launch_pbar_planes(d, p->prec, p->d_ms, (int)p->ms.size(), p->max_Lp, v_tab, p->tab_plane, s));
  HIP_TRY(launch_fft_tables(d, p->prec, p->d_cls, (int)p->classes.size(), p->classes.data(), v_fft, s));
  HIP_TRY(fft_set_max_lds(std::max(p->lds_syn, p->lds_ana)));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  return SHT_OK;
}

}  // namespace

extern "C" {

int sht_plan_create(sht_plan_t* out, int truncation, int grid, int nfields, int precision, void* hip_stream) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (truncation < 1 || nfields < 1) return SHT_EINVAL;
  if (grid != SHT_GRID_FULL && grid != SHT_GRID_OCTAHEDRAL) return SHT_EINVAL;
  if (precision != SHT_FP64 && precision != SHT_FP32 && precision != SHT_BF16X3) return SHT_EINVAL;
  sht_plan_s* p = new (std::nothrow) sht_plan_s();
  if (!p) return SHT_ENOMEM;
  p->N = truncation;
  p->grid = grid;
  p->F = nfields;
  p->prec = precision;
  p->elem = (precision == SHT_FP64) ? 8 : 4;
  int rc = build_host(p);
  if (rc == SHT_OK) rc = build_device(p, (hipStream_t)hip_stream);
  if (rc != SHT_OK) {
    if (p->arena) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p->arena);
    }
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
    if (e == hipSuccess) e = hipFree(p->arena);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  delete p;
  return rc;
}

int sht_plan_info(sht_plan_t p, sht_info* out) {
  if (!p || !out) return SHT_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->truncation = p->N;
  out->grid = p->grid;
  out->nfields = p->F;
  out->precision = p->prec;
  out->nlat = p->nlat;
  out->fpad = p->Fp;
  out->npts = p->npts;
  out->nspec = p->nspec;
  out->nfour = p->nfour;
  out->workspace_bytes = (int64_t)sht_workspace_size(p);
  out->table_bytes = (int64_t)p->tab_bytes;
  out->plan_bytes = (int64_t)p->arena_bytes;
  out->elem_bytes = p->elem;
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
  if (!p || m < 0 || m > p->N) return SHT_EINVAL;
  const MInfo& mi = p->ms[m];
  if (first_ring) *first_ring = mi.first_ring;
  if (!out) return SHT_OK;
  const size_t n = (size_t)mi.L * (p->N - m + 1);
  if (n == 0) return SHT_OK;
  double* tmp = nullptr;
  HIP_TRY(hipMalloc(&tmp, n * sizeof(double)));
  hipError_t e = launch_table_export_planes(p->dp, p->prec, mi, p->tab_plane, tmp, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, tmp, n * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e);
  return SHT_OK;
}

size_t sht_workspace_size(sht_plan_t p) {
  if (!p) return 0;
  return (size_t)p->nfour * p->Fp * 2 * p->elem;
}

int sht_legendre_inverse(sht_plan_t p, const void* spec, void* four, void* stream) {
  if (!p || !spec || !four) return SHT_EINVAL;
  HIP_TRY(launch_legendre_inverse(p->dp, p->prec, p->d_inv, (int)p->inv_items.size(), p->tab_plane, spec, four,
                                  (hipStream_t)stream));
  return SHT_OK;
}

int sht_fourier_synthesis(sht_plan_t p, const void* four, void* grid, void* stream) {
  if (!p || !four || !grid) return SHT_EINVAL;
  HIP_TRY(launch_fourier_synthesis(p->dp, p->prec, p->d_syn, (int)p->syn_items.size(), p->lds_syn, four, grid,
                                   (hipStream_t)stream));
  return SHT_OK;
}

int sht_fourier_analysis(sht_plan_t p, const void* grid, void* four, void* stream) {
  if (!p || !four || !grid) return SHT_EINVAL;
  HIP_TRY(launch_fourier_analysis(p->dp, p->prec, p->d_ana, (int)p->ana_items.size(), p->lds_ana, grid, four,
                                  (hipStream_t)stream));
  return SHT_OK;
}

int sht_legendre_direct(sht_plan_t p, const void* four, void* spec, void* stream) {
  if (!p || !spec || !four) return SHT_EINVAL;
  HIP_TRY(launch_legendre_direct(p->dp, p->prec, p->d_dir, (int)p->dir_items.size(), p->tab_plane, four, spec,
                                 (hipStream_t)stream));
  return SHT_OK;
}

int sht_inverse(sht_plan_t p, const void* spec, void* grid, void* ws, void* stream) {
  if (!p || !spec || !grid || !ws) return SHT_EINVAL;
  int rc = sht_legendre_inverse(p, spec, ws, stream);
  if (rc != SHT_OK) return rc;
  return sht_fourier_synthesis(p, ws, grid, stream);
}

int sht_direct(sht_plan_t p, const void* grid, void* spec, void* ws, void* stream) {
  if (!p || !spec || !grid || !ws) return SHT_EINVAL;
  int rc = sht_fourier_analysis(p, grid, ws, stream);
  if (rc != SHT_OK) return rc;
  return sht_legendre_direct(p, ws, spec, stream);
}

const char* sht_strerror(int status) {
  switch (status) {
    case SHT_OK: return "success";
    case SHT_EINVAL: return "invalid argument";
    case SHT_EUNSUPPORTED: return "unsupported truncation, grid or precision";
    case SHT_ENOMEM: return "device allocation failed";
    case SHT_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int sht_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
