// Host side of the C ABI declared in include/stmf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/stmf.h"
#include "stmf_internal.h"

namespace stmf {

// kernels (stmf_fit.hip, stmf_prims.hip, stmf_setup.hip)
__global__ void fit_kernel(const FitDev* fits, int nfits, int max_rows, unsigned* queue, int qgroup,
                           FitCtl* gctl, BarTree* gbar);
__global__ void fit_kernel_sel(const FitDev* fits, int nfits, int max_rows, unsigned* queue,
                               int qgroup, FitCtl* gctl, BarTree* gbar);
__global__ void fit_kernel_matrix(const FitDev* fits, int nfits, int max_rows, unsigned* queue,
                                  int qgroup, FitCtl* gctl, BarTree* gbar);
__global__ void fit_kernel_wide(const FitDev* fits, int nfits, int max_rows, unsigned* queue,
                                int qgroup, FitCtl* gctl, BarTree* gbar);
size_t fit_smem_bytes();
size_t masked_error_ws(int m, int n);
hipError_t launch_maxplus(const float*, const float*, int, int, int, float*, int32_t*, hipStream_t);
hipError_t launch_masked_error(const float*, const uint8_t*, const float*, const float*, int, int,
                               int, double*, double*, void*, hipStream_t);
hipError_t launch_update(int, const float*, const uint8_t*, float*, float*, int, int, int, int, int,
                         int, float*, float*, double*, void*, hipStream_t);
__global__ void check_count_kernel(const float*, const uint8_t*, int, int, int*, int*, CheckOut*);
__global__ void check_empty_kernel(const int*, const int*, int, int, CheckOut*);
__global__ void fill_u32_kernel(unsigned*, size_t, unsigned);
__global__ void pack_kernel(const float*, const uint8_t*, int, int, int, int, int, int, const int*,
                            const int*,
                            float*);
__global__ void transpose_kernel(const float*, int, int, float*);
__global__ void rowmin_kernel(const float*, const uint8_t*, int, int, int, float*);
__global__ void rank_perm_kernel(const float*, int, int*);
__global__ void iota_kernel(int*, int);
__global__ void u0_given_kernel(const float*, int, int, int, float*);
__global__ void u0_acol_kernel(const float*, int, int, int, int, int, int, const int*, float*);
__global__ void vinit_kernel(const float*, const float*, int, int, int, int, int, float*);
__global__ void output_kernel(const float*, const float*, int, int, int, int, int, int, const int*,
                              const int*,
                              float*, float*);
__global__ void copy_f64_kernel(const double*, double*, int);

// ---------------------------------------------------------------- randomness
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): a Weyl sequence with step
// 0x9E3779B97F4A7C15 passed through a 64-bit mixing finaliser.
struct Rng {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform in [0, bound): reject draws below 2^64 mod bound, then reduce
  uint64_t below(uint64_t bound) {
    const uint64_t floor_ = (~bound + 1) % bound;
    for (;;) {
      uint64_t x = next();
      if (x >= floor_) return x % bound;
    }
  }
};

// ---------------------------------------------------------------- helpers
static inline size_t al256(size_t x) { return (x + 255) / 256 * 256; }
static inline int rup(int x, int a) { return (x + a - 1) / a * a; }

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return STMF_EHIP;            \
  } while (0)

struct DevProps {
  int cus = 0;
  int coresident = 0;  // fit_kernel workgroups that fit at once
  bool ok = false;
};

static std::mutex g_props_mu;
static DevProps g_props[64];

static int device_props(DevProps& out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return STMF_EHIP;
  std::lock_guard<std::mutex> lk(g_props_mu);
  DevProps& p = g_props[dev];
  if (!p.ok) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    p.cus = prop.multiProcessorCount;
    const size_t smem = fit_smem_bytes();
    HIPCHK(hipFuncSetAttribute((const void*)fit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)smem));
    HIPCHK(hipFuncSetAttribute((const void*)fit_kernel_sel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    HIPCHK(hipFuncSetAttribute((const void*)fit_kernel_matrix,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    HIPCHK(hipFuncSetAttribute((const void*)fit_kernel_wide,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    // the fit kernels share the LDS layout; the group size must suit all
    int per = 0, per_sel = 0, per_mat = 0, per_wide = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)fit_kernel, NTHR, smem));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_sel, (const void*)fit_kernel_sel, NTHR,
                                                        smem));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_mat, (const void*)fit_kernel_matrix,
                                                        NTHR, smem));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_wide, (const void*)fit_kernel_wide,
                                                        NTHR, smem));
    p.coresident = std::min(std::min(per, per_sel), std::min(per_mat, per_wide)) * p.cus;
    // a group barrier holds up to GROUP_MAX workgroups
    p.coresident = std::min(p.coresident, GROUP_MAX);
    p.ok = true;
  }
  out = p;
  return STMF_OK;
}

void options_default(stmf_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->init_mode = 0;
  o->init_lo = 0.0f;
  o->init_hi = 100.0f;
  o->acol_p = 5;
  o->noop_rule = 1;
  o->batch_first = 0;
  o->batch_max = 0;
}

static int check_options(const stmf_options& o) {
  if (o.init_mode < 0 || o.init_mode > 2) return STMF_EINVAL;
  if (o.init_mode == 2 && !o.U0) return STMF_EINVAL;
  if (o.init_mode == 0 && !(o.init_hi >= o.init_lo)) return STMF_EINVAL;
  if (o.init_mode == 1 && o.acol_p < 1) return STMF_EINVAL;
  if (o.count_scope < 0 || o.count_scope > 1) return STMF_EINVAL;
  if (o.batch_first < 0 || o.batch_max < 0 || o.batch_max > TMAX) return STMF_EINVAL;
  if (o.group_size < 0 || o.log_cap < 0 || o.max_row_visits < 0) return STMF_EINVAL;
  if (!(o.eps >= 0.0)) return STMF_EINVAL;
  if (o.selection < 0 || o.selection > 3 || o.perm_mode < 0 || o.perm_mode > 3) return STMF_EINVAL;
  if (o.strategy < 0 || o.strategy > 2) return STMF_EINVAL;
  return STMF_OK;
}

// ---------------------------------------------------------------- layout
struct Layout {
  int m, n, r, iters;
  int mw, nw, ldm, ldn, nrt, nct, ldmax, G, acol_p, tmax;
  int transposed;
  size_t Rw, RwT, Uc, V, td, tdpart, crow, ccol, colst, rowst, colpart, rowpart, order, rowt,
      rord, tdrow, tvec, epart, eprime, closed, traj, ctl, bar, dev, perm, cperm, stage, check, rowc,
      colc, mtd, mfk, mkey, mtdr, mtdc, mhist, mcnt, mgat_u, mgat_q, mlist_q, mlist_k;
  bool matrix;
  size_t total;
};

// Largest batch when the caller leaves it to the library: a power of two,
// 2048 / tiles per workgroup, between 64 and TMAX (the trial buffers of the
// layout are sized by it).
static int auto_batch_max(int tiles, int G) {
  const int per = (tiles + G - 1) / G;
  int t = 64;
  while (t * 2 <= 2048 / per && t * 2 <= TMAX) t *= 2;
  return t;
}

// `matrix`: room for the ByMatrix buffers (per cell of the working matrix).
static void make_layout(int m, int n, int r, int iters, int G, int acol_p, int batch_max,
                        Layout& L, bool matrix = false) {
  L.m = m; L.n = n; L.r = r; L.iters = iters; L.G = G; L.acol_p = acol_p;
  L.transposed = m > n;
  L.mw = L.transposed ? n : m;
  L.nw = L.transposed ? m : n;
  L.ldm = rup(L.mw, TS);
  L.ldn = rup(L.nw, TS);
  L.nrt = L.ldm / TS;
  L.nct = L.ldn / TS;
  L.ldmax = std::max(L.ldm, L.ldn);
  L.tmax = batch_max > 0 ? batch_max : auto_batch_max(L.nrt * L.nct, G);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += al256(bytes); return at; };
  L.Rw = take((size_t)L.ldm * L.ldn * 4);
  L.RwT = take((size_t)L.ldn * L.ldm * 4);
  L.Uc = take((size_t)r * L.ldm * 4);
  L.V = take((size_t)r * L.ldn * 4);
  L.td = take((size_t)L.ldn * 8);
  L.tdpart = take((size_t)L.nrt * L.ldn * 8);
  L.crow = take((size_t)2 * L.ldm * r * 4);
  L.ccol = take((size_t)2 * L.ldn * r * 4);
  L.colst = take((size_t)r * L.ldn * sizeof(Top2));
  L.rowst = take((size_t)r * L.ldm * sizeof(Top2));
  L.colpart = take((size_t)L.nrt * L.ldn * sizeof(Top2));
  L.rowpart = take((size_t)L.nct * L.ldm * sizeof(Top2));
  L.order = take((size_t)L.ldn * 4);
  L.rord = take((size_t)L.ldn * 4);
  L.tdrow = take((size_t)L.ldn * 8);
  L.tvec = take((size_t)2 * L.tmax * L.ldmax * 4);
  L.epart = take((size_t)L.tmax * L.nrt * L.nct * 8);
  L.eprime = take((size_t)L.tmax * 8);
  L.closed = take((size_t)r * 4);
  L.rowt = take((size_t)L.mw * 4);
  L.traj = take((size_t)(iters + 1) * 8);
  L.ctl = take(sizeof(FitCtl));
  L.bar = take(sizeof(BarTree));
  L.dev = take(sizeof(FitDev));
  L.perm = take((size_t)L.mw * 4);
  L.cperm = take((size_t)L.nw * 4);
  L.stage = take(std::max({(size_t)L.mw * r * 4, (size_t)r * acol_p * 4, (size_t)L.nw * 4}));
  L.check = take(sizeof(CheckOut));
  L.rowc = take((size_t)m * 4);
  L.colc = take((size_t)n * 4);
  L.matrix = matrix;
  const size_t cells = matrix ? (size_t)L.mw * L.nw : 0, mt = matrix ? (size_t)L.tmax : 0;
  L.mtd = take(cells * 8);
  L.mfk = take(cells * 4);
  L.mkey = take(cells * 8);
  L.mtdr = take(matrix ? (size_t)L.mw * 8 : 0);
  L.mtdc = take(matrix ? (size_t)L.nw * 8 : 0);
  L.mhist = take(matrix ? (size_t)MATRIX_HIST * 256 * 4 : 0);
  L.mcnt = take(matrix ? 16 : 0);
  L.mgat_u = take(mt * 8);
  L.mgat_q = take(mt * 4);
  L.mlist_q = take(mt * 4);
  L.mlist_k = take(mt * 4);
  L.total = o;
}

// Smallest first batch of a row visit when the caller leaves it to the
// library.  A batch costs its synchronisation and, for every tile a
// workgroup sweeps, the tile's staging plus the trials' evaluation; trials
// after the accepted one are wasted.  The floor shrinks as each workgroup's
// share of tiles grows: 512 / tiles per workgroup, a power of two, at least
// 4, never above the largest batch.  A row's first visit starts at the
// power of two at or above the trials the last row visit needed, if that is
// more (the first pass of a fit that accepts early, on groups that sweep many
// tiles, wastes little); later visits from the row's own previous visit.
static int auto_batch_first(const Layout& L) {
  const int tiles = L.nrt * L.nct;
  const int per = (tiles + L.G - 1) / L.G;
  int t = 4;
  while (t * 2 <= 512 / per && t * 2 <= L.tmax) t *= 2;
  return std::min(t, L.tmax);
}

// What the fit kernel runs: a ByRow selection, or ByElement.
static int kernel_sel(const stmf_options& o) {
  return o.strategy == 2 ? (int)SEL_MATRIX : o.strategy == 1 ? (int)SEL_ELEM : o.selection;
}

static FitDev make_dev(const Layout& L, char* base, const stmf_options& o, int observed) {
  FitDev d;
  std::memset(&d, 0, sizeof(d));
  d.m = L.mw; d.n = L.nw; d.r = L.r;
  d.ldm = L.ldm; d.ldn = L.ldn; d.nrt = L.nrt; d.nct = L.nct;
  d.iters = L.iters;
  d.noop_rule = o.noop_rule; d.count_scope = o.count_scope;
  d.tmax = L.tmax;
  d.t0 = std::min(o.batch_first > 0 ? o.batch_first : auto_batch_first(L), L.tmax);
  d.log_cap = o.decision_log ? o.log_cap : 0;
  d.eps = o.eps;
  d.omega = observed;
  d.sel = kernel_sel(o);
  d.Rw = (const float*)(base + L.Rw);
  d.RwT = (const float*)(base + L.RwT);
  d.Uc = (float*)(base + L.Uc);
  d.V = (float*)(base + L.V);
  d.td = (double*)(base + L.td);
  d.tdpart = (double*)(base + L.tdpart);
  d.crow = (int*)(base + L.crow);
  d.ccol = (int*)(base + L.ccol);
  d.colst = (Top2*)(base + L.colst);
  d.rowst = (Top2*)(base + L.rowst);
  d.colpart = (Top2*)(base + L.colpart);
  d.rowpart = (Top2*)(base + L.rowpart);
  d.order = (int*)(base + L.order);
  d.rord = (int*)(base + L.rord);
  d.tdrow = (double*)(base + L.tdrow);
  d.tvec = (unsigned*)(base + L.tvec);
  d.epart = (double*)(base + L.epart);
  d.eprime = (double*)(base + L.eprime);
  d.closed = (int*)(base + L.closed);
  d.rowt = (int*)(base + L.rowt);
  d.traj = (double*)(base + L.traj);
  d.log = (LogRec*)o.decision_log;
  d.ctl = (FitCtl*)(base + L.ctl);
  d.bar = (BarTree*)(base + L.bar);
  d.ldmax = L.ldmax;
  d.gsize = L.G;
  d.bar_wait = o.barrier_wait_us < 0 ? -1 : (long long)o.barrier_wait_us * 100;
  if (L.matrix) {
    d.mtd = (double*)(base + L.mtd);
    d.mfk = (int*)(base + L.mfk);
    d.mkey = (unsigned long long*)(base + L.mkey);
    d.mtdr = (double*)(base + L.mtdr);
    d.mtdc = (double*)(base + L.mtdc);
    d.mhist = (int*)(base + L.mhist);
    d.mcnt = (int*)(base + L.mcnt);
    d.mgat_u = (unsigned long long*)(base + L.mgat_u);
    d.mgat_q = (int*)(base + L.mgat_q);
    d.mlist_q = (int*)(base + L.mlist_q);
    d.mlist_k = (int*)(base + L.mlist_k);
  }
  return d;
}

static int fill_u32(void* p, size_t count, unsigned v, hipStream_t s) {
  if (!count) return STMF_OK;
  size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned*)p, count, v);
  return hipGetLastError() == hipSuccess ? STMF_OK : STMF_EHIP;
}

// Check R and M (synchronous): empty lines, non-finite observed values,
// magnitudes.  Uses the layout's rowc/colc/check scratch.
static int check_inputs(const float* R, const uint8_t* M, const Layout& L, char* base, int int_exact,
                        hipStream_t s, int* observed = nullptr) {
  int st = fill_u32(base + L.rowc, (size_t)L.m, 0, s);
  if (!st) st = fill_u32(base + L.colc, (size_t)L.n, 0, s);
  if (!st) st = fill_u32(base + L.check, sizeof(CheckOut) / 4, 0, s);
  if (st) return st;
  const size_t total = (size_t)L.m * L.n;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(check_count_kernel, dim3(blocks), dim3(256), 0, s, R, M, L.m, L.n,
                     (int*)(base + L.rowc), (int*)(base + L.colc), (CheckOut*)(base + L.check));
  const int mx = std::max(L.m, L.n);
  hipLaunchKernelGGL(check_empty_kernel, dim3((mx + 255) / 256), dim3(256), 0, s,
                     (const int*)(base + L.rowc), (const int*)(base + L.colc), L.m, L.n,
                     (CheckOut*)(base + L.check));
  HIPCHK(hipGetLastError());
  CheckOut h;
  HIPCHK(hipMemcpyAsync(&h, base + L.check, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (observed) *observed = h.observed;
  if (h.empty_rows || h.empty_cols) return STMF_EEMPTY_LINE;
  if (h.nonfinite) return STMF_EINVAL;
  if (h.too_big) return STMF_ERANGE;
  if (int_exact && h.not_int24) return STMF_ERANGE;
  return STMF_OK;
}

// Draws of a fit from its seed: the working permutation (unless given, or
// PermR / none), then the initial U (random integers) or the Random Acol
// column indices.  The PermR order is data-dependent: prepare_fit computes it
// on the device, and perm holds the identity until then.
static int draw_setup(const Layout& L, uint64_t seed, const stmf_options& o,
                      std::vector<int32_t>& perm, std::vector<float>& U0, std::vector<int32_t>& cols) {
  Rng g{seed};
  perm.resize(L.mw);
  if (o.perm) {
    std::vector<char> hit(L.mw, 0);
    for (int a = 0; a < L.mw; ++a) {
      int p = o.perm[a];
      if (p < 0 || p >= L.mw || hit[p]) return STMF_EINVAL;
      hit[p] = 1;
      perm[a] = p;
    }
  } else {
    for (int a = 0; a < L.mw; ++a) perm[a] = a;
    for (int a = o.perm_mode == 0 ? L.mw - 1 : 0; a >= 1; --a) {
      int b = (int)g.below((uint64_t)a + 1);
      std::swap(perm[a], perm[b]);
    }
  }
  if (o.init_mode == 0) {
    const int64_t lo = (int64_t)o.init_lo, hi = (int64_t)o.init_hi;
    const uint64_t span = (uint64_t)(hi - lo + 1);
    U0.resize((size_t)L.mw * L.r);
    for (size_t q = 0; q < U0.size(); ++q) U0[q] = (float)(lo + (int64_t)g.below(span));
  } else if (o.init_mode == 1) {
    cols.resize((size_t)L.r * o.acol_p);
    for (size_t q = 0; q < cols.size(); ++q) cols[q] = (int)g.below((uint64_t)L.nw);
  } else {
    U0.assign(o.U0, o.U0 + (size_t)L.mw * L.r);
  }
  return STMF_OK;
}

// Working matrix, initial U and V, control block: everything a fit kernel
// needs, stream-ordered.  Host vectors must outlive the copies: the caller
// synchronises before they go out of scope.
static int prepare_fit(const float* R, const uint8_t* M, const Layout& L, char* base,
                       const stmf_options& o, const std::vector<int32_t>& perm,
                       const std::vector<float>& U0, const std::vector<int32_t>& cols,
                       hipStream_t s) {
  if (o.integer_exact && o.init_mode != 1)
    for (float x : U0)
      if (!(std::fabs(x) < 16777216.0f)) return STMF_ERANGE;
  for (float x : U0)
    if (!std::isfinite(x) || std::fabs(x) >= 1e30f) return STMF_ERANGE;
  if (o.perm_mode == 1 && !o.perm) {
    // PermR: minimum observed value of every working row, then the stable
    // order by it (both on the device; the minima use the staging buffer,
    // which the initial U overwrites later in stream order)
    hipLaunchKernelGGL(rowmin_kernel, dim3(L.mw), dim3(256), 0, s, R, M, L.n, L.nw, L.transposed,
                       (float*)(base + L.stage));
    hipLaunchKernelGGL(rank_perm_kernel, dim3((L.mw + 255) / 256), dim3(256), 0, s,
                       (const float*)(base + L.stage), L.mw, (int*)(base + L.perm));
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(base + L.perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, s));
  }
  if (o.perm_mode == 3) {
    // PermC: minimum observed value of every working column, then the stable
    // order by it (a working column is an original column, or an original
    // row when transposed)
    hipLaunchKernelGGL(rowmin_kernel, dim3(L.nw), dim3(256), 0, s, R, M, L.n, L.mw, !L.transposed,
                       (float*)(base + L.stage));
    hipLaunchKernelGGL(rank_perm_kernel, dim3((L.nw + 255) / 256), dim3(256), 0, s,
                       (const float*)(base + L.stage), L.nw, (int*)(base + L.cperm));
  } else {
    hipLaunchKernelGGL(iota_kernel, dim3((L.nw + 255) / 256), dim3(256), 0, s,
                       (int*)(base + L.cperm), L.nw);
  }
  HIPCHK(hipGetLastError());
  {
    dim3 grid((L.ldn + 255) / 256, L.ldm);
    hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, s, R, M, L.n, L.mw, L.nw, L.ldm, L.ldn,
                       L.transposed, (const int*)(base + L.perm), (const int*)(base + L.cperm),
                       (float*)(base + L.Rw));
    dim3 tg(L.ldn / TS, L.ldm / TS);
    hipLaunchKernelGGL(transpose_kernel, tg, dim3(256), 0, s, (const float*)(base + L.Rw), L.ldm,
                       L.ldn, (float*)(base + L.RwT));
  }
  if (o.init_mode == 1) {
    HIPCHK(hipMemcpyAsync(base + L.stage, cols.data(), cols.size() * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(u0_acol_kernel, dim3((L.ldm + 255) / 256), dim3(256), 0, s,
                       (const float*)(base + L.Rw), L.mw, L.nw, L.ldm, L.ldn, L.r, o.acol_p,
                       (const int*)(base + L.stage), (float*)(base + L.Uc));
  } else {
    HIPCHK(hipMemcpyAsync(base + L.stage, U0.data(), U0.size() * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(u0_given_kernel, dim3((L.ldm + 255) / 256, L.r), dim3(256), 0, s,
                       (const float*)(base + L.stage), L.mw, L.r, L.ldm, (float*)(base + L.Uc));
  }
  hipLaunchKernelGGL(vinit_kernel, dim3((L.ldn + 255) / 256, L.r), dim3(256), 0, s,
                     (const float*)(base + L.Rw), (const float*)(base + L.Uc), L.mw, L.nw, L.ldm,
                     L.ldn, L.r, (float*)(base + L.V));
  HIPCHK(hipGetLastError());
  int st = fill_u32(base + L.ctl, sizeof(FitCtl) / 4, 0, s);
  if (!st) st = fill_u32(base + L.bar, sizeof(BarTree) / 4, 0, s);
  if (!st) st = fill_u32(base + L.closed, (size_t)L.r, 0, s);
  if (!st) st = fill_u32(base + L.rowt, (size_t)L.mw, 0, s);
  if (!st) st = fill_u32(base + L.traj, (size_t)(L.iters + 1) * 2, 0, s);
  return st;
}

static int launch_output(const Layout& L, char* base, float* U_out, float* V_out, hipStream_t s) {
  const int mx = std::max(L.mw, L.nw);
  hipLaunchKernelGGL(output_kernel, dim3((mx + 255) / 256, L.r), dim3(256), 0, s,
                     (const float*)(base + L.Uc), (const float*)(base + L.V), L.mw, L.nw, L.ldm,
                     L.ldn, L.r, L.transposed, (const int*)(base + L.perm),
                     (const int*)(base + L.cperm), U_out, V_out);
  return hipGetLastError() == hipSuccess ? STMF_OK : STMF_EHIP;
}

// sel: the ByRow selection of every fit of the launch (TD_A runs the kernel
// compiled for it alone, in its own build for launches with a fit wider than
// SORT_MAX columns: `wide`).  queue: the grid is cut into groups of qgroup
// workgroups that take fits from the queue one after another, each group
// publishing its fit through its control block in gctl (zeroed before the
// launch); null: the fits own consecutive ranges of gsize workgroups.  Every
// launch is a plain one whose grid stays within the co-resident count (one
// fit-kernel workgroup per CU: its LDS takes most of a CU's), so on an
// otherwise idle device every group is resident at once; the group
// barrier's bounded wait turns anything else into STMF_ETIMEOUT.  (No
// cooperative launch: it adds nothing the bounded wait does not cover, and
// a process that made one ended with a segmentation fault at exit under the
// profiler.)
static int launch_fit_kernel(const FitDev* dev_fits, int nfits, int grid, int max_rows,
                             unsigned* queue, int qgroup, FitCtl* gctl, BarTree* gbar, int sel,
                             bool wide, hipStream_t s) {
  const size_t smem = fit_smem_bytes();
  const void* k = sel == SEL_TD_A     ? (wide ? (const void*)fit_kernel_wide : (const void*)fit_kernel)
                  : sel == SEL_MATRIX ? (const void*)fit_kernel_matrix
                                      : (const void*)fit_kernel_sel;
  void* args[] = {(void*)&dev_fits, (void*)&nfits, (void*)&max_rows, (void*)&queue,
                  (void*)&qgroup,   (void*)&gctl,  (void*)&gbar};
  HIPCHK(hipLaunchKernel(k, dim3(grid), dim3(NTHR), args, smem, s));
  return STMF_OK;
}

static void fill_info(stmf_fit_info* info, const FitCtl& c, const Layout& L) {
  if (!info) return;
  info->trials += c.trials;
  info->spec_trials += c.spec_trials;
  info->noops += c.noops;
  info->accepted += c.accepted;
  info->row_visits += c.row_visits;
  info->cells += c.cells;
  info->iters_done = c.iters_done;
  info->transposed = L.transposed;
  info->m_work = L.mw;
  info->n_work = L.nw;
  info->group_size = L.G;
  info->nlog += c.nlog;
  info->batches += c.batches;
  for (int q = 0; q < 8; ++q) info->phase_ms[q] += (double)c.phase_ticks[q] * 1e-5;
}

static int auto_group(const Layout& L, const DevProps& P, int requested) {
  const int ntiles = L.nrt * L.nct;
  int G = requested > 0 ? requested : ntiles;
  G = std::min(G, ntiles);
  G = std::min(G, P.coresident);
  return std::max(G, 1);
}

}  // namespace stmf

using namespace stmf;

// ================================================================ C ABI
extern "C" {

const char* stmf_status_str(int s) {
  switch (s) {
    case STMF_OK: return "ok";
    case STMF_EINVAL: return "invalid argument";
    case STMF_EEMPTY_LINE: return "a row or column has no observed cell";
    case STMF_ERANGE: return "value out of the supported range";
    case STMF_ENOMEM: return "workspace too small or misaligned";
    case STMF_EHIP: return "HIP runtime error";
    case STMF_EBUSY: return "no free slot or memory";
    case STMF_ETIMEOUT: return "fit timed out at a group barrier";
    default: return "unknown status";
  }
}

const char* stmf_version(void) { return "0.1.0"; }

void stmf_options_default(stmf_options* o) {
  if (o) options_default(o);
}

int stmf_maxplus_product(const float* U, const float* V, int m, int r, int n, float* P,
                         int32_t* argmax, void* stream) {
  if (!U || !V || (!P && !argmax) || m < 1 || n < 1 || r < 1 || r > RMAX) return STMF_EINVAL;
  HIPCHK(launch_maxplus(U, V, m, r, n, P, argmax, (hipStream_t)stream));
  return STMF_OK;
}

size_t stmf_masked_error_workspace(int m, int n, int r) {
  (void)r;
  if (m < 1 || n < 1) return 0;
  return masked_error_ws(m, n);
}

int stmf_masked_error(const float* R, const uint8_t* M, const float* U, const float* V, int m,
                      int n, int r, double* err, double* td_col, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!R || !M || !U || !V || !err || m < 1 || n < 1 || r < 1 || r > RMAX) return STMF_EINVAL;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < masked_error_ws(m, n)) return STMF_ENOMEM;
  HIPCHK(launch_masked_error(R, M, U, V, m, n, r, err, td_col, ws, (hipStream_t)stream));
  return STMF_OK;
}

size_t stmf_update_workspace(int m, int n, int r) { return stmf_masked_error_workspace(m, n, r); }

static int update_common(int op, const float* R, const uint8_t* M, float* U, float* V, int m, int n,
                         int r, int i, int j, int k, float* Ub, float* Vb, double* err, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!R || !M || !U || !V || !Ub || !Vb || !err || m < 1 || n < 1 || r < 1 || r > RMAX)
    return STMF_EINVAL;
  if (i < 0 || i >= m || j < 0 || j >= n || k < 0 || k >= r) return STMF_EINVAL;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < masked_error_ws(m, n)) return STMF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  // a residual over a row or column with no observed cell is undefined: the
  // mask is read back and every line checked before anything is launched
  std::vector<uint8_t> hm((size_t)m * n);
  HIPCHK(hipMemcpyAsync(hm.data(), M, hm.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<char> col_seen(n, 0);
  for (int t = 0; t < m; ++t) {
    bool row_seen = false;
    for (int c = 0; c < n; ++c)
      if (hm[(size_t)t * n + c]) { row_seen = true; col_seen[c] = 1; }
    if (!row_seen) return STMF_EEMPTY_LINE;
  }
  for (int c = 0; c < n; ++c)
    if (!col_seen[c]) return STMF_EEMPTY_LINE;
  const uint8_t obs = hm[(size_t)i * n + j];
  if (!obs) return STMF_EINVAL;
  HIPCHK(launch_update(op, R, M, U, V, m, n, r, i, j, k, Ub, Vb, err, ws, s));
  return STMF_OK;
}

int stmf_update_U(const float* R, const uint8_t* M, float* U, float* V, int m, int n, int r, int i,
                  int j, int k, float* Ub, float* Vb, double* err, void* ws, size_t ws_bytes,
                  void* stream) {
  return update_common(0, R, M, U, V, m, n, r, i, j, k, Ub, Vb, err, ws, ws_bytes, stream);
}

int stmf_update_V(const float* R, const uint8_t* M, float* U, float* V, int m, int n, int r, int i,
                  int j, int k, float* Ub, float* Vb, double* err, void* ws, size_t ws_bytes,
                  void* stream) {
  return update_common(1, R, M, U, V, m, n, r, i, j, k, Ub, Vb, err, ws, ws_bytes, stream);
}

static int resolve(const stmf_options* opt, stmf_options& o) {
  if (opt) o = *opt; else options_default(&o);
  return check_options(o);
}

size_t stmf_fit_workspace(int m, int n, int rank, int iters, const stmf_options* opt) {
  stmf_options o;
  if (resolve(opt, o) || m < 1 || n < 1 || rank < 1 || rank > RMAX || iters < 0) return 0;
  DevProps P;
  if (device_props(P)) return 0;
  Layout L;
  make_layout(m, n, rank, iters, 1, o.acol_p, o.batch_max, L, o.strategy == 2);
  const int G = auto_group(L, P, o.group_size);
  make_layout(m, n, rank, iters, G, o.acol_p, o.batch_max, L, o.strategy == 2);
  return L.total;
}

int stmf_draw_init(int m, int n, int rank, uint64_t seed, const stmf_options* opt,
                   int32_t* perm_out, float* U0_out) {
  stmf_options o;
  int st = resolve(opt, o);
  if (st) return st;
  if (m < 1 || n < 1 || rank < 1 || rank > RMAX) return STMF_EINVAL;
  if (o.perm_mode == 1 && !o.perm) return STMF_EINVAL;  // the PermR order is not a draw
  Layout L;
  make_layout(m, n, rank, 0, 1, o.acol_p, o.batch_max, L);
  std::vector<int32_t> perm, cols;
  std::vector<float> U0;
  st = draw_setup(L, seed, o, perm, U0, cols);
  if (st) return st;
  if (perm_out) std::memcpy(perm_out, perm.data(), perm.size() * 4);
  if (U0_out) {
    if (o.init_mode == 1)
      for (size_t q = 0; q < cols.size(); ++q) U0_out[q] = (float)cols[q];
    else
      std::memcpy(U0_out, U0.data(), U0.size() * 4);
  }
  return STMF_OK;
}

int stmf_fit(const float* R, const uint8_t* M, int m, int n, int rank, int iters, uint64_t seed,
             float* U_out, float* V_out, double* err_traj, const stmf_options* opt,
             stmf_fit_info* info, void* ws, size_t ws_bytes, void* stream) {
  stmf_options o;
  int st = resolve(opt, o);
  if (st) return st;
  if (!R || !M || !U_out || !V_out || m < 1 || n < 1 || rank < 1 || rank > RMAX || iters < 0)
    return STMF_EINVAL;
  if (o.decision_log && o.log_cap <= 0) return STMF_EINVAL;
  DevProps P;
  st = device_props(P);
  if (st) return st;
  Layout L;
  make_layout(m, n, rank, iters, 1, o.acol_p, o.batch_max, L, o.strategy == 2);
  const int G = auto_group(L, P, o.group_size);
  make_layout(m, n, rank, iters, G, o.acol_p, o.batch_max, L, o.strategy == 2);
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < L.total) return STMF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  int observed = 0;
  st = check_inputs(R, M, L, base, o.integer_exact, s, &observed);
  if (st) return st;
  std::vector<int32_t> perm, cols;
  std::vector<float> U0;
  st = draw_setup(L, seed, o, perm, U0, cols);
  if (st) return st;
  st = prepare_fit(R, M, L, base, o, perm, U0, cols, s);
  if (st) return st;
  FitDev d = make_dev(L, base, o, observed);
  d.seed_ops = seed ^ MATRIX_OP_STREAM;
  HIPCHK(hipMemcpyAsync(base + L.dev, &d, sizeof(d), hipMemcpyHostToDevice, s));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, s));
  st = launch_fit_kernel((const FitDev*)(base + L.dev), 1, G, o.max_row_visits, nullptr, 1,
                         nullptr, nullptr, kernel_sel(o), L.nw > SORT_MAX, s);
  if (st) { (void)hipEventDestroy(ev0); (void)hipEventDestroy(ev1); return st; }
  HIPCHK(hipEventRecord(ev1, s));
  FitCtl c;
  HIPCHK(hipMemcpyAsync(&c, base + L.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float kms = 0.0f;
  if (hipEventElapsedTime(&kms, ev0, ev1) != hipSuccess) kms = 0.0f;
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (c.status == STMF_ETIMEOUT) return STMF_ETIMEOUT;
  if (c.status != 0) return STMF_EHIP;
  st = launch_output(L, base, U_out, V_out, s);
  if (st) return st;
  if (err_traj)
    HIPCHK(hipMemcpyAsync(err_traj, base + L.traj, (size_t)(iters + 1) * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    fill_info(info, c, L);
    info->kernel_ms = kms;
  }
  return STMF_OK;
}

// ---------------------------------------------------------------- batched
struct BatchPlan {
  std::vector<Layout> L;       // one per fit (problem-major, restart-minor)
  std::vector<size_t> off;     // workspace offset of each fit
  std::vector<int> prob;       // problem of each fit
  std::vector<uint64_t> seed;  // seed of each fit
  int qgroup = 1;              // workgroups per group of the persistent launch
  int ngroups = 1;             // groups in the launch
  size_t table, queue, gctl, gbar, total;
};

// Estimated work of a fit, for ordering the queue (largest first) and
// sizing groups: rows visited per pass x tiles swept per trial x rank.
static double fit_work(const Layout& L) {
  return (double)L.mw * (double)(L.nrt * L.nct) * (double)L.r;
}

// Workgroups per fit when the caller leaves it to the library.  A fit's time
// scales with its group (measured: the same CU-time on groups of 4 to 64),
// so with fits handed out largest first the launch ends no sooner than
// W / (co-resident count) or w_max / G (W the total, w_max the largest
// fit's work).  G is the power of two at or above 4 co-resident w_max / W
// (a margin for the work estimate), between 1 and 64 and at most the largest
// fit's tiles.
static int auto_qgroup(double w_total, double w_max, int max_tiles, int coresident) {
  const double want = 4.0 * coresident * w_max / std::max(w_total, 1.0);
  int g = 1;
  while (g < want && g * 2 <= 64 && g * 2 <= max_tiles) g *= 2;
  return g;
}

static void plan_batched(const stmf_problem* probs, int nprob, int restarts, const stmf_options& o,
                         int coresident, BatchPlan& B) {
  const int F = nprob * restarts;
  int max_tiles = 1;
  double w_total = 0.0, w_max = 0.0;
  for (int p = 0; p < nprob; ++p) {
    Layout L;
    make_layout(probs[p].m, probs[p].n, probs[p].rank, probs[p].iters, 1, o.acol_p, o.batch_max, L);
    max_tiles = std::max(max_tiles, L.nrt * L.nct);
    w_total += restarts * fit_work(L);
    w_max = std::max(w_max, fit_work(L));
  }
  B.qgroup = o.group_size > 0 ? std::min(o.group_size, coresident)
                              : auto_qgroup(w_total, w_max, max_tiles, coresident);
  B.ngroups = std::max(1, std::min(coresident / B.qgroup, F));
  size_t o_ = 0;
  for (int p = 0; p < nprob; ++p) {
    Rng g{probs[p].seed};
    for (int q = 0; q < restarts; ++q) {
      // a fit's layout takes its group (the batch sizes depend on it; its
      // results do not)
      Layout L;
      make_layout(probs[p].m, probs[p].n, probs[p].rank, probs[p].iters, 1, o.acol_p, o.batch_max, L);
      const int G = std::min(B.qgroup, L.nrt * L.nct);
      if (G > 1)
        make_layout(probs[p].m, probs[p].n, probs[p].rank, probs[p].iters, G, o.acol_p,
                    o.batch_max, L);
      B.L.push_back(L);
      B.off.push_back(o_);
      B.prob.push_back(p);
      B.seed.push_back(restarts == 1 ? probs[p].seed : g.next());
      o_ += L.total;
    }
  }
  B.table = o_;
  o_ += al256(B.L.size() * sizeof(FitDev));
  B.queue = o_;
  o_ += 256;
  B.gctl = o_;
  o_ += al256((size_t)B.ngroups * sizeof(FitCtl));
  B.gbar = o_;
  o_ += al256((size_t)B.ngroups * sizeof(BarTree));
  B.total = o_;
}

// Whether a launch over these fits takes the wide build of the TD_A kernel.
static bool any_wide(const FitDev* fits, int n) {
  for (int f = 0; f < n; ++f)
    if (fits[f].n > SORT_MAX) return true;
  return false;
}

// The device side of a batched call, recorded on stream c: queue and group
// control blocks cleared by fill kernels, the persistent fit launch, then the
// output (un-permuted, un-transposed factors) and trajectory of every fit.
static int record_batched(const BatchPlan& B, const std::vector<int>& fit_ids,
                          const std::vector<FitDev>& table, stmf_problem* probs, int restarts,
                          char* base, int sel, int max_rows, hipStream_t c) {
  int st = fill_u32(base + B.queue, 1, 0, c);
  if (!st) st = fill_u32(base + B.gctl, (size_t)B.ngroups * sizeof(FitCtl) / 4, 0, c);
  if (!st) st = fill_u32(base + B.gbar, (size_t)B.ngroups * sizeof(BarTree) / 4, 0, c);
  if (st) return st;
  const int n = (int)table.size();
  const int ngroups = std::min(B.ngroups, n);
  st = launch_fit_kernel((const FitDev*)(base + B.table), n, ngroups * B.qgroup, max_rows,
                         (unsigned*)(base + B.queue), B.qgroup, (FitCtl*)(base + B.gctl),
                         (BarTree*)(base + B.gbar), sel,
                         any_wide(table.data(), n), c);
  if (st) return st;
  for (int f : fit_ids) {
    const Layout& L = B.L[f];
    char* fb = base + B.off[f];
    const int p = B.prob[f];
    const int q = f - p * restarts;
    float* Uo = probs[p].U_out + (size_t)q * L.m * L.r;
    float* Vo = probs[p].V_out + (size_t)q * L.r * L.n;
    st = launch_output(L, fb, Uo, Vo, c);
    if (st) return st;
    if (probs[p].err_traj)
      hipLaunchKernelGGL(copy_f64_kernel, dim3((L.iters + 1 + 255) / 256), dim3(256), 0, c,
                         (const double*)(fb + L.traj), probs[p].err_traj + (size_t)q * (L.iters + 1),
                         L.iters + 1);
  }
  HIPCHK(hipGetLastError());
  return STMF_OK;
}

size_t stmf_fit_batched_workspace(const stmf_problem* probs, int nprob, int restarts,
                                  const stmf_options* opt) {
  stmf_options o;
  if (resolve(opt, o) || !probs || nprob < 1 || restarts < 1) return 0;
  for (int p = 0; p < nprob; ++p)
    if (probs[p].m < 1 || probs[p].n < 1 || probs[p].rank < 1 || probs[p].rank > RMAX ||
        probs[p].iters < 0)
      return 0;
  DevProps P;
  if (device_props(P)) return 0;
  BatchPlan B;
  plan_batched(probs, nprob, restarts, o, P.coresident, B);
  return B.total;
}

int stmf_fit_batched(stmf_problem* probs, int nprob, int restarts, const stmf_options* opt,
                     stmf_fit_info* info, void* ws, size_t ws_bytes, void* stream) {
  stmf_options o;
  int st = resolve(opt, o);
  if (st) return st;
  if (!probs || nprob < 1 || restarts < 1) return STMF_EINVAL;
  if (o.decision_log || o.perm || o.init_mode == 2 || o.max_row_visits < 0) return STMF_EINVAL;
  if (o.strategy == 2) return STMF_EINVAL;  // ByMatrix runs through stmf_fit only
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].R || !probs[p].M || !probs[p].U_out || !probs[p].V_out || probs[p].m < 1 ||
        probs[p].n < 1 || probs[p].rank < 1 || probs[p].rank > RMAX || probs[p].iters < 0)
      return STMF_EINVAL;
  DevProps P;
  st = device_props(P);
  if (st) return st;
  BatchPlan B;
  plan_batched(probs, nprob, restarts, o, P.coresident, B);
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < B.total) return STMF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  const int F = (int)B.L.size();
  // input checks, one problem at a time (restarts share the input)
  std::vector<int> observed(nprob, 0);
  for (int p = 0; p < nprob; ++p) {
    int first = p * restarts;
    probs[p].status = check_inputs(probs[p].R, probs[p].M, B.L[first], base + B.off[first],
                                   o.integer_exact, s, &observed[p]);
  }
  std::vector<FitDev> table;
  std::vector<std::vector<int32_t>> perms(F), colss(F);
  std::vector<std::vector<float>> U0s(F);
  std::vector<int> fit_ids;
  for (int f = 0; f < F; ++f) {
    const int p = B.prob[f];
    if (probs[p].status) continue;
    const Layout& L = B.L[f];
    char* fb = base + B.off[f];
    int s2 = draw_setup(L, B.seed[f], o, perms[f], U0s[f], colss[f]);
    if (!s2) s2 = prepare_fit(probs[p].R, probs[p].M, L, fb, o, perms[f], U0s[f], colss[f], s);
    if (s2) { probs[p].status = s2; continue; }
    fit_ids.push_back(f);
  }
  // largest fits first (the queue hands them out in table order)
  std::stable_sort(fit_ids.begin(), fit_ids.end(),
                   [&](int a, int b) { return fit_work(B.L[a]) > fit_work(B.L[b]); });
  for (int f : fit_ids) table.push_back(make_dev(B.L[f], base + B.off[f], o, observed[B.prob[f]]));
  if (!table.empty()) {
    HIPCHK(hipMemcpyAsync(base + B.table, table.data(), table.size() * sizeof(FitDev),
                          hipMemcpyHostToDevice, s));
    // the whole device side (one persistent launch and the outputs) as one
    // captured graph, launched on the caller's stream
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    auto cleanup = [&]() {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (graph) (void)hipGraphDestroy(graph);
      if (cap) (void)hipStreamDestroy(cap);
    };
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) { cleanup(); return STMF_EHIP; }
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      cleanup();
      return STMF_EHIP;
    }
    st = record_batched(B, fit_ids, table, probs, restarts, base, kernel_sel(o), o.max_row_visits,
                        cap);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(cap, &g);
    graph = g;
    if (st || ce != hipSuccess) { cleanup(); return st ? st : STMF_EHIP; }
    if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess ||
        hipGraphLaunch(gexec, s) != hipSuccess) {
      cleanup();
      return STMF_EHIP;
    }
    const hipError_t se = hipStreamSynchronize(s);  // host staging vectors go out of scope after this
    cleanup();
    if (se != hipSuccess) return STMF_EHIP;
  } else {
    HIPCHK(hipStreamSynchronize(s));
  }
  if (info) std::memset(info, 0, sizeof(*info));
  for (int f : fit_ids) {
    const Layout& L = B.L[f];
    char* fb = base + B.off[f];
    const int p = B.prob[f];
    FitCtl c;
    HIPCHK(hipMemcpyAsync(&c, fb + L.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c.status) { probs[p].status = c.status == STMF_ETIMEOUT ? STMF_ETIMEOUT : STMF_EHIP; continue; }
    fill_info(info, c, L);
  }
  if (info) info->group_size = B.qgroup;
  return STMF_OK;
}

}  // extern "C"

// ================================================================ serving
// A continuous-batching engine: jobs are admitted into slots of a
// caller-owned arena (first-fit over a free list, by footprint), each tick
// advances every active job by a bounded number of row visits (state kept in
// the arena between ticks), and finished jobs are retired to free their
// memory for new admissions.  A job runs on a group of G workgroups, G the
// smaller of the engine's group size (0: the co-resident count) and the
// job's tile count, fixed at admission: its result is that of stmf_fit with
// group_size G, which is stmf_fit's own choice when the group size is 0.  With G = 1
// for every job a tick is one launch whose workgroups take jobs from a
// queue; otherwise the jobs are laid side by side over the grid, as many
// per launch as the co-resident workgroups hold, in slot order.
struct stmf_engine {
  char* arena = nullptr;
  size_t bytes = 0;
  int max_slots = 0;
  int gcap = 1;        // workgroups per job, at most
  int coresident = 0;  // fit-kernel workgroups resident at once
  stmf_options opt;
  size_t table_off = 0, queue_off = 0, gctl_off = 0, heap_off = 0;
  struct Slot {
    bool used = false;
    size_t off = 0, len = 0;
    Layout L;
    FitDev dev;
    int G = 1;
    std::vector<int32_t> perm, cols;
    std::vector<float> U0;
  };
  std::vector<Slot> slots;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, length), by offset
  std::mutex mu;
  // A tick is a captured graph (queue reset by a fill kernel and one fit
  // launch, or one fit launch per pack of jobs), re-captured when its launch
  // plan changes; the device table of resident jobs is uploaded only when the
  // resident set changes.
  bool use_graph = true;
  std::vector<FitDev> uploaded;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> g_plan;  // the captured plan (first, count, grid, wide per launch)
  int g_rows = -1, g_sel = -1;
  ~stmf_engine() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

static bool arena_alloc(stmf_engine* e, size_t len, size_t& off) {
  for (size_t q = 0; q < e->free_list.size(); ++q) {
    auto& fb = e->free_list[q];
    if (fb.second >= len) {
      off = fb.first;
      fb.first += len;
      fb.second -= len;
      if (!fb.second) e->free_list.erase(e->free_list.begin() + q);
      return true;
    }
  }
  return false;
}

static void arena_free(stmf_engine* e, size_t off, size_t len) {
  auto& F = e->free_list;
  auto it = std::lower_bound(F.begin(), F.end(), std::make_pair(off, (size_t)0));
  it = F.insert(it, {off, len});
  // merge with the next and previous blocks
  size_t q = (size_t)(it - F.begin());
  if (q + 1 < F.size() && F[q].first + F[q].second == F[q + 1].first) {
    F[q].second += F[q + 1].second;
    F.erase(F.begin() + q + 1);
  }
  if (q > 0 && F[q - 1].first + F[q - 1].second == F[q].first) {
    F[q - 1].second += F[q].second;
    F.erase(F.begin() + q);
  }
}

extern "C" {

size_t stmf_job_footprint(int m, int n, int rank, int iters) {
  if (m < 1 || n < 1 || rank < 1 || rank > RMAX || iters < 0) return 0;
  Layout L;
  make_layout(m, n, rank, iters, 1, 5, 0, L);
  return L.total;
}

size_t stmf_engine_job_footprint(const stmf_engine* e, int m, int n, int rank, int iters) {
  if (!e || m < 1 || n < 1 || rank < 1 || rank > RMAX || iters < 0) return 0;
  Layout L;
  make_layout(m, n, rank, iters, 1, e->opt.acol_p, e->opt.batch_max, L);
  const int G = std::min(e->gcap, L.nrt * L.nct);
  if (G > 1) make_layout(m, n, rank, iters, G, e->opt.acol_p, e->opt.batch_max, L);
  return L.total;
}

int stmf_engine_create(void* ws, size_t ws_bytes, int max_slots, const stmf_options* opt,
                       stmf_engine** out) {
  if (!out || max_slots < 1) return STMF_EINVAL;
  stmf_options o;
  int st = resolve(opt, o);
  if (st) return st;
  if (o.decision_log || o.perm || o.init_mode == 2 || o.max_row_visits) return STMF_EINVAL;
  if (o.strategy == 2) return STMF_EINVAL;  // ByMatrix runs through stmf_fit only
  if (!ws || ((uintptr_t)ws & 255)) return STMF_ENOMEM;
  DevProps P;
  st = device_props(P);
  if (st) return st;
  const size_t table = al256((size_t)max_slots * sizeof(FitDev));
  // control blocks of the one-workgroup groups of a queue launch
  const size_t gctl = al256((size_t)P.coresident * sizeof(FitCtl));
  if (ws_bytes < table + 256 + gctl + 256) return STMF_ENOMEM;
  stmf_engine* e = new (std::nothrow) stmf_engine();
  if (!e) return STMF_ENOMEM;
  e->arena = (char*)ws;
  e->bytes = ws_bytes;
  e->max_slots = max_slots;
  // group_size 0: as stmf_fit, every job on as many workgroups as it has tiles
  e->gcap = o.group_size > 0 ? std::min(o.group_size, P.coresident) : P.coresident;
  e->coresident = P.coresident;
  e->opt = o;
  e->table_off = 0;
  e->queue_off = table;
  e->gctl_off = table + 256;
  e->heap_off = table + 256 + gctl;
  e->slots.resize(max_slots);
  e->free_list.push_back({e->heap_off, (ws_bytes - e->heap_off) / 256 * 256});
  *out = e;
  return STMF_OK;
}

void stmf_engine_destroy(stmf_engine* e) { delete e; }

int stmf_engine_admit(stmf_engine* e, const float* R, const uint8_t* M, int m, int n, int rank,
                      int iters, uint64_t seed, int* slot, void* stream) {
  if (!e || !R || !M || !slot || m < 1 || n < 1 || rank < 1 || rank > RMAX || iters < 0)
    return STMF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  int sidx = -1;
  for (int q = 0; q < e->max_slots; ++q)
    if (!e->slots[q].used) { sidx = q; break; }
  if (sidx < 0) return STMF_EBUSY;
  stmf_engine::Slot& S = e->slots[sidx];
  make_layout(m, n, rank, iters, 1, e->opt.acol_p, e->opt.batch_max, S.L);
  const int G = std::min(e->gcap, S.L.nrt * S.L.nct);
  if (G > 1) make_layout(m, n, rank, iters, G, e->opt.acol_p, e->opt.batch_max, S.L);
  size_t off = 0;
  if (!arena_alloc(e, S.L.total, off)) return STMF_EBUSY;
  hipStream_t s = (hipStream_t)stream;
  char* base = e->arena + off;
  int observed = 0;
  int st = check_inputs(R, M, S.L, base, e->opt.integer_exact, s, &observed);
  if (!st) st = draw_setup(S.L, seed, e->opt, S.perm, S.U0, S.cols);
  if (!st) st = prepare_fit(R, M, S.L, base, e->opt, S.perm, S.U0, S.cols, s);
  if (st) {
    arena_free(e, off, S.L.total);
    return st;
  }
  S.used = true;
  S.G = G;
  S.off = off;
  S.len = S.L.total;
  S.dev = make_dev(S.L, base, e->opt, observed);
  *slot = sidx;
  return STMF_OK;
}

// The tick's launches on stream s.  plan: (first, count, grid, wide) per
// launch; a grid of -1 marks the queue launch of one-workgroup jobs (queue
// reset by a fill kernel, then the fit kernel over every job).
static int tick_work(stmf_engine* e, const std::vector<int>& plan, int max_rows, hipStream_t s) {
  const FitDev* table = (const FitDev*)(e->arena + e->table_off);
  const int sel = kernel_sel(e->opt);
  for (size_t q = 0; q < plan.size(); q += 4) {
    const int first = plan[q], count = plan[q + 1], grid = plan[q + 2];
    const bool wide = plan[q + 3] != 0;
    int st;
    if (grid < 0) {
      const int groups = std::min(count, e->coresident);
      st = fill_u32(e->arena + e->queue_off, 1, 0, s);
      if (!st) st = fill_u32(e->arena + e->gctl_off, (size_t)groups * sizeof(FitCtl) / 4, 0, s);
      if (!st)
        st = launch_fit_kernel(table + first, count, groups, max_rows,
                               (unsigned*)(e->arena + e->queue_off), 1,
                               (FitCtl*)(e->arena + e->gctl_off), nullptr, sel, wide, s);
    } else {
      // every group of the launch is resident at once: grid <= coresident
      st = launch_fit_kernel(table + first, count, grid, max_rows, nullptr, 1, nullptr, nullptr,
                             sel, wide, s);
    }
    if (st) return st;
  }
  return STMF_OK;
}

int stmf_batch_tick(stmf_engine* e, int max_rows, void* stream) {
  if (!e || max_rows < 0) return STMF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  std::vector<FitDev> table;
  std::vector<int> gs;
  for (auto& S : e->slots)
    if (S.used) { table.push_back(S.dev); gs.push_back(S.G); }
  if (table.empty()) return STMF_OK;
  hipStream_t s = (hipStream_t)stream;
  const int nfits = (int)table.size();
  if (table.size() != e->uploaded.size() ||
      std::memcmp(table.data(), e->uploaded.data(), table.size() * sizeof(FitDev)) != 0) {
    HIPCHK(hipMemcpyAsync(e->arena + e->table_off, table.data(), table.size() * sizeof(FitDev),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    e->uploaded = table;
  }
  std::vector<int> plan;
  if (e->gcap == 1) {
    plan = {0, nfits, -1, any_wide(table.data(), nfits) ? 1 : 0};
  } else {
    int first = 0, grid = 0;
    for (int f = 0; f <= nfits; ++f) {
      if (f == nfits || grid + gs[f] > e->coresident) {
        plan.insert(plan.end(),
                    {first, f - first, grid, any_wide(table.data() + first, f - first) ? 1 : 0});
        first = f;
        grid = 0;
      }
      if (f < nfits) grid += gs[f];
    }
  }
  int st;
  if (!e->use_graph) {
    st = tick_work(e, plan, max_rows, s);
    if (st) return st;
  } else {
    const int sel = kernel_sel(e->opt);
    if (!e->gexec || e->g_plan != plan || e->g_rows != max_rows || e->g_sel != sel) {
      if (e->gexec) { HIPCHK(hipGraphExecDestroy(e->gexec)); e->gexec = nullptr; }
      if (e->graph) { HIPCHK(hipGraphDestroy(e->graph)); e->graph = nullptr; }
      e->g_plan.clear();
      if (!e->cap) HIPCHK(hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
      st = tick_work(e, plan, max_rows, e->cap);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(e->cap, &g);
      if (st) { if (g) (void)hipGraphDestroy(g); return st; }
      if (ec != hipSuccess) return STMF_EHIP;
      e->graph = g;
      HIPCHK(hipGraphInstantiate(&e->gexec, e->graph, nullptr, nullptr, 0));
      e->g_plan = plan; e->g_rows = max_rows; e->g_sel = sel;
    }
    HIPCHK(hipGraphLaunch(e->gexec, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return STMF_OK;
}

int stmf_engine_set_graph(stmf_engine* e, int on) {
  if (!e) return STMF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  e->use_graph = on != 0;
  return STMF_OK;
}

int stmf_engine_poll(stmf_engine* e, int slot, int* done, void* stream) {
  if (!e || !done || slot < 0 || slot >= e->max_slots) return STMF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  stmf_engine::Slot& S = e->slots[slot];
  if (!S.used) return STMF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  FitCtl c;
  HIPCHK(hipMemcpyAsync(&c, e->arena + S.off + S.L.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (c.status) return c.status == STMF_ETIMEOUT ? STMF_ETIMEOUT : STMF_EHIP;
  *done = c.phase == 2;
  return STMF_OK;
}

int stmf_engine_retire(stmf_engine* e, int slot, float* U_out, float* V_out, double* err_traj,
                       stmf_fit_info* info, void* stream) {
  if (!e || slot < 0 || slot >= e->max_slots) return STMF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  stmf_engine::Slot& S = e->slots[slot];
  if (!S.used) return STMF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* base = e->arena + S.off;
  int st = STMF_OK;
  if (U_out && V_out) {
    FitCtl c;
    HIPCHK(hipMemcpyAsync(&c, base + S.L.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c.phase != 2) return STMF_EINVAL;
    st = launch_output(S.L, base, U_out, V_out, s);
    if (st) return st;
    if (err_traj)
      HIPCHK(hipMemcpyAsync(err_traj, base + S.L.traj, (size_t)(S.L.iters + 1) * 8,
                            hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (info) {
      std::memset(info, 0, sizeof(*info));
      fill_info(info, c, S.L);
    }
  }
  arena_free(e, S.off, S.len);
  S.used = false;
  S.perm.clear(); S.U0.clear(); S.cols.clear();
  return st;
}

}  // extern "C"
