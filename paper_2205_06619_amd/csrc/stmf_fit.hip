// FastSTMF fit engine for gfx950: one persistent kernel runs Algorithm 3
// (ByRow, random row permutation, TD_A, wide orientation) on device, with no
// host round trip per trial.
//
// A "group" of G workgroups owns one fit (G = 1 for batched fits, up to one
// per tile for a served job or one fit, at most the whole chip).  The working
// matrix is cut into 64 x 64 tiles; workgroup g of the group takes tiles
// g, g + G, ...
//
// Every trial of a row visit starts from the same state (a rejected F-ULF or
// F-URF restores U_.k and V_k., Algorithm 3), so the trials of a row are
// independent and are evaluated in speculative batches; the first trial in
// the method's order (candidate by td_col descending, F-ULF before F-URF)
// whose error strictly decreases is the one the method accepts.  This is
// exact: no trial's outcome depends on another's.
//
// Per trial (i, j, k):
//   F-ULF (Algorithm 1): u = R_ij - V_kj; V'_k. = column residual of U with
//     U_ik = u, which differs from the current one only through row i:
//     V'_kc = min(min_{t != i} (R_tc - U_tk), R_ic - u), taken from a top-2
//     summary per column (exact: min is exact); then U''_.k = row residual of
//     V'_k. (one pass, atomic min across tiles; exact) and the b-norm.
//   F-URF (Algorithm 2): the mirror image with rows and columns swapped.
//   The new product is P' = max(P without k, U''_tk + V'_kc), bit-identical
//   to a full max over components (max is exact and order-free).
// Every value operation is one correctly rounded FP32 operation; |R - P'| is
// widened to FP64 and summed in a fixed order (lane, row, tile, chunks of
// tiles, a tree over the chunks) that depends on the working shape alone, so
// a trial's error depends only on the state and the trial, never on how many
// workgroups share the fit.
//
// Per row visit: batches (residual pass, group barrier, error pass, group
// barrier with the decision taken by the last workgroup to arrive); after an
// acceptance the refresh pass (new component written, argmax counts, td_col
// partials, residual summaries of the component), one barrier, the summary
// combine while one workgroup sorts the columns by td_col, one barrier.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#define STMF_FIT_KERNEL_TU
#include "stmf_internal.h"

namespace stmf {

#define DEV __device__ __forceinline__

static constexpr float FINF = __builtin_huge_valf();
static constexpr unsigned long long BARRIER_TIMEOUT = 400000000ull;  // 4 s at 100 MHz
static constexpr int ST_TIMEOUT = 7;
static constexpr int ST_INTERNAL = 8;   // an internal consistency check failed (a re-evaluated
                                        // trial's error, a selection's count)
static constexpr int RPW = TS / NWAVE;  // tile rows (or columns) per wave
static constexpr int CQ_CAP = NTHR + CW + 128;
static constexpr int KB = 8;            // components whose summaries are staged together

DEV unsigned fmap(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
DEV float funmap(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}
static constexpr unsigned FMAP_INF = 0xFF800000u;  // fmap(+inf)

DEV float excl(const Top2& s, int idx) { return s.a1 == idx ? s.m2 : s.m1; }

DEV Top2 top2_id() { Top2 s; s.m1 = FINF; s.a1 = 0x7fffffff; s.m2 = FINF; s.pad = 0; return s; }

// Combine two summaries: smallest (value, index) first, second smallest after.
DEV Top2 top2_comb(Top2 a, Top2 b) {
  if (b.m1 < a.m1 || (b.m1 == a.m1 && b.a1 < a.a1)) { Top2 t = a; a = b; b = t; }
  a.m2 = fminf(a.m2, b.m1);
  return a;
}
DEV Top2 top2_add(Top2 s, float v, int idx) {
  Top2 one; one.m1 = v; one.a1 = idx; one.m2 = FINF; one.pad = 0;
  return top2_comb(s, one);
}

#if defined(__HIP_DEVICE_COMPILE__)
#define GA __attribute__((address_space(1)))
#else
#define GA
#endif

template <typename T>
DEV T ld_atomic(const GA T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-coherent access to data that other workgroups of the group write or
// read during the fit (relaxed agent-scope atomics: coherent across XCDs
// without cache maintenance).  The working matrix, which nothing writes
// during the fit, is read with plain cached loads.
template <typename T>
DEV void st_coh(GA T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV Top2 ld_top2(const GA Top2* p) {
  const GA unsigned long long* q = reinterpret_cast<const GA unsigned long long*>(p);
  unsigned long long a = ld_atomic(q), b = ld_atomic(q + 1);
  Top2 s;
  s.m1 = __uint_as_float((unsigned)a);
  s.a1 = (int)(a >> 32);
  s.m2 = __uint_as_float((unsigned)b);
  s.pad = 0;
  return s;
}
DEV void st_top2(GA Top2* p, Top2 s) {
  GA unsigned long long* q = reinterpret_cast<GA unsigned long long*>(p);
  st_coh(q, (unsigned long long)__float_as_uint(s.m1) | ((unsigned long long)(unsigned)s.a1 << 32));
  st_coh(q + 1, (unsigned long long)__float_as_uint(s.m2));
}
DEV void atomic_min_g(GA unsigned* p, unsigned v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void atomic_add_g(GA int* p, int v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exact max and min of the value path.  No NaN ever enters it (missing cells
// are +inf sentinels, or FLT_MAX in the error pass), so IEEE maximum/minimum
// equal max/min here; unlike fmaxf/fminf they need no input canonicalisation
// and pair up into the three-operand instructions.
DEV float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }
DEV float vmin(float a, float b) { return __builtin_elementwise_minimum(a, b); }

// ------------------------------------------------------------ LDS layout
struct EvalVectors {
  float sA[TCH][TS];         // per staged trial: changed U column at the tile rows
  float sB[TCH][TS];         // per staged trial: changed V row at the tile columns
};
struct BatchScratch {
  union {
    EvalVectors e;           // error pass
    float sX[2 * TCH][TS];   // residual pass: the one vector each trial needs
  } v;
  double epl[TCH][2][4];     // error pass: per staged trial, row half and 16-lane
                             // row, partial error
  float pc[TS][TS];          // error pass: the product without the current
                             // component at every cell of the tile
};
struct RefreshScratch {
  int hc[TS][RMAX + 1];      // argmax histogram of the tile columns (rows padded:
                             // the lanes of a wave count into distinct banks)
  int hr[TS][RMAX + 1];      // argmax histogram of the tile rows
  double tdw[NWAVE][TS];
  Top2 csw[NWAVE][TS];
  Top2 rsw[NWAVE][TS];
};
struct SortScratch {
  double key[SORT_MAX];
  int idx[SORT_MAX];
};
struct CombineScratch {
  Top2 part[2048];           // staged partial summaries
  double dpart[2048];        // staged td_col partials
};
struct ReduceScratch {
  double v[4096];            // chunk sums of the trials being reduced
};
struct Smem {
  union {
    BatchScratch b;
    RefreshScratch f;
    SortScratch s;
    CombineScratch c;
    ReduceScratch r;
  } u;
  float Ut[RMAX][TS];        // U of the tile rows, every component
  float Vt[RMAX][TS];        // V of the tile columns, every component
  float uk[TS], vk[TS];      // new component values of the tile (refresh)
  Trial trials[TMAX];
  int trow[TMAX];            // ByMatrix: each trial's row (a batch mixes rows)
  int noops_before[TMAX];    // no-op skips preceding each trial in the batch
  int byk[TMAX];             // trial indices by key op * RMAX + k (stable)
  int kst[2 * RMAX + 1];     // key q: byk[kst[q] .. kst[q + 1])
  int kcnt[2 * RMAX];        // per key: trial count, then the next free position
  int wk[NWAVE][2 * RMAX];   // per wave and key: trial count, then offset
  float Ri[TS];              // R of the visited row at the tile columns
  // summaries of a block of up to KB components (kb0, kb0 + 1, ...) at the tile
  float colb[KB][TS];        // F-ULF: column residual without row i, excl(colst_kc, i)
  float2 cmm[KB][TS];        // ByMatrix: colst_kc's (m1, m2), and a1 (the exclusion
  int ca1[KB][TS];           // depends on each trial's row; selected as values)
  float2 rmm[KB][TS];        // F-URF: row residual summaries of the tile rows: (m1, m2)
  int ra1[KB][TS];           // and a1 (both values are read and one is selected)
  float urow_i[RMAX];        // U of the visited row, every component
  int closed_s[RMAX];        // closed flags at the start of the row visit
  int crow_i[RMAX];          // argmax counts of the visited row
  int cq[CQ_CAP];            // queue of candidate columns of the visited row
  int cq_head, cq_n, ord_pos;
  int prev_nt;
  int nt;
  int batch_noops;
  int cur_op;
  int exhausted;
  int is_last;
  unsigned bar_e;            // group barrier: the episode being released
  int status;
  int dec;
  int wcount[NWAVE];
  int wnoop[NWAVE];
  int wcn[NWAVE];
  int wlast[NWAVE];
  // candidate window
  int cj[CW], ck[CW];
  float cvu[CW], cvv[CW];
  int cnu[CW], cnv[CW];
  int cskip[CW];             // ByElement: an exact entry (td = 0), not a trial
  int kbest[CW][4], kval[CW][4];
  float kvalf[CW][4];
  // TD_B: U of the first working row, and (U (x) V) and its argmax at (i, j0)
  float urow0[RMAX];
  float p_ij0;
  int f_ij0;
  // ByMatrix selection
  unsigned long long m_pref;
  int m_want, m_count, m_used;
  unsigned m_qpref;
};

static_assert(sizeof(Smem) <= 160 * 1024, "LDS layout exceeds a CU's 160 KB");
static_assert(2 * CW <= NTHR, "one thread per candidate pair");
static_assert(CW % (NTHR / 4) == 0, "whole rounds of four threads per candidate");
static_assert(RMAX == 64, "one lane per component (two group keys) in the batch grouping");
static_assert(TCH <= NTHR, "one thread per staged trial in the error reduction");
static_assert(KB * TS == NTHR, "one thread per staged summary");

struct Grp {
  const FitDev* d;
  GA FitCtl* ctl;
  GA BarTree* bar;   // the group barrier's counters (unused by a group of one)
  unsigned long long wait;  // bound of a barrier wait (100 MHz ticks)
  int g, G;
  int lane, wave, tid;
};

// ------------------------------------------------------------ group barrier
// Two-level barrier over the group's workgroups with a bounded wait.  A
// workgroup arrives on its subgroup's counter; the last member of each
// subgroup to arrive goes on to the top counter, and the last arrival there
// runs `last_work` (if any) and releases the episode to every subgroup.  The
// others wait on their subgroup's release word, so at most BAR_SUB
// workgroups contend for any one counter or word (with one counter for the
// whole group, its 256 serialised atomics made each barrier about 10 us;
// two levels about 2 us).  The counters only grow: an arrival's episode is
// its count divided by the arrivals per episode, which also holds for a fit
// resumed by a later launch.  A wait longer than the group's bound
// (BARRIER_TIMEOUT unless the fit sets another; a bound of 0 ends a wait at
// its first unanswered poll), or another workgroup's abort, sets the fit's
// status and leaves.  Returns false when
// this workgroup left on an abort.
//
// Ordering: data that crosses workgroups is written and read only with
// device-scope accesses; a workgroup arrives after s_waitcnt(0) (its stores
// are complete at the device level), and only thread 0 waits, between two
// workgroup barriers, so no thread's later access can be issued (or moved
// by the compiler) before the release has been seen.
template <typename F>
DEV bool group_sync_last(Grp& gp, Smem& S, F last_work) {
  GA FitCtl* ctl = gp.ctl;
  GA BarTree* bar = gp.bar;
  // every wave's stores (all device-coherent) are complete before arriving
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int G = gp.G, q = gp.g / BAR_SUB, nq = (G + BAR_SUB - 1) / BAR_SUB;
  if (gp.tid == 0) {
    int st = 0, last = 1;
    unsigned e = 0;
    if (G > 1) {
      const unsigned members = (unsigned)(q == nq - 1 ? G - BAR_SUB * q : BAR_SUB);
      const unsigned old = __hip_atomic_fetch_add(&bar->sub[q][0], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      e = old / members + 1;
      last = old % members == members - 1;
      if (last && nq > 1) {
        const unsigned o2 = __hip_atomic_fetch_add(&bar->top[0], 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        last = o2 % (unsigned)nq == (unsigned)nq - 1;
      }
      if (!last) {
        unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while ((int)(ld_atomic(&bar->rel[q][0]) - e) < 0) {
          st = ld_atomic(&ctl->status);
          if (st != 0) break;
          if (__builtin_amdgcn_s_memrealtime() - t0 > gp.wait) {
            int zero = 0;
            __hip_atomic_compare_exchange_strong(&ctl->status, &zero, ST_TIMEOUT, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st = ST_TIMEOUT;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    S.is_last = last;
    S.bar_e = e;
    S.status = st;
  }
  __syncthreads();
  if (S.is_last) {
    last_work();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (G > 1 && gp.tid == 0) {
      for (int r = 0; r < nq; ++r) st_coh(&bar->rel[r][0], S.bar_e);
    }
  }
  __syncthreads();
  return S.status == 0;
}

DEV bool group_sync(Grp& gp, Smem& S) {
  return group_sync_last(gp, S, [] {});
}

// Contiguous slice [lo, hi) of [0, n) owned by workgroup g of G.
DEV void slice(int n, int g, int G, int& lo, int& hi) {
  int per = (n + G - 1) / G;
  lo = g * per;
  hi = lo + per;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
}

// ------------------------------------------------------------ per-trial vectors
// Row-side value of trial tr at working row t (the changed U column):
//   F-ULF: U''_tk from the atomic-min pass; F-URF: U'_tk from the top-2 row
//   summary; null trial: the current U_tk.  Padding rows: 0.
DEV float row_side(const FitDev& d, const Trial& tr, int par, int slot, int t) {
  if (t >= d.m) return 0.0f;
  if (tr.op == OP_ULF)
    return funmap(ld_atomic(&d.tvec[((size_t)par * d.tmax + slot) * d.ldmax + t]));
  if (tr.op == OP_URF) {
    Top2 s = ld_top2(&d.rowst[(size_t)tr.k * d.ldm + t]);
    float x = d.RwT[(size_t)tr.j * d.ldm + t] - tr.val;
    return fminf(excl(s, tr.j), x);
  }
  return ld_atomic(&d.Uc[(size_t)tr.k * d.ldm + t]);
}

// Column-side value of trial tr at working column c (the changed V row).
DEV float col_side(const FitDev& d, const Trial& tr, int par, int slot, int c, int i) {
  if (c >= d.n) return 0.0f;
  if (tr.op == OP_ULF) {
    Top2 s = ld_top2(&d.colst[(size_t)tr.k * d.ldn + c]);
    float x = d.Rw[(size_t)i * d.ldn + c] - tr.val;
    return fminf(excl(s, i), x);
  }
  if (tr.op == OP_URF)
    return funmap(ld_atomic(&d.tvec[((size_t)par * d.tmax + slot) * d.ldmax + c]));
  return ld_atomic(&d.V[(size_t)tr.k * d.ldn + c]);
}

// U of the tile rows and V of the tile columns for every component, staged in
// LDS in one round of independent loads.
DEV void stage_uv(Grp& gp, Smem& S, int r0, int c0) {
  // descriptor fields are read once: a device-coherent access makes the
  // compiler reload anything it would read from memory after it
  const FitDev& d = *gp.d;
  const auto Uc = d.Uc;
  const auto V = d.V;
  const size_t ldm = d.ldm, ldn = d.ldn;
  const int ne = d.r * TS;
  for (int e = gp.tid; e < ne; e += NTHR) {
    const int l = e / TS, x = e % TS;
    S.Ut[l][x] = ld_atomic(&Uc[l * ldm + r0 + x]);
    S.Vt[l][x] = ld_atomic(&V[l * ldn + c0 + x]);
  }
}

// ------------------------------------------------------------ trial staging
// The first residual of a trial, restricted to a tile, from data staged once
// per tile and block of components (every trial of a batch shares the
// visited row i):
//   F-ULF, tile column x: V'_kc = min(excl(colst_kc, i), R_ic - u)
//   F-URF, tile row x:    U'_tk = min(excl(rowst_kt, j), R_tj - v)
// Padding rows and columns take 0.
DEV void stage_ri(Grp& gp, Smem& S, int i, int c0) {
  const FitDev& d = *gp.d;
  if (gp.tid < TS) S.Ri[gp.tid] = d.Rw[(size_t)i * d.ldn + c0 + gp.tid];
}

// Summaries of components kb0 .. kb0 + nb - 1 (nb <= KB) at the tile, one
// thread per component and tile index, all loads in one round: the column
// summaries without row i (cols) and the row summaries (rows).
template <bool MR = false>
DEV void stage_block(Grp& gp, Smem& S, int kb0, int nb, bool cols, bool rows, int r0, int c0,
                     int i) {
  const FitDev& d = *gp.d;
  const auto colst = d.colst;
  const auto rowst = d.rowst;
  const size_t ldm = d.ldm, ldn = d.ldn;
  const int b = gp.tid / TS, x = gp.tid % TS;
  if (b < nb) {
    if (cols) {
      const Top2 t = ld_top2(&colst[(kb0 + b) * ldn + c0 + x]);
      if (MR) {
        S.cmm[b][x] = make_float2(t.m1, t.m2);
        S.ca1[b][x] = t.a1;
      } else {
        S.colb[b][x] = excl(t, i);
      }
    }
    if (rows) {
      const Top2 t = ld_top2(&rowst[(kb0 + b) * ldm + r0 + x]);
      S.rmm[b][x] = make_float2(t.m1, t.m2);
      S.ra1[b][x] = t.a1;
    }
  }
}

// Position p of a trial list made of two byk ranges [a0, a0 + n0) and
// [a1, ...): the trial index.
DEV int list_at(const Smem& S, int p, int a0, int n0, int a1) {
  return S.byk[p < n0 ? a0 + p : a1 + p - n0];
}

// A wave's trials of a chunk, one per lane: lane l < NE holds the trial at
// chunk position w + NWAVE * l (slot q = -1 past the chunk's end).  Fetched
// in one round of LDS reads; the per-trial steps take the fields by
// v_readlane (wave-uniform scalars).
struct WaveTrials {
  int q, j, k, op;
  float val;
  int i;                     // ByMatrix: the trial's row
};
// Chunk positions cs .. cs + cn - 1 of the trial list made of the byk ranges
// [a0, a0 + n0) and [a1, ...).
template <int NE, bool MR = false>
DEV WaveTrials wave_trials(const Grp& gp, const Smem& S, int cs, int cn, int a0, int n0, int a1) {
  WaveTrials w;
  w.q = -1; w.j = 0; w.k = 0; w.op = OP_NULL; w.val = 0.0f; w.i = 0;
  const int sl = gp.wave + NWAVE * gp.lane;
  if (gp.lane < NE && sl < cn) {
    w.q = list_at(S, cs + sl, a0, n0, a1);
    const Trial tr = S.trials[w.q];
    w.j = tr.j; w.k = tr.k; w.op = tr.op; w.val = tr.val;
    if (MR) w.i = S.trow[w.q];
  }
  return w;
}
// The same for the byk range [base, base + cn).
template <int NE, bool MR = false>
DEV WaveTrials wave_trials_range(const Grp& gp, const Smem& S, int base, int cn) {
  WaveTrials w;
  w.q = -1; w.j = 0; w.k = 0; w.op = OP_NULL; w.val = 0.0f; w.i = 0;
  const int sl = gp.wave + NWAVE * gp.lane;
  if (gp.lane < NE && sl < cn) {
    w.q = S.byk[base + sl];
    const Trial tr = S.trials[w.q];
    w.j = tr.j; w.k = tr.k; w.op = tr.op; w.val = tr.val;
    if (MR) w.i = S.trow[w.q];
  }
  return w;
}
DEV int lane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
DEV float lane_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

// The R values the first residuals of a chunk's trials need (wave w: trials
// w, w + NWAVE, ... of the chunk's cn): F-URF (side 1), column j of R at the
// tile rows; F-ULF with rows of their own (MR), row i at the tile columns;
// plain F-ULF takes row i from LDS and loads nothing.  Every slot loads,
// unconditionally: one without a trial reads element 0 (a valid address, the
// value unused).  Under branches the compiler merged each load into the
// register array where it was issued and waited for it there.
template <int NE, bool MR>
DEV void residual_loads(const Grp& gp, const WaveTrials& w, int side, int cn, const GA float* Rw,
                        const GA float* RwT, size_t ldn, size_t ldm, int r0, int c0,
                        float (&raw)[NE]) {
  const int x = gp.lane;
  if (side) {
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      const int sl = gp.wave + m * NWAVE;
      raw[m] = RwT[sl < cn ? (size_t)lane_i(w.j, m) * ldm + r0 + x : 0];
    }
  } else if (MR) {
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      const int sl = gp.wave + m * NWAVE;
      raw[m] = Rw[sl < cn ? (size_t)lane_i(w.i, m) * ldn + c0 + x : 0];
    }
  }
}

// ------------------------------------------------------------ pass 1 of a batch
// Second residual of every trial over this workgroup's tiles, combined across
// tiles with an atomic min on order-preserving integer images (exact).  The
// F-ULF trials come first (lanes over the tile rows, the tile's R rows in
// registers), then the F-URF trials (lanes over the tile columns).  Per block
// of components the summaries are staged once; each trial then stages the
// one first-residual vector it needs, 2 * TCH trials at a time (wave w takes
// trials w, w + NWAVE, ...); the trial records and global loads of the next
// chunk are issued before the current chunk is evaluated.
// With MR (ByMatrix) the trials of a batch have rows of their own: the F-ULF
// first residual takes R's row and the column summary's exclusion per trial.
template <bool MR = false>
DEV void batch_residual_pass(Grp& gp, Smem& S, int i, int par) {
  const FitDev& d = *gp.d;
  // descriptor fields, read once (the atomics below would force reloads)
  const auto Rw = d.Rw;
  const auto RwT = d.RwT;
  const auto tv = d.tvec + (size_t)par * d.tmax * d.ldmax;
  const size_t ldx = d.ldmax, ldm = d.ldm, ldn = d.ldn;
  const int dm = d.m, dn = d.n, dr = d.r, nct = d.nct;
  const int ntile = d.nrt * d.nct;
  constexpr int NE = 2 * TCH / NWAVE;
  const int x = gp.lane;
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / nct, ct = tile % nct;
    const int r0 = rt * TS, c0 = ct * TS;
    __syncthreads();
    stage_ri(gp, S, i, c0);
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      // side 0, F-ULF: U''_tk = min over the tile columns of R_tc - V'_kc
      // side 1, F-URF: V''_kc = min over the tile rows of R_tc - U'_tk
      if (S.kst[side * RMAX + dr] == S.kst[side * RMAX]) continue;
      const GA float* rb = side ? Rw + r0 * ldn + c0 + gp.lane : RwT + c0 * ldm + r0 + gp.lane;
      const size_t rs = side ? ldn : ldm;
      float Rv[TS];
#pragma unroll
      for (int y = 0; y < TS; ++y) Rv[y] = rb[y * rs];
      const int own = (side ? c0 : r0) + gp.lane;
      const bool in = side ? r0 + x < dm : c0 + x < dn;
#pragma unroll 1
      for (int kb0 = 0; kb0 < dr; kb0 += KB) {
        const int nb = dr - kb0 < KB ? dr - kb0 : KB;
        const int lo = S.kst[side * RMAX + kb0], hi = S.kst[side * RMAX + kb0 + nb];
        if (lo == hi) continue;
        __syncthreads();
        stage_block<MR>(gp, S, kb0, nb, side == 0, side == 1, r0, c0, i);
        // the first chunk's trial records and loads; each later chunk's are
        // taken while the chunk before it is evaluated
        WaveTrials w = wave_trials_range<NE, MR>(gp, S, lo, hi - lo < 2 * TCH ? hi - lo : 2 * TCH);
        float raw[NE];
        residual_loads<NE, MR>(gp, w, side, hi - lo, Rw, RwT, ldn, ldm, r0, c0, raw);
#pragma unroll 1
        for (int cs = lo; cs < hi; cs += 2 * TCH) {
          const int cn = hi - cs < 2 * TCH ? hi - cs : 2 * TCH;
          __syncthreads();
          if (side == 0 && MR) {
#pragma unroll
            for (int m = 0; m < NE; ++m) {
              const int sl = gp.wave + m * NWAVE;
              if (sl < cn) {
                const int b = lane_i(w.k, m) - kb0;
                const float2 mm = S.cmm[b][x];
                const float ex = S.ca1[b][x] == lane_i(w.i, m) ? mm.y : mm.x;
                S.u.b.v.sX[sl][x] = in ? vmin(ex, raw[m] - lane_f(w.val, m)) : 0.0f;
              }
            }
          } else if (side == 0) {
            const float ri = S.Ri[x];
#pragma unroll
            for (int m = 0; m < NE; ++m) {
              const int sl = gp.wave + m * NWAVE;
              if (sl < cn)
                S.u.b.v.sX[sl][x] =
                    in ? vmin(S.colb[lane_i(w.k, m) - kb0][x], ri - lane_f(w.val, m)) : 0.0f;
            }
          } else {
#pragma unroll
            for (int m = 0; m < NE; ++m) {
              const int sl = gp.wave + m * NWAVE;
              if (sl < cn) {
                const int b = lane_i(w.k, m) - kb0;
                const float2 mm = S.rmm[b][x];
                const float ex = S.ra1[b][x] == lane_i(w.j, m) ? mm.y : mm.x;
                S.u.b.v.sX[sl][x] = in ? vmin(ex, raw[m] - lane_f(w.val, m)) : 0.0f;
              }
            }
          }
          // the next chunk's (past the range's end: no trials, and every
          // load reads element 0)
          const int ns = cs + 2 * TCH;
          w = wave_trials_range<NE, MR>(gp, S, ns, hi - ns < 2 * TCH ? hi - ns : 2 * TCH);
          residual_loads<NE, MR>(gp, w, side, hi - ns, Rw, RwT, ldn, ldm, r0, c0, raw);
          __syncthreads();
          // Each trial's 16 broadcast LDS reads are kept AHEAD deep in
          // flight, and the next trial's first AHEAD are issued before this
          // trial's reduction and atomic: the scheduling fences stop the
          // compiler from issuing each read just before its use (by itself
          // it keeps two in flight, and with two waves per SIMD the reads'
          // latency shows).  A read past the chunk's last trial stays inside
          // the staging array and its value is never used.
          constexpr int NQ = TS / 4, AHEAD = 4;
          float4 qn[AHEAD];
#pragma unroll
          for (int c4 = 0; c4 < AHEAD; ++c4)
            qn[c4] = reinterpret_cast<const float4*>(S.u.b.v.sX[gp.wave])[c4];
#pragma unroll 1
          for (int sl = gp.wave; sl < cn; sl += NWAVE) {
            const float4* sx = reinterpret_cast<const float4*>(S.u.b.v.sX[sl]);
            const int q = S.byk[cs + sl];
            float4 sq[NQ];
#pragma unroll
            for (int c4 = 0; c4 < AHEAD; ++c4) sq[c4] = qn[c4];
            __builtin_amdgcn_sched_barrier(0);
            float x0 = FINF, x1 = FINF, x2 = FINF, x3 = FINF;
#pragma unroll
            for (int c4 = 0; c4 < NQ; ++c4) {
              const float4 s = sq[c4];
              const int c = 4 * c4;
              if (c4 & 1) {
                x2 = vmin(vmin(x2, Rv[c + 0] - s.x), Rv[c + 1] - s.y);
                x3 = vmin(vmin(x3, Rv[c + 2] - s.z), Rv[c + 3] - s.w);
              } else {
                x0 = vmin(vmin(x0, Rv[c + 0] - s.x), Rv[c + 1] - s.y);
                x1 = vmin(vmin(x1, Rv[c + 2] - s.z), Rv[c + 3] - s.w);
              }
              if (c4 + AHEAD < NQ) sq[c4 + AHEAD] = sx[c4 + AHEAD];
              __builtin_amdgcn_sched_barrier(0);
            }
            const int nx = sl + NWAVE < 2 * TCH ? sl + NWAVE : sl;
#pragma unroll
            for (int c4 = 0; c4 < AHEAD; ++c4)
              qn[c4] = reinterpret_cast<const float4*>(S.u.b.v.sX[nx])[c4];
            __builtin_amdgcn_sched_barrier(0);
            const float xm = vmin(vmin(x0, x1), vmin(x2, x3));
            // +inf: no observed cell of this row (column) in the tile
            if (xm != FINF) atomic_min_g(&tv[q * ldx + own], fmap(xm));
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ pass 2 of a batch
// b-norm of every trial over this workgroup's tiles, component by component
// (the F-ULF and F-URF trials of component k together); per tile and
// component the product without k is formed once.  Wave w takes the tile
// rows of half w & 1 (lane = tile column) for the staged trials (w >> 1),
// (w >> 1) + 4, ..., holding that half's R and product without k in
// registers.  Per lane and trial the half-column sum runs over its 32 rows in
// four interleaved FP64 accumulators; the lanes of each 16-lane row are then
// added by DPP steps in a fixed pattern, and one thread per trial adds the
// eight row sums (half 0 first) in a fixed order; the tile's sum is added to
// the workgroup's per-trial sum in tile order.
//
// Chunks of up to TCH trials are software-pipelined: while chunk c is
// evaluated, the global loads of chunk c + 1 are in flight, and chunk c's
// lane sums are reduced while chunk c + 1 is being staged.

// One DPP exchange (control CTRL) of a double, added.
template <int CTRL>
DEV double dpp_add(double a) {
  const unsigned long long b = __double_as_longlong(a);
  // every lane reads a lane of its own 16-lane row: no lane keeps an old
  // value, so the moves need none (no zeroing before each exchange)
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return a + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Sum over a 16-lane row, in lane 16 * row: quad exchanges (permutations
// 1, 0, 3, 2 and 2, 3, 0, 1), then rotations of the row by 4 and by 8.
DEV double row_sum(double v) {
  return dpp_add<0x128>(dpp_add<0x124>(dpp_add<0x4E>(dpp_add<0xB1>(v))));
}
// The same for two values at once: a's row sum in lane 16 * row, b's in lane
// 16 * row + 1, each bit-identical to row_sum's.  In the first exchange even
// lanes keep a and odd lanes b, each receiving from its partner the value it
// keeps; the later exchanges stay within a parity.  Every addition has the
// operands of the corresponding one of row_sum (b's in swapped order, which
// IEEE addition does not see).
DEV double pair_row_sum(double a, double b, bool odd) {
  const double send = odd ? a : b, keep = odd ? b : a;
  const unsigned long long s = __double_as_longlong(send);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)s, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(s >> 32), 0xB1, 0xF, 0xF, false);
  const double w = keep + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  return dpp_add<0x128>(dpp_add<0x124>(dpp_add<0x4E>(w)));
}

// A chunk of a batch's trial list: component k's trials [cs, cs + cn) of
// the two byk ranges [a0, a0 + n0) (F-ULF) and [a1, a1 + n1) (F-URF).
struct Chunk {
  int k, cs, cn, a0, n0, a1;
};
// The chunk at or after component k, position cs; k == r when none is left.
DEV Chunk chunk_at(const Smem& S, int r, int k, int cs) {
  Chunk c;
  for (; k < r; ++k, cs = 0) {
    const int a0 = S.kst[k], n0 = S.kst[k + 1] - a0;
    const int a1 = S.kst[RMAX + k], n1 = S.kst[RMAX + k + 1] - a1;
    if (cs < n0 + n1) {
      c.k = k; c.cs = cs; c.cn = n0 + n1 - cs < TCH ? n0 + n1 - cs : TCH;
      c.a0 = a0; c.n0 = n0; c.a1 = a1;
      return c;
    }
  }
  c.k = r; c.cs = 0; c.cn = 0; c.a0 = c.n0 = c.a1 = 0;
  return c;
}

// Global loads of a chunk's trials (wave w: trials w, w + NWAVE, ...):
// F-ULF: the second residual at the tile rows; F-URF: R's column j at the
// tile rows and the second residual at the tile columns.
template <int NE, bool MR = false>
DEV void chunk_loads(Grp& gp, const WaveTrials& w, const Chunk& c, int par, int r0, int c0,
                     float (&rawA)[NE], unsigned (&rawB)[NE]) {
  const FitDev& d = *gp.d;
  const auto tv = d.tvec + (size_t)par * d.tmax * d.ldmax;
  const auto RwT = d.RwT;
  const size_t ldx = d.ldmax, ldm = d.ldm;
  const int x = gp.lane;
  // Every slot loads, unconditionally: a slot without a trial of either
  // operation reads element 0 of the target array and of R's transpose
  // (valid addresses, values unused).  With the loads under branches the
  // compiler merged each into the register array right away and waited for
  // it there, so the chunk's loads went one at a time.
#pragma unroll
  for (int m = 0; m < NE; ++m) {
    const bool has = gp.wave + m * NWAVE < c.cn;
    const int q = has ? lane_i(w.q, m) : 0, op = has ? lane_i(w.op, m) : OP_NULL;
    const bool ulf = op == OP_ULF, urf = op == OP_URF;
    const size_t ob = ulf ? (size_t)q * ldx + r0 + x : urf ? (size_t)q * ldx + c0 + x : 0;
    rawB[m] = ld_atomic(&tv[ob]);
    if (MR) {
      const size_t oa = urf ? (size_t)lane_i(w.j, m) * ldm + r0 + x : 0;
      const size_t oc = ulf ? (size_t)lane_i(w.i, m) * d.ldn + c0 + x : 0;
      rawA[m] = ulf ? d.Rw[oc] : RwT[oa];
    } else {
      rawA[m] = RwT[urf ? (size_t)lane_i(w.j, m) * ldm + r0 + x : 0];
    }
  }
}

// The trials' two vectors into LDS: the first residual from the staged
// summaries (block b of the component), the second from the loads.  The null
// trial of the initial evaluation (always alone) takes the current component.
template <int NE, bool MR = false>
DEV void chunk_stage(Grp& gp, Smem& S, const WaveTrials& w, const Chunk& c, int b, int r0, int c0,
                     const float (&rawA)[NE], const unsigned (&rawB)[NE]) {
  const FitDev& d = *gp.d;
  const int x = gp.lane;
  const bool rin = r0 + x < d.m, cin = c0 + x < d.n;
  if (S.trials[list_at(S, c.cs, c.a0, c.n0, c.a1)].op == OP_NULL) {
    if (gp.wave == 0) {
      S.u.b.v.e.sA[0][x] = rin ? ld_atomic(&d.Uc[(size_t)c.k * d.ldm + r0 + x]) : 0.0f;
      S.u.b.v.e.sB[0][x] = cin ? ld_atomic(&d.V[(size_t)c.k * d.ldn + c0 + x]) : 0.0f;
    }
    return;
  }
  const float cb = S.colb[b][x], ri = S.Ri[x];
  const float2 mm = S.rmm[b][x];
  const float m1 = mm.x, m2 = mm.y;
  const int a1 = S.ra1[b][x];
#pragma unroll
  for (int m = 0; m < NE; ++m) {
    const int sl = gp.wave + m * NWAVE;
    if (sl < c.cn) {
      const float val = lane_f(w.val, m);
      float va, vb;
      if (lane_i(w.op, m) == OP_ULF) {
        va = funmap(rawB[m]);
        if (MR) {
          const float2 cm = S.cmm[b][x];
          const float ex = S.ca1[b][x] == lane_i(w.i, m) ? cm.y : cm.x;
          vb = vmin(ex, rawA[m] - val);
        } else {
          vb = vmin(cb, ri - val);
        }
      } else {
        va = vmin(a1 == lane_i(w.j, m) ? m2 : m1, rawA[m] - val);
        vb = funmap(rawB[m]);
      }
      S.u.b.v.e.sA[sl][x] = rin ? va : 0.0f;
      S.u.b.v.e.sB[sl][x] = cin ? vb : 0.0f;
    }
  }
}

// Per trial of an evaluated chunk: the eight row sums (half 0 first) in a
// fixed order, the tile's partial error of the trial (epart[trial][tile]).
DEV void chunk_reduce(Grp& gp, Smem& S, const Chunk& c, GA double* epart, int ntile, int tile) {
  if (gp.tid < c.cn) {
    const double* p = &S.u.b.epl[gp.tid][0][0];
    const double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    st_coh(&epart[(size_t)list_at(S, c.cs + gp.tid, c.a0, c.n0, c.a1) * ntile + tile], s);
  }
}

template <bool MR = false>
DEV void batch_eval_pass(Grp& gp, Smem& S, int i, int par) {
  const FitDev& d = *gp.d;
  const auto Rw = d.Rw;
  const auto epart = d.epart;
  const size_t ldn = d.ldn;
  const int dr = d.r, nct = d.nct;
  constexpr int NE = TCH / NWAVE;
  const int ntile = d.nrt * d.nct;
  const int half = gp.wave & 1, h0 = half * (TS / 2);
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / nct, ct = tile % nct;
    const int r0 = rt * TS, c0 = ct * TS;
    __syncthreads();
    stage_uv(gp, S, r0, c0);
    stage_ri(gp, S, i, c0);
    __syncthreads();
    // an unobserved cell takes R = P = FLT_MAX, which contributes |d| = 0
    float Rev[TS / 2], Pc[TS / 2];
    unsigned obs = 0;
#pragma unroll
    for (int t = 0; t < TS / 2; ++t) {
      const float rv = Rw[(r0 + h0 + t) * ldn + c0 + gp.lane];
      const bool o = rv != FINF;
      obs |= (unsigned)o << t;
      Rev[t] = o ? rv : FLT_MAX;
    }
    float rawA[NE];
    unsigned rawB[NE];
    Chunk cur = chunk_at(S, dr, 0, 0), prev;
    prev.cn = 0;
    WaveTrials wcur = wave_trials<NE, MR>(gp, S, cur.cs, cur.cn, cur.a0, cur.n0, cur.a1);
    chunk_loads<NE, MR>(gp, wcur, cur, par, r0, c0, rawA, rawB);
    int kb0 = -KB, kcur = -1;
#pragma unroll 1
    while (cur.k < dr) {
      const bool newk = cur.k != kcur;
      if (newk) {
        // summaries of the component's block (read by the staging after the
        // chunk's barrier; the previous chunk's staging is done with them)
        if (cur.k >= kb0 + KB) {
          kb0 = cur.k;
          stage_block<MR>(gp, S, kb0, dr - kb0 < KB ? dr - kb0 : KB, true, true, r0, c0, i);
        }
        // the product without k at the tile, from the staged U and V: wave w
        // forms rows 8 (w >> 1) .. of its half into LDS (the four waves of a
        // half share the work), read back by every wave after the barrier
        const int rb = h0 + 8 * (gp.wave >> 1);
        float P8[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) P8[t] = -FINF;
        for (int l = 0; l < dr; ++l) {
          if (l == cur.k) continue;
          const float v = S.Vt[l][gp.lane];
          const float4* u4 = reinterpret_cast<const float4*>(&S.Ut[l][rb]);
#pragma unroll
          for (int t4 = 0; t4 < 2; ++t4) {
            const float4 u = u4[t4];
            P8[4 * t4 + 0] = vmax(P8[4 * t4 + 0], u.x + v);
            P8[4 * t4 + 1] = vmax(P8[4 * t4 + 1], u.y + v);
            P8[4 * t4 + 2] = vmax(P8[4 * t4 + 2], u.z + v);
            P8[4 * t4 + 3] = vmax(P8[4 * t4 + 3], u.w + v);
          }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) S.u.b.pc[rb + t][gp.lane] = P8[t];
        kcur = cur.k;
      }
      __syncthreads();
      if (newk) {
#pragma unroll
        for (int t = 0; t < TS / 2; ++t)
          Pc[t] = ((obs >> t) & 1u) ? S.u.b.pc[h0 + t][gp.lane] : FLT_MAX;
      }
      chunk_stage<NE, MR>(gp, S, wcur, cur, cur.k - kb0, r0, c0, rawA, rawB);
      chunk_reduce(gp, S, prev, epart, ntile, tile);
      const Chunk next = chunk_at(S, dr, cur.k, cur.cs + TCH);
      const WaveTrials wnext =
          wave_trials<NE, MR>(gp, S, next.cs, next.cn, next.a0, next.n0, next.a1);
      chunk_loads<NE, MR>(gp, wnext, next, par, r0, c0, rawA, rawB);
      __syncthreads();
      // Two trials per step (sl and sl + 4, the wave's consecutive ones): the
      // two cell loops interleave, and one DPP reduction adds both (the last
      // trial of an odd count goes alone, its partner reading its vectors).
#pragma unroll 1
      for (int sl = gp.wave >> 1; sl < cur.cn; sl += NWAVE) {
        const int slb = sl + NWAVE / 2;
        const bool two = slb < cur.cn;
        const int sb = two ? slb : sl;
        const float vsa = S.u.b.v.e.sB[sl][gp.lane], vsb = S.u.b.v.e.sB[sb][gp.lane];
        const float4* saa = reinterpret_cast<const float4*>(&S.u.b.v.e.sA[sl][h0]);
        const float4* sab = reinterpret_cast<const float4*>(&S.u.b.v.e.sA[sb][h0]);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
#pragma unroll
        for (int t4 = 0; t4 < TS / 8; ++t4) {
          const float4 x = saa[t4], y = sab[t4];
          const int t = 4 * t4;
          a0 += fabs((double)(Rev[t + 0] - vmax(Pc[t + 0], x.x + vsa)));
          a1 += fabs((double)(Rev[t + 1] - vmax(Pc[t + 1], x.y + vsa)));
          a2 += fabs((double)(Rev[t + 2] - vmax(Pc[t + 2], x.z + vsa)));
          a3 += fabs((double)(Rev[t + 3] - vmax(Pc[t + 3], x.w + vsa)));
          b0 += fabs((double)(Rev[t + 0] - vmax(Pc[t + 0], y.x + vsb)));
          b1 += fabs((double)(Rev[t + 1] - vmax(Pc[t + 1], y.y + vsb)));
          b2 += fabs((double)(Rev[t + 2] - vmax(Pc[t + 2], y.z + vsb)));
          b3 += fabs((double)(Rev[t + 3] - vmax(Pc[t + 3], y.w + vsb)));
        }
        const double v = pair_row_sum((a0 + a1) + (a2 + a3), (b0 + b1) + (b2 + b3), gp.lane & 1);
        if ((gp.lane & 15) == 0) S.u.b.epl[sl][half][gp.lane >> 4] = v;
        else if (two && (gp.lane & 15) == 1) S.u.b.epl[slb][half][gp.lane >> 4] = v;
      }
      prev = cur;
      cur = next;
      wcur = wnext;
    }
    __syncthreads();
    chunk_reduce(gp, S, prev, epart, ntile, tile);
  }
}

// Errors of this workgroup's slice of trials from the per-tile partials, in
// an order fixed by the tile count alone: chunks of consecutive tiles (RCH,
// or more when there are over 4096 chunks), each summed in tile order, then
// a pairwise tree over the chunk sums.  How the tiles were spread over the
// group's workgroups does not enter, so a fit's errors (and with them its
// decisions) are the same on any group size.
static constexpr int RCH = 32;

DEV void reduce_errors(Grp& gp, Smem& S, int nt) {
  const FitDev& d = *gp.d;
  const auto epart = d.epart;
  const auto eprime = d.eprime;
  const int ntile = d.nrt * d.nct;
  const int per = ntile <= 4096 * RCH ? RCH : (ntile + 4095) / 4096;
  const int nch = (ntile + per - 1) / per;
  int lo, hi;
  slice(nt, gp.g, gp.G, lo, hi);
  // trials staged at a time: their chunk sums (<= 4096 doubles)
  const int qb = 4096 / nch;
  for (int q0 = lo; q0 < hi; q0 += qb) {
    const int qn = hi - q0 < qb ? hi - q0 : qb;
    __syncthreads();
    for (int e = gp.tid; e < qn * nch; e += NTHR) {
      const int qq = e / nch, c = e % nch;
      const GA double* p = epart + (size_t)(q0 + qq) * ntile + (size_t)c * per;
      const int len = ntile - c * per < per ? ntile - c * per : per;
      double sum = 0.0;
      for (int t0 = 0; t0 < len; t0 += RCH) {
        double v[RCH];
#pragma unroll
        for (int t = 0; t < RCH; ++t) v[t] = t0 + t < len ? ld_atomic(&p[t0 + t]) : 0.0;
#pragma unroll
        for (int t = 0; t < RCH; ++t)
          if (t0 + t < len) sum += v[t];
      }
      S.u.r.v[e] = sum;
    }
    __syncthreads();
    for (int qq = gp.tid; qq < qn; qq += NTHR) {
      double* v = S.u.r.v + qq * nch;
      for (int w = 1; w < nch; w *= 2)
        for (int c = 0; c + w < nch; c += 2 * w) v[c] += v[c + w];
      st_coh(&eprime[q0 + qq], v[0]);
    }
  }
}

// Decision of a batch (last workgroup to arrive), among the trials whose
// error is strictly below thr: the first one, or with `best` the one of
// smallest error (the first of them on ties).
DEV void decide(Grp& gp, Smem& S, int nt, double thr, bool best) {
  const auto eprime = gp.d->eprime;
  if (gp.tid == 0) S.dec = 0x7fffffff;
  __syncthreads();
  if (!best) {
    for (int q = gp.tid; q < nt; q += NTHR)
      if (ld_atomic(&eprime[q]) < thr) atomicMin(&S.dec, q);
  } else {
    double bv = thr;
    int bq = 0x7fffffff;
    for (int q = gp.tid; q < nt; q += NTHR) {
      const double v = ld_atomic(&eprime[q]);
      if (v < bv) { bv = v; bq = q; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oq = __shfl_xor(bq, off, 64);
      if (ov < bv || (ov == bv && oq < bq)) { bv = ov; bq = oq; }
    }
    if (gp.lane == 0) { S.u.r.v[gp.wave] = bv; S.wcount[gp.wave] = bq; }
    __syncthreads();
    if (gp.tid == 0) {
      for (int w = 1; w < NWAVE; ++w) {
        const double ov = S.u.r.v[w];
        const int oq = S.wcount[w];
        if (ov < bv || (ov == bv && oq < bq)) { bv = ov; bq = oq; }
      }
      S.dec = bq;
    }
  }
  __syncthreads();
  if (gp.tid == 0) {
    const int dec = S.dec == 0x7fffffff ? -1 : S.dec;
    st_coh(&gp.ctl->decision, dec);
    st_coh(&gp.ctl->e_new, dec >= 0 ? ld_atomic(&eprime[dec]) : 0.0);
    // the deciding workgroup changes from batch to batch: device-coherent
    st_coh(&gp.ctl->batches, ld_atomic(&gp.ctl->batches) + 1);
  }
}

// Clear the atomic-min targets used by the previous batch (other parity).
DEV void clear_prev(Grp& gp, Smem& S, int par_prev) {
  const FitDev& d = *gp.d;
  const size_t total = (size_t)S.prev_nt * d.ldmax;
  GA unsigned* v = d.tvec + (size_t)par_prev * d.tmax * d.ldmax;
  for (size_t e = (size_t)gp.g * NTHR + gp.tid; e < total; e += (size_t)gp.G * NTHR)
    st_coh(&v[e], FMAP_INF);
}

// ------------------------------------------------------------ refresh
// After an accepted update (has_acc: component k takes the trial acc's
// vectors, written here by the owner tiles) and at initialisation: argmax
// counts of every row and column into count buffer cb, td_col partials per
// row tile, and the top-2 residual partials of component k.  With `full` it
// also clears the other count buffer.
DEV void refresh_tiles(Grp& gp, Smem& S, int k, bool has_acc, Trial acc, int par, int slot, int i,
                       bool full, int cb) {
  const FitDev& d = *gp.d;
  const int ntile = d.nrt * d.nct;
  GA int* crow = d.crow + (size_t)cb * d.ldm * d.r;
  GA int* ccol = d.ccol + (size_t)cb * d.ldn * d.r;
  if (full) {
    GA int* orow = d.crow + (size_t)(cb ^ 1) * d.ldm * d.r;
    GA int* ocol = d.ccol + (size_t)(cb ^ 1) * d.ldn * d.r;
    int lo, hi;
    slice(d.m * d.r, gp.g, gp.G, lo, hi);
    for (int x = lo + gp.tid; x < hi; x += NTHR) st_coh(&orow[x], 0);
    slice(d.n * d.r, gp.g, gp.G, lo, hi);
    for (int x = lo + gp.tid; x < hi; x += NTHR) st_coh(&ocol[x], 0);
  }
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / d.nct, ct = tile % d.nct;
    const int r0 = rt * TS, c0 = ct * TS;
    // the tile's R values (lanes over columns, the wave's rows) and R's
    // transpose (lanes over rows, the wave's columns), loaded first: they
    // arrive while the component's vectors are staged
    const int c = c0 + gp.lane;
    const int tl0 = gp.wave * RPW;
    const int tb = r0 + tl0;
    const int cl0 = gp.wave * RPW;
    float R[RPW], RT[RPW];
#pragma unroll
    for (int tt = 0; tt < RPW; ++tt) R[tt] = d.Rw[(size_t)(tb + tt) * d.ldn + c];
#pragma unroll
    for (int cc = 0; cc < RPW; ++cc) RT[cc] = d.RwT[(size_t)(c0 + cl0 + cc) * d.ldm + r0 + gp.lane];
    __syncthreads();
    if (full) {
      // only the rank's components of each histogram row are used
      const int dr = d.r;
      for (int e = gp.tid; e < TS * dr; e += NTHR) {
        const int x = e / dr, l = e - x * dr;
        S.u.f.hc[x][l] = 0;
        S.u.f.hr[x][l] = 0;
      }
    }
    if (gp.tid < TS) {
      const int t = r0 + gp.tid;
      const float v = has_acc ? row_side(d, acc, par, slot, t) : ld_atomic(&d.Uc[(size_t)k * d.ldm + t]);
      S.uk[gp.tid] = v;
      if (has_acc && ct == 0) st_coh(&d.Uc[(size_t)k * d.ldm + t], v);
    } else if (gp.tid < 2 * TS) {
      const int c = c0 + gp.tid - TS;
      const float v = has_acc ? col_side(d, acc, par, slot, c, i) : ld_atomic(&d.V[(size_t)k * d.ldn + c]);
      S.vk[gp.tid - TS] = v;
      if (has_acc && rt == 0) st_coh(&d.V[(size_t)k * d.ldn + c], v);
    }
    if (full) stage_uv(gp, S, r0, c0);
    __syncthreads();
    if (full) {
      float P[RPW];
      int A[RPW];
#pragma unroll
      for (int tt = 0; tt < RPW; ++tt) { P[tt] = -FINF; A[tt] = 0; }
      for (int l = 0; l < d.r; ++l) {
        if (l == k) {
          const float v = S.vk[gp.lane];
#pragma unroll
          for (int tt = 0; tt < RPW; ++tt) {
            float x = S.uk[tl0 + tt] + v;
            if (l == 0 || x > P[tt]) { P[tt] = x; A[tt] = l; }
          }
        } else {
          const float v = S.Vt[l][gp.lane];
#pragma unroll
          for (int tt = 0; tt < RPW; ++tt) {
            float x = S.Ut[l][tl0 + tt] + v;
            if (l == 0 || x > P[tt]) { P[tt] = x; A[tt] = l; }
          }
        }
      }
      double tdl = 0.0;
#pragma unroll
      for (int tt = 0; tt < RPW; ++tt) {
        const int t = tb + tt;
        const bool obs = R[tt] != FINF;
        if (obs) tdl += fabs((double)(R[tt] - P[tt]));
        const bool cnt = d.count_scope ? (t < d.m && c < d.n) : obs;
        if (cnt) {
          atomicAdd(&S.u.f.hc[gp.lane][A[tt]], 1);
          atomicAdd(&S.u.f.hr[tl0 + tt][A[tt]], 1);
        }
      }
      S.u.f.tdw[gp.wave][gp.lane] = tdl;
    }
    {
      Top2 cs = top2_id();
#pragma unroll
      for (int tt = 0; tt < RPW; ++tt) cs = top2_add(cs, R[tt] - S.uk[tl0 + tt], tb + tt);
      S.u.f.csw[gp.wave][gp.lane] = cs;
    }
    {
      // lanes over rows: row summary over this wave's columns
      Top2 rs = top2_id();
#pragma unroll
      for (int cc = 0; cc < RPW; ++cc)
        rs = top2_add(rs, RT[cc] - S.vk[cl0 + cc], c0 + cl0 + cc);
      S.u.f.rsw[gp.wave][gp.lane] = rs;
    }
    __syncthreads();
    if (gp.wave == 0) {
      Top2 cs = S.u.f.csw[0][gp.lane];
      for (int w = 1; w < NWAVE; ++w) cs = top2_comb(cs, S.u.f.csw[w][gp.lane]);
      st_top2(&d.colpart[(size_t)rt * d.ldn + c], cs);
      if (full) {
        double s = S.u.f.tdw[0][gp.lane];
        for (int w = 1; w < NWAVE; ++w) s += S.u.f.tdw[w][gp.lane];
        st_coh(&d.tdpart[(size_t)rt * d.ldn + c], s);
      }
    } else if (gp.wave == 1) {
      Top2 rs = S.u.f.rsw[0][gp.lane];
      for (int w = 1; w < NWAVE; ++w) rs = top2_comb(rs, S.u.f.rsw[w][gp.lane]);
      st_top2(&d.rowpart[(size_t)ct * d.ldm + r0 + gp.lane], rs);
    }
    if (full) {
      for (int e = gp.tid; e < TS * d.r; e += NTHR) {
        int x = e / d.r, l = e % d.r;
        int hcv = S.u.f.hc[x][l], hrv = S.u.f.hr[x][l];
        if (hcv && c0 + x < d.n) atomic_add_g(&ccol[(size_t)(c0 + x) * d.r + l], hcv);
        if (hrv && r0 + x < d.m) atomic_add_g(&crow[(size_t)(r0 + x) * d.r + l], hrv);
      }
    }
  }
  if (has_acc && gp.g == 0 && gp.tid == 0) st_coh(&d.closed[k], 1);
}

// Residual summaries of component k from the per-tile partials (fixed tile
// order), for this workgroup's slice of columns and rows; with with_td also
// td_col.
DEV void combine_summaries(Grp& gp, Smem& S, int k, bool with_td) {
  const FitDev& d = *gp.d;
  int lo, hi;
  // columns: chunks of columns whose (column, row tile) partials fit the buffer
  slice(d.n, gp.g, gp.G, lo, hi);
  {
    const int per_chunk = 2048 / d.nrt > 0 ? 2048 / d.nrt : 1;
    for (int c0 = lo; c0 < hi; c0 += per_chunk) {
      const int cn = hi - c0 < per_chunk ? hi - c0 : per_chunk;
      __syncthreads();
      for (int e = gp.tid; e < cn * d.nrt; e += NTHR) {
        const int cc = e / d.nrt, rt = e % d.nrt;
        S.u.c.part[e] = ld_top2(&d.colpart[(size_t)rt * d.ldn + c0 + cc]);
        if (with_td) S.u.c.dpart[e] = ld_atomic(&d.tdpart[(size_t)rt * d.ldn + c0 + cc]);
      }
      __syncthreads();
      for (int cc = gp.tid; cc < cn; cc += NTHR) {
        Top2 cs = top2_id();
        double sum = 0.0;
        for (int rt = 0; rt < d.nrt; ++rt) {
          cs = top2_comb(cs, S.u.c.part[cc * d.nrt + rt]);
          if (with_td) sum += S.u.c.dpart[cc * d.nrt + rt];
        }
        st_top2(&d.colst[(size_t)k * d.ldn + c0 + cc], cs);
        if (with_td) st_coh(&d.td[c0 + cc], sum);
      }
    }
  }
  slice(d.m, gp.g, gp.G, lo, hi);
  {
    const int per_chunk = 2048 / d.nct > 0 ? 2048 / d.nct : 1;
    for (int t0 = lo; t0 < hi; t0 += per_chunk) {
      const int tn = hi - t0 < per_chunk ? hi - t0 : per_chunk;
      __syncthreads();
      for (int e = gp.tid; e < tn * d.nct; e += NTHR) {
        const int tt = e / d.nct, ct = e % d.nct;
        S.u.c.part[e] = ld_top2(&d.rowpart[(size_t)ct * d.ldm + t0 + tt]);
      }
      __syncthreads();
      for (int tt = gp.tid; tt < tn; tt += NTHR) {
        Top2 rs = top2_id();
        for (int ct = 0; ct < d.nct; ++ct) rs = top2_comb(rs, S.u.c.part[tt * d.nct + ct]);
        st_top2(&d.rowst[(size_t)k * d.ldm + t0 + tt], rs);
      }
    }
  }
  __syncthreads();
}

// Ranking by counting: the rank of key c is the number of keys x with
// key[x] > key[c], or key[x] == key[c] and x < c (descending, index
// ascending on ties).  A workgroup ranks up to 64 of its keys at a time:
// with w = their count rounded up to a power of two, thread t counts for key
// t % w over the keys x = t / w, t / w + P, ... (P = NTHR / w partitions), so
// every thread has work however few keys the slice holds; the counts of one
// key are summed over a wave's lanes (xor shuffles) and then over the waves.
struct RankChunk {
  int nk, lg, j, p, P;
};

DEV RankChunk rank_chunk(const Grp& gp, int cb, int hi) {
  RankChunk q;
  q.nk = hi - cb < 64 ? hi - cb : 64;
  q.lg = q.nk <= 1 ? 0 : 32 - __builtin_clz((unsigned)(q.nk - 1));
  q.j = gp.lane & ((1 << q.lg) - 1);
  q.p = gp.tid >> q.lg;
  q.P = NTHR >> q.lg;
  return q;
}

// Counts of the staged keys key_lds[0 .. len) (global indices x0 + x) that
// precede key kc of index c.
DEV int rank_count(const double* key_lds, int len, int x0, int p, int P, double kc, int c) {
  int cnt = 0;
  int x = p;
  for (; x + 3 * P < len; x += 4 * P) {
    const double o0 = key_lds[x], o1 = key_lds[x + P];
    const double o2 = key_lds[x + 2 * P], o3 = key_lds[x + 3 * P];
    cnt += (o0 > kc || (o0 == kc && x0 + x < c)) ? 1 : 0;
    cnt += (o1 > kc || (o1 == kc && x0 + x + P < c)) ? 1 : 0;
    cnt += (o2 > kc || (o2 == kc && x0 + x + 2 * P < c)) ? 1 : 0;
    cnt += (o3 > kc || (o3 == kc && x0 + x + 3 * P < c)) ? 1 : 0;
  }
  for (; x < len; x += P) {
    const double o = key_lds[x];
    cnt += (o > kc || (o == kc && x0 + x < c)) ? 1 : 0;
  }
  return cnt;
}

// Sum of the chunk's counts per key; out[rank] = cb + j for its keys.
DEV void rank_write(Grp& gp, Smem& S, const RankChunk& q, int cb, int cnt, GA int* out) {
  int* part = S.u.s.idx;  // NWAVE x 64 counts
  for (int off = 1 << q.lg; off < 64; off <<= 1) cnt += __shfl_xor(cnt, off);
  if (gp.lane < (1 << q.lg)) part[gp.wave * 64 + gp.lane] = cnt;
  __syncthreads();
  if (gp.tid < q.nk) {
    int rank = 0;
    for (int w = 0; w < NWAVE; ++w) rank += part[w * 64 + gp.tid];
    st_coh(&out[rank], cb + gp.tid);
  }
  __syncthreads();
}

// Rank sort of the keys S.u.s.key[0 .. n) (n <= SORT_MAX), in every
// workgroup at once: each workgroup ranks its slice and writes out[rank] =
// column and, if keys_out is given, keys_out[column] = key.
DEV void rank_slice_lds(Grp& gp, Smem& S, int n, GA int* out, GA double* keys_out) {
  int lo, hi;
  slice(n, gp.g, gp.G, lo, hi);
  for (int cb = lo; cb < hi; cb += 64) {
    const RankChunk q = rank_chunk(gp, cb, hi);
    const int c = cb + q.j;
    int cnt = 0;
    if (q.j < q.nk) cnt = rank_count(S.u.s.key, n, 0, q.p, q.P, S.u.s.key[c], c);
    if (keys_out && gp.tid < q.nk) st_coh(&keys_out[cb + gp.tid], S.u.s.key[cb + gp.tid]);
    rank_write(gp, S, q, cb, cnt, out);
  }
}

// Column order by (td_col descending, index ascending), for up to SORT_MAX
// columns: td_col of every column from the row-tile partials (fixed order)
// into LDS in every workgroup, then the ranks of each workgroup's slice.
DEV void sort_small(Grp& gp, Smem& S) {
  const FitDev& d = *gp.d;
  const auto tdpart = d.tdpart;
  const size_t ldn = d.ldn;
  const int n = d.n, nrt = d.nrt;
  __syncthreads();
  for (int x = gp.tid; x < n; x += NTHR) {
    double v[8];
    double sum = 0.0;
    for (int rt0 = 0; rt0 < nrt; rt0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = rt0 + u < nrt ? ld_atomic(&tdpart[(rt0 + u) * ldn + x]) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += v[u];
    }
    S.u.s.key[x] = sum;
  }
  __syncthreads();
  rank_slice_lds(gp, S, n, d.order, d.td);
}

// Order of wide matrices: every workgroup ranks its slice of columns against
// all the keys (descending, index ascending on ties), staged through LDS in
// chunks of SORT_MAX; 64 columns at a time, lane = column, wave w counting
// the keys x = w, w + NWAVE, ... of each chunk, the eight counts added at
// the end; out[rank] = column.
DEV void sort_by_rank(Grp& gp, Smem& S, const GA double* keys, GA int* out) {
  const FitDev& d = *gp.d;
  const int n = d.n;
  int lo, hi;
  slice(n, gp.g, gp.G, lo, hi);
  // the wave counts live beside the staged keys (SORT_MAX doubles)
  int* part = S.u.s.idx;
  for (int cb = lo; cb < hi; cb += 64) {
    const int c = cb + gp.lane;
    const bool valid = c < hi;
    const double kc = valid ? ld_atomic(&keys[c]) : 0.0;
    int cnt = 0;
    for (int x0 = 0; x0 < n; x0 += SORT_MAX) {
      const int len = n - x0 < SORT_MAX ? n - x0 : SORT_MAX;
      __syncthreads();
      for (int x = gp.tid; x < len; x += NTHR) S.u.s.key[x] = ld_atomic(&keys[x0 + x]);
      __syncthreads();
      int x = gp.wave;
      for (; x + 3 * NWAVE < len; x += 4 * NWAVE) {
        const double o0 = S.u.s.key[x], o1 = S.u.s.key[x + NWAVE];
        const double o2 = S.u.s.key[x + 2 * NWAVE], o3 = S.u.s.key[x + 3 * NWAVE];
        cnt += (o0 > kc || (o0 == kc && x0 + x < c)) ? 1 : 0;
        cnt += (o1 > kc || (o1 == kc && x0 + x + NWAVE < c)) ? 1 : 0;
        cnt += (o2 > kc || (o2 == kc && x0 + x + 2 * NWAVE < c)) ? 1 : 0;
        cnt += (o3 > kc || (o3 == kc && x0 + x + 3 * NWAVE < c)) ? 1 : 0;
      }
      for (; x < len; x += NWAVE) {
        const double o = S.u.s.key[x];
        cnt += (o > kc || (o == kc && x0 + x < c)) ? 1 : 0;
      }
    }
    part[gp.wave * 64 + gp.lane] = cnt;
    __syncthreads();
    if (gp.wave == 0 && valid) {
      int rank = 0;
      for (int w = 0; w < NWAVE; ++w) rank += part[w * 64 + gp.lane];
      st_coh(&out[rank], c);
    }
    __syncthreads();
  }
}

// The same order with every thread counting (the ranking of up to 4096
// columns above) and four staged loads in flight per thread.  Compiled only
// into the kernel for matrices wider than SORT_MAX, so that the register
// allocation of the others stays as it is.
DEV void sort_by_rank_all(Grp& gp, Smem& S, const GA double* keys, GA int* out) {
  const FitDev& d = *gp.d;
  const int n = d.n;
  int lo, hi;
  slice(n, gp.g, gp.G, lo, hi);
  for (int cb = lo; cb < hi; cb += 64) {
    const RankChunk q = rank_chunk(gp, cb, hi);
    const int c = cb + q.j;
    const double kc = q.j < q.nk ? ld_atomic(&keys[c]) : 0.0;
    int cnt = 0;
    for (int x0 = 0; x0 < n; x0 += SORT_MAX) {
      const int len = n - x0 < SORT_MAX ? n - x0 : SORT_MAX;
      __syncthreads();
      for (int x = gp.tid; x < len; x += 4 * NTHR) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          v[u] = x + u * NTHR < len ? ld_atomic(&keys[x0 + x + u * NTHR]) : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (x + u * NTHR < len) S.u.s.key[x + u * NTHR] = v[u];
      }
      __syncthreads();
      if (q.j < q.nk) cnt += rank_count(S.u.s.key, len, x0, q.p, q.P, kc, c);
    }
    rank_write(gp, S, q, cb, cnt, out);
  }
}

// Whole refresh: tile pass, barrier, summaries (and, for matrices up to
// SORT_MAX columns, the column order), barrier.
template <bool WIDE = false>
DEV bool refresh(Grp& gp, Smem& S, int k, bool has_acc, Trial acc, int par, int slot, int i, bool full,
                 int cb) {
  const FitDev& d = *gp.d;
  refresh_tiles(gp, S, k, has_acc, acc, par, slot, i, full, cb);
  if (!group_sync(gp, S)) return false;
  const bool small = d.n <= SORT_MAX;
  combine_summaries(gp, S, k, full && !small);
  if (full && small) sort_small(gp, S);
  if (!group_sync(gp, S)) return false;
  if (full && !small) {
    if (WIDE)
      sort_by_rank_all(gp, S, d.td, d.order);
    else
      sort_by_rank(gp, S, d.td, d.order);
    if (!group_sync(gp, S)) return false;
  }
  return true;
}

// ------------------------------------------------------------ row visit pieces
// Start a row visit: argmax counts, U and closed flags of row i into LDS,
// candidate queue empty.
DEV void row_begin(Grp& gp, Smem& S, int i, int cb, int sel, int start = 0) {
  const FitDev& d = *gp.d;
  if (gp.tid < d.r) {
    S.crow_i[gp.tid] = ld_atomic(&d.crow[((size_t)cb * d.ldm + i) * d.r + gp.tid]);
    S.urow_i[gp.tid] = ld_atomic(&d.Uc[(size_t)gp.tid * d.ldm + i]);
    S.closed_s[gp.tid] = ld_atomic(&d.closed[gp.tid]);
  }
  if (sel == SEL_TD_B) {
    // i0 = the first working row (the column error td_col does not depend on
    // the row, so every row ties and the lowest index is taken); j0 = the
    // column of largest td_col, the first of the order
    if (gp.tid < d.r) S.urow0[gp.tid] = ld_atomic(&d.Uc[(size_t)gp.tid * d.ldm]);
    if (gp.tid == 0) {
      const int j0 = ld_atomic(&d.order[0]);
      float best = 0.0f;
      int kb = 0;
      for (int l = 0; l < d.r; ++l) {
        const float x = ld_atomic(&d.Uc[(size_t)l * d.ldm + i]) + ld_atomic(&d.V[(size_t)l * d.ldn + j0]);
        if (l == 0 || x > best) { best = x; kb = l; }
      }
      S.p_ij0 = best;
      S.f_ij0 = kb;
    }
  }
  if (gp.tid == 0) { S.cq_head = 0; S.cq_n = 0; S.ord_pos = start; S.cur_op = 0; }
  __syncthreads();
}

// TD (Sec. 3.2.1): the visited row's columns by the entry error
// |R_ic - (U (x) V)_ic| descending, index ascending on ties, into d.rord
// (unobserved columns last, key -1).  Values in FP32 as everywhere on the
// value path; the key is the exact widening of the FP32 difference.
DEV double td_entry_key(const FitDev& d, const Smem& S, int i, int c) {
  const float rv = d.Rw[(size_t)i * d.ldn + c];
  if (rv == FINF) return -1.0;
  float p = S.urow_i[0] + ld_atomic(&d.V[c]);
  for (int l = 1; l < d.r; ++l) p = vmax(p, S.urow_i[l] + ld_atomic(&d.V[(size_t)l * d.ldn + c]));
  return (double)fabsf(rv - p);
}

DEV bool row_order_td(Grp& gp, Smem& S, int i) {
  const FitDev& d = *gp.d;
  if (d.n <= SORT_MAX) {
    // every workgroup computes every key in LDS, then ranks its slice
    for (int c = gp.tid; c < d.n; c += NTHR) S.u.s.key[c] = td_entry_key(d, S, i, c);
    __syncthreads();
    rank_slice_lds(gp, S, d.n, d.rord, nullptr);
  } else {
    int lo, hi;
    slice(d.n, gp.g, gp.G, lo, hi);
    for (int c = lo + gp.tid; c < hi; c += NTHR) st_coh(&d.tdrow[c], td_entry_key(d, S, i, c));
    if (!group_sync(gp, S)) return false;
    sort_by_rank(gp, S, d.tdrow, d.rord);
  }
  return group_sync(gp, S);
}

// Keep at least CW candidates of row i queued (observed columns in the
// current order), unless the order is exhausted.  Every workgroup of the
// group builds the same queue.
DEV void refill_candidates(Grp& gp, Smem& S, int i, int sel) {
  const FitDev& d = *gp.d;
  const GA float* Ri = d.Rw + (size_t)i * d.ldn;
  // TD_A, TD_B: the column order; TD: the row's own order; SEQ: every
  // (column, component) pair, both ascending (entry j * RMAX + k);
  // ByElement: the working columns in order
  const bool seq = sel == SEL_SEQ, elem = sel == SEL_ELEM;
  const GA int* ord = sel == SEL_TD ? d.rord : d.order;
  const int total = seq ? d.n * d.r : d.n;
  while (S.cq_n - S.cq_head < CW && S.ord_pos < total) {
    // move the unconsumed tail to the front
    const int keep = S.cq_n - S.cq_head;
    int v = 0;
    if (gp.tid < keep) v = S.cq[S.cq_head + gp.tid];
    __syncthreads();
    if (gp.tid < keep) S.cq[gp.tid] = v;
    const int pos = S.ord_pos + gp.tid;
    int j = -1;
    if (pos < total) {
      if (seq) {
        const int c = pos / d.r;
        j = Ri[c] == FINF ? -1 : c * RMAX + (pos - c * d.r);
      } else if (elem) {
        j = Ri[pos] == FINF ? -1 : pos;
      } else {
        j = ld_atomic(&ord[pos]);
        if (Ri[j] == FINF) j = -1;
      }
    }
    const unsigned long long m = __ballot(j >= 0);
    const int below = __popcll(m & ((1ull << gp.lane) - 1ull));
    if (gp.lane == 0) S.wcount[gp.wave] = __popcll(m);
    __syncthreads();
    int off = keep;
    for (int w = 0; w < gp.wave; ++w) off += S.wcount[w];
    if (j >= 0) S.cq[off + below] = j;
    __syncthreads();
    if (gp.tid == 0) {
      int tot = keep;
      for (int w = 0; w < NWAVE; ++w) tot += S.wcount[w];
      S.cq_head = 0;
      S.cq_n = tot;
      S.ord_pos += NTHR;
    }
    __syncthreads();
  }
}

// Group the trials of S.trials[0 .. nt) for the two passes by key
// op * RMAX + k (operation-major, then component, stable within a key):
// S.byk and the key ranges S.kst.
DEV void group_trials(Grp& gp, Smem& S) {
  // Key counts first (LDS atomics), key starts by a scan; then, NTHR
  // trials at a time in order, ranks within a wave by ballot and offsets
  // from per-wave counts.
  if (gp.tid < 2 * RMAX) S.kcnt[gp.tid] = 0;
  __syncthreads();
  for (int q = gp.tid; q < S.nt; q += NTHR) atomicAdd(&S.kcnt[S.trials[q].op * RMAX + S.trials[q].k], 1);
  __syncthreads();
  if (gp.wave == 0) {
    // lane l: keys l and RMAX + l (F-ULF keys first)
    const int t0 = S.kcnt[gp.lane], t1 = S.kcnt[RMAX + gp.lane];
    int i0 = t0, i1 = t1;
    for (int sft = 1; sft < 64; sft <<= 1) {
      const int v0 = __shfl_up(i0, sft, 64), v1 = __shfl_up(i1, sft, 64);
      if (gp.lane >= sft) { i0 += v0; i1 += v1; }
    }
    const int nulf = __shfl(i0, 63, 64);
    S.kst[gp.lane] = S.kcnt[gp.lane] = i0 - t0;
    S.kst[RMAX + gp.lane] = S.kcnt[RMAX + gp.lane] = nulf + i1 - t1;
    if (gp.lane == 63) S.kst[2 * RMAX] = nulf + i1;
  }
  __syncthreads();
  for (int base = 0; base < S.nt; base += NTHR) {
    const int q = base + gp.tid;
    const bool valid = q < S.nt;
    const int key = valid ? S.trials[q].op * RMAX + S.trials[q].k : -1;
    const unsigned long long below = (1ull << gp.lane) - 1ull;
    int rank = 0, c0 = 0, c1 = 0;  // rank among the wave's trials of the key;
                                   // lane l: the wave's trials of keys l, RMAX + l
    unsigned long long rem = __ballot(valid);
    while (rem) {
      const int kl = __shfl(key, __ffsll((long long)rem) - 1, 64);
      const unsigned long long m = __ballot(valid && key == kl);
      if (valid && key == kl) rank = __popcll(m & below);
      if (gp.lane == kl % RMAX) {
        if (kl >= RMAX) c1 = __popcll(m); else c0 = __popcll(m);
      }
      rem &= ~m;
    }
    S.wk[gp.wave][gp.lane] = c0;
    S.wk[gp.wave][RMAX + gp.lane] = c1;
    __syncthreads();
    if (gp.wave == 0) {
      // every wave's share of each key starts after the earlier trials'
      int run0 = S.kcnt[gp.lane], run1 = S.kcnt[RMAX + gp.lane];
      for (int w = 0; w < NWAVE; ++w) {
        const int a = S.wk[w][gp.lane], b = S.wk[w][RMAX + gp.lane];
        S.wk[w][gp.lane] = run0;
        S.wk[w][RMAX + gp.lane] = run1;
        run0 += a;
        run1 += b;
      }
      S.kcnt[gp.lane] = run0;
      S.kcnt[RMAX + gp.lane] = run1;
    }
    __syncthreads();
    if (valid) S.byk[S.wk[gp.wave][key] + rank] = q;
    __syncthreads();
  }
}

// Next batch of up to T trials from the cursor, in the method's order:
// candidate by candidate, F-ULF then F-URF, skipping no-op trials.  Every
// workgroup of the group computes the same list.
DEV void build_batch(Grp& gp, Smem& S, int i, int T, int cb, int sel) {
  const FitDev& d = *gp.d;
  if (T > d.tmax) T = d.tmax;  // never more trials than the trial buffers hold
  const GA int* ccol = d.ccol + (size_t)cb * d.ldn * d.r;
  if (gp.tid == 0) { S.nt = 0; S.batch_noops = 0; }
  __syncthreads();
  while (true) {
    refill_candidates(gp, S, i, sel);
    const int avail0 = S.cq_n - S.cq_head;
    if (S.nt >= T || avail0 == 0) break;
    const int avail = avail0 < CW ? avail0 : CW;
    // Component of each candidate in the window, four threads per candidate,
    // each over components l = sub, sub + 4, ... (for TD_A the column counts,
    // otherwise V_lj, loaded in one round), NTHR / 4 candidates per round:
    //   TD_A: the index counted most often in row i's and column j's argmax
    //         multisets (lowest on ties);
    //   TD:   f(i, j), the lowest argmax of U_il + V_lj;
    //   TD_B: f(i, j0) if (U (x) V)_{i j0} >= (U (x) V)_{i0 j}, else f(i0, j);
    //   SEQ:  the candidate's own component;
    //   ByElement: f(i, j), and an entry with R_ij = (U (x) V)_ij is skipped.
    {
      const int sub = gp.tid & 3;
#pragma unroll 1
      for (int p0 = 0; p0 < CW; p0 += NTHR / 4) {
        const int p = p0 + (gp.tid >> 2);
        if (p0 < avail && p < avail) {
          const int e = S.cq[S.cq_head + p];
          const int j = sel == SEL_SEQ ? e / RMAX : e;
          if (sel == SEL_TD_A) {
            int cnt[RMAX / 4];
#pragma unroll
            for (int u = 0; u < RMAX / 4; ++u) {
              const int l = sub + 4 * u;
              cnt[u] = l < d.r ? ld_atomic(&ccol[(size_t)j * d.r + l]) : 0;
            }
            int best = -1, kb = 0;
#pragma unroll
            for (int u = 0; u < RMAX / 4; ++u) {
              const int l = sub + 4 * u;
              if (l < d.r) {
                const int v = S.crow_i[l] + cnt[u];
                if (v > best) { best = v; kb = l; }
              }
            }
            S.kval[p][sub] = best;
            S.kbest[p][sub] = kb;
          } else if (sel != SEL_SEQ) {
            float vv[RMAX / 4];
#pragma unroll
            for (int u = 0; u < RMAX / 4; ++u) {
              const int l = sub + 4 * u;
              vv[u] = l < d.r ? ld_atomic(&d.V[(size_t)l * d.ldn + j]) : 0.0f;
            }
            // row i (TD) or row i0 (TD_B): value selects, not address selects
            const bool own = sel == SEL_TD || sel == SEL_ELEM;
            float best = 0.0f;
            int kb = -1;
#pragma unroll
            for (int u = 0; u < RMAX / 4; ++u) {
              const int l = sub + 4 * u;
              if (l < d.r) {
                const float uv = own ? S.urow_i[l] : S.urow0[l];
                const float x = uv + vv[u];
                if (kb < 0 || x > best) { best = x; kb = l; }
              }
            }
            S.kvalf[p][sub] = best;
            S.kbest[p][sub] = kb;
          }
        }
      }
      __syncthreads();
      if (gp.tid < avail) {
        const int q = gp.tid;
        int k = 0;
        int skip = 0;
        if (sel == SEL_TD_A) {
          int best = -1;
          for (int u = 0; u < 4; ++u) {
            const int v = S.kval[q][u], kb = S.kbest[q][u];
            if (v > best || (v == best && kb < k)) { best = v; k = kb; }
          }
        } else if (sel == SEL_SEQ) {
          k = S.cq[S.cq_head + q] % RMAX;
        } else {
          float best = 0.0f;
          int kb = -1;
          for (int u = 0; u < 4; ++u) {
            const int c = S.kbest[q][u];
            if (c < 0) continue;
            const float v = S.kvalf[q][u];
            if (kb < 0 || v > best || (v == best && c < kb)) { best = v; kb = c; }
          }
          k = kb;
          if (sel == SEL_TD_B && S.p_ij0 >= best) k = S.f_ij0;
          if (sel == SEL_ELEM) skip = d.Rw[(size_t)i * d.ldn + S.cq[S.cq_head + q]] == best;
        }
        S.ck[q] = k;
        S.cskip[q] = skip;
      }
    }
    __syncthreads();
    if (gp.tid < avail) {
      // V_kj is loaded again rather than kept from the loads above (V does
      // not change while a batch list is built), next to R_ij
      const int p = gp.tid;
      const int e = S.cq[S.cq_head + p];
      const int j = sel == SEL_SEQ ? e / RMAX : e;
      const int k = S.ck[p];
      const float Rij = d.Rw[(size_t)i * d.ldn + j];
      const float Vkj = ld_atomic(&d.V[(size_t)k * d.ldn + j]);
      const float Uik = S.urow_i[k];
      const float vu = Rij - Vkj, vv2 = Rij - Uik;
      const bool cl = d.noop_rule && S.closed_s[k];
      S.cj[p] = j; S.cvu[p] = vu; S.cvv[p] = vv2;
      S.cnu[p] = cl && vu == Uik;
      S.cnv[p] = cl && vv2 == Vkj;
    }
    __syncthreads();
    // Walk the (candidate, operation) pairs of the window in order: pair
    // x = 2p + op, starting at the cursor's operation.  A pair is consumed
    // while fewer than T - nt trials precede it; consumed no-op pairs count as
    // skipped trials.  Prefix counts by ballot.
    const int nt0 = S.nt, room = T - nt0, nn0 = S.batch_noops, op0 = S.cur_op;
    // A skipped (exact) candidate's pairs are consumed without a trial.
    const int x = gp.tid;
    const bool valid = x < 2 * avail && x >= op0;
    bool noop = false, skip = false;
    if (valid) {
      skip = S.cskip[x >> 1];
      noop = !skip && ((x & 1) ? S.cnv[x >> 1] : S.cnu[x >> 1]);
    }
    const bool kept = valid && !noop && !skip;
    const unsigned long long mk = __ballot(kept);
    const unsigned long long mn = __ballot(valid && noop);
    const unsigned long long below_mask = (1ull << gp.lane) - 1ull;
    if (gp.lane == 0) { S.wcount[gp.wave] = __popcll(mk); S.wnoop[gp.wave] = __popcll(mn); }
    __syncthreads();
    int kept_before = __popcll(mk & below_mask), noop_before = __popcll(mn & below_mask);
    for (int w = 0; w < gp.wave; ++w) { kept_before += S.wcount[w]; noop_before += S.wnoop[w]; }
    const bool consumed = valid && kept_before < room;
    if (consumed && kept) {
      const int slot = nt0 + kept_before;
      Trial tr;
      tr.j = S.cj[x >> 1]; tr.k = S.ck[x >> 1]; tr.op = x & 1;
      tr.val = (x & 1) ? S.cvv[x >> 1] : S.cvu[x >> 1];
      S.trials[slot] = tr;
      S.noops_before[slot] = nn0 + noop_before;
    }
    // the consumed pairs are a prefix of the valid ones: find the last one and
    // count the consumed no-op pairs
    const unsigned long long mc = __ballot(consumed);
    const unsigned long long mcn = __ballot(consumed && noop);
    if (gp.lane == 0) {
      S.wlast[gp.wave] = mc ? gp.wave * 64 + 63 - __clzll(mc) : -1;
      S.wcn[gp.wave] = __popcll(mcn);
    }
    __syncthreads();
    if (gp.tid == 0) {
      int last = -1, kt = 0, nn = 0;
      for (int w = 0; w < NWAVE; ++w) {
        last = S.wlast[w] > last ? S.wlast[w] : last;
        kt += S.wcount[w];
        nn += S.wcn[w];
      }
      S.nt = nt0 + (kt < room ? kt : room);
      S.batch_noops = nn0 + nn;
      const int nxt = last + 1;       // next pair after the last consumed one
      S.cq_head += nxt >> 1;
      S.cur_op = nxt & 1;
    }
    __syncthreads();
  }
  if (gp.tid == 0)
    S.exhausted = (S.cq_n - S.cq_head) == 0 && S.ord_pos >= (sel == SEL_SEQ ? d.n * d.r : d.n);
  group_trials(gp, S);
}

// Evaluate the batch in S.trials: residual pass, error pass, per-trial
// reduction, and the decision (the first trial with e' < thr, or with `best`
// the smallest such e') made by the last workgroup to arrive.
template <bool MR = false, typename Lap>
DEV bool run_batch(Grp& gp, Smem& S, int i, int par, double thr, bool best, Lap& lap) {
  batch_residual_pass<MR>(gp, S, i, par);
  if (!group_sync(gp, S)) return false;
  lap(2);
  batch_eval_pass<MR>(gp, S, i, par);
  clear_prev(gp, S, par ^ 1);
  if (!group_sync(gp, S)) return false;
  lap(6);
  reduce_errors(gp, S, S.nt);
  const bool ok = group_sync_last(gp, S, [&] { decide(gp, S, S.nt, thr, best); });
  lap(3);
  return ok;
}

// A batch of the one trial tr (its key range and list position).
DEV void single_trial(Grp& gp, Smem& S, Trial tr) {
  __syncthreads();
  if (gp.tid == 0) {
    const int key = tr.op * RMAX + tr.k;
    S.trials[0] = tr;
    S.noops_before[0] = 0;
    S.nt = 1;
    S.batch_noops = 0;
    for (int q = 0; q <= 2 * RMAX; ++q) S.kst[q] = q <= key ? 0 : 1;
    S.byk[0] = 0;
  }
  __syncthreads();
}

DEV void clear_trial_vectors(Grp& gp) {
  const FitDev& d = *gp.d;
  const size_t total = (size_t)2 * d.tmax * d.ldmax;
  for (size_t x = (size_t)gp.g * NTHR + gp.tid; x < total; x += (size_t)gp.G * NTHR)
    st_coh(&d.tvec[x], FMAP_INF);
}

// Initial state: residual summaries of every component, counts, td_col,
// the order, and the error of the current state through the same pass as
// every trial (a null trial).
template <bool WIDE = false>
DEV bool fit_init(Grp& gp, Smem& S) {
  const FitDev& d = *gp.d;
  clear_trial_vectors(gp);
  {
    int lo, hi;
    slice(2 * d.ldm * d.r, gp.g, gp.G, lo, hi);
    for (int x = lo + gp.tid; x < hi; x += NTHR) st_coh(&d.crow[x], 0);
    slice(2 * d.ldn * d.r, gp.g, gp.G, lo, hi);
    for (int x = lo + gp.tid; x < hi; x += NTHR) st_coh(&d.ccol[x], 0);
  }
  if (!group_sync(gp, S)) return false;
  for (int k = 0; k < d.r; ++k)
    if (!refresh<WIDE>(gp, S, k, false, Trial{}, 0, 0, 0, k == d.r - 1, 0)) return false;
  if (gp.tid == 0) {
    Trial tr; tr.j = 0; tr.k = 0; tr.op = OP_NULL; tr.val = 0.0f;
    S.trials[0] = tr; S.nt = 1;
    for (int q = 0; q <= 2 * RMAX; ++q) S.kst[q] = q == 0 ? 0 : 1;  // key 0: the null trial
    S.byk[0] = 0; S.prev_nt = 0;
  }
  __syncthreads();
  batch_eval_pass(gp, S, 0, 0);
  if (!group_sync(gp, S)) return false;
  reduce_errors(gp, S, 1);
  if (!group_sync_last(gp, S, [&] {
        if (gp.tid == 0) {
          const double s = ld_atomic(&d.eprime[0]);
          st_coh(&gp.ctl->e, s);
          st_coh(&d.traj[0], s);
          st_coh(&gp.ctl->phase, d.iters > 0 ? 1 : 2);
          st_coh(&gp.ctl->it, 1);
          st_coh(&gp.ctl->row, 0);
          st_coh(&gp.ctl->acc_in_pass, 0);
          st_coh(&gp.ctl->cells, 0ll);
          st_coh(&gp.ctl->cbuf, 0);
        }
      }))
    return false;
  return true;
}

// Statistics and the decision record of a finished row visit (ByRow) or
// segment of one (ByElement), by one thread of the group.
DEV void book(Grp& gp, int it, int i, long long trials, long long noops, long long spec, int acc_j,
              int acc_k, int acc_op, double e_cur) {
  const FitDev& d = *gp.d;
  GA FitCtl* ctl = gp.ctl;
  if (gp.g != 0 || gp.tid != 0) return;
  ctl->trials += trials;
  ctl->spec_trials += spec;
  ctl->noops += noops;
  ctl->cells += trials * (long long)d.omega;
  if (acc_j >= 0) { ctl->accepted += 1; ctl->e = e_cur; }
  if (d.log && ctl->nlog < d.log_cap) {
    LogRec rec;
    rec.iter = it; rec.row = i; rec.trials = (int)trials; rec.noops = (int)noops;
    rec.j = acc_j; rec.k = acc_k; rec.op = acc_op; rec.pad = 0; rec.e = e_cur;
    d.log[ctl->nlog] = rec;
  }
  ctl->nlog += 1;
}

// ------------------------------------------------------------ ByMatrix
// Sec. 3.2.3 and its supplementary pseudocode.  One iteration keys every
// observed cell of the working matrix by
//   err(i, j) = (td_row(i) + td_col(j)) - td(i, j)
// (FP64; td_row summed over j ascending, td_col over i ascending, one thread
// per line, the same order as a plain loop), and tries the cells by err
// descending, ties in row-major order, each with k = f(i, j) of the
// iteration's state and one operation drawn from a counter-based SplitMix64
// stream, until the first strict decrease.  The candidates come in rounds of
// up to T_max: a radix select over the group (8-bit digits of the order-mapped
// key, then of the cell position among equal keys) finds the round's last
// cell, the cells up to it are gathered and ranked, and the next round starts
// after it.

// SplitMix64 output mixing (Steele, Lea, Flood 2014).
DEV unsigned long long sm_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Operation of the c-th cell tried in the fit (c from 0): the c-th output of
// SplitMix64 seeded with seed_ops; F-URF when its top bit is set (a uniform
// draw of at least 1/2), else F-ULF.
DEV int matrix_op(unsigned long long seed_ops, long long c) {
  return (int)(sm_mix(seed_ops + (unsigned long long)(c + 1) * 0x9E3779B97F4A7C15ull) >> 63);
}
// Order-preserving image of a double (0 is never an image of a key >= 0,
// and marks an unobserved cell).
DEV unsigned long long fmap64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Keys of every cell for the iteration (three group barriers).
DEV bool matrix_keys(Grp& gp, Smem& S) {
  const FitDev& d = *gp.d;
  const int m = d.m, n = d.n, r = d.r;
  const size_t cells = (size_t)m * n, stride = (size_t)gp.G * NTHR;
  const size_t first = (size_t)gp.g * NTHR + gp.tid;
  for (size_t q = first; q < cells; q += stride) {
    const int i = (int)(q / n), j = (int)(q % n);
    const float rv = d.Rw[(size_t)i * d.ldn + j];
    float best = ld_atomic(&d.Uc[i]) + ld_atomic(&d.V[j]);
    int arg = 0;
    for (int l = 1; l < r; ++l) {
      const float x = ld_atomic(&d.Uc[(size_t)l * d.ldm + i]) + ld_atomic(&d.V[(size_t)l * d.ldn + j]);
      if (x > best) { best = x; arg = l; }
    }
    st_coh(&d.mfk[q], arg);
    st_coh(&d.mtd[q], rv == FINF ? -1.0 : (double)fabsf(rv - best));
  }
  if (!group_sync(gp, S)) return false;
  for (size_t x = first; x < (size_t)(m + n); x += stride) {
    double sum = 0.0;
    if (x < (size_t)m) {
      for (int j = 0; j < n; ++j) {
        const double t = ld_atomic(&d.mtd[x * n + j]);
        if (t >= 0.0) sum += t;
      }
      st_coh(&d.mtdr[x], sum);
    } else {
      const int j = (int)(x - m);
      for (int i = 0; i < m; ++i) {
        const double t = ld_atomic(&d.mtd[(size_t)i * n + j]);
        if (t >= 0.0) sum += t;
      }
      st_coh(&d.mtdc[j], sum);
    }
  }
  if (!group_sync(gp, S)) return false;
  for (size_t q = first; q < cells; q += stride) {
    const double t = ld_atomic(&d.mtd[q]);
    unsigned long long u = 0;
    if (t >= 0.0) u = fmap64((ld_atomic(&d.mtdr[q / n]) + ld_atomic(&d.mtdc[q % n])) - t);
    st_coh(&d.mkey[q], u);
  }
  return group_sync(gp, S);
}

// A cell after the cursor (have, cu, cq) in the order (key desc, position asc).
DEV bool after_cursor(unsigned long long u, long long q, bool have, unsigned long long cu,
                      long long cq) {
  return u != 0 && (!have || u < cu || (u == cu && q > cq));
}

// One radix-select pass: every workgroup counts the digits of its cells that
// pass `in` into LDS and adds the counts into histogram h; after the barrier
// one thread walks h (from the top digit down, or up with `up`) to the digit
// holding the want-th cell (S.m_want), and want becomes the rank within that
// digit.  The digit goes to `digit` (-1 if h holds fewer cells); false when
// the fit was aborted.
template <typename In>
DEV bool radix_pass(Grp& gp, Smem& S, GA int* h, In in, bool up, int& want, int& digit) {
  const FitDev& d = *gp.d;
  const size_t cells = (size_t)d.m * d.n, stride = (size_t)gp.G * NTHR;
  int* lh = S.u.s.idx;
  if (gp.tid < 256) lh[gp.tid] = 0;
  __syncthreads();
  for (size_t q = (size_t)gp.g * NTHR + gp.tid; q < cells; q += stride) {
    int dig;
    if (in(q, dig)) atomicAdd(&lh[dig], 1);
  }
  __syncthreads();
  if (gp.tid < 256 && lh[gp.tid]) atomic_add_g(&h[gp.tid], lh[gp.tid]);
  if (!group_sync(gp, S)) return false;
  if (gp.tid == 0) {
    int w = S.m_want, found = -1;
    for (int x = 0; x < 256; ++x) {
      const int b = up ? x : 255 - x;
      const int c = ld_atomic(&h[b]);
      if (w <= c) { found = b; break; }
      w -= c;
    }
    S.m_want = w;
    S.m_count = found;
  }
  __syncthreads();
  want = S.m_want;
  digit = S.m_count;
  __syncthreads();
  return true;
}

// The next round of candidates after the cursor into mlist_q / mlist_k, in
// order; S.m_count gets their number (0: none left).  The cursor moves to
// the round's last cell.
DEV bool matrix_select(Grp& gp, Smem& S, bool have) {
  const FitDev& d = *gp.d;
  GA FitCtl* ctl = gp.ctl;
  const unsigned long long cu = have ? ld_atomic(&ctl->mlast_u) : 0ull;
  const long long cq = have ? ld_atomic(&ctl->mlast_q) : -1ll;
  const auto mkey = d.mkey;
  {
    int lo, hi;
    slice(MATRIX_HIST * 256, gp.g, gp.G, lo, hi);
    for (int x = lo + gp.tid; x < hi; x += NTHR) st_coh(&d.mhist[x], 0);
    if (gp.g == 0 && gp.tid == 0) st_coh(&d.mcnt[0], 0);
  }
  if (!group_sync(gp, S)) return false;
  // the eligible count first (pass 0 counts every digit), then the key of
  // the round's last cell digit by digit
  unsigned long long pref = 0;
  int want = 0, digit = 0;
  if (gp.tid == 0) S.m_want = 1;
  __syncthreads();
  for (int p = 0; p < 8; ++p) {
    const int sh = 56 - 8 * p;
    const unsigned long long pp = pref;
    auto in = [&](size_t q, int& dig) {
      const unsigned long long u = ld_atomic(&mkey[q]);
      if (!after_cursor(u, (long long)q, have, cu, cq)) return false;
      if (p > 0 && (u >> (sh + 8)) != (pp >> (sh + 8))) return false;
      dig = (int)((u >> sh) & 255);
      return true;
    };
    if (p == 0) {
      // total of the first histogram: the round takes min(T_max, eligible)
      if (!radix_pass(gp, S, d.mhist, in, false, want, digit)) return false;
      if (gp.tid == 0) {
        long long tot = 0;
        for (int x = 0; x < 256; ++x) tot += ld_atomic(&d.mhist[x]);
        S.m_pref = (unsigned long long)tot;
      }
      __syncthreads();
      const long long tot = (long long)S.m_pref;
      if (tot == 0) {
        if (gp.tid == 0) S.m_count = 0;
        __syncthreads();
        return true;
      }
      // redo the walk of histogram 0 with the round's size
      if (gp.tid == 0) {
        int w = tot < d.tmax ? (int)tot : d.tmax, bb = 255;
        for (; bb >= 0; --bb) {
          const int c = ld_atomic(&d.mhist[bb]);
          if (w <= c) break;
          w -= c;
        }
        S.m_want = w;
        S.m_count = bb;
        S.m_used = tot < d.tmax ? (int)tot : d.tmax;  // the round's size
      }
      __syncthreads();
      want = S.m_want;
      pref |= (unsigned long long)S.m_count << sh;
    } else {
      if (!radix_pass(gp, S, d.mhist + p * 256, in, false, want, digit)) return false;
      pref |= (unsigned long long)digit << sh;
    }
  }
  const int round = S.m_used;
  // among the cells with that key, the want-th smallest position
  unsigned qpref = 0;
  for (int p = 0; p < 4; ++p) {
    const int sh = 24 - 8 * p;
    const unsigned qp = qpref;
    auto in = [&](size_t q, int& dig) {
      const unsigned long long u = ld_atomic(&mkey[q]);
      if (u != pref || !after_cursor(u, (long long)q, have, cu, cq)) return false;
      if (p > 0 && ((unsigned)q >> (sh + 8)) != (qp >> (sh + 8))) return false;
      dig = (int)(((unsigned)q >> sh) & 255u);
      return true;
    };
    if (!radix_pass(gp, S, d.mhist + (8 + p) * 256, in, true, want, digit)) return false;
    qpref |= (unsigned)digit << sh;
  }
  // gather the round's cells (any order), then rank them
  {
    const size_t cells = (size_t)d.m * d.n, stride = (size_t)gp.G * NTHR;
    for (size_t q = (size_t)gp.g * NTHR + gp.tid; q < cells; q += stride) {
      const unsigned long long u = ld_atomic(&mkey[q]);
      if (!after_cursor(u, (long long)q, have, cu, cq)) continue;
      if (u > pref || (u == pref && (unsigned)q <= qpref)) {
        const int slot = __hip_atomic_fetch_add(&d.mcnt[0], 1, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        if (slot < round) {
          st_coh(&d.mgat_u[slot], u);
          st_coh(&d.mgat_q[slot], (int)q);
        }
      }
    }
  }
  if (!group_sync(gp, S)) return false;
  if (ld_atomic(&d.mcnt[0]) != round) {
    // the gathered cells must be exactly the selected ones
    if (gp.tid == 0) {
      int zero = 0;
      __hip_atomic_compare_exchange_strong(&ctl->status, &zero, ST_INTERNAL, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return false;
  }
  unsigned long long* ku = reinterpret_cast<unsigned long long*>(S.u.s.key);
  int* kq = S.u.s.idx;
  for (int e = gp.tid; e < round; e += NTHR) {
    ku[e] = ld_atomic(&d.mgat_u[e]);
    kq[e] = ld_atomic(&d.mgat_q[e]);
  }
  __syncthreads();
  int lo, hi;
  slice(round, gp.g, gp.G, lo, hi);
  for (int e = lo + gp.tid; e < hi; e += NTHR) {
    const unsigned long long u = ku[e];
    const int q = kq[e];
    int rank = 0;
    for (int x = 0; x < round; ++x) rank += (ku[x] > u || (ku[x] == u && kq[x] < q)) ? 1 : 0;
    st_coh(&d.mlist_q[rank], q);
    st_coh(&d.mlist_k[rank], ld_atomic(&d.mfk[q]));
    if (rank == round - 1) {
      st_coh(&ctl->mlast_u, u);
      st_coh(&ctl->mlast_q, (long long)q);
    }
  }
  if (gp.tid == 0) S.m_count = round;
  return group_sync(gp, S);
}

// Next batch of up to T trials from list position pos: one operation per
// candidate (drawn by its position in the fit's draw sequence, draw0 being
// that of position pos), no-op skips, trials in order with their rows in
// S.trow.  Returns the candidates consumed.
DEV int build_batch_matrix(Grp& gp, Smem& S, int pos, int L, int T, long long draw0) {
  const FitDev& d = *gp.d;
  if (T > d.tmax) T = d.tmax;
  if (gp.tid == 0) { S.nt = 0; S.batch_noops = 0; S.m_used = 0; }
  __syncthreads();
  while (true) {
    const int used = S.m_used, nt0 = S.nt, nn0 = S.batch_noops;
    const int left = L - pos - used;
    if (nt0 >= T || left <= 0) break;
    const int x = gp.tid;
    const bool valid = x < left;
    bool noop = false;
    Trial tr;
    tr.j = 0; tr.k = 0; tr.op = OP_ULF; tr.val = 0.0f;
    int row = 0;
    if (valid) {
      const int q = ld_atomic(&d.mlist_q[pos + used + x]);
      const int k = ld_atomic(&d.mlist_k[pos + used + x]);
      const int i = q / d.n, j = q - i * d.n;
      const int op = matrix_op(d.seed_ops, draw0 + used + x);
      const float Rij = d.Rw[(size_t)i * d.ldn + j];
      const float Uik = ld_atomic(&d.Uc[(size_t)k * d.ldm + i]);
      const float Vkj = ld_atomic(&d.V[(size_t)k * d.ldn + j]);
      const float val = op == OP_ULF ? Rij - Vkj : Rij - Uik;
      noop = d.noop_rule && S.closed_s[k] && (op == OP_ULF ? val == Uik : val == Vkj);
      tr.j = j; tr.k = k; tr.op = op; tr.val = val;
      row = i;
    }
    const bool kept = valid && !noop;
    const unsigned long long mk = __ballot(kept);
    const unsigned long long mn = __ballot(valid && noop);
    const unsigned long long below = (1ull << gp.lane) - 1ull;
    if (gp.lane == 0) { S.wcount[gp.wave] = __popcll(mk); S.wnoop[gp.wave] = __popcll(mn); }
    __syncthreads();
    int kept_before = __popcll(mk & below), noop_before = __popcll(mn & below);
    for (int w = 0; w < gp.wave; ++w) { kept_before += S.wcount[w]; noop_before += S.wnoop[w]; }
    const int room = T - nt0;
    const bool consumed = valid && kept_before < room;
    if (consumed && kept) {
      S.trials[nt0 + kept_before] = tr;
      S.trow[nt0 + kept_before] = row;
      S.noops_before[nt0 + kept_before] = nn0 + noop_before;
    }
    const unsigned long long mc = __ballot(consumed);
    const unsigned long long mcn = __ballot(consumed && noop);
    if (gp.lane == 0) {
      S.wlast[gp.wave] = mc ? gp.wave * 64 + 63 - __clzll(mc) : -1;
      S.wcn[gp.wave] = __popcll(mcn);
    }
    __syncthreads();
    if (gp.tid == 0) {
      int last = -1, kt = 0, nn = 0;
      for (int w = 0; w < NWAVE; ++w) {
        last = S.wlast[w] > last ? S.wlast[w] : last;
        kt += S.wcount[w];
        nn += S.wcn[w];
      }
      S.nt = nt0 + (kt < room ? kt : room);
      S.batch_noops = nn0 + nn;
      S.m_used = used + last + 1;
    }
    __syncthreads();
  }
  if (gp.tid == 0) S.exhausted = pos + S.m_used >= L;
  group_trials(gp, S);
  return S.m_used;
}

// One ByMatrix iteration: keys, then rounds of candidates in batches until
// the first accepted update or none is left (then *acc_iter stays false).
template <typename Lap>
DEV bool matrix_iteration(Grp& gp, Smem& S, int it, int& cb, int& par, double& e_cur,
                          bool& acc_iter, int& seg_t, Lap& lap) {
  const FitDev& d = *gp.d;
  GA FitCtl* ctl = gp.ctl;
  acc_iter = false;
  if (gp.tid < d.r) S.closed_s[gp.tid] = ld_atomic(&d.closed[gp.tid]);
  __syncthreads();
  if (!matrix_keys(gp, S)) return false;
  lap(0);
  long long draws = ld_atomic(&ctl->mdraws);
  long long trials = 0, noops = 0, spec = 0;
  int acc_row = -1, acc_j = -1, acc_k = -1, acc_op = -1;
  bool have = false;
  while (!acc_iter) {
    if (!matrix_select(gp, S, have)) return false;
    have = true;
    const int L = S.m_count;
    lap(1);
    if (L == 0) break;
    int pos = 0, T = seg_t;
    while (pos < L) {
      const int used = build_batch_matrix(gp, S, pos, L, T, draws + pos);
      lap(1);
      const int nt = S.nt;
      if (nt == 0) { noops += S.batch_noops; pos += used; continue; }
      if (!run_batch<true>(gp, S, 0, par, e_cur, false, lap)) return false;
      const int dec = ld_atomic(&ctl->decision);
      spec += nt;
      if (gp.tid == 0) S.prev_nt = nt;
      if (dec >= 0) {
        trials += dec + 1;
        noops += S.noops_before[dec];
        const Trial tr = S.trials[dec];
        acc_row = S.trow[dec];
        acc_j = tr.j; acc_k = tr.k; acc_op = tr.op;
        draws += pos + dec + S.noops_before[dec] + 1;
        e_cur = ld_atomic(&ctl->e_new);
        // the keys of the next iteration are computed afresh: no counts or order
        if (!refresh(gp, S, tr.k, true, tr, par, dec, acc_row, false, cb ^ 1)) return false;
        cb ^= 1;
        lap(4);
        par ^= 1;
        acc_iter = true;
        break;
      }
      trials += nt;
      noops += S.batch_noops;
      par ^= 1;
      pos += used;
      T = T * 2 > d.tmax ? d.tmax : T * 2;
    }
    if (!acc_iter) draws += L;
    int t = 16;
    while (t < trials) t *= 2;
    seg_t = t > d.tmax ? d.tmax : t;
  }
  if (gp.g == 0 && gp.tid == 0) st_coh(&ctl->mdraws, draws);
  book(gp, it, acc_row, trials, noops, spec, acc_j, acc_k, acc_op, e_cur);
  return true;
}


// ByElement row visit (Sec. 3.2.2): the row's observed entries in working
// column order, k = f(i, j), exact entries skipped, F-ULF then F-URF.  An
// accepted update ends a segment (its record is written) and the visit goes
// on from the next entry with the new state; the last segment closes the
// visit with j = -1.  Each segment's first batch is sized from the trials
// the previous segment needed.
template <typename Lap>
DEV bool elem_row_visit(Grp& gp, Smem& S, int i, int it, int& cb, int& par, double& e_cur,
                        int& acc_pass, int& seg_t, Lap& lap) {
  const FitDev& d = *gp.d;
  GA FitCtl* ctl = gp.ctl;
  int start = 0;
  while (true) {
    row_begin(gp, S, i, cb, SEL_ELEM, start);
    lap(0);
    int T = seg_t;
    long long trials = 0, noops = 0, spec = 0;
    int acc_j = -1, acc_k = -1, acc_op = -1;
    while (true) {
      build_batch(gp, S, i, T, cb, SEL_ELEM);
      lap(1);
      const int nt = S.nt;
      if (nt == 0) { noops += S.batch_noops; break; }
      if (!run_batch(gp, S, i, par, e_cur, false, lap)) return false;
      const int dec = ld_atomic(&ctl->decision);
      spec += nt;
      if (gp.tid == 0) S.prev_nt = nt;
      if (dec >= 0) {
        trials += dec + 1;
        noops += S.noops_before[dec];
        const Trial tr = S.trials[dec];
        acc_j = tr.j; acc_k = tr.k; acc_op = tr.op;
        e_cur = ld_atomic(&ctl->e_new);
        // ByElement needs neither the argmax counts nor the column order
        if (!refresh(gp, S, tr.k, true, tr, par, dec, i, false, cb ^ 1)) return false;
        cb ^= 1;
        lap(4);
        par ^= 1;
        break;
      }
      trials += nt;
      noops += S.batch_noops;
      par ^= 1;
      if (S.exhausted) break;
      T = T * 2 > d.tmax ? d.tmax : T * 2;
    }
    int t = 16;
    while (t < trials) t *= 2;
    seg_t = t > d.tmax ? d.tmax : t;
    if (acc_j >= 0) ++acc_pass;
    book(gp, it, i, trials, noops, spec, acc_j, acc_k, acc_op, e_cur);
    lap(5);
    if (acc_j < 0) return true;
    start = acc_j + 1;
  }
}

// Run the fit from its saved state for at most max_rows row visits (0: no
// limit).  All workgroups of the group execute the same control flow.
// MODE 0 is FastSTMF's TD_A alone, compiled without the code of the other
// selections (MODE 3: the same for matrices wider than SORT_MAX, with the
// all-thread ranking of the column order); MODE 1 runs any ByRow selection
// or ByElement; MODE 2 ByMatrix (batches of trials of different rows).  A ByRow row visit (Algorithm 3; the selections of
// Sec. 3.2.1) runs batches of trials until the first accepted update (SEQ:
// every trial, then the best), its refresh and the visit's record; it stays
// written out here rather than in a function of its own, which measured
// 1.3% slower on the TD_A fit (register allocation around the passes).
template <int MODE>
DEV void fit_run(Grp& gp, Smem& S, int max_rows) {
  const FitDev& d = *gp.d;
  const int sel = MODE == 0 || MODE == 3 ? (int)SEL_TD_A : MODE == 2 ? (int)SEL_MATRIX : d.sel;
  GA FitCtl* ctl = gp.ctl;
  if (gp.tid == 0) { S.prev_nt = 0; S.status = 0; }
  __syncthreads();
  if (ld_atomic(&ctl->phase) == 0) {
    if (!fit_init<MODE == 3>(gp, S)) return;
  } else {
    // a resumed launch: the trial vectors of both parities must start clean
    clear_trial_vectors(gp);
    if (!group_sync(gp, S)) return;
  }
  double e_cur = ld_atomic(&ctl->e);
  int it = ld_atomic(&ctl->it), row = ld_atomic(&ctl->row);
  int acc_pass = ld_atomic(&ctl->acc_in_pass);
  int phase = ld_atomic(&ctl->phase);
  int cb = ld_atomic(&ctl->cbuf);
  int rows_done = 0;
  int par = 0;
  // leader-side phase timers: 0 row start, 1 batch list, 2 residual pass,
  // 6 error pass, 3 error reduction and decision, 4 refresh, 5 bookkeeping
  long long ticks[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long tmark = __builtin_amdgcn_s_memrealtime();
  auto lap = [&](int which) {
    unsigned long long now = __builtin_amdgcn_s_memrealtime();
    ticks[which] += (long long)(now - tmark);
    tmark = now;
  };
  int seg_t = d.t0;  // ByElement, ByMatrix: first batch of the next segment or round
  int last_trials = 0;  // ByRow: trials the last row visit needed (0: none yet)
  while (MODE == 2 && phase == 1) {
    // one ByMatrix iteration per step (counted as a row visit)
    if (max_rows > 0 && rows_done >= max_rows) break;
    bool acc_iter = false;
    if (!matrix_iteration(gp, S, it, cb, par, e_cur, acc_iter, seg_t, lap)) return;
    ++rows_done;
    if (gp.g == 0 && gp.tid == 0) {
      ctl->row_visits += 1;
      st_coh(&d.traj[it], e_cur);
    }
    const bool small = d.eps > 0.0 && (ld_atomic(&d.traj[it - 1]) - e_cur) < d.eps;
    if (!acc_iter || small || it == d.iters) {
      if (gp.g == 0 && gp.tid == 0)
        for (int q = it + 1; q <= d.iters; ++q) d.traj[q] = e_cur;
      phase = 2;
    }
    if (gp.g == 0 && gp.tid == 0) {
      ctl->iters_done = it;
      ctl->it = it + 1; ctl->row = 0; ctl->acc_in_pass = 0; ctl->phase = phase; ctl->cbuf = cb;
    }
    ++it;
    lap(5);
  }
  while (MODE != 2 && phase == 1) {
    if (max_rows > 0 && rows_done >= max_rows) break;
    const int i = row;
    if (sel == SEL_ELEM) {
      if (!elem_row_visit(gp, S, i, it, cb, par, e_cur, acc_pass, seg_t, lap)) return;
    } else {
      row_begin(gp, S, i, cb, sel);
      if (sel == SEL_TD && !row_order_td(gp, S, i)) return;
      lap(0);
      // SEQ evaluates every trial of the row: full batches, the best one kept
      const bool seq = sel == SEL_SEQ;
      // first batch: sized from the trials this row's previous visit needed,
      // or on a row's first visit from the trials the last row visit needed
      // (at least t0, the batch whose evaluation costs about what a batch's
      // fixed steps do); batch sizes change which trials are evaluated
      // speculatively, never the outcome
      const int prev_trials = ld_atomic(&d.rowt[i]);
      int T = d.t0;
      if (seq) {
        T = d.tmax;
      } else if (prev_trials > 0) {
        T = 16;
        while (T < prev_trials) T *= 2;
      } else {
        while (T < last_trials) T *= 2;
      }
      if (T > d.tmax) T = d.tmax;  // the trial buffers hold tmax trials
      long long row_trials = 0, row_noops = 0, row_spec = 0;
      int acc_j = -1, acc_k = -1, acc_op = -1;
      double e_best = e_cur;
      Trial best_tr;
      best_tr.j = -1; best_tr.k = 0; best_tr.op = OP_NULL; best_tr.val = 0.0f;
      while (true) {
        build_batch(gp, S, i, T, cb, sel);
        lap(1);
        const int nt = S.nt;
        if (nt == 0) { row_noops += S.batch_noops; break; }
        if (!run_batch(gp, S, i, par, seq ? e_best : e_cur, seq, lap)) return;
        const int dec = ld_atomic(&ctl->decision);
        row_spec += nt;
        if (gp.tid == 0) S.prev_nt = nt;
        if (seq) {
          row_trials += nt;
          row_noops += S.batch_noops;
          if (dec >= 0) { best_tr = S.trials[dec]; e_best = ld_atomic(&ctl->e_new); }
          par ^= 1;
          if (S.exhausted) break;
          continue;
        }
        if (dec >= 0) {
          row_trials += dec + 1;
          row_noops += S.noops_before[dec];
          const Trial tr = S.trials[dec];
          acc_j = tr.j; acc_k = tr.k; acc_op = tr.op;
          e_cur = ld_atomic(&ctl->e_new);
          // the argmax counts and the column order serve TD_A and TD_B only
          if (!refresh<MODE == 3>(gp, S, tr.k, true, tr, par, dec, i, sel == SEL_TD_A || sel == SEL_TD_B,
                       cb ^ 1))
            return;
          cb ^= 1;
          lap(4);
          par ^= 1;
          break;
        }
        row_trials += nt;
        row_noops += S.batch_noops;
        par ^= 1;
        if (S.exhausted) break;
        T = T * 2 > d.tmax ? d.tmax : T * 2;
      }
      if (seq && best_tr.j >= 0) {
        // the chosen trial once more, alone, for its vectors (the evaluation is
        // deterministic: it reproduces the error it was chosen for)
        single_trial(gp, S, best_tr);
        if (!run_batch(gp, S, i, par, e_cur, false, lap)) return;
        row_spec += 1;
        if (gp.tid == 0) S.prev_nt = 1;
        if (ld_atomic(&ctl->decision) != 0 || ld_atomic(&ctl->e_new) != e_best) {
          if (gp.tid == 0) {
            int zero = 0;
            __hip_atomic_compare_exchange_strong(&ctl->status, &zero, ST_INTERNAL, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          return;
        }
        acc_j = best_tr.j; acc_k = best_tr.k; acc_op = best_tr.op;
        e_cur = e_best;
        if (!refresh(gp, S, best_tr.k, true, best_tr, par, 0, i, false, cb ^ 1)) return;
        cb ^= 1;
        lap(4);
        par ^= 1;
      }
      if (acc_j >= 0) ++acc_pass;
      last_trials = (int)(row_trials > 0 ? row_trials : 1);
      if (gp.g == 0 && gp.tid == 0) st_coh(&d.rowt[i], last_trials);
      book(gp, it, i, row_trials, row_noops, row_spec, acc_j, acc_k, acc_op, e_cur);
    }
    if (gp.g == 0 && gp.tid == 0) ctl->row_visits += 1;
    ++row;
    ++rows_done;
    if (row == d.m) {
      if (gp.g == 0 && gp.tid == 0) st_coh(&d.traj[it], e_cur);
      const bool fixed = acc_pass == 0;
      const bool small = d.eps > 0.0 && (ld_atomic(&d.traj[it - 1]) - e_cur) < d.eps;
      if (fixed || small || it == d.iters) {
        if (gp.g == 0 && gp.tid == 0)
          for (int q = it + 1; q <= d.iters; ++q) d.traj[q] = e_cur;
        phase = 2;
      }
      if (gp.g == 0 && gp.tid == 0) ctl->iters_done = it;
      ++it;
      row = 0;
      acc_pass = 0;
    }
    if (gp.g == 0 && gp.tid == 0) {
      ctl->it = it; ctl->row = row; ctl->acc_in_pass = acc_pass; ctl->phase = phase;
      ctl->cbuf = cb;
    }
    lap(5);
  }
  if (gp.g == 0 && gp.tid == 0)
    for (int q = 0; q < 8; ++q) ctl->phase_ticks[q] += ticks[q];
  group_sync(gp, S);
}

// Which fit each workgroup works on.  With a queue (batched fits) the grid
// is cut into groups of qgroup workgroups; each group takes fits from the
// queue one after another (its first workgroup takes the next index and
// publishes it through the group's control block gctl[group], behind a
// group barrier) and runs each on its qgroup workgroups; a group leaves once
// the queue is exhausted.  Without a queue the fits own consecutive ranges
// of the grid, fits[f].gsize workgroups each in table order (one fit over
// the whole grid, or several side by side), and a workgroup beyond the last
// range has nothing to do.  fit_run has one call site, so it is expanded
// once per kernel.
template <int MODE>
DEV void fit_kernel_body(const FitDev* __restrict__ fits, int nfits, int max_rows,
                         unsigned* __restrict__ queue, int qgroup, FitCtl* __restrict__ gctl,
                         BarTree* __restrict__ gbar) {
  extern __shared__ __align__(16) char smem_raw[];
  Smem& S = *reinterpret_cast<Smem*>(smem_raw);
  Grp gp;
  gp.tid = threadIdx.x;
  gp.lane = threadIdx.x & 63;
  gp.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int b = (int)blockIdx.x;
  while (true) {
    int fid;
    if (queue) {
      // the group's own barrier, on its control block
      Grp gq = gp;
      gq.g = b % qgroup;
      gq.G = qgroup;
      gq.d = nullptr;
      gq.wait = BARRIER_TIMEOUT;
      gq.ctl = (GA FitCtl*)(gctl + b / qgroup);
      gq.bar = gbar ? (GA BarTree*)(gbar + b / qgroup) : nullptr;
      if (gq.g == 0 && gq.tid == 0) st_coh(&gq.ctl->decision, (int)atomicAdd(queue, 1u));
      if (!group_sync(gq, S)) break;
      fid = ld_atomic(&gq.ctl->decision);
      // every workgroup has read the index before the next one is taken
      if (!group_sync(gq, S)) break;
      gp.g = gq.g;
      gp.G = qgroup;
    } else {
      if (b < 0) break;
      fid = 0;
      while (fid < nfits && b >= fits[fid].gsize) b -= fits[fid].gsize, ++fid;
      gp.g = b;
      gp.G = fid < nfits ? fits[fid].gsize : 1;
      b = -1;
    }
    if (fid >= nfits) break;
    gp.d = &fits[fid];
    gp.ctl = fits[fid].ctl;
    gp.bar = fits[fid].bar;
    gp.wait = fits[fid].bar_wait < 0 ? 0ull
              : fits[fid].bar_wait > 0 ? (unsigned long long)fits[fid].bar_wait : BARRIER_TIMEOUT;
    if (ld_atomic(&gp.ctl->phase) != 2) fit_run<MODE>(gp, S, max_rows);
  }
}

// FastSTMF (TD_A) fits.
__global__ void __launch_bounds__(NTHR) fit_kernel(const FitDev* __restrict__ fits, int nfits,
                                                   int max_rows,
                                                   unsigned* __restrict__ queue, int qgroup, FitCtl* __restrict__ gctl,
    BarTree* __restrict__ gbar) {
  fit_kernel_body<0>(fits, nfits, max_rows, queue, qgroup, gctl, gbar);
}

// Fits with any ByRow selection (all fits of one launch share it).
__global__ void __launch_bounds__(NTHR) fit_kernel_sel(const FitDev* __restrict__ fits, int nfits,
                                                       int max_rows,
                                                       unsigned* __restrict__ queue, int qgroup, FitCtl* __restrict__ gctl,
    BarTree* __restrict__ gbar) {
  fit_kernel_body<1>(fits, nfits, max_rows, queue, qgroup, gctl, gbar);
}

// FastSTMF (TD_A) fits on matrices wider than SORT_MAX columns (the same
// fit; the column order ranked with every thread counting).
__global__ void __launch_bounds__(NTHR) fit_kernel_wide(const FitDev* __restrict__ fits, int nfits,
                                                        int max_rows,
                                                        unsigned* __restrict__ queue, int qgroup, FitCtl* __restrict__ gctl,
    BarTree* __restrict__ gbar) {
  fit_kernel_body<3>(fits, nfits, max_rows, queue, qgroup, gctl, gbar);
}

// ByMatrix fits.
__global__ void __launch_bounds__(NTHR) fit_kernel_matrix(const FitDev* __restrict__ fits,
                                                          int nfits, int max_rows,
                                                          unsigned* __restrict__ queue, int qgroup, FitCtl* __restrict__ gctl,
    BarTree* __restrict__ gbar) {
  fit_kernel_body<2>(fits, nfits, max_rows, queue, qgroup, gctl, gbar);
}

size_t fit_smem_bytes() { return sizeof(Smem); }

}  // namespace stmf
