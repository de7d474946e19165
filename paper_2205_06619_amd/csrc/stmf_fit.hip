// FastSTMF fit engine for gfx950: one persistent kernel runs Algorithm 3
// (ByRow, random row permutation, TD_A, wide orientation) on device, with no
// host round trip per trial.
//
// A "group" of G workgroups owns one fit (G = 1 for the batched and serving
// paths, G = the whole grid for one large fit).  The working matrix is cut
// into 64 x 64 tiles; workgroup g of the group takes tiles g, g + G, ...
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
// widened to FP64 and summed in a fixed order (lane, tile, workgroup), so a
// trial's error depends only on the state and the trial.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "stmf_internal.h"

namespace stmf {

#define DEV __device__ __forceinline__

static constexpr float FINF = __builtin_huge_valf();
static constexpr unsigned long long BARRIER_TIMEOUT = 400000000ull;  // 4 s at 100 MHz
static constexpr int ST_TIMEOUT = 7;

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

template <typename T>
DEV T ld_atomic(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ LDS layout
struct BatchScratch {
  float sA[TMAX][TS];        // per trial: value of the changed U column at the tile rows
  float sB[TMAX][TS];        // per trial: value of the changed V row at the tile columns
  double wacc[TMAX][TS];     // per trial, per lane running FP64 sums over this WG's tiles
};
struct RefreshScratch {
  int hc[TS][RMAX];          // argmax histogram of the tile columns
  int hr[TS][RMAX];          // argmax histogram of the tile rows
  double tdw[NWAVE][TS];
  Top2 csw[NWAVE][TS];
  Top2 rsw[NWAVE][TS];
};
struct Smem {
  union {
    BatchScratch b;
    RefreshScratch f;
  } u;
  float Ps[TS][TS + 1];      // tile of max over l != k of U_tl + V_lc
  Trial trials[TMAX];
  int noops_before[TMAX];
  int prev_ops[TMAX];
  int kdistinct[TMAX];
  int prev_nt;
  int nt;
  int nk;
  int batch_noops;
  int cur_q, cur_op;         // cursor in the candidate list
  int exhausted;
  int is_last;
  int status;
  // candidate scan scratch
  int cj[64], ck[64];
  float cvu[64], cvv[64];
  int cnu[64], cnv[64];
  int scan[NTHR + 1];
};

struct Grp {
  const FitDev* d;
  FitCtl* ctl;
  int g, G;
  int lane, wave, tid;
};

// ------------------------------------------------------------ group barrier
// Sense-reversing barrier over the group's workgroups with a bounded wait: a
// wait longer than BARRIER_TIMEOUT (or any other workgroup's abort) sets the
// fit's status and every workgroup leaves the fit.  If `last_work` is set, the
// last workgroup to arrive runs it before releasing the others.  Returns false
// when the fit has been aborted.
template <typename F>
DEV bool group_sync_last(Grp& gp, Smem& S, F last_work) {
  FitCtl* ctl = gp.ctl;
  __syncthreads();
  if (gp.G == 1) {
    S.is_last = 1;
  } else if (gp.tid == 0) {
    unsigned gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned old = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT);
    S.is_last = (old == (unsigned)gp.G - 1) ? 1 : 0;
    if (!S.is_last) {
      unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (__builtin_amdgcn_s_memrealtime() - t0 > BARRIER_TIMEOUT) {
          int zero = 0;
          __hip_atomic_compare_exchange_strong(&ctl->status, &zero, ST_TIMEOUT, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
  if (S.is_last) {
    last_work();
    __syncthreads();
    if (gp.G > 1 && gp.tid == 0) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (gp.tid == 0)
    S.status = __hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
//   summary; null trial: the current U_tk.
DEV float row_side(const FitDev& d, const Trial& tr, int par, int slot, int t, int i) {
  (void)i;
  if (t >= d.m) return 0.0f;
  if (tr.op == OP_ULF)
    return funmap(ld_atomic(&d.tvec[((size_t)par * TMAX + slot) * d.ldmax + t]));
  if (tr.op == OP_URF) {
    Top2 s = d.rowst[(size_t)tr.k * d.ldm + t];
    float x = d.RwT[(size_t)tr.j * d.ldm + t] - tr.val;
    return fminf(excl(s, tr.j), x);
  }
  return d.Uc[(size_t)tr.k * d.ldm + t];
}

// Column-side value of trial tr at working column c (the changed V row).
DEV float col_side(const FitDev& d, const Trial& tr, int par, int slot, int c, int i) {
  if (c >= d.n) return 0.0f;
  if (tr.op == OP_ULF) {
    Top2 s = d.colst[(size_t)tr.k * d.ldn + c];
    float x = d.Rw[(size_t)i * d.ldn + c] - tr.val;
    return fminf(excl(s, i), x);
  }
  if (tr.op == OP_URF)
    return funmap(ld_atomic(&d.tvec[((size_t)par * TMAX + slot) * d.ldmax + c]));
  return d.V[(size_t)tr.k * d.ldn + c];
}

// ------------------------------------------------------------ pass 1 of a batch
// Second residual of every trial over this workgroup's tiles, combined across
// tiles with an atomic min on order-preserving integer images (exact).
DEV void batch_residual_pass(Grp& gp, Smem& S, int i, int par) {
  const FitDev& d = *gp.d;
  const int nt = S.nt;
  bool anyU = false, anyV = false;
  for (int q = 0; q < nt; ++q) {
    anyU |= S.trials[q].op == OP_ULF;
    anyV |= S.trials[q].op == OP_URF;
  }
  const int ntile = d.nrt * d.nct;
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / d.nct, ct = tile % d.nct;
    const int r0 = rt * TS, c0 = ct * TS;
    __syncthreads();
    // incremental first residuals for the tile: ULF needs V'_k. on the tile
    // columns, URF needs U'_.k on the tile rows
    for (int e = gp.tid; e < nt * TS; e += NTHR) {
      int q = e / TS, x = e % TS;
      const Trial& tr = S.trials[q];
      if (tr.op == OP_ULF) S.u.b.sB[q][x] = col_side(d, tr, par, q, c0 + x, i);
      else if (tr.op == OP_URF) S.u.b.sA[q][x] = row_side(d, tr, par, q, r0 + x, i);
    }
    __syncthreads();
    if (anyU) {
      // lanes over rows: U''_tk = min over the tile columns of R_tc - V'_kc
      float Rrow[TS];
#pragma unroll
      for (int c = 0; c < TS; ++c) Rrow[c] = d.RwT[(size_t)(c0 + c) * d.ldm + r0 + gp.lane];
      for (int q = gp.wave; q < nt; q += NWAVE) {
        if (S.trials[q].op != OP_ULF) continue;
        float x = FINF;
#pragma unroll
        for (int c = 0; c < TS; ++c) x = fminf(x, Rrow[c] - S.u.b.sB[q][c]);
        if (x != FINF)
          atomicMin(&d.tvec[((size_t)par * TMAX + q) * d.ldmax + r0 + gp.lane], fmap(x));
      }
    }
    if (anyV) {
      // lanes over columns: V''_kc = min over the tile rows of R_tc - U'_tk
      float Rcol[TS];
#pragma unroll
      for (int t = 0; t < TS; ++t) Rcol[t] = d.Rw[(size_t)(r0 + t) * d.ldn + c0 + gp.lane];
      for (int q = gp.wave; q < nt; q += NWAVE) {
        if (S.trials[q].op != OP_URF) continue;
        float y = FINF;
#pragma unroll
        for (int t = 0; t < TS; ++t) y = fminf(y, Rcol[t] - S.u.b.sA[q][t]);
        if (y != FINF)
          atomicMin(&d.tvec[((size_t)par * TMAX + q) * d.ldmax + c0 + gp.lane], fmap(y));
      }
    }
  }
}

// Max over l != k of U_tl + V_lc for the tile (cooperative: wave w fills rows
// 16w..16w+15), left in S.Ps.  With rank 1 the set is empty (-inf).
DEV void compute_pnotk(Grp& gp, Smem& S, int r0, int c0, int k) {
  const FitDev& d = *gp.d;
  const int c = c0 + gp.lane;
  float P[TS / NWAVE];
#pragma unroll
  for (int tt = 0; tt < TS / NWAVE; ++tt) P[tt] = -FINF;
  const int tb = r0 + gp.wave * (TS / NWAVE);
  for (int l = 0; l < d.r; ++l) {
    if (l == k) continue;
    const float v = d.V[(size_t)l * d.ldn + c];
    const float* u = d.Uc + (size_t)l * d.ldm + tb;
#pragma unroll
    for (int tt = 0; tt < TS / NWAVE; ++tt) P[tt] = fmaxf(P[tt], u[tt] + v);
  }
#pragma unroll
  for (int tt = 0; tt < TS / NWAVE; ++tt) S.Ps[gp.wave * (TS / NWAVE) + tt][gp.lane] = P[tt];
}

// ------------------------------------------------------------ pass 2 of a batch
// b-norm of every trial over this workgroup's tiles.  Per lane and trial the
// sum runs over the tile rows in four interleaved FP64 accumulators, is added
// to a per-lane running sum in tile order, and reduced across lanes at the end.
DEV void batch_eval_pass(Grp& gp, Smem& S, int i, int par) {
  const FitDev& d = *gp.d;
  const int nt = S.nt;
  for (int e = gp.tid; e < nt * TS; e += NTHR) S.u.b.wacc[e / TS][e % TS] = 0.0;
  const int ntile = d.nrt * d.nct;
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / d.nct, ct = tile % d.nct;
    const int r0 = rt * TS, c0 = ct * TS;
    __syncthreads();
    for (int e = gp.tid; e < nt * TS; e += NTHR) {
      int q = e / TS, x = e % TS;
      const Trial& tr = S.trials[q];
      S.u.b.sA[q][x] = row_side(d, tr, par, q, r0 + x, i);
      S.u.b.sB[q][x] = col_side(d, tr, par, q, c0 + x, i);
    }
    float Rev[TS];
#pragma unroll
    for (int t = 0; t < TS; ++t) {
      float rv = d.Rw[(size_t)(r0 + t) * d.ldn + c0 + gp.lane];
      Rev[t] = (rv == FINF) ? FLT_MAX : rv;   // unobserved: R = P = FLT_MAX gives d = 0
    }
    for (int kq = 0; kq < S.nk; ++kq) {
      const int k = S.kdistinct[kq];
      __syncthreads();
      compute_pnotk(gp, S, r0, c0, k);
      __syncthreads();
      float Pc[TS];
#pragma unroll
      for (int t = 0; t < TS; ++t) Pc[t] = (Rev[t] == FLT_MAX) ? FLT_MAX : S.Ps[t][gp.lane];
      for (int q = gp.wave; q < nt; q += NWAVE) {
        if (S.trials[q].k != k) continue;
        const float vs = S.u.b.sB[q][gp.lane];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int t = 0; t < TS; t += 4) {
          float n0 = S.u.b.sA[q][t + 0] + vs, n1 = S.u.b.sA[q][t + 1] + vs;
          float n2 = S.u.b.sA[q][t + 2] + vs, n3 = S.u.b.sA[q][t + 3] + vs;
          float d0 = Rev[t + 0] - fmaxf(Pc[t + 0], n0);
          float d1 = Rev[t + 1] - fmaxf(Pc[t + 1], n1);
          float d2 = Rev[t + 2] - fmaxf(Pc[t + 2], n2);
          float d3 = Rev[t + 3] - fmaxf(Pc[t + 3], n3);
          a0 += fabs((double)d0);
          a1 += fabs((double)d1);
          a2 += fabs((double)d2);
          a3 += fabs((double)d3);
        }
        S.u.b.wacc[q][gp.lane] += (a0 + a1) + (a2 + a3);
      }
    }
  }
  __syncthreads();
  // lane butterfly (fixed pattern), one FP64 partial per trial and workgroup
  for (int q = gp.wave; q < nt; q += NWAVE) {
    double v = S.u.b.wacc[q][gp.lane];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    if (gp.lane == 0) d.epart[(size_t)q * d.gsize + gp.g] = v;
  }
}

// Clear the atomic-min targets used by the previous batch (other parity).
DEV void clear_prev(Grp& gp, Smem& S, int par_prev) {
  const FitDev& d = *gp.d;
  for (int q = 0; q < S.prev_nt; ++q) {
    int op = S.prev_ops[q];
    int len = op == OP_ULF ? d.ldm : (op == OP_URF ? d.ldn : 0);
    unsigned* v = d.tvec + ((size_t)par_prev * TMAX + q) * d.ldmax;
    for (int x = gp.g * NTHR + gp.tid; x < len; x += gp.G * NTHR) v[x] = FMAP_INF;
  }
}

// ------------------------------------------------------------ refresh
// After an accepted update (and at initialisation): argmax counts of every
// row and column, td_col, and the top-2 residual summaries of component k.
DEV bool refresh(Grp& gp, Smem& S, int k, bool full) {
  const FitDev& d = *gp.d;
  const int ntile = d.nrt * d.nct;
  const int rows16 = TS / NWAVE;
  for (int tile = gp.g; tile < ntile; tile += gp.G) {
    const int rt = tile / d.nct, ct = tile % d.nct;
    const int r0 = rt * TS, c0 = ct * TS;
    __syncthreads();
    if (full)
      for (int e = gp.tid; e < TS * RMAX; e += NTHR) {
        (&S.u.f.hc[0][0])[e] = 0;
        (&S.u.f.hr[0][0])[e] = 0;
      }
    __syncthreads();
    const int c = c0 + gp.lane;
    const int tb = r0 + gp.wave * rows16;
    float R[TS / NWAVE];
#pragma unroll
    for (int tt = 0; tt < rows16; ++tt) R[tt] = d.Rw[(size_t)(tb + tt) * d.ldn + c];
    if (full) {
      float P[TS / NWAVE];
      int A[TS / NWAVE];
      {
        const float v = d.V[c];
#pragma unroll
        for (int tt = 0; tt < rows16; ++tt) { P[tt] = d.Uc[tb + tt] + v; A[tt] = 0; }
      }
      for (int l = 1; l < d.r; ++l) {
        const float v = d.V[(size_t)l * d.ldn + c];
        const float* u = d.Uc + (size_t)l * d.ldm + tb;
#pragma unroll
        for (int tt = 0; tt < rows16; ++tt) {
          float x = u[tt] + v;
          if (x > P[tt]) { P[tt] = x; A[tt] = l; }
        }
      }
      double tdl = 0.0;
#pragma unroll
      for (int tt = 0; tt < rows16; ++tt) {
        const int t = tb + tt;
        const bool obs = R[tt] != FINF;
        if (obs) tdl += fabs((double)(R[tt] - P[tt]));
        const bool cnt = d.count_scope ? (t < d.m && c < d.n) : obs;
        if (cnt) {
          atomicAdd(&S.u.f.hc[gp.lane][A[tt]], 1);
          atomicAdd(&S.u.f.hr[gp.wave * rows16 + tt][A[tt]], 1);
        }
      }
      S.u.f.tdw[gp.wave][gp.lane] = tdl;
    }
    {
      Top2 cs = top2_id();
      const float* u = d.Uc + (size_t)k * d.ldm + tb;
#pragma unroll
      for (int tt = 0; tt < rows16; ++tt) cs = top2_add(cs, R[tt] - u[tt], tb + tt);
      S.u.f.csw[gp.wave][gp.lane] = cs;
    }
    {
      // lanes over rows: row summary over this wave's 16 columns
      const int t = r0 + gp.lane;
      const int cb = c0 + gp.wave * rows16;
      const float* vk = d.V + (size_t)k * d.ldn + cb;
      Top2 rs = top2_id();
#pragma unroll
      for (int cc = 0; cc < rows16; ++cc)
        rs = top2_add(rs, d.RwT[(size_t)(cb + cc) * d.ldm + t] - vk[cc], cb + cc);
      S.u.f.rsw[gp.wave][gp.lane] = rs;
    }
    __syncthreads();
    if (gp.wave == 0) {
      Top2 cs = top2_comb(top2_comb(top2_comb(S.u.f.csw[0][gp.lane], S.u.f.csw[1][gp.lane]),
                                    S.u.f.csw[2][gp.lane]), S.u.f.csw[3][gp.lane]);
      d.colpart[(size_t)rt * d.ldn + c] = cs;
      if (full)
        d.tdpart[(size_t)rt * d.ldn + c] =
            ((S.u.f.tdw[0][gp.lane] + S.u.f.tdw[1][gp.lane]) + S.u.f.tdw[2][gp.lane]) + S.u.f.tdw[3][gp.lane];
    } else if (gp.wave == 1) {
      Top2 rs = top2_comb(top2_comb(top2_comb(S.u.f.rsw[0][gp.lane], S.u.f.rsw[1][gp.lane]),
                                    S.u.f.rsw[2][gp.lane]), S.u.f.rsw[3][gp.lane]);
      d.rowpart[(size_t)ct * d.ldm + r0 + gp.lane] = rs;
    }
    if (full) {
      for (int e = gp.tid; e < TS * d.r; e += NTHR) {
        int x = e / d.r, l = e % d.r;
        int hcv = S.u.f.hc[x][l], hrv = S.u.f.hr[x][l];
        if (hcv && c0 + x < d.n) atomicAdd(&d.ccol[(size_t)(c0 + x) * d.r + l], hcv);
        if (hrv && r0 + x < d.m) atomicAdd(&d.crow[(size_t)(r0 + x) * d.r + l], hrv);
      }
    }
  }
  if (!group_sync(gp, S)) return false;
  // combine partials in fixed tile order
  {
    int lo, hi;
    slice(d.n, gp.g, gp.G, lo, hi);
    for (int c = lo + gp.tid; c < hi; c += NTHR) {
      Top2 cs = top2_id();
      double s = 0.0;
      for (int rt = 0; rt < d.nrt; ++rt) {
        cs = top2_comb(cs, d.colpart[(size_t)rt * d.ldn + c]);
        if (full) s += d.tdpart[(size_t)rt * d.ldn + c];
      }
      d.colst[(size_t)k * d.ldn + c] = cs;
      if (full) d.td[c] = s;
    }
    slice(d.m, gp.g, gp.G, lo, hi);
    for (int t = lo + gp.tid; t < hi; t += NTHR) {
      Top2 rs = top2_id();
      for (int ct = 0; ct < d.nct; ++ct) rs = top2_comb(rs, d.rowpart[(size_t)ct * d.ldm + t]);
      d.rowst[(size_t)k * d.ldm + t] = rs;
    }
  }
  if (!full) return group_sync(gp, S);
  if (!group_sync(gp, S)) return false;
  // order of the columns by (td_col descending, index ascending), by ranking
  {
    int lo, hi;
    slice(d.n, gp.g, gp.G, lo, hi);
    for (int c0 = lo; c0 < hi; c0 += NTHR) {
      const int c = c0 + gp.tid;
      const double key = c < hi ? d.td[c] : 0.0;
      int rank = 0;
      for (int x = 0; x < d.n; ++x) {
        const double o = d.td[x];
        rank += (o > key || (o == key && x < c)) ? 1 : 0;
      }
      if (c < hi) d.order[rank] = c;
    }
  }
  return group_sync(gp, S);
}

// ------------------------------------------------------------ row visit pieces
// Candidate list of row i (workgroup 0 of the group): observed columns in
// the current order.
DEV void build_candidates(Grp& gp, Smem& S, int i) {
  const FitDev& d = *gp.d;
  const float* Ri = d.Rw + (size_t)i * d.ldn;
  const int per = (d.n + NTHR - 1) / NTHR;
  const int lo = gp.tid * per;
  int hi = lo + per;
  if (hi > d.n) hi = d.n;
  int cnt = 0;
  for (int q = lo; q < hi; ++q) cnt += Ri[d.order[q]] != FINF;
  S.scan[gp.tid] = cnt;
  __syncthreads();
  if (gp.tid == 0) {
    int acc = 0;
    for (int x = 0; x < NTHR; ++x) { int v = S.scan[x]; S.scan[x] = acc; acc += v; }
    S.scan[NTHR] = acc;
    gp.ctl->ncand = acc;
  }
  __syncthreads();
  int pos = S.scan[gp.tid];
  for (int q = lo; q < hi; ++q) {
    int c = d.order[q];
    if (Ri[c] != FINF) d.cand[pos++] = c;
  }
}

// Next batch of up to T trials from the cursor, in the method's order:
// candidate by candidate, F-ULF then F-URF, skipping no-op trials.  Every
// workgroup of the group computes the same list.
DEV void build_batch(Grp& gp, Smem& S, int i, int T, int ncand) {
  const FitDev& d = *gp.d;
  if (gp.tid == 0) { S.nt = 0; S.batch_noops = 0; }
  __syncthreads();
  while (true) {
    const int qbase = S.cur_q;
    if (S.nt >= T || qbase >= ncand) break;
    if (gp.tid < 64) {
      const int p = gp.tid, q = qbase + p;
      if (q < ncand) {
        const int j = d.cand[q];
        int best = -1, k = 0;
        for (int l = 0; l < d.r; ++l) {
          int v = ld_atomic(&d.crow[(size_t)i * d.r + l]) + ld_atomic(&d.ccol[(size_t)j * d.r + l]);
          if (v > best) { best = v; k = l; }
        }
        const float Rij = d.Rw[(size_t)i * d.ldn + j];
        const float Uik = d.Uc[(size_t)k * d.ldm + i];
        const float Vkj = d.V[(size_t)k * d.ldn + j];
        const float vu = Rij - Vkj, vv = Rij - Uik;
        const bool cl = d.noop_rule && d.closed[k];
        S.cj[p] = j; S.ck[p] = k; S.cvu[p] = vu; S.cvv[p] = vv;
        S.cnu[p] = cl && vu == Uik;
        S.cnv[p] = cl && vv == Vkj;
      }
    }
    __syncthreads();
    if (gp.tid == 0) {
      int p = 0, op = S.cur_op;
      int nt = S.nt, nn = S.batch_noops;
      while (nt < T && qbase + p < ncand && p < 64) {
        const bool noop = op == 0 ? S.cnu[p] : S.cnv[p];
        if (noop) {
          ++nn;
        } else {
          Trial tr;
          tr.j = S.cj[p]; tr.k = S.ck[p]; tr.op = op; tr.val = op == 0 ? S.cvu[p] : S.cvv[p];
          S.trials[nt] = tr;
          S.noops_before[nt] = nn;
          ++nt;
        }
        if (op == 0) op = 1; else { op = 0; ++p; }
      }
      S.nt = nt; S.batch_noops = nn;
      S.cur_q = qbase + p; S.cur_op = op;
    }
    __syncthreads();
  }
  if (gp.tid == 0) {
    S.exhausted = S.cur_q >= ncand;
    int nk = 0;
    for (int q = 0; q < S.nt; ++q) {
      int k = S.trials[q].k, seen = 0;
      for (int x = 0; x < nk; ++x) seen |= S.kdistinct[x] == k;
      if (!seen) S.kdistinct[nk++] = k;
    }
    S.nk = nk;
  }
  __syncthreads();
}

// Apply the accepted trial: U_.k and V_k. take the trial's vectors.  Also
// clears the argmax counts for the refresh that follows.
DEV void apply_trial(Grp& gp, Smem& S, int i, int par, int slot) {
  const FitDev& d = *gp.d;
  const Trial tr = S.trials[slot];
  int lo, hi;
  slice(d.ldm, gp.g, gp.G, lo, hi);
  for (int t = lo + gp.tid; t < hi; t += NTHR) {
    float v = row_side(d, tr, par, slot, t, i);
    d.Uc[(size_t)tr.k * d.ldm + t] = v;
  }
  slice(d.ldn, gp.g, gp.G, lo, hi);
  for (int c = lo + gp.tid; c < hi; c += NTHR) {
    float v = col_side(d, tr, par, slot, c, i);
    d.V[(size_t)tr.k * d.ldn + c] = v;
  }
  slice(d.m * d.r, gp.g, gp.G, lo, hi);
  for (int x = lo + gp.tid; x < hi; x += NTHR) d.crow[x] = 0;
  slice(d.n * d.r, gp.g, gp.G, lo, hi);
  for (int x = lo + gp.tid; x < hi; x += NTHR) d.ccol[x] = 0;
  if (gp.g == 0 && gp.tid == 0) d.closed[tr.k] = 1;
}

DEV void zero_counts(Grp& gp) {
  const FitDev& d = *gp.d;
  int lo, hi;
  slice(d.m * d.r, gp.g, gp.G, lo, hi);
  for (int x = lo + gp.tid; x < hi; x += NTHR) d.crow[x] = 0;
  slice(d.n * d.r, gp.g, gp.G, lo, hi);
  for (int x = lo + gp.tid; x < hi; x += NTHR) d.ccol[x] = 0;
}

// Evaluate the batch in S.trials: residual pass, error pass, and the
// decision (first trial with e' < e) made by the last workgroup to arrive.
DEV bool run_batch(Grp& gp, Smem& S, int i, int par, double e_cur) {
  const FitDev& d = *gp.d;
  batch_residual_pass(gp, S, i, par);
  if (!group_sync(gp, S)) return false;
  batch_eval_pass(gp, S, i, par);
  clear_prev(gp, S, par ^ 1);
  return group_sync_last(gp, S, [&] {
    if (gp.tid < 64) {
      const int q = gp.tid;
      double s = 0.0;
      if (q < S.nt)
        for (int g = 0; g < gp.G; ++g) s += d.epart[(size_t)q * d.gsize + g];
      S.u.b.wacc[0][q] = s;   // reuse as scratch
    }
    __syncthreads();
    if (gp.tid == 0) {
      int dec = -1;
      for (int q = 0; q < S.nt; ++q)
        if (S.u.b.wacc[0][q] < e_cur) { dec = q; break; }
      gp.ctl->decision = dec;
      gp.ctl->e_new = dec >= 0 ? S.u.b.wacc[0][dec] : (S.nt ? S.u.b.wacc[0][0] : 0.0);
    }
  });
}

// Initial state: residual summaries of every component, counts, td_col,
// the order, and the error of the current state through the same pass as
// every trial (a null trial).
DEV bool fit_init(Grp& gp, Smem& S) {
  const FitDev& d = *gp.d;
  // clear both parities of the trial vectors
  {
    size_t total = (size_t)2 * TMAX * d.ldmax;
    for (size_t x = (size_t)gp.g * NTHR + gp.tid; x < total; x += (size_t)gp.G * NTHR)
      d.tvec[x] = FMAP_INF;
  }
  zero_counts(gp);
  if (!group_sync(gp, S)) return false;
  for (int k = 0; k < d.r; ++k)
    if (!refresh(gp, S, k, k == d.r - 1)) return false;
  if (gp.tid == 0) {
    Trial tr; tr.j = 0; tr.k = 0; tr.op = OP_NULL; tr.val = 0.0f;
    S.trials[0] = tr; S.nt = 1; S.nk = 1; S.kdistinct[0] = 0; S.prev_nt = 0;
  }
  __syncthreads();
  batch_eval_pass(gp, S, 0, 0);
  if (!group_sync_last(gp, S, [&] {
        if (gp.tid == 0) {
          double s = 0.0;
          for (int g = 0; g < gp.G; ++g) s += d.epart[g];
          gp.ctl->e = s;
          d.traj[0] = s;
          gp.ctl->phase = d.iters > 0 ? 1 : 2;
          gp.ctl->it = 1;
          gp.ctl->row = 0;
          gp.ctl->acc_in_pass = 0;
          gp.ctl->cells = 0;
        }
      }))
    return false;
  return true;
}

// Run the fit from its saved state for at most max_rows row visits (0: no
// limit).  All workgroups of the group execute the same control flow.
DEV void fit_run(Grp& gp, Smem& S, int max_rows) {
  const FitDev& d = *gp.d;
  FitCtl* ctl = gp.ctl;
  if (gp.tid == 0) { S.prev_nt = 0; S.status = 0; }
  __syncthreads();
  if (ld_atomic(&ctl->phase) == 0) {
    if (!fit_init(gp, S)) return;
  } else {
    // a resumed launch: the trial vectors of both parities must start clean
    size_t total = (size_t)2 * TMAX * d.ldmax;
    for (size_t x = (size_t)gp.g * NTHR + gp.tid; x < total; x += (size_t)gp.G * NTHR)
      d.tvec[x] = FMAP_INF;
    if (!group_sync(gp, S)) return;
  }
  double e_cur = ld_atomic(&ctl->e);
  int it = ld_atomic(&ctl->it), row = ld_atomic(&ctl->row);
  int acc_pass = ld_atomic(&ctl->acc_in_pass);
  int phase = ld_atomic(&ctl->phase);
  int rows_done = 0;
  int par = 0;
  while (phase == 1) {
    if (max_rows > 0 && rows_done >= max_rows) break;
    const int i = row;
    if (gp.g == 0) build_candidates(gp, S, i);
    if (!group_sync(gp, S)) return;
    const int ncand = ld_atomic(&ctl->ncand);
    if (gp.tid == 0) { S.cur_q = 0; S.cur_op = 0; }
    __syncthreads();
    int T = d.t0;
    long long row_trials = 0, row_noops = 0, row_spec = 0;
    int acc_j = -1, acc_k = -1, acc_op = -1;
    while (true) {
      build_batch(gp, S, i, T, ncand);
      const int nt = S.nt;
      if (nt == 0) { row_noops += S.batch_noops; break; }
      if (!run_batch(gp, S, i, par, e_cur)) return;
      const int dec = ld_atomic(&ctl->decision);
      row_spec += nt;
      if (gp.tid == 0) {
        S.prev_nt = nt;
        for (int q = 0; q < nt; ++q) S.prev_ops[q] = S.trials[q].op;
      }
      if (dec >= 0) {
        row_trials += dec + 1;
        row_noops += S.noops_before[dec];
        const Trial tr = S.trials[dec];
        acc_j = tr.j; acc_k = tr.k; acc_op = tr.op;
        e_cur = ld_atomic(&ctl->e_new);
        apply_trial(gp, S, i, par, dec);
        if (!group_sync(gp, S)) return;
        if (!refresh(gp, S, tr.k, true)) return;
        par ^= 1;
        break;
      }
      row_trials += nt;
      row_noops += S.batch_noops;
      par ^= 1;
      if (S.exhausted) break;
      T = T * 2 > d.tmax ? d.tmax : T * 2;
    }
    if (acc_j >= 0) ++acc_pass;
    // bookkeeping by one thread of the group
    if (gp.g == 0 && gp.tid == 0) {
      ctl->trials += row_trials;
      ctl->spec_trials += row_spec;
      ctl->noops += row_noops;
      ctl->row_visits += 1;
      ctl->cells += row_trials * (long long)d.omega;
      if (acc_j >= 0) { ctl->accepted += 1; ctl->e = e_cur; }
      if (d.log && ctl->nlog < d.log_cap) {
        LogRec rec;
        rec.iter = it; rec.row = i; rec.trials = (int)row_trials; rec.noops = (int)row_noops;
        rec.j = acc_j; rec.k = acc_k; rec.op = acc_op; rec.pad = 0; rec.e = e_cur;
        d.log[ctl->nlog] = rec;
      }
      ctl->nlog += 1;
    }
    ++row;
    ++rows_done;
    if (row == d.m) {
      if (gp.g == 0 && gp.tid == 0) d.traj[it] = e_cur;
      const bool fixed = acc_pass == 0;
      const bool small = d.eps > 0.0 && (d.traj[it - 1] - e_cur) < d.eps;
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
    }
  }
  group_sync(gp, S);
}

// One fit per group of gsize workgroups.  With nfits > 1 every group takes
// fits from a queue (ctl of fit 0 holds the counter).
__global__ void __launch_bounds__(NTHR) fit_kernel(const FitDev* __restrict__ fits, int nfits,
                                                   int gsize, int max_rows,
                                                   unsigned* __restrict__ queue) {
  extern __shared__ char smem_raw[];
  Smem& S = *reinterpret_cast<Smem*>(smem_raw);
  Grp gp;
  gp.tid = threadIdx.x;
  gp.lane = threadIdx.x & 63;
  gp.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  gp.g = blockIdx.x % gsize;
  gp.G = gsize;
  if (nfits == 1 && gsize == (int)gridDim.x) {
    gp.d = &fits[0];
    gp.ctl = fits[0].ctl;
    if (ld_atomic(&gp.ctl->phase) != 2) fit_run(gp, S, max_rows);
    return;
  }
  // queue of fits, one workgroup per fit
  __shared__ int fid_s;
  while (true) {
    if (gp.tid == 0) fid_s = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int fid = fid_s;
    __syncthreads();
    if (fid >= nfits) break;
    gp.d = &fits[fid];
    gp.ctl = fits[fid].ctl;
    gp.g = 0;
    gp.G = 1;
    if (ld_atomic(&gp.ctl->phase) != 2) fit_run(gp, S, max_rows);
  }
}

size_t fit_smem_bytes() { return sizeof(Smem); }

}  // namespace stmf
