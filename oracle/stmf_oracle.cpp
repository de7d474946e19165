// CPU oracle for sparse tropical matrix factorization (FastSTMF).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or helper with the HIP library; it is a plain, slow,
// deliberately unblocked restatement of the paper's definitions:
//
//   * max-plus product          (A (x) B)_ij = max_k A_ik + B_kj      Sec. 2
//   * masked min-plus residual  (A (x)* B)_ij = min over given A_ik, B_kj
//                                of A_ik + B_kj                        Sec. 2
//   * b-norm                    ||W||_b = sum |W_ij|, over given cells Sec. 3.6
//   * argmax f(i,j), lowest index on ties                     Sec. 3.2.1 (TD)
//   * td_col(j) = sum over rows of td(t, j)                   Sec. 3.2.1
//   * TD_A k-selection from the additive union of the two
//     argmax multisets                                        Sec. 3.2.1
//   * F-ULF / F-URF                                           Algorithms 1, 2
//   * FastSTMF = ByRow, random row permutation, TD_A, wide    Algorithm 3
//   * the other ByRow selections TD, TD_B and SEQ, and the row orders PermR
//     (rows by increasing minimum) and none                   Sec. 3.2.1, 3.3
//   * ByElement with PermC (columns by increasing minimum), TD
//     selection of k                          Sec. 3.2.2, 3.3, supplementary
//                                             ByElement pseudocode
//   * ByMatrix without permutation, TD selection of k, a random operation
//                                             Sec. 3.2.3, supplementary
//                                             ByMatrix pseudocode
//
// Every routine is a template over the value type T.  T = double is "the FP64
// oracle": all value arithmetic in double on exactly promoted FP32 inputs.
// T = float takes every value operation as one correctly rounded FP32
// operation (the precision in which the GPU library decides accept/reject,
// argmax and ordering), with error sums widened to double.  The b-norm is
// summed row by row: each row's |d| in column order, then the row sums in row
// order; td_col(j) adds its rows in row order.  The row loops of the
// residuals and of the evaluation may run on several threads (OpenMP): every
// sum keeps that order, so the results do not depend on the thread count.
// Built with -ffp-contract=off and no fast-math.
//
// Readings of points the paper leaves open (each is listed in the design
// notes of the repository):
//   - error, td and td_col range over observed cells only;
//   - transpose iff rows > columns ("wide" means m <= n);
//   - TD_A counts range over observed cells of row i and column j, the union
//     is additive, ties go to the lowest index;
//   - candidates j are the observed columns of row i ordered by td_col
//     descending, ties by ascending j; F-URF is tried with the same (j, k)
//     after F-ULF is rejected, and the first strict decrease (e' < e) ends the
//     row;
//   - initial V is the residual (-U)^T (x)* R for every component;
//   - no-op rule: an operation whose step-2 write leaves the stored value
//     unchanged, on a component last written by a completed operation, is
//     counted as rejected without evaluation (exact arithmetic gives e' = e);
//   - a pass with no accepted update is a fixed point: the rest of the
//     trajectory is padded with the current error;
//   - random draws: SplitMix64 (Steele, Lea, Flood 2014), bounded integers by
//     rejection of x < 2^64 mod b then x mod b, Durstenfeld's Fisher-Yates
//     from the last index down; draw order: permutation, then U0 (with PermR
//     or no permutation the stream starts with U0);
//   - TD: candidates by td(i, j) = |R_ij - (U (x) V)_ij| descending, ties by
//     ascending j, k = f(i, j);
//   - TD_B: candidates as TD_A; j0 = the column of largest td_col (lowest on
//     ties); ByRow's err(t, j) = td_col(j) does not depend on the row t, so
//     every row ties for i0 and the lowest working row is taken;
//     k = f(i, j0) if (U (x) V)_{i j0} >= (U (x) V)_{i0 j}, else f(i0, j);
//   - SEQ: every (j, k, operation) of row i is evaluated, j and k ascending,
//     F-ULF before F-URF; the one with the smallest error below the current
//     one is applied (ties: the first in that order);
//   - PermR: working rows by increasing minimum observed value, ties by the
//     lower original index.
//   - ByElement: the working rows in order (PermC permutes only columns),
//     in each row its observed columns in working column order; k = f(i, j);
//     an entry with R_ij = (U (x) V)_ij (td = 0) is not updated; F-ULF, and
//     F-URF after a rejected F-ULF; an accepted update does not end the row
//     visit, the next element follows; a pass with no accepted update is a
//     fixed point.  Log: one record per accepted update (trials and no-op
//     skips since the previous record of the visit) and one closing record
//     per row visit (j = -1);
//   - PermC: working columns by increasing minimum observed value, ties by
//     the lower working index; V's columns are put back at the output.
//   - ByMatrix: one iteration keys every observed cell by
//     err = (td_row(i) + td_col(j)) - td(i, j) (FP64, td_row summed over j
//     ascending, td_col over i ascending) in the iteration's state and tries
//     the cells by err descending, ties in row-major order, with k = f(i, j)
//     from that state; the operation of the c-th cell tried in the fit
//     (no-op skips included) is F-URF if the top bit of the c-th output of
//     SplitMix64 seeded with seed ^ 0xA0761D6478BD642F is set, else F-ULF
//     (a uniform draw below 1/2 selects F-ULF); the first strict decrease
//     ends the iteration; an iteration without one is a fixed point.  Log:
//     one record per iteration (row = the accepted row, else -1).
//
// Parity of the TD_A counting scope, the candidate tie order, the Random-Acol
// column count and the random stream is unpinned: the paper fixes none of
// them.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

enum { OK = 0, EINVAL_ = 1, EEMPTY = 2, ERANGE_ = 3 };

// ---------------------------------------------------------------- randomness
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

uint64_t draw_below(SplitMix64& g, uint64_t bound) {
  uint64_t reject_under = (0ull - bound) % bound;  // 2^64 mod bound
  while (true) {
    uint64_t x = g.next();
    if (x >= reject_under) return x % bound;
  }
}

// Loops over fewer cells than this stay on the calling thread.
constexpr int64_t PAR_CELLS = 16384;

// ---------------------------------------------------------------- primitives
// (U (x) V)_ij = max_l U_il + V_lj; A gets the lowest l reaching the maximum.
template <class T>
void maxplus(const T* U, const T* V, int m, int r, int n, T* P, int32_t* A) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      T best = U[(size_t)i * r + 0] + V[j];
      int arg = 0;
      for (int l = 1; l < r; ++l) {
        T x = U[(size_t)i * r + l] + V[(size_t)l * n + j];
        if (x > best) { best = x; arg = l; }
      }
      if (P) P[(size_t)i * n + j] = best;
      if (A) A[(size_t)i * n + j] = arg;
    }
}

// Column residual of component k: V_kj <- min over observed t of R_tj - U_tk.
// This is (-U_.k)^T (x)* R restricted to the given cells of column j.
template <class T>
void col_res(const T* R, const uint8_t* M, int m, int n, int r, int k,
             const T* U, T* V) {
#pragma omp parallel for schedule(static) if ((int64_t)m * n >= PAR_CELLS)
  for (int j = 0; j < n; ++j) {
    bool seen = false;
    T best = 0;
    for (int t = 0; t < m; ++t) {
      if (!M[(size_t)t * n + j]) continue;
      T x = R[(size_t)t * n + j] - U[(size_t)t * r + k];
      if (!seen || x < best) { best = x; seen = true; }
    }
    V[(size_t)k * n + j] = best;
  }
}

// Row residual of component k: U_tk <- min over observed j of R_tj - V_kj.
// This is R (x)* (-V_k.)^T restricted to the given cells of row t.
template <class T>
void row_res(const T* R, const uint8_t* M, int m, int n, int r, int k,
             const T* V, T* U) {
#pragma omp parallel for schedule(static) if ((int64_t)m * n >= PAR_CELLS)
  for (int t = 0; t < m; ++t) {
    bool seen = false;
    T best = 0;
    for (int j = 0; j < n; ++j) {
      if (!M[(size_t)t * n + j]) continue;
      T x = R[(size_t)t * n + j] - V[(size_t)k * n + j];
      if (!seen || x < best) { best = x; seen = true; }
    }
    U[(size_t)t * r + k] = best;
  }
}

// b-norm of R - U (x) V over the observed cells (Sec. 3.6), in double: each
// row's |d| summed in column order, then the row sums in row order.  The
// per-cell difference is taken in T and then widened.  td_col[j] (nullable)
// gets the sum over the observed rows of column j, in row order; A (nullable)
// the argmax of every cell (observed or not).
template <class T>
double masked_error(const T* R, const uint8_t* M, const T* U, const T* V,
                    int m, int n, int r, double* td_col, int32_t* A) {
  // |d| of every cell (0 where unobserved) and the row sums
  static thread_local std::vector<double> ad, rows;
  if (td_col && ad.size() < (size_t)m * n) ad.resize((size_t)m * n);
  if (rows.size() < (size_t)m) rows.resize((size_t)m);
  const bool par = (int64_t)m * n >= PAR_CELLS;
  double* adp = td_col ? ad.data() : nullptr;
  double* rowp = rows.data();
#pragma omp parallel for schedule(static) if (par)
  for (int t = 0; t < m; ++t) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) {
      T best = U[(size_t)t * r + 0] + V[j];
      int arg = 0;
      for (int l = 1; l < r; ++l) {
        T x = U[(size_t)t * r + l] + V[(size_t)l * n + j];
        if (x > best) { best = x; arg = l; }
      }
      if (A) A[(size_t)t * n + j] = arg;
      double a = 0.0;
      if (M[(size_t)t * n + j]) {
        T d = R[(size_t)t * n + j] - best;
        a = std::fabs((double)d);
      }
      if (adp) adp[(size_t)t * n + j] = a;
      rs += a;
    }
    rowp[t] = rs;
  }
  double e = 0.0;
  for (int t = 0; t < m; ++t) e += rowp[t];
  if (td_col) {
#pragma omp parallel for schedule(static) if (par)
    for (int j = 0; j < n; ++j) {
      double c = 0.0;
      for (int t = 0; t < m; ++t) c += adp[(size_t)t * n + j];
      td_col[j] = c;
    }
  }
  return e;
}

// Algorithm 1 (F-ULF) at (i, j, k): back up U_.k and V_k., write
// U_ik <- R_ij - V_kj, then V_k. <- column residual of U_.k, then
// U_.k <- row residual of V_k., and return the new b-norm.
template <class T>
double f_ulf(const T* R, const uint8_t* M, T* U, T* V, int m, int n, int r,
             int i, int j, int k, T* Ubak, T* Vbak, double* td_col, int32_t* A) {
  for (int t = 0; t < m; ++t) Ubak[t] = U[(size_t)t * r + k];
  for (int c = 0; c < n; ++c) Vbak[c] = V[(size_t)k * n + c];
  U[(size_t)i * r + k] = R[(size_t)i * n + j] - V[(size_t)k * n + j];
  col_res(R, M, m, n, r, k, U, V);
  row_res(R, M, m, n, r, k, V, U);
  return masked_error(R, M, U, V, m, n, r, td_col, A);
}

// Algorithm 2 (F-URF) at (i, j, k): the same with V_kj <- R_ij - U_ik and the
// two residual steps in the other order.
template <class T>
double f_urf(const T* R, const uint8_t* M, T* U, T* V, int m, int n, int r,
             int i, int j, int k, T* Ubak, T* Vbak, double* td_col, int32_t* A) {
  for (int t = 0; t < m; ++t) Ubak[t] = U[(size_t)t * r + k];
  for (int c = 0; c < n; ++c) Vbak[c] = V[(size_t)k * n + c];
  V[(size_t)k * n + j] = R[(size_t)i * n + j] - U[(size_t)i * r + k];
  row_res(R, M, m, n, r, k, V, U);
  col_res(R, M, m, n, r, k, U, V);
  return masked_error(R, M, U, V, m, n, r, td_col, A);
}

}  // namespace

// ============================================================ C interface
extern "C" {

struct oracle_opts {
  int init_mode;         // 0 random ints, 1 random Acol, 2 given U0
  float init_lo, init_hi;// random-int range, inclusive
  int acol_p;            // columns averaged per U column (random Acol)
  const float* U0;       // given U0, working orientation (m' x r)
  const int32_t* perm;   // nullable explicit working-row permutation
  double eps;            // 0: run exactly `iters` passes (bar fixed points)
  int count_scope;       // 0 observed cells, 1 every index
  int noop_rule;         // 1: skip no-op trials as rejected
  int integer_exact;     // 1: reject |value| >= 2^24
  int selection;         // 0 TD_A, 1 TD, 2 TD_B, 3 SEQ
  int perm_mode;         // 0 random, 1 PermR (increasing minimum), 2 none,
                         // 3 PermC (columns by increasing minimum, rows as given)
  int strategy;          // 0 ByRow, 1 ByElement, 2 ByMatrix
};

struct oracle_log {      // ByRow: one record per row visit; ByElement: one per
                         // accepted update and one closing each row visit;
                         // ByMatrix: one per iteration (row = accepted row)
  int32_t iter, row, trials, noops, j, k, op;  // j = -1: nothing accepted
  int32_t pad;
  double e;
};

struct oracle_stats {
  int64_t trials;        // evaluated trials
  int64_t noops;         // trials skipped by the no-op rule
  int64_t accepted;
  int64_t row_visits;
  int32_t iters_done;
  int32_t transposed;
  int64_t evaluated_cells;  // sum over evaluations of |Omega|
};

// ---- primitive entry points (f64: T = double, f32: T = float) ----
#define ORACLE_PRIMS(SUF, T)                                                   \
  void oracle_maxplus_##SUF(const T* U, const T* V, int m, int r, int n, T* P, \
                            int32_t* A) {                                      \
    maxplus<T>(U, V, m, r, n, P, A);                                           \
  }                                                                            \
  double oracle_masked_error_##SUF(const T* R, const uint8_t* M, const T* U,   \
                                   const T* V, int m, int n, int r,            \
                                   double* td_col, int32_t* A) {               \
    return masked_error<T>(R, M, U, V, m, n, r, td_col, A);                    \
  }                                                                            \
  void oracle_col_res_##SUF(const T* R, const uint8_t* M, int m, int n, int r, \
                            int k, const T* U, T* V) {                         \
    col_res<T>(R, M, m, n, r, k, U, V);                                        \
  }                                                                            \
  void oracle_row_res_##SUF(const T* R, const uint8_t* M, int m, int n, int r, \
                            int k, const T* V, T* U) {                         \
    row_res<T>(R, M, m, n, r, k, V, U);                                        \
  }                                                                            \
  double oracle_update_U_##SUF(const T* R, const uint8_t* M, T* U, T* V,       \
                               int m, int n, int r, int i, int j, int k,       \
                               T* Ubak, T* Vbak, double* td_col) {             \
    return f_ulf<T>(R, M, U, V, m, n, r, i, j, k, Ubak, Vbak, td_col, nullptr);\
  }                                                                            \
  double oracle_update_V_##SUF(const T* R, const uint8_t* M, T* U, T* V,       \
                               int m, int n, int r, int i, int j, int k,       \
                               T* Ubak, T* Vbak, double* td_col) {             \
    return f_urf<T>(R, M, U, V, m, n, r, i, j, k, Ubak, Vbak, td_col, nullptr);\
  }

ORACLE_PRIMS(f64, double)
ORACLE_PRIMS(f32, float)

// First `count` outputs of SplitMix64 seeded with `seed`.
void oracle_splitmix64(uint64_t seed, int count, uint64_t* out) {
  SplitMix64 g{seed};
  for (int c = 0; c < count; ++c) out[c] = g.next();
}

}  // extern "C"

namespace {

// Working orientation: transpose iff m > n, then rows permuted by perm.
struct Working {
  int m, n;            // working shape
  bool transposed;
  std::vector<float> R;
  std::vector<uint8_t> M;
  std::vector<int32_t> perm;
  std::vector<int32_t> cperm;  // working column b is column cperm[b]
};

int build_working(const float* R, const uint8_t* M, int m, int n,
                  const oracle_opts* o, uint64_t seed, Working& w,
                  SplitMix64& g) {
  w.transposed = m > n;
  w.m = w.transposed ? n : m;
  w.n = w.transposed ? m : n;
  w.perm.resize(w.m);
  if (o && (o->perm_mode < 0 || o->perm_mode > 3)) return EINVAL_;
  // minimum observed value of working line a (a row, or with cols a column)
  auto line_min = [&](int a, bool cols) {
    float mn = 0.0f;
    bool seen = false;
    const int len = cols ? w.m : w.n;
    for (int b = 0; b < len; ++b) {
      const int wr = cols ? b : a, wc = cols ? a : b;
      size_t s = w.transposed ? ((size_t)wc * n + wr) : ((size_t)wr * n + wc);
      if (!M[s]) continue;
      float v = R[s] + 0.0f;
      if (!seen || v < mn) { mn = v; seen = true; }
    }
    return mn;
  };
  w.cperm.resize(w.n);
  for (int b = 0; b < w.n; ++b) w.cperm[b] = b;
  if (o && o->perm_mode == 3) {
    // PermC: working columns by increasing minimum observed value, stable
    std::vector<float> mn(w.n);
    for (int b = 0; b < w.n; ++b) mn[b] = line_min(b, true);
    std::stable_sort(w.cperm.begin(), w.cperm.end(), [&](int x, int y) { return mn[x] < mn[y]; });
  }
  if (o && o->perm) {
    std::vector<char> hit(w.m, 0);
    for (int a = 0; a < w.m; ++a) {
      int p = o->perm[a];
      if (p < 0 || p >= w.m || hit[p]) return EINVAL_;
      hit[p] = 1;
      w.perm[a] = p;
    }
  } else if (o && o->perm_mode == 1) {
    // PermR: working rows by increasing minimum observed value, stable
    std::vector<float> mn(w.m, 0.0f);
    for (int a = 0; a < w.m; ++a) mn[a] = line_min(a, false);
    for (int a = 0; a < w.m; ++a) w.perm[a] = a;
    std::stable_sort(w.perm.begin(), w.perm.end(), [&](int x, int y) { return mn[x] < mn[y]; });
  } else if (o && (o->perm_mode == 2 || o->perm_mode == 3)) {
    for (int a = 0; a < w.m; ++a) w.perm[a] = a;
  } else {
    for (int a = 0; a < w.m; ++a) w.perm[a] = a;
    for (int a = w.m - 1; a >= 1; --a) {
      int b = (int)draw_below(g, (uint64_t)a + 1);
      std::swap(w.perm[a], w.perm[b]);
    }
  }
  (void)seed;
  w.R.assign((size_t)w.m * w.n, 0.0f);
  w.M.assign((size_t)w.m * w.n, 0);
  for (int a = 0; a < w.m; ++a)
    for (int b = 0; b < w.n; ++b) {
      int src = w.perm[a], csrc = w.cperm[b];
      size_t s = w.transposed ? ((size_t)csrc * n + src) : ((size_t)src * n + csrc);
      uint8_t obs = M[s] ? 1 : 0;
      w.M[(size_t)a * w.n + b] = obs;
      // -0 becomes +0; unobserved values are never read into arithmetic.
      w.R[(size_t)a * w.n + b] = obs ? (R[s] + 0.0f) : 0.0f;
    }
  return OK;
}

int init_U0(const Working& w, int r, const oracle_opts* o, SplitMix64& g,
            std::vector<float>& U0) {
  U0.assign((size_t)w.m * r, 0.0f);
  int mode = o ? o->init_mode : 0;
  if (mode == 2) {
    if (!o->U0) return EINVAL_;
    for (size_t q = 0; q < U0.size(); ++q) U0[q] = o->U0[q] + 0.0f;
  } else if (mode == 0) {
    float lo = o ? o->init_lo : 0.0f, hi = o ? o->init_hi : 100.0f;
    int64_t span = (int64_t)hi - (int64_t)lo + 1;
    if (span < 1) return EINVAL_;
    for (int t = 0; t < w.m; ++t)
      for (int l = 0; l < r; ++l)
        U0[(size_t)t * r + l] =
            (float)((int64_t)lo + (int64_t)draw_below(g, (uint64_t)span));
  } else if (mode == 1) {
    int p = (o && o->acol_p > 0) ? o->acol_p : 5;
    std::vector<int> cols((size_t)r * p);
    for (int l = 0; l < r; ++l)
      for (int q = 0; q < p; ++q)
        cols[(size_t)l * p + q] = (int)draw_below(g, (uint64_t)w.n);
    for (int t = 0; t < w.m; ++t) {
      // fallback: mean of the row's observed values
      double rs = 0.0;
      int rc = 0;
      for (int b = 0; b < w.n; ++b)
        if (w.M[(size_t)t * w.n + b]) { rs += (double)w.R[(size_t)t * w.n + b]; ++rc; }
      for (int l = 0; l < r; ++l) {
        double s = 0.0;
        int c = 0;
        for (int q = 0; q < p; ++q) {
          int b = cols[(size_t)l * p + q];
          if (w.M[(size_t)t * w.n + b]) { s += (double)w.R[(size_t)t * w.n + b]; ++c; }
        }
        double mean = c ? s / (double)c : rs / (double)rc;
        U0[(size_t)t * r + l] = (float)mean + 0.0f;
      }
    }
  } else {
    return EINVAL_;
  }
  return OK;
}

template <class T>
int fit(const float* Rin, const uint8_t* Min, int m_in, int n_in, int r,
        int iters, uint64_t seed, const oracle_opts* o, float* U_out,
        float* V_out, double* traj, oracle_log* log, int log_cap, int* log_len,
        oracle_stats* st, int row_limit) {
  if (m_in < 1 || n_in < 1 || r < 1 || r > 64 || iters < 0) return EINVAL_;
  for (int i = 0; i < m_in; ++i) {
    int c = 0;
    for (int j = 0; j < n_in; ++j) c += Min[(size_t)i * n_in + j] ? 1 : 0;
    if (!c) return EEMPTY;
  }
  for (int j = 0; j < n_in; ++j) {
    int c = 0;
    for (int i = 0; i < m_in; ++i) c += Min[(size_t)i * n_in + j] ? 1 : 0;
    if (!c) return EEMPTY;
  }
  const bool int_exact = o && o->integer_exact;
  if (int_exact)
    for (size_t q = 0; q < (size_t)m_in * n_in; ++q)
      if (Min[q] && !(std::fabs(Rin[q]) < 16777216.0f)) return ERANGE_;

  SplitMix64 g{seed};
  Working w;
  int s = build_working(Rin, Min, m_in, n_in, o, seed, w, g);
  if (s) return s;
  std::vector<float> U0;
  s = init_U0(w, r, o, g, U0);
  if (s) return s;
  if (int_exact)
    for (float x : U0)
      if (!(std::fabs(x) < 16777216.0f)) return ERANGE_;

  const int m = w.m, n = w.n;
  std::vector<T> R((size_t)m * n), U((size_t)m * r), V((size_t)r * n);
  for (size_t q = 0; q < R.size(); ++q) R[q] = (T)w.R[q];
  for (size_t q = 0; q < U.size(); ++q) U[q] = (T)U0[q];
  const uint8_t* M = w.M.data();
  for (int k = 0; k < r; ++k) col_res(R.data(), M, m, n, r, k, U.data(), V.data());

  std::vector<double> td((size_t)n);
  std::vector<int32_t> A((size_t)m * n);
  std::vector<T> Ubak((size_t)m), Vbak((size_t)n);
  std::vector<char> closed((size_t)r, 0);
  int64_t omega = 0;
  for (size_t q = 0; q < (size_t)m * n; ++q) omega += M[q];

  double e = masked_error(R.data(), M, U.data(), V.data(), m, n, r, td.data(), A.data());
  if (traj) traj[0] = e;
  oracle_stats S{};
  S.transposed = w.transposed;
  S.evaluated_cells = omega;
  int nlog = 0;
  const int scope_all = o && o->count_scope == 1;
  const int noop_rule = o ? o->noop_rule : 1;
  const double eps = o ? o->eps : 0.0;
  const int sel = o ? o->selection : 0;
  if (sel < 0 || sel > 3) return EINVAL_;
  const int strategy = o ? o->strategy : 0;
  if (strategy < 0 || strategy > 2) return EINVAL_;

  int it_done = 0;
  bool stop = false;
  int rows_left = row_limit > 0 ? row_limit : -1;
  if (strategy == 2) {
    // ByMatrix: one iteration = every observed cell keyed by
    // err = td_row(i) + td_col(j) - td(i, j) from the iteration's state,
    // tried in decreasing order (ties: row-major order) with k = f(i, j) and
    // one operation drawn per cell (F-ULF when the draw is below 1/2) until
    // the first strict decrease; at most one accepted update per iteration.
    SplitMix64 gop{seed ^ 0xA0761D6478BD642Full};
    std::vector<double> tdr((size_t)m), tdc((size_t)n), tij((size_t)m * n), key((size_t)m * n);
    std::vector<int32_t> fk((size_t)m * n);
    std::vector<int64_t> order;
    double e_prev_it = e;
    for (int it = 1; it <= iters && !stop; ++it) {
      if (rows_left == 0) break;
      if (rows_left > 0) --rows_left;
      std::fill(tdr.begin(), tdr.end(), 0.0);
      std::fill(tdc.begin(), tdc.end(), 0.0);
      order.clear();
      for (int t = 0; t < m; ++t)
        for (int j = 0; j < n; ++j) {
          const size_t q = (size_t)t * n + j;
          T best = U[(size_t)t * r] + V[j];
          int arg = 0;
          for (int l = 1; l < r; ++l) {
            T x = U[(size_t)t * r + l] + V[(size_t)l * n + j];
            if (x > best) { best = x; arg = l; }
          }
          fk[q] = arg;
          if (!M[q]) continue;
          const T d = R[q] - best;
          tij[q] = std::fabs((double)d);
          tdr[t] += tij[q];
          tdc[j] += tij[q];
          order.push_back((int64_t)q);
        }
      for (int64_t q : order) key[q] = (tdr[q / n] + tdc[q % n]) - tij[q];
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t a, int64_t b) { return key[a] > key[b]; });
      oracle_log rec{it, -1, 0, 0, -1, -1, -1, 0, e};
      bool accepted = false;
      for (int64_t q : order) {
        const int i = (int)(q / n), j = (int)(q % n), k = fk[q];
        const int op = (gop.next() >> 63) ? 1 : 0;
        T* Uik = &U[(size_t)i * r + k];
        T* Vkj = &V[(size_t)k * n + j];
        const T Rij = R[q];
        if (noop_rule && closed[k]) {
          const bool same = op == 0 ? (T)(Rij - *Vkj) == *Uik : (T)(Rij - *Uik) == *Vkj;
          if (same) { rec.noops++; S.noops++; continue; }
        }
        const double e2 = op == 0
            ? f_ulf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k,
                    Ubak.data(), Vbak.data(), nullptr, nullptr)
            : f_urf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k,
                    Ubak.data(), Vbak.data(), nullptr, nullptr);
        rec.trials++;
        S.trials++;
        S.evaluated_cells += omega;
        if (e2 < e) {
          e = e2;
          masked_error(R.data(), M, U.data(), V.data(), m, n, r, td.data(), A.data());
          closed[k] = 1;
          accepted = true;
          rec.row = i; rec.j = j; rec.k = k; rec.op = op; rec.e = e;
          S.accepted++;
          break;
        }
        for (int t = 0; t < m; ++t) U[(size_t)t * r + k] = Ubak[t];
        for (int c = 0; c < n; ++c) V[(size_t)k * n + c] = Vbak[c];
      }
      if (log && nlog < log_cap) log[nlog] = rec;
      nlog++;
      it_done = it;
      if (traj) traj[it] = e;
      // a fixed point, or (Sec. 3.3) a decrease below eps, ends the fit
      const bool small_step = eps > 0.0 && (e_prev_it - e < eps);
      e_prev_it = e;
      if (!accepted || small_step) {
        if (traj)
          for (int qq = it + 1; qq <= iters; ++qq) traj[qq] = e;
        stop = true;
      }
    }
  } else {
    double e_prev_pass = e;  // error at the end of the previous pass
    for (int it = 1; it <= iters && !stop; ++it) {
      int64_t acc_this_pass = 0;
      for (int i = 0; i < m; ++i) {
        if (rows_left == 0) { stop = true; break; }
        if (rows_left > 0) --rows_left;
        oracle_log rec{it, i, 0, 0, -1, -1, -1, 0, e};
        bool accepted = false;
        // One trial on the current state (U, V changed; restore() undoes it).
        // Returns false for a no-op skip, counted as a rejection.
        auto try_op = [&](int j, int k, int op, double& e2) -> bool {
          T* Uik = &U[(size_t)i * r + k];
          T* Vkj = &V[(size_t)k * n + j];
          T Rij = R[(size_t)i * n + j];
          if (noop_rule && closed[k]) {
            bool same = op == 0 ? (T)(Rij - *Vkj) == *Uik : (T)(Rij - *Uik) == *Vkj;
            if (same) { rec.noops++; S.noops++; return false; }
          }
          e2 = op == 0
              ? f_ulf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k,
                      Ubak.data(), Vbak.data(), nullptr, nullptr)
              : f_urf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k,
                      Ubak.data(), Vbak.data(), nullptr, nullptr);
          rec.trials++;
          S.trials++;
          S.evaluated_cells += omega;
          return true;
        };
        auto restore = [&](int k) {
          for (int t = 0; t < m; ++t) U[(size_t)t * r + k] = Ubak[t];
          for (int c = 0; c < n; ++c) V[(size_t)k * n + c] = Vbak[c];
        };
        auto accept = [&](int j, int k, int op, double e2) {
          e = e2;
          masked_error(R.data(), M, U.data(), V.data(), m, n, r, td.data(), A.data());
          closed[k] = 1;
          accepted = true;
          rec.j = j; rec.k = k; rec.op = op; rec.e = e;
          S.accepted++;
          acc_this_pass++;
        };
        // (U (x) V)_tj of the current state
        auto prod = [&](int t, int j) {
          T best = U[(size_t)t * r + 0] + V[j];
          for (int l = 1; l < r; ++l) {
            T x = U[(size_t)t * r + l] + V[(size_t)l * n + j];
            if (x > best) best = x;
          }
          return best;
        };
        if (strategy == 1) {
          // ByElement: every observed (i, j) of the row in working column
          // order, k = f(i, j), F-ULF then F-URF; a perfect entry (td = 0) is
          // not updated; after an accepted update the visit goes on with the
          // next element
          for (int j = 0; j < n; ++j) {
            if (!M[(size_t)i * n + j]) continue;
            T best = U[(size_t)i * r] + V[j];
            int k = 0;
            for (int l = 1; l < r; ++l) {
              T x = U[(size_t)i * r + l] + V[(size_t)l * n + j];
              if (x > best) { best = x; k = l; }
            }
            if ((T)(R[(size_t)i * n + j] - best) == (T)0) continue;
            accepted = false;
            for (int op = 0; op < 2 && !accepted; ++op) {
              double e2;
              if (!try_op(j, k, op, e2)) continue;
              if (e2 < e) accept(j, k, op, e2);
              else restore(k);
            }
            if (accepted) {
              if (log && nlog < log_cap) log[nlog] = rec;
              nlog++;
              rec = oracle_log{it, i, 0, 0, -1, -1, -1, 0, e};
            }
          }
          rec.e = e;
          if (log && nlog < log_cap) log[nlog] = rec;
          nlog++;
          continue;
        }
        std::vector<int> cand;  // observed columns of row i
        for (int j = 0; j < n; ++j)
          if (M[(size_t)i * n + j]) cand.push_back(j);

        if (sel == 3) {
          // SEQ: every (j, k, operation), the smallest error below e wins
          int bj = -1, bk = -1, bop = -1;
          double be = e;
          for (int j : cand)
            for (int k = 0; k < r; ++k)
              for (int op = 0; op < 2; ++op) {
                double e2;
                if (!try_op(j, k, op, e2)) continue;
                if (e2 < be) { be = e2; bj = j; bk = k; bop = op; }
                restore(k);
              }
          if (bj >= 0) {
            // apply the chosen update again (the same arithmetic, the same result)
            double e2 = bop == 0
                ? f_ulf(R.data(), M, U.data(), V.data(), m, n, r, i, bj, bk,
                        Ubak.data(), Vbak.data(), nullptr, nullptr)
                : f_urf(R.data(), M, U.data(), V.data(), m, n, r, i, bj, bk,
                        Ubak.data(), Vbak.data(), nullptr, nullptr);
            accept(bj, bk, bop, e2);
          }
        } else {
          // candidate order and the component of each candidate
          std::vector<int> kof((size_t)n, 0);
          if (sel == 1) {
            // TD: entry error td(i, j) descending; k = f(i, j)
            std::vector<double> tij((size_t)n, 0.0);
            for (int j : cand) {
              T d = R[(size_t)i * n + j] - prod(i, j);
              tij[j] = std::fabs((double)d);
              kof[j] = A[(size_t)i * n + j];
            }
            std::stable_sort(cand.begin(), cand.end(),
                             [&](int a, int b) { return tij[a] > tij[b]; });
          } else {
            // TD_A and TD_B: td_col descending
            std::stable_sort(cand.begin(), cand.end(),
                             [&](int a, int b) { return td[a] > td[b]; });
            if (sel == 0) {
              // TD_A: the index counted most often in the two argmax multisets
              std::vector<int> crow((size_t)r, 0);
              for (int t = 0; t < n; ++t)
                if (scope_all || M[(size_t)i * n + t]) crow[A[(size_t)i * n + t]]++;
              for (int j : cand) {
                std::vector<int> cnt(crow);
                for (int t = 0; t < m; ++t)
                  if (scope_all || M[(size_t)t * n + j]) cnt[A[(size_t)t * n + j]]++;
                int k = 0;
                for (int l = 1; l < r; ++l)
                  if (cnt[l] > cnt[k]) k = l;
                kof[j] = k;
              }
            } else {
              // TD_B: j0 = largest td_col, i0 = the first working row
              int j0 = 0;
              for (int t = 1; t < n; ++t)
                if (td[t] > td[j0]) j0 = t;
              const int i0 = 0;
              const T p_ij0 = prod(i, j0);
              const int f_ij0 = A[(size_t)i * n + j0];
              for (int j : cand)
                kof[j] = p_ij0 >= prod(i0, j) ? f_ij0 : A[(size_t)i0 * n + j];
            }
          }
          for (int j : cand) {
            const int k = kof[j];
            for (int op = 0; op < 2 && !accepted; ++op) {
              double e2;
              if (!try_op(j, k, op, e2)) continue;
              if (e2 < e) accept(j, k, op, e2);
              else restore(k);
            }
            if (accepted) break;
          }
        }
        S.row_visits++;
        if (log && nlog < log_cap) log[nlog] = rec;
        nlog++;
      }
      if (stop && rows_left == 0) break;
      it_done = it;
      if (traj) traj[it] = e;
      // Sec. 3.3: stop once a pass lowers the error by less than eps
      bool fixed_point = acc_this_pass == 0;
      bool small_step = eps > 0.0 && (e_prev_pass - e < eps);
      e_prev_pass = e;
      if (fixed_point || small_step) {
        if (traj)
          for (int q = it + 1; q <= iters; ++q) traj[q] = e;
        stop = true;
      }
    }
  }

  S.iters_done = it_done;
  if (log_len) *log_len = nlog;
  if (st) *st = S;

  // un-permute and un-transpose (Algorithm 3, output step)
  std::vector<float> Uw((size_t)m * r);
  for (int a = 0; a < m; ++a)
    for (int l = 0; l < r; ++l) Uw[(size_t)w.perm[a] * r + l] = (float)U[(size_t)a * r + l];
  // working column b goes back to column cperm[b]
  std::vector<float> Vw((size_t)r * n);
  for (int l = 0; l < r; ++l)
    for (int b = 0; b < n; ++b) Vw[(size_t)l * n + w.cperm[b]] = (float)V[(size_t)l * n + b];
  if (!w.transposed) {
    if (U_out) std::memcpy(U_out, Uw.data(), sizeof(float) * Uw.size());
    if (V_out) std::memcpy(V_out, Vw.data(), sizeof(float) * Vw.size());
  } else {
    // original is n x m' ... U_out (m_in x r) = V_w^T, V_out (r x n_in) = U_unperm^T
    if (U_out)
      for (int a = 0; a < m_in; ++a)
        for (int l = 0; l < r; ++l) U_out[(size_t)a * r + l] = Vw[(size_t)l * n + a];
    if (V_out)
      for (int l = 0; l < r; ++l)
        for (int b = 0; b < n_in; ++b) V_out[(size_t)l * n_in + b] = Uw[(size_t)b * r + l];
  }
  return OK;
}

}  // namespace

extern "C" {

// Algorithm 3.  U_out (m x rank), V_out (rank x n) in the original
// orientation; traj gets iters + 1 values; log (nullable) one record per row
// visit.  row_limit > 0 stops after that many row visits (prefix runs).
int oracle_fit_f64(const float* R, const uint8_t* M, int m, int n, int rank,
                   int iters, uint64_t seed, const oracle_opts* o, float* U_out,
                   float* V_out, double* traj, oracle_log* log, int log_cap,
                   int* log_len, oracle_stats* st, int row_limit) {
  return fit<double>(R, M, m, n, rank, iters, seed, o, U_out, V_out, traj, log,
                     log_cap, log_len, st, row_limit);
}
int oracle_fit_f32(const float* R, const uint8_t* M, int m, int n, int rank,
                   int iters, uint64_t seed, const oracle_opts* o, float* U_out,
                   float* V_out, double* traj, oracle_log* log, int log_cap,
                   int* log_len, oracle_stats* st, int row_limit) {
  return fit<float>(R, M, m, n, rank, iters, seed, o, U_out, V_out, traj, log,
                    log_cap, log_len, st, row_limit);
}

// Setup draws of a fit, for checking a library's own random stream: the
// working permutation (m' entries) and U0 (m' x rank, working orientation).
int oracle_draw_init(const float* R, const uint8_t* M, int m, int n, int rank,
                     uint64_t seed, const oracle_opts* o, int32_t* perm_out,
                     float* U0_out) {
  SplitMix64 g{seed};
  Working w;
  int s = build_working(R, M, m, n, o, seed, w, g);
  if (s) return s;
  std::vector<float> U0;
  s = init_U0(w, rank, o, g, U0);
  if (s) return s;
  if (perm_out) std::memcpy(perm_out, w.perm.data(), sizeof(int32_t) * w.perm.size());
  if (U0_out) std::memcpy(U0_out, U0.data(), sizeof(float) * U0.size());
  return OK;
}

}  // extern "C"

// ============================================================ lockstep
// The FP32-value oracle (the precision in which the GPU library takes its
// decisions) checked decision by decision against FP64 arithmetic, for the
// FastSTMF method (ByRow, TD_A).  The FP32 run goes its own way; before every
// row visit its state is promoted exactly to double (the FP64 side is
// re-synchronised to it), and every decision of the visit is recomputed in
// FP64 from that state:
//   - the candidate order: each pair of consecutive candidates, up to the
//     accepted one, must also be in order by the FP64 td_col;
//   - the component of each tried candidate: the TD_A count argmax from the
//     FP64 argmax of every counted cell;
//   - every trial (a no-op skip counting as a rejection): the same operation
//     applied in FP64 to the promoted state, accepted iff its FP64 error is
//     below the FP64 error of the promoted state.
// A decision the FP64 side takes the other way is a rounding flip when the
// quantity deciding it is within `band` (relative) of the tie on either side
// (|e' - e| / e, the gap between two td_col keys, the gap between the two
// max-plus terms of a counted cell), and a mismatch otherwise.  The
// trajectory of the FP64 side is the FP64 error of the synchronised state
// at the end of each pass.
namespace {

int validate_input(const float* Rin, const uint8_t* Min, int m_in, int n_in, int r, int iters,
                   bool int_exact) {
  if (m_in < 1 || n_in < 1 || r < 1 || r > 64 || iters < 0) return EINVAL_;
  for (int i = 0; i < m_in; ++i) {
    int c = 0;
    for (int j = 0; j < n_in; ++j) c += Min[(size_t)i * n_in + j] ? 1 : 0;
    if (!c) return EEMPTY;
  }
  for (int j = 0; j < n_in; ++j) {
    int c = 0;
    for (int i = 0; i < m_in; ++i) c += Min[(size_t)i * n_in + j] ? 1 : 0;
    if (!c) return EEMPTY;
  }
  if (int_exact)
    for (size_t q = 0; q < (size_t)m_in * n_in; ++q)
      if (Min[q] && !(std::fabs(Rin[q]) < 16777216.0f)) return ERANGE_;
  return OK;
}

}  // namespace

extern "C" {

struct oracle_lock_report {
  int64_t row_visits;
  int64_t trials;            // operations the FP32 run decided (evaluated or skipped)
  int64_t agree;             // decisions the FP64 replay takes the same way
  int64_t flips;             // taken the other way, within the band of a tie
  int64_t flips_f32_accepts; // of those: the FP32 run accepts, FP64 rejects
  int64_t mismatches;        // taken the other way beyond it
  int64_t order_pairs;       // candidate pairs checked
  int64_t order_flips, order_mismatches;
  int64_t k_checked;         // components checked
  int64_t k_flips, k_mismatches;
  int32_t iters_done;
  int32_t first_bad_iter;    // first mismatch of any kind (-1: none)
  int32_t first_bad_row;
  int32_t pad;
  double max_rel_traj;       // max over passes of |traj_f32 - traj_f64| / traj_f64
  double max_flip_margin;    // largest relative margin among the flips
};

void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

int oracle_lockstep(const float* Rin, const uint8_t* Min, int m_in, int n_in, int r, int iters,
                    uint64_t seed, const oracle_opts* o, double band, double* traj_f,
                    double* traj_d, oracle_log* log, int log_cap, int* log_len,
                    oracle_lock_report* rep) {
  if (o && (o->selection != 0 || o->strategy != 0)) return EINVAL_;
  const bool int_exact = o && o->integer_exact;
  int s = validate_input(Rin, Min, m_in, n_in, r, iters, int_exact);
  if (s) return s;
  SplitMix64 g{seed};
  Working w;
  s = build_working(Rin, Min, m_in, n_in, o, seed, w, g);
  if (s) return s;
  std::vector<float> U0;
  s = init_U0(w, r, o, g, U0);
  if (s) return s;
  const int m = w.m, n = w.n;
  const uint8_t* M = w.M.data();
  const int scope_all = o && o->count_scope == 1;
  const int noop_rule = o ? o->noop_rule : 1;
  const double eps = o ? o->eps : 0.0;

  // the FP32 run's state, and the FP64 side's arrays
  std::vector<float> R = w.R, U = U0, V((size_t)r * n);
  std::vector<double> Rd((size_t)m * n), Ud((size_t)m * r), Vd((size_t)r * n);
  for (size_t q = 0; q < R.size(); ++q) Rd[q] = (double)R[q];
  for (int k = 0; k < r; ++k) col_res(R.data(), M, m, n, r, k, U.data(), V.data());
  std::vector<double> td((size_t)n), tdd((size_t)n);
  std::vector<int32_t> A((size_t)m * n), Ad((size_t)m * n);
  std::vector<float> Ubak((size_t)m), Vbak((size_t)n);
  std::vector<double> Udb((size_t)m), Vdb((size_t)n);
  std::vector<char> closed((size_t)r, 0);
  oracle_lock_report Q{};
  Q.first_bad_iter = Q.first_bad_row = -1;
  auto bad = [&](int it, int i) {
    if (Q.first_bad_iter < 0) { Q.first_bad_iter = it; Q.first_bad_row = i; }
  };
  auto promote = [&]() {
    for (size_t q = 0; q < U.size(); ++q) Ud[q] = (double)U[q];
    for (size_t q = 0; q < V.size(); ++q) Vd[q] = (double)V[q];
    return masked_error(Rd.data(), M, Ud.data(), Vd.data(), m, n, r, tdd.data(), Ad.data());
  };
  auto rel = [](double a, double b) {
    const double s = std::max(std::fabs(a), std::fabs(b));
    return s > 0.0 ? std::fabs(a - b) / s : 0.0;
  };

  double e = masked_error(R.data(), M, U.data(), V.data(), m, n, r, td.data(), A.data());
  double ed = promote();
  if (traj_f) traj_f[0] = e;
  if (traj_d) traj_d[0] = ed;
  Q.max_rel_traj = rel(e, ed);
  int nlog = 0;
  double e_prev_pass = e;
  bool stop = false;
  for (int it = 1; it <= iters && !stop; ++it) {
    int64_t acc_pass = 0;
    for (int i = 0; i < m; ++i) {
      ed = promote();
      oracle_log rec{it, i, 0, 0, -1, -1, -1, 0, e};
      std::vector<int> cand;
      for (int j = 0; j < n; ++j)
        if (M[(size_t)i * n + j]) cand.push_back(j);
      std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return td[a] > td[b]; });
      // TD_A counts of row i, in both precisions
      std::vector<int> crow((size_t)r, 0), crowd((size_t)r, 0);
      for (int t = 0; t < n; ++t)
        if (scope_all || M[(size_t)i * n + t]) {
          crow[A[(size_t)i * n + t]]++;
          crowd[Ad[(size_t)i * n + t]]++;
        }
      // a counted cell whose argmax differs between the two precisions: a
      // near-tie of two max-plus terms in FP64?
      auto cell_near_tie = [&](int t, int c) {
        const int a = A[(size_t)t * n + c], b = Ad[(size_t)t * n + c];
        if (a == b) return true;
        const double pa = Ud[(size_t)t * r + a] + Vd[(size_t)a * n + c];
        const double pb = Ud[(size_t)t * r + b] + Vd[(size_t)b * n + c];
        return rel(pa, pb) <= band;
      };
      bool accepted = false;
      size_t pos = 0;
      for (; pos < cand.size() && !accepted; ++pos) {
        const int j = cand[pos];
        std::vector<int> cnt(crow), cntd(crowd);
        for (int t = 0; t < m; ++t)
          if (scope_all || M[(size_t)t * n + j]) {
            cnt[A[(size_t)t * n + j]]++;
            cntd[Ad[(size_t)t * n + j]]++;
          }
        int k = 0, kd = 0;
        for (int l = 1; l < r; ++l) {
          if (cnt[l] > cnt[k]) k = l;
          if (cntd[l] > cntd[kd]) kd = l;
        }
        Q.k_checked++;
        if (k != kd) {
          bool ties = true;
          for (int t = 0; t < n && ties; ++t)
            if (scope_all || M[(size_t)i * n + t]) ties = cell_near_tie(i, t);
          for (int t = 0; t < m && ties; ++t)
            if (scope_all || M[(size_t)t * n + j]) ties = cell_near_tie(t, j);
          if (ties) Q.k_flips++;
          else { Q.k_mismatches++; bad(it, i); }
        }
        for (int op = 0; op < 2 && !accepted; ++op) {
          // FP32 run
          const float Rij = R[(size_t)i * n + j];
          bool skip_f = false;
          double e2 = e;
          if (noop_rule && closed[k]) {
            const float Uik = U[(size_t)i * r + k], Vkj = V[(size_t)k * n + j];
            skip_f = op == 0 ? (float)(Rij - Vkj) == Uik : (float)(Rij - Uik) == Vkj;
          }
          if (skip_f) {
            rec.noops++;
          } else {
            e2 = op == 0 ? f_ulf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k, Ubak.data(),
                                 Vbak.data(), nullptr, nullptr)
                         : f_urf(R.data(), M, U.data(), V.data(), m, n, r, i, j, k, Ubak.data(),
                                 Vbak.data(), nullptr, nullptr);
            rec.trials++;
          }
          const bool acc_f = !skip_f && e2 < e;
          // FP64 replay of the same operation from the promoted state
          const double Rijd = Rd[(size_t)i * n + j];
          bool skip_d = false;
          double e2d = ed;
          if (noop_rule && closed[k]) {
            const double Uik = Ud[(size_t)i * r + k], Vkj = Vd[(size_t)k * n + j];
            skip_d = op == 0 ? (Rijd - Vkj) == Uik : (Rijd - Uik) == Vkj;
          }
          if (!skip_d) {
            e2d = op == 0 ? f_ulf(Rd.data(), M, Ud.data(), Vd.data(), m, n, r, i, j, k, Udb.data(),
                                  Vdb.data(), nullptr, nullptr)
                          : f_urf(Rd.data(), M, Ud.data(), Vd.data(), m, n, r, i, j, k, Udb.data(),
                                  Vdb.data(), nullptr, nullptr);
            for (int t = 0; t < m; ++t) Ud[(size_t)t * r + k] = Udb[t];
            for (int c = 0; c < n; ++c) Vd[(size_t)k * n + c] = Vdb[c];
          }
          const bool acc_d = !skip_d && e2d < ed;
          Q.trials++;
          if (acc_f == acc_d) {
            Q.agree++;
          } else {
            const double mf = rel(e2, e), md = rel(e2d, ed);
            if (std::min(mf, md) <= band) {
              Q.flips++;
              if (acc_f) Q.flips_f32_accepts++;
              Q.max_flip_margin = std::max(Q.max_flip_margin, std::min(mf, md));
            } else {
              Q.mismatches++;
              bad(it, i);
            }
          }
          if (acc_f) {
            e = e2;
            masked_error(R.data(), M, U.data(), V.data(), m, n, r, td.data(), A.data());
            closed[k] = 1;
            accepted = true;
            rec.j = j; rec.k = k; rec.op = op; rec.e = e;
            acc_pass++;
          } else if (!skip_f) {
            for (int t = 0; t < m; ++t) U[(size_t)t * r + k] = Ubak[t];
            for (int c = 0; c < n; ++c) V[(size_t)k * n + c] = Vbak[c];
          }
        }
      }
      // candidate order up to (and including the pair after) the last tried
      // candidate, by the FP64 td_col of the visit's starting state
      const size_t last = std::min(pos, cand.size() - 1);
      for (size_t p = 0; p < last; ++p) {
        const int a = cand[p], b = cand[p + 1];
        Q.order_pairs++;
        const bool ok = tdd[a] > tdd[b] || (tdd[a] == tdd[b] && a < b);
        if (!ok) {
          if (rel(tdd[a], tdd[b]) <= band) Q.order_flips++;
          else { Q.order_mismatches++; bad(it, i); }
        }
      }
      Q.row_visits++;
      if (log && nlog < log_cap) log[nlog] = rec;
      nlog++;
    }
    ed = promote();
    if (traj_f) traj_f[it] = e;
    if (traj_d) traj_d[it] = ed;
    Q.max_rel_traj = std::max(Q.max_rel_traj, rel(e, ed));
    Q.iters_done = it;
    const bool fixed_point = acc_pass == 0;
    const bool small_step = eps > 0.0 && (e_prev_pass - e < eps);
    e_prev_pass = e;
    if (fixed_point || small_step) {
      for (int q = it + 1; q <= iters; ++q) {
        if (traj_f) traj_f[q] = e;
        if (traj_d) traj_d[q] = ed;
      }
      stop = true;
    }
  }
  if (log_len) *log_len = nlog;
  if (rep) *rep = Q;
  return OK;
}

}  // extern "C"
