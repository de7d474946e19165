// Internal layout shared by the HIP kernels and the host side of the library.
// (Not part of the public ABI; the public declarations live in include/stmf.h.)
#pragma once
#include <stdint.h>

// The fit kernel's device code sees the workspace arrays of a fit as
// global-address-space pointers (plain global loads instead of flat ones);
// every other translation unit sees plain pointers.  The layout is the same.
#if defined(__HIP_DEVICE_COMPILE__) && defined(STMF_FIT_KERNEL_TU)
#define STMF_G(T) __attribute__((address_space(1))) T*
#else
#define STMF_G(T) T*
#endif

namespace stmf {

constexpr int TS = 64;          // tile side: 64 rows x 64 columns of the working matrix
constexpr int NWAVE = 8;        // waves per workgroup
constexpr int NTHR = 64 * NWAVE;
constexpr int TMAX = 1024;      // trials per speculative batch (upper bound)
constexpr int TCH = 64;         // trials staged in LDS at a time
constexpr int CW = 256;         // candidate columns examined at a time
constexpr int RMAX = 64;        // largest supported rank
constexpr int SORT_MAX = 4096;  // widest matrix sorted in one workgroup's LDS

// Top-2 summary of a residual line: smallest value, its (lowest) index, and
// the second smallest value (equal to m1 on ties; +inf if the line has one
// observed cell).
struct Top2 {
  float m1;
  int a1;
  float m2;
  int pad;
};

enum Op : int { OP_ULF = 0, OP_URF = 1, OP_NULL = 2 };

// ByRow selections of (j, k) within a row visit (Sec. 3.2.1), and the
// ByElement (Sec. 3.2.2) and ByMatrix (Sec. 3.2.3) strategies, which the fit
// kernel runs as two more.
enum Sel : int { SEL_TD_A = 0, SEL_TD = 1, SEL_TD_B = 2, SEL_SEQ = 3, SEL_ELEM = 4, SEL_MATRIX = 5 };

// ByMatrix: the operation of the c-th cell tried in a fit comes from the
// SplitMix64 stream seeded with the fit's seed XOR this constant.
constexpr unsigned long long MATRIX_OP_STREAM = 0xA0761D6478BD642Full;
constexpr int MATRIX_HIST = 12;  // radix-select passes: 8 key digits, 4 position digits

struct Trial {
  int j, k, op;
  float val;   // the step-2 value written at (i, k) of U (F-ULF) or (k, j) of V (F-URF)
};

// Results of the input checks of a fit.
struct CheckOut {
  int empty_rows, empty_cols;
  int nonfinite;   // an observed value that is not finite
  int too_big;     // an observed |R| >= 1e30
  int not_int24;   // an observed |R| >= 2^24
  int observed;    // observed cells
  int pad[2];
};

// One record per row visit (decision log).
struct LogRec {
  int32_t iter, row, trials, noops, j, k, op, pad;
  double e;
};

// Two-level group barrier: workgroup g of a group belongs to subgroup
// g / BAR_SUB; the counters only grow (from zero at the fit's preparation),
// each on a 128-byte line of its own.
constexpr int BAR_SUB = 16;                    // workgroups per subgroup
constexpr int BAR_NSUB = 16;                   // subgroups
constexpr int GROUP_MAX = BAR_SUB * BAR_NSUB;  // largest group
struct alignas(128) BarTree {
  unsigned top[32];             // [0]: arrivals of the subgroups' last members
  unsigned sub[BAR_NSUB][32];   // [q][0]: arrivals of subgroup q's members
  unsigned rel[BAR_NSUB][32];   // [q][0]: episodes released to subgroup q
};

// Control block of one fit (device memory).  Everything a resumed launch
// needs to continue a fit lives here or in the arrays of FitDev.
struct FitCtl {
  double e;              // current b-norm (FP64)
  double e_new;          // error of the trial chosen by the last batch
  int decision;          // index of the first improving trial of the batch, -1 none
  int status;            // 0 ok; nonzero aborts the fit
  int phase;             // 0 needs init, 1 iterating, 2 done
  int it;                // current pass (1-based) while iterating
  int row;               // next working row to visit
  int acc_in_pass;       // acceptances in the current pass
  int ncand;             // candidates of the current row
  int iters_done;
  unsigned queue;        // batched launches: next fit to take (only in ctl[0])
  unsigned pad0;
  long long trials;      // trials the method evaluates (up to the accepted one)
  long long spec_trials; // trials evaluated including speculative ones
  long long noops;       // trials skipped by the no-op rule
  long long accepted;
  long long row_visits;
  long long batches;
  long long cells;       // sum over evaluated trials of |Omega| (method count)
  int nlog;
  int cbuf;              // which of the two argmax-count buffers is current
  long long phase_ticks[8];  // leader's wall time per phase (100 MHz ticks)
  long long mdraws;      // ByMatrix: operation draws consumed so far
  unsigned long long mlast_u;  // ByMatrix: key and position of the last
  long long mlast_q;           // selected cell (the next selection's cursor)
};

// Device-side descriptor of one fit.  All arrays live in the caller's
// workspace.  Working orientation: m <= n, rows permuted.
struct FitDev {
  int m, n, r;           // working shape and rank
  int ldm, ldn;          // padded extents (multiples of TS)
  int nrt, nct;          // tile counts
  int iters;
  int noop_rule, count_scope;
  int tmax;              // largest batch
  int t0;                // first batch of a row visit
  int log_cap;
  int omega;             // number of observed cells
  int sel;               // Sel
  double eps;
  unsigned long long seed_ops;  // ByMatrix: seed ^ MATRIX_OP_STREAM
  STMF_G(const float) Rw;    // ldm x ldn, +inf at unobserved and padding cells
  STMF_G(const float) RwT;   // ldn x ldm, the transpose
  STMF_G(float) Uc;          // r x ldm: Uc[l*ldm + t] = U_tl
  STMF_G(float) V;           // r x ldn: V[l*ldn + c]  = V_lc
  STMF_G(double) td;         // ldn: td_col
  STMF_G(double) tdpart;     // nrt x ldn
  STMF_G(int) crow;          // 2 x ldm x r: argmax counts of every row (two buffers)
  STMF_G(int) ccol;          // 2 x ldn x r: argmax counts of every column (two buffers)
  STMF_G(Top2) colst;        // r x ldn: top-2 of R_tc - U_tk over t (per component)
  STMF_G(Top2) rowst;        // r x ldm: top-2 of R_tc - V_kc over c
  STMF_G(Top2) colpart;      // nrt x ldn: per row-tile partial of colst (one component)
  STMF_G(Top2) rowpart;      // nct x ldm
  STMF_G(int) order;         // ldn: columns by (td_col desc, index asc)
  STMF_G(int) rord;          // ldn: TD order of the visited row's columns
  STMF_G(double) tdrow;      // ldn: TD keys of the visited row (wide matrices)
  // ByMatrix (null otherwise): per cell of the m x n working matrix (row-major,
  // unpadded) td (-1 unobserved), f and the order-mapped key; line sums;
  // radix-select histograms; the gathered and the ordered candidates
  STMF_G(double) mtd;
  STMF_G(int) mfk;
  STMF_G(unsigned long long) mkey;
  STMF_G(double) mtdr;       // m
  STMF_G(double) mtdc;       // n
  STMF_G(int) mhist;         // MATRIX_HIST x 256
  STMF_G(int) mcnt;          // 1: gathered count
  STMF_G(unsigned long long) mgat_u;  // tmax
  STMF_G(int) mgat_q;        // tmax
  STMF_G(int) mlist_q;       // tmax: candidates in order (cell position)
  STMF_G(int) mlist_k;       // tmax: their component f(i, j)
  STMF_G(unsigned) tvec;     // 2 x TMAX x ldmax: atomic-min targets (order-mapped floats)
  STMF_G(double) epart;      // tmax x tiles: per-tile partial errors of every trial
  STMF_G(double) eprime;     // TMAX: error of every trial of the batch
  STMF_G(int) closed;        // r
  STMF_G(int) rowt;          // m': trials the last visit of each row evaluated (0: none yet)
  STMF_G(double) traj;       // iters + 1
  STMF_G(LogRec) log;        // nullable
  STMF_G(FitCtl) ctl;
  STMF_G(BarTree) bar;       // the group barrier's counters
  int ldmax;
  int gsize;             // workgroups cooperating on this fit
  long long bar_wait;    // bound of a group-barrier wait in 100 MHz ticks: 0 the
                         // default, negative none (a wait ends at its first
                         // unanswered poll)
};

}  // namespace stmf
