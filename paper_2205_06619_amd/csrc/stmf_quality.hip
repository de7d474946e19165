// Completion quality (Sec. 3.6) of a factorization on a held-out split
// (Sec. 3.7): RMSE-A over the training cells, RMSE-P over the held-out
// cells, and the distance correlation (DC) of the held-out cells' original
// and approximated values.
//
// The product P = U (x) V is formed in FP32 as everywhere else in the
// library; R - P and every sum are FP64, in fixed orders (per row by a fixed
// tree, rows in order; DC per sample over all samples in order, samples by a
// fixed split and tree), so the results do not depend on timing.
//
// Distance correlation (Szekely, Rizzo and Bakirov, Ann. Statist. 35(6),
// 2007), V-statistic form, without the N x N matrices: with a_kl = |x_k - x_l|,
// b_kl = |y_k - y_l|, row means ra_k, rb_k and grand means ga, gb, the
// double-centred products sum to
//   sum_kl A_kl B_kl = sum_kl a_kl b_kl - 2 N sum_k ra_k rb_k + N^2 ga gb
// (A and B have zero row and column sums), so one pass over the pairs
// collecting per sample k the sums of a, b, a b, a^2 and b^2 gives dCov^2,
// dVar^2(x) and dVar^2(y).  The pass is FP64 vector-ALU work, 10 operations
// per pair.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/stmf.h"
#include "stmf_internal.h"

namespace stmf {

static constexpr int QT = 256;          // threads per workgroup of these kernels
static constexpr int DC_CHUNK = 2048;   // samples staged in LDS at a time

// Sum of v over a workgroup of QT threads by a fixed tree (result in thread 0).
__device__ double block_sum(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = QT / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  const double out = s[0];
  __syncthreads();
  return out;
}

// (U (x) V)_ij in FP32 from U's row staged in LDS.
__device__ float product_at(const float* urow, const float* __restrict__ V, int n, int r, int j) {
  float p = urow[0] + V[j];
  for (int l = 1; l < r; ++l) p = fmaxf(p, urow[l] + V[(size_t)l * n + j]);
  return p;
}

// Per row i: sums of (R - P)^2 over its training and held-out cells, and the
// counts of both (one workgroup per row).
__global__ void __launch_bounds__(QT) quality_rows_kernel(
    const float* __restrict__ R, const uint8_t* __restrict__ Mtr, const uint8_t* __restrict__ Mte,
    const float* __restrict__ U, const float* __restrict__ V, int n, int r,
    double* __restrict__ sq, int* __restrict__ cnt) {
  __shared__ float urow[RMAX];
  __shared__ double red[QT];
  const int i = blockIdx.x;
  if ((int)threadIdx.x < r) urow[threadIdx.x] = U[(size_t)i * r + threadIdx.x];
  __syncthreads();
  double s_tr = 0.0, s_te = 0.0;
  int c_tr = 0, c_te = 0;
  for (int j = threadIdx.x; j < n; j += QT) {
    const size_t q = (size_t)i * n + j;
    const bool tr = Mtr[q] != 0, te = Mte[q] != 0;
    if (!tr && !te) continue;
    const double d = (double)R[q] - (double)product_at(urow, V, n, r, j);
    if (tr) { s_tr += d * d; ++c_tr; }
    if (te) { s_te += d * d; ++c_te; }
  }
  s_tr = block_sum(s_tr, red);
  s_te = block_sum(s_te, red);
  const double n_tr = block_sum((double)c_tr, red);
  const double n_te = block_sum((double)c_te, red);
  if (threadIdx.x == 0) {
    sq[2 * i] = s_tr;
    sq[2 * i + 1] = s_te;
    cnt[2 * i] = (int)n_tr;
    cnt[2 * i + 1] = (int)n_te;
  }
}

// One workgroup: the rows' held-out offsets (exclusive scan, row order) and
// the totals: tot[0] training squared sum, tot[1] held-out squared sum,
// tot[2], tot[3] the two counts.
__global__ void __launch_bounds__(QT) quality_scan_kernel(const double* __restrict__ sq,
                                                         const int* __restrict__ cnt, int m,
                                                         int* __restrict__ off,
                                                         double* __restrict__ tot) {
  __shared__ double red[QT];
  __shared__ int base;
  double s_tr = 0.0, s_te = 0.0, n_tr = 0.0;
  for (int i = threadIdx.x; i < m; i += QT) {
    s_tr += sq[2 * i];
    s_te += sq[2 * i + 1];
    n_tr += (double)cnt[2 * i];
  }
  s_tr = block_sum(s_tr, red);
  s_te = block_sum(s_te, red);
  n_tr = block_sum(n_tr, red);
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  // exclusive scan of the held-out counts, QT rows at a time (waves by
  // shuffles, then the wave totals in order)
  __shared__ int wtot[QT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < m; i0 += QT) {
    const int i = i0 + threadIdx.x;
    const int c = i < m ? cnt[2 * i + 1] : 0;
    int incl = c;
    for (int s = 1; s < 64; s <<= 1) {
      const int v = __shfl_up(incl, s, 64);
      if (lane >= s) incl += v;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int before = base;
    for (int w = 0; w < wave; ++w) before += wtot[w];
    if (i < m) off[i] = before + incl - c;
    __syncthreads();
    if (threadIdx.x == QT - 1) base = before + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tot[0] = s_tr;
    tot[1] = s_te;
    tot[2] = n_tr;
    tot[3] = (double)base;
  }
}

// Held-out cells in row-major order: x = R, y = P (one workgroup per row).
__global__ void __launch_bounds__(QT) quality_gather_kernel(
    const float* __restrict__ R, const uint8_t* __restrict__ Mte, const float* __restrict__ U,
    const float* __restrict__ V, int n, int r, const int* __restrict__ off,
    float* __restrict__ x, float* __restrict__ y) {
  __shared__ float urow[RMAX];
  __shared__ int wcnt[QT / 64];
  const int i = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((int)threadIdx.x < r) urow[threadIdx.x] = U[(size_t)i * r + threadIdx.x];
  __syncthreads();
  int pos = off[i];
  for (int j0 = 0; j0 < n; j0 += QT) {
    const int j = j0 + threadIdx.x;
    const bool te = j < n && Mte[(size_t)i * n + j] != 0;
    const unsigned long long b = __ballot(te);
    if (lane == 0) wcnt[wave] = __popcll(b);
    __syncthreads();
    int at = pos + __popcll(b & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) at += wcnt[w];
    if (te) {
      x[at] = R[(size_t)i * n + j];
      y[at] = product_at(urow, V, n, r, j);
    }
    int tot = 0;
    for (int w = 0; w < QT / 64; ++w) tot += wcnt[w];
    pos += tot;
    __syncthreads();
  }
}

// Per sample k: sums over all l of a_kl, b_kl, a_kl b_kl, a_kl^2, b_kl^2
// (terms[5k .. 5k + 4]); samples l staged in LDS, in order.
__global__ void __launch_bounds__(QT) dcor_rows_kernel(const float* __restrict__ x,
                                                      const float* __restrict__ y, int N,
                                                      double* __restrict__ terms) {
  __shared__ float2 xy[DC_CHUNK];
  const int k = blockIdx.x * QT + threadIdx.x;
  const double xk = k < N ? (double)x[k] : 0.0, yk = k < N ? (double)y[k] : 0.0;
  double sa = 0.0, sb = 0.0, sab = 0.0, saa = 0.0, sbb = 0.0;
  for (int l0 = 0; l0 < N; l0 += DC_CHUNK) {
    const int len = N - l0 < DC_CHUNK ? N - l0 : DC_CHUNK;
    __syncthreads();
    for (int e = threadIdx.x; e < len; e += QT) xy[e] = make_float2(x[l0 + e], y[l0 + e]);
    __syncthreads();
#pragma unroll 4
    for (int e = 0; e < len; ++e) {
      const float2 v = xy[e];
      const double a = fabs(xk - (double)v.x), b = fabs(yk - (double)v.y);
      sa += a;
      sb += b;
      sab += a * b;
      saa += a * a;
      sbb += b * b;
    }
  }
  if (k < N) {
    double* t = terms + (size_t)5 * k;
    t[0] = sa; t[1] = sb; t[2] = sab; t[3] = saa; t[4] = sbb;
  }
}

// One workgroup: dCov^2, dVar^2(x), dVar^2(y) and dCor from the per-sample
// sums (res[0] dCor, res[1] dCov^2, res[2] dVar^2(x), res[3] dVar^2(y)).
__global__ void __launch_bounds__(QT) dcor_final_kernel(const double* __restrict__ terms, int N,
                                                       double* __restrict__ res) {
  __shared__ double red[QT];
  const double nn = (double)N;
  double sa = 0.0, sb = 0.0, sab = 0.0, saa = 0.0, sbb = 0.0, rab = 0.0, raa = 0.0, rbb = 0.0;
  for (int k = threadIdx.x; k < N; k += QT) {
    const double* t = terms + (size_t)5 * k;
    const double ra = t[0] / nn, rb = t[1] / nn;
    sa += t[0]; sb += t[1]; sab += t[2]; saa += t[3]; sbb += t[4];
    rab += ra * rb; raa += ra * ra; rbb += rb * rb;
  }
  sa = block_sum(sa, red);
  sb = block_sum(sb, red);
  sab = block_sum(sab, red);
  saa = block_sum(saa, red);
  sbb = block_sum(sbb, red);
  rab = block_sum(rab, red);
  raa = block_sum(raa, red);
  rbb = block_sum(rbb, red);
  if (threadIdx.x == 0) {
    double dcov2 = 0.0, vx = 0.0, vy = 0.0, dc = 0.0;
    if (N > 0) {
      const double n2 = nn * nn, ga = sa / n2, gb = sb / n2;
      dcov2 = (sab - 2.0 * nn * rab + n2 * ga * gb) / n2;
      vx = (saa - 2.0 * nn * raa + n2 * ga * ga) / n2;
      vy = (sbb - 2.0 * nn * rbb + n2 * gb * gb) / n2;
      const double den = sqrt(vx * vy);
      dc = den > 0.0 ? sqrt((dcov2 > 0.0 ? dcov2 : 0.0) / den) : 0.0;
    }
    res[0] = dc; res[1] = dcov2; res[2] = vx; res[3] = vy;
  }
}

static inline size_t al256q(size_t v) { return (v + 255) / 256 * 256; }

static size_t dcor_ws(size_t N) { return al256q(N * 5 * sizeof(double)) + al256q(4 * sizeof(double)); }

static hipError_t launch_dcor(const float* x, const float* y, int N, double* terms, double* res,
                              hipStream_t s) {
  if (N > 0)
    hipLaunchKernelGGL(dcor_rows_kernel, dim3((N + QT - 1) / QT), dim3(QT), 0, s, x, y, N, terms);
  hipLaunchKernelGGL(dcor_final_kernel, dim3(1), dim3(QT), 0, s, terms, N, res);
  return hipGetLastError();
}

}  // namespace stmf

using namespace stmf;

#define QCHK(expr)                                  \
  do {                                              \
    if ((expr) != hipSuccess) return STMF_EHIP;     \
  } while (0)

extern "C" {

size_t stmf_dcor_workspace(int N) { return N < 0 ? 0 : dcor_ws((size_t)N); }

int stmf_distance_correlation(const float* x, const float* y, int N, double* out,
                              double* row_terms, void* ws, size_t ws_bytes, void* stream) {
  if (N < 0 || !out || (N > 0 && (!x || !y))) return STMF_EINVAL;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < dcor_ws((size_t)N)) return STMF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  double* terms = row_terms ? row_terms : (double*)ws;
  double* res = (double*)((char*)ws + al256q((size_t)N * 5 * sizeof(double)));
  QCHK(launch_dcor(x, y, N, terms, res, s));
  QCHK(hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  QCHK(hipStreamSynchronize(s));
  return STMF_OK;
}

size_t stmf_completion_metrics_workspace(int m, int n, int r) {
  if (m < 1 || n < 1 || r < 1 || r > RMAX) return 0;
  const size_t cells = (size_t)m * n;
  return al256q((size_t)m * 2 * sizeof(double)) + al256q((size_t)m * 2 * sizeof(int)) +
         al256q((size_t)m * sizeof(int)) + al256q(4 * sizeof(double)) +
         2 * al256q(cells * sizeof(float)) + dcor_ws(cells);
}

int stmf_completion_metrics(const float* R, const uint8_t* M_train, const uint8_t* M_test,
                            const float* U, const float* V, int m, int n, int r, double* out,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!R || !M_train || !M_test || !U || !V || !out || m < 1 || n < 1 || r < 1 || r > RMAX)
    return STMF_EINVAL;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < stmf_completion_metrics_workspace(m, n, r))
    return STMF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const size_t cells = (size_t)m * n;
  char* p = (char*)ws;
  double* sq = (double*)p;  p += al256q((size_t)m * 2 * sizeof(double));
  int* cnt = (int*)p;       p += al256q((size_t)m * 2 * sizeof(int));
  int* off = (int*)p;       p += al256q((size_t)m * sizeof(int));
  double* tot = (double*)p; p += al256q(4 * sizeof(double));
  float* x = (float*)p;     p += al256q(cells * sizeof(float));
  float* y = (float*)p;     p += al256q(cells * sizeof(float));
  double* terms = (double*)p;
  double* res = (double*)(p + al256q(cells * 5 * sizeof(double)));
  hipLaunchKernelGGL(quality_rows_kernel, dim3(m), dim3(QT), 0, s, R, M_train, M_test, U, V, n, r,
                     sq, cnt);
  hipLaunchKernelGGL(quality_scan_kernel, dim3(1), dim3(QT), 0, s, sq, cnt, m, off, tot);
  QCHK(hipGetLastError());
  double h[4];
  QCHK(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
  QCHK(hipStreamSynchronize(s));
  const int N = (int)h[3];
  if (N > 0)
    hipLaunchKernelGGL(quality_gather_kernel, dim3(m), dim3(QT), 0, s, R, M_test, U, V, n, r, off,
                       x, y);
  QCHK(launch_dcor(x, y, N, terms, res, s));
  double d[4];
  QCHK(hipMemcpyAsync(d, res, sizeof(d), hipMemcpyDeviceToHost, s));
  QCHK(hipStreamSynchronize(s));
  out[0] = h[2] > 0 ? sqrt(h[0] / h[2]) : 0.0;
  out[1] = N > 0 ? sqrt(h[1] / (double)N) : 0.0;
  out[2] = d[0];
  out[3] = h[2];
  out[4] = (double)N;
  return STMF_OK;
}

}  // extern "C"
