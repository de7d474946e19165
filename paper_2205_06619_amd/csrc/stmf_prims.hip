// Primitive operations on the caller's layout (R, M m x n row-major, U m x r,
// V r x n): the max-plus product and argmax (Section 2, Section 3.2.1), the
// masked b-norm with per-column sums (Sections 3.6 and 3.2.1), and the two
// masked min-plus residual steps of F-ULF / F-URF (Algorithms 1 and 2).
//
// Every value operation is one correctly rounded FP32 operation; error sums
// are FP64 in a fixed order: per column over 64-row tiles (row order), the
// tiles in order, then the columns by a fixed 256-way split and tree.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "stmf.h"
#include "stmf_internal.h"

namespace stmf {

static constexpr float PINF = __builtin_huge_valf();

// P and argmax of a 64 x 64 output tile: lanes over columns, wave w rows
// 16w..16w+15.  U rows of the tile staged in LDS.
__global__ void __launch_bounds__(256) maxplus_kernel(const float* __restrict__ U,
                                                      const float* __restrict__ V, int m,
                                                      int r, int n, float* __restrict__ P,
                                                      int32_t* __restrict__ A) {
  __shared__ float Us[TS][RMAX + 1];
  const int r0 = blockIdx.y * TS, c0 = blockIdx.x * TS;
  for (int e = threadIdx.x; e < TS * r; e += blockDim.x) {
    int t = e / r, l = e % r;
    Us[t][l] = (r0 + t < m) ? U[(size_t)(r0 + t) * r + l] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = c0 + lane;
  if (c >= n) return;
  for (int tt = 0; tt < 16; ++tt) {
    const int tl = wave * 16 + tt, t = r0 + tl;
    if (t >= m) break;
    float best = Us[tl][0] + V[c];
    int arg = 0;
    for (int l = 1; l < r; ++l) {
      float x = Us[tl][l] + V[(size_t)l * n + c];
      if (x > best) { best = x; arg = l; }
    }
    if (P) P[(size_t)t * n + c] = best;
    if (A) A[(size_t)t * n + c] = arg;
  }
}

// Per (row tile, column) FP64 partial of |R - P| over observed cells.
__global__ void __launch_bounds__(256) masked_err_tiles(const float* __restrict__ R,
                                                        const uint8_t* __restrict__ M,
                                                        const float* __restrict__ U,
                                                        const float* __restrict__ V, int m,
                                                        int n, int r, int ldp,
                                                        double* __restrict__ part) {
  __shared__ float Us[TS][RMAX + 1];
  __shared__ double wsum[4][TS];
  const int r0 = blockIdx.y * TS, c0 = blockIdx.x * TS;
  for (int e = threadIdx.x; e < TS * r; e += blockDim.x) {
    int t = e / r, l = e % r;
    Us[t][l] = (r0 + t < m) ? U[(size_t)(r0 + t) * r + l] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = c0 + lane;
  double acc = 0.0;
  if (c < n) {
    for (int tt = 0; tt < 16; ++tt) {
      const int tl = wave * 16 + tt, t = r0 + tl;
      if (t >= m) break;
      if (!M[(size_t)t * n + c]) continue;
      float best = Us[tl][0] + V[c];
      for (int l = 1; l < r; ++l) best = fmaxf(best, Us[tl][l] + V[(size_t)l * n + c]);
      float d = R[(size_t)t * n + c] - best;
      acc += fabs((double)d);
    }
  }
  wsum[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && c < n)
    part[(size_t)blockIdx.y * ldp + c] = ((wsum[0][lane] + wsum[1][lane]) + wsum[2][lane]) + wsum[3][lane];
}

// td_col[c] = sum over row tiles (in order); err = fixed 256-way split over
// columns (thread x sums columns x, x + 256, ... in order) and a fixed tree.
__global__ void __launch_bounds__(256) masked_err_final(const double* __restrict__ part, int nrt,
                                                        int n, int ldp, double* __restrict__ td,
                                                        double* __restrict__ err) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    double v = 0.0;
    for (int rt = 0; rt < nrt; ++rt) v += part[(size_t)rt * ldp + c];
    if (td) td[c] = v;
    acc += v;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) err[0] = s[0];
}

// Backups of U[:,k] and V[k,:].
__global__ void backup_kernel(const float* __restrict__ U, const float* __restrict__ V, int m,
                              int n, int r, int k, float* __restrict__ Ub,
                              float* __restrict__ Vb) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < m) Ub[x] = U[(size_t)x * r + k];
  if (x < n) Vb[x] = V[(size_t)k * n + x];
}

// Step 2 of F-ULF (op 0: U_ik <- R_ij - V_kj) or F-URF (op 1: V_kj <- R_ij - U_ik).
__global__ void step2_kernel(const float* __restrict__ R, float* U, float* V, int n, int r,
                             int i, int j, int k, int op) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const float Rij = R[(size_t)i * n + j];
    if (op == 0) U[(size_t)i * r + k] = Rij - V[(size_t)k * n + j];
    else V[(size_t)k * n + j] = Rij - U[(size_t)i * r + k];
  }
}

// Column residual: V_kc <- min over observed t of R_tc - U_tk (one thread per
// column, reads coalesced across the columns of a row).
__global__ void colres_kernel(const float* __restrict__ R, const uint8_t* __restrict__ M,
                              const float* U, float* V, int m, int n, int r, int k) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float best = PINF;
  for (int t = 0; t < m; ++t)
    if (M[(size_t)t * n + c]) best = fminf(best, R[(size_t)t * n + c] - U[(size_t)t * r + k]);
  V[(size_t)k * n + c] = best;
}

// Row residual: U_tk <- min over observed c of R_tc - V_kc (one wave per row).
__global__ void __launch_bounds__(256) rowres_kernel(const float* __restrict__ R,
                                                     const uint8_t* __restrict__ M, float* U,
                                                     const float* V, int m, int n, int r,
                                                     int k) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= m) return;
  float best = PINF;
  for (int c = lane; c < n; c += 64)
    if (M[(size_t)t * n + c]) best = fminf(best, R[(size_t)t * n + c] - V[(size_t)k * n + c]);
  for (int s = 32; s >= 1; s >>= 1) best = fminf(best, __shfl_xor(best, s, 64));
  if (lane == 0) U[(size_t)t * r + k] = best;
}

// ---------------------------------------------------------------- launchers
size_t masked_error_ws(int m, int n) {
  const int nrt = (m + TS - 1) / TS;
  const size_t ldp = (size_t)((n + 63) / 64) * 64;
  return ((size_t)nrt * ldp * sizeof(double) + 255) / 256 * 256;
}

hipError_t launch_maxplus(const float* U, const float* V, int m, int r, int n, float* P,
                          int32_t* A, hipStream_t s) {
  dim3 grid((n + TS - 1) / TS, (m + TS - 1) / TS);
  hipLaunchKernelGGL(maxplus_kernel, grid, dim3(256), 0, s, U, V, m, r, n, P, A);
  return hipGetLastError();
}

hipError_t launch_masked_error(const float* R, const uint8_t* M, const float* U, const float* V,
                               int m, int n, int r, double* err, double* td, void* ws,
                               hipStream_t s) {
  const int nrt = (m + TS - 1) / TS;
  const int ldp = (n + 63) / 64 * 64;
  double* part = (double*)ws;
  dim3 grid((n + TS - 1) / TS, nrt);
  hipLaunchKernelGGL(masked_err_tiles, grid, dim3(256), 0, s, R, M, U, V, m, n, r, ldp, part);
  hipLaunchKernelGGL(masked_err_final, dim3(1), dim3(256), 0, s, part, nrt, n, ldp, td, err);
  return hipGetLastError();
}

hipError_t launch_update(int op, const float* R, const uint8_t* M, float* U, float* V, int m,
                         int n, int r, int i, int j, int k, float* Ub, float* Vb, double* err,
                         void* ws, hipStream_t s) {
  const int mx = m > n ? m : n;
  hipLaunchKernelGGL(backup_kernel, dim3((mx + 255) / 256), dim3(256), 0, s, U, V, m, n, r, k, Ub,
                     Vb);
  hipLaunchKernelGGL(step2_kernel, dim3(1), dim3(64), 0, s, R, U, V, n, r, i, j, k, op);
  if (op == 0) {
    hipLaunchKernelGGL(colres_kernel, dim3((n + 255) / 256), dim3(256), 0, s, R, M, U, V, m, n, r, k);
    hipLaunchKernelGGL(rowres_kernel, dim3((m + 3) / 4), dim3(256), 0, s, R, M, U, V, m, n, r, k);
  } else {
    hipLaunchKernelGGL(rowres_kernel, dim3((m + 3) / 4), dim3(256), 0, s, R, M, U, V, m, n, r, k);
    hipLaunchKernelGGL(colres_kernel, dim3((n + 255) / 256), dim3(256), 0, s, R, M, U, V, m, n, r, k);
  }
  return launch_masked_error(R, M, U, V, m, n, r, err, nullptr, ws, s);
}

// ---------------------------------------------------------------- no allocation
// Scratch of stmf_masked_error_noalloc: the per (row tile, column) partials,
// up to NOALLOC_PARTIALS doubles (8 MiB; every device the library runs on
// holds its own copy until the process ends).  Its device address is looked
// up once per device, with that device current; the host-side name is never
// passed to a kernel or a copy.
static constexpr size_t NOALLOC_PARTIALS = (size_t)1 << 20;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return STMF_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return STMF_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return STMF_OK;
}

}  // namespace stmf

extern "C" int stmf_masked_error_noalloc(const float* R, const uint8_t* M, const float* U,
                                         const float* V, int m, int n, int r, double* err,
                                         double* td_col, void* stream) {
  using namespace stmf;
  if (!R || !M || !U || !V || !err || m < 1 || n < 1 || r < 1 || r > RMAX) return STMF_EINVAL;
  // the partials of this shape must fit the static scratch
  if (masked_error_ws(m, n) > sizeof(scratch)) return STMF_ENOMEM;
  void* ws = nullptr;
  const int st = scratch_address(&ws);
  if (st) return st;
  // every partial the final reduction reads is written first: nothing to clear
  if (launch_masked_error(R, M, U, V, m, n, r, err, td_col, ws, (hipStream_t)stream) != hipSuccess)
    return STMF_EHIP;
  return STMF_OK;
}
