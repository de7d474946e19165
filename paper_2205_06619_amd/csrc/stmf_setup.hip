// Set-up and output steps of a fit (Algorithm 3): input checks, the working
// matrix (transposed when R is not wide, rows permuted or in the PermR order
// of Sec. 3.2, missing cells as
// +inf), the initial U (given, random integers drawn on the host, or Random
// Acol averages), the initial V = (-U)^T (x)* R for every component, and the
// un-permuted, un-transposed output.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stmf_internal.h"

namespace stmf {

static constexpr float SINF = __builtin_huge_valf();


// Observed counts of every row and column (atomics) and value checks.
__global__ void check_count_kernel(const float* __restrict__ R, const uint8_t* __restrict__ M,
                                   int m, int n, int* __restrict__ rowc, int* __restrict__ colc,
                                   CheckOut* out) {
  const size_t total = (size_t)m * n;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (size_t)gridDim.x * blockDim.x) {
    if (!M[x]) continue;
    const int i = (int)(x / n), j = (int)(x % n);
    atomicAdd(&rowc[i], 1);
    atomicAdd(&colc[j], 1);
    const float v = R[x];
    if (!(v == v) || v == SINF || v == -SINF) atomicOr(&out->nonfinite, 1);
    else {
      if (fabsf(v) >= 1e30f) atomicOr(&out->too_big, 1);
      if (fabsf(v) >= 16777216.0f) atomicOr(&out->not_int24, 1);
    }
  }
}

__global__ void check_empty_kernel(const int* __restrict__ rowc, const int* __restrict__ colc,
                                   int m, int n, CheckOut* out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < m && rowc[x] == 0) atomicAdd(&out->empty_rows, 1);
  if (x < m && rowc[x] > 0) atomicAdd(&out->observed, rowc[x]);
  if (x < n && colc[x] == 0) atomicAdd(&out->empty_cols, 1);
}

__global__ void fill_u32_kernel(unsigned* __restrict__ p, size_t count, unsigned v) {
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < count;
       x += (size_t)gridDim.x * blockDim.x)
    p[x] = v;
}

// Working matrix: Rw[a][b] = R at original (perm[a], cperm[b]), or
// (cperm[b], perm[a]) when transposed; +inf at missing and padding cells; -0
// becomes +0.
__global__ void pack_kernel(const float* __restrict__ R, const uint8_t* __restrict__ M, int n_in,
                            int mw, int nw, int ldm, int ldn, int transposed,
                            const int* __restrict__ perm, const int* __restrict__ cperm,
                            float* __restrict__ Rw) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (b >= ldn || a >= ldm) return;
  float v = SINF;
  if (a < mw && b < nw) {
    const int src = perm[a], csrc = cperm[b];
    const size_t idx = transposed ? ((size_t)csrc * n_in + src) : ((size_t)src * n_in + csrc);
    if (M[idx]) v = R[idx] + 0.0f;
  }
  Rw[(size_t)a * ldn + b] = v;
}

// PermR / PermC (Sec. 3.3), first step: mn[a] = the minimum observed value
// of line a: original row a (elements R[a][b], b < nw), or with `transposed`
// original column a (elements R[b][a]); one workgroup of 256 threads per
// line.  Every line has an observed cell (checked before).  -0 and +0 compare equal, so the order never depends on the sign
// of a zero.
__global__ void __launch_bounds__(256) rowmin_kernel(const float* __restrict__ R,
                                                     const uint8_t* __restrict__ M, int n_in,
                                                     int nw, int transposed, float* __restrict__ mn) {
  __shared__ float part[256];
  const int a = blockIdx.x;
  float best = SINF;
  for (int b = threadIdx.x; b < nw; b += 256) {
    const size_t idx = transposed ? ((size_t)b * n_in + a) : ((size_t)a * n_in + b);
    if (M[idx]) best = fminf(best, R[idx]);
  }
  part[threadIdx.x] = best;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] = fminf(part[threadIdx.x], part[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) mn[a] = part[0] + 0.0f;
}

// PermR / PermC, second step: the stable order of the lines by increasing
// minimum, perm[rank of a] = a, the rank counting the lines with a smaller
// minimum or an equal one at a lower index.
__global__ void rank_perm_kernel(const float* __restrict__ mn, int mw, int* __restrict__ perm) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= mw) return;
  const float v = mn[a];
  int rank = 0;
  for (int b = 0; b < mw; ++b) {
    const float o = mn[b];
    rank += (o < v || (o == v && b < a)) ? 1 : 0;
  }
  perm[rank] = a;
}

// perm[a] = a for a < count.
__global__ void iota_kernel(int* __restrict__ perm, int count) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < count) perm[a] = a;
}

// RwT = Rw^T through 64 x 64 LDS tiles.
__global__ void __launch_bounds__(256) transpose_kernel(const float* __restrict__ Rw, int ldm,
                                                        int ldn, float* __restrict__ RwT) {
  __shared__ float tile[TS][TS + 1];
  const int r0 = blockIdx.y * TS, c0 = blockIdx.x * TS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = wave; t < TS; t += 4) tile[t][lane] = Rw[(size_t)(r0 + t) * ldn + c0 + lane];
  __syncthreads();
  for (int c = wave; c < TS; c += 4) RwT[(size_t)(c0 + c) * ldm + r0 + lane] = tile[lane][c];
}

// Uc[l][t] = U0[t][l] (working orientation, row-major m' x r); padding 0.
__global__ void u0_given_kernel(const float* __restrict__ U0, int mw, int r, int ldm,
                                float* __restrict__ Uc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (t >= ldm) return;
  Uc[(size_t)l * ldm + t] = t < mw ? U0[(size_t)t * r + l] + 0.0f : 0.0f;
}

// Random Acol: U_tl = mean of the observed values of working row t at the
// drawn columns cols[l][0..p), summed in double in draw order; a row with
// none of them observed takes the mean of all its observed values (column
// order).  Rounded once to float.
__global__ void u0_acol_kernel(const float* __restrict__ Rw, int mw, int nw, int ldm, int ldn,
                               int r, int p, const int* __restrict__ cols,
                               float* __restrict__ Uc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ldm) return;
  if (t >= mw) {
    for (int l = 0; l < r; ++l) Uc[(size_t)l * ldm + t] = 0.0f;
    return;
  }
  const float* row = Rw + (size_t)t * ldn;
  double rs = 0.0;
  int rc = 0;
  for (int b = 0; b < nw; ++b)
    if (row[b] != SINF) { rs += (double)row[b]; ++rc; }
  for (int l = 0; l < r; ++l) {
    double s = 0.0;
    int c = 0;
    for (int q = 0; q < p; ++q) {
      const float v = row[cols[l * p + q]];
      if (v != SINF) { s += (double)v; ++c; }
    }
    const double mean = c ? s / (double)c : rs / (double)rc;
    Uc[(size_t)l * ldm + t] = (float)mean + 0.0f;
  }
}

// Initial V: V_lc = min over observed t of R_tc - U_tl, for every component.
__global__ void vinit_kernel(const float* __restrict__ Rw, const float* __restrict__ Uc, int mw,
                             int nw, int ldm, int ldn, int r, float* __restrict__ V) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (c >= ldn) return;
  float best = 0.0f;
  if (c < nw) {
    best = SINF;
    for (int t = 0; t < mw; ++t) best = fminf(best, Rw[(size_t)t * ldn + c] - Uc[(size_t)l * ldm + t]);
  }
  V[(size_t)l * ldn + c] = best;
}

// Output (Algorithm 3, last step): U_unperm[perm[a]] = U_w[a] and
// V_unperm[:, cperm[c]] = V_w[:, c]; if transposed, U_out = V_unperm^T and
// V_out = U_unperm^T, else U_out = U_unperm, V_out = V_unperm.
__global__ void output_kernel(const float* __restrict__ Uc, const float* __restrict__ V, int mw,
                              int nw, int ldm, int ldn, int r, int transposed,
                              const int* __restrict__ perm, const int* __restrict__ cperm,
                              float* __restrict__ U_out, float* __restrict__ V_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (!transposed) {
    // original m = mw rows, n = nw columns
    if (x < mw) U_out[(size_t)perm[x] * r + l] = Uc[(size_t)l * ldm + x];
    if (x < nw) V_out[(size_t)l * nw + cperm[x]] = V[(size_t)l * ldn + x];
  } else {
    // original m = nw rows, n = mw columns
    if (x < nw) U_out[(size_t)cperm[x] * r + l] = V[(size_t)l * ldn + x];
    if (x < mw) V_out[(size_t)l * mw + perm[x]] = Uc[(size_t)l * ldm + x];
  }
}

// Device-to-device copy of the error trajectory out of a fit's workspace.
__global__ void copy_f64_kernel(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) dst[x] = src[x];
}


}  // namespace stmf
