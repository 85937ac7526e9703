// Kernels of the field-circuit coupled step (Sec. 3.1): the dense
// right-hand-side CG start of the set-up solves Z = A^-1 B^T, and the
// per-column elimination of the circuit unknowns after a step's linear solve.
// Every sum runs in a fixed order, so a column's result does not depend on
// the batch it is computed in, except that a one-column batch (the
// sequential steppers, the coarsest level's steps) spreads the rows of each
// partial dot over the lanes of its wave.
#include <hip/hip_runtime.h>

#include "circuit.h"

namespace mg {
namespace {

__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// x = 0, r^ = S b; partials r^.r^, r.r (= b.b) and b.b per row block, summed
// over the block's four waves in a fixed order.
__global__ __launch_bounds__(kBlock) void k_circ_rhs_init(int n, const double* __restrict__ sc,
                                                          const double* __restrict__ B, int64_t ldb,
                                                          int ncols, int rpb, int64_t ld,
                                                          double* __restrict__ x, double* __restrict__ r,
                                                          double* __restrict__ part, int nrb,
                                                          int* __restrict__ flags) {
  __shared__ double red[3][4][kWave];
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = blockIdx.x * kWave + lane;
  const int rb = blockIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (c < ncols) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const double b = B[static_cast<int64_t>(i) * ldb + c];
      const double rh = sc[i] * b;
      x[static_cast<int64_t>(i) * ld + c] = 0.0;
      r[static_cast<int64_t>(i) * ld + c] = rh;
      acc[0] += rh * rh;
      acc[1] += b * b;
      acc[2] += b * b;
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) red[q][wv][lane] = acc[q];
  __syncthreads();
  if (wv == 0 && c < ncols) {
    const int64_t qs = static_cast<int64_t>(nrb) * ld;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      part[q * qs + static_cast<int64_t>(rb) * ld + c] =
          ((red[q][0][lane] + red[q][1][lane]) + red[q][2][lane]) + red[q][3][lane];
  }
}

// One wave per partial p (kCircRowsPerWave consecutive rows), one lane per
// column: part[p][j][c] = sum_i Bt[i][j] (y[i][c] - a[i][c]), rows in order.
__global__ __launch_bounds__(kBlock) void k_circ_dots(int n, int k, int ncols,
                                                      const double* __restrict__ Bt,
                                                      const double* __restrict__ y, int64_t ldy,
                                                      const double* __restrict__ a, int64_t lda,
                                                      double* __restrict__ part, int64_t ldp,
                                                      int nparts) {
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = blockIdx.x * kWave + lane;
  const int p = blockIdx.y * 4 + wv;
  if (p >= nparts || c >= ncols) return;
  double acc[kCircMax];
#pragma unroll
  for (int j = 0; j < kCircMax; ++j) acc[j] = 0.0;
  const int i0 = p * kCircRowsPerWave;
  const int i1 = (i0 + kCircRowsPerWave < n) ? i0 + kCircRowsPerWave : n;
  // unrolled so that several rows' loads are in flight (narrow batches, one
  // column in sequential stepping, are latency-bound); the order of the sums
  // is unchanged
#pragma unroll 8
  for (int i = i0; i < i1; ++i) {
    const double d = y[static_cast<int64_t>(i) * ldy + c] - a[static_cast<int64_t>(i) * lda + c];
    const double* b = Bt + static_cast<int64_t>(i) * k;
#pragma unroll
    for (int j = 0; j < kCircMax; ++j)
      if (j < k) acc[j] = fma(b[j], d, acc[j]);
  }
  double* o = part + static_cast<int64_t>(p) * k * ldp + c;
#pragma unroll
  for (int j = 0; j < kCircMax; ++j)
    if (j < k) o[static_cast<int64_t>(j) * ldp] = acc[j];
}

// As k_circ_dots, with the residual of the step's inexact solve folded in.
// The solve left y with A y = (M/dt) a - r, r its residual (recomputed here
// row by row); A is symmetric, so the error of y seen by the circuit rows is
// B A^-1 r = Z^T r, and the exact B (y* - a) is B (y - a) + Z^T r:
//   part[p][j][c] = sum_i Bt[i][j] (y - a)[i][c] + Z[i][j] r[i][c], rows in order.
// The circuit unknowns then carry no error of the solve, and a' = y + Z w
// differs from the exact step by the solve's own error only.
template <int W>
__global__ __launch_bounds__(kBlock) void k_circ_dots_res(
    int n, int k, int ncols, const double* __restrict__ Bt, const double* __restrict__ Z,
    const int* __restrict__ col, const double* __restrict__ av, const double* __restrict__ mm,
    const uint8_t* __restrict__ has_mass, const double* __restrict__ y, int64_t ldy,
    const double* __restrict__ a, int64_t lda, double* __restrict__ part, int64_t ldp, int nparts) {
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = blockIdx.x * kWave + lane;
  const int p = blockIdx.y * 4 + wv;
  if (p >= nparts || c >= ncols) return;
  double acc[kCircMax];
#pragma unroll
  for (int j = 0; j < kCircMax; ++j) acc[j] = 0.0;
  const int i0 = p * kCircRowsPerWave;
  const int i1 = (i0 + kCircRowsPerWave < n) ? i0 + kCircRowsPerWave : n;
#pragma unroll 2
  for (int i = i0; i < i1; ++i) {
    const int* ci = col + static_cast<int64_t>(i) * W;
    double bv = 0.0;
    if (has_mass[i]) {
      const double* mi = mm + static_cast<int64_t>(i) * W;
#pragma unroll
      for (int t = 0; t < W; ++t) bv += mi[t] * a[static_cast<int64_t>(ci[t]) * lda + c];
    }
    const double* ai = av + static_cast<int64_t>(i) * W;
    double ax = 0.0;
#pragma unroll
    for (int t = 0; t < W; ++t) ax += ai[t] * y[static_cast<int64_t>(ci[t]) * ldy + c];
    const double r = bv - ax;
    const double d = y[static_cast<int64_t>(i) * ldy + c] - a[static_cast<int64_t>(i) * lda + c];
    const double* b = Bt + static_cast<int64_t>(i) * k;
    const double* z = Z + static_cast<int64_t>(i) * k;
#pragma unroll
    for (int j = 0; j < kCircMax; ++j)
      if (j < k) acc[j] = fma(z[j], r, fma(b[j], d, acc[j]));
  }
  double* o = part + static_cast<int64_t>(p) * k * ldp + c;
#pragma unroll
  for (int j = 0; j < kCircMax; ++j)
    if (j < k) o[static_cast<int64_t>(j) * ldp] = acc[j];
}

__global__ void k_circ_sum(int k, int ncols, int nparts, const double* __restrict__ part, int64_t ldp,
                           double* __restrict__ d, int64_t ldd) {
  const int c = blockIdx.x * kWave + static_cast<int>(threadIdx.x);
  const int j = blockIdx.y;
  if (c >= ncols || j >= k) return;
  double t = 0.0;
#pragma unroll 8
  for (int p = 0; p < nparts; ++p) t += part[(static_cast<int64_t>(p) * k + j) * ldp + c];
  d[static_cast<int64_t>(j) * ldd + c] = t;
}

// One column of the dots on one column: wave p sums the rows of partial p,
// row i0 + q * 64 + lane on lane `lane`, then reduces over its lanes by a
// butterfly (the same order on every call).
__global__ __launch_bounds__(kBlock) void k_circ_dots1(int n, int k, const double* __restrict__ Bt,
                                                       const double* __restrict__ y, int64_t ldy,
                                                       const double* __restrict__ a, int64_t lda,
                                                       double* __restrict__ part, int64_t ldp, int nparts) {
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int p = blockIdx.x * 4 + wv;
  if (p >= nparts) return;   // wave-uniform
  double acc[kCircMax];
#pragma unroll
  for (int j = 0; j < kCircMax; ++j) acc[j] = 0.0;
  const int i0 = p * kCircRowsPerWave;
#pragma unroll
  for (int q = 0; q < kCircRowsPerWave / kWave; ++q) {
    const int i = i0 + q * kWave + lane;
    if (i < n) {
      const double d = y[static_cast<int64_t>(i) * ldy] - a[static_cast<int64_t>(i) * lda];
      const double* b = Bt + static_cast<int64_t>(i) * k;
#pragma unroll
      for (int j = 0; j < kCircMax; ++j)
        if (j < k) acc[j] = fma(b[j], d, acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < kCircMax; ++j) {
    if (j < k) {
      double v = acc[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[j] = v;
    }
  }
  if (lane == 0) {
    double* o = part + static_cast<int64_t>(p) * k * ldp;
#pragma unroll
    for (int j = 0; j < kCircMax; ++j)
      if (j < k) o[static_cast<int64_t>(j) * ldp] = acc[j];
  }
}

// One thread per column and circuit unknown j.
__global__ void k_circ_solve(int k, int ncols, const double* __restrict__ d, int64_t ldd,
                             const double* __restrict__ src, int64_t lds,
                             const double* __restrict__ cS, double* __restrict__ w, int64_t ldw) {
  const int c = blockIdx.x * kWave + static_cast<int>(threadIdx.x);
  const int j = blockIdx.y;
  if (c >= ncols || j >= k) return;
  const double v0 = src[c], v1 = src[lds + c], v2 = src[2 * lds + c];
  const double* row = cS + static_cast<int64_t>(j) * (3 + k);
  double t = (row[0] * v0 + row[1] * v1) + row[2] * v2;
#pragma unroll
  for (int l = 0; l < kCircMax; ++l)
    if (l < k) t = fma(-row[3 + l], d[static_cast<int64_t>(l) * ldd + c], t);
  w[static_cast<int64_t>(j) * ldw + c] = t;
}

// x[i][c] += sum_j Z[i][j] w[j][c]: one lane per column, a wave walks 64 rows.
__global__ __launch_bounds__(kBlock) void k_circ_apply(int n, int k, int ncols,
                                                       const double* __restrict__ Z,
                                                       const double* __restrict__ w, int64_t ldw,
                                                       double* __restrict__ x, int64_t ldx) {
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = blockIdx.x * kWave + lane;
  if (c >= ncols) return;
  double wc[kCircMax];
#pragma unroll
  for (int j = 0; j < kCircMax; ++j) wc[j] = (j < k) ? w[static_cast<int64_t>(j) * ldw + c] : 0.0;
  const int i0 = (blockIdx.y * 4 + wv) * kWave;
  const int i1 = (i0 + kWave < n) ? i0 + kWave : n;
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const double* z = Z + static_cast<int64_t>(i) * k;
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kCircMax; ++j)
      if (j < k) t = fma(z[j], wc[j], t);
    x[static_cast<int64_t>(i) * ldx + c] += t;
  }
}

// x[i] += sum_j Z[i][j] w[j] for one column: one thread per row (the sum in
// the order of k_circ_apply).
__global__ void k_circ_apply1(int n, int k, const double* __restrict__ Z, const double* __restrict__ w,
                              int64_t ldw, double* __restrict__ x, int64_t ldx) {
  const int i = blockIdx.x * blockDim.x + static_cast<int>(threadIdx.x);
  if (i >= n) return;
  const double* z = Z + static_cast<int64_t>(i) * k;
  double t = 0.0;
#pragma unroll
  for (int j = 0; j < kCircMax; ++j)
    if (j < k) t = fma(z[j], w[static_cast<int64_t>(j) * ldw], t);
  x[static_cast<int64_t>(i) * ldx] += t;
}

// w[j][c] = -wt[j][i], i the column's time point (0 outside [0, nt)).
__global__ void k_circ_recall(int k, int ncols, const int64_t* __restrict__ t_list, int64_t t_base,
                              int64_t t_stride, const double* __restrict__ wt, int64_t nt,
                              double* __restrict__ w, int64_t ldw) {
  const int c = blockIdx.x * kWave + static_cast<int>(threadIdx.x);
  const int j = blockIdx.y;
  if (c >= ncols || j >= k) return;
  const int64_t i = t_list ? t_list[c] : t_base + static_cast<int64_t>(c) * t_stride;
  w[static_cast<int64_t>(j) * ldw + c] = (i >= 0 && i < nt) ? -wt[static_cast<int64_t>(j) * nt + i] : 0.0;
}

// wt[j][i] = w[j][c], i the column's time point (skipped outside [0, nt)).
__global__ void k_circ_keep(int k, int ncols, const int64_t* __restrict__ t_list, int64_t t_base,
                            int64_t t_stride, const double* __restrict__ w, int64_t ldw,
                            double* __restrict__ wt, int64_t nt) {
  const int c = blockIdx.x * kWave + static_cast<int>(threadIdx.x);
  const int j = blockIdx.y;
  if (c >= ncols || j >= k) return;
  const int64_t i = t_list ? t_list[c] : t_base + static_cast<int64_t>(c) * t_stride;
  if (i >= 0 && i < nt) wt[static_cast<int64_t>(j) * nt + i] = w[static_cast<int64_t>(j) * ldw + c];
}

}  // namespace

void launch_circ_rhs_init(hipStream_t s, const DevLevel& L, PcgWork& w, const double* B, int64_t ldb,
                          int ncols) {
  if (ncols <= 0) return;
  if (ncols > w.cap) fail(MGRIT_INVALID_ARGUMENT, "circuit set-up solve wider than its workspace");
  hipLaunchKernelGGL(k_circ_rhs_init, dim3(cdiv(ncols, kWave), w.nrb), dim3(kBlock), 0, s, L.n, L.s64, B,
                     ldb, ncols, w.rows_per_block, w.ld, w.x, w.r, w.part, w.nrb, w.flags);
  MG_HIP(hipGetLastError());
}

int circ_parts(int n) { return cdiv(n, kCircRowsPerWave); }

void launch_circ_dots(hipStream_t s, int n, int k, int ncols, const double* Bt, CView y, CView a,
                      double* part, int64_t ldp) {
  if (ncols <= 0 || n <= 0) return;
  if (k < 1 || k > kCircMax || ldp < ncols) fail(MGRIT_INVALID_ARGUMENT, "circuit dots: bad sizes");
  const int np = circ_parts(n);
  if (ncols == 1)
    hipLaunchKernelGGL(k_circ_dots1, dim3(cdiv(np, 4)), dim3(kBlock), 0, s, n, k, Bt, y.p, y.ld, a.p, a.ld,
                       part, ldp, np);
  else
    hipLaunchKernelGGL(k_circ_dots, dim3(cdiv(ncols, kWave), cdiv(np, 4)), dim3(kBlock), 0, s, n, k, ncols,
                       Bt, y.p, y.ld, a.p, a.ld, part, ldp, np);
  MG_HIP(hipGetLastError());
}

void launch_circ_dots_res(hipStream_t s, const DevLevel& L, int k, int ncols, const double* Bt,
                          const double* Z, CView y, CView a, double* part, int64_t ldp) {
  if (ncols <= 0 || L.n <= 0) return;
  if (k < 1 || k > kCircMax || ldp < ncols) fail(MGRIT_INVALID_ARGUMENT, "circuit dots: bad sizes");
  if (L.W != 8 && L.W != 16) fail(MGRIT_INVALID_ARGUMENT, "circuit dots: unsupported row width");
  const int np = circ_parts(L.n);
  auto kern = (L.W == 8) ? k_circ_dots_res<8> : k_circ_dots_res<16>;
  hipLaunchKernelGGL(kern, dim3(cdiv(ncols, kWave), cdiv(np, 4)), dim3(kBlock), 0, s, L.n, k, ncols, Bt, Z,
                     L.col, L.a64, L.m64, L.has_mass, y.p, y.ld, a.p, a.ld, part, ldp, np);
  MG_HIP(hipGetLastError());
}

void launch_circ_sum(hipStream_t s, int k, int ncols, int nparts, const double* part, int64_t ldp,
                     double* d, int64_t ldd) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_circ_sum, dim3(cdiv(ncols, kWave), k), dim3(kWave), 0, s, k, ncols, nparts, part,
                     ldp, d, ldd);
  MG_HIP(hipGetLastError());
}

void launch_circ_solve(hipStream_t s, int k, int ncols, const double* d, int64_t ldd,
                       const double* src, int64_t lds, const double* cS, double* w, int64_t ldw) {
  if (ncols <= 0) return;
  if (k < 1 || k > kCircMax) fail(MGRIT_INVALID_ARGUMENT, "circuit solve: bad sizes");
  hipLaunchKernelGGL(k_circ_solve, dim3(cdiv(ncols, kWave), k), dim3(kWave), 0, s, k, ncols, d, ldd, src, lds,
                     cS, w, ldw);
  MG_HIP(hipGetLastError());
}

void launch_circ_apply(hipStream_t s, int n, int k, int ncols, const double* Z, const double* w,
                       int64_t ldw, double* x, int64_t ldx) {
  if (ncols <= 0 || n <= 0) return;
  if (k < 1 || k > kCircMax) fail(MGRIT_INVALID_ARGUMENT, "circuit apply: bad sizes");
  if (ncols == 1)
    hipLaunchKernelGGL(k_circ_apply1, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, k, Z, w, ldw, x, ldx);
  else
    hipLaunchKernelGGL(k_circ_apply, dim3(cdiv(ncols, kWave), cdiv(n, 4 * kWave)), dim3(kBlock), 0, s, n, k,
                       ncols, Z, w, ldw, x, ldx);
  MG_HIP(hipGetLastError());
}

void launch_circ_recall(hipStream_t s, int k, int ncols, const int64_t* t_list, int64_t t_base,
                        int64_t t_stride, const double* wt, int64_t nt, double* w, int64_t ldw) {
  if (ncols <= 0) return;
  if (k < 1 || k > kCircMax || ldw < ncols) fail(MGRIT_INVALID_ARGUMENT, "circuit recall: bad sizes");
  hipLaunchKernelGGL(k_circ_recall, dim3(cdiv(ncols, kWave), k), dim3(kWave), 0, s, k, ncols, t_list, t_base,
                     t_stride, wt, nt, w, ldw);
  MG_HIP(hipGetLastError());
}

void launch_circ_keep(hipStream_t s, int k, int ncols, const int64_t* t_list, int64_t t_base,
                      int64_t t_stride, const double* w, int64_t ldw, double* wt, int64_t nt) {
  if (ncols <= 0) return;
  if (k < 1 || k > kCircMax || ldw < ncols) fail(MGRIT_INVALID_ARGUMENT, "circuit keep: bad sizes");
  hipLaunchKernelGGL(k_circ_keep, dim3(cdiv(ncols, kWave), k), dim3(kWave), 0, s, k, ncols, t_list, t_base,
                     t_stride, w, ldw, wt, nt);
  MG_HIP(hipGetLastError());
}

}  // namespace mg
