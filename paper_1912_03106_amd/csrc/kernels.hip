// HIP kernels of the MGRIT library (gfx950).
//
// Data layout of every batched kernel: a "column block" [n][ld] holds one
// state vector per column (node-major, columns contiguous).  The columns are
// the coarse time intervals of an F/C sweep (or the points of a coarse level),
// so every column shares the sparsity pattern and the matrix values of the
// level.  A wave owns 64 consecutive columns of one row at a time: the row's
// pattern and values are wave-uniform (scalar loads), each lane streams its
// own column, and the loads of a row's neighbours are 512-byte coalesced
// segments.  A workgroup (4 waves) covers `rpb` consecutive rows of one
// 64-column chunk; the chunk -> XCD mapping keeps the rows a chunk re-reads
// (neighbours at +-1 and +-n_theta) inside one XCD's L2.
//
// Reductions (dot products, norms) are deterministic: per-workgroup partial
// sums in a fixed order, then a fixed-order reduction per column.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>

#include "internal.h"
#include "source_dev.h"

namespace mg {

namespace {

__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

// Work-group -> (row block, 64-column chunk).  Work-groups are dispatched
// round-robin over the 8 XCDs (XCD = id % 8).  The tiles, ordered chunk by
// chunk and row block by row block within a chunk, are cut into 8 contiguous
// ranges of nearly equal size, one per XCD, which walks its range in order:
// the +-n_theta neighbour rows a tile reads belong to tiles of the same XCD
// run at about the same time, and so are L2 hits.  A bijection on the grid
// (gridDim.x = row blocks x chunks), whatever the chunk count.
__device__ __forceinline__ void tile_decode(int w, int nrb, int ncc, int& rb, int& cc) {
  const int nrb_ = nrb;
  (void)ncc;
  const int T = static_cast<int>(gridDim.x);   // = row blocks x chunks
  const int x = w & 7, k = w >> 3, q = T >> 3, rem = T & 7;
  const int tile = x * q + (x < rem ? x : rem) + k;
  cc = tile / nrb_;
  rb = tile - cc * nrb_;
}

// Sum the per-lane values v[0..NQ) of the 4 waves of a work-group in a fixed
// order and store them, for every lane's column, at out[q * qstride + c].
template <int NQ>
__device__ __forceinline__ void block_partials(const double (&v)[NQ], double* out,
                                               int64_t qstride, int c, bool on) {
  __shared__ double red[NQ][4][kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][wv][lane] = v[q];
  __syncthreads();
  if (wv == 0 && on) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      out[q * qstride + c] = ((red[q][0][lane] + red[q][1][lane]) + red[q][2][lane]) + red[q][3][lane];
  }
}

// ----------------------------------------------------------------------------
// Setup: element geometry and assembly (P1 Galerkin, eq. 7).

__global__ void k_elem_geometry(int n_tri, const double* __restrict__ xy,
                                const int* __restrict__ tri, double* __restrict__ area,
                                double* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_tri) return;
  const int v0 = tri[3 * e], v1 = tri[3 * e + 1], v2 = tri[3 * e + 2];
  const double x0 = xy[2 * v0], y0 = xy[2 * v0 + 1];
  const double x1 = xy[2 * v1], y1 = xy[2 * v1 + 1];
  const double x2 = xy[2 * v2], y2 = xy[2 * v2 + 1];
  const double det = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
  area[e] = 0.5 * det;
  // grad(phi_a) = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / det
  const double inv = 1.0 / det;
  double* g = grad + 6 * e;
  g[0] = (y1 - y2) * inv; g[1] = (x2 - x1) * inv;
  g[2] = (y2 - y0) * inv; g[3] = (x0 - x2) * inv;
  g[4] = (y0 - y1) * inv; g[5] = (x1 - x0) * inv;
}

// One thread per stored entry (row i, slot k): K and M/dt are sums over the
// (element, a, b) contributions listed for that entry, in a fixed order.
__global__ void k_assemble_linear(int n, int W, double inv_dt, const int* __restrict__ cptr,
                                  const int* __restrict__ contrib, const double* __restrict__ area,
                                  const double* __restrict__ grad, const double* __restrict__ nu_e,
                                  const double* __restrict__ sigma_e, double* __restrict__ a64,
                                  float* __restrict__ a32, double* __restrict__ m64) {
  const int64_t slot = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (slot >= static_cast<int64_t>(n) * W) return;
  double kv = 0.0, mv = 0.0;
  for (int t = cptr[slot]; t < cptr[slot + 1]; ++t) {
    const int code = contrib[t];
    const int e = code / 9, a = (code % 9) / 3, b = code % 3;
    const double* g = grad + 6 * e;
    kv += nu_e[e] * area[e] * (g[2 * a] * g[2 * b] + g[2 * a + 1] * g[2 * b + 1]);
    mv += sigma_e[e] * area[e] * ((a == b) ? 2.0 : 1.0) / 12.0;
  }
  const double md = mv * inv_dt;
  m64[slot] = md;
  a64[slot] = md + kv;
  a32[slot] = static_cast<float>(md + kv);
}

__global__ void k_diag_inverse(int n, int W, const int* __restrict__ diag_slot,
                               const double* __restrict__ a64, const double* __restrict__ m64,
                               double* __restrict__ dinv64, float* __restrict__ dinv32,
                               uint8_t* __restrict__ has_mass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = a64[static_cast<int64_t>(i) * W + diag_slot[i]];
  dinv64[i] = 1.0 / d;
  dinv32[i] = static_cast<float>(1.0 / d);
  uint8_t hm = 0;
  for (int k = 0; k < W; ++k) hm |= (m64[static_cast<int64_t>(i) * W + k] != 0.0);
  has_mass[i] = hm;
}

// F_p[i] = sum over the elements touching node i with phase p of sign*area/3
// (the diagonal entry's contribution list is exactly those elements).
__global__ void k_load_vectors(int n, int W, const int* __restrict__ cptr,
                               const int* __restrict__ contrib, const int* __restrict__ diag_slot,
                               const double* __restrict__ area, const int* __restrict__ cell_phase,
                               const int* __restrict__ cell_sign, double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t slot = static_cast<int64_t>(i) * W + diag_slot[i];
  double f[3] = {0.0, 0.0, 0.0};
  for (int t = cptr[slot]; t < cptr[slot + 1]; ++t) {
    const int e = contrib[t] / 9;
    const int p = cell_phase[e];
    if (p >= 0 && p < 3) f[p] += cell_sign[e] * area[e] / 3.0;
  }
  F[i] = f[0];
  F[n + i] = f[1];
  F[2 * n + i] = f[2];
}

// ----------------------------------------------------------------------------
// Batched Phi / PCG.

// table[p][c] = J0*amp * b_p(t) at the new time t = (i_from(c) + 1) * dt;
// optional per-column amplitude factors and phase shifts (training data).
__global__ void k_source_table(SourceDev s, double dt, int ncols, const int64_t* __restrict__ t_list,
                               int64_t t_base, int64_t t_stride, const double* __restrict__ amp,
                               const double* __restrict__ dphi, double* __restrict__ table,
                               int64_t ld) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int64_t i_from = t_list ? t_list[c] : t_base + static_cast<int64_t>(c) * t_stride;
  const double t = static_cast<double>(i_from + 1) * dt;
  SourceDev sc = s;
  if (amp) sc.scale *= amp[c];
  if (dphi)
    for (int p = 0; p < 3; ++p) sc.phi[p] += dphi[c];
  const double a = source_scale(t, sc);
#pragma unroll
  for (int p = 0; p < 3; ++p) table[p * ld + c] = a * pwm(t, sc, p);
}

__global__ void k_axpby3(int n, int ncols, double* __restrict__ out, int64_t ldo, double sx,
                         const double* __restrict__ x, int64_t ldx, double sa,
                         const double* __restrict__ a, int64_t lda, double sb,
                         const double* __restrict__ b, int64_t ldb) {
  const int c = blockIdx.x * kWave + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= ncols || i >= n) return;
  double v = 0.0;
  if (x) v += sx * x[i * ldx + c];
  if (a) v += sa * a[i * lda + c];
  if (b) v += sb * b[i * ldb + c];
  out[i * ldo + c] = v;
}

// Sum of squares of every column over a row block.
__global__ __launch_bounds__(kBlock) void k_colsq(int n, int ncols, int nrb, int ncc, int rpb,
                                                  const double* __restrict__ X, int64_t ldx,
                                                  double* __restrict__ part, int64_t ldp) {
  int rb, cc;
  tile_decode(blockIdx.x, nrb, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols;
  double acc[1] = {0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const double v = X[i * ldx + c];
      acc[0] += v * v;
    }
  }
  block_partials<1>(acc, part + rb * ldp, static_cast<int64_t>(nrb) * ldp, c, on);
}

// Joule-loss partial sums (Sec. 3.1): per column c, d = a[:, c] - b[:, c] and
// the row-block sums of d_i (M/dt d)_i over the rows with a mass entry (the
// conductor nodes); the caller divides the column total by dt.
__global__ __launch_bounds__(kBlock) void k_joule(int n, int W, const int* __restrict__ col,
                                                  const double* __restrict__ mdt,
                                                  const uint8_t* __restrict__ has_mass, int ncols,
                                                  int nrb, int ncc, int rpb,
                                                  const double* __restrict__ a, int64_t lda,
                                                  const double* __restrict__ b, int64_t ldb,
                                                  double* __restrict__ part, int64_t ldp) {
  int rb, cc;
  tile_decode(blockIdx.x, nrb, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols;
  double acc[1] = {0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      if (!has_mass[i]) continue;
      double md = 0.0;
      for (int t = 0; t < W; ++t) {
        const int j = col[static_cast<int64_t>(i) * W + t];
        md += mdt[static_cast<int64_t>(i) * W + t] * (a[j * lda + c] - b[j * ldb + c]);
      }
      acc[0] += (a[i * lda + c] - b[i * ldb + c]) * md;
    }
  }
  block_partials<1>(acc, part + rb * ldp, static_cast<int64_t>(nrb) * ldp, c, on);
}

// Y = alpha * T X + beta * Y for a fixed-width transfer operator.
template <int W>
__global__ __launch_bounds__(kBlock) void k_transfer(int n_out, const int* __restrict__ col,
                                                     const double* __restrict__ val, int ncols,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     double alpha, double* __restrict__ Y,
                                                     int64_t ldy, double beta) {
  const int c = blockIdx.x * kWave + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + wave_index();
  if (c >= ncols || i >= n_out) return;
  const int* ci = col + static_cast<int64_t>(i) * W;
  const double* vi = val + static_cast<int64_t>(i) * W;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < W; ++t) s += vi[t] * X[ci[t] * ldx + c];
  const int64_t o = i * ldy + c;
  Y[o] = (beta == 0.0) ? alpha * s : alpha * s + beta * Y[o];
}

// Tiled transposes between time-major trajectories and slabs.
// Tile: 64 nodes x 64 slab columns of one slab (blockIdx.z = slab).
__global__ __launch_bounds__(kBlock) void k_tm_to_slabs(int n, int64_t npts, int m,
                                                        const double* __restrict__ tm,
                                                        double* __restrict__ slabs, int64_t ld,
                                                        int64_t ss, const int* __restrict__ nat) {
  __shared__ double tile[64][65];
  const int j = blockIdx.z;
  const int64_t k0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int i0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int q = ty; q < 64; q += 4) {
    const int64_t t = (k0 + q) * m + j;
    const int i = i0 + tx;
    tile[q][tx] = (t < npts && i < n) ? tm[t * n + (nat ? nat[i] : i)] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 64; q += 4) {
    const int i = i0 + q;
    const int64_t k = k0 + tx;
    const int64_t t = k * m + j;
    if (i < n && t < npts) slabs[j * ss + i * ld + k] = tile[tx][q];
  }
}

__global__ __launch_bounds__(kBlock) void k_slabs_to_tm(int n, int64_t npts, int m,
                                                        const double* __restrict__ slabs,
                                                        int64_t ld, int64_t ss,
                                                        double* __restrict__ tm,
                                                        const int* __restrict__ nat) {
  __shared__ double tile[64][65];
  const int j = blockIdx.z;
  const int64_t k0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int i0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int q = ty; q < 64; q += 4) {
    const int i = i0 + q;
    const int64_t k = k0 + tx;
    const int64_t t = k * m + j;
    tile[q][tx] = (i < n && t < npts) ? slabs[j * ss + i * ld + k] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 64; q += 4) {
    const int64_t t = (k0 + q) * m + j;
    const int i = i0 + tx;
    if (t < npts && i < n) tm[t * n + (nat ? nat[i] : i)] = tile[tx][q];
  }
}

__global__ void k_cols_to_slabs(int n, int64_t npts, int m, const double* __restrict__ src,
                                int64_t lds, double* __restrict__ slabs, int64_t ld, int64_t ss) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= npts) return;
  for (int i = blockIdx.y; i < n; i += gridDim.y)
    slabs[(t % m) * ss + static_cast<int64_t>(i) * ld + t / m] = src[static_cast<int64_t>(i) * lds + t];
}

__global__ void k_slabs_to_cols(int n, int64_t npts, int m, const double* __restrict__ slabs,
                                int64_t ld, int64_t ss, double* __restrict__ dst, int64_t ldd) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= npts) return;
  for (int i = blockIdx.y; i < n; i += gridDim.y)
    dst[static_cast<int64_t>(i) * ldd + t] = slabs[(t % m) * ss + static_cast<int64_t>(i) * ld + t / m];
}

// ----------------------------------------------------------------------------
// Single-work-group sequential stepper (coarsest level, small sequential
// baselines).  Vectors in global memory (L2-resident at these sizes); block
// reductions in a fixed order.

__device__ double block_sum(double v, double* sh) {
  // wave reduction (fixed butterfly), then the 16 wave sums in order
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += sh[k];
  return t;
}

template <int W>
__global__ __launch_bounds__(kSeqThreads) void k_seq_small(
    int n, const int* __restrict__ col, const double* __restrict__ a,
    const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
    const double* __restrict__ dinv, const double* __restrict__ F, SourceDev src, double dt,
    int nsteps, int64_t t0, double* __restrict__ U, int64_t ldu, const double* __restrict__ G,
    int64_t ldg, double* __restrict__ ws, double tol, int maxit, int warm,
    int* __restrict__ flags) {
  __shared__ double sh[32];
  __shared__ double sgn[3];
  __shared__ int stop;
  if (threadIdx.x == 0) stop = 0;
  double* x = ws;
  double* r = ws + n;
  double* p = ws + 2 * n;
  double* q = ws + 3 * n;
  const double tol2 = tol * tol;
  int total_iters = 0;
  for (int s = 1; s <= nsteps; ++s) {
    if (threadIdx.x == 0) {
      const double t = static_cast<double>(t0 + s) * dt;
      const double amp = source_scale(t, src);
      for (int k = 0; k < 3; ++k) sgn[k] = amp * pwm(t, src, k);
    }
    __syncthreads();
    const double s0 = sgn[0], s1 = sgn[1], s2 = sgn[2];
    // initial guess
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double g = warm ? U[i * ldu + s] : U[i * ldu + s - 1];
      if (warm && G) g -= G[i * ldg + s];
      x[i] = g;
    }
    __syncthreads();
    double lrz = 0.0, lrr = 0.0, lbb = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int* ci = col + static_cast<int64_t>(i) * W;
      double bv = 0.0;
      if (has_mass[i]) {
        const double* mi = mm + static_cast<int64_t>(i) * W;
        for (int t = 0; t < W; ++t) bv += mi[t] * U[ci[t] * ldu + s - 1];
      }
      bv += (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      const double* ai = a + static_cast<int64_t>(i) * W;
      double ax = 0.0;
      for (int t = 0; t < W; ++t) ax += ai[t] * x[ci[t]];
      const double rv = bv - ax;
      const double z = dinv[i] * rv;
      r[i] = rv;
      p[i] = z;
      lrz += rv * z;
      lrr += rv * rv;
      lbb += bv * bv;
    }
    double rz = block_sum(lrz, sh);
    double rr = block_sum(lrr, sh + 16);
    double bb = block_sum(lbb, sh);
    if (bb == 0.0) bb = rr;
    int it = 0;
    while (rr > tol2 * bb) {
      if (it >= maxit) {
        if (threadIdx.x == 0) {
          atomicOr(flags + 1, 2);
          stop = 1;
        }
        break;
      }
      __syncthreads();
      double lpq = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int* ci = col + static_cast<int64_t>(i) * W;
        const double* ai = a + static_cast<int64_t>(i) * W;
        double sq = 0.0;
        for (int t = 0; t < W; ++t) sq += ai[t] * p[ci[t]];
        q[i] = sq;
        lpq += p[i] * sq;
      }
      const double pq = block_sum(lpq, sh);
      const double al = rz / pq;
      double lz = 0.0;
      lrr = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[i] += al * p[i];
        const double rv = r[i] - al * q[i];
        r[i] = rv;
        lz += rv * (dinv[i] * rv);
        lrr += rv * rv;
      }
      const double rzn = block_sum(lz, sh + 16);
      rr = block_sum(lrr, sh);
      const double be = rzn / rz;
      rz = rzn;
      if (!isfinite(rr)) {
        if (threadIdx.x == 0) {
          atomicOr(flags + 1, 1);
          stop = 1;
        }
        break;
      }
      for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = dinv[i] * r[i] + be * p[i];
      __syncthreads();
      ++it;
    }
    total_iters += it;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double v = x[i];
      if (G) v += G[i * ldg + s];
      U[i * ldu + s] = v;
    }
    __syncthreads();
    if (stop) break;
  }
  if (threadIdx.x == 0) atomicAdd(flags + 2, total_iters);
}

// Batched implicit-Euler right-hand sides b[i][c] = (M/dt) u[:, c] + f_c
// (f from the per-column source table src[3][ld]).
__global__ void k_ie_rhs_batch(int n, int W, int ncols, const int* __restrict__ col,
                               const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
                               const double* __restrict__ F, const double* __restrict__ src,
                               int64_t lds, const double* __restrict__ U, int64_t ldu,
                               double* __restrict__ B, int64_t ldb) {
  const int c = blockIdx.x * kWave + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= ncols || i >= n) return;
  double bv = 0.0;
  if (has_mass[i])
    for (int k = 0; k < W; ++k)
      bv += mm[static_cast<int64_t>(i) * W + k] * U[col[static_cast<int64_t>(i) * W + k] * ldu + c];
  bv += (src[c] * F[i] + src[lds + c] * F[n + i]) + src[2 * lds + c] * F[2 * n + i];
  B[i * ldb + c] = bv;
}

// X[i][c] = sum_j Ainv[i][j] B[j][c]: one wave per (row, column), lanes
// stride over j, fixed-order shuffle reduction (the same arithmetic for one
// column or many, so batched and single-step coarse steps agree bitwise).
__global__ __launch_bounds__(kBlock) void k_inv_apply(int n, int ncols, const double* __restrict__ Ainv,
                                                      int64_t lda, const double* __restrict__ B,
                                                      int64_t ldb, double* __restrict__ X,
                                                      int64_t ldx) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x;
  const int i = blockIdx.y * 4 + wave_index();
  if (i >= n || c >= ncols) return;
  const double* row = Ainv + static_cast<int64_t>(i) * lda;
  double acc = 0.0;
  for (int j = lane; j < n; j += kWave) acc += row[j] * B[static_cast<int64_t>(j) * ldb + c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) X[i * ldx + c] = acc;
}

// ----------------------------------------------------------------------------
// Cooperative sequential stepper (the GPU sequential baseline): one grid of
// co-resident work-groups advances U[:, s] = Phi(U[:, s-1]) step after step
// with Jacobi-PCG spread over all work-groups.  Rows are distributed over the
// grid's threads; a CG iteration is two phases separated by grid barriers
// (A: p = D^{-1} r + beta p' with neighbours formed on the fly, q = A p,
// partials of p.q;  B: x += alpha p, r -= alpha q, partials of r.z, r.r).
// Reductions: per-block partials, summed by every block in block order.
// The barrier spins a bounded number of times; on timeout it sets an error
// bit and the kernel returns, so a launch always ends.

constexpr unsigned kSpinLimit = 1u << 24;
constexpr int kMaxCoopBlocks = 1024;
constexpr int kFlagStride = 16;   // one 64-byte line per block flag

// Flag barrier: block b publishes its epoch in arrive[b] (its own cache
// line, one release store); block 0 polls every flag with one thread per
// flag (relaxed loads), then publishes the epoch in *release; the other
// blocks poll it (relaxed) and take one acquire fence.  Release/acquire
// operations are kept to one each per block and barrier because each one
// maintains the XCD's L2.  Every wait is bounded.
struct GridBar {
  unsigned* arrive;   // [gridDim.x * kFlagStride], zeroed before the launch
  unsigned* release;  // one word, zeroed before the launch
  int* flags;
};

__device__ bool grid_sync(const GridBar& g, unsigned& epoch) {
  __shared__ int ok;
  ++epoch;
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(g.arrive + blockIdx.x * kFlagStride, epoch, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0) {
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
      unsigned spins = 0;
      while (__hip_atomic_load(g.arrive + b * kFlagStride, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(g.flags + 1, 4);
          ok = 0;
          break;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
      __hip_atomic_store(g.release, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(g.release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicOr(g.flags + 1, 4);
        ok = 0;
        break;
      }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
  }
  __syncthreads();
  return ok != 0;
}

// Sum v over the block (fixed order) and store it at part[blockIdx.x * 8 + q].
__device__ void block_store(double v, double* sh, double* part, int q) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) t += sh[k];
    part[blockIdx.x * 8 + q] = t;
  }
  __syncthreads();
}

// Totals of partial quantities q0 .. q0+NQ-1 over all blocks: thread t
// loads block t's partials, then a fixed butterfly per wave and the waves in
// order.  Every block computes the same bits.
template <int NQ>
__device__ void grid_totals(const double* part, int q0, double (&out)[NQ], double* sh) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += part[b * 8 + q0 + q];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    if (lane == 0) sh[wv * NQ + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double t = 0.0;
    for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) t += sh[k * NQ + q];
    out[q] = t;
  }
  __syncthreads();
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_seq_coop(
    int n, const int* __restrict__ col, const double* __restrict__ a,
    const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
    const double* __restrict__ dinv, const double* __restrict__ F, SourceDev src, double dt,
    int64_t t0, int s_begin, int s_end, double* __restrict__ U, int64_t ldu,
    double* __restrict__ ws, double* __restrict__ part, GridBar bar, double tol, int maxit) {
  __shared__ double sh[16];
  __shared__ double shg[48];
  double* x = ws;
  double* r = ws + n;
  double* pb[2] = {ws + 2 * n, ws + 3 * n};
  double* q = ws + 4 * n;
  const int T = gridDim.x * blockDim.x;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const double tol2 = tol * tol;
  int iters = 0;
  unsigned epoch = 0;
  for (int s = s_begin; s < s_end; ++s) {
    const double t = static_cast<double>(t0 + s) * dt;
    const double amp = source_scale(t, src);
    const double s0 = amp * pwm(t, src, 0), s1 = amp * pwm(t, src, 1), s2 = amp * pwm(t, src, 2);
    double lrz = 0.0, lrr = 0.0, lbb = 0.0;
    for (int i = tid; i < n; i += T) {
      const int* ci = col + static_cast<int64_t>(i) * W;
      double bv = 0.0;
      if (has_mass[i]) {
        const double* mi = mm + static_cast<int64_t>(i) * W;
        for (int k = 0; k < W; ++k) bv += mi[k] * U[ci[k] * ldu + s - 1];
      }
      bv += (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      const double* ai = a + static_cast<int64_t>(i) * W;
      double ax = 0.0;
      for (int k = 0; k < W; ++k) ax += ai[k] * U[ci[k] * ldu + s - 1];
      const double rv = bv - ax;
      x[i] = U[i * ldu + s - 1];
      r[i] = rv;
      lrz += rv * (dinv[i] * rv);
      lrr += rv * rv;
      lbb += bv * bv;
    }
    block_store(lrz, sh, part, 3);
    block_store(lrr, sh, part, 4);
    block_store(lbb, sh, part, 5);
    if (!grid_sync(bar, epoch)) return;
    double tot3[3];
    grid_totals<3>(part, 3, tot3, shg);
    double rz = tot3[0], rr = tot3[1], bb = tot3[2];
    if (bb == 0.0) bb = rr;
    double beta = 0.0;
    int par = 0, it = 0;
    while (rr > tol2 * bb) {
      if (it >= maxit) {
        if (tid == 0) atomicOr(bar.flags + 1, 2);
        return;
      }
      const double* po = pb[par];
      double* pn = pb[par ^ 1];
      double lpq = 0.0;
      for (int i = tid; i < n; i += T) {
        const int* ci = col + static_cast<int64_t>(i) * W;
        const double* ai = a + static_cast<int64_t>(i) * W;
        double qs = 0.0;
        for (int k = 0; k < W; ++k) {
          const int j = ci[k];
          qs += ai[k] * fma(beta, po[j], dinv[j] * r[j]);
        }
        const double pi = fma(beta, po[i], dinv[i] * r[i]);
        pn[i] = pi;
        q[i] = qs;
        lpq += pi * qs;
      }
      block_store(lpq, sh, part, 0);
      if (!grid_sync(bar, epoch)) return;
      double tot1[1];
      grid_totals<1>(part, 0, tot1, shg);
      const double alpha = rz / tot1[0];
      double lz = 0.0;
      lrr = 0.0;
      for (int i = tid; i < n; i += T) {
        x[i] += alpha * pn[i];
        const double rv = r[i] - alpha * q[i];
        r[i] = rv;
        lz += rv * (dinv[i] * rv);
        lrr += rv * rv;
      }
      block_store(lz, sh, part, 1);
      block_store(lrr, sh, part, 2);
      if (!grid_sync(bar, epoch)) return;
      double tot2[2];
      grid_totals<2>(part, 1, tot2, shg);
      const double rzn = tot2[0];
      rr = tot2[1];
      if (!isfinite(rr)) {
        if (tid == 0) atomicOr(bar.flags + 1, 1);
        return;
      }
      beta = rzn / rz;
      rz = rzn;
      par ^= 1;
      ++it;
    }
    iters += it;
    for (int i = tid; i < n; i += T) U[i * ldu + s] = x[i];
    if (!grid_sync(bar, epoch)) return;
  }
  if (tid == 0) atomicAdd(bar.flags + 2, iters);
}

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

// ----------------------------------------------------------------------------
// Launch wrappers.

void launch_elem_geometry(hipStream_t s, int n_tri, const double* xy, const int* tri,
                          double* area, double* grad) {
  hipLaunchKernelGGL(k_elem_geometry, dim3(ceil_div(n_tri, 256)), dim3(256), 0, s, n_tri, xy, tri,
                     area, grad);
  MG_HIP(hipGetLastError());
}

void launch_assemble_linear(hipStream_t s, const DevLevel& L, const int* cptr, const int* contrib,
                            const double* area, const double* grad, const double* nu_e,
                            const double* sigma_e) {
  const int64_t slots = static_cast<int64_t>(L.n) * L.W;
  hipLaunchKernelGGL(k_assemble_linear, dim3(ceil_div(slots, 256)), dim3(256), 0, s, L.n, L.W,
                     1.0 / L.dt, cptr, contrib, area, grad, nu_e, sigma_e, L.a64, L.a32, L.m64);
  MG_HIP(hipGetLastError());
}

void launch_diag_inverse(hipStream_t s, const DevLevel& L, const int* diag_slot) {
  hipLaunchKernelGGL(k_diag_inverse, dim3(ceil_div(L.n, 256)), dim3(256), 0, s, L.n, L.W,
                     diag_slot, L.a64, L.m64, L.dinv64, L.dinv32, L.has_mass);
  MG_HIP(hipGetLastError());
}

void launch_load_vectors(hipStream_t s, const DevLevel& L, const int* cptr, const int* contrib,
                         const int* diag_slot, const double* area, const int* cell_phase,
                         const int* cell_sign) {
  hipLaunchKernelGGL(k_load_vectors, dim3(ceil_div(L.n, 256)), dim3(256), 0, s, L.n, L.W, cptr,
                     contrib, diag_slot, area, cell_phase, cell_sign, L.F);
  MG_HIP(hipGetLastError());
}

void launch_source_table(hipStream_t s, const SourceDev& src, double dt, int ncols,
                         const int64_t* t_list, int64_t t_base, int64_t t_stride, double* table,
                         int64_t ld, const double* amp, const double* dphi) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_source_table, dim3(ceil_div(ncols, 256)), dim3(256), 0, s, src, dt, ncols,
                     t_list, t_base, t_stride, amp, dphi, table, ld);
  MG_HIP(hipGetLastError());
}

void launch_axpby3(hipStream_t s, int n, int ncols, double* out, int64_t ldo, double sx, CView x,
                   double sa, CView a, double sb, CView b) {
  if (n <= 0 || ncols <= 0) return;
  dim3 grid(ceil_div(ncols, kWave), ceil_div(n, 4));
  hipLaunchKernelGGL(k_axpby3, grid, dim3(kBlock), 0, s, n, ncols, out, ldo, sx, x.p, x.ld, sa, a.p,
                     a.ld, sb, b.p, b.ld);
  MG_HIP(hipGetLastError());
}

static int grid_tiles(const PcgWork& w, int ncols, int& ncc) {
  ncc = ceil_div(ncols, kWave);
  return w.nrb * ncc;
}

void launch_colsq(hipStream_t s, PcgWork& w, int n, int ncols, CView X) {
  int ncc;
  const int nb = grid_tiles(w, ncols, ncc);
  hipLaunchKernelGGL(k_colsq, dim3(nb), dim3(kBlock), 0, s, n, ncols, w.nrb, ncc, w.rows_per_block,
                     X.p, X.ld, w.part, w.ld);
  MG_HIP(hipGetLastError());
}

void launch_joule(hipStream_t s, PcgWork& w, const DevLevel& L, int ncols, CView a, CView b) {
  if (ncols <= 0) return;
  int ncc;
  const int nb = grid_tiles(w, ncols, ncc);
  hipLaunchKernelGGL(k_joule, dim3(nb), dim3(kBlock), 0, s, L.n, L.W, L.col, L.m64, L.has_mass, ncols,
                     w.nrb, ncc, w.rows_per_block, a.p, a.ld, b.p, b.ld, w.part, w.ld);
  MG_HIP(hipGetLastError());
}

void launch_transfer(hipStream_t s, const DevTransfer& T, int ncols, CView X, double alpha,
                     double* Y, int64_t ldy, double beta) {
  if (ncols <= 0) return;
  dim3 grid(ceil_div(ncols, kWave), ceil_div(T.n_out, 4));
  switch (T.W) {
    case 2:
      hipLaunchKernelGGL(k_transfer<2>, grid, dim3(kBlock), 0, s, T.n_out, T.col, T.val, ncols, X.p,
                         X.ld, alpha, Y, ldy, beta);
      break;
    case 4:
      hipLaunchKernelGGL(k_transfer<4>, grid, dim3(kBlock), 0, s, T.n_out, T.col, T.val, ncols, X.p,
                         X.ld, alpha, Y, ldy, beta);
      break;
    case 8:
      hipLaunchKernelGGL(k_transfer<8>, grid, dim3(kBlock), 0, s, T.n_out, T.col, T.val, ncols, X.p,
                         X.ld, alpha, Y, ldy, beta);
      break;
    default:
      hipLaunchKernelGGL(k_transfer<16>, grid, dim3(kBlock), 0, s, T.n_out, T.col, T.val, ncols,
                         X.p, X.ld, alpha, Y, ldy, beta);
      break;
  }
  MG_HIP(hipGetLastError());
}

void launch_tm_to_slabs(hipStream_t s, int n, int64_t npts, int m, const double* tm, double* slabs,
                        int64_t ld, int64_t ss, const int* nat) {
  const int64_t cols = (npts + m - 1) / m;
  dim3 grid(ceil_div(cols, 64), ceil_div(n, 64), m);
  hipLaunchKernelGGL(k_tm_to_slabs, grid, dim3(kBlock), 0, s, n, npts, m, tm, slabs, ld, ss, nat);
  MG_HIP(hipGetLastError());
}

void launch_slabs_to_tm(hipStream_t s, int n, int64_t npts, int m, const double* slabs, int64_t ld,
                        int64_t ss, double* tm, const int* nat) {
  const int64_t cols = (npts + m - 1) / m;
  dim3 grid(ceil_div(cols, 64), ceil_div(n, 64), m);
  hipLaunchKernelGGL(k_slabs_to_tm, grid, dim3(kBlock), 0, s, n, npts, m, slabs, ld, ss, tm, nat);
  MG_HIP(hipGetLastError());
}

void launch_cols_to_slabs(hipStream_t s, int n, int64_t npts, int m, const double* src,
                          int64_t lds, double* slabs, int64_t ld, int64_t ss) {
  dim3 grid(ceil_div(npts, 256), n < 4096 ? n : 4096);
  hipLaunchKernelGGL(k_cols_to_slabs, grid, dim3(256), 0, s, n, npts, m, src, lds, slabs, ld, ss);
  MG_HIP(hipGetLastError());
}

void launch_slabs_to_cols(hipStream_t s, int n, int64_t npts, int m, const double* slabs,
                          int64_t ld, int64_t ss, double* dst, int64_t ldd) {
  dim3 grid(ceil_div(npts, 256), n < 4096 ? n : 4096);
  hipLaunchKernelGGL(k_slabs_to_cols, grid, dim3(256), 0, s, n, npts, m, slabs, ld, ss, dst, ldd);
  MG_HIP(hipGetLastError());
}

void launch_ie_rhs_batch(hipStream_t s, const DevLevel& L, int ncols, const double* src, int64_t lds,
                         CView u, double* B, int64_t ld) {
  if (ncols <= 0) return;
  dim3 grid(ceil_div(ncols, kWave), ceil_div(L.n, 4));
  hipLaunchKernelGGL(k_ie_rhs_batch, grid, dim3(kBlock), 0, s, L.n, L.W, ncols, L.col, L.m64,
                     L.has_mass, L.F, src, lds, u.p, u.ld, B, ld);
  MG_HIP(hipGetLastError());
}

void launch_ie_inverse_batch(hipStream_t s, const DevLevel& L, int ncols, const double* src, int64_t lds,
                             CView u, const double* Ainv, int64_t lda, double* B, double* X,
                             int64_t ld) {
  if (ncols <= 0) return;
  dim3 grid(ceil_div(ncols, kWave), ceil_div(L.n, 4));
  hipLaunchKernelGGL(k_ie_rhs_batch, grid, dim3(kBlock), 0, s, L.n, L.W, ncols, L.col, L.m64,
                     L.has_mass, L.F, src, lds, u.p, u.ld, B, ld);
  hipLaunchKernelGGL(k_inv_apply, dim3(ncols, ceil_div(L.n, 4)), dim3(kBlock), 0, s, L.n, ncols, Ainv, lda,
                     B, ld, X, ld);
  MG_HIP(hipGetLastError());
}

int seq_coop_blocks() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  MG_HIP(hipGetDevice(&dev));
  MG_HIP(hipGetDeviceProperties(&prop, dev));
  MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_seq_coop<8>, kBlock, 0));
  const int fit = per_cu * prop.multiProcessorCount;
  int want = 128;
  if (const char* e = std::getenv("MGRIT_COOP_BLOCKS")) want = std::atoi(e);
  if (want < 1) want = 1;
  want = fit < want ? fit : want;
  return want < kMaxCoopBlocks ? want : kMaxCoopBlocks;
}

void launch_seq_coop(hipStream_t s, const DevLevel& L, const SourceDev& src, int s_begin,
                     int s_end, double* U, int64_t ldu, double* ws, double* part,
                     unsigned* bar_state, int* flags, double tol, int maxit, int blocks) {
  if (s_end <= s_begin) return;
  if (L.W != 8) fail(MGRIT_UNSUPPORTED, "cooperative stepper needs rows of width 8");
  GridBar bar{bar_state + kFlagStride, bar_state, flags};
  int64_t t0 = 0;
  int n = L.n;
  const int* col = L.col;
  const double* a = L.a64;
  const double* mm = L.m64;
  const uint8_t* hm = L.has_mass;
  const double* dinv = L.dinv64;
  const double* F = L.F;
  SourceDev sd = src;
  double dt = L.dt;
  void* args[] = {&n, &col, &a, &mm, &hm, &dinv, &F, &sd, &dt, &t0, &s_begin, &s_end,
                  &U, &ldu, &ws, &part, &bar, &tol, &maxit};
  MG_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_seq_coop<8>), dim3(blocks),
                                    dim3(kBlock), args, 0, s));
}

void launch_seq_small(hipStream_t s, const DevLevel& L, const SourceDev& src, int nsteps,
                      int64_t t0, double* U, int64_t ldu, const double* G, int64_t ldg, double* ws,
                      double tol, int maxit, int warm, int* flags) {
  if (nsteps <= 0) return;
  if (L.W == 8) {
    hipLaunchKernelGGL(k_seq_small<8>, dim3(1), dim3(kSeqThreads), 0, s, L.n, L.col, L.a64, L.m64,
                       L.has_mass, L.dinv64, L.F, src, L.dt, nsteps, t0, U, ldu, G, ldg, ws, tol,
                       maxit, warm, flags);
  } else {
    hipLaunchKernelGGL(k_seq_small<16>, dim3(1), dim3(kSeqThreads), 0, s, L.n, L.col, L.a64,
                       L.m64, L.has_mass, L.dinv64, L.F, src, L.dt, nsteps, t0, U, ldu, G, ldg, ws,
                       tol, maxit, warm, flags);
  }
  MG_HIP(hipGetLastError());
}

}  // namespace mg
