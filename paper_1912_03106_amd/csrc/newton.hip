// Batched Newton for the saturating-iron model (Sec. 3.1, eq. 7-8 with
// nu = nu(|grad A|^2); damped Newton of the time stepper, Sec. 5).
//
// Every column is an independent nonlinear system
//     R(u) = (M/dt)(u - u_prev) + K(u) u - f(t) = 0,
// K(u) assembled with nu_e = k1 exp(k2 B_e^2) + k3 in iron elements
// (B_e^2 = |grad u_e|^2), the linear nu elsewhere.  Newton step:
//     J(u) d = -R(u),  J = M/dt + sum_e [nu_e G_e + (2 nu'_e / area_e)(G_e u_e)(G_e u_e)^T],
// G_e = area_e grad(phi) grad(phi)^T, nu' = d nu / d(B^2).
// The Jacobian values are per column on the level's shared pattern
// ([n][W][ld], column contiguous), Jacobi-scaled per column, and solved by
// the same two-pass CG as the linear propagator with per-lane matrix values.
//
// Data per column: element fields (nu, nu', grad u) [T][ld]; residual R and
// diag(J) [n][ld] in FP64; scaled Jacobian, scaling and CG vectors in the
// inner precision.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "source_dev.h"

namespace mg {
namespace {

__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

__device__ __forceinline__ void tile_decode(int w, int ncc, int& rb, int& cc) {
  const int nrb_ = static_cast<int>(gridDim.x) / ncc;
  const int T = static_cast<int>(gridDim.x);   // = row blocks x chunks
  const int x = w & 7, k = w >> 3, q = T >> 3, rem = T & 7;
  const int tile = x * q + (x < rem ? x : rem) + k;
  cc = tile / nrb_;
  rb = tile - cc * nrb_;
}

template <int NQ>
__device__ __forceinline__ void block_partials(const double (&v)[NQ], double* out, int64_t qstride,
                                               int c, bool on) {
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

// Element fields of every column: g = grad u_e, nu_e, nu'_e.
// One wave per element (4 per work-group), lanes over columns.
__global__ __launch_bounds__(kBlock) void k_nl_elem(
    int n_tri, const int* __restrict__ tri_u, const double* __restrict__ grad,
    const double* __restrict__ nu_lin, const uint8_t* __restrict__ iron, double k1, double k2,
    double k3, int ncols, int64_t ld, const uint8_t* __restrict__ outer,
    const double* __restrict__ u, int64_t ldu, double* __restrict__ nu_e,
    double* __restrict__ dnu_e, double* __restrict__ gx, double* __restrict__ gy) {
  const int c = blockIdx.x * kWave + (threadIdx.x & 63);
  const int e = blockIdx.y * 4 + wave_index();
  if (e >= n_tri || c >= ncols) return;
  if (outer && !outer[c]) return;
  const int* v = tri_u + 3 * e;
  const double* gr = grad + 6 * e;
  double ux = 0.0, uy = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int vk = v[k];
    const double uk = vk >= 0 ? u[vk * ldu + c] : 0.0;
    ux += uk * gr[2 * k];
    uy += uk * gr[2 * k + 1];
  }
  double nu = nu_lin[e], dnu = 0.0;
  if (iron[e]) {
    const double ex = exp(k2 * (ux * ux + uy * uy));
    nu = k1 * ex + k3;
    dnu = k1 * k2 * ex;
  }
  const int64_t o = static_cast<int64_t>(e) * ld + c;
  nu_e[o] = nu;
  dnu_e[o] = dnu;
  gx[o] = ux;
  gy[o] = uy;
}

// R_i = sum_t (M/dt)_it (u - u_prev)_col(t) + sum_{e at i} nu_e area_e grad(phi_a).g_e - f_i
// (the diagonal entry's contribution list enumerates the elements at node i
// with the node's local index a); partials of R.R.
template <int W>
__global__ __launch_bounds__(kBlock) void k_nl_residual(
    int n, const int* __restrict__ col, const double* __restrict__ mm,
    const uint8_t* __restrict__ has_mass, const double* __restrict__ F,
    const int* __restrict__ cptr, const int* __restrict__ contrib,
    const int* __restrict__ diag_slot, const double* __restrict__ area,
    const double* __restrict__ grad, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ outer, const double* __restrict__ src,
    const double* __restrict__ u, int64_t ldu, const double* __restrict__ uprev, int64_t ldp,
    const double* __restrict__ nu_e, const double* __restrict__ gx,
    const double* __restrict__ gy, double* __restrict__ R, double* __restrict__ part, int nrb) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols && (!outer || outer[c]);
  double acc[1] = {0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on) {
    const double s0 = src[c], s1 = src[ld + c], s2 = src[2 * ld + c];
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      double rv = 0.0;
      if (has_mass[i]) {
        const int* ci = col + static_cast<int64_t>(i) * W;
        const double* mi = mm + static_cast<int64_t>(i) * W;
#pragma unroll
        for (int t = 0; t < W; ++t) {
          const int j = ci[t];
          rv += mi[t] * (u[j * ldu + c] - uprev[j * ldp + c]);
        }
      }
      const int64_t slot = static_cast<int64_t>(i) * W + diag_slot[i];
      for (int q = cptr[slot]; q < cptr[slot + 1]; ++q) {
        const int code = contrib[q];
        const int e = code / 9, a = (code % 9) / 3;
        const int64_t o = static_cast<int64_t>(e) * ld + c;
        rv += nu_e[o] * area[e] * (grad[6 * e + 2 * a] * gx[o] + grad[6 * e + 2 * a + 1] * gy[o]);
      }
      rv -= (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      R[i * ld + c] = rv;
      acc[0] += rv * rv;
    }
  }
  block_partials<1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Jacobian values per column on the shared pattern, and its diagonal.
template <int W, typename T>
__global__ __launch_bounds__(kBlock) void k_nl_jacobian(
    int n, const double* __restrict__ mm, const int* __restrict__ cptr,
    const int* __restrict__ contrib, const int* __restrict__ diag_slot,
    const double* __restrict__ area, const double* __restrict__ grad, int ncols, int ncc, int rpb,
    int64_t ld, const uint8_t* __restrict__ outer, const double* __restrict__ nu_e,
    const double* __restrict__ dnu_e, const double* __restrict__ gx,
    const double* __restrict__ gy, T* __restrict__ J, double* __restrict__ dg) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  if (!(c < ncols && outer[c])) return;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  for (int k = 0; k < rpw; ++k) {
    const int i = i0 + k;
    if (i >= n) break;
    const int ds = diag_slot[i];
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int64_t slot = static_cast<int64_t>(i) * W + t;
      double v = mm[slot];
      for (int q = cptr[slot]; q < cptr[slot + 1]; ++q) {
        const int code = contrib[q];
        const int e = code / 9, a = (code % 9) / 3, b = code % 3;
        const int64_t o = static_cast<int64_t>(e) * ld + c;
        const double* g = grad + 6 * e;
        const double gag = g[2 * a] * gx[o] + g[2 * a + 1] * gy[o];
        const double gbg = g[2 * b] * gx[o] + g[2 * b + 1] * gy[o];
        v += area[e] * (nu_e[o] * (g[2 * a] * g[2 * b] + g[2 * a + 1] * g[2 * b + 1]) +
                        2.0 * dnu_e[o] * gag * gbg);
      }
      J[slot * ld + c] = static_cast<T>(v);
      if (t == ds) dg[i * ld + c] = v;
    }
  }
}

// J^ = S J S with S = diag(J)^{-1/2} per column; stores S.
template <int W, typename T>
__global__ __launch_bounds__(kBlock) void k_nl_scale(int n, const int* __restrict__ col, int ncols,
                                                     int ncc, int rpb, int64_t ld,
                                                     const uint8_t* __restrict__ outer,
                                                     const double* __restrict__ dg,
                                                     T* __restrict__ J, T* __restrict__ sc) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  if (!(c < ncols && outer[c])) return;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  for (int k = 0; k < rpw; ++k) {
    const int i = i0 + k;
    if (i >= n) break;
    const double si = 1.0 / sqrt(dg[i * ld + c]);
    sc[i * ld + c] = static_cast<T>(si);
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int64_t slot = static_cast<int64_t>(i) * W + t;
      const int j = col[slot];
      const double sj = 1.0 / sqrt(dg[j * ld + c]);
      J[slot * ld + c] = static_cast<T>(si * static_cast<double>(J[slot * ld + c]) * sj);
    }
  }
}

// Inner CG start for J d = -R: r^ = S(-R), d = 0; partials r^.r^, ||R||^2,
// ||R||^2 (the inner tolerance is relative to the Newton residual).
// Columns that are not refining contribute zeros (they stay inactive).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nl_cg_init(int n, int ncols, int ncc, int rpb,
                                                       int64_t ld, const uint8_t* __restrict__ outer,
                                                       const double* __restrict__ R,
                                                       const T* __restrict__ sc, T* __restrict__ r,
                                                       T* __restrict__ x, double* __restrict__ part,
                                                       int nrb, int* __restrict__ flags) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols;
  const bool live = on && outer[c];
  double acc[3] = {0.0, 0.0, 0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (live) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const int64_t o = i * ld + c;
      const double rv = -R[o];
      const T rh = static_cast<T>(static_cast<double>(sc[o]) * rv);
      r[o] = rh;
      x[o] = T(0);
      const double rd = static_cast<double>(rh);
      acc[0] += rd * rd;
      acc[1] += rv * rv;
      acc[2] += rv * rv;
    }
  }
  block_partials<3>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Pass A with per-column matrix values J^[i][t][c].
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_cgj_pass_a(
    int n, const int* __restrict__ col, const T* __restrict__ J, int ncols, int ncc, int rpb,
    int64_t ld, const uint8_t* __restrict__ active, const double* __restrict__ beta, int first,
    const T* __restrict__ r, const T* __restrict__ pold, T* __restrict__ pnew,
    double* __restrict__ part, int nrb, int* __restrict__ flags, int* __restrict__ hist) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int it = flags[4];
    hist[it] = flags[0];
    flags[4] = it + 1;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols && active[c];
  double acc[1] = {0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on) {
    const T be = first ? T(0) : static_cast<T>(beta[c]);
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      T s = T(0);
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const int j = ci[t];
        const T a = J[(static_cast<int64_t>(i) * W + t) * ld + c];
        const T pj = first ? r[j * ld + c] : fma(be, pold[j * ld + c], r[j * ld + c]);
        s += a * pj;
      }
      const int64_t o = i * ld + c;
      const T pi = first ? r[o] : fma(be, pold[o], r[o]);
      pnew[o] = pi;
      acc[0] += static_cast<double>(pi) * static_cast<double>(s);
    }
  }
  block_partials<1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Pass B with per-column matrix values; x += alpha S p^, r^ -= alpha J^ p^.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_cgj_pass_b(
    int n, const int* __restrict__ col, const T* __restrict__ J, const T* __restrict__ sc,
    const double* __restrict__ dg, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ active, const double* __restrict__ alpha,
    const T* __restrict__ p, T* __restrict__ x, T* __restrict__ r, double* __restrict__ part,
    int nrb) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols && active[c];
  double acc[2] = {0.0, 0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on) {
    const T al = static_cast<T>(alpha[c]);
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      T q = T(0);
#pragma unroll
      for (int t = 0; t < W; ++t)
        q += J[(static_cast<int64_t>(i) * W + t) * ld + c] * p[ci[t] * ld + c];
      const int64_t o = i * ld + c;
      x[o] = fma(al * sc[o], p[o], x[o]);
      const T rv = r[o] - al * q;
      r[o] = rv;
      const double rd = static_cast<double>(rv);
      acc[0] += rd * rd;
      acc[1] += dg[o] * (rd * rd);
    }
  }
  block_partials<2>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// ---------------------------------------------------------------------------
// Diagonal-window Jacobian (periodic polar stencil, angle-major numbering,
// R radial unknowns per ray).  Only the upper half is stored, by offset:
// Jd[(i*4 + s)*ld + c] for s = 0, 1, 2, 3 <-> offsets 0, +1, +R, +R+1
// (mod n); an offset without a pattern entry holds 0.  The CG passes walk
// consecutive rows per wave with sliding register windows of the direction.

__device__ __forceinline__ int wrap_row(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

// Upper-half Jacobian values per column (unscaled) and diag(J).
template <int W, typename T>
__global__ __launch_bounds__(kBlock) void k_nl_jacobian_dia(
    int n, int R, const int* __restrict__ col, const double* __restrict__ mm,
    const int* __restrict__ cptr, const int* __restrict__ contrib,
    const int* __restrict__ diag_slot, const double* __restrict__ area,
    const double* __restrict__ grad, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ outer, const double* __restrict__ nu_e,
    const double* __restrict__ dnu_e, const double* __restrict__ gx, const double* __restrict__ gy,
    T* __restrict__ Jd, double* __restrict__ dg) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  if (!(c < ncols && outer[c])) return;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  const int offs[4] = {0, 1, R, R + 1};
  for (int k = 0; k < rpw; ++k) {
    const int i = i0 + k;
    if (i >= n) break;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      // the pattern pads short rows with zero entries in the diagonal
      // column: the diagonal is the row's diagonal slot, every other offset
      // appears at most once
      const int j = wrap_row(i + offs[sl], n);
      int t = -1;
      if (sl == 0) {
        t = diag_slot[i];
      } else {
#pragma unroll
        for (int q = 0; q < W; ++q)
          if (t < 0 && col[static_cast<int64_t>(i) * W + q] == j) t = q;
      }
      double v = 0.0;
      if (t >= 0) {
        const int64_t slot = static_cast<int64_t>(i) * W + t;
        v = mm[slot];
        for (int q = cptr[slot]; q < cptr[slot + 1]; ++q) {
          const int code = contrib[q];
          const int e = code / 9, a = (code % 9) / 3, b = code % 3;
          const int64_t o = static_cast<int64_t>(e) * ld + c;
          const double* g = grad + 6 * e;
          const double gag = g[2 * a] * gx[o] + g[2 * a + 1] * gy[o];
          const double gbg = g[2 * b] * gx[o] + g[2 * b + 1] * gy[o];
          v += area[e] * (nu_e[o] * (g[2 * a] * g[2 * b] + g[2 * a + 1] * g[2 * b + 1]) +
                          2.0 * dnu_e[o] * gag * gbg);
        }
      }
      Jd[(static_cast<int64_t>(i) * 4 + sl) * ld + c] = static_cast<T>(v);
      if (sl == 0) dg[i * ld + c] = v;
    }
  }
}

// J^ = S J S on the upper half, S = diag(J)^{-1/2}; stores S.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nl_scale_dia(int n, int R, int ncols, int ncc, int rpb,
                                                         int64_t ld, const uint8_t* __restrict__ outer,
                                                         const double* __restrict__ dg,
                                                         T* __restrict__ Jd, T* __restrict__ sc) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  if (!(c < ncols && outer[c])) return;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  const int offs[4] = {0, 1, R, R + 1};
  for (int k = 0; k < rpw; ++k) {
    const int i = i0 + k;
    if (i >= n) break;
    const double si = 1.0 / sqrt(dg[i * ld + c]);
    sc[i * ld + c] = static_cast<T>(si);
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const double sj = 1.0 / sqrt(dg[wrap_row(i + offs[sl], n) * ld + c]);
      const int64_t o = (static_cast<int64_t>(i) * 4 + sl) * ld + c;
      Jd[o] = static_cast<T>(si * static_cast<double>(Jd[o]) * sj);
    }
  }
}

// Pass A: p^ = r^ + beta p^_old (row i stored), partials of p^.J^p^ from the
// upper half: p_i (J_ii p_i + 2 (J_i,i+1 p_i+1 + J_i,i+R p_i+R + J_i,i+R+1 p_i+R+1)).
// Window rows i, i+1, i+R, i+R+1: two new direction rows per row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgj_pass_a_dia(
    int n, int R, const T* __restrict__ Jd, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ active, const double* __restrict__ beta, int first,
    const T* __restrict__ r, const T* __restrict__ pold, T* __restrict__ pnew,
    double* __restrict__ part, int nrb, int* __restrict__ flags, int* __restrict__ hist) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int it = flags[4];
    hist[it] = flags[0];
    flags[4] = it + 1;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols && active[c];
  double acc[1] = {0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on && i0 < n) {
    const int iend = (i0 + rpw < n) ? i0 + rpw : n;
    const T be = first ? T(0) : static_cast<T>(beta[c]);
    auto dir = [&](int row) {
      const int64_t o = static_cast<int64_t>(row) * ld + c;
      return first ? r[o] : fma(be, pold[o], r[o]);
    };
    T m1 = dir(i0), hi0 = dir(wrap_row(i0 + R, n));
    // unrolled so that the loads of the next rows are issued before this
    // row's arithmetic waits for its own (the walk is latency-bound on narrow
    // batches); the arithmetic and its order are unchanged
#pragma unroll 4
    for (int i = i0; i < iend; ++i) {
      const T m2 = dir(wrap_row(i + 1, n)), hi1 = dir(wrap_row(i + R + 1, n));
      const T* a = Jd + static_cast<int64_t>(i) * 4 * ld + c;
      const T up = a[ld] * m2 + a[2 * ld] * hi0 + a[3 * ld] * hi1;
      const T s = a[0] * m1 + T(2) * up;
      acc[0] += static_cast<double>(m1) * static_cast<double>(s);
      pnew[static_cast<int64_t>(i) * ld + c] = m1;
      m1 = m2;
      hi0 = hi1;
    }
  }
  block_partials<1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Pass B: q^ = J^ p^ from the upper half of row i and the upper entries of
// the rows i-1 (offset +1), i-R (+R) and i-R-1 (+R+1) that reach row i;
// x += alpha S p^, r^ -= alpha q^, partials of r^.r^ and diag(J) r^.r^.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgj_pass_b_dia(
    int n, int R, const T* __restrict__ Jd, const T* __restrict__ sc, const double* __restrict__ dg,
    int ncols, int ncc, int rpb, int64_t ld, const uint8_t* __restrict__ active,
    const double* __restrict__ alpha, const T* __restrict__ p, T* __restrict__ x,
    T* __restrict__ r, double* __restrict__ part, int nrb) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  const bool on = c < ncols && active[c];
  double acc[2] = {0.0, 0.0};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on && i0 < n) {
    const int iend = (i0 + rpw < n) ? i0 + rpw : n;
    const T al = static_cast<T>(alpha[c]);
    auto pv = [&](int row) { return p[static_cast<int64_t>(row) * ld + c]; };
    auto jv = [&](int row, int sl) { return Jd[(static_cast<int64_t>(row) * 4 + sl) * ld + c]; };
    T lo0 = pv(wrap_row(i0 - R - 1, n)), m0 = pv(wrap_row(i0 - 1, n));
    T m1 = pv(i0), hi0 = pv(wrap_row(i0 + R, n));
    T jm = jv(wrap_row(i0 - 1, n), 1);   // J_{i-1,i}
#pragma unroll 4
    for (int i = i0; i < iend; ++i) {
      const T lo1 = pv(wrap_row(i - R, n)), m2 = pv(wrap_row(i + 1, n)), hi1 = pv(wrap_row(i + R + 1, n));
      const T j0 = jv(i, 0), j1 = jv(i, 1), j2 = jv(i, 2), j3 = jv(i, 3);
      const T jl = jv(wrap_row(i - R, n), 2), jll = jv(wrap_row(i - R - 1, n), 3);
      const T q = jll * lo0 + jl * lo1 + jm * m0 + j0 * m1 + j1 * m2 + j2 * hi0 + j3 * hi1;
      const int64_t o = static_cast<int64_t>(i) * ld + c;
      x[o] = fma(al * sc[o], m1, x[o]);
      const T rv = r[o] - al * q;
      r[o] = rv;
      const double rd = static_cast<double>(rv);
      acc[0] += rd * rd;
      acc[1] += dg[o] * (rd * rd);
      lo0 = lo1;
      m0 = m1;
      m1 = m2;
      hi0 = hi1;
      jm = j1;
    }
  }
  block_partials<2>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// u += d for the columns still refining.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nl_update(int n, int ncols, int ncc, int rpb, int64_t ld,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ fac,
                                                      const T* __restrict__ d,
                                                      double* __restrict__ u) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  if (!(c < ncols && mask[c])) return;
  const double f = fac[c];
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  for (int k = 0; k < rpw; ++k) {
    const int i = i0 + k;
    if (i >= n) break;
    u[i * ld + c] += f * static_cast<double>(d[i * ld + c]);
  }
}

// Start of the damped step of every refining column: trial length 1.
__global__ void k_nl_ls_start(int ncols, const uint8_t* __restrict__ outer,
                              uint8_t* __restrict__ ls, double* __restrict__ lam,
                              double* __restrict__ fac, int* __restrict__ flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) flags[3] = 0;
  if (c >= ncols) return;
  ls[c] = outer[c];
  lam[c] = 1.0;
  fac[c] = 1.0;
}

// Step-length test of every searching column (one wave per column; Armijo
// rule on the residual 2-norm, Sec. 5.1 damping): t = ||R(u + lam d)||^2.
// Accept when t < (1 - 1e-4 lam)^2 ||R(u)||^2, or when lam has reached
// lam_min; an accepted column keeps refining while t > tol2 ref.  A rejected
// column moves back to u + (lam/2) d (fac = -lam/2 for the next update).
// flags[0] counts searching columns, flags[3] the refining columns accepted.
__global__ __launch_bounds__(kBlock) void k_nl_ls(int ncols, int nrb, int64_t ld, double tol2,
                                                  double lam_min, const double* __restrict__ part,
                                                  const double* __restrict__ ref,
                                                  double* __restrict__ rcur, double* __restrict__ lam,
                                                  double* __restrict__ fac, uint8_t* __restrict__ ls,
                                                  uint8_t* __restrict__ outer,
                                                  int* __restrict__ flags) {
  __shared__ int cnt[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wv;
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  __syncthreads();
  const bool on = c < ncols && ls[c];
  double t = 0.0;
  if (on) {
    for (int rb = lane; rb < nrb; rb += kWave) t += part[rb * ld + c];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  }
  if (lane == 0 && on) {
    const double l = lam[c];
    const double shrink = 1.0 - 1e-4 * l;
    const bool ok = isfinite(t) && t < shrink * shrink * rcur[c];
    if (ok || l <= lam_min) {
      rcur[c] = t;
      ls[c] = 0;
      const int act = t > tol2 * ref[c];
      outer[c] = static_cast<uint8_t>(act);
      if (!isfinite(t)) atomicOr(flags + 1, 1);
      if (act) atomicAdd(&cnt[1], 1);
    } else {
      fac[c] = -0.5 * l;
      lam[c] = 0.5 * l;
      atomicAdd(&cnt[0], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt[0] > 0) atomicAdd(flags, cnt[0]);
  if (threadIdx.x == 1 && cnt[1] > 0) atomicAdd(flags + 3, cnt[1]);
}

// Newton bookkeeping per column (one wave per column): sums the R.R partials
// and, in REF mode, stores the reference ||R(u_prev)||^2 and marks every
// column as refining; in TEST mode, keeps refining the columns with
// ||R||^2 > tol2 ref.  Counts refining columns into flags[0].
__global__ __launch_bounds__(kBlock) void k_nl_test(int ncols, int nrb, int64_t ld, int ref_mode,
                                                    double tol2, double eta2,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ ref,
                                                    double* __restrict__ rcur,
                                                    uint8_t* __restrict__ outer,
                                                    int* __restrict__ flags) {
  __shared__ int cnt;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wv;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const bool on = c < ncols && (ref_mode || outer[c]);
  double t = 0.0;
  if (on) {
    for (int rb = lane; rb < nrb; rb += kWave) t += part[rb * ld + c];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  }
  if (lane == 0 && c < ncols) {
    int act = 0;
    // eta2 > 0: also stop once ||R||^2 <= eta2 times that of the initial
    // guess (ref is kept as threshold / tol2)
    if (ref_mode) {
      ref[c] = eta2 > 0.0 ? fmax(t, (eta2 / tol2) * t) : t;
      rcur[c] = t;
      act = t > 0.0;
    } else if (on) {
      rcur[c] = t;
      if (eta2 > 0.0) ref[c] = fmax(ref[c], (eta2 / tol2) * t);
      act = t > tol2 * ref[c];
    }
    outer[c] = static_cast<uint8_t>(act);
    if (!isfinite(t)) atomicOr(flags + 1, 1);
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt > 0) atomicAdd(flags, cnt);
}

__global__ void k_zero_flag0(int* flags) { flags[0] = 0; }

// ---------------------------------------------------------------------------
// Persistent single-work-group damped-Newton stepper for small levels (the
// coarsest level's sequential solve u_s = Phi(u_{s-1}) + g_s, and small
// sequential baselines).  One work-group runs every step, every Newton
// iteration, every inner CG iteration and every step-length trial of the
// whole sweep without returning to the host: the same arithmetic as the
// batched Newton (element fields, FP64 residual, Jacobian on the shared
// pattern, symmetric Jacobi scaling, CG to the inner tolerance, Armijo step
// lengths), with the vectors in global memory (L2-resident at these sizes)
// and block reductions in a fixed order.

__device__ double nl_block_sum(double v, double* sh) {
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

struct SeqNewtonArgs {
  int n, W, n_tri;
  const int* col;
  const double* mm;          // M/dt on the pattern
  const uint8_t* has_mass;
  const double* F;           // [3][n]
  const int* tri_u;
  const double* grad;
  const double* area;
  const double* nu_lin;
  const uint8_t* iron;
  const int* cptr;
  const int* contrib;
  const int* diag_slot;
  double k1, k2, k3;
  double dt;
  int nsteps;
  int64_t t0;                // step offset: step s samples the source at (t0 + s) dt
  double* U;                 // column s = point s
  int64_t ldu;
  const double* G;           // FAS right-hand side (or null)
  int64_t ldg;
  int warm;                  // start from U[:, s] - G[:, s] instead of U[:, s-1]
  int add_g;                 // store Phi(u_{s-1}) + g_s (1) or Phi(u_{s-1}) alone (0)
  double tol2;               // (Newton tolerance)^2, relative to ||R(u_prev)||^2
  int newton_max;
  double lam_min;
  double tin2;               // (inner CG tolerance)^2
  int cg_max;
  double* ws;                // workspace, see seq_newton_ws_doubles
  int* flags;                // [1] bits: 1 non-finite, 2 inner CG cap, 8 Newton cap; [2] CG its; [3] Newton its
};

// Element fields of u: gradient, nu, d nu / d B^2.
__device__ void sn_elem(const SeqNewtonArgs& a, const double* u, double* gx, double* gy, double* nu,
                        double* dnu) {
  for (int e = threadIdx.x; e < a.n_tri; e += blockDim.x) {
    const int* v = a.tri_u + 3 * e;
    const double* gr = a.grad + 6 * e;
    double ux = 0.0, uy = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double uk = v[k] >= 0 ? u[v[k]] : 0.0;
      ux += uk * gr[2 * k];
      uy += uk * gr[2 * k + 1];
    }
    double nv = a.nu_lin[e], dv = 0.0;
    if (a.iron[e]) {
      const double ex = exp(a.k2 * (ux * ux + uy * uy));
      nv = a.k1 * ex + a.k3;
      dv = a.k1 * a.k2 * ex;
    }
    gx[e] = ux;
    gy[e] = uy;
    nu[e] = nv;
    dnu[e] = dv;
  }
  __syncthreads();
}

// R = (M/dt)(u - u_prev) + K(u) u - f; returns ||R||^2.
__device__ double sn_residual(const SeqNewtonArgs& a, const double* u, const double* up, double s0,
                              double s1, double s2, const double* gx, const double* gy,
                              const double* nu, double* R, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) {
    double rv = 0.0;
    if (a.has_mass[i]) {
      for (int t = 0; t < a.W; ++t) {
        const int64_t sl = static_cast<int64_t>(i) * a.W + t;
        const int j = a.col[sl];
        rv += a.mm[sl] * (u[j] - up[j]);
      }
    }
    const int64_t slot = static_cast<int64_t>(i) * a.W + a.diag_slot[i];
    for (int q = a.cptr[slot]; q < a.cptr[slot + 1]; ++q) {
      const int code = a.contrib[q];
      const int e = code / 9, al = (code % 9) / 3;
      rv += nu[e] * a.area[e] * (a.grad[6 * e + 2 * al] * gx[e] + a.grad[6 * e + 2 * al + 1] * gy[e]);
    }
    rv -= (s0 * a.F[i] + s1 * a.F[a.n + i]) + s2 * a.F[2 * a.n + i];
    R[i] = rv;
    acc += rv * rv;
  }
  return nl_block_sum(acc, sh);
}

// Workspace of one column: x, xt, u_prev, R, r, p, q, y, S (n each), the
// scaled Jacobian (n W), element fields (4 T).
struct SnBufs {
  double *x, *xt, *up, *R, *r, *p, *q, *y, *sc, *J, *gx, *gy, *nu, *dnu;
};

__device__ SnBufs sn_bufs(const SeqNewtonArgs& a, double* ws) {
  const int n = a.n, T = a.n_tri;
  SnBufs b;
  b.x = ws;
  b.xt = b.x + n;
  b.up = b.xt + n;
  b.R = b.up + n;
  b.r = b.R + n;
  b.p = b.r + n;
  b.q = b.p + n;
  b.y = b.q + n;
  b.sc = b.y + n;
  b.J = b.sc + n;
  b.gx = b.J + static_cast<int64_t>(n) * a.W;
  b.gy = b.gx + T;
  b.nu = b.gy + T;
  b.dnu = b.nu + T;
  return b;
}

// One damped-Newton step of one column by the calling work-group: b.x holds
// the start on entry and the solution on exit, b.up = u_prev, s0..s2 the
// source values at the new time.  Returns the Newton iterations; on failure
// sets the bits of a.flags[1] and *stop (shared).
__device__ int sn_newton(const SeqNewtonArgs& a, const SnBufs& b, double s0, double s1, double s2,
                         double* sh, int* stop, int* cg_its) {
  const int n = a.n, W = a.W;
  double* x = b.x;
  double* xt = b.xt;
  double* up = b.up;
  double* R = b.R;
  double* r = b.r;
  double* p = b.p;
  double* q = b.q;
  double* y = b.y;
  double* sc = b.sc;
  double* J = b.J;
  double *gx = b.gx, *gy = b.gy, *nu = b.nu, *dnu = b.dnu;
  // reference ||R(u_prev)||^2, then the residual of the start
  sn_elem(a, up, gx, gy, nu, dnu);
  const double ref = sn_residual(a, up, up, s0, s1, s2, gx, gy, nu, R, sh);
  sn_elem(a, x, gx, gy, nu, dnu);
  double rcur = sn_residual(a, x, up, s0, s1, s2, gx, gy, nu, R, sh);
  if (!isfinite(rcur) || !isfinite(ref)) {
    if (threadIdx.x == 0) { atomicOr(a.flags + 1, 1); *stop = 1; }
  }
  __syncthreads();
  if (*stop) return 0;
  int k = 0;
  while (rcur > a.tol2 * ref) {
    if (k >= a.newton_max) {
      if (threadIdx.x == 0) { atomicOr(a.flags + 1, 8); *stop = 1; }
      break;
    }
    ++k;
    // Jacobian at x (element fields of x are current), diag, scaling
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      for (int t = 0; t < W; ++t) {
        const int64_t slot = static_cast<int64_t>(i) * W + t;
        double v = a.mm[slot];
        for (int qq = a.cptr[slot]; qq < a.cptr[slot + 1]; ++qq) {
          const int code = a.contrib[qq];
          const int e = code / 9, al = (code % 9) / 3, bl = code % 3;
          const double* g = a.grad + 6 * e;
          const double gag = g[2 * al] * gx[e] + g[2 * al + 1] * gy[e];
          const double gbg = g[2 * bl] * gx[e] + g[2 * bl + 1] * gy[e];
          v += a.area[e] * (nu[e] * (g[2 * al] * g[2 * bl] + g[2 * al + 1] * g[2 * bl + 1]) +
                            2.0 * dnu[e] * gag * gbg);
        }
        J[slot] = v;
        if (t == a.diag_slot[i]) sc[i] = 1.0 / sqrt(v);
      }
    }
    __syncthreads();
    // J^ = S J S; CG on J^ y = S (-R), y = 0
    double lrr = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double si = sc[i];
      for (int t = 0; t < W; ++t) {
        const int64_t slot = static_cast<int64_t>(i) * W + t;
        J[slot] = si * J[slot] * sc[a.col[slot]];
      }
      const double rv = -si * R[i];
      r[i] = rv;
      p[i] = rv;
      y[i] = 0.0;
      lrr += rv * rv;
    }
    double rr = nl_block_sum(lrr, sh);
    const double rr0 = rr;
    int it = 0;
    while (rr > a.tin2 * rr0) {
      if (it >= a.cg_max) {
        if (threadIdx.x == 0) { atomicOr(a.flags + 1, 2); *stop = 1; }
        break;
      }
      double lpq = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double sq = 0.0;
        for (int t = 0; t < W; ++t) {
          const int64_t slot = static_cast<int64_t>(i) * W + t;
          sq += J[slot] * p[a.col[slot]];
        }
        q[i] = sq;
        lpq += p[i] * sq;
      }
      const double pq = nl_block_sum(lpq, sh);
      const double al = rr / pq;
      double lr = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        y[i] += al * p[i];
        const double rv = r[i] - al * q[i];
        r[i] = rv;
        lr += rv * rv;
      }
      const double rrn = nl_block_sum(lr, sh);
      if (!isfinite(rrn)) {
        if (threadIdx.x == 0) { atomicOr(a.flags + 1, 1); *stop = 1; }
        break;
      }
      const double be = rrn / rr;
      rr = rrn;
      for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + be * p[i];
      __syncthreads();
      ++it;
    }
    *cg_its += it;
    __syncthreads();
    if (*stop) break;
    // damped update: the first lambda in 1, 1/2, ... with
    // ||R(x + lambda d)|| < (1 - 1e-4 lambda) ||R(x)||, else lam_min
    double lam = 1.0;
    while (true) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) xt[i] = x[i] + lam * (sc[i] * y[i]);
      __syncthreads();
      sn_elem(a, xt, gx, gy, nu, dnu);
      const double t = sn_residual(a, xt, up, s0, s1, s2, gx, gy, nu, R, sh);
      const double shrink = 1.0 - 1e-4 * lam;
      const bool ok = isfinite(t) && t < shrink * shrink * rcur;
      if (ok || lam <= a.lam_min) {
        if (!isfinite(t)) {
          if (threadIdx.x == 0) { atomicOr(a.flags + 1, 1); *stop = 1; }
        }
        rcur = t;
        break;
      }
      lam *= 0.5;
    }
    __syncthreads();
    if (*stop) break;
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = xt[i];
    __syncthreads();
    // the element fields and R now belong to x
  }
  __syncthreads();
  return k;
}

__global__ __launch_bounds__(kSeqThreads) void k_seq_newton(SeqNewtonArgs a, SourceDev src) {
  __shared__ double sh[32];
  __shared__ double sgn[3];
  __shared__ int stop;
  if (threadIdx.x == 0) stop = 0;
  const int n = a.n;
  const SnBufs b = sn_bufs(a, a.ws);
  int cg_total = 0, newton_total = 0;
  for (int s = 1; s <= a.nsteps; ++s) {
    if (threadIdx.x == 0) {
      const double t = static_cast<double>(a.t0 + s) * a.dt;
      const double amp = source_scale(t, src);
      for (int k = 0; k < 3; ++k) sgn[k] = amp * pwm(t, src, k);
    }
    __syncthreads();
    const double s0 = sgn[0], s1 = sgn[1], s2 = sgn[2];
    // u_prev and the start as contiguous vectors
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double g = a.warm ? a.U[i * a.ldu + s] : a.U[i * a.ldu + s - 1];
      if (a.warm && a.G) g -= a.G[i * a.ldg + s];
      b.x[i] = g;
      b.up[i] = a.U[i * a.ldu + s - 1];
    }
    __syncthreads();
    newton_total += sn_newton(a, b, s0, s1, s2, sh, &stop, &cg_total);
    if (stop) break;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double v = b.x[i];
      if (a.G && a.add_g) v += a.G[i * a.ldg + s];
      a.U[i * a.ldu + s] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(a.flags + 2, cg_total);
    atomicAdd(a.flags + 3, newton_total);
  }
}

// Narrow batches of independent steps: work-group c takes column c,
// u_prev = uin[:, c], the start and the result in x[:, c], the step from
// t_{i_c} to t_{i_c + 1} with i_c = t_list[c] (or t_base + c t_stride).
__global__ __launch_bounds__(kSeqThreads) void k_seq_newton_batch(SeqNewtonArgs a, SourceDev src,
                                                                  const double* __restrict__ uin,
                                                                  int64_t ldin, double* __restrict__ xio,
                                                                  int64_t ldx,
                                                                  const int64_t* __restrict__ t_list,
                                                                  int64_t t_base, int64_t t_stride,
                                                                  int64_t ws_stride) {
  __shared__ double sh[32];
  __shared__ double sgn[3];
  __shared__ int stop;
  const int c = blockIdx.x;
  if (threadIdx.x == 0) {
    stop = 0;
    const int64_t i_from = t_list ? t_list[c] : t_base + static_cast<int64_t>(c) * t_stride;
    const double t = static_cast<double>(i_from + 1) * a.dt;
    const double amp = source_scale(t, src);
    for (int k = 0; k < 3; ++k) sgn[k] = amp * pwm(t, src, k);
  }
  const int n = a.n;
  const SnBufs b = sn_bufs(a, a.ws + static_cast<int64_t>(c) * ws_stride);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    b.x[i] = xio[static_cast<int64_t>(i) * ldx + c];
    b.up[i] = uin[static_cast<int64_t>(i) * ldin + c];
  }
  __syncthreads();
  int cg = 0;
  const int nk = sn_newton(a, b, sgn[0], sgn[1], sgn[2], sh, &stop, &cg);
  if (!stop)
    for (int i = threadIdx.x; i < n; i += blockDim.x) xio[static_cast<int64_t>(i) * ldx + c] = b.x[i];
  if (threadIdx.x == 0) {
    atomicAdd(a.flags + 2, cg);
    atomicAdd(a.flags + 3, nk);
  }
}

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

int64_t seq_newton_ws_doubles(int n, int W, int n_tri) {
  return 9LL * n + static_cast<int64_t>(n) * W + 4LL * n_tri;
}

static SeqNewtonArgs seq_newton_args(const DevLevel& L, const NlLevel& N, double newton_tol,
                                     int newton_max, double lam_min, double inner_tol, int cg_max,
                                     double* ws, int* flags) {
  SeqNewtonArgs a{};
  a.n = L.n;
  a.W = L.W;
  a.n_tri = N.n_tri;
  a.col = L.col;
  a.mm = L.m64;
  a.has_mass = L.has_mass;
  a.F = L.F;
  a.tri_u = N.tri_u;
  a.grad = N.grad;
  a.area = N.area;
  a.nu_lin = N.nu_lin;
  a.iron = N.iron;
  a.cptr = N.cptr;
  a.contrib = N.contrib;
  a.diag_slot = N.diag;
  a.k1 = N.k1;
  a.k2 = N.k2;
  a.k3 = N.k3;
  a.dt = L.dt;
  a.tol2 = newton_tol * newton_tol;
  a.newton_max = newton_max;
  a.lam_min = lam_min;
  a.tin2 = inner_tol * inner_tol;
  a.cg_max = cg_max;
  a.ws = ws;
  a.flags = flags;
  return a;
}

void launch_seq_newton_batch(hipStream_t s, const DevLevel& L, const NlLevel& N, const SourceDev& src,
                             int ncols, CView uin, double* x, int64_t ldx, const int64_t* t_list,
                             int64_t t_base, int64_t t_stride, double newton_tol, int newton_max,
                             double lam_min, double inner_tol, int cg_max, double* ws, int* flags) {
  if (ncols <= 0) return;
  const SeqNewtonArgs a = seq_newton_args(L, N, newton_tol, newton_max, lam_min, inner_tol, cg_max, ws, flags);
  hipLaunchKernelGGL(k_seq_newton_batch, dim3(ncols), dim3(kSeqThreads), 0, s, a, src, uin.p, uin.ld, x, ldx,
                     t_list, t_base, t_stride, seq_newton_ws_doubles(L.n, L.W, N.n_tri));
  MG_HIP(hipGetLastError());
}

void launch_seq_newton(hipStream_t s, const DevLevel& L, const NlLevel& N, const SourceDev& src,
                       int nsteps, int64_t t0, double* U, int64_t ldu, const double* G, int64_t ldg,
                       int warm, double newton_tol, int newton_max, double lam_min, double inner_tol,
                       int cg_max, double* ws, int* flags, bool add_g) {
  if (nsteps <= 0) return;
  SeqNewtonArgs a = seq_newton_args(L, N, newton_tol, newton_max, lam_min, inner_tol, cg_max, ws, flags);
  a.add_g = add_g ? 1 : 0;
  a.nsteps = nsteps;
  a.t0 = t0;
  a.U = U;
  a.ldu = ldu;
  a.G = G;
  a.ldg = ldg;
  a.warm = warm;
  hipLaunchKernelGGL(k_seq_newton, dim3(1), dim3(kSeqThreads), 0, s, a, src);
  MG_HIP(hipGetLastError());
}

// ----------------------------------------------------------------------------

static int tiles(const PcgWork& w, int ncols, int& ncc) {
  ncc = ceil_div(ncols, kWave);
  return w.nrb * ncc;
}

void launch_nl_elem(hipStream_t s, const NlLevel& N, int ncols, int64_t ld, const uint8_t* outer,
                    CView u, NlWork& nw) {
  dim3 grid(ceil_div(ncols, kWave), ceil_div(N.n_tri, 4));
  hipLaunchKernelGGL(k_nl_elem, grid, dim3(kBlock), 0, s, N.n_tri, N.tri_u, N.grad, N.nu_lin, N.iron,
                     N.k1, N.k2, N.k3, ncols, ld, outer, u.p, u.ld, nw.nu, nw.dnu, nw.gx, nw.gy);
  MG_HIP(hipGetLastError());
}

void launch_nl_residual(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                        int ncols, const uint8_t* outer, CView u, CView uprev) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  auto k = (L.W == 8) ? k_nl_residual<8> : k_nl_residual<16>;
  hipLaunchKernelGGL(k, dim3(nb), dim3(kBlock), 0, s, L.n, L.col, L.m64, L.has_mass, L.F, N.cptr,
                     N.contrib, N.diag, N.area, N.grad, ncols, ncc, w.rows_per_block, w.ld, outer,
                     w.src, u.p, u.ld, uprev.p, uprev.ld, nw.nu, nw.gx, nw.gy, nw.R, w.part, w.nrb);
  MG_HIP(hipGetLastError());
}

void launch_nl_test(hipStream_t s, PcgWork& w, NlWork& nw, int ncols, int ref_mode, double tol2,
                    double eta2) {
  hipLaunchKernelGGL(k_zero_flag0, dim3(1), dim3(1), 0, s, w.flags);
  hipLaunchKernelGGL(k_nl_test, dim3(ceil_div(ncols, 4)), dim3(kBlock), 0, s, ncols, w.nrb, w.ld,
                     ref_mode, tol2, eta2, w.part, nw.ref, nw.rcur, w.outer, w.flags);
  MG_HIP(hipGetLastError());
}

template <typename T>
static void jac_impl(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                     int ncols, T* J, T* sc) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  if (L.W == 8) {
    hipLaunchKernelGGL((k_nl_jacobian<8, T>), dim3(nb), dim3(kBlock), 0, s, L.n, L.m64, N.cptr,
                       N.contrib, N.diag, N.area, N.grad, ncols, ncc, w.rows_per_block, w.ld,
                       w.outer, nw.nu, nw.dnu, nw.gx, nw.gy, J, nw.dg);
    hipLaunchKernelGGL((k_nl_scale<8, T>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, ncols, ncc,
                       w.rows_per_block, w.ld, w.outer, nw.dg, J, sc);
  } else {
    hipLaunchKernelGGL((k_nl_jacobian<16, T>), dim3(nb), dim3(kBlock), 0, s, L.n, L.m64, N.cptr,
                       N.contrib, N.diag, N.area, N.grad, ncols, ncc, w.rows_per_block, w.ld,
                       w.outer, nw.nu, nw.dnu, nw.gx, nw.gy, J, nw.dg);
    hipLaunchKernelGGL((k_nl_scale<16, T>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, ncols, ncc,
                       w.rows_per_block, w.ld, w.outer, nw.dg, J, sc);
  }
  MG_HIP(hipGetLastError());
}

template <typename T>
static void jac_dia_impl(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                         int ncols, T* Jd, T* sc) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  auto k = (L.W == 8) ? k_nl_jacobian_dia<8, T> : k_nl_jacobian_dia<16, T>;
  hipLaunchKernelGGL(k, dim3(nb), dim3(kBlock), 0, s, L.n, nw.dia_R, L.col, L.m64, N.cptr, N.contrib,
                     N.diag, N.area, N.grad, ncols, ncc, w.rows_per_block, w.ld, w.outer, nw.nu, nw.dnu, nw.gx,
                     nw.gy, Jd, nw.dg);
  hipLaunchKernelGGL(k_nl_scale_dia<T>, dim3(nb), dim3(kBlock), 0, s, L.n, nw.dia_R, ncols, ncc,
                     w.rows_per_block, w.ld, w.outer, nw.dg, Jd, sc);
  MG_HIP(hipGetLastError());
}

void launch_nl_jacobian(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                        int ncols) {
  if (nw.dia_R > 0) {
    if (nw.fp32) jac_dia_impl<float>(s, L, N, w, nw, ncols, nw.J32, nw.s32);
    else jac_dia_impl<double>(s, L, N, w, nw, ncols, nw.J64, nw.s64);
    return;
  }
  if (nw.fp32) jac_impl<float>(s, L, N, w, nw, ncols, nw.J32, nw.s32);
  else jac_impl<double>(s, L, N, w, nw, ncols, nw.J64, nw.s64);
}

void launch_nl_cg_init(hipStream_t s, PcgWork& w, NlWork& nw, int ncols) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  if (nw.fp32)
    hipLaunchKernelGGL(k_nl_cg_init<float>, dim3(nb), dim3(kBlock), 0, s, w.n, ncols, ncc,
                       w.rows_per_block, w.ld, w.outer, nw.R, nw.s32, w.r32, w.x32, w.part, w.nrb,
                       w.flags);
  else
    hipLaunchKernelGGL(k_nl_cg_init<double>, dim3(nb), dim3(kBlock), 0, s, w.n, ncols, ncc,
                       w.rows_per_block, w.ld, w.outer, nw.R, nw.s64, nw.r64, nw.d64, w.part,
                       w.nrb, w.flags);
  MG_HIP(hipGetLastError());
}

template <typename T, int W>
static void cgj_a(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first, const T* J,
                  const T* r, T* pold, T* pnew) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  hipLaunchKernelGGL((k_cgj_pass_a<T, W>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, J, ncols, ncc,
                     w.rows_per_block, w.ld, w.active, w.scal + 4 * w.ld, first, r, pold, pnew,
                     w.part, w.nrb, w.flags, w.hist);
}

template <typename T, int W>
static void cgj_b(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols, const T* J,
                  const T* sc, const T* p, T* x, T* r) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  hipLaunchKernelGGL((k_cgj_pass_b<T, W>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, J, sc, nw.dg,
                     ncols, ncc, w.rows_per_block, w.ld, w.active, w.scal + 3 * w.ld, p, x, r,
                     w.part, w.nrb);
}

template <typename T>
static void cgj_a_dia(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols, int first,
                      const T* J, const T* r, T* pold, T* pnew) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  hipLaunchKernelGGL(k_cgj_pass_a_dia<T>, dim3(nb), dim3(kBlock), 0, s, L.n, nw.dia_R, J, ncols, ncc,
                     w.rows_per_block, w.ld, w.active, w.scal + 4 * w.ld, first, r, pold, pnew, w.part,
                     w.nrb, w.flags, w.hist);
}

template <typename T>
static void cgj_b_dia(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols, const T* J,
                      const T* sc, const T* p, T* x, T* r) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  hipLaunchKernelGGL(k_cgj_pass_b_dia<T>, dim3(nb), dim3(kBlock), 0, s, L.n, nw.dia_R, J, sc, nw.dg,
                     ncols, ncc, w.rows_per_block, w.ld, w.active, w.scal + 3 * w.ld, p, x, r, w.part,
                     w.nrb);
}

void launch_nl_pass_a(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols,
                      int first) {
  if (nw.dia_R > 0) {
    if (nw.fp32) cgj_a_dia<float>(s, L, w, nw, ncols, first, nw.J32, w.r32, w.p32[w.parity],
                                  w.p32[w.parity ^ 1]);
    else cgj_a_dia<double>(s, L, w, nw, ncols, first, nw.J64, nw.r64, nw.p64[w.parity],
                           nw.p64[w.parity ^ 1]);
    w.parity ^= 1;
    MG_HIP(hipGetLastError());
    return;
  }
  if (nw.fp32) {
    float* po = w.p32[w.parity];
    float* pn = w.p32[w.parity ^ 1];
    if (L.W == 8) cgj_a<float, 8>(s, L, w, ncols, first, nw.J32, w.r32, po, pn);
    else cgj_a<float, 16>(s, L, w, ncols, first, nw.J32, w.r32, po, pn);
  } else {
    double* po = nw.p64[w.parity];
    double* pn = nw.p64[w.parity ^ 1];
    if (L.W == 8) cgj_a<double, 8>(s, L, w, ncols, first, nw.J64, nw.r64, po, pn);
    else cgj_a<double, 16>(s, L, w, ncols, first, nw.J64, nw.r64, po, pn);
  }
  w.parity ^= 1;
  MG_HIP(hipGetLastError());
}

void launch_nl_pass_b(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols) {
  if (nw.dia_R > 0) {
    if (nw.fp32) cgj_b_dia<float>(s, L, w, nw, ncols, nw.J32, nw.s32, w.p32[w.parity], w.x32, w.r32);
    else cgj_b_dia<double>(s, L, w, nw, ncols, nw.J64, nw.s64, nw.p64[w.parity], nw.d64, nw.r64);
    MG_HIP(hipGetLastError());
    return;
  }
  if (nw.fp32) {
    const float* p = w.p32[w.parity];
    if (L.W == 8) cgj_b<float, 8>(s, L, w, nw, ncols, nw.J32, nw.s32, p, w.x32, w.r32);
    else cgj_b<float, 16>(s, L, w, nw, ncols, nw.J32, nw.s32, p, w.x32, w.r32);
  } else {
    const double* p = nw.p64[w.parity];
    if (L.W == 8) cgj_b<double, 8>(s, L, w, nw, ncols, nw.J64, nw.s64, p, nw.d64, nw.r64);
    else cgj_b<double, 16>(s, L, w, nw, ncols, nw.J64, nw.s64, p, nw.d64, nw.r64);
  }
  MG_HIP(hipGetLastError());
}

void launch_nl_update(hipStream_t s, PcgWork& w, NlWork& nw, int ncols) {
  int ncc;
  const int nb = tiles(w, ncols, ncc);
  if (nw.fp32)
    hipLaunchKernelGGL(k_nl_update<float>, dim3(nb), dim3(kBlock), 0, s, w.n, ncols, ncc,
                       w.rows_per_block, w.ld, nw.ls, nw.fac, w.x32, w.x);
  else
    hipLaunchKernelGGL(k_nl_update<double>, dim3(nb), dim3(kBlock), 0, s, w.n, ncols, ncc,
                       w.rows_per_block, w.ld, nw.ls, nw.fac, nw.d64, w.x);
  MG_HIP(hipGetLastError());
}

void launch_nl_ls_start(hipStream_t s, PcgWork& w, NlWork& nw, int ncols) {
  hipLaunchKernelGGL(k_nl_ls_start, dim3(ceil_div(ncols, kBlock)), dim3(kBlock), 0, s, ncols,
                     w.outer, nw.ls, nw.lam, nw.fac, w.flags);
  MG_HIP(hipGetLastError());
}

void launch_nl_ls(hipStream_t s, PcgWork& w, NlWork& nw, int ncols, double tol2, double lam_min) {
  hipLaunchKernelGGL(k_zero_flag0, dim3(1), dim3(1), 0, s, w.flags);
  hipLaunchKernelGGL(k_nl_ls, dim3(ceil_div(ncols, 4)), dim3(kBlock), 0, s, ncols, w.nrb, w.ld,
                     tol2, lam_min, w.part, nw.ref, nw.rcur, nw.lam, nw.fac, nw.ls, w.outer, w.flags);
  MG_HIP(hipGetLastError());
}

}  // namespace mg
