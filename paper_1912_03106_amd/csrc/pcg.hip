// Batched Jacobi-preconditioned CG for the one-step propagator Phi.
//
// Every column of a column block [n][ld] is an independent linear system
// (M/dt + K) x = (M/dt) u_prev + f(t) with the same matrix: the columns are
// the time intervals of an F- or C-relaxation sweep.  CG runs on the
// symmetrically scaled system  A^ = S A S,  S = diag(A)^{-1/2}, whose
// iterates are those of Jacobi-PCG on A (same Krylov space, same stopping
// residual); the scaling removes the preconditioner from the inner loop.
// Vectors r^ (scaled residual) and p^ (scaled direction) live in the scaled
// space, x stays in the original one (x += alpha S p^).
//
// One iteration = two passes over the column block, each containing one
// product with A^, plus two small per-column reductions:
//   pass A: p^ = r^ + beta p^_old (own rows stored into a second buffer),
//           partials of p^.(A^ p^), the neighbours' p^ formed on the fly;
//   pass B: q^ = A^ p^ (recomputed), x += alpha S p^, r^ -= alpha q^,
//           partials of r^.r^ and ||r||^2 = sum_i diag_i r^_i^2.
// 8 vector passes per iteration (r, p_old read + p written; p, x, r read +
// x, r written) instead of 11 for the textbook split.
//
// Mapping: a wave owns CPL x 64 consecutive columns of one row at a time
// (CPL = columns per lane, 1 or 2); the row's pattern and values are
// wave-uniform scalar loads.  A work-group (4 waves) covers `rpb` rows of one
// column chunk; chunks are pinned to XCDs when their count allows.  Both
// knobs are chosen per level by the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace mg {
namespace {

__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

// Work-group -> (row block, column chunk): contiguous tile ranges per XCD, as
// in kernels.hip.
__device__ __forceinline__ void tile_decode(int w, int ncc, int& rb, int& cc) {
  const int nrb_ = static_cast<int>(gridDim.x) / ncc;
  const int T = static_cast<int>(gridDim.x);   // = row blocks x chunks
  const int x = w & 7, k = w >> 3, q = T >> 3, rem = T & 7;
  const int tile = x * q + (x < rem ? x : rem) + k;
  cc = tile / nrb_;
  rb = tile - cc * nrb_;
}

template <typename T, int CPL>
struct Vec;
template <typename T>
struct Vec<T, 1> {
  T v[1];
  __device__ __forceinline__ static Vec load(const T* p) { return Vec{{p[0]}}; }
  __device__ __forceinline__ void store(T* p) const { p[0] = v[0]; }
};
template <>
struct Vec<double, 2> {
  double v[2];
  __device__ __forceinline__ static Vec load(const double* p) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    return Vec{{t.x, t.y}};
  }
  __device__ __forceinline__ void store(double* p) const {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  }
};
template <>
struct Vec<float, 2> {
  float v[2];
  __device__ __forceinline__ static Vec load(const float* p) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    return Vec{{t.x, t.y}};
  }
  __device__ __forceinline__ void store(float* p) const {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  }
};

// Sum the per-column values of the 4 waves in a fixed order and store them
// at out[q * qstride + c] for the columns of this work-group's chunk.
template <int NQ, int CPL>
__device__ __forceinline__ void block_partials(const double (&v)[NQ][CPL], double* out,
                                               int64_t qstride, int c0, const bool (&on)[CPL]) {
  __shared__ double red[NQ][4][kWave * CPL];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int k = 0; k < CPL; ++k) red[q][wv][lane * CPL + k] = v[q][k];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      if (!on[k]) continue;
      const int l = lane * CPL + k;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        out[q * qstride + c0 + k] = ((red[q][0][l] + red[q][1][l]) + red[q][2][l]) + red[q][3][l];
    }
  }
}

// r = b - A x with b = (M/dt) u_in + f(t) (original scaling, FP64);
// stores r^ = S r; partials r^.r^, r.r, b.b.  Block 0 clears the
// active-column counter for the reduce that follows.
template <int W>
__global__ __launch_bounds__(kBlock) void k_cg_init(
    int n, const int* __restrict__ col, const double* __restrict__ a,
    const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
    const double* __restrict__ sc, const double* __restrict__ F, int ncols, int ncc, int rpb,
    const double* __restrict__ uin, int64_t ldu, const double* __restrict__ src, int64_t ld,
    const double* __restrict__ x, double* __restrict__ r, double* __restrict__ part,
    int nrb, int* __restrict__ flags) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  bool on[1] = {c < ncols};
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (on[0]) { s0 = src[c]; s1 = src[ld + c]; s2 = src[2 * ld + c]; }
  double acc[3][1] = {{0.0}, {0.0}, {0.0}};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on[0]) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      double bv = 0.0;
      if (has_mass[i]) {
        const double* mi = mm + static_cast<int64_t>(i) * W;
#pragma unroll
        for (int t = 0; t < W; ++t) bv += mi[t] * uin[ci[t] * ldu + c];
      }
      bv += (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      const double* ai = a + static_cast<int64_t>(i) * W;
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < W; ++t) ax += ai[t] * x[ci[t] * ld + c];
      const double rv = bv - ax;
      const double rh = sc[i] * rv;
      r[i * ld + c] = rh;
      acc[0][0] += rh * rh;
      acc[1][0] += rv * rv;
      acc[2][0] += bv * bv;
    }
  }
  block_partials<3, 1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Pass A.  first != 0: p^ = r^ (beta and p_old unused).  Block 0 records the
// number of columns this iteration works on (the count left by the previous
// reduce) in hist[flags[4]] and advances flags[4].
template <typename T, int W, int CPL>
__global__ __launch_bounds__(kBlock) void k_cg_pass_a(
    int n, const int* __restrict__ col, const T* __restrict__ ah, int ncols, int ncc, int rpb,
    int64_t ld, const uint8_t* __restrict__ active, const double* __restrict__ beta, int first,
    const T* __restrict__ r, const T* __restrict__ pold, T* __restrict__ pnew,
    double* __restrict__ part, int nrb, int* __restrict__ flags, int* __restrict__ hist) {
  using V = Vec<T, CPL>;
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int it = flags[4];
    hist[it] = flags[0];
    flags[4] = it + 1;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c0 = (cc * kWave + lane) * CPL;
  bool on[CPL];
  bool any = false;
  T be[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    on[k] = (c0 + k < ncols) && active[c0 + k];
    any |= on[k];
    be[k] = (first || !on[k]) ? T(0) : static_cast<T>(beta[c0 + k]);
  }
  double acc[1][CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[0][k] = 0.0;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (any) {
    for (int kk = 0; kk < rpw; ++kk) {
      const int i = i0 + kk;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      const T* ai = ah + static_cast<int64_t>(i) * W;
      T s[CPL];
#pragma unroll
      for (int k = 0; k < CPL; ++k) s[k] = T(0);
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const int64_t o = ci[t] * ld + c0;
        const V rv = V::load(r + o);
        if (first) {
#pragma unroll
          for (int k = 0; k < CPL; ++k) s[k] += ai[t] * rv.v[k];
        } else {
          const V pv = V::load(pold + o);
#pragma unroll
          for (int k = 0; k < CPL; ++k) s[k] += ai[t] * fma(be[k], pv.v[k], rv.v[k]);
        }
      }
      const int64_t o = i * ld + c0;
      V pi = V::load(r + o);
      if (!first) {
        const V pv = V::load(pold + o);
#pragma unroll
        for (int k = 0; k < CPL; ++k) pi.v[k] = fma(be[k], pv.v[k], pi.v[k]);
      }
      pi.store(pnew + o);
#pragma unroll
      for (int k = 0; k < CPL; ++k) acc[0][k] += static_cast<double>(pi.v[k]) * static_cast<double>(s[k]);
    }
  }
  block_partials<1, CPL>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c0, on);
}

// Pass B: q^ = A^ p^, x += alpha S p^, r^ -= alpha q^ (columns that are not
// active are left untouched), partials r^.r^ and sum diag_i r^_i^2.
template <typename T, int W, int CPL>
__global__ __launch_bounds__(kBlock) void k_cg_pass_b(
    int n, const int* __restrict__ col, const T* __restrict__ ah, const T* __restrict__ sc,
    const double* __restrict__ dg, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ active, const double* __restrict__ alpha, const T* __restrict__ p,
    T* __restrict__ x, T* __restrict__ r, double* __restrict__ part, int nrb) {
  using V = Vec<T, CPL>;
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c0 = (cc * kWave + lane) * CPL;
  bool on[CPL];
  bool any = false, all = true;
  T al[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    on[k] = (c0 + k < ncols) && active[c0 + k];
    any |= on[k];
    all &= on[k];
    al[k] = on[k] ? static_cast<T>(alpha[c0 + k]) : T(0);
  }
  double acc[2][CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[0][k] = acc[1][k] = 0.0;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (any) {
    for (int kk = 0; kk < rpw; ++kk) {
      const int i = i0 + kk;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      const T* ai = ah + static_cast<int64_t>(i) * W;
      T q[CPL];
#pragma unroll
      for (int k = 0; k < CPL; ++k) q[k] = T(0);
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const V pv = V::load(p + ci[t] * ld + c0);
#pragma unroll
        for (int k = 0; k < CPL; ++k) q[k] += ai[t] * pv.v[k];
      }
      const int64_t o = i * ld + c0;
      const T si = sc[i];
      const double di = dg[i];
      const V pi = V::load(p + o);
      V xi = V::load(x + o);
      V ri = V::load(r + o);
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        xi.v[k] = fma(al[k] * si, pi.v[k], xi.v[k]);
        ri.v[k] = ri.v[k] - al[k] * q[k];
        const double rd = static_cast<double>(ri.v[k]);
        acc[0][k] += rd * rd;
        acc[1][k] += di * (rd * rd);
      }
      if (all) {
        xi.store(x + o);
        ri.store(r + o);
      } else {
#pragma unroll
        for (int k = 0; k < CPL; ++k)
          if (on[k]) {
            x[o + k] = xi.v[k];
            r[o + k] = ri.v[k];
          }
      }
    }
  }
  block_partials<2, CPL>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c0, on);
}

// ---------------------------------------------------------------------------
// Diagonal-window variants.  When every row's entries sit at the offsets
// {-(R+1), -R, -1, 0, +1, +R, +R+1} (mod n) -- the P1 operator of a periodic
// polar mesh numbered angle-major, R = radial unknowns per ray -- the
// values are stored per offset (dv[i][8], slot order as listed, slot 7 = 0)
// and a wave walking consecutive rows keeps three sliding windows in
// registers: (i-R-1, i-R), (i-1, i, i+1), (i+R, i+R+1).  Moving to the next
// row loads three new rows instead of seven.

__device__ __forceinline__ int wrap_index(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

template <typename T, int CPL>
struct PDir {
  // p^ = r^ + beta p^_old formed while loading (first: p^ = r^)
  const T* r;
  const T* pold;
  int64_t ld;
  int c0;
  bool first;
  T be[CPL];
  __device__ __forceinline__ Vec<T, CPL> load(int row) const {
    const int64_t o = row * ld + c0;
    Vec<T, CPL> v = Vec<T, CPL>::load(r + o);
    if (!first) {
      const Vec<T, CPL> q = Vec<T, CPL>::load(pold + o);
#pragma unroll
      for (int k = 0; k < CPL; ++k) v.v[k] = fma(be[k], q.v[k], v.v[k]);
    }
    return v;
  }
};

// The three new window rows of a row (and the row's own streams) are loaded
// D rows ahead into a ring of D register slots, so that a wave walking rpw
// rows keeps D rows of loads in flight instead of waiting for one row's loads
// per row; the arithmetic of a row, and its order, do not depend on D.

// Pass A needs p^.A^p^ only, and A^ is symmetric: with the upper offsets
// o = +1, +R, +R+1 (mod n) every off-diagonal pair is met once, from its
// lower row, so
//   p^.A^p^ = sum_i p_i (a_ii p_i + 2 (a_i,i+1 p_i+1 + a_i,i+R p_i+R + a_i,i+R+1 p_i+R+1))
// and a wave's window is the rows i, i+1, i+R, i+R+1: two new rows per row.
template <typename T, int CPL, int D>
__global__ __launch_bounds__(kBlock) void k_cg_pass_a_dia(
    int n, int R, const T* __restrict__ dv, int ncols, int ncc, int rpb, int64_t ld,
    const uint8_t* __restrict__ active, const double* __restrict__ beta, int first,
    const T* __restrict__ r, const T* __restrict__ pold, T* __restrict__ pnew,
    double* __restrict__ part, int nrb, int* __restrict__ flags, int* __restrict__ hist) {
  using V = Vec<T, CPL>;
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int it = flags[4];
    hist[it] = flags[0];
    flags[4] = it + 1;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c0 = (cc * kWave + lane) * CPL;
  bool on[CPL];
  bool any = false;
  PDir<T, CPL> P{r, pold, ld, c0, first != 0, {}};
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    on[k] = (c0 + k < ncols) && active[c0 + k];
    any |= on[k];
    P.be[k] = (first || !on[k]) ? T(0) : static_cast<T>(beta[c0 + k]);
  }
  double acc[1][CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[0][k] = 0.0;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (any && i0 < n) {
    const int iend = (i0 + rpw < n) ? i0 + rpw : n;
    // slot d holds, for a row j = d (mod D), the r^ and p^_old values of the
    // rows j+1 and j+R+1 (index 0, 1)
    V sr[D][2], sp[D][2];
    auto fill = [&](int d, int j) {
      const int rows[2] = {wrap_index(j + 1, n), wrap_index(j + R + 1, n)};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t o = rows[e] * ld + c0;
        sr[d][e] = V::load(r + o);
        if (!P.first) sp[d][e] = V::load(pold + o);
      }
    };
    auto take = [&](int d, int e) {
      V v = sr[d][e];
      if (!P.first) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) v.v[k] = fma(P.be[k], sp[d][e].v[k], v.v[k]);
      }
      return v;
    };
    V m1 = P.load(i0), hi0 = P.load(wrap_index(i0 + R, n));
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (i0 + d < iend) fill(d, i0 + d);
    for (int ib = i0; ib < iend; ib += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = ib + d;
        if (i < iend) {
          const V m2 = take(d, 0), hi1 = take(d, 1);
          if (i + D < iend) fill(d, i + D);
          const T* a = dv + static_cast<int64_t>(i) * 8;
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const T up = a[4] * m2.v[k] + a[5] * hi0.v[k] + a[6] * hi1.v[k];
            const T s = a[3] * m1.v[k] + T(2) * up;
            acc[0][k] += static_cast<double>(m1.v[k]) * static_cast<double>(s);
          }
          m1.store(pnew + i * ld + c0);
          m1 = m2;
          hi0 = hi1;
        }
      }
    }
  }
  block_partials<1, CPL>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c0, on);
}

template <typename T, int CPL, int D>
__global__ __launch_bounds__(kBlock) void k_cg_pass_b_dia(
    int n, int R, const T* __restrict__ dv, const T* __restrict__ sc, const double* __restrict__ dg,
    int ncols, int ncc, int rpb, int64_t ld, const uint8_t* __restrict__ active,
    const double* __restrict__ alpha, const T* __restrict__ p, T* __restrict__ x,
    T* __restrict__ r, double* __restrict__ part, int nrb) {
  using V = Vec<T, CPL>;
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c0 = (cc * kWave + lane) * CPL;
  bool on[CPL];
  bool any = false, all = true;
  T al[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    on[k] = (c0 + k < ncols) && active[c0 + k];
    any |= on[k];
    all &= on[k];
    al[k] = on[k] ? static_cast<T>(alpha[c0 + k]) : T(0);
  }
  double acc[2][CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[0][k] = acc[1][k] = 0.0;
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  auto ld_p = [&](int row) { return V::load(p + row * ld + c0); };
  if (any && i0 < n) {
    const int iend = (i0 + rpw < n) ? i0 + rpw : n;
    // slot d holds, for a row j = d (mod D), p^ of the rows j-R, j+1, j+R+1
    // and x, r^ of row j
    V sl[D], sm[D], sh[D], sx[D], sr[D];
    auto fill = [&](int d, int j) {
      sl[d] = ld_p(wrap_index(j - R, n));
      sm[d] = ld_p(wrap_index(j + 1, n));
      sh[d] = ld_p(wrap_index(j + R + 1, n));
      sx[d] = V::load(x + j * ld + c0);
      sr[d] = V::load(r + j * ld + c0);
    };
    V lo0 = ld_p(wrap_index(i0 - R - 1, n)), m0 = ld_p(wrap_index(i0 - 1, n));
    V m1 = ld_p(i0), hi0 = ld_p(wrap_index(i0 + R, n));
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (i0 + d < iend) fill(d, i0 + d);
    for (int ib = i0; ib < iend; ib += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = ib + d;
        if (i < iend) {
          const V lo1 = sl[d], m2 = sm[d], hi1 = sh[d];
          V xi = sx[d], ri = sr[d];
          // the stores of row i go to other addresses than the loads of row i + D
          if (i + D < iend) fill(d, i + D);
          const T* a = dv + static_cast<int64_t>(i) * 8;
          const int64_t o = i * ld + c0;
          const T si = sc[i];
          const double di = dg[i];
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const T q = a[0] * lo0.v[k] + a[1] * lo1.v[k] + a[2] * m0.v[k] + a[3] * m1.v[k] +
                        a[4] * m2.v[k] + a[5] * hi0.v[k] + a[6] * hi1.v[k];
            xi.v[k] = fma(al[k] * si, m1.v[k], xi.v[k]);
            ri.v[k] = ri.v[k] - al[k] * q;
            const double rd = static_cast<double>(ri.v[k]);
            acc[0][k] += rd * rd;
            acc[1][k] += di * (rd * rd);
          }
          if (all) {
            xi.store(x + o);
            ri.store(r + o);
          } else {
#pragma unroll
            for (int k = 0; k < CPL; ++k)
              if (on[k]) {
                x[o + k] = xi.v[k];
                r[o + k] = ri.v[k];
              }
          }
          lo0 = lo1;
          m0 = m1;
          m1 = m2;
          hi0 = hi1;
        }
      }
    }
  }
  block_partials<2, CPL>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c0, on);
}

// CG start on the periodic polar stencil: b = (M/dt) u_in + f (original
// scaling) and r^ = S (b - A x) = S b - A^ (S^-1 x), with A^ by offset and the
// window rows of S^-1 x (rows i-R-1 .. i+R+1) kept in registers while a wave
// walks its rows (three new rows per row); partials r^.r^, r.r, b.b as in
// k_cg_init.  The mass term gathers u_in only on the conductor rows.
template <int W>
__global__ __launch_bounds__(kBlock) void k_cg_init_dia(
    int n, int R, const double* __restrict__ dv, const int* __restrict__ col,
    const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
    const double* __restrict__ sc, const double* __restrict__ F, int ncols, int ncc, int rpb,
    const double* __restrict__ uin, int64_t ldu, const double* __restrict__ src, int64_t ld,
    const double* __restrict__ x, double* __restrict__ r, double* __restrict__ part,
    int nrb, int* __restrict__ flags) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  bool on[1] = {c < ncols};
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (on[0]) { s0 = src[c]; s1 = src[ld + c]; s2 = src[2 * ld + c]; }
  double acc[3][1] = {{0.0}, {0.0}, {0.0}};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on[0] && i0 < n) {
    const int iend = (i0 + rpw < n) ? i0 + rpw : n;
    auto xs = [&](int row) { return x[static_cast<int64_t>(row) * ld + c] / sc[row]; };
    double lo0 = xs(wrap_index(i0 - R - 1, n)), m0 = xs(wrap_index(i0 - 1, n));
    double m1 = xs(i0), hi0 = xs(wrap_index(i0 + R, n));
    for (int i = i0; i < iend; ++i) {
      const double lo1 = xs(wrap_index(i - R, n)), m2 = xs(wrap_index(i + 1, n));
      const double hi1 = xs(wrap_index(i + R + 1, n));
      double bv = 0.0;
      if (has_mass[i]) {
        const int* ci = col + static_cast<int64_t>(i) * W;
        const double* mi = mm + static_cast<int64_t>(i) * W;
#pragma unroll
        for (int t = 0; t < W; ++t) bv += mi[t] * uin[ci[t] * ldu + c];
      }
      bv += (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      const double* a = dv + static_cast<int64_t>(i) * 8;
      const double ax = a[0] * lo0 + a[1] * lo1 + a[2] * m0 + a[3] * m1 + a[4] * m2 + a[5] * hi0 +
                        a[6] * hi1;
      const double si = sc[i];
      const double rh = si * bv - ax;
      r[static_cast<int64_t>(i) * ld + c] = rh;
      const double rv = rh / si;
      acc[0][0] += rh * rh;
      acc[1][0] += rv * rv;
      acc[2][0] += bv * bv;
      lo0 = lo1;
      m0 = m1;
      m1 = m2;
      hi0 = hi1;
    }
  }
  block_partials<3, 1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Scatter the scaled operator into the per-offset layout; flags[0] counts
// entries whose offset is not one of the seven (then the layout is unusable).
__global__ void k_build_dia(int n, int W, int R, const int* __restrict__ col,
                            const double* __restrict__ ah, double* __restrict__ dv64,
                            float* __restrict__ dv32, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int nbad = 0;
  for (int t = 0; t < W; ++t) {
    const double a = ah[static_cast<int64_t>(i) * W + t];
    int off = col[static_cast<int64_t>(i) * W + t] - i;
    if (off > n / 2) off -= n;
    if (off < -(n / 2)) off += n;
    int slot = -1;
    if (off == -R - 1) slot = 0;
    else if (off == -R) slot = 1;
    else if (off == -1) slot = 2;
    else if (off == 0) slot = 3;
    else if (off == 1) slot = 4;
    else if (off == R) slot = 5;
    else if (off == R + 1) slot = 6;
    if (slot < 0) {
      if (a != 0.0) ++nbad;
      continue;
    }
    v[slot] += a;
  }
  for (int t = 0; t < 8; ++t) {
    dv64[static_cast<int64_t>(i) * 8 + t] = v[t];
    dv32[static_cast<int64_t>(i) * 8 + t] = static_cast<float>(v[t]);
  }
  if (nbad) atomicAdd(bad, nbad);
}

// CG start for A x = e_(j0 + c) (columns of the inverse), x = 0:
// r^ = S e, partials r^.r^, r.r = 1, b.b = 1.
__global__ __launch_bounds__(kBlock) void k_cg_init_identity(
    int n, int j0, const double* __restrict__ sc, int ncols, int ncc, int rpb, int64_t ld,
    double* __restrict__ x, double* __restrict__ r, double* __restrict__ part, int nrb,
    int* __restrict__ flags) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  bool on[1] = {c < ncols};
  double acc[3][1] = {{0.0}, {0.0}, {0.0}};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on[0]) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const double rv = (i == j0 + c) ? 1.0 : 0.0;
      const double rh = sc[i] * rv;
      x[i * ld + c] = 0.0;
      r[i * ld + c] = rh;
      acc[0][0] += rh * rh;
      acc[1][0] += rv * rv;
      acc[2][0] += rv * rv;
    }
  }
  block_partials<3, 1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Refinement sweep, FP64 part: r = b - A x (FP64) for the columns that have
// not reached the outer tolerance; the FP32 inner solve starts from
// r^32 = float(S r) with correction d = 0.  Partials: r^32.r^32 (inner
// start), r.r and b.b (outer test).
template <int W>
__global__ __launch_bounds__(kBlock) void k_ir_residual(
    int n, const int* __restrict__ col, const double* __restrict__ a,
    const double* __restrict__ mm, const uint8_t* __restrict__ has_mass,
    const double* __restrict__ sc, const double* __restrict__ F, int ncols, int ncc, int rpb,
    const double* __restrict__ uin, int64_t ldu, const double* __restrict__ src, int64_t ld,
    const uint8_t* __restrict__ outer, const double* __restrict__ x, float* __restrict__ r32,
    float* __restrict__ d32, double* __restrict__ part, int nrb, int* __restrict__ flags) {
  int rb, cc;
  tile_decode(blockIdx.x, ncc, rb, cc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[4] = 0;
  }
  const int lane = threadIdx.x & 63, wv = wave_index();
  const int c = cc * kWave + lane;
  bool on[1] = {c < ncols && outer[c]};
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (on[0]) { s0 = src[c]; s1 = src[ld + c]; s2 = src[2 * ld + c]; }
  double acc[3][1] = {{0.0}, {0.0}, {0.0}};
  const int rpw = rpb >> 2;
  const int i0 = rb * rpb + wv * rpw;
  if (on[0]) {
    for (int k = 0; k < rpw; ++k) {
      const int i = i0 + k;
      if (i >= n) break;
      const int* ci = col + static_cast<int64_t>(i) * W;
      double bv = 0.0;
      if (has_mass[i]) {
        const double* mi = mm + static_cast<int64_t>(i) * W;
#pragma unroll
        for (int t = 0; t < W; ++t) bv += mi[t] * uin[ci[t] * ldu + c];
      }
      bv += (s0 * F[i] + s1 * F[n + i]) + s2 * F[2 * n + i];
      const double* ai = a + static_cast<int64_t>(i) * W;
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < W; ++t) ax += ai[t] * x[ci[t] * ld + c];
      const double rv = bv - ax;
      const float rf = static_cast<float>(sc[i] * rv);
      r32[i * ld + c] = rf;
      d32[i * ld + c] = 0.0f;
      const double rd = static_cast<double>(rf);
      acc[0][0] += rd * rd;
      acc[1][0] += rv * rv;
      acc[2][0] += bv * bv;
    }
  }
  block_partials<3, 1>(acc, part + rb * ld, static_cast<int64_t>(nrb) * ld, c, on);
}

// Refinement sweep, FP64 update: x += d for the columns of the sweep.
__global__ __launch_bounds__(kBlock) void k_ir_update(int n, int ncols, int ncc, int rpb, int64_t ld,
                                                      const uint8_t* __restrict__ outer,
                                                      const float* __restrict__ d32,
                                                      double* __restrict__ x) {
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
    x[i * ld + c] += static_cast<double>(d32[i * ld + c]);
  }
}

// Per-column reduction of the row-block partials, in a fixed order, followed
// by the CG scalar updates.  One wave per column (4 columns per work-group):
// lane l sums row blocks l, l+64, ... in order, then a fixed butterfly.
//   INIT:    rz, rr, bb; active = rr > tol2 bb (bb = 0: relative to rr)
//   ALPHA:   alpha = rz / p.Ap (0 for columns that are not active)
//   BETA:    beta = rz_new / rz, convergence test (beta = 0 once converged)
//   SUM:     plain sums into sums_out
//   IR_INIT: outer test on the FP64 residual; inner start (rz, reference rr)
__global__ __launch_bounds__(kBlock) void k_reduce(int ncols, int nrb, int64_t ld, int mode,
                                                   int nq, double tol2, double eta2,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ scal,
                                                   uint8_t* __restrict__ active,
                                                   int* __restrict__ flags,
                                                   double* __restrict__ sums_out,
                                                   uint8_t* __restrict__ outer) {
  __shared__ int cnt;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wv;
  if (threadIdx.x == 0) cnt = 0;
  if (mode == RED_ALPHA && blockIdx.x == 0 && threadIdx.x == 0) flags[0] = 0;
  __syncthreads();
  bool on = c < ncols;
  if (on && (mode == RED_ALPHA || mode == RED_BETA)) on = active[c] != 0;
  if (on && (mode == RED_IR_INIT || mode == RED_IR_FIRST)) on = outer[c] != 0;
  double T[3] = {0.0, 0.0, 0.0};
  if (on) {
    const int64_t qs = static_cast<int64_t>(nrb) * ld;
    for (int rb = lane; rb < nrb; rb += kWave)
      for (int q = 0; q < nq; ++q) T[q] += part[q * qs + rb * ld + c];
    for (int q = 0; q < nq; ++q)
      for (int off = 32; off > 0; off >>= 1) T[q] += __shfl_xor(T[q], off, 64);
  }
  if (lane == 0 && c < ncols) {
    double* rz = scal;
    double* rr = scal + ld;
    double* bb = scal + 2 * ld;
    double* al = scal + 3 * ld;
    double* be = scal + 4 * ld;
    double* thr = scal + 6 * ld;       // outer stopping threshold (refinement)
    int act = 0;
    bool bad = false;
    if (mode == RED_INIT) {
      double b2 = T[2];
      if (b2 == 0.0) b2 = T[1];
      if (eta2 > 0.0) b2 = fmax(b2, (eta2 / tol2) * T[1]);
      rz[c] = T[0];
      rr[c] = T[1];
      bb[c] = b2;
      al[c] = 0.0;
      be[c] = 0.0;
      act = T[1] > tol2 * b2;
      active[c] = static_cast<uint8_t>(act);
      bad = !isfinite(T[0]) || !isfinite(T[1]) || !isfinite(T[2]);
    } else if (mode == RED_ALPHA) {
      double a = 0.0;
      if (on) {
        a = rz[c] / T[0];
        bad = !isfinite(a);
        if (bad) a = 0.0;
      }
      al[c] = a;
    } else if (mode == RED_BETA) {
      double b = 0.0;
      if (on) {
        b = T[0] / rz[c];
        rz[c] = T[0];
        rr[c] = T[1];
        act = T[1] > tol2 * bb[c];
        active[c] = static_cast<uint8_t>(act);
        bad = !isfinite(b) || !isfinite(T[1]);
        if (!act || bad) b = 0.0;
      }
      be[c] = b;
    } else if (mode == RED_IR_INIT || mode == RED_IR_FIRST) {
      if (on) {
        if (mode == RED_IR_FIRST) {
          double b2 = T[2];
          if (b2 == 0.0) b2 = T[1];
          thr[c] = fmax(tol2 * b2, eta2 * T[1]);
        }
        act = T[1] > thr[c];           // outer (FP64) convergence test
        outer[c] = static_cast<uint8_t>(act);
        rz[c] = T[0];
        rr[c] = T[1];
        bb[c] = T[1];                  // inner tolerance is relative to this residual
        bad = !isfinite(T[0]) || !isfinite(T[1]) || !isfinite(T[2]);
      }
      al[c] = 0.0;
      be[c] = 0.0;
      active[c] = static_cast<uint8_t>(act);
    } else {
      sums_out[c] = T[0];
      bad = !isfinite(T[0]);
    }
    if (bad) atomicOr(flags + 1, 1);
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt > 0 &&
      (mode == RED_INIT || mode == RED_BETA || mode == RED_IR_INIT || mode == RED_IR_FIRST))
    atomicAdd(flags, cnt);
}

// A^ = S A S, S = diag(A)^{-1/2}, and the diagonal itself.
__global__ void k_scale_matrix(int n, int W, const int* __restrict__ col,
                               const double* __restrict__ a, const int* __restrict__ diag_slot,
                               double* __restrict__ s64, float* __restrict__ s32,
                               double* __restrict__ d64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = a[static_cast<int64_t>(i) * W + diag_slot[i]];
  d64[i] = d;
  s64[i] = 1.0 / sqrt(d);
  s32[i] = static_cast<float>(1.0 / sqrt(d));
}

__global__ void k_scale_entries(int n, int W, const int* __restrict__ col,
                                const double* __restrict__ a, const double* __restrict__ s64,
                                double* __restrict__ ah64, float* __restrict__ ah32) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * W) return;
  const int i = static_cast<int>(e / W);
  const double v = s64[i] * a[e] * s64[col[e]];
  ah64[e] = v;
  ah32[e] = static_cast<float>(v);
}

// --- column compaction ------------------------------------------------------

template <typename T>
__global__ void k_compact_retire(int n, int cur, int64_t ld, const uint8_t* __restrict__ active,
                                 const int* __restrict__ gmap, int first, int all_cols,
                                 const T* __restrict__ x, T* __restrict__ ox) {
  const int c = blockIdx.x * kWave + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= cur || i >= n) return;
  if (!all_cols && active[c]) return;
  const int g = first ? c : gmap[c];
  ox[i * ld + g] = x[i * ld + c];
}

// Serial (one thread, cur <= a few thousand): deterministic and in place, as
// cmap[j] >= j makes the forward copies safe.
// One work-group: the iterating columns keep their order and move to the
// front, with their CG scalars (rz, rr, bb, beta) and original column ids;
// cmap[j] = the old position of new column j.  In place, chunk by chunk: a
// column's new position j never exceeds its old one c, positions of chunk
// t + 1 are all >= every target of chunk t, and within a chunk every value is
// read before any is written.
constexpr int kCompactThreads = 1024;
__global__ __launch_bounds__(kCompactThreads) void k_compact_map(
    int cur, int64_t ld, int first, uint8_t* __restrict__ active, int* __restrict__ cmap,
    int* __restrict__ gmap, double* __restrict__ scal) {
  constexpr int kWaves = kCompactThreads / kWave;
  __shared__ int wsum[kWaves];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int base = 0;
  for (int c0 = 0; c0 < cur; c0 += kCompactThreads) {
    const int c = c0 + t;
    const bool on = (c < cur) && active[c];
    const unsigned long long bal = __ballot(on);
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int off = base, total = 0;
    for (int k = 0; k < kWaves; ++k) {
      if (k < wv) off += wsum[k];
      total += wsum[k];
    }
    const int j = off + __popcll(bal & ((1ull << lane) - 1ull));
    int g = 0;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v4 = 0.0;
    if (on) {
      g = first ? c : gmap[c];
      v0 = scal[c];            // rz
      v1 = scal[ld + c];       // rr
      v2 = scal[2 * ld + c];   // bb (stopping threshold)
      v4 = scal[4 * ld + c];   // beta
    }
    __syncthreads();
    if (on) {
      cmap[j] = c;
      gmap[j] = g;
      scal[j] = v0;
      scal[ld + j] = v1;
      scal[2 * ld + j] = v2;
      scal[4 * ld + j] = v4;
    }
    base += total;
    __syncthreads();
  }
  for (int k = t; k < cur; k += kCompactThreads) active[k] = k < base ? 1 : 0;
}

template <typename T>
__global__ void k_compact_gather(int n, int count, int64_t ld, const int* __restrict__ cmap,
                                 const T* __restrict__ x, const T* __restrict__ r,
                                 const T* __restrict__ p, T* __restrict__ xd, T* __restrict__ rd,
                                 T* __restrict__ pd) {
  const int j = blockIdx.x * kWave + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (j >= count || i >= n) return;
  const int64_t src = i * ld + cmap[j], dst = i * ld + j;
  xd[dst] = x[src];
  rd[dst] = r[src];
  pd[dst] = p[src];
}

__global__ void k_fill_u8(uint8_t* p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

// ----------------------------------------------------------------------------
// Launch wrappers.

static int grid_tiles(const PcgWork& w, int ncols, int cpl, int& ncc) {
  ncc = ceil_div(ncols, kWave * cpl);
  return w.nrb * ncc;
}

void launch_scale_matrix(hipStream_t s, DevLevel& L, const int* diag_slot) {
  hipLaunchKernelGGL(k_scale_matrix, dim3(ceil_div(L.n, 256)), dim3(256), 0, s, L.n, L.W, L.col,
                     L.a64, diag_slot, L.s64, L.s32, L.d64);
  const int64_t e = static_cast<int64_t>(L.n) * L.W;
  hipLaunchKernelGGL(k_scale_entries, dim3(ceil_div(e, 256)), dim3(256), 0, s, L.n, L.W, L.col,
                     L.a64, L.s64, L.ah64, L.ah32);
  MG_HIP(hipGetLastError());
}

void launch_compact_retire(hipStream_t s, int n, int cur, int ld, bool fp32, const uint8_t* active,
                           const int* gmap, bool first, bool all_cols, const void* x, void* orig_x) {
  dim3 grid(ceil_div(cur, kWave), ceil_div(n, 4));
  if (fp32)
    hipLaunchKernelGGL(k_compact_retire<float>, grid, dim3(kBlock), 0, s, n, cur, static_cast<int64_t>(ld),
                       active, gmap, first ? 1 : 0, all_cols ? 1 : 0, static_cast<const float*>(x),
                       static_cast<float*>(orig_x));
  else
    hipLaunchKernelGGL(k_compact_retire<double>, grid, dim3(kBlock), 0, s, n, cur, static_cast<int64_t>(ld),
                       active, gmap, first ? 1 : 0, all_cols ? 1 : 0, static_cast<const double*>(x),
                       static_cast<double*>(orig_x));
  MG_HIP(hipGetLastError());
}

void launch_compact_map(hipStream_t s, int cur, int64_t ld, bool first, uint8_t* active, int* cmap,
                        int* gmap, double* scal) {
  hipLaunchKernelGGL(k_compact_map, dim3(1), dim3(kCompactThreads), 0, s, cur, ld, first ? 1 : 0, active, cmap, gmap,
                     scal);
  MG_HIP(hipGetLastError());
}

void launch_compact_gather(hipStream_t s, int n, int count, int64_t ld, bool fp32, const int* cmap,
                           const void* x, const void* r, const void* p, void* xd, void* rd, void* pd) {
  if (count <= 0) return;
  dim3 grid(ceil_div(count, kWave), ceil_div(n, 4));
  if (fp32)
    hipLaunchKernelGGL(k_compact_gather<float>, grid, dim3(kBlock), 0, s, n, count, ld, cmap,
                       static_cast<const float*>(x), static_cast<const float*>(r),
                       static_cast<const float*>(p), static_cast<float*>(xd), static_cast<float*>(rd),
                       static_cast<float*>(pd));
  else
    hipLaunchKernelGGL(k_compact_gather<double>, grid, dim3(kBlock), 0, s, n, count, ld, cmap,
                       static_cast<const double*>(x), static_cast<const double*>(r),
                       static_cast<const double*>(p), static_cast<double*>(xd), static_cast<double*>(rd),
                       static_cast<double*>(pd));
  MG_HIP(hipGetLastError());
}

void launch_fill_u8(hipStream_t s, uint8_t* p, int n, uint8_t v) {
  hipLaunchKernelGGL(k_fill_u8, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, n, v);
  MG_HIP(hipGetLastError());
}

void launch_pcg_init(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, CView u_in) {
  int ncc;
  const int nb = grid_tiles(w, ncols, 1, ncc);
  if (w.dia && L.dia_R > 0) {
    auto kd = (L.W == 8) ? k_cg_init_dia<8> : k_cg_init_dia<16>;
    hipLaunchKernelGGL(kd, dim3(nb), dim3(kBlock), 0, s, L.n, L.dia_R, L.dv64, L.col, L.m64, L.has_mass,
                       L.s64, L.F, ncols, ncc, w.rows_per_block, u_in.p, u_in.ld, w.src, w.ld, w.x, w.r,
                       w.part, w.nrb, w.flags);
    MG_HIP(hipGetLastError());
    return;
  }
  auto k = (L.W == 8) ? k_cg_init<8> : k_cg_init<16>;
  hipLaunchKernelGGL(k, dim3(nb), dim3(kBlock), 0, s, L.n, L.col, L.a64, L.m64, L.has_mass, L.s64,
                     L.F, ncols, ncc, w.rows_per_block, u_in.p, u_in.ld, w.src, w.ld, w.x, w.r,
                     w.part, w.nrb, w.flags);
  MG_HIP(hipGetLastError());
}

void launch_cg_init_identity(hipStream_t s, const DevLevel& L, PcgWork& w, int j0, int ncols) {
  int ncc;
  const int nb = grid_tiles(w, ncols, 1, ncc);
  hipLaunchKernelGGL(k_cg_init_identity, dim3(nb), dim3(kBlock), 0, s, L.n, j0, L.s64, ncols, ncc,
                     w.rows_per_block, w.ld, w.x, w.r, w.part, w.nrb, w.flags);
  MG_HIP(hipGetLastError());
}

void launch_reduce(hipStream_t s, PcgWork& w, int ncols, int mode, double tol2, int nq,
                   double* sums_out, double eta2) {
  hipLaunchKernelGGL(k_reduce, dim3(ceil_div(ncols, 4)), dim3(kBlock), 0, s, ncols, w.nrb, w.ld,
                     mode, nq, tol2, eta2, w.part, w.scal, w.active, w.flags, sums_out, w.outer);
  MG_HIP(hipGetLastError());
}

template <typename T, int W, int CPL>
static void pass_a_impl(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first,
                        const T* ah, const T* r, T* pold, T* pnew) {
  int ncc;
  const int nb = grid_tiles(w, ncols, CPL, ncc);
  hipLaunchKernelGGL((k_cg_pass_a<T, W, CPL>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, ah, ncols,
                     ncc, w.rows_per_block, w.ld, w.active, w.scal + 4 * w.ld, first, r, pold, pnew,
                     w.part, w.nrb, w.flags, w.hist);
}

template <typename T, int W, int CPL>
static void pass_b_impl(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, const T* ah,
                        const T* sc, const T* p, T* x, T* r) {
  int ncc;
  const int nb = grid_tiles(w, ncols, CPL, ncc);
  hipLaunchKernelGGL((k_cg_pass_b<T, W, CPL>), dim3(nb), dim3(kBlock), 0, s, L.n, L.col, ah, sc,
                     L.d64, ncols, ncc, w.rows_per_block, w.ld, w.active, w.scal + 3 * w.ld, p, x,
                     r, w.part, w.nrb);
}

template <typename T, int CPL, int D>
static void pass_a_dia_d(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first,
                         const T* dv, const T* r, T* pold, T* pnew) {
  int ncc;
  const int nb = grid_tiles(w, ncols, CPL, ncc);
  hipLaunchKernelGGL((k_cg_pass_a_dia<T, CPL, D>), dim3(nb), dim3(kBlock), 0, s, L.n, L.dia_R, dv,
                     ncols, ncc, w.rows_per_block, w.ld, w.active, w.scal + 4 * w.ld, first, r, pold,
                     pnew, w.part, w.nrb, w.flags, w.hist);
}

template <typename T, int CPL>
static void pass_a_dia(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first,
                       const T* dv, const T* r, T* pold, T* pnew) {
  if (w.depth >= 4) pass_a_dia_d<T, CPL, 4>(s, L, w, ncols, first, dv, r, pold, pnew);
  else if (w.depth == 2) pass_a_dia_d<T, CPL, 2>(s, L, w, ncols, first, dv, r, pold, pnew);
  else pass_a_dia_d<T, CPL, 1>(s, L, w, ncols, first, dv, r, pold, pnew);
}

template <typename T, int CPL, int D>
static void pass_b_dia_d(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, const T* dv,
                         const T* sc, const T* p, T* x, T* r) {
  int ncc;
  const int nb = grid_tiles(w, ncols, CPL, ncc);
  hipLaunchKernelGGL((k_cg_pass_b_dia<T, CPL, D>), dim3(nb), dim3(kBlock), 0, s, L.n, L.dia_R, dv,
                     sc, L.d64, ncols, ncc, w.rows_per_block, w.ld, w.active, w.scal + 3 * w.ld, p,
                     x, r, w.part, w.nrb);
}

template <typename T, int CPL>
static void pass_b_dia(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, const T* dv,
                       const T* sc, const T* p, T* x, T* r) {
  if (w.depth >= 4) pass_b_dia_d<T, CPL, 4>(s, L, w, ncols, dv, sc, p, x, r);
  else if (w.depth == 2) pass_b_dia_d<T, CPL, 2>(s, L, w, ncols, dv, sc, p, x, r);
  else pass_b_dia_d<T, CPL, 1>(s, L, w, ncols, dv, sc, p, x, r);
}

void launch_build_dia(hipStream_t s, DevLevel& L, int* bad) {
  hipLaunchKernelGGL(k_build_dia, dim3(ceil_div(L.n, 256)), dim3(256), 0, s, L.n, L.W, L.dia_R,
                     L.col, L.ah64, L.dv64, L.dv32, bad);
  MG_HIP(hipGetLastError());
}

void launch_pcg_pass_a(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first) {
  double* pold = w.pbuf[w.parity];
  double* pnew = w.pbuf[w.parity ^ 1];
  if (w.dia) {
    if (w.cpl == 2) pass_a_dia<double, 2>(s, L, w, ncols, first, L.dv64, w.r, pold, pnew);
    else pass_a_dia<double, 1>(s, L, w, ncols, first, L.dv64, w.r, pold, pnew);
  } else if (L.W == 8) {
    if (w.cpl == 2) pass_a_impl<double, 8, 2>(s, L, w, ncols, first, L.ah64, w.r, pold, pnew);
    else pass_a_impl<double, 8, 1>(s, L, w, ncols, first, L.ah64, w.r, pold, pnew);
  } else {
    pass_a_impl<double, 16, 1>(s, L, w, ncols, first, L.ah64, w.r, pold, pnew);
  }
  w.parity ^= 1;
  MG_HIP(hipGetLastError());
}

void launch_pcg_pass_b(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols) {
  const double* p = w.pbuf[w.parity];
  if (w.dia) {
    if (w.cpl == 2) pass_b_dia<double, 2>(s, L, w, ncols, L.dv64, L.s64, p, w.x, w.r);
    else pass_b_dia<double, 1>(s, L, w, ncols, L.dv64, L.s64, p, w.x, w.r);
  } else if (L.W == 8) {
    if (w.cpl == 2) pass_b_impl<double, 8, 2>(s, L, w, ncols, L.ah64, L.s64, p, w.x, w.r);
    else pass_b_impl<double, 8, 1>(s, L, w, ncols, L.ah64, L.s64, p, w.x, w.r);
  } else {
    pass_b_impl<double, 16, 1>(s, L, w, ncols, L.ah64, L.s64, p, w.x, w.r);
  }
  MG_HIP(hipGetLastError());
}

void launch_pcg_pass_a32(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first) {
  float* pold = w.p32[w.parity];
  float* pnew = w.p32[w.parity ^ 1];
  if (w.dia) {
    if (w.cpl == 2) pass_a_dia<float, 2>(s, L, w, ncols, first, L.dv32, w.r32, pold, pnew);
    else pass_a_dia<float, 1>(s, L, w, ncols, first, L.dv32, w.r32, pold, pnew);
  } else if (L.W == 8) {
    if (w.cpl == 2) pass_a_impl<float, 8, 2>(s, L, w, ncols, first, L.ah32, w.r32, pold, pnew);
    else pass_a_impl<float, 8, 1>(s, L, w, ncols, first, L.ah32, w.r32, pold, pnew);
  } else {
    pass_a_impl<float, 16, 1>(s, L, w, ncols, first, L.ah32, w.r32, pold, pnew);
  }
  w.parity ^= 1;
  MG_HIP(hipGetLastError());
}

void launch_pcg_pass_b32(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols) {
  const float* p = w.p32[w.parity];
  if (w.dia) {
    if (w.cpl == 2) pass_b_dia<float, 2>(s, L, w, ncols, L.dv32, L.s32, p, w.x32, w.r32);
    else pass_b_dia<float, 1>(s, L, w, ncols, L.dv32, L.s32, p, w.x32, w.r32);
  } else if (L.W == 8) {
    if (w.cpl == 2) pass_b_impl<float, 8, 2>(s, L, w, ncols, L.ah32, L.s32, p, w.x32, w.r32);
    else pass_b_impl<float, 8, 1>(s, L, w, ncols, L.ah32, L.s32, p, w.x32, w.r32);
  } else {
    pass_b_impl<float, 16, 1>(s, L, w, ncols, L.ah32, L.s32, p, w.x32, w.r32);
  }
  MG_HIP(hipGetLastError());
}

void launch_ir_residual(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, CView u_in) {
  int ncc;
  const int nb = grid_tiles(w, ncols, 1, ncc);
  auto k = (L.W == 8) ? k_ir_residual<8> : k_ir_residual<16>;
  hipLaunchKernelGGL(k, dim3(nb), dim3(kBlock), 0, s, L.n, L.col, L.a64, L.m64, L.has_mass, L.s64,
                     L.F, ncols, ncc, w.rows_per_block, u_in.p, u_in.ld, w.src, w.ld, w.outer, w.x,
                     w.r32, w.x32, w.part, w.nrb, w.flags);
  MG_HIP(hipGetLastError());
}

void launch_ir_update(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols) {
  int ncc;
  const int nb = grid_tiles(w, ncols, 1, ncc);
  hipLaunchKernelGGL(k_ir_update, dim3(nb), dim3(kBlock), 0, s, L.n, ncols, ncc, w.rows_per_block,
                     w.ld, w.outer, w.x32, w.x);
  MG_HIP(hipGetLastError());
}

}  // namespace mg
