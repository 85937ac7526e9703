// Learned coarse propagator (gfx950): a 3-layer message-passing network on
// the coarsest mesh that corrects the implicit-Euler coarse step,
//
//     Psi(u) = p + s_out * delta(x),   p = Phi_IE(u),
//
// with inference, training (forward, manual backward, Adam) and the source
// features all computed here.  Rows of every activation array are
// (node i, sample s) pairs, r = i * S + s, with the 64 features of a row
// contiguous ([rows][64], FP32).  Weights are stored as an FP32 master copy
// and used as bfloat16 (round to nearest even); products accumulate in FP32.
//
// Dense layer products run on 64-row tiles: a work-group of 256 threads
// stages the tile (transposed) and the 64 x 64 weight block in LDS and each
// thread accumulates a 4-row x 4-feature block.  Weight gradients are
// per-work-group partial sums reduced in a fixed order (deterministic).

#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "setup.h"
#include "source_dev.h"

namespace mg {

namespace {

constexpr int kH = 64;        // width
constexpr int kTile = 64;     // rows per work-group tile
constexpr int kXS = 68;       // LDS stride of a transposed tile (64 rows + pad)
constexpr int kFP = 32;       // padded input feature count

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(r >> 16);
}

// acc[4 rows][4 features] += Xs^T[k][rows] * Wl[k][features] over k < K.
template <int K>
__device__ __forceinline__ void tile_mm(const float* __restrict__ Xs, const float* __restrict__ Wl,
                                        int rb, int fb, float (&acc)[4][4]) {
#pragma unroll 8
  for (int k = 0; k < K; ++k) {
    const float4 xv = *reinterpret_cast<const float4*>(Xs + k * kXS + rb * 4);
    const float4 wv = *reinterpret_cast<const float4*>(Wl + k * kH + fb * 4);
    const float xa[4] = {xv.x, xv.y, xv.z, xv.w};
    const float wa[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xa[i], wa[j], acc[i][j]);
  }
}

// Stage a [64 rows][64] tile of a row-major array (rows >= nrows read as 0)
// transposed into Xs[k][row].
__device__ __forceinline__ void stage_tile_t(const float* __restrict__ A, int64_t r0, int64_t nrows,
                                             float* __restrict__ Xs) {
  for (int q = threadIdx.x; q < kTile * 16; q += blockDim.x) {
    const int row = q >> 4, k4 = q & 15;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + row < nrows) v = *reinterpret_cast<const float4*>(A + (r0 + row) * kH + k4 * 4);
    Xs[(k4 * 4 + 0) * kXS + row] = v.x;
    Xs[(k4 * 4 + 1) * kXS + row] = v.y;
    Xs[(k4 * 4 + 2) * kXS + row] = v.z;
    Xs[(k4 * 4 + 3) * kXS + row] = v.w;
  }
}

// Stage a bf16 weight block W[k][f] (k < K, 64 columns) as floats, or its
// transpose (Wl[f][k] = W[k][f], K = 64 only).
__device__ __forceinline__ void stage_w(const uint16_t* __restrict__ W, int K, int Kvalid,
                                        bool transpose, float* __restrict__ Wl) {
  for (int e = threadIdx.x; e < K * kH; e += blockDim.x) {
    const int k = e / kH, f = e % kH;
    const float v = (k < Kvalid) ? bf16_to_f32(W[k * kH + f]) : 0.f;
    if (transpose) Wl[f * kH + k] = v;
    else Wl[k * kH + f] = v;
  }
}

// ---------------------------------------------------------------------------
// Source table: tab[(s*(m+1) + j)*3 + p] = amplitude(t) * b_p(t) at
// t = k_s dT + j dT/m, with the sample's amplitude factor and phase shift.
__global__ void k_gnn_srctab(int S, int m, double dT, const int64_t* __restrict__ k_list,
                             int64_t k_base, int64_t k_stride, SourceDev src,
                             const double* __restrict__ amp, const double* __restrict__ dphi,
                             double* __restrict__ tab) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * (m + 1)) return;
  const int s = e / (m + 1), j = e % (m + 1);
  const int64_t k = k_list ? k_list[s] : k_base + static_cast<int64_t>(s) * k_stride;
  const double t = static_cast<double>(k) * dT + static_cast<double>(j) * (dT / m);
  SourceDev sc = src;
  if (amp) sc.scale *= amp[s];
  if (dphi)
    for (int p = 0; p < 3; ++p) sc.phi[p] += dphi[s];
  const double a = source_scale(t, sc);
  for (int p = 0; p < 3; ++p) tab[static_cast<int64_t>(e) * 3 + p] = a * pwm(t, sc, p);
}

// Encoder: features x (FP64 arithmetic, stored FP32) and h0 = tanh(x W_in + b_in).
__global__ __launch_bounds__(kBlock) void k_gnn_encode(
    int n, int S, int m, int F, const double* __restrict__ u, int64_t ldu,
    const double* __restrict__ p, int64_t ldp, const double* __restrict__ tab,
    const double* __restrict__ F3, const float* __restrict__ flags, const float* __restrict__ scales,
    const uint16_t* __restrict__ W_in, const uint16_t* __restrict__ b_in, float* __restrict__ x_out,
    float* __restrict__ h0) {
  __shared__ float Xs[kFP * kXS];
  __shared__ float Wl[kFP * kH];
  const int64_t nrows = static_cast<int64_t>(n) * S;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kTile;
  const double su = scales[0], sf = scales[1];
  for (int e = threadIdx.x; e < kTile * kFP; e += blockDim.x) {
    const int row = e / kFP, f = e % kFP;
    const int64_t r = r0 + row;
    double v = 0.0;
    if (r < nrows && f < F) {
      const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
      if (f == 0) v = u[i * ldu + s] / su;
      else if (f == 1) v = p[i * ldp + s] / su;
      else if (f < m + 3) {
        const double* tb = tab + (static_cast<int64_t>(s) * (m + 1) + (f - 2)) * 3;
        v = ((tb[0] * F3[i] + tb[1] * F3[n + i]) + tb[2] * F3[2 * n + i]) / sf;
      } else {
        v = flags[i * 4 + (f - m - 3)];
      }
    }
    const float fv = static_cast<float>(v);
    Xs[f * kXS + row] = fv;
    if (x_out && r < nrows) x_out[r * kFP + f] = fv;
  }
  stage_w(W_in, kFP, F, false, Wl);
  __syncthreads();
  const int fb = threadIdx.x & 15, rb = threadIdx.x >> 4;
  float acc[4][4] = {};
  tile_mm<kFP>(Xs, Wl, rb, fb, acc);
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + rb * 4 + i;
    if (r >= nrows) continue;
    float4 o;
    o.x = tanhf(acc[i][0] + bf16_to_f32(b_in[fb * 4 + 0]));
    o.y = tanhf(acc[i][1] + bf16_to_f32(b_in[fb * 4 + 1]));
    o.z = tanhf(acc[i][2] + bf16_to_f32(b_in[fb * 4 + 2]));
    o.w = tanhf(acc[i][3] + bf16_to_f32(b_in[fb * 4 + 3]));
    *reinterpret_cast<float4*>(h0 + r * kH + fb * 4) = o;
  }
}

// Message-passing layer: a = mean of neighbour rows, h' = h + tanh(h Ws + a Wn + b).
__global__ __launch_bounds__(kBlock) void k_gnn_layer(
    int n, int S, const int* __restrict__ gptr, const int* __restrict__ gidx,
    const float* __restrict__ hin, const uint16_t* __restrict__ Ws, const uint16_t* __restrict__ Wn,
    const uint16_t* __restrict__ b, float* __restrict__ hout, float* __restrict__ a_out,
    float* __restrict__ t_out) {
  __shared__ float Hs[kH * kXS];
  __shared__ float As[kH * kXS];
  __shared__ float Wl[kH * kH];
  const int64_t nrows = static_cast<int64_t>(n) * S;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kTile;
  stage_tile_t(hin, r0, nrows, Hs);
  for (int q = threadIdx.x; q < kTile * 16; q += blockDim.x) {
    const int row = q >> 4, k4 = q & 15;
    const int64_t r = r0 + row;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < nrows) {
      const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
      const int j0 = gptr[i], j1 = gptr[i + 1];
      for (int jj = j0; jj < j1; ++jj) {
        const float4 v =
            *reinterpret_cast<const float4*>(hin + (static_cast<int64_t>(gidx[jj]) * S + s) * kH + k4 * 4);
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
      }
      const float inv = 1.f / static_cast<float>(j1 - j0);
      acc.x *= inv;
      acc.y *= inv;
      acc.z *= inv;
      acc.w *= inv;
      if (a_out) *reinterpret_cast<float4*>(a_out + r * kH + k4 * 4) = acc;
    }
    As[(k4 * 4 + 0) * kXS + row] = acc.x;
    As[(k4 * 4 + 1) * kXS + row] = acc.y;
    As[(k4 * 4 + 2) * kXS + row] = acc.z;
    As[(k4 * 4 + 3) * kXS + row] = acc.w;
  }
  stage_w(Ws, kH, kH, false, Wl);
  __syncthreads();
  const int fb = threadIdx.x & 15, rb = threadIdx.x >> 4;
  float acc[4][4] = {};
  tile_mm<kH>(Hs, Wl, rb, fb, acc);
  __syncthreads();
  stage_w(Wn, kH, kH, false, Wl);
  __syncthreads();
  tile_mm<kH>(As, Wl, rb, fb, acc);
  for (int i = 0; i < 4; ++i) {
    const int row = rb * 4 + i;
    const int64_t r = r0 + row;
    if (r >= nrows) continue;
    float tv[4], hv[4];
    for (int j = 0; j < 4; ++j) {
      const int f = fb * 4 + j;
      tv[j] = tanhf(acc[i][j] + bf16_to_f32(b[f]));
      hv[j] = Hs[f * kXS + row] + tv[j];
    }
    *reinterpret_cast<float4*>(hout + r * kH + fb * 4) = make_float4(hv[0], hv[1], hv[2], hv[3]);
    if (t_out)
      *reinterpret_cast<float4*>(t_out + r * kH + fb * 4) = make_float4(tv[0], tv[1], tv[2], tv[3]);
  }
}

// Decoder: out(i, s) = p(i, s) + s_out * (h_L w_out + b_out); 16 lanes per row.
__global__ __launch_bounds__(kBlock) void k_gnn_decode(int n, int S, const float* __restrict__ h,
                                                       const uint16_t* __restrict__ w_out,
                                                       const uint16_t* __restrict__ b_out,
                                                       const float* __restrict__ scales,
                                                       const double* __restrict__ p, int64_t ldp,
                                                       double* __restrict__ out, int64_t ldo) {
  const int64_t nrows = static_cast<int64_t>(n) * S;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 16 + (threadIdx.x >> 4);
  const int l = threadIdx.x & 15;
  float d = 0.f;
  if (r < nrows) {
    const float4 v = *reinterpret_cast<const float4*>(h + r * kH + l * 4);
    d = v.x * bf16_to_f32(w_out[l * 4]) + v.y * bf16_to_f32(w_out[l * 4 + 1]) +
        v.z * bf16_to_f32(w_out[l * 4 + 2]) + v.w * bf16_to_f32(w_out[l * 4 + 3]);
  }
  for (int off = 8; off > 0; off >>= 1) d += __shfl_xor(d, off, 16);
  if (r < nrows && l == 0) {
    const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
    const double delta = static_cast<double>(d) + static_cast<double>(bf16_to_f32(b_out[0]));
    out[i * ldo + s] = p[i * ldp + s] + static_cast<double>(scales[2]) * delta;
  }
}

// Loss: d = (psi - y) / s_out; dd = dL/d(delta) = 2 d / N; per-block sums of d^2.
__global__ __launch_bounds__(kBlock) void k_gnn_loss(int64_t nrows, const double* __restrict__ psi,
                                                     const double* __restrict__ y,
                                                     const float* __restrict__ scales,
                                                     float* __restrict__ dd,
                                                     double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (r < nrows) {
    const double d = (psi[r] - y[r]) / static_cast<double>(scales[2]);
    v = d * d;
    dd[r] = static_cast<float>(2.0 * d / static_cast<double>(nrows));
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Decoder backward: g[r][k] = dd[r] w_out[k]; partials of dw_out = sum h dd,
// db_out = sum dd over the block's 64 rows.
__global__ __launch_bounds__(kBlock) void k_gnn_decode_bwd(int64_t nrows, const float* __restrict__ h,
                                                           const float* __restrict__ dd,
                                                           const uint16_t* __restrict__ w_out,
                                                           float* __restrict__ g,
                                                           float* __restrict__ part_w,
                                                           float* __restrict__ part_b) {
  __shared__ float red[16][kH + 1];
  const int k4 = threadIdx.x & 15, rq = threadIdx.x >> 4;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kTile;
  float aw[4] = {0.f, 0.f, 0.f, 0.f};
  float ab = 0.f;
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + rq * 4 + i;
    if (r >= nrows) continue;
    const float d = dd[r];
    const float4 hv = *reinterpret_cast<const float4*>(h + r * kH + k4 * 4);
    float4 gv;
    gv.x = d * bf16_to_f32(w_out[k4 * 4 + 0]);
    gv.y = d * bf16_to_f32(w_out[k4 * 4 + 1]);
    gv.z = d * bf16_to_f32(w_out[k4 * 4 + 2]);
    gv.w = d * bf16_to_f32(w_out[k4 * 4 + 3]);
    *reinterpret_cast<float4*>(g + r * kH + k4 * 4) = gv;
    aw[0] += hv.x * d;
    aw[1] += hv.y * d;
    aw[2] += hv.z * d;
    aw[3] += hv.w * d;
    ab += d;
  }
  for (int j = 0; j < 4; ++j) red[rq][k4 * 4 + j] = aw[j];
  __syncthreads();
  if (threadIdx.x < kH) {
    float s = 0.f;
    for (int q = 0; q < 16; ++q) s += red[q][threadIdx.x];
    part_w[static_cast<int64_t>(blockIdx.x) * kH + threadIdx.x] = s;
  }
  __syncthreads();
  if (k4 == 0) red[rq][0] = ab;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int q = 0; q < 16; ++q) s += red[q][0];
    part_b[blockIdx.x] = s;
  }
}

// Layer backward, part 1: dz = g (1 - t^2); gp = g + dz Ws^T; y = dz Wn^T.
__global__ __launch_bounds__(kBlock) void k_gnn_layer_bwd1(
    int64_t nrows, const float* __restrict__ g, const float* __restrict__ t,
    const uint16_t* __restrict__ Ws, const uint16_t* __restrict__ Wn, float* __restrict__ dz_out,
    float* __restrict__ y_out, float* __restrict__ gp_out) {
  __shared__ float Ds[kH * kXS];
  __shared__ float W1[kH * kH];
  __shared__ float W2[kH * kH];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kTile;
  for (int q = threadIdx.x; q < kTile * 16; q += blockDim.x) {
    const int row = q >> 4, k4 = q & 15;
    const int64_t r = r0 + row;
    float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < nrows) {
      const float4 gv = *reinterpret_cast<const float4*>(g + r * kH + k4 * 4);
      const float4 tv = *reinterpret_cast<const float4*>(t + r * kH + k4 * 4);
      d.x = gv.x * (1.f - tv.x * tv.x);
      d.y = gv.y * (1.f - tv.y * tv.y);
      d.z = gv.z * (1.f - tv.z * tv.z);
      d.w = gv.w * (1.f - tv.w * tv.w);
      *reinterpret_cast<float4*>(dz_out + r * kH + k4 * 4) = d;
    }
    Ds[(k4 * 4 + 0) * kXS + row] = d.x;
    Ds[(k4 * 4 + 1) * kXS + row] = d.y;
    Ds[(k4 * 4 + 2) * kXS + row] = d.z;
    Ds[(k4 * 4 + 3) * kXS + row] = d.w;
  }
  stage_w(Ws, kH, kH, true, W1);
  stage_w(Wn, kH, kH, true, W2);
  __syncthreads();
  const int fb = threadIdx.x & 15, rb = threadIdx.x >> 4;
  float a1[4][4] = {}, a2[4][4] = {};
  tile_mm<kH>(Ds, W1, rb, fb, a1);
  tile_mm<kH>(Ds, W2, rb, fb, a2);
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + rb * 4 + i;
    if (r >= nrows) continue;
    const float4 gv = *reinterpret_cast<const float4*>(g + r * kH + fb * 4);
    *reinterpret_cast<float4*>(gp_out + r * kH + fb * 4) =
        make_float4(gv.x + a1[i][0], gv.y + a1[i][1], gv.z + a1[i][2], gv.w + a1[i][3]);
    *reinterpret_cast<float4*>(y_out + r * kH + fb * 4) =
        make_float4(a2[i][0], a2[i][1], a2[i][2], a2[i][3]);
  }
}

// Layer backward, part 2: gp(j, s) += sum over neighbours i of j of y(i, s) / deg_i.
__global__ __launch_bounds__(kBlock) void k_gnn_layer_bwd2(int n, int S, const int* __restrict__ gptr,
                                                           const int* __restrict__ gidx,
                                                           const float* __restrict__ y,
                                                           float* __restrict__ gp) {
  const int64_t nrows = static_cast<int64_t>(n) * S;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = q >> 4;
  const int k4 = static_cast<int>(q & 15);
  if (r >= nrows) return;
  const int j = static_cast<int>(r / S), s = static_cast<int>(r % S);
  float4 acc = *reinterpret_cast<const float4*>(gp + r * kH + k4 * 4);
  for (int e = gptr[j]; e < gptr[j + 1]; ++e) {
    const int i = gidx[e];
    const float inv = 1.f / static_cast<float>(gptr[i + 1] - gptr[i]);
    const float4 v = *reinterpret_cast<const float4*>(y + (static_cast<int64_t>(i) * S + s) * kH + k4 * 4);
    acc.x += v.x * inv;
    acc.y += v.y * inv;
    acc.z += v.z * inv;
    acc.w += v.w * inv;
  }
  *reinterpret_cast<float4*>(gp + r * kH + k4 * 4) = acc;
}

// Encoder backward: dz0 = g (1 - h0^2), in place.
__global__ void k_gnn_tanh_bwd(int64_t count, const float* __restrict__ h0, float* __restrict__ g) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  g[e] *= 1.f - h0[e] * h0[e];
}

// Weight-gradient partials over 256 rows per work-group:
//   part_w[blk][k][f] = sum_r A[r][k] D[r][f]  (k < K, A row stride lda)
//   part_b[blk][f]    = sum_r D[r][f]
__global__ __launch_bounds__(kBlock) void k_gnn_wgrad(int64_t nrows, int K, const float* __restrict__ A,
                                                      int lda, const float* __restrict__ D,
                                                      float* __restrict__ part_w,
                                                      float* __restrict__ part_b) {
  __shared__ float As_[kTile][kH + 4];
  __shared__ float Ds_[kTile][kH + 4];
  const int fb = threadIdx.x & 15, kb = threadIdx.x >> 4;
  float acc[4][4] = {};
  float bacc[4] = {0.f, 0.f, 0.f, 0.f};
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 4 * kTile;
  for (int sub = 0; sub < 4; ++sub) {
    const int64_t r0 = base + sub * kTile;
    __syncthreads();
    for (int q = threadIdx.x; q < kTile * 16; q += blockDim.x) {
      const int row = q >> 4, c4 = q & 15;
      const int64_t r = r0 + row;
      float4 dv = make_float4(0.f, 0.f, 0.f, 0.f), av = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < nrows) {
        dv = *reinterpret_cast<const float4*>(D + r * kH + c4 * 4);
        if (c4 * 4 < K) av = *reinterpret_cast<const float4*>(A + r * lda + c4 * 4);
      }
      *reinterpret_cast<float4*>(&Ds_[row][c4 * 4]) = dv;
      *reinterpret_cast<float4*>(&As_[row][c4 * 4]) = av;
    }
    __syncthreads();
    if (kb * 4 < K) {
      for (int row = 0; row < kTile; ++row) {
        const float4 av = *reinterpret_cast<const float4*>(&As_[row][kb * 4]);
        const float4 dv = *reinterpret_cast<const float4*>(&Ds_[row][fb * 4]);
        const float aa[4] = {av.x, av.y, av.z, av.w};
        const float da[4] = {dv.x, dv.y, dv.z, dv.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(aa[i], da[j], acc[i][j]);
        if (kb == 0)
#pragma unroll
          for (int j = 0; j < 4; ++j) bacc[j] += da[j];
      }
    }
  }
  if (kb * 4 < K) {
    float* out = part_w + static_cast<int64_t>(blockIdx.x) * K * kH;
    for (int i = 0; i < 4 && kb * 4 + i < K; ++i)
      *reinterpret_cast<float4*>(out + (kb * 4 + i) * kH + fb * 4) =
          make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
  }
  if (kb == 0)
    *reinterpret_cast<float4*>(part_b + static_cast<int64_t>(blockIdx.x) * kH + fb * 4) =
        make_float4(bacc[0], bacc[1], bacc[2], bacc[3]);
}

// out[e] = sum over blocks b (in order) of part[b * count + e], e < count.
__global__ void k_gnn_sum(int nblk, int count, const float* __restrict__ part, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[static_cast<int64_t>(b) * count + e];
  out[e] = s;
}

__global__ void k_gnn_sum_loss(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b];
  *out += s;
}

// Adam on the trained entries (e >= first); bf16 copies of every entry.
__global__ void k_gnn_adam(int64_t np, int first, float* __restrict__ w, uint16_t* __restrict__ wbf,
                           const float* __restrict__ g, float* __restrict__ m1,
                           float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= np) return;
  if (e >= first) {
    const float gv = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gv;
    const float b = b2 * m2[e] + (1.f - b2) * gv * gv;
    m1[e] = a;
    m2[e] = b;
    w[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
  wbf[e] = f32_to_bf16(w[e]);
}

__global__ void k_gnn_round(int64_t np, const float* __restrict__ w, uint16_t* __restrict__ wbf) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < np) wbf[e] = f32_to_bf16(w[e]);
}

// Gather columns idx[s] of a [n][ld] block into a dense [n][S] block.
__global__ void k_gnn_gather(int n, int S, const int64_t* __restrict__ idx,
                             const double* __restrict__ src, int64_t ld, double* __restrict__ dst) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * S) return;
  const int i = static_cast<int>(e / S), s = static_cast<int>(e % S);
  dst[e] = src[i * ld + idx[s]];
}

__global__ void k_gnn_gather_meta(int S, const int64_t* __restrict__ idx, const int64_t* __restrict__ k_all,
                                  const double* __restrict__ amp_all, const double* __restrict__ dphi_all,
                                  int64_t* __restrict__ k_b, double* __restrict__ amp_b,
                                  double* __restrict__ dphi_b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int64_t j = idx[s];
  k_b[s] = k_all[j];
  amp_b[s] = amp_all[j];
  dphi_b[s] = dphi_all[j];
}

// Per-column sums of squares of (a - b) (or of a when b is null) over the
// n rows of [n][ld] blocks: out[c] += ...  (one wave per column).
__global__ __launch_bounds__(kBlock) void k_gnn_colsq(int n, int ncols, const double* __restrict__ a,
                                                      const double* __restrict__ b, int64_t ld,
                                                      double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= ncols) return;
  double s = 0.0;
  for (int i = lane; i < n; i += kWave) {
    const double d = b ? a[i * ld + c] - b[i * ld + c] : a[i * ld + c];
    s += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[c] = s;
}

// ---------------------------------------------------------------------------
// FP64 inference (the propagator inside MGRIT).  A coarse correction of FAS
// is a difference of two evaluations of the propagator; with FP32 features
// and activations that difference is noise below ~1e-7 of the state, which
// would stall MGRIT near its 1e-8 tolerance, so the network is evaluated in
// FP64 there (same bf16 weights).  A wave owns one row; lane f computes
// output feature f.

__global__ __launch_bounds__(kBlock) void k_gnn64_features(
    int n, int S, int m, int F, const double* __restrict__ u, int64_t ldu,
    const double* __restrict__ p, int64_t ldp, const double* __restrict__ tab,
    const double* __restrict__ F3, const float* __restrict__ flags, const float* __restrict__ scales,
    double* __restrict__ x) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = e / kFP;
  const int f = static_cast<int>(e % kFP);
  if (r >= static_cast<int64_t>(n) * S) return;
  const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
  double v = 0.0;
  if (f == 0) v = u[i * ldu + s] / static_cast<double>(scales[0]);
  else if (f == 1) v = p[i * ldp + s] / static_cast<double>(scales[0]);
  else if (f < m + 3) {
    const double* tb = tab + (static_cast<int64_t>(s) * (m + 1) + (f - 2)) * 3;
    v = ((tb[0] * F3[i] + tb[1] * F3[n + i]) + tb[2] * F3[2 * n + i]) / static_cast<double>(scales[1]);
  } else if (f < F) {
    v = flags[i * 4 + (f - m - 3)];
  }
  x[r * kFP + f] = v;
}

__global__ __launch_bounds__(kBlock) void k_gnn64_in(int64_t nrows, int F, const double* __restrict__ x,
                                                     const uint16_t* __restrict__ W,
                                                     const uint16_t* __restrict__ b,
                                                     double* __restrict__ h) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int f = threadIdx.x & 63;
  if (r >= nrows) return;
  double z = 0.0;
  for (int k = 0; k < F; ++k) z += x[r * kFP + k] * static_cast<double>(bf16_to_f32(W[k * kH + f]));
  h[r * kH + f] = tanh(z + static_cast<double>(bf16_to_f32(b[f])));
}

__global__ __launch_bounds__(kBlock) void k_gnn64_agg(int n, int S, const int* __restrict__ gptr,
                                                      const int* __restrict__ gidx,
                                                      const double* __restrict__ h,
                                                      double* __restrict__ a) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int f = threadIdx.x & 63;
  if (r >= static_cast<int64_t>(n) * S) return;
  const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
  double acc = 0.0;
  for (int e = gptr[i]; e < gptr[i + 1]; ++e) acc += h[(static_cast<int64_t>(gidx[e]) * S + s) * kH + f];
  a[r * kH + f] = acc / static_cast<double>(gptr[i + 1] - gptr[i]);
}

__global__ __launch_bounds__(kBlock) void k_gnn64_layer(int64_t nrows, const double* __restrict__ h,
                                                        const double* __restrict__ a,
                                                        const uint16_t* __restrict__ Ws,
                                                        const uint16_t* __restrict__ Wn,
                                                        const uint16_t* __restrict__ b,
                                                        double* __restrict__ hout) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int f = threadIdx.x & 63;
  if (r >= nrows) return;
  double z = 0.0;
  for (int k = 0; k < kH; ++k)
    z += h[r * kH + k] * static_cast<double>(bf16_to_f32(Ws[k * kH + f])) +
         a[r * kH + k] * static_cast<double>(bf16_to_f32(Wn[k * kH + f]));
  hout[r * kH + f] = h[r * kH + f] + tanh(z + static_cast<double>(bf16_to_f32(b[f])));
}

__global__ __launch_bounds__(kBlock) void k_gnn64_out(int n, int S, const double* __restrict__ h,
                                                      const uint16_t* __restrict__ w_out,
                                                      const uint16_t* __restrict__ b_out,
                                                      const float* __restrict__ scales,
                                                      const double* __restrict__ p, int64_t ldp,
                                                      double* __restrict__ out, int64_t ldo) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int f = threadIdx.x & 63;
  if (r >= static_cast<int64_t>(n) * S) return;
  double d = h[r * kH + f] * static_cast<double>(bf16_to_f32(w_out[f]));
  for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
  if (f == 0) {
    const int i = static_cast<int>(r / S), s = static_cast<int>(r % S);
    const double delta = d + static_cast<double>(bf16_to_f32(b_out[0]));
    out[i * ldo + s] = p[i * ldp + s] + static_cast<double>(scales[2]) * delta;
  }
}

// X'[:, b] = X[:, b] + alpha[b] (X[:, perm[b]] - X[:, b]) for b < nt.
__global__ void k_gnn_mix(int n, int nt, const double* __restrict__ X, int64_t ld,
                          const int* __restrict__ perm, const double* __restrict__ alpha,
                          double* __restrict__ Y) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * nt) return;
  const int i = static_cast<int>(e / nt), b = static_cast<int>(e % nt);
  const double x = X[i * ld + b];
  Y[i * ld + b] = x + alpha[b] * (X[i * ld + perm[b]] - x);
}

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

void gnn_mix(hipStream_t s, int n, int nt, const double* X, int64_t ld, const int* perm,
             const double* alpha, double* Y) {
  hipLaunchKernelGGL(k_gnn_mix, dim3(cdiv(static_cast<int64_t>(n) * nt, 256)), dim3(256), 0, s, n, nt, X,
                     ld, perm, alpha, Y);
  MG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------

GnnOffsets gnn_offsets(int m) {
  GnnOffsets o;
  o.F = m + 7;
  o.w_in = 4;
  o.b_in = o.w_in + static_cast<int64_t>(o.F) * kH;
  int64_t p = o.b_in + kH;
  for (int l = 0; l < 3; ++l) {
    o.ws[l] = p;
    o.wn[l] = p + kH * kH;
    o.b[l] = p + 2 * kH * kH;
    p += 2 * kH * kH + kH;
  }
  o.w_out = p;
  o.b_out = p + kH;
  o.n_params = p + kH + 1;
  return o;
}

void gnn_alloc_rows(GnnModel& g, DeviceArena& arena, int64_t rows) {
  if (rows <= g.rows_cap) return;
  g.rows_cap = rows;
  const size_t act = static_cast<size_t>(rows) * kH;
  for (int l = 0; l < 4; ++l) g.h[l] = arena.alloc<float>(act);
  for (int l = 0; l < 3; ++l) {
    g.a[l] = arena.alloc<float>(act);
    g.t[l] = arena.alloc<float>(act);
  }
  g.x = arena.alloc<float>(static_cast<size_t>(rows) * kFP);
  g.g0 = arena.alloc<float>(act);
  g.g1 = arena.alloc<float>(act);
  g.dz = arena.alloc<float>(act);
  g.y = arena.alloc<float>(act);
  g.dd = arena.alloc<float>(rows);
  const int64_t nblk_w = cdiv(rows, 4 * kTile);
  g.part_w = arena.alloc<float>(static_cast<size_t>(nblk_w) * kH * kH);
  g.part_b = arena.alloc<float>(static_cast<size_t>(cdiv(rows, kTile)) * kH);
  g.part_loss = arena.alloc<double>(static_cast<size_t>(cdiv(rows, kBlock)));
}

void gnn_alloc_samples(GnnModel& g, DeviceArena& arena, int S) {
  if (S <= g.s_cap) return;
  g.s_cap = S;
  g.tab = arena.alloc<double>(static_cast<size_t>(S) * (g.m + 1) * 3);
}

void gnn_alloc_rows64(GnnModel& g, DeviceArena& arena, int64_t rows) {
  if (rows <= g.rows64_cap) return;
  g.rows64_cap = rows;
  const size_t act = static_cast<size_t>(rows) * kH;
  g.x64 = arena.alloc<double>(static_cast<size_t>(rows) * kFP);
  g.h64[0] = arena.alloc<double>(act);
  g.h64[1] = arena.alloc<double>(act);
  g.a64 = arena.alloc<double>(act);
}

void gnn_forward64(hipStream_t s, GnnModel& g, const SourceDev& src, int S, const int64_t* k_list,
                   int64_t k_base, int64_t k_stride, const double* amp, const double* dphi, CView u,
                   CView p, double* out, int64_t ldo) {
  const int n = g.n;
  const int64_t rows = static_cast<int64_t>(n) * S;
  if (rows > g.rows64_cap || S > g.s_cap) fail(MGRIT_INVALID_ARGUMENT, "learned propagator workspace too small");
  const GnnOffsets& o = g.off;
  hipLaunchKernelGGL(k_gnn_srctab, dim3(cdiv(static_cast<int64_t>(S) * (g.m + 1), 256)), dim3(256), 0, s,
                     S, g.m, g.dT, k_list, k_base, k_stride, src, amp, dphi, g.tab);
  hipLaunchKernelGGL(k_gnn64_features, dim3(cdiv(rows * kFP, kBlock)), dim3(kBlock), 0, s, n, S, g.m, o.F,
                     u.p, u.ld, p.p, p.ld, g.tab, g.F3, g.flags, g.w32, g.x64);
  const int nb = cdiv(rows, 4);
  hipLaunchKernelGGL(k_gnn64_in, dim3(nb), dim3(kBlock), 0, s, rows, o.F, g.x64, g.wbf + o.w_in,
                     g.wbf + o.b_in, g.h64[0]);
  for (int l = 0; l < 3; ++l) {
    const double* hin = g.h64[l & 1];
    double* hout = g.h64[(l + 1) & 1];
    hipLaunchKernelGGL(k_gnn64_agg, dim3(nb), dim3(kBlock), 0, s, n, S, g.gptr, g.gidx, hin, g.a64);
    hipLaunchKernelGGL(k_gnn64_layer, dim3(nb), dim3(kBlock), 0, s, rows, hin, g.a64, g.wbf + o.ws[l],
                       g.wbf + o.wn[l], g.wbf + o.b[l], hout);
  }
  hipLaunchKernelGGL(k_gnn64_out, dim3(nb), dim3(kBlock), 0, s, n, S, g.h64[1], g.wbf + o.w_out,
                     g.wbf + o.b_out, g.w32, p.p, p.ld, out, ldo);
  MG_HIP(hipGetLastError());
}

void gnn_round_weights(hipStream_t s, GnnModel& g) {
  hipLaunchKernelGGL(k_gnn_round, dim3(cdiv(g.off.n_params, 256)), dim3(256), 0, s, g.off.n_params,
                     g.w32, g.wbf);
  MG_HIP(hipGetLastError());
}

void gnn_forward(hipStream_t s, GnnModel& g, const SourceDev& src, int S, const int64_t* k_list,
                 int64_t k_base, int64_t k_stride, const double* amp, const double* dphi,
                 CView u, CView p, double* out, int64_t ldo, bool keep) {
  const int n = g.n;
  const int64_t rows = static_cast<int64_t>(n) * S;
  if (rows > g.rows_cap || S > g.s_cap) fail(MGRIT_INVALID_ARGUMENT, "learned propagator workspace too small");
  const GnnOffsets& o = g.off;
  hipLaunchKernelGGL(k_gnn_srctab, dim3(cdiv(static_cast<int64_t>(S) * (g.m + 1), 256)), dim3(256), 0, s,
                     S, g.m, g.dT, k_list, k_base, k_stride, src, amp, dphi, g.tab);
  hipLaunchKernelGGL(k_gnn_encode, dim3(cdiv(rows, kTile)), dim3(kBlock), 0, s, n, S, g.m, o.F, u.p, u.ld,
                     p.p, p.ld, g.tab, g.F3, g.flags, g.w32, g.wbf + o.w_in, g.wbf + o.b_in,
                     keep ? g.x : nullptr, g.h[0]);
  for (int l = 0; l < 3; ++l)
    hipLaunchKernelGGL(k_gnn_layer, dim3(cdiv(rows, kTile)), dim3(kBlock), 0, s, n, S, g.gptr, g.gidx,
                       g.h[l], g.wbf + o.ws[l], g.wbf + o.wn[l], g.wbf + o.b[l], g.h[l + 1],
                       keep ? g.a[l] : nullptr, keep ? g.t[l] : nullptr);
  hipLaunchKernelGGL(k_gnn_decode, dim3(cdiv(rows, 16)), dim3(kBlock), 0, s, n, S, g.h[3],
                     g.wbf + o.w_out, g.wbf + o.b_out, g.w32, p.p, p.ld, out, ldo);
  MG_HIP(hipGetLastError());
}

void gnn_backward(hipStream_t s, GnnModel& g, int S, const double* psi, const double* y,
                  double* loss_acc) {
  const int n = g.n;
  const int64_t rows = static_cast<int64_t>(n) * S;
  const GnnOffsets& o = g.off;
  const int nb_loss = cdiv(rows, kBlock);
  hipLaunchKernelGGL(k_gnn_loss, dim3(nb_loss), dim3(kBlock), 0, s, rows, psi, y, g.w32, g.dd,
                     g.part_loss);
  hipLaunchKernelGGL(k_gnn_sum_loss, dim3(1), dim3(64), 0, s, nb_loss, g.part_loss, loss_acc);
  const int nb_t = cdiv(rows, kTile);
  hipLaunchKernelGGL(k_gnn_decode_bwd, dim3(nb_t), dim3(kBlock), 0, s, rows, g.h[3], g.dd,
                     g.wbf + o.w_out, g.g0, g.part_b, g.part_w);
  // part_b holds the w_out partials [nb_t][64], part_w the b_out partials [nb_t]
  hipLaunchKernelGGL(k_gnn_sum, dim3(1), dim3(kH), 0, s, nb_t, kH, g.part_b, g.grad + o.w_out);
  hipLaunchKernelGGL(k_gnn_sum, dim3(1), dim3(kH), 0, s, nb_t, 1, g.part_w, g.grad + o.b_out);
  const int nb_w = cdiv(rows, 4 * kTile);
  float* gcur = g.g0;
  float* gnext = g.g1;
  for (int l = 2; l >= 0; --l) {
    hipLaunchKernelGGL(k_gnn_layer_bwd1, dim3(nb_t), dim3(kBlock), 0, s, rows, gcur, g.t[l],
                       g.wbf + o.ws[l], g.wbf + o.wn[l], g.dz, g.y, gnext);
    hipLaunchKernelGGL(k_gnn_layer_bwd2, dim3(cdiv(rows * 16, kBlock)), dim3(kBlock), 0, s, n, S,
                       g.gptr, g.gidx, g.y, gnext);
    hipLaunchKernelGGL(k_gnn_wgrad, dim3(nb_w), dim3(kBlock), 0, s, rows, kH, g.h[l], kH, g.dz,
                       g.part_w, g.part_b);
    hipLaunchKernelGGL(k_gnn_sum, dim3(cdiv(kH * kH, 256)), dim3(256), 0, s, nb_w, kH * kH, g.part_w,
                       g.grad + o.ws[l]);
    hipLaunchKernelGGL(k_gnn_sum, dim3(1), dim3(kH), 0, s, nb_w, kH, g.part_b, g.grad + o.b[l]);
    hipLaunchKernelGGL(k_gnn_wgrad, dim3(nb_w), dim3(kBlock), 0, s, rows, kH, g.a[l], kH, g.dz,
                       g.part_w, g.part_b);
    hipLaunchKernelGGL(k_gnn_sum, dim3(cdiv(kH * kH, 256)), dim3(256), 0, s, nb_w, kH * kH, g.part_w,
                       g.grad + o.wn[l]);
    float* tmp = gcur;
    gcur = gnext;
    gnext = tmp;
  }
  hipLaunchKernelGGL(k_gnn_tanh_bwd, dim3(cdiv(rows * kH, 256)), dim3(256), 0, s, rows * kH, g.h[0], gcur);
  hipLaunchKernelGGL(k_gnn_wgrad, dim3(nb_w), dim3(kBlock), 0, s, rows, o.F, g.x, kFP, gcur, g.part_w,
                     g.part_b);
  hipLaunchKernelGGL(k_gnn_sum, dim3(cdiv(o.F * kH, 256)), dim3(256), 0, s, nb_w, o.F * kH, g.part_w,
                     g.grad + o.w_in);
  hipLaunchKernelGGL(k_gnn_sum, dim3(1), dim3(kH), 0, s, nb_w, kH, g.part_b, g.grad + o.b_in);
  MG_HIP(hipGetLastError());
}

void gnn_adam(hipStream_t s, GnnModel& g, double lr, int step) {
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
  hipLaunchKernelGGL(k_gnn_adam, dim3(cdiv(g.off.n_params, 256)), dim3(256), 0, s, g.off.n_params, 4,
                     g.w32, g.wbf, g.grad, g.m1, g.m2, static_cast<float>(lr), static_cast<float>(b1),
                     static_cast<float>(b2), 1e-8f, static_cast<float>(c1), static_cast<float>(c2));
  MG_HIP(hipGetLastError());
}

void gnn_gather(hipStream_t s, int n, int S, const int64_t* idx, const double* src, int64_t ld,
                double* dst) {
  hipLaunchKernelGGL(k_gnn_gather, dim3(cdiv(static_cast<int64_t>(n) * S, 256)), dim3(256), 0, s, n, S,
                     idx, src, ld, dst);
  MG_HIP(hipGetLastError());
}

void gnn_gather_meta(hipStream_t s, int S, const int64_t* idx, const int64_t* k_all,
                     const double* amp_all, const double* dphi_all, int64_t* k_b, double* amp_b,
                     double* dphi_b) {
  hipLaunchKernelGGL(k_gnn_gather_meta, dim3(cdiv(S, 256)), dim3(256), 0, s, S, idx, k_all, amp_all,
                     dphi_all, k_b, amp_b, dphi_b);
  MG_HIP(hipGetLastError());
}

void gnn_colsq(hipStream_t s, int n, int ncols, const double* a, const double* b, int64_t ld,
               double* out) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_gnn_colsq, dim3(cdiv(ncols, 4)), dim3(kBlock), 0, s, n, ncols, a, b, ld, out);
  MG_HIP(hipGetLastError());
}

}  // namespace mg
