// Stored-inverse step of an intermediate level: X = A^{-1} B for a batch of
// columns, in FP64 on the matrix cores.
//
// The right-hand sides and results are column blocks [n][ld] (row i of
// column c at p[i * ld + c]); A^{-1} is stored [n][lda] (symmetric).  As a
// product of matrices indexed (column c, row k):
//     X(c, j) = sum_k B(c, k) Ainv(k, j),   B(c, k) = Bp[k * ldb + c],
//     Ainv(k, j) = A[k * lda + j],          X(c, j) = Xp[j * ldx + c].
// A work-group computes a 64 x 64 tile of X (64 columns c times 64 rows j)
// over one slice of k; its 4 waves each own a 32 x 32 quarter as 2 x 2
// blocks of the 16 x 16 x 4 FP64 MFMA.  Chunks of 16 values of k of both
// operands are staged in LDS, the next chunk's global loads in flight while
// the current one is multiplied.  With few columns (the relaxation sweeps of
// an intermediate level: 64) the k range is split over several work-groups
// so that the grid fills the chip; the slices' partial tiles are summed in a
// fixed order by a second kernel, so every result is independent of the
// batch width and of the split.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace mg {
namespace {

constexpr int kTileM = 64;   // columns c per work-group
constexpr int kTileN = 64;   // rows j per work-group
constexpr int kChunk = 16;   // values of k per LDS stage
constexpr int kGemmThreads = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kGemmThreads) void k_inv_gemm(int M, int N, int K, int kslice,
                                                           const double* __restrict__ Bp, int64_t ldb,
                                                           const double* __restrict__ A, int64_t lda,
                                                           double* __restrict__ out, int64_t ldo,
                                                           int64_t split_stride) {
  __shared__ double Bs[kChunk][kTileM];
  __shared__ double As[kChunk][kTileN];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int mt = blockIdx.x, nt = blockIdx.y, split = blockIdx.z;
  const int c0 = mt * kTileM, j0 = nt * kTileN;
  const int kb = split * kslice;
  const int ke = (kb + kslice < K) ? kb + kslice : K;
  // staging: thread t loads 4 consecutive values of one chunk row of each operand
  const int lr = tid >> 4;            // chunk row 0..15
  const int lc = (tid & 15) * 4;      // first of 4 columns
  double rb[4], ra[4];
  auto gload = [&](int k) {
    const int kk = k + lr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + lc + e, j = j0 + lc + e;
      rb[e] = (kk < ke && c < M) ? Bp[static_cast<int64_t>(kk) * ldb + c] : 0.0;
      ra[e] = (kk < ke && j < N) ? A[static_cast<int64_t>(kk) * lda + j] : 0.0;
    }
  };
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  // this wave's quarter of the tile and its lane's operand coordinates
  const int wc = (wv & 1) * 32, wj = (wv >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  if (kb < ke) gload(kb);
  for (int k = kb; k < ke; k += kChunk) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Bs[lr][lc + e] = rb[e];
      As[lr][lc + e] = ra[e];
    }
    __syncthreads();
    if (k + kChunk < ke) gload(k + kChunk);
#pragma unroll
    for (int s4 = 0; s4 < kChunk; s4 += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = Bs[s4 + lk][wc + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = As[s4 + lk][wj + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  }
  // lane l of a 16 x 16 block holds rows l / 16 + 4 r, r = 0..3, of
  // column l % 16 (rows = c, columns = j here)
  double* o = out + split * split_stride;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + wj + b * 16 + li;
      if (j >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = c0 + wc + a * 16 + lk + 4 * r;
        if (c < M) o[static_cast<int64_t>(j) * ldo + c] = acc[a][b][r];
      }
    }
}

// X[j][c] = sum over the splits s (in order) of P[s][j][c].
__global__ void k_inv_gemm_sum(int M, int N, int splits, const double* __restrict__ P, int64_t ldp,
                               int64_t split_stride, double* __restrict__ X, int64_t ldx) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= M || j >= N) return;
  double v = 0.0;
  for (int s = 0; s < splits; ++s) v += P[s * split_stride + static_cast<int64_t>(j) * ldp + c];
  X[static_cast<int64_t>(j) * ldx + c] = v;
}

// y = A x for one contiguous column (the stored-inverse sequential stepper):
// a wave owns 4 rows, its lanes read 16-byte pairs of each row and of x
// (x once for the 4 rows), two pairs in flight per row, then a fixed-order
// shuffle reduction.  A streams from HBM once; x stays in the caches.
constexpr int kGemvRows = 4;

__global__ __launch_bounds__(256) void k_inv_gemv(int n, const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int r0 = (blockIdx.x * 4 + wv) * kGemvRows;
  if (r0 >= n) return;
  double acc[kGemvRows][2];
#pragma unroll
  for (int r = 0; r < kGemvRows; ++r) acc[r][0] = acc[r][1] = 0.0;
  const int npair = n >> 1;                 // full 16-byte pairs of a row
  int p = lane;
  for (; p + 64 < npair; p += 128) {
    const double2 xa = reinterpret_cast<const double2*>(x)[p];
    const double2 xb = reinterpret_cast<const double2*>(x)[p + 64];
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) {
      const int row = (r0 + r < n) ? r0 + r : n - 1;
      const double2* ar = reinterpret_cast<const double2*>(A + static_cast<int64_t>(row) * lda);
      const double2 a0 = ar[p], a1 = ar[p + 64];
      acc[r][0] = fma(a0.x, xa.x, acc[r][0]);
      acc[r][1] = fma(a0.y, xa.y, acc[r][1]);
      acc[r][0] = fma(a1.x, xb.x, acc[r][0]);
      acc[r][1] = fma(a1.y, xb.y, acc[r][1]);
    }
  }
  for (; p < npair; p += 64) {
    const double2 xa = reinterpret_cast<const double2*>(x)[p];
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) {
      const int row = (r0 + r < n) ? r0 + r : n - 1;
      const double2 a0 = reinterpret_cast<const double2*>(A + static_cast<int64_t>(row) * lda)[p];
      acc[r][0] = fma(a0.x, xa.x, acc[r][0]);
      acc[r][1] = fma(a0.y, xa.y, acc[r][1]);
    }
  }
  if ((n & 1) && lane == 0) {
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) {
      const int row = (r0 + r < n) ? r0 + r : n - 1;
      acc[r][0] = fma(A[static_cast<int64_t>(row) * lda + n - 1], x[n - 1], acc[r][0]);
    }
  }
#pragma unroll
  for (int r = 0; r < kGemvRows; ++r) {
    double t = acc[r][0] + acc[r][1];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0 && r0 + r < n) y[r0 + r] = t;
  }
}

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace

void launch_inv_gemv(hipStream_t s, int n, const double* A, int64_t lda, const double* x, double* y) {
  if (n <= 0) return;
  if ((lda & 1) || (reinterpret_cast<uintptr_t>(A) & 15) || (reinterpret_cast<uintptr_t>(x) & 15))
    fail(MGRIT_INVALID_ARGUMENT, "inverse GEMV: A, its stride and x must be 16-byte aligned");
  hipLaunchKernelGGL(k_inv_gemv, dim3(cdiv(n, 4 * kGemvRows)), dim3(256), 0, s, n, A, lda, x, y);
  MG_HIP(hipGetLastError());
}

// Slices of k for M columns: enough work-groups for two per compute unit.
static int inv_gemm_slices(int M, int N, int& kslice) {
  const int tiles = cdiv(M, kTileM) * cdiv(N, kTileN);
  int want = cdiv(512, tiles);
  want = want < 1 ? 1 : (want > 8 ? 8 : want);
  kslice = cdiv(cdiv(N, want), kChunk) * kChunk;
  return cdiv(N, kslice);
}

int64_t inv_gemm_part_doubles(int max_cols, int N) {
  int64_t best = 0;
  for (int mt = 1; mt <= cdiv(max_cols, kTileM); ++mt) {
    int kslice = 0;
    const int S = inv_gemm_slices(mt * kTileM, N, kslice);
    if (S > 1) best = std::max<int64_t>(best, static_cast<int64_t>(S) * N * mt * kTileM);
  }
  return best;
}

void launch_inv_gemm(hipStream_t s, int M, int N, const double* B, int64_t ldb, const double* A,
                     int64_t lda, double* X, int64_t ldx, double* part, int64_t part_size) {
  if (M <= 0 || N <= 0) return;
  int kslice = 0;
  const int S = inv_gemm_slices(M, N, kslice);
  const int64_t ldp = static_cast<int64_t>(cdiv(M, kTileM)) * kTileM;
  dim3 grid(cdiv(M, kTileM), cdiv(N, kTileN), S);
  if (S == 1) {
    hipLaunchKernelGGL(k_inv_gemm, grid, dim3(kGemmThreads), 0, s, M, N, N, kslice, B, ldb, A, lda, X,
                       ldx, int64_t(0));
  } else {
    const int64_t stride = static_cast<int64_t>(N) * ldp;
    if (!part || S * stride > part_size) fail(MGRIT_INVALID_ARGUMENT, "inverse GEMM: partial-sum buffer too small");
    hipLaunchKernelGGL(k_inv_gemm, grid, dim3(kGemmThreads), 0, s, M, N, N, kslice, B, ldb, A, lda,
                       part, ldp, stride);
    hipLaunchKernelGGL(k_inv_gemm_sum, dim3(cdiv(M, 64), cdiv(N, 4)), dim3(256), 0, s, M, N, S, part,
                       ldp, stride, X, ldx);
  }
  MG_HIP(hipGetLastError());
}

}  // namespace mg
