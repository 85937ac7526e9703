// Internal declarations of the MGRIT library: device data structures and the
// launch wrappers of every kernel.  Not part of the public ABI (see mgrit.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mgrit.h"

namespace mg {

// ---------------------------------------------------------------------------
// Errors: thrown inside the library, turned into mgrit_status at the C ABI.
struct Fail {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define MG_HIP(x) ::mg::hip_check((x), #x)

constexpr int kWave = 64;
constexpr int kBlock = 256;        // threads of the batched kernels (4 waves)
constexpr int kSeqThreads = 1024;  // threads of the single-workgroup stepper

// Source parameters evaluated on the device (PWM, Sec. 3.2-3.3).
struct SourceDev {
  double scale;        // J0 * amplitude
  double freq, f_carrier;
  double phi[3];       // phases[p] + phase_offset
  int carrier;         // 0 triangle, 1 sawtooth
  double ramp_span;    // start-up ramp length in seconds (0 = none)
  int signal = 0;      // 0 PWM, 1 the sine references themselves (nested-iteration start)
  double t0 = 0.0;     // time origin: the source is sampled at t0 + t
};

// Column-block view: entry (row i, column c) at p[i * ld + c].
struct CView {
  const double* p = nullptr;
  int64_t ld = 0;
};

// Operators of one level on the device.  The sparsity pattern is stored with a
// fixed row width W (rows padded with a zero entry pointing at the row itself).
struct DevLevel {
  int n = 0, W = 0;
  double dt = 0.0;
  int* col = nullptr;          // [n*W]
  double* a64 = nullptr;       // [n*W] A = M/dt + K (linear model)
  float* a32 = nullptr;        // [n*W]
  double* m64 = nullptr;       // [n*W] M/dt
  uint8_t* has_mass = nullptr; // [n] row of M/dt is not identically zero
  double* dinv64 = nullptr;    // [n] 1 / diag(A)
  float* dinv32 = nullptr;
  double* F = nullptr;         // [3][n] phase load vectors (unit current density x sign)
  // symmetric Jacobi scaling used by the batched CG: A^ = S A S, S = diag(A)^{-1/2}
  double* s64 = nullptr;       // [n] S
  float* s32 = nullptr;
  double* d64 = nullptr;       // [n] diag(A)
  double* ah64 = nullptr;      // [n*W] A^
  float* ah32 = nullptr;
  // A^ by offset when the pattern is the periodic 7-diagonal polar stencil
  // (offsets 0, +-1, +-R, +-(R+1) mod n); dia_R = 0 when it is not
  int dia_R = 0;
  double* dv64 = nullptr;      // [n][8]
  float* dv32 = nullptr;
};

// Spatial transfer (rows = output nodes), fixed row width.
struct DevTransfer {
  int n_out = 0, n_in = 0, W = 0;
  int* col = nullptr;
  double* val = nullptr;
};

// Element data of a level for the nonlinear model (device).
struct NlLevel {
  int n_tri = 0;
  const int* tri_u = nullptr;     // [T][3] unknown index of each vertex, -1 = Dirichlet
  const double* grad = nullptr;   // [T][3][2]
  const double* area = nullptr;   // [T]
  const double* nu_lin = nullptr; // [T] linear reluctivity
  const uint8_t* iron = nullptr;  // [T] saturating law applies
  const int* cptr = nullptr;      // contribution lists of the stored entries
  const int* contrib = nullptr;
  const int* diag = nullptr;      // [n] slot of the diagonal entry
  double k1 = 0, k2 = 0, k3 = 0;
};

struct NlWork;

// Batched-PCG workspace for up to `cap` columns of an n-row level.
struct PcgWork {
  int n = 0, cap = 0, nrb = 0, rows_per_block = 0;
  int prec = 0;                 // MGRIT_FP64 or MGRIT_FP32_IR (this workspace's solves)
  int cpl = 1;                  // columns per lane of the CG passes (1 or 2)
  bool dia = false;             // use the diagonal-window CG passes
  int depth = 1;                // rows of loads in flight per wave (diagonal-window passes: 1, 2, 4)
  int rpb_narrow = 0;           // rows per work-group once few columns iterate (0 = keep)
  int64_t ld = 0;
  double *x = nullptr, *r = nullptr;
  double* pbuf[2] = {nullptr, nullptr};  // search directions, ping-pong
  int parity = 0;                        // pbuf[parity] holds the current p
  double* part = nullptr;       // [3][nrb][ld] per-row-block partial sums
  double* scal = nullptr;       // [8][ld]: rz, rr, bb, alpha, beta, (spare)
  double* src = nullptr;        // [3][ld] source value per phase and column
  uint8_t* active = nullptr;    // [ld] column still iterating (inner solve)
  uint8_t* outer = nullptr;     // [ld] column still refining (FP32 + FP64 refinement)
  float *r32 = nullptr, *x32 = nullptr;  // FP32 inner solve (residual, correction)
  float* p32[2] = {nullptr, nullptr};
  int* flags = nullptr;         // [8]: 0 active count, 1 error bits, 2 iterations of the
                                //      sequential stepper, 4 pass-A launches of this solve
  int* host_flags = nullptr;    // pinned copy of flags
  int* hist = nullptr;          // [max_iter] active columns of every PCG iteration
  int* host_hist = nullptr;     // pinned copy
  int hist_cap = 0;
  NlWork* nl = nullptr;         // Newton buffers (nonlinear model, allocated on first use)
  // column compaction (allocated on first use): two alternate sets of the CG
  // vectors of the workspace's precision, the compact -> caller column map,
  // and the per-step gather map
  void* alt_x[2] = {nullptr, nullptr};
  void* alt_r[2] = {nullptr, nullptr};
  void* alt_p[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int* gmap = nullptr;
  int* cmap = nullptr;
};

// Newton workspace of a PcgWork (same n, ld).
struct NlWork {
  bool fp32 = false;                   // inner solve in FP32
  // periodic polar stencil (DevLevel::dia_R > 0): the Jacobian is stored as
  // its upper half by offset, J[i][s][ld] for the offsets 0, +1, +R, +R+1
  // (mod n) of row i; the lower entries of row i are the upper entries of
  // the rows i-1, i-R, i-R-1 (J is symmetric)
  int dia_R = 0;
  double *nu = nullptr, *dnu = nullptr, *gx = nullptr, *gy = nullptr;  // [T][ld]
  double* R = nullptr;                 // [n][ld] Newton residual
  double* dg = nullptr;                // [n][ld] diag(J)
  double* ref = nullptr;               // [ld] ||R(u_prev)||^2
  double* rcur = nullptr;              // [ld] ||R(u)||^2 at the current iterate
  double* lam = nullptr;               // [ld] trial step length (damping)
  double* fac = nullptr;               // [ld] factor of d in the next update
  uint8_t* ls = nullptr;               // [ld] column still choosing its step length
  float* J32 = nullptr;                // [n][W][ld] scaled Jacobian (FP32 inner)
  float* s32 = nullptr;                // [n][ld] scaling
  double* J64 = nullptr;               // FP64 inner
  double* s64 = nullptr;
  double* r64 = nullptr;
  double* p64[2] = {nullptr, nullptr};
  double* d64 = nullptr;               // FP64 inner correction
};

void launch_nl_elem(hipStream_t s, const NlLevel& N, int ncols, int64_t ld, const uint8_t* outer,
                    CView u, NlWork& nw);
void launch_nl_residual(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                        int ncols, const uint8_t* outer, CView u, CView uprev);
// ref_mode 1: ref = ||R||^2, every column with R != 0 refines; 0: refine while ||R||^2 > tol2 ref
// eta2 > 0: the stopping threshold becomes max(tol2 ||R(u_prev)||^2, eta2 ||R(guess)||^2)
// (in ref_mode the guess is u_prev itself, pass 0 when it is not)
void launch_nl_test(hipStream_t s, PcgWork& w, NlWork& nw, int ncols, int ref_mode, double tol2,
                    double eta2 = 0.0);
void launch_nl_jacobian(hipStream_t s, const DevLevel& L, const NlLevel& N, PcgWork& w, NlWork& nw,
                        int ncols);
void launch_nl_cg_init(hipStream_t s, PcgWork& w, NlWork& nw, int ncols);
void launch_nl_pass_a(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols, int first);
// Persistent one-work-group damped-Newton stepper: nsteps sequential steps
// u_s = Phi(u_{s-1}) + g_s on the column block U (column s = point s), the
// whole Newton / CG / step-length loop on the device.  ws: seq_newton_ws_doubles.
// flags[1] bits: 1 non-finite, 2 inner CG cap, 8 Newton cap; flags[2] += CG
// iterations, flags[3] += Newton iterations.
int64_t seq_newton_ws_doubles(int n, int W, int n_tri);
void launch_seq_newton(hipStream_t s, const DevLevel& L, const NlLevel& N, const SourceDev& src,
                       int nsteps, int64_t t0, double* U, int64_t ldu, const double* G, int64_t ldg,
                       int warm, double newton_tol, int newton_max, double lam_min, double inner_tol,
                       int cg_max, double* ws, int* flags, bool add_g = true);
// The same per-column Newton for a narrow batch of independent steps, one
// work-group per column: u_prev = uin[:, c], start and result in x[:, c], the
// step from t_i to t_{i+1} with i = t_list[c] (or t_base + c t_stride); ws
// holds ncols workspaces of seq_newton_ws_doubles each.
void launch_seq_newton_batch(hipStream_t s, const DevLevel& L, const NlLevel& N, const SourceDev& src,
                             int ncols, CView uin, double* x, int64_t ldx, const int64_t* t_list,
                             int64_t t_base, int64_t t_stride, double newton_tol, int newton_max,
                             double lam_min, double inner_tol, int cg_max, double* ws, int* flags);
void launch_nl_pass_b(hipStream_t s, const DevLevel& L, PcgWork& w, NlWork& nw, int ncols);
// u += fac[c] d on the columns with ls[c] set
void launch_nl_update(hipStream_t s, PcgWork& w, NlWork& nw, int ncols);
// ls = outer, lam = fac = 1, flags[3] = 0
void launch_nl_ls_start(hipStream_t s, PcgWork& w, NlWork& nw, int ncols);
// step-length test of the searching columns; flags[0] = still searching,
// flags[3] += refining columns accepted
void launch_nl_ls(hipStream_t s, PcgWork& w, NlWork& nw, int ncols, double tol2, double lam_min);

enum ReduceMode { RED_INIT = 0, RED_ALPHA = 1, RED_BETA = 2, RED_SUM = 3, RED_IR_INIT = 4, RED_IR_FIRST = 5 };

// --- setup kernels ---------------------------------------------------------
void launch_elem_geometry(hipStream_t s, int n_tri, const double* xy, const int* tri,
                          double* area, double* grad);
void launch_assemble_linear(hipStream_t s, const DevLevel& L, const int* cptr, const int* contrib,
                            const double* area, const double* grad, const double* nu_e,
                            const double* sigma_e);
void launch_diag_inverse(hipStream_t s, const DevLevel& L, const int* diag_slot);
void launch_load_vectors(hipStream_t s, const DevLevel& L, const int* cptr, const int* contrib,
                         const int* diag_slot, const double* area, const int* cell_phase,
                         const int* cell_sign);

// --- batched Phi / PCG kernels (FP64) ---------------------------------------
// Column compaction of a batched CG (T = double or float vectors):
// retire: orig_x[:, gmap[c]] = x[:, c] for the columns c < cur that are
//   inactive (all of them when all_cols), gmap = identity when first;
// map: cmap = active columns in order, gmap = gmap[cmap], the CG scalars
//   (rz, rr, bb, beta) gathered in place, active = 1 for the first count
//   columns and 0 up to cur; gather: dst[:, j] = src[:, cmap[j]] for x, r, p.
void launch_compact_retire(hipStream_t s, int n, int cur, int ld, bool fp32, const uint8_t* active,
                           const int* gmap, bool first, bool all_cols, const void* x, void* orig_x);
void launch_compact_map(hipStream_t s, int cur, int64_t ld, bool first, uint8_t* active, int* cmap,
                        int* gmap, double* scal);
void launch_compact_gather(hipStream_t s, int n, int count, int64_t ld, bool fp32, const int* cmap,
                           const void* x, const void* r, const void* p, void* xd, void* rd, void* pd);

// amp / dphi: optional per-column amplitude factors and phase shifts
void launch_source_table(hipStream_t s, const SourceDev& src, double dt, int ncols,
                         const int64_t* t_list, int64_t t_base, int64_t t_stride,
                         double* table, int64_t ld, const double* amp = nullptr,
                         const double* dphi = nullptr);
void launch_axpby3(hipStream_t s, int n, int ncols, double* out, int64_t ldo, double sx,
                   CView x, double sa, CView a, double sb, CView b);
void launch_pcg_init(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, CView u_in);
// eta2 > 0 (RED_INIT, RED_IR_FIRST): a column also stops once its residual
// is below eta2 times its initial residual (squared norms).
void launch_reduce(hipStream_t s, PcgWork& w, int ncols, int mode, double tol2, int nq,
                   double* sums_out, double eta2 = 0.0);
// CG on the scaled system (pcg.hip).
// pass A: p^ = r^ + beta p^_old, partials of p^.A^p^ (flips w.parity)
void launch_pcg_pass_a(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first);
// pass B: x += alpha S p^, r^ -= alpha A^ p^, partials of r^.r^ and ||r||^2
void launch_pcg_pass_b(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols);
void launch_scale_matrix(hipStream_t s, DevLevel& L, const int* diag_slot);
// per-offset copy of A^ (L.dia_R set); *bad (device) counts entries off the stencil
void launch_build_dia(hipStream_t s, DevLevel& L, int* bad);

// FP32 inner solve of the refinement: the same two passes on r32/p32/x32.
void launch_pcg_pass_a32(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, int first);
void launch_pcg_pass_b32(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols);
// FP64 residual of a refinement sweep (and FP32 inner start), FP64 update.
void launch_ir_residual(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols, CView u_in);
void launch_ir_update(hipStream_t s, const DevLevel& L, PcgWork& w, int ncols);
void launch_fill_u8(hipStream_t s, uint8_t* p, int n, uint8_t v);

// Y = alpha * T X + beta * Y for a transfer operator (beta = 0: overwrite).
void launch_transfer(hipStream_t s, const DevTransfer& T, int ncols, CView X, double alpha,
                     double* Y, int64_t ldy, double beta);
// Sum of squares of every column: per-column partials into w.part, reduced into sums.
void launch_colsq(hipStream_t s, PcgWork& w, int n, int ncols, CView X);
// row-block partials (w.part, quantity 0) of (a - b)^T (M/dt) (a - b) per column
void launch_joule(hipStream_t s, PcgWork& w, const DevLevel& L, int ncols, CView a, CView b);

// Layout conversions.
// time-major [npts][n] (user order) <-> slabs (internal order): point t ->
// slab t % m, column t / m; internal row i is user row nat[i] (nat may be null).
void launch_tm_to_slabs(hipStream_t s, int n, int64_t npts, int m, const double* tm,
                        double* slabs, int64_t ld, int64_t slab_stride, const int* nat);
void launch_slabs_to_tm(hipStream_t s, int n, int64_t npts, int m, const double* slabs,
                        int64_t ld, int64_t slab_stride, double* tm, const int* nat);
// column block [n][lds] (column t = point t) <-> slabs.
void launch_cols_to_slabs(hipStream_t s, int n, int64_t npts, int m, const double* src,
                          int64_t lds, double* slabs, int64_t ld, int64_t slab_stride);
void launch_slabs_to_cols(hipStream_t s, int n, int64_t npts, int m, const double* slabs,
                          int64_t ld, int64_t slab_stride, double* dst, int64_t ldd);

// Columns j0 .. j0+ncols-1 of the identity as CG right-hand sides (x = 0).
void launch_cg_init_identity(hipStream_t s, const DevLevel& L, PcgWork& w, int j0, int ncols);

// Cooperative sequential stepper: steps s_begin .. s_end-1 of U[:, s] =
// Phi(U[:, s-1]) on `blocks` co-resident work-groups.  ws: [5n] doubles,
// part: [blocks*8] doubles, bar_state: coop_bar_words(blocks) zeroed unsigned; flags as for
// launch_seq_small (bit 4 of flags[1]: a grid barrier timed out).
int seq_coop_blocks();
inline size_t coop_bar_words(int blocks) { return 16 * (static_cast<size_t>(blocks) + 1); }
void launch_seq_coop(hipStream_t s, const DevLevel& L, const SourceDev& src, int s_begin,
                     int s_end, double* U, int64_t ldu, double* ws, double* part,
                     unsigned* bar_state, int* flags, double tol, int maxit, int blocks);

// Single-workgroup sequential stepper for small levels: for s = 1..nsteps,
// U[:, s] = Phi(U[:, s-1]) + G[:, s] (G may be null) by Jacobi-PCG.
void launch_seq_small(hipStream_t s, const DevLevel& L, const SourceDev& src, int nsteps,
                      int64_t t0, double* U, int64_t ldu, const double* G, int64_t ldg,
                      double* ws, double tol, int maxit, int warm, int* flags);

// ---------------------------------------------------------------------------
// Learned coarse propagator (gnn.hip).  Weight blob (FP32 master, used as
// bf16): [s_u, s_f, s_out, 0], W_in [F][64], b_in [64], per layer Ws [64][64],
// Wn [64][64], b [64], then w_out [64], b_out [1]; F = m + 7 features.
struct GnnOffsets {
  int F = 0;
  int64_t w_in = 0, b_in = 0, ws[3] = {0, 0, 0}, wn[3] = {0, 0, 0}, b[3] = {0, 0, 0};
  int64_t w_out = 0, b_out = 0, n_params = 0;
};
GnnOffsets gnn_offsets(int m);

struct GnnModel {
  int n = 0, m = 0;
  double dT = 0.0;              // coarse step
  GnnOffsets off;
  int* gptr = nullptr;          // [n+1] neighbour lists (internal numbering)
  int* gidx = nullptr;
  float* flags = nullptr;       // [n][4] conductor, iron, coil, normalised radius
  const double* F3 = nullptr;   // [3][n] phase load vectors of the level
  float* w32 = nullptr;         // [n_params] master weights
  uint16_t* wbf = nullptr;      // [n_params] bf16 copies
  float* grad = nullptr;        // [n_params]
  float *m1 = nullptr, *m2 = nullptr;   // Adam moments
  int adam_step = 0;
  bool ready = false;           // weights set or trained
  // activations (rows = n * samples)
  int64_t rows_cap = 0;
  int s_cap = 0;
  float* h[4] = {nullptr, nullptr, nullptr, nullptr};
  float* a[3] = {nullptr, nullptr, nullptr};
  float* t[3] = {nullptr, nullptr, nullptr};
  float *x = nullptr, *g0 = nullptr, *g1 = nullptr, *dz = nullptr, *y = nullptr, *dd = nullptr;
  float *part_w = nullptr, *part_b = nullptr;
  double* part_loss = nullptr;
  double* tab = nullptr;        // [S][m+1][3] source samples
  // FP64 inference workspace
  int64_t rows64_cap = 0;
  double* x64 = nullptr;
  double* h64[2] = {nullptr, nullptr};
  double* a64 = nullptr;
};

struct DeviceArena;
void gnn_alloc_rows(GnnModel& g, DeviceArena& arena, int64_t rows);
void gnn_alloc_samples(GnnModel& g, DeviceArena& arena, int S);
void gnn_alloc_rows64(GnnModel& g, DeviceArena& arena, int64_t rows);
void gnn_round_weights(hipStream_t s, GnnModel& g);
// The same network evaluated in FP64 (the propagator used inside MGRIT).
void gnn_forward64(hipStream_t s, GnnModel& g, const SourceDev& src, int S, const int64_t* k_list,
                   int64_t k_base, int64_t k_stride, const double* amp, const double* dphi, CView u,
                   CView p, double* out, int64_t ldo);
// out(i, s) = p(i, s) + s_out delta for S samples with input coarse steps
// k_list[s] (or k_base + s k_stride); keep = store activations for backward
void gnn_forward(hipStream_t s, GnnModel& g, const SourceDev& src, int S, const int64_t* k_list,
                 int64_t k_base, int64_t k_stride, const double* amp, const double* dphi,
                 CView u, CView p, double* out, int64_t ldo, bool keep);
// loss of the last forward (psi, y dense [n][S]) added to *loss_acc; gradients into g.grad
void gnn_backward(hipStream_t s, GnnModel& g, int S, const double* psi, const double* y,
                  double* loss_acc);
void gnn_adam(hipStream_t s, GnnModel& g, double lr, int step);
void gnn_gather(hipStream_t s, int n, int S, const int64_t* idx, const double* src, int64_t ld,
                double* dst);
void gnn_gather_meta(hipStream_t s, int S, const int64_t* idx, const int64_t* k_all,
                     const double* amp_all, const double* dphi_all, int64_t* k_b, double* amp_b,
                     double* dphi_b);
// B = (M/dt) u + f for ncols columns (f from the source table src[3][lds]).
void launch_ie_rhs_batch(hipStream_t s, const DevLevel& L, int ncols, const double* src, int64_t lds,
                         CView u, double* B, int64_t ld);
// Implicit Euler with a stored inverse for ncols columns: B = (M/dt) u + f
// (f from the source table src[3][lds]), X = Ainv B; B and X are [n][ld].
void launch_ie_inverse_batch(hipStream_t s, const DevLevel& L, int ncols, const double* src, int64_t lds,
                             CView u, const double* Ainv, int64_t lda, double* B, double* X,
                             int64_t ld);
// X = Ainv B for M columns of [N][ld] blocks (FP64 MFMA): X[j*ldx + c] =
// sum_k Ainv[k*lda + j] B[k*ldb + c]; part: partial sums of the k slices
// (inv_gemm_part_doubles(max columns, N) doubles), unused for wide batches.
int64_t inv_gemm_part_doubles(int max_cols, int N);
void launch_inv_gemm(hipStream_t s, int M, int N, const double* B, int64_t ldb, const double* A,
                     int64_t lda, double* X, int64_t ldx, double* part, int64_t part_size);
// y = A x for one contiguous column, A row-major [n][lda] (stored-inverse
// sequential stepping); A, lda and x 16-byte aligned.
void launch_inv_gemv(hipStream_t s, int n, const double* A, int64_t lda, const double* x, double* y);
// Y[:, b] = X[:, b] + alpha[b] (X[:, perm[b]] - X[:, b]), b < nt (Y != X)
void gnn_mix(hipStream_t s, int n, int nt, const double* X, int64_t ld, const int* perm,
             const double* alpha, double* Y);
// out[c] = sum_i (a - b)^2 (b may be null) over the n rows of column c
void gnn_colsq(hipStream_t s, int n, int ncols, const double* a, const double* b, int64_t ld,
               double* out);

}  // namespace mg
