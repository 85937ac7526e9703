// MGRIT engine and C ABI.
//
// Space-time storage of a level with N steps and coarsening factor m
// (non-coarsest level): m "slabs" [n][ld], slab j holding the points
// k*m + j (column k), so that one F-relaxation step j (all intervals at once)
// reads slab j-1 and writes slab j with coalesced column blocks; the
// C-points are slab 0 (columns 0..N/m).  The coarsest level is one column
// block [n][ld] with column t = point t.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "circuit.h"
#include "internal.h"
#include "setup.h"

namespace mg {

struct LevelState {
  DevLevel op;
  ElementData elem;
  int n = 0;
  int64_t N = 0;     // steps on this level
  int m = 0;         // temporal coarsening factor to the next level (non-coarsest levels)
  int64_t NT = 0;    // intervals (N / m) on non-coarsest levels
  bool coarsest = false;
  int prec = 0;      // arithmetic of this level's linear solves (MGRIT_FP64 / MGRIT_FP32_IR)
  int64_t ld = 0;    // column stride of the storage
  int64_t ss = 0;    // slab stride
  double* U = nullptr;
  double* G = nullptr;
  double* RES = nullptr;                          // [n][ld] C-point residual
  // warm_start = 2 (level 0): change of the input of the next F-point solve,
  // and the C-points as the previous F-relaxation started from them
  double* dlt = nullptr;
  double* csnap = nullptr;
  double *U2 = nullptr, *G2 = nullptr, *RR = nullptr;  // next level, C-point columns
  bool has_transfer = false;
  DevTransfer R, P;
  PcgWork pcg;       // batched Phi on this level (capacity N + 1 columns)
  PcgWork user;      // phi_step workspace (grown on demand)
  double* seq_ws = nullptr;
  NlLevel nl;             // element data for the nonlinear model (n_tri = 0 if linear)
  int* nat = nullptr;     // internal unknown -> user-facing index
  double* Ainv = nullptr; // coarsest level, linear model: A^{-1} [n][ld_inv]
  int64_t ld_inv = 0;
  double* bvec = nullptr; // [n] right-hand side of one coarse step
  double* u0r = nullptr;  // [n] initial value restricted to this level's mesh (nested start)
  double* nl_ws = nullptr; // persistent Newton stepper workspace (coarsest nonlinear level)
  double* nl_batch_ws = nullptr; // per-column persistent Newton workspaces of narrow batches (lazy)
  double* gemm_part = nullptr;   // partial sums of the stored-inverse product (intermediate levels)
  int64_t gemm_part_size = 0;
  // field-circuit coupling: coupling rows B^T and Z = A^-1 B^T ([n][k] each),
  // the eliminated circuit system [k][3 + k], and per-column work buffers
  // ([parts][k][c_ld] partial dots, [k][c_ld] dots and circuit unknowns)
  double* cBt = nullptr;
  double* cZ = nullptr;
  double* cS = nullptr;
  double* cpart = nullptr;
  double* cd = nullptr;
  double* cw = nullptr;
  int64_t c_ld = 0;
  double* cwt = nullptr;  // [k][c_nt]: circuit unknowns of the latest step from each time point
  int64_t c_nt = 0;
  bool relaxed = false;   // F-points hold a previous iterate (warm starts)
  bool cvalid = false;    // C-points hold a previous iterate
};

struct Handle {
  hipStream_t stream = nullptr;
  mgrit_params par{};
  mgrit_physics phys{};
  SourceDev src{};
  int m = 2;
  std::vector<LevelState> lv;
  DeviceArena arena;
  std::string last_error;
  double* tm_stage = nullptr;     // time-major staging [(N+1)][n0] (lazy)
  double* host_sums = nullptr;    // pinned [ld0]
  double* u0_dev = nullptr;       // [n0]
  double* seq_U = nullptr;        // sequential trajectory [n0][ld] (lazy)
  double* seq_ws = nullptr;
  double* seq_nl_ws = nullptr;    // persistent Newton stepper of the sequential solve (lazy)
  bool circ_guess = false;        // coupled solves start from the stored circuit unknowns
  double* seq_inv = nullptr;      // finest level's A^-1 of the stored-inverse sequential solve (lazy)
  int64_t seq_ld_inv = 0;
  double* seq_bvec = nullptr;
  int coop_blocks = 0;            // cooperative stepper (lazy)
  double* coop_ws = nullptr;
  double* coop_part = nullptr;
  unsigned* coop_bar = nullptr;
  mgrit_stats* st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> ev;     // 4 per PCG iteration of a chunk (profiling)
  std::vector<std::unique_ptr<NlWork>> nl_keep;
  // hipGraphs of one check interval of CG iterations, keyed by what the
  // captured launches depend on
  // (workspace buffers are arena allocations, never reused while the handle
  // lives, so a buffer address names one workspace)
  struct GraphKey {
    const void* x;
    const void* L;
    const void* nl;
    int rpb, cpl, dia, depth, parity, ncols, kind, chunk;
    double tol2;
    auto tie() const {
      return std::tie(x, L, nl, rpb, cpl, dia, depth, parity, ncols, kind, chunk, tol2);
    }
    bool operator<(const GraphKey& o) const { return tie() < o.tie(); }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  // learned coarse propagator on the coarsest level
  GnnModel gnn;
  bool has_gnn = false;
  bool learned_off = false;  // switched back to implicit Euler in this solve
  double* gnn_tmp = nullptr; // [n_c][ld_c] implicit-Euler part of a coarse step
  const double* col_amp = nullptr;   // per-column source amplitude factors / phase
  const double* col_dphi = nullptr;  // shifts of phi_batch (training data only)
  bool circ = false;         // field-circuit coupling (phys.circuit = 1)
  int circ_k = 0;            // circuit unknowns: 3 phase currents + bar voltages
  std::vector<double> circ_Cinv;  // level 0: inverse of the cage matrix C (host, nb x nb)
  double* circ_stage = nullptr;   // mgrit_circuit_values staging (lazy)
  bool verbose = false;      // MGRIT_VERBOSE: one line per MGRIT iteration on stderr
  int device = 0;           // HIP device the handle was set up on
  bool solved = false;      // level 0 holds the iterate of a completed mgrit_solve
  bool noalloc = false;     // inside phi_step_noalloc: no graph capture, no compaction buffers
  bool timing = false;      // a LevelTimer is running
  double tol_now = 1e-12;   // relative residual of the linear solves
  double eta_now = 0.0;     // > 0: linear solves also stop at eta times their initial residual
  hipStream_t capture_stream = nullptr;
};

static int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

constexpr int kMinRowsPerBlock = 16;
constexpr size_t kMaxGraphs = 256;       // cached CG-interval graphs per handle
constexpr int kMaxInverseN = 8192;        // largest coarsest level given a stored inverse
constexpr int kMaxInverseNCoarse = 16384; // largest intermediate level given one (coarse_inverse = 2)
constexpr int kMaxPersistentN = 16384;    // largest level given the persistent one-work-group Newton sweep
static const int kRowsPerBlockCandidates[] = {16, 32, 64, 128, 256};

static void alloc_pcg(Handle& h, PcgWork& w, int n, int cap, int rows_per_block, int prec) {
  w.n = n;
  w.cap = cap;
  w.ld = round_up(cap > 0 ? cap : 1, kWave);
  w.rows_per_block = rows_per_block;
  w.nrb = static_cast<int>((n + rows_per_block - 1) / rows_per_block);
  const int nrb_max = static_cast<int>((n + kMinRowsPerBlock - 1) / kMinRowsPerBlock);
  const size_t vec = static_cast<size_t>(n) * w.ld;
  w.x = h.arena.alloc<double>(vec);
  w.r = h.arena.alloc<double>(vec);
  w.pbuf[0] = h.arena.alloc<double>(vec);
  w.pbuf[1] = h.arena.alloc<double>(vec);
  w.parity = 0;
  w.hist_cap = h.par.pcg_max_iter + 64;
  w.hist = h.arena.alloc<int>(w.hist_cap);
  w.host_hist = static_cast<int*>(h.arena.alloc_host(sizeof(int) * w.hist_cap));
  w.part = h.arena.alloc<double>(3 * static_cast<size_t>(std::max(w.nrb, nrb_max)) * w.ld);
  w.scal = h.arena.alloc<double>(8 * static_cast<size_t>(w.ld));
  w.src = h.arena.alloc<double>(3 * static_cast<size_t>(w.ld));
  w.active = h.arena.alloc<uint8_t>(w.ld);
  w.outer = h.arena.alloc<uint8_t>(w.ld);
  w.prec = prec;
  if (prec == MGRIT_FP32_IR) {
    w.r32 = h.arena.alloc<float>(vec);
    w.x32 = h.arena.alloc<float>(vec);
    w.p32[0] = h.arena.alloc<float>(vec);
    w.p32[1] = h.arena.alloc<float>(vec);
  }
  w.flags = h.arena.alloc<int>(8);
  w.host_flags = static_cast<int*>(h.arena.alloc_host(8 * sizeof(int)));
  MG_HIP(hipMemsetAsync(w.flags, 0, 8 * sizeof(int), h.stream));
}


static int rows_per_block_for(int n) {
  (void)n;
  return 64;
}

static void set_rows_per_block(PcgWork& w, int rpb) {
  w.rows_per_block = rpb;
  w.nrb = (w.n + rpb - 1) / rpb;
}

// Autotuner: time pass A + pass B of the batched PCG on the level's own
// matrix with every column active, for each candidate rows-per-work-group,
// and keep the fastest.  Results are cached per (n, W, columns, precision)
// for the life of the process.
struct TuneKey {
  int n, W, cols, prec, dia, depth, narrow, rpb, cpl;
  bool operator<(const TuneKey& o) const {
    return std::tie(n, W, cols, prec, dia, depth, narrow, rpb, cpl) <
           std::tie(o.n, o.W, o.cols, o.prec, o.dia, o.depth, o.narrow, o.rpb, o.cpl);
  }
};
struct TuneChoice {
  int rpb, cpl;
  bool dia;
  int depth, rpb_narrow;
};
// Once at most this many columns of a batched CG still iterate, its passes
// switch to the narrow rows-per-work-group choice: a wave's walk over its rows
// is a chain of dependent loads, so with few columns a launch is as long as
// the walk, and shorter walks in more work-groups finish sooner.
constexpr int kNarrowCols = 128;
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;

static void autotune(Handle& h, LevelState& S) {
  PcgWork& w = S.pcg;
  const int ncols = w.cap;
  w.dia = (h.par.pcg_kernel == 2);
  const int forced_depth = h.par.pcg_prefetch;
  w.depth = forced_depth > 0 ? forced_depth : 1;
  const int forced_narrow = h.par.pcg_rows_narrow;
  w.rpb_narrow = forced_narrow > 0 ? forced_narrow : 0;
  const int forced_rpb = h.par.pcg_rows_per_block, forced_cpl = h.par.pcg_cols_per_lane;
  if (forced_rpb > 0) set_rows_per_block(w, forced_rpb);
  if (forced_cpl > 0) w.cpl = forced_cpl;
  if (!h.par.autotune || S.n < 4096 || ncols < kWave) {
    if (w.cpl == 2 && !w.dia && S.op.W != 8)
      fail(MGRIT_INVALID_ARGUMENT, "two columns per lane need the 8-wide row family or the diagonal window");
    return;
  }
  const bool fp32 = w.prec == MGRIT_FP32_IR;
  const TuneKey key{S.n, S.op.W, ncols, w.prec, S.op.dia_R * 4 + h.par.pcg_kernel, forced_depth,
                    forced_narrow, forced_rpb, forced_cpl};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      set_rows_per_block(w, it->second.rpb);
      w.cpl = it->second.cpl;
      w.dia = it->second.dia;
      w.depth = it->second.depth;
      w.rpb_narrow = it->second.rpb_narrow;
      return;
    }
  }
  hipStream_t s = h.stream;
  const size_t vec = static_cast<size_t>(S.n) * w.ld;
  if (fp32) {
    MG_HIP(hipMemsetAsync(w.r32, 0, sizeof(float) * vec, s));
    MG_HIP(hipMemsetAsync(w.x32, 0, sizeof(float) * vec, s));
    MG_HIP(hipMemsetAsync(w.p32[0], 0, sizeof(float) * vec, s));
    MG_HIP(hipMemsetAsync(w.p32[1], 0, sizeof(float) * vec, s));
  } else {
    MG_HIP(hipMemsetAsync(w.r, 0, sizeof(double) * vec, s));
    MG_HIP(hipMemsetAsync(w.x, 0, sizeof(double) * vec, s));
    MG_HIP(hipMemsetAsync(w.pbuf[0], 0, sizeof(double) * vec, s));
    MG_HIP(hipMemsetAsync(w.pbuf[1], 0, sizeof(double) * vec, s));
  }
  MG_HIP(hipMemsetAsync(w.scal, 0, sizeof(double) * 8 * w.ld, s));
  launch_fill_u8(s, w.active, ncols, 1);
  const int reps = 4;
  float best = 1e30f;
  int best_rpb = w.rows_per_block, best_cpl = 1, best_depth = 1;
  bool best_dia = false;
  const int nr = static_cast<int>(sizeof(kRowsPerBlockCandidates) / sizeof(int));
  static const int kDepths[3] = {1, 2, 4};
  for (int cand = 0; cand < 4 * nr * 3; ++cand) {
    const int rpb = kRowsPerBlockCandidates[cand % nr];
    const int cpl = 1 + ((cand / nr) & 1);
    const bool dia = ((cand / (2 * nr)) & 1) != 0;
    const int depth = kDepths[cand / (4 * nr)];
    if (dia && S.op.dia_R == 0) continue;
    if ((dia && h.par.pcg_kernel == 1) || (!dia && h.par.pcg_kernel == 2)) continue;
    if (!dia && cpl == 2 && S.op.W != 8) continue;
    // depth applies to the diagonal-window family and needs rows to walk
    if ((!dia || depth > rpb / 4) && depth != 1) continue;
    if (forced_depth > 0 && dia && depth != forced_depth) continue;
    if ((forced_rpb > 0 && rpb != forced_rpb) || (forced_cpl > 0 && cpl != forced_cpl)) continue;
    set_rows_per_block(w, rpb);
    w.cpl = cpl;
    w.dia = dia;
    w.depth = depth;
    for (int warm = 0; warm < 2; ++warm) {
      if (warm) MG_HIP(hipEventRecord(h.ev0, s));
      for (int r = 0; r < reps; ++r) {
        // one CG iteration as the solver runs it (the reduces only sum
        // partials here: every column stays active with alpha = beta = 0)
        if (fp32) launch_pcg_pass_a32(s, S.op, w, ncols, 0);
        else launch_pcg_pass_a(s, S.op, w, ncols, 0);
        launch_reduce(s, w, ncols, RED_SUM, 0.0, 1, w.scal + 6 * w.ld);
        if (fp32) launch_pcg_pass_b32(s, S.op, w, ncols);
        else launch_pcg_pass_b(s, S.op, w, ncols);
        launch_reduce(s, w, ncols, RED_SUM, 0.0, 2, w.scal + 6 * w.ld);
      }
    }
    MG_HIP(hipEventRecord(h.ev1, s));
    MG_HIP(hipEventSynchronize(h.ev1));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, h.ev0, h.ev1));
    if (ms < best) {
      best = ms;
      best_rpb = rpb;
      best_cpl = cpl;
      best_dia = dia;
      best_depth = depth;
    }
    if (std::getenv("MGRIT_TUNE_LOG")) {
      const double unit = fp32 ? 4.0 : 8.0;
      const double bytes = 8.0 * unit * S.n * static_cast<double>(ncols);  // A + B vector passes
      std::fprintf(stderr, "[mgrit tune] n=%d cols=%d %s %s rpb=%d cpl=%d depth=%d: iteration %.1f us, %.0f GB/s\n",
                   S.n, ncols, fp32 ? "fp32" : "fp64", dia ? "diag" : "ell", rpb, cpl, depth,
                   1e3 * ms / reps, bytes / (1e-3 * ms / reps) / 1e9);
    }
  }
  w.parity = 0;
  set_rows_per_block(w, best_rpb);
  w.cpl = best_cpl;
  w.dia = best_dia;
  w.depth = best_dia ? best_depth : 1;
  // narrow column sets: the same kernels with shorter walks
  w.rpb_narrow = forced_narrow > 0 ? forced_narrow : 0;
  if (forced_narrow == 0 && ncols > kNarrowCols) {
    float best_n = 1e30f;
    for (int rpb : kRowsPerBlockCandidates) {
      if (rpb > best_rpb || rpb / 4 < w.depth) continue;
      set_rows_per_block(w, rpb);
      for (int warm = 0; warm < 2; ++warm) {
        if (warm) MG_HIP(hipEventRecord(h.ev0, s));
        for (int r = 0; r < reps; ++r) {
          if (fp32) launch_pcg_pass_a32(s, S.op, w, kNarrowCols, 0);
          else launch_pcg_pass_a(s, S.op, w, kNarrowCols, 0);
          launch_reduce(s, w, kNarrowCols, RED_SUM, 0.0, 1, w.scal + 6 * w.ld);
          if (fp32) launch_pcg_pass_b32(s, S.op, w, kNarrowCols);
          else launch_pcg_pass_b(s, S.op, w, kNarrowCols);
          launch_reduce(s, w, kNarrowCols, RED_SUM, 0.0, 2, w.scal + 6 * w.ld);
        }
      }
      MG_HIP(hipEventRecord(h.ev1, s));
      MG_HIP(hipEventSynchronize(h.ev1));
      float ms = 0.f;
      MG_HIP(hipEventElapsedTime(&ms, h.ev0, h.ev1));
      if (std::getenv("MGRIT_TUNE_LOG"))
        std::fprintf(stderr, "[mgrit tune] n=%d narrow cols=%d rpb=%d: iteration %.1f us\n", S.n,
                     kNarrowCols, rpb, 1e3 * ms / reps);
      if (ms < best_n) {
        best_n = ms;
        w.rpb_narrow = rpb;
      }
    }
    if (w.rpb_narrow == best_rpb) w.rpb_narrow = 0;
    set_rows_per_block(w, best_rpb);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = {best_rpb, best_cpl, best_dia, w.depth, w.rpb_narrow};
}

// ---------------------------------------------------------------------------
// Batched PCG iterations on an initialised state (after a reduce that set
// rz, the reference norms and the active flags; `active` columns remain).
// Each iteration is pass A, reduce (alpha), pass B, reduce (beta,
// convergence); converged columns drop out of every kernel.  The host reads
// the active-column count every pcg_check_every iterations.  Returns the
// number of iterations in which some column was active.
enum IterKind { IT_LIN64 = 0, IT_LIN32 = 1, IT_JAC = 2 };

static void ensure_compaction_buffers(Handle& h, PcgWork& w) {
  if (w.gmap) return;
  const size_t bytes = sizeof(double) * static_cast<size_t>(w.n) * w.ld;   // large enough for either type
  for (int st = 0; st < 2; ++st) {
    w.alt_x[st] = h.arena.alloc_bytes(bytes);
    w.alt_r[st] = h.arena.alloc_bytes(bytes);
    w.alt_p[st][0] = h.arena.alloc_bytes(bytes);
    w.alt_p[st][1] = h.arena.alloc_bytes(bytes);
  }
  w.gmap = h.arena.alloc<int>(w.ld);
  w.cmap = h.arena.alloc<int>(w.ld);
}

static int pcg_iterate(Handle& h, int level, const DevLevel& L, PcgWork& w, int ncols, double tol2,
                       int kind, int active, bool fail_at_cap, int max_iter = -1) {
  hipStream_t s = h.stream;
  const bool prof = h.par.profile_kernels && h.st && level < MGRIT_MAX_LEVELS;
  int it = 0, used = 0;
  // narrow batches (coarse levels) gain nothing from compaction checks, and
  // every check is a device-to-host round trip: check less often
  const int every = (ncols <= kNarrowCols && h.par.pcg_check_narrow > 0) ? h.par.pcg_check_narrow
                                                                         : h.par.pcg_check_every;
  const int chunk = std::max(1, std::min(every > 0 ? every : 16, static_cast<int>(h.ev.size() / 4)));
  const int cap = std::min(max_iter > 0 ? max_iter : h.par.pcg_max_iter, w.hist_cap);
  int64_t cols = 0, launches = 0;
  w.parity = 0;
  // Column compaction: once at most compact_fraction of the current columns iterate,
  // converged columns hand their x back to the caller's buffer and the rest
  // are gathered densely into an alternate buffer set (each column's
  // arithmetic does not depend on its position, so the iterates are the
  // same).  set = -1: the caller's buffers; 0 / 1: alternate sets.
  const bool fp32 = (kind == IT_LIN32);
  const bool can_compact = h.par.compact_columns > 0 && kind != IT_JAC && !h.noalloc;
  void* ox = fp32 ? static_cast<void*>(w.x32) : static_cast<void*>(w.x);
  void* orr = fp32 ? static_cast<void*>(w.r32) : static_cast<void*>(w.r);
  void* op0 = fp32 ? static_cast<void*>(w.p32[0]) : static_cast<void*>(w.pbuf[0]);
  void* op1 = fp32 ? static_cast<void*>(w.p32[1]) : static_cast<void*>(w.pbuf[1]);
  int set = -1, cur = ncols;
  auto vx = [&](int st) { return st < 0 ? ox : w.alt_x[st]; };
  auto vr = [&](int st) { return st < 0 ? orr : w.alt_r[st]; };
  auto vp = [&](int st, int k) { return st < 0 ? (k ? op1 : op0) : w.alt_p[st][k]; };
  auto point = [&](int st) {
    if (fp32) {
      w.x32 = static_cast<float*>(vx(st));
      w.r32 = static_cast<float*>(vr(st));
      w.p32[0] = static_cast<float*>(vp(st, 0));
      w.p32[1] = static_cast<float*>(vp(st, 1));
    } else {
      w.x = static_cast<double*>(vx(st));
      w.r = static_cast<double*>(vr(st));
      w.pbuf[0] = static_cast<double*>(vp(st, 0));
      w.pbuf[1] = static_cast<double*>(vp(st, 1));
    }
  };
  const int rpb_full = w.rows_per_block;
  struct Restore {
    std::function<void()> f;
    ~Restore() { f(); }
  } restore{[&] {
    point(-1);
    if (w.rows_per_block != rpb_full) set_rows_per_block(w, rpb_full);
  }};
  while (active > 0) {
    if (it >= cap) {
      if (fail_at_cap)
        fail(MGRIT_PCG_NOT_CONVERGED, "PCG did not converge in pcg_max_iter iterations (" +
                                          std::to_string(active) + " columns left)");
      break;
    }
    const int k = std::min(chunk, cap - it);
    // Later check intervals replay a captured graph of the same k launches
    // (the first carries the `first` iteration and runs eagerly).  HIP events
    // recorded inside a graph do not time its kernels reliably, so profiled
    // solves launch eagerly; compacted column sets change every interval.
    const bool graph = h.par.use_graphs && !prof && !h.noalloc && set < 0 && it > 0 && k == chunk &&
                       (chunk % 2) == 0;
    if (graph) {
      const Handle::GraphKey key{w.x, &L, w.nl, w.rows_per_block, w.cpl, w.dia ? 1 : 0, w.depth, w.parity,
                                 cur, kind, chunk, tol2};
      auto found = h.graphs.find(key);
      if (found == h.graphs.end()) {
        if (h.graphs.size() >= kMaxGraphs) {   // many distinct shapes: start over
          MG_HIP(hipStreamSynchronize(s));
          for (auto& g : h.graphs) (void)hipGraphExecDestroy(g.second);
          h.graphs.clear();
        }
        hipStream_t cs = h.capture_stream;
        MG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int keep_parity = w.parity;
        for (int t = 0; t < k; ++t) {
          if (kind == IT_JAC) launch_nl_pass_a(cs, L, w, *w.nl, cur, 0);
          else if (kind == IT_LIN32) launch_pcg_pass_a32(cs, L, w, cur, 0);
          else launch_pcg_pass_a(cs, L, w, cur, 0);
          launch_reduce(cs, w, cur, RED_ALPHA, tol2, 1, nullptr);
          if (kind == IT_JAC) launch_nl_pass_b(cs, L, w, *w.nl, cur);
          else if (kind == IT_LIN32) launch_pcg_pass_b32(cs, L, w, cur);
          else launch_pcg_pass_b(cs, L, w, cur);
          launch_reduce(cs, w, cur, RED_BETA, tol2, 2, nullptr);
        }
        w.parity = keep_parity;
        hipGraph_t g = nullptr;
        MG_HIP(hipStreamEndCapture(cs, &g));
        hipGraphExec_t ex = nullptr;
        MG_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        MG_HIP(hipGraphDestroy(g));
        found = h.graphs.emplace(key, ex).first;
      }
      MG_HIP(hipGraphLaunch(found->second, s));
    }
    for (int t = 0; t < k && !graph; ++t) {
      if (prof) MG_HIP(hipEventRecord(h.ev[4 * t], s));
      if (kind == IT_JAC) launch_nl_pass_a(s, L, w, *w.nl, cur, it + t == 0);
      else if (kind == IT_LIN32) launch_pcg_pass_a32(s, L, w, cur, it + t == 0);
      else launch_pcg_pass_a(s, L, w, cur, it + t == 0);
      if (prof) MG_HIP(hipEventRecord(h.ev[4 * t + 1], s));
      launch_reduce(s, w, cur, RED_ALPHA, tol2, 1, nullptr);
      if (prof) MG_HIP(hipEventRecord(h.ev[4 * t + 2], s));
      if (kind == IT_JAC) launch_nl_pass_b(s, L, w, *w.nl, cur);
      else if (kind == IT_LIN32) launch_pcg_pass_b32(s, L, w, cur);
      else launch_pcg_pass_b(s, L, w, cur);
      if (prof) MG_HIP(hipEventRecord(h.ev[4 * t + 3], s));
      launch_reduce(s, w, cur, RED_BETA, tol2, 2, nullptr);
    }
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipMemcpyAsync(w.host_hist, w.hist + it, sizeof(int) * k, hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (w.host_flags[1]) fail(MGRIT_NONFINITE, "non-finite value in a linear solve");
    for (int t = 0; t < k; ++t) {
      const int a = w.host_hist[t];
      if (a > 0) {
        ++used;
        cols += a;
      }
      if (prof) {
        float ta = 0.f, tb = 0.f;
        MG_HIP(hipEventElapsedTime(&ta, h.ev[4 * t], h.ev[4 * t + 1]));
        MG_HIP(hipEventElapsedTime(&tb, h.ev[4 * t + 2], h.ev[4 * t + 3]));
        h.st->kernel_time_s[0][level] += 1e-3 * ta;
        h.st->kernel_time_s[1][level] += 1e-3 * tb;
      }
    }
    launches += k;
    it += k;
    active = w.host_flags[0];
    // few columns left: shorter walks (decided by the active count alone, so
    // that runs with and without compaction take the same partial sums)
    if (w.rpb_narrow > 0 && w.rows_per_block != w.rpb_narrow && active <= kNarrowCols)
      set_rows_per_block(w, w.rpb_narrow);
    if (can_compact && active > 0 && it < cap &&
        static_cast<double>(active) <= h.par.compact_fraction * cur && cur - active >= h.par.compact_columns) {
      ensure_compaction_buffers(h, w);
      const bool first = set < 0;
      if (!first) launch_compact_retire(s, w.n, cur, static_cast<int>(w.ld), fp32, w.active, w.gmap,
                                        false, false, vx(set), ox);
      launch_compact_map(s, cur, w.ld, first, w.active, w.cmap, w.gmap, w.scal);
      const int nxt = first ? 0 : (set ^ 1);
      launch_compact_gather(s, w.n, active, w.ld, fp32, w.cmap, vx(set), vr(set), vp(set, w.parity),
                            vx(nxt), vr(nxt), vp(nxt, w.parity));
      set = nxt;
      point(set);
      cur = active;
    }
  }
  if (set >= 0)
    launch_compact_retire(s, w.n, cur, static_cast<int>(w.ld), fp32, w.active, w.gmap, false, true, vx(set),
                          ox);
  if (h.st && level < MGRIT_MAX_LEVELS) {
    h.st->kernel_launches[0][level] += launches;
    h.st->kernel_launches[1][level] += launches;
    h.st->kernel_columns[level] += cols;
  }
  return used;
}

// Solves (M/dt + K) x = (M/dt) u_in + f(t) for every column, x initialised in
// w.x, to ||b - A x|| <= pcg_tol ||b||.
//  FP64:     Jacobi-PCG in FP64.
//  FP32_IR:  refinement sweeps: r = b - A x in FP64; if not converged, solve
//            A d = r by FP32 Jacobi-PCG to ir_inner_tol (relative), x += d.
static int pcg_solve(Handle& h, int level, const DevLevel& L, PcgWork& w, int ncols, CView in) {
  hipStream_t s = h.stream;
  const double tol2 = h.tol_now * h.tol_now;
  const double eta2 = h.eta_now * h.eta_now;
  if (w.prec == MGRIT_FP64) {
    launch_pcg_init(s, L, w, ncols, in);
    launch_reduce(s, w, ncols, RED_INIT, tol2, 3, nullptr, eta2);
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (w.host_flags[1]) fail(MGRIT_NONFINITE, "non-finite value in a linear solve");
    return pcg_iterate(h, level, L, w, ncols, tol2, IT_LIN64, w.host_flags[0], true);
  }
  // inner FP32 tolerance: ir_inner_tol, or the reduction the outer test asks
  // for when that is looser (half of eta, so one sweep normally suffices)
  const double tin = std::min(0.1, std::max(h.par.ir_inner_tol, 0.5 * h.eta_now));
  const double tin2 = tin * tin;
  launch_fill_u8(s, w.outer, ncols, 1);
  int total = 0;
  for (int sweep = 0;; ++sweep) {
    launch_ir_residual(s, L, w, ncols, in);
    launch_reduce(s, w, ncols, sweep == 0 ? RED_IR_FIRST : RED_IR_INIT, tol2, 3, nullptr, eta2);
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (w.host_flags[1]) fail(MGRIT_NONFINITE, "non-finite value in a linear solve");
    const int active = w.host_flags[0];
    if (active == 0) break;
    if (sweep >= h.par.ir_max_iter)
      fail(MGRIT_PCG_NOT_CONVERGED, "iterative refinement did not converge in ir_max_iter sweeps (" +
                                        std::to_string(active) + " columns left)");
    total += pcg_iterate(h, level, L, w, ncols, tin2, IT_LIN32, active, false);
    launch_ir_update(s, L, w, ncols);
  }
  return total;
}

// Newton buffers of a workspace (allocated on first use).
static NlWork& nl_work(Handle& h, LevelState& S, PcgWork& w) {
  if (w.nl) return *w.nl;
  auto* nw = new NlWork();
  h.nl_keep.emplace_back(nw);
  nw->fp32 = (w.prec == MGRIT_FP32_IR);
  // the symmetric Jacobian by offset (upper half, 4 values per row) on the
  // periodic polar stencil, unless the general sparse-row kernels are forced
  nw->dia_R = (h.par.pcg_kernel != 1) ? S.op.dia_R : 0;
  const size_t ev = static_cast<size_t>(S.nl.n_tri) * w.ld;
  const size_t vec = static_cast<size_t>(w.n) * w.ld;
  const size_t mat = vec * (nw->dia_R > 0 ? 4 : S.op.W);
  nw->nu = h.arena.alloc<double>(ev);
  nw->dnu = h.arena.alloc<double>(ev);
  nw->gx = h.arena.alloc<double>(ev);
  nw->gy = h.arena.alloc<double>(ev);
  nw->R = h.arena.alloc<double>(vec);
  nw->dg = h.arena.alloc<double>(vec);
  nw->ref = h.arena.alloc<double>(w.ld);
  nw->rcur = h.arena.alloc<double>(w.ld);
  nw->lam = h.arena.alloc<double>(w.ld);
  nw->fac = h.arena.alloc<double>(w.ld);
  nw->ls = h.arena.alloc<uint8_t>(w.ld);
  if (nw->fp32) {
    nw->J32 = h.arena.alloc<float>(mat);
    nw->s32 = h.arena.alloc<float>(vec);
  } else {
    nw->J64 = h.arena.alloc<double>(mat);
    nw->s64 = h.arena.alloc<double>(vec);
    nw->r64 = h.arena.alloc<double>(vec);
    nw->p64[0] = h.arena.alloc<double>(vec);
    nw->p64[1] = h.arena.alloc<double>(vec);
    nw->d64 = h.arena.alloc<double>(vec);
  }
  w.nl = nw;
  return *nw;
}

// Batched Newton (saturating iron): x (= w.x, initialised with the guess)
// is driven to ||R(x)|| <= newton_tol ||R(u_prev)|| per column.  Each step
// assembles the per-column Jacobian, solves J d = -R by CG on the Jacobi-
// scaled Jacobian to ir_inner_tol (FP32 for MGRIT_FP32_IR, else FP64) and
// updates x in FP64.  Returns the number of inner CG iterations.
static int newton_solve(Handle& h, int level, LevelState& S, PcgWork& w, int ncols, CView in,
                        bool guess_is_input) {
  hipStream_t s = h.stream;
  NlWork& nw = nl_work(h, S, w);
  const double tol2 = h.par.newton_tol * h.par.newton_tol;
  // inexact Newton: one step with a relative inner tolerance tau cuts the
  // residual by about tau, so a solve that stops at eta times its warm-start
  // residual needs no inner tolerance below eta / 2 (as for the refinement)
  const double tin = h.eta_now > 0.0 ? std::min(0.1, std::max(h.par.ir_inner_tol, 0.5 * h.eta_now))
                                      : h.par.ir_inner_tol;
  const double tin2 = tin * tin;
  const double lam_min = std::ldexp(1.0, -h.par.newton_halvings);
  // reference ||R(u_prev)||
  launch_nl_elem(s, S.nl, ncols, w.ld, nullptr, in, nw);
  launch_nl_residual(s, S.op, S.nl, w, nw, ncols, nullptr, in, in);
  // level-0 relaxation with pcg_tol_eta: Newton also stops at eta times the
  // residual of its warm start
  const double eta2 = h.eta_now * h.eta_now;
  launch_nl_test(s, w, nw, ncols, 1, tol2, guess_is_input ? eta2 : 0.0);
  if (!guess_is_input) {
    launch_nl_elem(s, S.nl, ncols, w.ld, w.outer, CView{w.x, w.ld}, nw);
    launch_nl_residual(s, S.op, S.nl, w, nw, ncols, w.outer, CView{w.x, w.ld}, in);
    launch_nl_test(s, w, nw, ncols, 0, tol2, eta2);
  }
  auto read_count = [&]() {
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (w.host_flags[1]) fail(MGRIT_NONFINITE, "non-finite value in a Newton step");
    return w.host_flags[0];
  };
  int refining = read_count();
  int inner = 0;
  for (int k = 0; refining > 0; ++k) {
    if (k >= h.par.newton_max_iter)
      fail(MGRIT_NEWTON_NOT_CONVERGED, "Newton did not converge in newton_max_iter iterations (" +
                                           std::to_string(refining) + " columns left)");
    launch_nl_jacobian(s, S.op, S.nl, w, nw, ncols);
    launch_nl_cg_init(s, w, nw, ncols);
    launch_reduce(s, w, ncols, RED_INIT, tin2, 3, nullptr);
    const int act = read_count();
    inner += pcg_iterate(h, level, S.op, w, ncols, tin2, IT_JAC, act, false);
    // damped update: per column, halve the step until the residual norm
    // decreases enough (at most newton_halvings times)
    launch_nl_ls_start(s, w, nw, ncols);
    while (true) {
      launch_nl_update(s, w, nw, ncols);
      launch_nl_elem(s, S.nl, ncols, w.ld, nw.ls, CView{w.x, w.ld}, nw);
      launch_nl_residual(s, S.op, S.nl, w, nw, ncols, nw.ls, CView{w.x, w.ld}, in);
      launch_nl_ls(s, w, nw, ncols, tol2, lam_min);
      if (read_count() == 0) break;
    }
    refining = w.host_flags[3];
    if (h.st && level < MGRIT_MAX_LEVELS) h.st->newton_sweeps[level] += 1;
  }
  return inner;
}

// Narrow batches on the coarse levels of the nonlinear model, on request
// (coarse_persistent = 1): one persistent work-group per column runs the
// column's whole damped Newton solve (every Newton, CG and step-length
// iteration on the device), the same per-column solver as the coarsest
// level's sequential sweep.  Measured on the nonlinear 64x512 workload
// (8192 steps, 16-column batches on 32x256) it is slower than the batched
// kernels (16.9 s against 11.0 s on that level): a column's CG then streams
// through one compute unit, and 16 columns leave most of the chip idle.
constexpr int kNarrowPersistentCols = 256;

static bool narrow_persistent(const Handle& h, int l, const LevelState& S, int ncols) {
  return S.nl.n_tri > 0 && l > 0 && ncols <= kNarrowPersistentCols && !h.noalloc && !h.col_amp &&
         !h.col_dphi && h.eta_now == 0.0 && h.par.coarse_persistent == 1;
}

// x[:, c] (start on entry, result on exit) = Phi(u_in[:, c]); returns the CG
// iterations summed over the columns.
static int newton_narrow(Handle& h, int l, LevelState& S, PcgWork& w, int ncols, CView in,
                         const int64_t* t_list, int64_t t_base, int64_t t_stride) {
  hipStream_t s = h.stream;
  const int64_t per = seq_newton_ws_doubles(S.n, S.op.W, S.nl.n_tri);
  if (!S.nl_batch_ws)
    S.nl_batch_ws = h.arena.alloc<double>(static_cast<size_t>(per) * kNarrowPersistentCols);
  MG_HIP(hipMemsetAsync(w.flags, 0, 4 * sizeof(int), s));
  launch_seq_newton_batch(s, S.op, S.nl, h.src, ncols, in, w.x, w.ld, t_list, t_base, t_stride,
                          h.par.newton_tol, h.par.newton_max_iter, std::ldexp(1.0, -h.par.newton_halvings),
                          h.par.ir_inner_tol, h.par.pcg_max_iter, S.nl_batch_ws, w.flags);
  MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  const int bits = w.host_flags[1];
  if (bits & 1) fail(MGRIT_NONFINITE, "non-finite value in a Newton step");
  if (bits & 8) fail(MGRIT_NEWTON_NOT_CONVERGED, "Newton did not converge in newton_max_iter iterations");
  if (bits & 2) fail(MGRIT_PCG_NOT_CONVERGED, "an inner CG of a Newton step hit pcg_max_iter");
  if (h.st && l < MGRIT_MAX_LEVELS) h.st->newton_sweeps[l] += w.host_flags[3];
  return w.host_flags[2];
}

// One batched application of Phi on level l:
//   x = Phi(u_in[:, c]) for c < ncols, input time index t_base + c*t_stride
//   (or t_list[c]), initial guess x0 = ga + sgb * gb,
//   out = osx * x + oa + osb * ob.
struct PhiCall {
  int ncols = 0;
  CView in;
  const int64_t* t_list = nullptr;
  int64_t t_base = 0, t_stride = 1;
  CView ga, gb;
  double sgb = 0.0;
  double* out = nullptr;
  int64_t ldo = 0;
  double osx = 1.0;
  CView oa, ob;
  double osb = 0.0;
  double* dout = nullptr;   // if set: dout = x - out (before out is written), ld = ldo
};

// profile_kernels = 1: wall time of a level's Phi applications (and of the
// coarsest sequential solve) with the stream drained on entry and exit; the
// outermost timer of a nest counts.
struct LevelTimer {
  Handle& h;
  int l;
  bool on;
  std::chrono::steady_clock::time_point t0;
  LevelTimer(Handle& hh, int ll)
      : h(hh), l(ll), on(hh.par.profile_kernels && hh.st && ll < MGRIT_MAX_LEVELS && !hh.timing) {
    if (!on) return;
    h.timing = true;
    MG_HIP(hipStreamSynchronize(h.stream));
    t0 = std::chrono::steady_clock::now();
  }
  ~LevelTimer() {
    if (!on) return;
    h.timing = false;
    if (hipStreamSynchronize(h.stream) != hipSuccess) return;
    h.st->time_phi_s[l] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static void circuit_buffers(Handle& h, LevelState& S, int ncols) {
  if (S.c_ld >= ncols) return;
  const int64_t ld = round_up(std::max<int64_t>(ncols, S.pcg.cap), kWave);
  const size_t k = static_cast<size_t>(h.circ_k);
  S.cpart = h.arena.alloc<double>(static_cast<size_t>(circ_parts(S.n)) * k * ld);
  S.cd = h.arena.alloc<double>(k * ld);
  S.cw = h.arena.alloc<double>(k * ld);
  S.c_ld = ld;
}

// a' = y + Z w, w = S^-1 (v(t'); 0) - S^-1 (l_z/dt) E B (y - u_in) per column
// (y[:, c] at y[i * ldy + c] on entry, a' on exit; the phase voltages are the
// source table src[q * lds + c]).
// inexact = true: y comes from an iterative solve, and the dots take its
// residual into account (Z^T r), so that the error of the solve is not
// multiplied by the elimination.
static void circuit_eliminate(Handle& h, LevelState& S, int ncols, double* y, int64_t ldy, CView in,
                              const double* src, int64_t lds, bool inexact = false) {
  hipStream_t s = h.stream;
  circuit_buffers(h, S, ncols);
  const int k = h.circ_k;
  if (inexact)
    launch_circ_dots_res(s, S.op, k, ncols, S.cBt, S.cZ, CView{y, ldy}, in, S.cpart, S.c_ld);
  else
    launch_circ_dots(s, S.n, k, ncols, S.cBt, CView{y, ldy}, in, S.cpart, S.c_ld);
  launch_circ_sum(s, k, ncols, circ_parts(S.n), S.cpart, S.c_ld, S.cd, S.c_ld);
  launch_circ_solve(s, k, ncols, S.cd, S.c_ld, src, lds, S.cS, S.cw, S.c_ld);
  launch_circ_apply(s, S.n, k, ncols, S.cZ, S.cw, S.c_ld, y, ldy);
}

static void circuit_step(Handle& h, LevelState& S, PcgWork& w, const PhiCall& c) {
  circuit_eliminate(h, S, c.ncols, w.x, w.ld, c.in, w.src, w.ld, S.Ainv == nullptr);
  if (h.circ_guess)
    launch_circ_keep(h.stream, h.circ_k, c.ncols, c.t_list, c.t_base, c.t_stride, S.cw, S.c_ld, S.cwt,
                     S.c_nt);
}

// Start of a coupled step's linear solve inside an MGRIT solve.  The solve
// is for y = a' - Z w, and its guess x0 is one of a' (the previous iterate at
// the same time point, plus the change of its input).  With the circuit
// unknowns w0 of the latest step from that point, y starts from x0 - Z w0:
// its start residual then shrinks as MGRIT converges, as in the uncoupled
// model, instead of holding the circuits' field A Z w0 = B^T w0, so a stop
// at eta times the start residual tightens with the iterations.
static void circuit_guess(Handle& h, LevelState& S, PcgWork& w, const PhiCall& c) {
  if (!h.circ_guess) return;
  circuit_buffers(h, S, c.ncols);
  launch_circ_recall(h.stream, h.circ_k, c.ncols, c.t_list, c.t_base, c.t_stride, S.cwt, S.c_nt, S.cw,
                     S.c_ld);
  launch_circ_apply(h.stream, S.n, h.circ_k, c.ncols, S.cZ, S.cw, S.c_ld, w.x, w.ld);
}

static void phi_batch(Handle& h, int l, PcgWork& w, const PhiCall& c) {
  if (c.ncols <= 0) return;
  LevelTimer timer(h, l);
  if (c.ncols > w.cap) fail(MGRIT_INVALID_ARGUMENT, "batched Phi wider than its workspace");
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  launch_source_table(s, h.src, S.op.dt, c.ncols, c.t_list, c.t_base, c.t_stride, w.src, w.ld,
                      h.col_amp, h.col_dphi);
  int it = 0;
  if (S.Ainv && S.coarsest) {
    // coarsest linear level: the stored inverse, the same kernels (and bits)
    // as its sequential solve
    launch_ie_inverse_batch(s, S.op, c.ncols, w.src, w.ld, c.in, S.Ainv, S.ld_inv, w.r, w.x, w.ld);
  } else if (S.Ainv) {
    // intermediate linear level: right-hand sides, then X = Ainv B on the
    // FP64 matrix cores
    launch_ie_rhs_batch(s, S.op, c.ncols, w.src, w.ld, c.in, w.r, w.ld);
    launch_inv_gemm(s, c.ncols, S.n, w.r, w.ld, S.Ainv, S.ld_inv, w.x, w.ld, S.gemm_part,
                    S.gemm_part_size);
  } else {
    launch_axpby3(s, S.n, c.ncols, w.x, w.ld, 0.0, CView{}, 1.0, c.ga, c.sgb, c.gb);
    if (h.circ) circuit_guess(h, S, w, c);
    if (S.nl.n_tri > 0 && narrow_persistent(h, l, S, c.ncols))
      it = newton_narrow(h, l, S, w, c.ncols, c.in, c.t_list, c.t_base, c.t_stride);
    else
      it = S.nl.n_tri > 0
               ? newton_solve(h, l, S, w, c.ncols, c.in, c.ga.p == c.in.p && c.gb.p == nullptr)
               : pcg_solve(h, l, S.op, w, c.ncols, c.in);
  }
  // field-circuit coupling: the solve gave y = A^-1 (M/dt) u_in; eliminate
  // the circuit unknowns and add Z w
  if (h.circ) circuit_step(h, S, w, c);
  if (c.dout)
    launch_axpby3(s, S.n, c.ncols, c.dout, c.ldo, 1.0, CView{w.x, w.ld}, -1.0, CView{c.out, c.ldo},
                  0.0, CView{});
  launch_axpby3(s, S.n, c.ncols, c.out, c.ldo, c.osx, CView{w.x, w.ld}, 1.0, c.oa, c.osb, c.ob);
  if (h.st && l < MGRIT_MAX_LEVELS) {
    h.st->phi_columns[l] += c.ncols;
    h.st->pcg_sweeps[l] += it;
  }
}

// The coarse propagator of level l: implicit Euler, or on the coarsest level
// with coarse_model = 1 implicit Euler plus the learned correction,
//   out = osx * (p + s_out delta) + oa + osb * ob,   p = Phi_IE(in).
static bool learned_active(const Handle& h, int l) {
  return h.par.coarse_model == 1 && !h.learned_off && l == static_cast<int>(h.lv.size()) - 1;
}

static void psi_batch(Handle& h, int l, PcgWork& w, const PhiCall& c) {
  if (!learned_active(h, l)) {
    phi_batch(h, l, w, c);
    return;
  }
  if (c.ncols <= 0) return;
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  PhiCall ie = c;
  ie.out = h.gnn_tmp;
  ie.ldo = S.ld;
  ie.osx = 1.0;
  ie.oa = CView{};
  ie.ob = CView{};
  ie.osb = 0.0;
  phi_batch(h, l, w, ie);
  gnn_forward64(s, h.gnn, h.src, c.ncols, c.t_list, c.t_base, c.t_stride, nullptr, nullptr, c.in,
                CView{h.gnn_tmp, S.ld}, h.gnn_tmp, S.ld);
  launch_axpby3(s, S.n, c.ncols, c.out, c.ldo, c.osx, CView{h.gnn_tmp, S.ld}, 1.0, c.oa, c.osb, c.ob);
}

static double* slab(LevelState& S, int j) { return S.U + static_cast<int64_t>(j) * S.ss; }
static double* gslab(LevelState& S, int j) {
  return S.G ? S.G + static_cast<int64_t>(j) * S.ss : nullptr;
}

static void f_relax(Handle& h, int l) {
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  const bool warm = S.relaxed && h.par.warm_start;
  // warm_start = 2: the previous iterate u_j was Phi(u_j-1^old); start from
  // u_j + (u_j-1 - u_j-1^old).  dlt carries the input change from one solve
  // to the next (dlt = x - u_j^old after solve j); for j = 1 it is the change
  // of the C-points since the previous F-relaxation (C-relaxation or coarse
  // correction).  Level 0 only: its FAS right-hand side is zero, so u_j^old
  // stays Phi(u_j-1^old).
  const bool delta = S.dlt && !S.G;
  const int nt = static_cast<int>(S.NT);
  if (delta) {
    if (warm)
      launch_axpby3(s, S.n, nt, S.dlt, S.ld, 0.0, CView{}, 1.0, CView{slab(S, 0), S.ld}, -1.0,
                    CView{S.csnap, S.ld});
    launch_axpby3(s, S.n, nt, S.csnap, S.ld, 0.0, CView{}, 1.0, CView{slab(S, 0), S.ld}, 0.0, CView{});
  }
  for (int j = 1; j < S.m; ++j) {
    PhiCall c;
    c.ncols = nt;
    c.in = CView{slab(S, j - 1), S.ld};
    c.t_base = j - 1;
    c.t_stride = S.m;
    if (warm && delta) {
      c.ga = CView{slab(S, j), S.ld};
      c.gb = CView{S.dlt, S.ld};
      c.sgb = 1.0;
    } else if (warm) {
      c.ga = CView{slab(S, j), S.ld};
      c.gb = CView{gslab(S, j), S.ld};
      c.sgb = -1.0;
    } else {
      c.ga = c.in;
    }
    c.out = slab(S, j);
    c.ldo = S.ld;
    c.oa = CView{gslab(S, j), S.ld};
    if (delta) c.dout = S.dlt;
    phi_batch(h, l, S.pcg, c);
  }
  S.relaxed = true;
}

static void c_relax(Handle& h, int l) {
  LevelState& S = h.lv[l];
  PhiCall c;
  c.ncols = static_cast<int>(S.NT);
  c.in = CView{slab(S, S.m - 1), S.ld};
  c.t_base = S.m - 1;
  c.t_stride = S.m;
  if (S.cvalid && h.par.warm_start) {
    c.ga = CView{slab(S, 0) + 1, S.ld};
    c.gb = CView{S.G ? gslab(S, 0) + 1 : nullptr, S.ld};
    c.sgb = -1.0;
  } else {
    c.ga = c.in;
  }
  c.out = slab(S, 0) + 1;
  c.ldo = S.ld;
  c.oa = CView{S.G ? gslab(S, 0) + 1 : nullptr, S.ld};
  phi_batch(h, l, S.pcg, c);
  S.cvalid = true;
}

static void relax(Handle& h, int l) {
  f_relax(h, l);
  for (int g = 0; g < h.par.gamma; ++g) {
    c_relax(h, l);
    f_relax(h, l);
  }
}

// RES[:, k] = g_km - u_km + Phi(u_km-1) (k >= 1), RES[:, 0] = g_0 - u_0.
// Level 0 stores no g: g_0 is the initial value, which u_0 holds exactly, so
// r_0 = 0 there.
static void c_residual(Handle& h, int l) {
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  if (S.G)
    launch_axpby3(s, S.n, 1, S.RES, S.ld, 0.0, CView{}, 1.0, CView{gslab(S, 0), S.ld}, -1.0,
                  CView{slab(S, 0), S.ld});
  else
    launch_axpby3(s, S.n, 1, S.RES, S.ld, 0.0, CView{}, 0.0, CView{}, 0.0, CView{});
  PhiCall c;
  c.ncols = static_cast<int>(S.NT);
  c.in = CView{slab(S, S.m - 1), S.ld};
  c.t_base = S.m - 1;
  c.t_stride = S.m;
  c.ga = CView{slab(S, 0) + 1, S.ld};
  c.gb = CView{S.G ? gslab(S, 0) + 1 : nullptr, S.ld};
  c.sgb = -1.0;
  c.out = S.RES + 1;
  c.ldo = S.ld;
  c.osx = 1.0;
  c.oa = c.gb;
  c.ob = CView{slab(S, 0) + 1, S.ld};
  c.osb = -1.0;
  phi_batch(h, l, S.pcg, c);
}

static double residual_norm(Handle& h, int l) {
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  const int ncols = static_cast<int>(S.NT + 1);
  launch_colsq(s, S.pcg, S.n, ncols, CView{S.RES, S.ld});
  double* sums = S.pcg.scal + 5 * S.pcg.ld;
  launch_reduce(s, S.pcg, ncols, RED_SUM, 0.0, 1, sums);
  MG_HIP(hipMemcpyAsync(h.host_sums, sums, sizeof(double) * ncols, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (int c = 0; c < ncols; ++c) t += h.host_sums[c];
  if (!std::isfinite(t)) fail(MGRIT_NONFINITE, "non-finite MGRIT residual");
  return std::sqrt(t);
}

static void coarsest_solve(Handle& h, int l) {
  LevelState& S = h.lv[l];
  hipStream_t s = h.stream;
  LevelTimer timer(h, l);
  // u_0 = g_0
  launch_axpby3(s, S.n, 1, S.U, S.ld, 0.0, CView{}, 1.0, CView{S.G, S.ld}, 0.0, CView{});
  if (S.Ainv && !h.circ) {
    // implicit Euler with the stored inverse (the same kernels as the batched
    // coarse steps of the FAS right-hand side, so both evaluate the same
    // propagator), the learned correction in place if active, then + g_s
    PcgWork& w = S.pcg;
    const bool learned = learned_active(h, l);
    for (int64_t st = 1; st <= S.N; ++st) {
      // one column: right-hand side and result contiguous (the product's
      // arithmetic does not depend on the strides)
      launch_source_table(s, h.src, S.op.dt, 1, nullptr, st - 1, 0, w.src, w.ld);
      launch_ie_inverse_batch(s, S.op, 1, w.src, w.ld, CView{S.U + st - 1, S.ld}, S.Ainv, S.ld_inv,
                              S.bvec, w.x, 1);
      if (learned)
        gnn_forward64(s, h.gnn, h.src, 1, nullptr, st - 1, 0, nullptr, nullptr, CView{S.U + st - 1, S.ld},
                      CView{w.x, 1}, w.x, 1);
      launch_axpby3(s, S.n, 1, S.U + st, S.ld, 1.0, CView{w.x, 1}, 1.0, CView{S.G + st, S.ld}, 0.0,
                    CView{});
    }
    if (h.st && l < MGRIT_MAX_LEVELS) h.st->phi_columns[l] += S.N;
    return;
  }
  if (S.nl.n_tri > 0 && S.nl_ws) {
    const double lam_min = std::ldexp(1.0, -h.par.newton_halvings);
    MG_HIP(hipMemsetAsync(S.pcg.flags, 0, 8 * sizeof(int), s));
    if (!learned_active(h, l)) {
      // the whole sequential Newton sweep in one persistent work-group
      launch_seq_newton(s, S.op, S.nl, h.src, static_cast<int>(S.N), 0, S.U, S.ld, S.G, S.ld, 1,
                        h.par.newton_tol, h.par.newton_max_iter, lam_min, h.par.ir_inner_tol,
                        h.par.pcg_max_iter, S.nl_ws, S.pcg.flags);
    } else {
      // learned propagator: per step the implicit-Euler Newton step in the
      // persistent work-group, the network correction, then + g_s
      PcgWork& w = S.pcg;
      for (int64_t st = 1; st <= S.N; ++st) {
        launch_seq_newton(s, S.op, S.nl, h.src, 1, st - 1, S.U + st - 1, S.ld, S.G + st - 1, S.ld, 1,
                          h.par.newton_tol, h.par.newton_max_iter, lam_min, h.par.ir_inner_tol,
                          h.par.pcg_max_iter, S.nl_ws, S.pcg.flags, false);
        launch_axpby3(s, S.n, 1, w.x, w.ld, 1.0, CView{S.U + st, S.ld}, 0.0, CView{}, 0.0, CView{});
        gnn_forward64(s, h.gnn, h.src, 1, nullptr, st - 1, 0, nullptr, nullptr, CView{S.U + st - 1, S.ld},
                      CView{w.x, w.ld}, w.x, w.ld);
        launch_axpby3(s, S.n, 1, S.U + st, S.ld, 1.0, CView{w.x, w.ld}, 1.0, CView{S.G + st, S.ld}, 0.0,
                      CView{});
      }
    }
    MG_HIP(hipMemcpyAsync(S.pcg.host_flags, S.pcg.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    const int bits = S.pcg.host_flags[1];
    if (bits & 1) fail(MGRIT_NONFINITE, "non-finite value in the coarsest Newton solve");
    if (bits & 8) fail(MGRIT_NEWTON_NOT_CONVERGED, "Newton did not converge in newton_max_iter iterations on the coarsest level");
    if (bits & 2) fail(MGRIT_PCG_NOT_CONVERGED, "inner CG did not converge on the coarsest level");
    if (h.st && l < MGRIT_MAX_LEVELS) {
      h.st->phi_columns[l] += S.N;
      h.st->pcg_sweeps[l] += S.pcg.host_flags[2];
      h.st->newton_sweeps[l] += S.pcg.host_flags[3];
    }
    return;
  }
  if (S.nl.n_tri > 0 || learned_active(h, l) || h.circ) {
    // one step at a time, u_s = Psi(u_{s-1}) + g_s (Newton for the nonlinear
    // model; the circuit elimination after each step of the coupled model)
    for (int64_t st = 1; st <= S.N; ++st) {
      PhiCall c;
      c.ncols = 1;
      c.in = CView{S.U + st - 1, S.ld};
      c.t_base = st - 1;
      c.ga = CView{S.U + st, S.ld};
      c.gb = CView{S.G + st, S.ld};
      c.sgb = -1.0;
      c.out = S.U + st;
      c.ldo = S.ld;
      c.oa = CView{S.G + st, S.ld};
      psi_batch(h, l, S.pcg, c);
    }
    return;
  }
  MG_HIP(hipMemsetAsync(S.pcg.flags, 0, 4 * sizeof(int), s));
  launch_seq_small(s, S.op, h.src, static_cast<int>(S.N), 0, S.U, S.ld, S.G, S.ld, S.seq_ws,
                   h.par.pcg_tol, h.par.pcg_max_iter, 1, S.pcg.flags);
  MG_HIP(hipMemcpyAsync(S.pcg.host_flags, S.pcg.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (S.pcg.host_flags[1] & 1) fail(MGRIT_NONFINITE, "non-finite value in the coarsest solve");
  if (S.pcg.host_flags[1] & 2) fail(MGRIT_PCG_NOT_CONVERGED, "PCG did not converge on the coarsest level");
  if (h.st && l < MGRIT_MAX_LEVELS) {
    h.st->phi_columns[l] += S.N;
    h.st->pcg_sweeps[l] += S.pcg.host_flags[2];
  }
}

enum CycleKind { CYCLE_V = 0, CYCLE_F = 1 };
static void cycle(Handle& h, int l, int kind);

// Algorithm 1, steps 4-9: restrict, FAS right-hand side, coarse solve, correct.
// The coarse problem is approximated by one V-cycle on level l+1, or for an
// F-cycle by an F-cycle followed by a V-cycle (Sec. 2.1, Fig. 4); on the
// coarsest level both are its one exact sequential solve.
static void coarse_correct(Handle& h, int l, int kind) {
  LevelState& S = h.lv[l];
  LevelState& C = h.lv[l + 1];
  hipStream_t s = h.stream;
  const int np = static_cast<int>(S.NT + 1);  // points of level l+1
  if (S.has_transfer) {
    launch_transfer(s, S.R, np, CView{slab(S, 0), S.ld}, 1.0, S.U2, S.ld, 0.0);
    launch_transfer(s, S.R, np, CView{S.RES, S.ld}, 1.0, S.RR, S.ld, 0.0);
  } else {
    launch_axpby3(s, C.n, np, S.U2, S.ld, 1.0, CView{slab(S, 0), S.ld}, 0.0, CView{}, 0.0, CView{});
    launch_axpby3(s, C.n, np, S.RR, S.ld, 1.0, CView{S.RES, S.ld}, 0.0, CView{}, 0.0, CView{});
  }
  // g2_0 = u2_0 + rr_0 ; g2_k = u2_k - Phi_{l+1}(u2_{k-1}) + rr_k
  launch_axpby3(s, C.n, 1, S.G2, S.ld, 1.0, CView{S.U2, S.ld}, 1.0, CView{S.RR, S.ld}, 0.0, CView{});
  PhiCall c;
  c.ncols = np - 1;
  c.in = CView{S.U2, S.ld};
  c.t_base = 0;
  c.t_stride = 1;
  c.ga = CView{S.U2 + 1, S.ld};
  c.out = S.G2 + 1;
  c.ldo = S.ld;
  c.osx = -1.0;
  c.oa = CView{S.U2 + 1, S.ld};
  c.ob = CView{S.RR + 1, S.ld};
  c.osb = 1.0;
  psi_batch(h, l + 1, C.pcg, c);
  // v = u2, load the coarse problem
  if (C.coarsest) {
    launch_axpby3(s, C.n, np, C.U, C.ld, 1.0, CView{S.U2, S.ld}, 0.0, CView{}, 0.0, CView{});
    launch_axpby3(s, C.n, np, C.G, C.ld, 1.0, CView{S.G2, S.ld}, 0.0, CView{}, 0.0, CView{});
  } else {
    launch_cols_to_slabs(s, C.n, np, C.m, S.U2, S.ld, C.U, C.ld, C.ss);
    launch_cols_to_slabs(s, C.n, np, C.m, S.G2, S.ld, C.G, C.ld, C.ss);
  }
  C.cvalid = true;
  cycle(h, l + 1, kind);
  if (kind == CYCLE_F && !C.coarsest) cycle(h, l + 1, CYCLE_V);
  // e = v - u2 (into RR), u_C += P_s e
  if (C.coarsest) {
    launch_axpby3(s, C.n, np, S.RR, S.ld, 1.0, CView{C.U, C.ld}, -1.0, CView{S.U2, S.ld}, 0.0, CView{});
  } else {
    launch_slabs_to_cols(s, C.n, np, C.m, C.U, C.ld, C.ss, S.RR, S.ld);
    launch_axpby3(s, C.n, np, S.RR, S.ld, 1.0, CView{S.RR, S.ld}, -1.0, CView{S.U2, S.ld}, 0.0, CView{});
  }
  if (S.has_transfer) {
    launch_transfer(s, S.P, np, CView{S.RR, S.ld}, 1.0, slab(S, 0), S.ld, 1.0);
  } else {
    launch_axpby3(s, S.n, np, slab(S, 0), S.ld, 1.0, CView{slab(S, 0), S.ld}, 1.0, CView{S.RR, S.ld},
                  0.0, CView{});
  }
}

static void cycle(Handle& h, int l, int kind) {
  LevelState& S = h.lv[l];
  if (S.coarsest) {
    coarsest_solve(h, l);
    return;
  }
  relax(h, l);
  c_residual(h, l);
  coarse_correct(h, l, kind);
  f_relax(h, l);
}

// Joule losses (Sec. 3.1) P = (u_a - u_b)^T M (u_a - u_b) / dt^2 (l_z = 1 m)
// of ncols column pairs of level 0, into host_sums[0 .. ncols).
static void joule_pairs(Handle& h, int ncols, CView a, CView b) {
  LevelState& S = h.lv[0];
  hipStream_t s = h.stream;
  launch_joule(s, S.pcg, S.op, ncols, a, b);
  double* sums = S.pcg.scal + 5 * S.pcg.ld;
  launch_reduce(s, S.pcg, ncols, RED_SUM, 0.0, 1, sums);
  MG_HIP(hipMemcpyAsync(h.host_sums, sums, sizeof(double) * ncols, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < ncols; ++c) h.host_sums[c] /= S.op.dt;
}

// Losses at the C-points k >= 1 of level 0 (u_km against u_km-1).
static void cpoint_losses(Handle& h, std::vector<double>& p) {
  LevelState& S = h.lv[0];
  const int nt = static_cast<int>(S.NT);
  joule_pairs(h, nt, CView{slab(S, 0) + 1, S.ld}, CView{slab(S, h.m - 1), S.ld});
  p.assign(h.host_sums, h.host_sums + nt);
  for (double v : p)
    if (!std::isfinite(v)) fail(MGRIT_NONFINITE, "non-finite Joule loss");
}

// Largest |p - q| / |p| over the points with p != 0 (Sec. 5.1 stop rule).
static double max_relative_change(const std::vector<double>& p, const std::vector<double>& q) {
  double worst = 0.0;
  bool any = false;
  for (size_t k = 0; k < p.size(); ++k) {
    if (p[k] == 0.0) continue;
    any = true;
    worst = std::max(worst, std::fabs(p[k] - q[k]) / std::fabs(p[k]));
  }
  if (!any) return p == q ? 0.0 : INFINITY;
  return worst;
}

// Nested-iteration start (Sec. 2.1; Sec. 4.1 drives it with the sine
// references): the coarsest level's time-stepping problem (g_0 = the
// restricted initial value, g_i = 0) is solved sequentially; on every finer
// level its points become the C-points (P_s in space), one V-cycle is applied
// to that level's own problem, and so on up to level 0.  On level 0 the
// V-cycle's last F-relaxation is left to the first MGRIT iteration, whose
// relaxation starts with it (F-relaxation depends on the C-points only).
static void nested_start(Handle& h) {
  const int L = static_cast<int>(h.lv.size());
  hipStream_t s = h.stream;
  struct Restore {
    Handle& h;
    bool learned_off;
    ~Restore() {
      h.src.signal = h.phys.signal;
      h.learned_off = learned_off;
    }
  } restore{h, h.learned_off};
  h.src.signal = 1;
  // the learned correction was trained on PWM-driven steps: the sine-driven
  // start steps the coarsest level by implicit Euler
  h.learned_off = true;
  h.tol_now = h.par.pcg_tol;
  h.eta_now = 0.0;
  LevelState& S0 = h.lv[0];
  // restricted initial values
  launch_axpby3(s, S0.n, 1, S0.u0r, 1, 1.0, CView{slab(S0, 0), S0.ld}, 0.0, CView{}, 0.0, CView{});
  for (int l = 0; l + 1 < L; ++l) {
    LevelState& S = h.lv[l];
    LevelState& C = h.lv[l + 1];
    if (S.has_transfer) launch_transfer(s, S.R, 1, CView{S.u0r, 1}, 1.0, C.u0r, 1, 0.0);
    else launch_axpby3(s, C.n, 1, C.u0r, 1, 1.0, CView{S.u0r, 1}, 0.0, CView{}, 0.0, CView{});
  }
  LevelState& C = h.lv[L - 1];
  MG_HIP(hipMemsetAsync(C.G, 0, sizeof(double) * C.ss, s));
  launch_axpby3(s, C.n, 1, C.G, C.ld, 1.0, CView{C.u0r, 1}, 0.0, CView{}, 0.0, CView{});
  coarsest_solve(h, L - 1);
  for (int l = L - 2; l >= 0; --l) {
    LevelState& S = h.lv[l];
    LevelState& Cn = h.lv[l + 1];
    const int np = static_cast<int>(S.NT + 1);
    // the coarse level's points in time order, then P_s onto the C-points
    if (Cn.coarsest)
      launch_axpby3(s, Cn.n, np, S.RR, S.ld, 1.0, CView{Cn.U, Cn.ld}, 0.0, CView{}, 0.0, CView{});
    else
      launch_slabs_to_cols(s, Cn.n, np, Cn.m, Cn.U, Cn.ld, Cn.ss, S.RR, S.ld);
    if (S.has_transfer) launch_transfer(s, S.P, np, CView{S.RR, S.ld}, 1.0, slab(S, 0), S.ld, 0.0);
    else launch_axpby3(s, S.n, np, slab(S, 0), S.ld, 1.0, CView{S.RR, S.ld}, 0.0, CView{}, 0.0, CView{});
    launch_axpby3(s, S.n, 1, slab(S, 0), S.ld, 1.0, CView{S.u0r, 1}, 0.0, CView{}, 0.0, CView{});
    S.relaxed = S.cvalid = false;
    if (l > 0) {
      MG_HIP(hipMemsetAsync(S.G, 0, sizeof(double) * S.ss * S.m, s));
      launch_axpby3(s, S.n, 1, S.G, S.ld, 1.0, CView{S.u0r, 1}, 0.0, CView{}, 0.0, CView{});
      cycle(h, l, CYCLE_V);
    } else {
      h.eta_now = h.par.pcg_tol_eta;
      relax(h, 0);
      h.eta_now = h.par.residual_eta;
      c_residual(h, 0);
      h.eta_now = 0.0;
      coarse_correct(h, 0, CYCLE_V);
    }
  }
  MG_HIP(hipStreamSynchronize(s));
}

// A^{-1} of the coarsest level (linear model), by batched CG on the columns
// of the identity to a relative residual of 1e-14.
static void build_coarse_inverse(Handle& h, LevelState& S) {
  hipStream_t s = h.stream;
  PcgWork w;
  const int chunk = std::min(S.n, 2048);
  const int keep_max = h.par.pcg_max_iter;
  h.par.pcg_max_iter = std::max(keep_max, 20000);   // history buffer size for this solve
  alloc_pcg(h, w, S.n, chunk, rows_per_block_for(S.n), MGRIT_FP64);
  h.par.pcg_max_iter = keep_max;
  // the level's own (autotuned) CG kernel shape
  set_rows_per_block(w, S.pcg.rows_per_block);
  w.cpl = S.pcg.cpl;
  w.dia = S.pcg.dia;
  w.depth = S.pcg.depth;
  S.ld_inv = round_up(S.n, kWave);
  S.Ainv = h.arena.alloc<double>(static_cast<size_t>(S.n) * S.ld_inv);
  S.bvec = h.arena.alloc<double>(S.n);
  const double tol2 = 1e-28;
  for (int j0 = 0; j0 < S.n; j0 += chunk) {
    const int nc = std::min(chunk, S.n - j0);
    launch_cg_init_identity(s, S.op, w, j0, nc);
    launch_reduce(s, w, nc, RED_INIT, tol2, 3, nullptr);
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    mgrit_stats* keep = h.st;
    h.st = nullptr;
    pcg_iterate(h, 0, S.op, w, nc, tol2, IT_LIN64, w.host_flags[0], true, w.hist_cap);
    h.st = keep;
    // columns j0.. of the inverse (symmetric: rows j0.. as well)
    launch_axpby3(s, S.n, nc, S.Ainv + j0, S.ld_inv, 1.0, CView{w.x, w.ld}, 0.0, CView{}, 0.0,
                  CView{});
  }
  MG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Field-circuit coupling set-up (Sec. 3.1): per level the coupling rows
// B = [X; Y'/l_z] (X_s = turns_density * integral of sign phi over the cells
// of phase s, Y'_k = integral of sigma phi over bar k), Z = A^-1 B^T by
// batched CG to 1e-14 relative residual, and the eliminated circuit system
// S = (l_z/dt) E B Z + diag(r_phase I_3, C), C = diag(G) + L / (2 ring_r),
// stored as [S^-1 columns 0..2 | S^-1 (l_z/dt) E] per row.

// Inverse of a small dense matrix (row-major k x k) by Gauss-Jordan
// elimination with partial pivoting.
static std::vector<double> small_inverse(std::vector<double> a, int k) {
  std::vector<double> inv(static_cast<size_t>(k) * k, 0.0);
  for (int i = 0; i < k; ++i) inv[static_cast<size_t>(i) * k + i] = 1.0;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(a[static_cast<size_t>(r) * k + c]) > std::fabs(a[static_cast<size_t>(piv) * k + c])) piv = r;
    if (!(std::fabs(a[static_cast<size_t>(piv) * k + c]) > 0.0))
      fail(MGRIT_INVALID_ARGUMENT, "field-circuit system is singular");
    if (piv != c)
      for (int j = 0; j < k; ++j) {
        std::swap(a[static_cast<size_t>(piv) * k + j], a[static_cast<size_t>(c) * k + j]);
        std::swap(inv[static_cast<size_t>(piv) * k + j], inv[static_cast<size_t>(c) * k + j]);
      }
    const double d = a[static_cast<size_t>(c) * k + c];
    for (int j = 0; j < k; ++j) {
      a[static_cast<size_t>(c) * k + j] /= d;
      inv[static_cast<size_t>(c) * k + j] /= d;
    }
    for (int r = 0; r < k; ++r) {
      if (r == c) continue;
      const double f = a[static_cast<size_t>(r) * k + c];
      if (f == 0.0) continue;
      for (int j = 0; j < k; ++j) {
        a[static_cast<size_t>(r) * k + j] -= f * a[static_cast<size_t>(c) * k + j];
        inv[static_cast<size_t>(r) * k + j] -= f * inv[static_cast<size_t>(c) * k + j];
      }
    }
  }
  return inv;
}

static void setup_circuit(Handle& h, const mgrit_problem* prob, const std::vector<HostPattern>& pats) {
  const mgrit_physics& ph = prob->phys;
  hipStream_t s = h.stream;
  const int nb = ph.n_bars, k = 3 + nb;
  h.circ_k = k;
  for (size_t l = 0; l < h.lv.size(); ++l) {
    LevelState& S = h.lv[l];
    const mgrit_mesh& m = prob->meshes[l];
    const HostPattern& P = pats[l];
    const int n = S.n;
    // coupling rows by unknown (device order), and the bars' conductances
    std::vector<double> Bt(static_cast<size_t>(n) * k, 0.0);
    std::vector<double> G(nb, 0.0);
    for (int e = 0; e < m.n_tri; ++e) {
      const int* v = m.tri + 3 * e;
      const double* p0 = m.xy + 2 * v[0];
      const double* p1 = m.xy + 2 * v[1];
      const double* p2 = m.xy + 2 * v[2];
      const double area = 0.5 * ((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
      const int ph_e = m.cell_phase[e];
      const double sig = ph.sigma[m.cell_mat[e]];
      const int bar = (nb > 0) ? m.cell_bar[e] : -1;
      if (bar >= 0) G[bar] += sig * area / ph.l_z;
      for (int a = 0; a < 3; ++a) {
        const int i = P.index[v[a]];
        if (i < 0) continue;
        if (ph_e >= 0) Bt[static_cast<size_t>(i) * k + ph_e] += ph.turns_density * m.cell_sign[e] * area / 3.0;
        if (bar >= 0) Bt[static_cast<size_t>(i) * k + 3 + bar] += sig * area / 3.0 / ph.l_z;
      }
    }
    for (int b = 0; b < nb; ++b)
      if (!(G[b] > 0.0)) fail(MGRIT_INVALID_ARGUMENT, "a rotor bar has no conducting cells on some level");
    S.cBt = h.arena.alloc<double>(Bt.size());
    MG_HIP(hipMemcpyAsync(S.cBt, Bt.data(), sizeof(double) * Bt.size(), hipMemcpyHostToDevice, s));
    // Z = A^-1 B^T: k columns of batched FP64 CG (the level's kernel shape)
    PcgWork w;
    const int keep_max = h.par.pcg_max_iter;
    h.par.pcg_max_iter = std::max(keep_max, 20000);
    alloc_pcg(h, w, n, k, rows_per_block_for(n), MGRIT_FP64);
    h.par.pcg_max_iter = keep_max;
    set_rows_per_block(w, S.pcg.rows_per_block);
    w.cpl = S.pcg.cpl;
    w.dia = S.pcg.dia;
    w.depth = S.pcg.depth;
    const double tol2 = 1e-28;
    launch_circ_rhs_init(s, S.op, w, S.cBt, k, k);
    launch_reduce(s, w, k, RED_INIT, tol2, 3, nullptr);
    MG_HIP(hipMemcpyAsync(w.host_flags, w.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    mgrit_stats* keep = h.st;
    h.st = nullptr;
    pcg_iterate(h, 0, S.op, w, k, tol2, IT_LIN64, w.host_flags[0], true, w.hist_cap);
    h.st = keep;
    S.cZ = h.arena.alloc<double>(static_cast<size_t>(n) * k);
    launch_axpby3(s, n, k, S.cZ, k, 1.0, CView{w.x, w.ld}, 0.0, CView{}, 0.0, CView{});
    std::vector<double> Z(static_cast<size_t>(n) * k);
    MG_HIP(hipMemcpyAsync(Z.data(), S.cZ, sizeof(double) * Z.size(), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    // S = (l_z/dt) E B Z + diag(r_phase I_3, C)
    const double f = ph.l_z / S.op.dt;
    std::vector<double> Sm(static_cast<size_t>(k) * k, 0.0);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < k; ++a) {
        const double ba = Bt[static_cast<size_t>(i) * k + a];
        if (ba == 0.0) continue;
        for (int b = 0; b < k; ++b) Sm[static_cast<size_t>(a) * k + b] += ba * Z[static_cast<size_t>(i) * k + b];
      }
    for (int a = 0; a < k; ++a) {
      const double e = a < 3 ? f : -f;
      for (int b = 0; b < k; ++b) Sm[static_cast<size_t>(a) * k + b] *= e;
    }
    for (int a = 0; a < 3; ++a) Sm[static_cast<size_t>(a) * k + a] += ph.r_phase;
    for (int b = 0; b < nb; ++b) {
      const int r = 3 + b;
      Sm[static_cast<size_t>(r) * k + r] += G[b] + 2.0 / (2.0 * ph.ring_r);
      Sm[static_cast<size_t>(r) * k + 3 + (b + 1) % nb] -= 1.0 / (2.0 * ph.ring_r);
      Sm[static_cast<size_t>(r) * k + 3 + (b + nb - 1) % nb] -= 1.0 / (2.0 * ph.ring_r);
    }
    if (l == 0 && nb > 0) {
      std::vector<double> Cm(static_cast<size_t>(nb) * nb, 0.0);
      for (int b = 0; b < nb; ++b) {
        Cm[static_cast<size_t>(b) * nb + b] += G[b] + 2.0 / (2.0 * ph.ring_r);
        Cm[static_cast<size_t>(b) * nb + (b + 1) % nb] -= 1.0 / (2.0 * ph.ring_r);
        Cm[static_cast<size_t>(b) * nb + (b + nb - 1) % nb] -= 1.0 / (2.0 * ph.ring_r);
      }
      h.circ_Cinv = small_inverse(Cm, nb);
    }
    const std::vector<double> Si = small_inverse(Sm, k);
    std::vector<double> cS(static_cast<size_t>(k) * (3 + k));
    for (int j = 0; j < k; ++j) {
      for (int q = 0; q < 3; ++q) cS[static_cast<size_t>(j) * (3 + k) + q] = Si[static_cast<size_t>(j) * k + q];
      for (int a = 0; a < k; ++a)
        cS[static_cast<size_t>(j) * (3 + k) + 3 + a] = Si[static_cast<size_t>(j) * k + a] * (a < 3 ? f : -f);
    }
    S.cS = h.arena.alloc<double>(cS.size());
    MG_HIP(hipMemcpyAsync(S.cS, cS.data(), sizeof(double) * cS.size(), hipMemcpyHostToDevice, s));
    // circuit unknowns of the latest coupled step from every time point (the
    // start of the next solve from the same point)
    S.c_nt = std::max<int64_t>(S.N, 1);
    S.cwt = h.arena.alloc<double>(static_cast<size_t>(k) * S.c_nt);
    MG_HIP(hipStreamSynchronize(s));
    circuit_buffers(h, S, S.pcg.cap);
  }
}

// ---------------------------------------------------------------------------
// Workspace of phi_step_noalloc: one static device array per GPU.  Host code
// never passes `scratch` itself to a kernel (in host code the name is a
// host-side stand-in, not a device address): set-up takes the array's device
// address once per device with hipGetSymbolAddress and the entry point carves
// every buffer out of that address.
constexpr int64_t kNoallocVec = int64_t(1) << 21;   // n * round_up(B, 64) at most
constexpr int64_t kNoallocCols = 32768;             // B at most
constexpr int64_t kNoallocHist = 65536;             // pcg_max_iter + 64 at most
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }
// worst case of noalloc_bytes(): 6 FP64 and 4 FP32 vectors, partial sums of
// 16-row blocks, the per-column scalars, source table, masks, flags, history
constexpr size_t kScratchBytes =
    align_up(6 * 8 * kNoallocVec) + align_up(4 * 4 * kNoallocVec) +
    align_up(3 * 8 * (kNoallocVec / 16 + kNoallocCols)) + align_up(8 * 8 * kNoallocCols) +
    align_up(3 * 8 * kNoallocCols) + 2 * align_up(kNoallocCols) + align_up(8 * 4) +
    align_up(4 * kNoallocHist);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken once per device).
static void init_scratch(Handle& h) {
  MG_HIP(hipGetDevice(&h.device));
  if (h.device < 0 || h.device >= kMaxDevices) fail(MGRIT_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[h.device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    fail(MGRIT_HIP_ERROR, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[h.device] = ptr;
}

// ---------------------------------------------------------------------------
// Setup.

static void setup_gnn(Handle& h, const mgrit_mesh& mesh, const HostPattern& pat, const mgrit_physics& ph);

static void setup_impl(Handle& h, const mgrit_problem* prob, const mgrit_params* par) {
  if (!prob || !par) fail(MGRIT_INVALID_ARGUMENT, "null problem or params");
  h.par = *par;
  h.tol_now = h.par.pcg_tol;
  h.verbose = std::getenv("MGRIT_VERBOSE") != nullptr;
  h.phys = prob->phys;
  const mgrit_physics& ph = prob->phys;
  const int L = prob->n_levels;
  if (L < 1 || L > MGRIT_MAX_LEVELS || !prob->meshes) fail(MGRIT_INVALID_ARGUMENT, "n_levels out of range");
  if (par->m < 2) fail(MGRIT_INVALID_ARGUMENT, "m must be > 1");
  if (par->gamma < 0) fail(MGRIT_INVALID_ARGUMENT, "gamma must be >= 0");
  if (!(par->pcg_tol > 0.0) || par->pcg_max_iter < 1 || !(par->pcg_tol_eta >= 0.0))
    fail(MGRIT_INVALID_ARGUMENT, "bad PCG settings");
  if (par->precision != MGRIT_FP64 && par->precision != MGRIT_FP32_IR)
    fail(MGRIT_INVALID_ARGUMENT, "precision must be MGRIT_FP64 or MGRIT_FP32_IR");
  if (par->precision_coarse != -1 && par->precision_coarse != MGRIT_FP64 &&
      par->precision_coarse != MGRIT_FP32_IR)
    fail(MGRIT_INVALID_ARGUMENT, "precision_coarse must be -1, MGRIT_FP64 or MGRIT_FP32_IR");
  if (par->pcg_kernel < 0 || par->pcg_kernel > 2) fail(MGRIT_INVALID_ARGUMENT, "pcg_kernel");
  if (par->warm_start < 0 || par->warm_start > 2) fail(MGRIT_INVALID_ARGUMENT, "warm_start must be 0, 1 or 2");
  if (par->pcg_prefetch != 0 && par->pcg_prefetch != 1 && par->pcg_prefetch != 2 &&
      par->pcg_prefetch != 4)
    fail(MGRIT_INVALID_ARGUMENT, "pcg_prefetch must be 0, 1, 2 or 4");
  if (!(par->residual_eta >= 0.0 && par->residual_eta < 1.0))
    fail(MGRIT_INVALID_ARGUMENT, "residual_eta must be in [0, 1)");
  {
    const int rn = par->pcg_rows_narrow;
    if (!(rn == 0 || rn == -1 || rn == 16 || rn == 32 || rn == 64 || rn == 128 || rn == 256))
      fail(MGRIT_INVALID_ARGUMENT, "pcg_rows_narrow must be 0, -1, 16, 32, 64, 128 or 256");
  }
  if (par->cycle != 0 && par->cycle != 1) fail(MGRIT_INVALID_ARGUMENT, "cycle must be 0 (V) or 1 (F)");
  if (par->nested != 0 && par->nested != 1) fail(MGRIT_INVALID_ARGUMENT, "nested must be 0 or 1");
  if (!(par->loss_tol >= 0.0)) fail(MGRIT_INVALID_ARGUMENT, "loss_tol must be >= 0");
  if (par->compact_columns < 0) fail(MGRIT_INVALID_ARGUMENT, "compact_columns must be >= 0");
  if (!(par->compact_fraction > 0.0 && par->compact_fraction < 1.0))
    fail(MGRIT_INVALID_ARGUMENT, "compact_fraction must be in (0, 1)");
  if (par->coarse_inverse < 0 || par->coarse_inverse > 2) fail(MGRIT_INVALID_ARGUMENT, "coarse_inverse");
  if (par->precision == MGRIT_FP32_IR && (!(par->ir_inner_tol > 0.0) || par->ir_max_iter < 1))
    fail(MGRIT_INVALID_ARGUMENT, "bad refinement settings");
  if (ph.nonlinear && !ph.iron) fail(MGRIT_INVALID_ARGUMENT, "the nonlinear model needs the iron flags");
  if (ph.nonlinear && (par->newton_max_iter < 1 || !(par->newton_tol > 0.0) || !(par->ir_inner_tol > 0.0) ||
                       par->newton_halvings < 0 || par->newton_halvings > 40))
    fail(MGRIT_INVALID_ARGUMENT, "bad Newton settings");
  if (ph.n_materials <= 0 || !ph.nu || !ph.sigma) fail(MGRIT_INVALID_ARGUMENT, "material table");
  if (!(ph.dt > 0.0) || ph.n_steps < 1) fail(MGRIT_INVALID_ARGUMENT, "time grid");
  if (ph.carrier != 0 && ph.carrier != 1) fail(MGRIT_INVALID_ARGUMENT, "carrier");
  if (par->m_coarse != 0 && par->m_coarse < 2) fail(MGRIT_INVALID_ARGUMENT, "m_coarse must be 0 or > 1");
  if (par->pcg_check_every < 0 || par->pcg_check_every > 64 || par->pcg_check_narrow < 0 ||
      par->pcg_check_narrow > 64)
    fail(MGRIT_INVALID_ARGUMENT, "pcg_check_every and pcg_check_narrow must be in 0..64");
  if (par->coarse_persistent < -1 || par->coarse_persistent > 1)
    fail(MGRIT_INVALID_ARGUMENT, "coarse_persistent must be -1, 0 or 1");
  {
    const int rb = par->pcg_rows_per_block;
    if (!(rb == 0 || rb == 16 || rb == 32 || rb == 64 || rb == 128 || rb == 256))
      fail(MGRIT_INVALID_ARGUMENT, "pcg_rows_per_block must be 0, 16, 32, 64, 128 or 256");
    if (par->pcg_cols_per_lane < 0 || par->pcg_cols_per_lane > 2)
      fail(MGRIT_INVALID_ARGUMENT, "pcg_cols_per_lane must be 0, 1 or 2");
  }
  h.m = par->m;
  // factor between levels l and l+1: m on level 0, m_coarse (or m) below
  auto factor = [&](int l) { return (l == 0 || par->m_coarse == 0) ? par->m : par->m_coarse; };
  int64_t mpow = 1;
  for (int l = 0; l + 1 < L; ++l) {
    mpow *= factor(l);
    if (ph.n_steps % mpow != 0)
      fail(MGRIT_INVALID_ARGUMENT, "n_steps must be divisible by the product of the coarsening factors");
  }
  h.src.scale = ph.J0 * ph.amplitude;
  h.src.freq = ph.freq;
  h.src.f_carrier = ph.f_carrier;
  for (int p = 0; p < 3; ++p) h.src.phi[p] = ph.phases[p] + ph.phase_offset;
  h.src.carrier = ph.carrier;
  if (!(ph.ramp_periods >= 0.0)) fail(MGRIT_INVALID_ARGUMENT, "ramp_periods must be >= 0");
  h.src.ramp_span = ph.ramp_periods > 0.0 ? ph.ramp_periods / ph.freq : 0.0;
  if (ph.signal != 0 && ph.signal != 1) fail(MGRIT_INVALID_ARGUMENT, "signal must be 0 (PWM) or 1 (sine)");
  h.src.signal = ph.signal;
  if (!std::isfinite(ph.t_start)) fail(MGRIT_INVALID_ARGUMENT, "t_start must be finite");
  h.src.t0 = ph.t_start;
  if (ph.circuit != 0 && ph.circuit != 1) fail(MGRIT_INVALID_ARGUMENT, "circuit must be 0 or 1");
  h.circ = ph.circuit == 1;
  if (h.circ) {
    if (ph.nonlinear) fail(MGRIT_UNSUPPORTED, "the field-circuit coupling needs the linear model");
    if (par->coarse_model != 0) fail(MGRIT_UNSUPPORTED, "the learned coarse propagator does not model the circuit");
    if (!(ph.turns_density > 0.0) || !(ph.l_z > 0.0) || !(ph.r_phase > 0.0) || !std::isfinite(ph.v0))
      fail(MGRIT_INVALID_ARGUMENT, "circuit: turns_density, l_z and r_phase must be > 0, v0 finite");
    if (ph.n_bars < 0 || ph.n_bars > kCircMax - 3) fail(MGRIT_INVALID_ARGUMENT, "circuit: n_bars must be 0..32");
    if (ph.n_bars > 0 && !(ph.ring_r > 0.0)) fail(MGRIT_INVALID_ARGUMENT, "circuit: ring_r must be > 0");
    for (int l = 0; l < L && ph.n_bars > 0; ++l) {
      const mgrit_mesh& mm = prob->meshes[l];
      if (!mm.cell_bar) fail(MGRIT_INVALID_ARGUMENT, "circuit: cell_bar is required with n_bars > 0");
      for (int e = 0; e < mm.n_tri; ++e)
        if (mm.cell_bar[e] < -1 || mm.cell_bar[e] >= ph.n_bars)
          fail(MGRIT_INVALID_ARGUMENT, "circuit: cell_bar out of range");
    }
    // the source table then holds the phase voltages v_s(t)
    h.src.scale = ph.v0 * ph.amplitude;
  }

  // host phase: validate every mesh, build patterns and transfers (no HIP call)
  std::vector<HostPattern> pats(L);
  for (int l = 0; l < L; ++l) {
    validate_mesh(prob->meshes[l], ph.n_materials);
    pats[l] = build_pattern(prob->meshes[l]);
  }
  std::vector<HostSparse> Ps(L), Rs(L);
  std::vector<bool> sc(L, false);
  for (int l = 0; l + 1 < L; ++l) {
    if (same_mesh(prob->meshes[l], prob->meshes[l + 1])) continue;
    Ps[l] = build_prolongation(prob->meshes[l], prob->meshes[l + 1], pats[l], pats[l + 1]);
    Rs[l] = build_restriction(Ps[l], par->restriction, prob->meshes[l], prob->meshes[l + 1],
                              pats[l], pats[l + 1]);
    sc[l] = true;
  }
  // device phase
  hipStream_t s = h.stream;
  init_scratch(h);
  h.lv.resize(L);
  double dt = ph.dt;
  int64_t N = ph.n_steps;
  for (int l = 0; l < L; ++l) {
    LevelState& S = h.lv[l];
    S.n = pats[l].n;
    S.N = N;
    S.coarsest = (l == L - 1);
    S.op = assemble_level(h.arena, s, prob->meshes[l], pats[l], ph, dt, &S.elem);
    // coupled model: the coils carry the circuit currents, not a source term
    if (h.circ) MG_HIP(hipMemsetAsync(S.op.F, 0, sizeof(double) * 3 * static_cast<size_t>(S.n), s));
    S.nat = upload_vec(h.arena, s, pats[l].nat);
    S.u0r = h.arena.alloc<double>(S.n);
    if (ph.nonlinear) {
      S.nl.n_tri = S.elem.n_tri;
      S.nl.tri_u = S.elem.tri_u;
      S.nl.grad = S.elem.grad;
      S.nl.area = S.elem.area;
      S.nl.nu_lin = S.elem.nu;
      S.nl.iron = S.elem.iron;
      S.nl.cptr = S.elem.cptr;
      S.nl.contrib = S.elem.contrib;
      S.nl.diag = S.elem.diag;
      S.nl.k1 = ph.bh_k1;
      S.nl.k2 = ph.bh_k2;
      S.nl.k3 = ph.bh_k3;
    }
    S.m = S.coarsest ? 0 : factor(l);
    if (!S.coarsest) {
      dt *= S.m;
      N /= S.m;
    }
  }
  for (int l = 0; l < L; ++l) {
    LevelState& S = h.lv[l];
    const int rpb = rows_per_block_for(S.n);
    if (S.coarsest) {
      S.ld = round_up(S.N + 1, kWave);
      S.ss = static_cast<int64_t>(S.n) * S.ld;
      S.U = h.arena.alloc<double>(S.ss);
      S.G = h.arena.alloc<double>(S.ss);
      S.seq_ws = h.arena.alloc<double>(4 * static_cast<size_t>(S.n));
      // nonlinear coarsest level: one persistent work-group runs the whole
      // sequential Newton sweep (latency-bound otherwise)
      const bool persistent = par->coarse_persistent == 1 ||
                              (par->coarse_persistent == 0 && S.n <= kMaxPersistentN);
      if (ph.nonlinear && L > 1 && persistent)
        S.nl_ws = h.arena.alloc<double>(
            static_cast<size_t>(seq_newton_ws_doubles(S.n, S.op.W, S.nl.n_tri)));
      MG_HIP(hipMemsetAsync(S.U, 0, sizeof(double) * S.ss, s));
      MG_HIP(hipMemsetAsync(S.G, 0, sizeof(double) * S.ss, s));
    } else {
      S.NT = S.N / S.m;
      S.ld = round_up(S.NT + 1, kWave);
      S.ss = static_cast<int64_t>(S.n) * S.ld;
      S.U = h.arena.alloc<double>(static_cast<size_t>(S.ss) * S.m);
      MG_HIP(hipMemsetAsync(S.U, 0, sizeof(double) * S.ss * S.m, s));
      if (l > 0) {
        S.G = h.arena.alloc<double>(static_cast<size_t>(S.ss) * S.m);
        MG_HIP(hipMemsetAsync(S.G, 0, sizeof(double) * S.ss * S.m, s));
      }
      S.RES = h.arena.alloc<double>(S.ss);
      if (l == 0 && par->warm_start == 2) {
        S.dlt = h.arena.alloc<double>(S.ss);
        S.csnap = h.arena.alloc<double>(S.ss);
      }
      const int nc = pats[l + 1].n;
      const size_t cs = static_cast<size_t>(nc) * S.ld;
      S.U2 = h.arena.alloc<double>(cs);
      S.G2 = h.arena.alloc<double>(cs);
      S.RR = h.arena.alloc<double>(cs);
      if (sc[l]) {
        S.P = upload_transfer(h.arena, s, Ps[l]);
        S.R = upload_transfer(h.arena, s, Rs[l]);
        S.has_transfer = true;
      }
    }
    // level l's batched Phi serves its own sweeps (NT columns) and, on
    // coarse levels, the FAS right-hand side (N columns)
    const int cap = static_cast<int>((l == 0 ? S.NT : S.N) + 1);
    S.prec = (l == 0 || par->precision_coarse < 0) ? par->precision : par->precision_coarse;
    alloc_pcg(h, S.pcg, S.n, cap, rpb, S.prec);
  }
  const int64_t ld0 = h.lv[0].pcg.ld > h.lv[0].ld ? h.lv[0].pcg.ld : h.lv[0].ld;
  h.host_sums = static_cast<double*>(h.arena.alloc_host(sizeof(double) * (ld0 + 64)));
  h.u0_dev = h.arena.alloc<double>(h.lv[0].n);
  MG_HIP(hipEventCreate(&h.ev0));
  MG_HIP(hipEventCreate(&h.ev1));
  MG_HIP(hipStreamCreateWithFlags(&h.capture_stream, hipStreamNonBlocking));
  h.ev.resize(4 * 64);   // 4 events per CG iteration of a check interval (<= 64 iterations)
  for (auto& e : h.ev) MG_HIP(hipEventCreate(&e));
  for (auto& S : h.lv) {
    if (par->pcg_kernel == 2 && S.op.dia_R == 0)
      fail(MGRIT_UNSUPPORTED, "diagonal-window kernels need the periodic polar stencil");
    autotune(h, S);
  }
  if (L > 1 && !ph.nonlinear && par->coarse_inverse && h.lv.back().n <= kMaxInverseN)
    build_coarse_inverse(h, h.lv.back());
  if (!ph.nonlinear && par->coarse_inverse == 2) {
    for (int l = 1; l + 1 < L; ++l)
      if (h.lv[l].n <= kMaxInverseNCoarse) {
        LevelState& S = h.lv[l];
        build_coarse_inverse(h, S);
        // partial sums of the k slices of narrow batches (phi_step_noalloc
        // may pass up to 2^21 / n columns)
        const int max_cols = std::max<int>(S.pcg.cap, static_cast<int>(kNoallocVec / S.n));
        S.gemm_part_size = inv_gemm_part_doubles(max_cols, S.n);
        if (S.gemm_part_size > 0) S.gemm_part = h.arena.alloc<double>(static_cast<size_t>(S.gemm_part_size));
      }
  }
  if (h.circ) setup_circuit(h, prob, pats);
  if (L > 1) setup_gnn(h, prob->meshes[L - 1], pats[L - 1], ph);
  if (par->coarse_model != 0 && par->coarse_model != 1)
    fail(MGRIT_INVALID_ARGUMENT, "coarse_model must be 0 or 1");
  if (par->coarse_model == 1 && !h.has_gnn)
    fail(MGRIT_UNSUPPORTED, "the learned coarse propagator needs two or more levels and m <= 25");
  MG_HIP(hipStreamSynchronize(s));
}

static double* stage(Handle& h) {
  if (!h.tm_stage) {
    const LevelState& S = h.lv[0];
    h.tm_stage = h.arena.alloc<double>(static_cast<size_t>(S.N + 1) * S.n);
  }
  return h.tm_stage;
}

static void load_u0(Handle& h, const double* u0) {
  LevelState& S = h.lv[0];
  if (u0) {
    MG_HIP(hipMemcpyAsync(h.u0_dev, u0, sizeof(double) * S.n,
                          h.par.device_pointers ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          h.stream));
  } else {
    MG_HIP(hipMemsetAsync(h.u0_dev, 0, sizeof(double) * S.n, h.stream));
  }
}

static void solve_impl(Handle& h, const double* u0, const double* u_init, double* u_out,
                       mgrit_stats* st) {
  hipStream_t s = h.stream;
  LevelState& S0 = h.lv[0];
  if (h.lv.size() < 2) fail(MGRIT_INVALID_ARGUMENT, "mgrit_solve needs at least two levels");
  if (!u_out) fail(MGRIT_INVALID_ARGUMENT, "u_out is null");
  for (auto& S : h.lv) S.relaxed = S.cvalid = false;
  const size_t tm_elems = static_cast<size_t>(S0.N + 1) * S0.n;
  const hipMemcpyKind h2d = h.par.device_pointers ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind d2h = h.par.device_pointers ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  load_u0(h, u0);
  if (u_init) {
    double* tm = stage(h);
    MG_HIP(hipMemcpyAsync(tm, u_init, sizeof(double) * tm_elems, h2d, s));
    launch_tm_to_slabs(s, S0.n, S0.N + 1, h.m, tm, S0.U, S0.ld, S0.ss, S0.nat);
  } else {
    MG_HIP(hipMemsetAsync(S0.U, 0, sizeof(double) * S0.ss * h.m, s));
  }
  launch_tm_to_slabs(s, S0.n, 1, 1, h.u0_dev, S0.U, S0.ld, 0, S0.nat);
  auto t0 = std::chrono::steady_clock::now();
  double rho0 = 0.0, rho_prev = 0.0;
  int status = MGRIT_OK;
  h.learned_off = false;
  h.solved = false;
  st->coarse_fallback = -1;
  // coupled steps start from the circuit unknowns of the previous step from
  // the same time point (zero before the first)
  struct GuessOff {
    Handle& h;
    ~GuessOff() { h.circ_guess = false; }
  } guess_off{h};
  if (h.circ) {
    for (auto& S : h.lv)
      if (S.cwt)
        launch_axpby3(s, h.circ_k, static_cast<int>(S.c_nt), S.cwt, S.c_nt, 0.0, CView{}, 0.0, CView{}, 0.0,
                      CView{});
    h.circ_guess = true;
  }
  if (h.par.coarse_model == 1 && !h.gnn.ready)
    fail(MGRIT_INVALID_ARGUMENT, "coarse_model = 1 needs trained or set coarse weights");
  if (h.par.nested) {
    nested_start(h);
    st->time_nested_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  const bool loss_stop = h.par.loss_tol > 0.0;
  std::vector<double> p_now, p_prev;
  for (int it = 0;; ++it) {
    // Only the level-0 relaxation stops its solves early (eta times the
    // warm-start residual, which shrinks as MGRIT converges).  Coarse levels
    // keep pcg_tol: their warm-start residuals do not shrink (the FAS right-
    // hand side and the coarse solve evaluate Phi at different inputs), so
    // loose coarse solves would leave an error floor in the correction.
    h.tol_now = h.par.pcg_tol;
    h.eta_now = h.par.pcg_tol_eta;
    MG_HIP(hipEventRecord(h.ev0, s));
    relax(h, 0);
    h.eta_now = 0.0;
    MG_HIP(hipEventRecord(h.ev1, s));
    MG_HIP(hipEventSynchronize(h.ev1));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, h.ev0, h.ev1));
    st->time_relax_s += 1e-3 * ms;
    // the C-point residual solves start from the current C-point values, so
    // their initial residual shrinks with the MGRIT residual: residual_eta
    // is a relative accuracy of the residual itself
    h.eta_now = h.par.residual_eta;
    c_residual(h, 0);
    h.eta_now = 0.0;
    const double rho = residual_norm(h, 0);
    if (st->n_history < MGRIT_MAX_HISTORY) st->rho[st->n_history++] = rho;
    if (it == 0) rho0 = rho;
    if (h.verbose) {
      std::fprintf(stderr, "[mgrit] iteration %d: rho/rho_0 = %.3e\n", it, rho0 > 0.0 ? rho / rho0 : 0.0);
      std::fflush(stderr);
    }
    // the learned coarse propagator is judged by the residual: if it grows,
    // the rest of the solve uses implicit Euler
    if (h.par.coarse_model == 1 && !h.learned_off && it > 0 && rho > rho_prev) {
      h.learned_off = true;
      st->coarse_fallback = it;
    }
    rho_prev = rho;
    if (loss_stop) {
      // Sec. 5.1: stop once no C-point loss changes by loss_tol or more
      // (relative) between two successive iterations
      cpoint_losses(h, p_now);
      const double ch = p_prev.empty() ? -1.0 : max_relative_change(p_now, p_prev);
      if (it < MGRIT_MAX_HISTORY) st->loss_change[it] = ch;
      if (h.verbose) {
        std::fprintf(stderr, "[mgrit] iteration %d: largest relative C-point loss change %.3e\n", it, ch);
        std::fflush(stderr);
      }
      if (!p_prev.empty() && ch < h.par.loss_tol) {
        st->converged = 1;
        break;
      }
      std::swap(p_prev, p_now);
    } else if (rho == 0.0 || rho <= h.par.tol * rho0) {
      st->converged = 1;
      break;
    }
    if (it >= h.par.max_iter) {
      status = MGRIT_NOT_CONVERGED;
      break;
    }
    coarse_correct(h, 0, h.par.cycle);
    st->iterations = it + 1;
  }
  h.solved = true;
  double* tm = h.par.device_pointers ? u_out : stage(h);
  launch_slabs_to_tm(s, S0.n, S0.N + 1, h.m, S0.U, S0.ld, S0.ss, tm, S0.nat);
  if (!h.par.device_pointers)
    MG_HIP(hipMemcpyAsync(u_out, tm, sizeof(double) * tm_elems, d2h, s));
  MG_HIP(hipStreamSynchronize(s));
  st->time_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status != MGRIT_OK) fail(status, "MGRIT did not reach tol within max_iter iterations");
}

// Joule losses at every point of the iterate of the last solve (p[0] = 0).
static void joule_impl(Handle& h, double* p) {
  if (!p) fail(MGRIT_INVALID_ARGUMENT, "p is null");
  if (!h.solved) fail(MGRIT_INVALID_ARGUMENT, "no completed mgrit_solve on this handle");
  LevelState& S = h.lv[0];
  const int nt = static_cast<int>(S.NT);
  std::vector<double> out(static_cast<size_t>(S.N + 1), 0.0);
  for (int j = 0; j < h.m; ++j) {
    // points k m + j against k m + j - 1: slab j against slab j-1 (same
    // column), or for j = 0 slab 0 from column 1 against slab m-1
    if (j > 0) joule_pairs(h, nt, CView{slab(S, j), S.ld}, CView{slab(S, j - 1), S.ld});
    else joule_pairs(h, nt, CView{slab(S, 0) + 1, S.ld}, CView{slab(S, h.m - 1), S.ld});
    for (int k = 0; k < nt; ++k) out[static_cast<size_t>(j > 0 ? k * h.m + j : (k + 1) * h.m)] = h.host_sums[k];
  }
  MG_HIP(hipMemcpyAsync(p, out.data(), sizeof(double) * out.size(),
                        h.par.device_pointers ? hipMemcpyHostToDevice : hipMemcpyHostToHost, h.stream));
  MG_HIP(hipStreamSynchronize(h.stream));
}

// Circuit quantities of the steps of a level-0 trajectory (time-major
// [(N+1)][n0], host or device): per step the k dot products with the
// coupling rows of u_i - u_{i-1} on the GPU, then on the host
//   i_s = (v_s(t_i) - (l_z/dt) d_s) / r_phase,  v_bar = C^-1 (l_z/dt) d_bar,
//   i_bar = -L v_bar / (2 ring_r).
static void circuit_values_impl(Handle& h, const double* u, double* out) {
  if (!h.circ) fail(MGRIT_UNSUPPORTED, "the problem has no circuit (circuit = 0)");
  if (!u || !out) fail(MGRIT_INVALID_ARGUMENT, "null trajectory or output");
  hipStream_t s = h.stream;
  LevelState& S = h.lv[0];
  const mgrit_physics& ph = h.phys;
  const int k = h.circ_k, nb = ph.n_bars, n = S.n;
  const int64_t N = S.N;
  const int chunk = 1024;                    // steps per pass
  const int64_t ldc = round_up(chunk + 1, kWave);
  if (!h.circ_stage)
    h.circ_stage = h.arena.alloc<double>(static_cast<size_t>(n) * (chunk + 1) + static_cast<size_t>(n) * ldc +
                                         3 * static_cast<size_t>(ldc));
  double* tm = h.circ_stage;
  double* cols = tm + static_cast<size_t>(n) * (chunk + 1);
  double* vtab = cols + static_cast<size_t>(n) * ldc;
  circuit_buffers(h, S, chunk);
  const double f = ph.l_z / S.op.dt;
  const int kout = 3 + 2 * nb;
  std::vector<double> d(static_cast<size_t>(k) * S.c_ld), v(3 * static_cast<size_t>(ldc));
  for (int64_t i0 = 0; i0 < N; i0 += chunk) {
    const int P = static_cast<int>(std::min<int64_t>(chunk, N - i0));   // steps i0+1 .. i0+P
    MG_HIP(hipMemcpyAsync(tm, u + static_cast<size_t>(i0) * n, sizeof(double) * static_cast<size_t>(P + 1) * n,
                          h.par.device_pointers ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    launch_tm_to_slabs(s, n, P + 1, 1, tm, cols, ldc, 0, S.nat);
    launch_circ_dots(s, n, k, P, S.cBt, CView{cols + 1, ldc}, CView{cols, ldc}, S.cpart, S.c_ld);
    launch_circ_sum(s, k, P, circ_parts(n), S.cpart, S.c_ld, S.cd, S.c_ld);
    launch_source_table(s, h.src, S.op.dt, P, nullptr, i0, 1, vtab, ldc);
    MG_HIP(hipMemcpyAsync(d.data(), S.cd, sizeof(double) * d.size(), hipMemcpyDeviceToHost, s));
    MG_HIP(hipMemcpyAsync(v.data(), vtab, sizeof(double) * v.size(), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < P; ++c) {
      double* o = out + static_cast<size_t>(i0 + c) * kout;
      for (int q = 0; q < 3; ++q)
        o[q] = (v[static_cast<size_t>(q) * ldc + c] - f * d[static_cast<size_t>(q) * S.c_ld + c]) / ph.r_phase;
      for (int b = 0; b < nb; ++b) {
        double t = 0.0;
        for (int a = 0; a < nb; ++a)
          t += h.circ_Cinv[static_cast<size_t>(b) * nb + a] * f * d[static_cast<size_t>(3 + a) * S.c_ld + c];
        o[3 + b] = t;
      }
      for (int b = 0; b < nb; ++b)
        o[3 + nb + b] = -(2.0 * o[3 + b] - o[3 + (b + 1) % nb] - o[3 + (b + nb - 1) % nb]) / (2.0 * ph.ring_r);
    }
  }
}

static void seq_impl(Handle& h, const double* u0, double* u_out, mgrit_stats* st) {
  hipStream_t s = h.stream;
  h.tol_now = h.par.pcg_tol;
  h.eta_now = 0.0;
  LevelState& S0 = h.lv[0];
  if (!u_out) fail(MGRIT_INVALID_ARGUMENT, "u_out is null");
  load_u0(h, u0);
  // trajectory as a column block [n][N+1] (column t = point t)
  const int64_t ld = round_up(S0.N + 1, kWave);
  if (!h.seq_U) {
    h.seq_U = h.arena.alloc<double>(static_cast<size_t>(S0.n) * ld);
    h.seq_ws = h.arena.alloc<double>(4 * static_cast<size_t>(S0.n));
  }
  double* U = h.seq_U;
  double* ws = h.seq_ws;
  MG_HIP(hipMemsetAsync(U, 0, sizeof(double) * S0.n * ld, s));
  launch_tm_to_slabs(s, S0.n, 1, 1, h.u0_dev, U, ld, 0, S0.nat);
  int* flags = S0.pcg.flags;
  MG_HIP(hipMemsetAsync(flags, 0, 8 * sizeof(int), s));
  const bool coop = h.par.seq_kernel == 2 || (h.par.seq_kernel == 0 && S0.n >= 4096 && S0.op.W == 8);
  if (h.par.seq_kernel < 0 || h.par.seq_kernel > 3) fail(MGRIT_INVALID_ARGUMENT, "seq_kernel must be 0..3");
  auto t0 = std::chrono::steady_clock::now();
  const bool nl_persistent = S0.nl.n_tri > 0 &&
                             (h.par.seq_kernel == 1 || (h.par.seq_kernel == 0 && S0.n <= 4096));
  if (h.par.seq_kernel == 3) {
    // linear model: every step is exact implicit Euler with the level's
    // stored inverse, one stream of A^{-1} per step (built here on first use)
    if (S0.nl.n_tri > 0) fail(MGRIT_UNSUPPORTED, "seq_kernel = 3 needs the linear model");
    if (!h.seq_inv) {
      const auto tb = std::chrono::steady_clock::now();
      build_coarse_inverse(h, S0);
      // kept apart from the level: the MGRIT solve of this handle still
      // steps level 0 by its batched solves
      h.seq_inv = S0.Ainv;
      h.seq_ld_inv = S0.ld_inv;
      h.seq_bvec = S0.bvec;
      S0.Ainv = nullptr;
      S0.bvec = nullptr;
      st->time_nested_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
    }
    PcgWork& w = S0.pcg;
    t0 = std::chrono::steady_clock::now();
    for (int64_t st_i = 1; st_i <= S0.N; ++st_i) {
      // right-hand side and result as contiguous vectors (stride 1), so that
      // the product streams A^{-1} and the right-hand side coalesced
      launch_source_table(s, h.src, S0.op.dt, 1, nullptr, st_i - 1, 0, w.src, w.ld);
      launch_ie_rhs_batch(s, S0.op, 1, w.src, w.ld, CView{U + st_i - 1, ld}, h.seq_bvec, 1);
      launch_inv_gemv(s, S0.n, h.seq_inv, h.seq_ld_inv, h.seq_bvec, w.x);
      // field-circuit coupling: eliminate the circuit unknowns of the step
      if (h.circ) circuit_eliminate(h, S0, 1, w.x, 1, CView{U + st_i - 1, ld}, w.src, w.ld);
      launch_axpby3(s, S0.n, 1, U + st_i, ld, 1.0, CView{w.x, 1}, 0.0, CView{}, 0.0, CView{});
    }
    MG_HIP(hipStreamSynchronize(s));
    std::memset(S0.pcg.host_flags, 0, 4 * sizeof(int));
  } else if (nl_persistent) {
    // nonlinear, small level: the whole sweep in one persistent work-group
    if (!h.seq_nl_ws)
      h.seq_nl_ws = h.arena.alloc<double>(
          static_cast<size_t>(seq_newton_ws_doubles(S0.n, S0.op.W, S0.nl.n_tri)));
    launch_seq_newton(s, S0.op, S0.nl, h.src, static_cast<int>(S0.N), 0, U, ld, nullptr, 0, 0,
                      h.par.newton_tol, h.par.newton_max_iter, std::ldexp(1.0, -h.par.newton_halvings),
                      h.par.ir_inner_tol, h.par.pcg_max_iter, h.seq_nl_ws, flags);
    MG_HIP(hipMemcpyAsync(S0.pcg.host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    const int bits = S0.pcg.host_flags[1];
    st->newton_sweeps[0] += S0.pcg.host_flags[3];
    st->pcg_sweeps[0] += S0.pcg.host_flags[2];
    if (bits & 8) fail(MGRIT_NEWTON_NOT_CONVERGED, "Newton did not converge in newton_max_iter iterations");
    S0.pcg.host_flags[1] = bits & 3;
    S0.pcg.host_flags[2] = 0;
  } else if (S0.nl.n_tri > 0 || h.circ) {
    // nonlinear: batched Newton on one column, step after step; coupled
    // model: the batched step and its circuit elimination
    for (int64_t st = 1; st <= S0.N; ++st) {
      PhiCall c;
      c.ncols = 1;
      c.in = CView{U + st - 1, ld};
      c.t_base = st - 1;
      c.ga = c.in;
      c.out = U + st;
      c.ldo = ld;
      phi_batch(h, 0, S0.pcg, c);
    }
    MG_HIP(hipStreamSynchronize(s));
    std::memset(S0.pcg.host_flags, 0, 4 * sizeof(int));
  } else if (coop) {
    if (!h.coop_ws) {
      h.coop_blocks = seq_coop_blocks();
      h.coop_ws = h.arena.alloc<double>(5 * static_cast<size_t>(S0.n));
      h.coop_part = h.arena.alloc<double>(8 * static_cast<size_t>(h.coop_blocks));
      h.coop_bar = h.arena.alloc<unsigned>(coop_bar_words(h.coop_blocks));
    }
    const int chunk = 512;
    for (int64_t s0 = 1; s0 <= S0.N; s0 += chunk) {
      const int64_t s1 = std::min<int64_t>(S0.N + 1, s0 + chunk);
      MG_HIP(hipMemsetAsync(h.coop_bar, 0, coop_bar_words(h.coop_blocks) * sizeof(unsigned), s));
      launch_seq_coop(s, S0.op, h.src, static_cast<int>(s0), static_cast<int>(s1), U, ld, h.coop_ws,
                      h.coop_part, h.coop_bar, flags, h.par.pcg_tol, h.par.pcg_max_iter,
                      h.coop_blocks);
      MG_HIP(hipMemcpyAsync(S0.pcg.host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
      if (S0.pcg.host_flags[1]) break;
    }
  } else {
    launch_seq_small(s, S0.op, h.src, static_cast<int>(S0.N), 0, U, ld, nullptr, 0, ws,
                     h.par.pcg_tol, h.par.pcg_max_iter, 0, flags);
    MG_HIP(hipMemcpyAsync(S0.pcg.host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
  }
  st->time_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (S0.nl.n_tri == 0 && !h.circ) {
    st->phi_columns[0] += S0.N;
    st->pcg_sweeps[0] += S0.pcg.host_flags[2];
  }
  if (S0.pcg.host_flags[1] & 4) fail(MGRIT_HIP_ERROR, "a grid barrier of the sequential stepper timed out");
  if (S0.pcg.host_flags[1] & 1) fail(MGRIT_NONFINITE, "non-finite value in sequential stepping");
  if (S0.pcg.host_flags[1] & 2) fail(MGRIT_PCG_NOT_CONVERGED, "PCG did not converge in sequential stepping");
  const size_t tm_elems = static_cast<size_t>(S0.N + 1) * S0.n;
  double* tm = h.par.device_pointers ? u_out : stage(h);
  launch_slabs_to_tm(s, S0.n, S0.N + 1, 1, U, ld, 0, tm, S0.nat);
  if (!h.par.device_pointers)
    MG_HIP(hipMemcpyAsync(u_out, tm, sizeof(double) * tm_elems, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
}

static void phi_step_impl(Handle& h, int level, int B, const int64_t* i_from, const double* u_prev,
                          double* u_next) {
  h.tol_now = h.par.pcg_tol;
  h.eta_now = 0.0;
  if (level < 0 || level >= static_cast<int>(h.lv.size())) fail(MGRIT_INVALID_ARGUMENT, "level");
  if (B < 0 || (B > 0 && (!i_from || !u_prev || !u_next))) fail(MGRIT_INVALID_ARGUMENT, "phi_step arguments");
  if (B == 0) return;
  LevelState& S = h.lv[level];
  hipStream_t s = h.stream;
  if (S.user.cap < B)
    alloc_pcg(h, S.user, S.n, static_cast<int>(round_up(B, kWave)), rows_per_block_for(S.n), S.prec);
  PcgWork& w = S.user;
  // same kernel family and tile shape as the level's own sweeps
  set_rows_per_block(w, S.pcg.rows_per_block);
  w.cpl = S.pcg.cpl;
  w.dia = S.pcg.dia;
  w.depth = S.pcg.depth;
  w.rpb_narrow = S.pcg.rpb_narrow;
  // staging: time-major input/output and the column-block copy of u_prev
  double* tm = h.arena.alloc<double>(static_cast<size_t>(B) * S.n);
  double* cols = h.arena.alloc<double>(static_cast<size_t>(S.n) * w.ld);
  double* outc = h.arena.alloc<double>(static_cast<size_t>(S.n) * w.ld);
  int64_t* tl = h.arena.alloc<int64_t>(B);
  MG_HIP(hipMemcpyAsync(tm, u_prev, sizeof(double) * B * S.n, hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(tl, i_from, sizeof(int64_t) * B, hipMemcpyHostToDevice, s));
  launch_tm_to_slabs(s, S.n, B, 1, tm, cols, w.ld, 0, S.nat);
  PhiCall c;
  c.ncols = B;
  c.in = CView{cols, w.ld};
  c.t_list = tl;
  c.ga = c.in;
  c.out = outc;
  c.ldo = w.ld;
  phi_batch(h, level, w, c);
  launch_slabs_to_tm(s, S.n, B, 1, outc, w.ld, 0, tm, S.nat);
  MG_HIP(hipMemcpyAsync(u_next, tm, sizeof(double) * B * S.n, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  // release the staging buffers of this call
  for (void* p : {static_cast<void*>(tm), static_cast<void*>(cols), static_cast<void*>(outc),
                  static_cast<void*>(tl)}) {
    for (size_t k = 0; k < h.arena.ptrs.size(); ++k)
      if (h.arena.ptrs[k] == p) {
        (void)hipFree(p);
        h.arena.ptrs.erase(h.arena.ptrs.begin() + k);
        break;
      }
  }
}

// phi_step on device arrays with every buffer carved out of the static
// scratch array of the handle's device: no allocation of any kind.
static void phi_step_noalloc_impl(Handle& h, int level, int B, const int64_t* i_from,
                                  const double* u_prev, double* u_next) {
  h.tol_now = h.par.pcg_tol;
  h.eta_now = 0.0;
  if (h.circ) fail(MGRIT_UNSUPPORTED, "phi_step_noalloc does not step the field-circuit model");
  if (level < 0 || level >= static_cast<int>(h.lv.size())) fail(MGRIT_INVALID_ARGUMENT, "level");
  if (B < 0 || (B > 0 && (!i_from || !u_prev || !u_next))) fail(MGRIT_INVALID_ARGUMENT, "phi_step arguments");
  if (B == 0) return;
  LevelState& S = h.lv[level];
  if (S.nl.n_tri > 0)
    fail(MGRIT_UNSUPPORTED, "phi_step_noalloc: the nonlinear model's Newton workspace does not fit the scratch array");
  const int64_t ld = round_up(B, kWave);
  if (ld > kNoallocCols || static_cast<int64_t>(S.n) * ld > kNoallocVec)
    fail(MGRIT_INVALID_ARGUMENT, "phi_step_noalloc: n * round_up(B, 64) must be <= 2^21 and B <= 32768 (scratch size)");
  const int hist_cap = h.par.pcg_max_iter + 64;
  if (hist_cap > kNoallocHist) fail(MGRIT_INVALID_ARGUMENT, "phi_step_noalloc: pcg_max_iter must be <= 65472");
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[h.device]);
  if (!base) fail(MGRIT_HIP_ERROR, "phi_step_noalloc: scratch address not initialised");
  int cur_dev = -1;
  MG_HIP(hipGetDevice(&cur_dev));
  if (cur_dev != h.device) fail(MGRIT_INVALID_ARGUMENT, "phi_step_noalloc: the handle's device is not current");
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    void* p = base + off;
    off += align_up(bytes);
    if (off > kScratchBytes) fail(MGRIT_INVALID_ARGUMENT, "phi_step_noalloc: scratch array too small");
    return p;
  };
  const size_t V = static_cast<size_t>(S.n) * ld;
  PcgWork w;
  w.n = S.n;
  w.cap = B;
  w.ld = ld;
  w.prec = S.prec;
  set_rows_per_block(w, S.pcg.rows_per_block);
  w.cpl = S.pcg.cpl;
  w.dia = S.pcg.dia;
  w.depth = S.pcg.depth;
  w.rpb_narrow = S.pcg.rpb_narrow;
  w.x = static_cast<double*>(carve(8 * V));
  w.r = static_cast<double*>(carve(8 * V));
  w.pbuf[0] = static_cast<double*>(carve(8 * V));
  w.pbuf[1] = static_cast<double*>(carve(8 * V));
  double* cols = static_cast<double*>(carve(8 * V));
  double* outc = static_cast<double*>(carve(8 * V));
  if (w.prec == MGRIT_FP32_IR) {
    w.r32 = static_cast<float*>(carve(4 * V));
    w.x32 = static_cast<float*>(carve(4 * V));
    w.p32[0] = static_cast<float*>(carve(4 * V));
    w.p32[1] = static_cast<float*>(carve(4 * V));
  }
  const int nrb_max = (S.n + kMinRowsPerBlock - 1) / kMinRowsPerBlock;
  w.part = static_cast<double*>(carve(8 * 3 * static_cast<size_t>(nrb_max) * ld));
  w.scal = static_cast<double*>(carve(8 * 8 * static_cast<size_t>(ld)));
  w.src = static_cast<double*>(carve(8 * 3 * static_cast<size_t>(ld)));
  w.active = static_cast<uint8_t*>(carve(ld));
  w.outer = static_cast<uint8_t*>(carve(ld));
  w.flags = static_cast<int*>(carve(8 * sizeof(int)));
  w.hist_cap = hist_cap;
  w.hist = static_cast<int*>(carve(sizeof(int) * hist_cap));
  // pinned host mirrors: the level's own (one handle per thread)
  w.host_flags = S.pcg.host_flags;
  w.host_hist = S.pcg.host_hist;
  if (S.pcg.hist_cap < hist_cap) fail(MGRIT_INVALID_ARGUMENT, "phi_step_noalloc: history mirror too small");
  hipStream_t s = h.stream;
  // the array keeps the previous call's contents: clear what must start at zero
  MG_HIP(hipMemsetAsync(w.flags, 0, 8 * sizeof(int), s));
  launch_tm_to_slabs(s, S.n, B, 1, u_prev, cols, ld, 0, S.nat);
  PhiCall c;
  c.ncols = B;
  c.in = CView{cols, ld};
  c.t_list = i_from;
  c.ga = c.in;
  c.out = outc;
  c.ldo = ld;
  struct Reset {
    Handle& h;
    ~Reset() { h.noalloc = false; }
  } reset{h};
  h.noalloc = true;
  phi_batch(h, level, w, c);
  launch_slabs_to_tm(s, S.n, B, 1, outc, ld, 0, u_next, S.nat);
  MG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Learned coarse propagator: model set-up, training data, training.

static void arena_free(Handle& h, void* p) {
  for (size_t k = 0; k < h.arena.ptrs.size(); ++k)
    if (h.arena.ptrs[k] == p) {
      (void)hipFree(p);
      h.arena.ptrs.erase(h.arena.ptrs.begin() + k);
      return;
    }
}

// Graph, node flags and weight storage of the coarsest level.
static void setup_gnn(Handle& h, const mgrit_mesh& mesh, const HostPattern& pat,
                      const mgrit_physics& ph) {
  LevelState& C = h.lv.back();
  GnnModel& g = h.gnn;
  g.n = C.n;
  g.m = h.lv[h.lv.size() - 2].m;
  g.dT = C.op.dt;
  g.off = gnn_offsets(g.m);
  if (g.off.F > 32) return;                  // input features are padded to 32
  hipStream_t s = h.stream;
  const int n = C.n, W = pat.W;
  std::vector<int> ptr(n + 1, 0), idx;
  for (int i = 0; i < n; ++i) {
    const size_t first = idx.size();
    for (int k = 0; k < W; ++k) {
      const int j = pat.col[static_cast<size_t>(i) * W + k];
      if (j == i) continue;
      bool seen = false;
      for (size_t q = first; q < idx.size(); ++q) seen = seen || idx[q] == j;
      if (!seen) idx.push_back(j);
    }
    if (idx.size() == first) fail(MGRIT_UNSUPPORTED, "coarsest mesh has an unknown without neighbours");
    ptr[i + 1] = static_cast<int>(idx.size());
  }
  // flags per unknown: conductor, iron, coil (touches such a cell), radius
  std::vector<float> flags(static_cast<size_t>(n) * 4, 0.f);
  for (int t = 0; t < mesh.n_tri; ++t) {
    const int mat = mesh.cell_mat[t];
    const bool cond = ph.sigma[mat] > 0.0;
    const bool iron = ph.iron && ph.iron[mat] != 0;
    const bool coil = mesh.cell_phase[t] >= 0 && mesh.cell_sign[t] != 0;
    for (int a = 0; a < 3; ++a) {
      const int k = pat.index[mesh.tri[3 * t + a]];
      if (k < 0) continue;
      if (cond) flags[4 * k + 0] = 1.f;
      if (iron) flags[4 * k + 1] = 1.f;
      if (coil) flags[4 * k + 2] = 1.f;
    }
  }
  const int N = mesh.n_nodes;
  const double rin = std::hypot(mesh.xy[0], mesh.xy[1]);
  const double rout = std::hypot(mesh.xy[2 * (N - 1)], mesh.xy[2 * (N - 1) + 1]);
  for (int v = 0; v < N; ++v) {
    const int k = pat.index[v];
    if (k < 0) continue;
    const double r = std::hypot(mesh.xy[2 * v], mesh.xy[2 * v + 1]);
    flags[4 * k + 3] = static_cast<float>((r - rin) / (rout - rin));
  }
  g.gptr = upload_vec(h.arena, s, ptr);
  g.gidx = upload_vec(h.arena, s, idx);
  g.flags = h.arena.alloc<float>(flags.size());
  MG_HIP(hipMemcpyAsync(g.flags, flags.data(), sizeof(float) * flags.size(), hipMemcpyHostToDevice, s));
  g.F3 = C.op.F;
  const size_t np = static_cast<size_t>(g.off.n_params);
  g.w32 = h.arena.alloc<float>(np);
  g.wbf = h.arena.alloc<uint16_t>(np);
  g.grad = h.arena.alloc<float>(np);
  g.m1 = h.arena.alloc<float>(np);
  g.m2 = h.arena.alloc<float>(np);
  MG_HIP(hipMemsetAsync(g.w32, 0, sizeof(float) * np, s));
  MG_HIP(hipMemsetAsync(g.wbf, 0, sizeof(uint16_t) * np, s));
  MG_HIP(hipMemsetAsync(g.grad, 0, sizeof(float) * np, s));
  MG_HIP(hipMemsetAsync(g.m1, 0, sizeof(float) * np, s));
  MG_HIP(hipMemsetAsync(g.m2, 0, sizeof(float) * np, s));
  h.gnn_tmp = h.arena.alloc<double>(static_cast<size_t>(C.n) * C.ld);
  if (h.par.coarse_model == 1) {
    gnn_alloc_samples(g, h.arena, static_cast<int>(C.N + 1));
    gnn_alloc_rows64(g, h.arena, static_cast<int64_t>(C.n) * (C.N + 1));
  }
  h.has_gnn = true;
}

static void set_weights_impl(Handle& h, const float* w, int64_t count) {
  if (!h.has_gnn) fail(MGRIT_UNSUPPORTED, "no learned coarse propagator on this hierarchy");
  GnnModel& g = h.gnn;
  if (!w || count != g.off.n_params) fail(MGRIT_INVALID_ARGUMENT, "weight vector size");
  if (!(w[0] > 0.f) || !(w[1] > 0.f) || !(w[2] > 0.f)) fail(MGRIT_INVALID_ARGUMENT, "scales must be > 0");
  hipStream_t s = h.stream;
  const size_t np = static_cast<size_t>(count);
  MG_HIP(hipMemcpyAsync(g.w32, w, sizeof(float) * np, hipMemcpyHostToDevice, s));
  MG_HIP(hipMemsetAsync(g.m1, 0, sizeof(float) * np, s));
  MG_HIP(hipMemsetAsync(g.m2, 0, sizeof(float) * np, s));
  g.adam_step = 0;
  gnn_round_weights(s, g);
  MG_HIP(hipStreamSynchronize(s));
  g.ready = true;
}

// Host rows [B][n] (user order) of up to three arrays -> dense [n][B] (internal order).
struct GnnStaging {
  Handle& h;
  std::vector<void*> bufs;
  explicit GnnStaging(Handle& hh) : h(hh) {}
  template <class T>
  T* alloc(size_t n) {
    T* p = h.arena.alloc<T>(n);
    bufs.push_back(p);
    return p;
  }
  ~GnnStaging() {
    (void)hipStreamSynchronize(h.stream);
    for (void* p : bufs) arena_free(h, p);
  }
};

static double* stage_rows(GnnStaging& st, const double* host, int B, int n, const int* nat) {
  hipStream_t s = st.h.stream;
  double* tm = st.alloc<double>(static_cast<size_t>(B) * n);
  double* cols = st.alloc<double>(static_cast<size_t>(B) * n);
  MG_HIP(hipMemcpyAsync(tm, host, sizeof(double) * B * n, hipMemcpyHostToDevice, s));
  launch_tm_to_slabs(s, n, B, 1, tm, cols, B, 0, nat);
  return cols;
}

// Forward (and optionally backward) of the network on host samples.
static void coarse_eval_impl(Handle& h, int B, const int64_t* k, const double* amp, const double* dphi,
                             const double* u, const double* p, const double* y, double* psi_out,
                             double* loss, float* grad) {
  if (!h.has_gnn) fail(MGRIT_UNSUPPORTED, "no learned coarse propagator on this hierarchy");
  GnnModel& g = h.gnn;
  if (!g.ready) fail(MGRIT_INVALID_ARGUMENT, "coarse weights are not set");
  if (B < 1 || !k || !u || !p) fail(MGRIT_INVALID_ARGUMENT, "coarse model arguments");
  LevelState& C = h.lv.back();
  hipStream_t s = h.stream;
  const int n = C.n;
  gnn_alloc_samples(g, h.arena, B);
  if (y) gnn_alloc_rows(g, h.arena, static_cast<int64_t>(n) * B);
  else gnn_alloc_rows64(g, h.arena, static_cast<int64_t>(n) * B);
  GnnStaging st(h);
  double* uc = stage_rows(st, u, B, n, C.nat);
  double* pc = stage_rows(st, p, B, n, C.nat);
  int64_t* kd = st.alloc<int64_t>(B);
  MG_HIP(hipMemcpyAsync(kd, k, sizeof(int64_t) * B, hipMemcpyHostToDevice, s));
  double *ad = nullptr, *dd = nullptr;
  if (amp) {
    ad = st.alloc<double>(B);
    MG_HIP(hipMemcpyAsync(ad, amp, sizeof(double) * B, hipMemcpyHostToDevice, s));
  }
  if (dphi) {
    dd = st.alloc<double>(B);
    MG_HIP(hipMemcpyAsync(dd, dphi, sizeof(double) * B, hipMemcpyHostToDevice, s));
  }
  double* psi = st.alloc<double>(static_cast<size_t>(n) * B);
  const bool train = (y != nullptr);
  if (train) gnn_forward(s, g, h.src, B, kd, 0, 0, ad, dd, CView{uc, B}, CView{pc, B}, psi, B, true);
  else gnn_forward64(s, g, h.src, B, kd, 0, 0, ad, dd, CView{uc, B}, CView{pc, B}, psi, B);
  if (train) {
    double* yc = stage_rows(st, y, B, n, C.nat);
    double* ld = st.alloc<double>(1);
    MG_HIP(hipMemsetAsync(ld, 0, sizeof(double), s));
    MG_HIP(hipMemsetAsync(g.grad, 0, sizeof(float) * g.off.n_params, s));
    gnn_backward(s, g, B, psi, yc, ld);
    double lsum = 0.0;
    MG_HIP(hipMemcpyAsync(&lsum, ld, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad) MG_HIP(hipMemcpyAsync(grad, g.grad, sizeof(float) * g.off.n_params, hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (loss) *loss = lsum / (static_cast<double>(n) * B);
  }
  if (psi_out) {
    double* tm = st.alloc<double>(static_cast<size_t>(B) * n);
    launch_slabs_to_tm(s, n, B, 1, psi, B, 0, tm, C.nat);
    MG_HIP(hipMemcpyAsync(psi_out, tm, sizeof(double) * B * n, hipMemcpyDeviceToHost, s));
  }
  MG_HIP(hipStreamSynchronize(s));
}

static void coarse_adam_impl(Handle& h, const float* grad, double lr) {
  if (!h.has_gnn || !h.gnn.ready) fail(MGRIT_INVALID_ARGUMENT, "coarse weights are not set");
  if (!grad || !(lr > 0.0)) fail(MGRIT_INVALID_ARGUMENT, "coarse Adam arguments");
  GnnModel& g = h.gnn;
  hipStream_t s = h.stream;
  MG_HIP(hipMemcpyAsync(g.grad, grad, sizeof(float) * g.off.n_params, hipMemcpyHostToDevice, s));
  gnn_adam(s, g, lr, ++g.adam_step);
  MG_HIP(hipStreamSynchronize(s));
}

static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform01(uint64_t& x) { return static_cast<double>(splitmix64(x) >> 11) * 0x1.0p-53; }

// Training data from the level above the coarsest (its own propagator, m of
// its steps per coarse step, restricted to the coarse mesh), implicit-Euler
// predictions on the coarsest level, then Adam on the scaled squared error.
static void train_impl(Handle& h, const mgrit_train_params* tp, mgrit_train_stats* ts) {
  if (!tp || !ts) fail(MGRIT_INVALID_ARGUMENT, "null training parameters or statistics");
  if (h.lv.size() < 2 || !h.has_gnn) fail(MGRIT_UNSUPPORTED, "no learned coarse propagator on this hierarchy");
  if (h.circ) fail(MGRIT_UNSUPPORTED, "the learned coarse propagator does not model the circuit");
  if (tp->n_traj < 2 || tp->epochs < 1 || tp->batch < 1 || !(tp->lr > 0.0) ||
      !(tp->perturb >= 0.0 && tp->perturb <= 1.0) ||
      !(tp->amp_spread >= 0.0 && tp->amp_spread < 1.0) ||
      !(tp->val_fraction >= 0.0 && tp->val_fraction < 1.0))
    fail(MGRIT_INVALID_ARGUMENT, "bad training parameters");
  *ts = mgrit_train_stats{};
  h.st = nullptr;
  h.tol_now = h.par.pcg_tol;
  h.eta_now = 0.0;
  hipStream_t s = h.stream;
  const int L = static_cast<int>(h.lv.size());
  LevelState& C = h.lv[L - 1];
  LevelState& Gl = h.lv[L - 2];
  GnnModel& g = h.gnn;
  const int nt = tp->n_traj, m = Gl.m, n = C.n;
  const int64_t Nc = C.N;
  auto t0 = std::chrono::steady_clock::now();
  GnnStaging st(h);

  // per-trajectory source amplitude factors and phase shifts
  uint64_t rng = tp->seed;
  std::vector<double> amp(nt), dphi(nt);
  for (int b = 0; b < nt; ++b) {
    amp[b] = 1.0 + tp->amp_spread * (2.0 * uniform01(rng) - 1.0);
    dphi[b] = 6.283185307179586 * (uniform01(rng) - 0.5);
  }
  double* amp_d = st.alloc<double>(nt);
  double* dphi_d = st.alloc<double>(nt);
  MG_HIP(hipMemcpyAsync(amp_d, amp.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(dphi_d, dphi.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));

  // trajectories on the generating level: at every coarse step the state is
  // moved towards another trajectory's by alpha in [-perturb, perturb] (so
  // that pairs also sample how deviations propagate), restricted, advanced
  // by m steps and restricted again: the pair (input, target)
  const int64_t ldt = round_up(nt, kWave);
  double* X = st.alloc<double>(static_cast<size_t>(Gl.n) * ldt);
  double* Xn = st.alloc<double>(static_cast<size_t>(Gl.n) * ldt);
  MG_HIP(hipMemsetAsync(X, 0, sizeof(double) * Gl.n * ldt, s));
  const int64_t nq = Nc * nt;
  const int64_t ldD = round_up(nq, kWave);
  double* D = st.alloc<double>(static_cast<size_t>(n) * ldD);   // inputs
  double* Y = st.alloc<double>(static_cast<size_t>(n) * ldD);   // targets
  double* P = st.alloc<double>(static_cast<size_t>(n) * ldD);   // implicit Euler of the inputs
  int* perm_d = st.alloc<int>(nt);
  double* alpha_d = st.alloc<double>(nt);
  std::vector<int> perm(nt);
  std::vector<double> alpha(nt);
  PcgWork gw, cw;
  alloc_pcg(h, gw, Gl.n, nt, Gl.pcg.rows_per_block, Gl.prec);
  gw.cpl = Gl.pcg.cpl;
  gw.dia = Gl.pcg.dia;
  gw.depth = Gl.pcg.depth;
  gw.rpb_narrow = Gl.pcg.rpb_narrow;
  alloc_pcg(h, cw, C.n, nt, C.pcg.rows_per_block, C.prec);
  cw.cpl = C.pcg.cpl;
  cw.dia = C.pcg.dia;
  cw.depth = C.pcg.depth;
  cw.rpb_narrow = C.pcg.rpb_narrow;
  h.col_amp = amp_d;
  h.col_dphi = dphi_d;
  struct Reset {
    Handle& h;
    ~Reset() { h.col_amp = h.col_dphi = nullptr; }
  } reset{h};
  auto restrict_to = [&](const double* src, double* dst) {
    if (Gl.has_transfer) launch_transfer(s, Gl.R, nt, CView{src, ldt}, 1.0, dst, ldD, 0.0);
    else launch_axpby3(s, n, nt, dst, ldD, 1.0, CView{src, ldt}, 0.0, CView{}, 0.0, CView{});
  };
  for (int64_t k = 0; k < Nc; ++k) {
    if (tp->perturb > 0.0 && k > 0) {
      for (int b = 0; b < nt; ++b) {
        perm[b] = static_cast<int>(splitmix64(rng) % static_cast<uint64_t>(nt));
        alpha[b] = tp->perturb * (2.0 * uniform01(rng) - 1.0);
      }
      MG_HIP(hipStreamSynchronize(s));      // the previous step's perm / alpha are consumed
      MG_HIP(hipMemcpyAsync(perm_d, perm.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
      MG_HIP(hipMemcpyAsync(alpha_d, alpha.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
      gnn_mix(s, Gl.n, nt, X, ldt, perm_d, alpha_d, Xn);
      std::swap(X, Xn);
    }
    restrict_to(X, D + k * nt);
    for (int j = 0; j < m; ++j) {
      PhiCall c;
      c.ncols = nt;
      c.in = CView{X, ldt};
      c.t_base = k * m + j;
      c.t_stride = 0;
      c.ga = c.in;
      c.out = Xn;
      c.ldo = ldt;
      phi_batch(h, L - 2, gw, c);
      std::swap(X, Xn);
    }
    restrict_to(X, Y + k * nt);
    if (h.verbose && ((k + 1) % 16 == 0 || k + 1 == Nc)) {
      MG_HIP(hipStreamSynchronize(s));
      std::fprintf(stderr, "[mgrit train] trajectories: %lld of %lld coarse steps, %.1f s\n",
                   static_cast<long long>(k + 1), static_cast<long long>(Nc),
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      std::fflush(stderr);
    }
  }
  for (int64_t k = 0; k < Nc; ++k) {
    PhiCall c;
    c.ncols = nt;
    c.in = CView{D + k * nt, ldD};
    c.t_base = k;
    c.t_stride = 0;
    c.ga = c.in;
    c.out = P + k * nt;
    c.ldo = ldD;
    phi_batch(h, L - 1, cw, c);
  }
  h.col_amp = h.col_dphi = nullptr;
  MG_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  ts->time_data_s = std::chrono::duration<double>(t1 - t0).count();

  // samples q = k nt + b: u = D[q], p = P[q], y = Y[q]
  const int ntr_traj = std::max(1, nt - static_cast<int>(std::lround(tp->val_fraction * nt)));
  std::vector<int64_t> k_all(nq), train, val;
  std::vector<double> amp_all(nq), dphi_all(nq);
  for (int64_t q = 0; q < nq; ++q) {
    const int b = static_cast<int>(q % nt);
    k_all[q] = q / nt;
    amp_all[q] = amp[b];
    dphi_all[q] = dphi[b];
    (b < ntr_traj ? train : val).push_back(q);
  }
  int64_t* k_all_d = st.alloc<int64_t>(nq);
  double* amp_all_d = st.alloc<double>(nq);
  double* dphi_all_d = st.alloc<double>(nq);
  MG_HIP(hipMemcpyAsync(k_all_d, k_all.data(), sizeof(int64_t) * nq, hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(amp_all_d, amp_all.data(), sizeof(double) * nq, hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(dphi_all_d, dphi_all.data(), sizeof(double) * nq, hipMemcpyHostToDevice, s));

  // scales: RMS state, peak nodal forcing, RMS implicit-Euler error
  double* csum = st.alloc<double>(static_cast<size_t>(nq));
  std::vector<double> hs(nq);
  gnn_colsq(s, n, static_cast<int>(nq), Y, nullptr, ldD, csum);
  MG_HIP(hipMemcpyAsync(hs.data(), csum, sizeof(double) * nq, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  double su2 = 0.0;
  for (int64_t q : train) su2 += hs[q];
  gnn_colsq(s, n, static_cast<int>(nq), Y, P, ldD, csum);
  MG_HIP(hipMemcpyAsync(hs.data(), csum, sizeof(double) * nq, hipMemcpyDeviceToHost, s));
  std::vector<double> F3(3 * static_cast<size_t>(n));
  MG_HIP(hipMemcpyAsync(F3.data(), C.op.F, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  double so2 = 0.0;
  for (int64_t q : train) so2 += hs[q];
  double fmax = 0.0;
  for (int i = 0; i < n; ++i)
    fmax = std::max(fmax, std::fabs(F3[i]) + std::fabs(F3[n + i]) + std::fabs(F3[2 * n + i]));
  const double cnt = static_cast<double>(train.size()) * n;
  const float s_u = static_cast<float>(std::sqrt(su2 / cnt));
  const float s_f = static_cast<float>(h.src.scale * (1.0 + tp->amp_spread) * fmax);
  const float s_out = static_cast<float>(std::sqrt(so2 / cnt));
  if (!(s_u > 0.f) || !(s_f > 0.f) || !(s_out > 0.f))
    fail(MGRIT_INVALID_ARGUMENT, "training data are identically zero (no source?)");

  // initial weights: Glorot-uniform hidden matrices, zero biases and output
  {
    const GnnOffsets& o = g.off;
    std::vector<float> w(static_cast<size_t>(o.n_params), 0.f);
    w[0] = s_u;
    w[1] = s_f;
    w[2] = s_out;
    uint64_t wr = tp->seed ^ 0x5DEECE66Dull;
    auto glorot = [&](int64_t off, int fan_in, int fan_out) {
      const double lim = std::sqrt(6.0 / (fan_in + fan_out));
      for (int64_t e = 0; e < static_cast<int64_t>(fan_in) * fan_out; ++e)
        w[off + e] = static_cast<float>(lim * (2.0 * uniform01(wr) - 1.0));
    };
    glorot(o.w_in, o.F, 64);
    for (int l = 0; l < 3; ++l) {
      glorot(o.ws[l], 64, 64);
      glorot(o.wn[l], 64, 64);
    }
    set_weights_impl(h, w.data(), o.n_params);
  }

  // Adam over shuffled minibatches, cosine decay of the rate to lr/10
  const int S = static_cast<int>(std::min<int64_t>(tp->batch, static_cast<int64_t>(train.size())));
  const int64_t spe = static_cast<int64_t>(train.size()) / S;
  gnn_alloc_samples(g, h.arena, S);
  gnn_alloc_rows(g, h.arena, static_cast<int64_t>(n) * S);
  double* Ub = st.alloc<double>(static_cast<size_t>(n) * S);
  double* Pb = st.alloc<double>(static_cast<size_t>(n) * S);
  double* Yb = st.alloc<double>(static_cast<size_t>(n) * S);
  double* Psib = st.alloc<double>(static_cast<size_t>(n) * S);
  int64_t* idx_d = st.alloc<int64_t>(static_cast<size_t>(spe) * S);
  int64_t* k_b = st.alloc<int64_t>(S);
  double* amp_b = st.alloc<double>(S);
  double* dphi_b = st.alloc<double>(S);
  double* loss_d = st.alloc<double>(tp->epochs);
  MG_HIP(hipMemsetAsync(loss_d, 0, sizeof(double) * tp->epochs, s));
  const int64_t total = spe * tp->epochs;
  int64_t step = 0;
  std::vector<int64_t> order(train);
  uint64_t sh = tp->seed ^ 0x9E3779B97F4A7C15ull;
  for (int e = 0; e < tp->epochs; ++e) {
    for (int64_t i = static_cast<int64_t>(order.size()) - 1; i > 0; --i) {
      const int64_t j = static_cast<int64_t>(splitmix64(sh) % static_cast<uint64_t>(i + 1));
      std::swap(order[i], order[j]);
    }
    MG_HIP(hipStreamSynchronize(s));          // the previous epoch's indices are consumed
    MG_HIP(hipMemcpyAsync(idx_d, order.data(), sizeof(int64_t) * spe * S, hipMemcpyHostToDevice, s));
    for (int64_t b = 0; b < spe; ++b, ++step) {
      const int64_t* ib = idx_d + b * S;
      gnn_gather(s, n, S, ib, D, ldD, Ub);
      gnn_gather(s, n, S, ib, P, ldD, Pb);
      gnn_gather(s, n, S, ib, Y, ldD, Yb);
      gnn_gather_meta(s, S, ib, k_all_d, amp_all_d, dphi_all_d, k_b, amp_b, dphi_b);
      const double lr = tp->lr * (0.1 + 0.45 * (1.0 + std::cos(3.141592653589793 * step / total)));
      gnn_forward(s, g, h.src, S, k_b, 0, 0, amp_b, dphi_b, CView{Ub, S}, CView{Pb, S}, Psib, S, true);
      MG_HIP(hipMemsetAsync(g.grad, 0, sizeof(float) * g.off.n_params, s));
      gnn_backward(s, g, S, Psib, Yb, loss_d + e);
      gnn_adam(s, g, lr, ++g.adam_step);
    }
    if (h.verbose) {
      double le = 0.0;
      MG_HIP(hipMemcpyAsync(&le, loss_d + e, sizeof(double), hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
      std::fprintf(stderr, "[mgrit train] epoch %d of %d: loss %.4e, %.1f s\n", e + 1, tp->epochs,
                   le / (static_cast<double>(spe) * S * n),
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
      std::fflush(stderr);
    }
  }
  std::vector<double> losses(tp->epochs);
  MG_HIP(hipMemcpyAsync(losses.data(), loss_d, sizeof(double) * tp->epochs, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  const double per_epoch = static_cast<double>(spe) * S * n;
  ts->loss_first = losses.front() / per_epoch;
  ts->loss_last = losses.back() / per_epoch;

  // relative errors of implicit Euler and of the learned step on both sets
  auto evaluate = [&](const std::vector<int64_t>& list, double& err_ie, double& err_l) {
    double se = 0.0, sl = 0.0, sd = 0.0;
    std::vector<double> a(S), b2(S), c(S);
    double* cs = st.alloc<double>(3 * static_cast<size_t>(S));
    for (size_t q0 = 0; q0 < list.size(); q0 += S) {
      const int B = static_cast<int>(std::min<size_t>(S, list.size() - q0));
      MG_HIP(hipStreamSynchronize(s));
      MG_HIP(hipMemcpyAsync(idx_d, list.data() + q0, sizeof(int64_t) * B, hipMemcpyHostToDevice, s));
      gnn_gather(s, n, B, idx_d, D, ldD, Ub);
      gnn_gather(s, n, B, idx_d, P, ldD, Pb);
      gnn_gather(s, n, B, idx_d, Y, ldD, Yb);
      gnn_gather_meta(s, B, idx_d, k_all_d, amp_all_d, dphi_all_d, k_b, amp_b, dphi_b);
      gnn_forward(s, g, h.src, B, k_b, 0, 0, amp_b, dphi_b, CView{Ub, B}, CView{Pb, B}, Psib, B, false);
      gnn_colsq(s, n, B, Pb, Yb, B, cs);
      gnn_colsq(s, n, B, Psib, Yb, B, cs + S);
      gnn_colsq(s, n, B, Yb, Ub, B, cs + 2 * S);
      MG_HIP(hipMemcpyAsync(a.data(), cs, sizeof(double) * B, hipMemcpyDeviceToHost, s));
      MG_HIP(hipMemcpyAsync(b2.data(), cs + S, sizeof(double) * B, hipMemcpyDeviceToHost, s));
      MG_HIP(hipMemcpyAsync(c.data(), cs + 2 * S, sizeof(double) * B, hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < B; ++q) {
        se += a[q];
        sl += b2[q];
        sd += c[q];
      }
    }
    err_ie = sd > 0.0 ? std::sqrt(se / sd) : 0.0;
    err_l = sd > 0.0 ? std::sqrt(sl / sd) : 0.0;
  };
  evaluate(train, ts->train_err_ie, ts->train_err_learned);
  evaluate(val, ts->val_err_ie, ts->val_err_learned);
  ts->n_train = static_cast<int64_t>(train.size());
  ts->n_val = static_cast<int64_t>(val.size());
  ts->steps = total;
  ts->time_train_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
}

}  // namespace mg

// ---------------------------------------------------------------------------
// C ABI.

namespace {
thread_local std::string g_setup_error;

template <class F>
int guarded(mg::Handle* h, F&& f) {
  try {
    f();
    return MGRIT_OK;
  } catch (const mg::Fail& e) {
    if (h) h->last_error = e.msg;
    else g_setup_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (h) h->last_error = "host allocation failed";
    else g_setup_error = "host allocation failed";
    return MGRIT_OUT_OF_MEMORY;
  } catch (...) {
    if (h) h->last_error = "unexpected error";
    else g_setup_error = "unexpected error";
    return MGRIT_HIP_ERROR;
  }
}
}  // namespace

extern "C" {

void mgrit_default_params(mgrit_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->m = 16;
  p->gamma = 1;
  p->precision = MGRIT_FP64;
  p->restriction = MGRIT_R_NORMALIZED;
  p->tol = 1e-8;
  p->max_iter = 64;
  p->pcg_tol = 1e-12;
  p->pcg_max_iter = 5000;
  p->pcg_check_every = 4;
  p->ir_inner_tol = 1e-5;
  p->ir_max_iter = 20;
  p->newton_tol = 1e-10;
  p->newton_max_iter = 8;
  p->warm_start = 1;
  p->device_pointers = 0;
  p->profile_kernels = 0;
  p->autotune = 1;
  p->pcg_kernel = 0;
  p->coarse_inverse = 2;
  p->seq_kernel = 0;
  p->use_graphs = 1;
  p->newton_halvings = 6;
  p->pcg_tol_eta = 0.0;
  p->precision_coarse = -1;
  p->compact_columns = 64;
  p->compact_fraction = 0.9;
  p->pcg_prefetch = 0;
  p->residual_eta = 0.0;
  p->pcg_rows_narrow = 0;
  p->cycle = 0;
  p->nested = 0;
  p->loss_tol = 0.0;
  p->m_coarse = 0;
  p->coarse_persistent = 0;
  p->pcg_check_narrow = 16;
  p->pcg_rows_per_block = 0;
  p->pcg_cols_per_lane = 0;
}

int mgrit_setup(const mgrit_problem* prob, const mgrit_params* par, void* hip_stream, void** out) {
  if (!out) return MGRIT_INVALID_ARGUMENT;
  *out = nullptr;
  auto h = std::make_unique<mg::Handle>();
  h->stream = static_cast<hipStream_t>(hip_stream);
  const int rc = guarded(nullptr, [&] { mg::setup_impl(*h, prob, par); });
  if (rc != MGRIT_OK) return rc;
  *out = h.release();
  return MGRIT_OK;
}

int mgrit_solve(void* hp, const double* u0, const double* u_init, double* u_out, mgrit_stats* st) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  mgrit_stats local;
  mgrit_stats* s = st ? st : &local;
  std::memset(s, 0, sizeof(*s));
  h->st = s;
  const int rc = guarded(h, [&] { mg::solve_impl(*h, u0, u_init, u_out, s); });
  h->st = nullptr;
  return rc;
}

int mgrit_seq_solve(void* hp, const double* u0, double* u_out, mgrit_stats* st) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  mgrit_stats local;
  mgrit_stats* s = st ? st : &local;
  std::memset(s, 0, sizeof(*s));
  h->st = s;
  const int rc = guarded(h, [&] { mg::seq_impl(*h, u0, u_out, s); });
  h->st = nullptr;
  return rc;
}

int phi_step(void* hp, int32_t level, int32_t B, const int64_t* i_from, const double* u_prev,
             double* u_next) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::phi_step_impl(*h, level, B, i_from, u_prev, u_next); });
}

int phi_step_noalloc(void* hp, int32_t level, int32_t B, const int64_t* i_from, const double* u_prev,
                     double* u_next) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::phi_step_noalloc_impl(*h, level, B, i_from, u_prev, u_next); });
}

int mgrit_joule_losses(void* hp, double* p) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::joule_impl(*h, p); });
}

int mgrit_circuit_values(void* hp, const double* u, double* out) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::circuit_values_impl(*h, u, out); });
}

int mgrit_level_info(void* hp, int32_t level, int64_t* n, int64_t* n_steps, int64_t* nnz,
                     int32_t* kernel_shape) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h || level < 0 || level >= static_cast<int>(h->lv.size())) return MGRIT_INVALID_ARGUMENT;
  const auto& S = h->lv[level];
  if (n) *n = S.n;
  if (n_steps) *n_steps = S.N;
  if (nnz) *nnz = static_cast<int64_t>(S.n) * S.op.W;
  if (kernel_shape) {
    kernel_shape[0] = S.pcg.rows_per_block;
    kernel_shape[1] = S.pcg.cpl;
    kernel_shape[2] = S.pcg.dia ? 2 : 1;
    kernel_shape[3] = S.pcg.dia ? S.pcg.depth : 1;
    kernel_shape[4] = S.pcg.rpb_narrow;
  }
  return MGRIT_OK;
}

int mgrit_train_coarse(void* hp, const mgrit_train_params* tp, mgrit_train_stats* ts) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::train_impl(*h, tp, ts); });
}

int64_t mgrit_coarse_n_params(void* hp) {
  auto* h = static_cast<mg::Handle*>(hp);
  return (h && h->has_gnn) ? h->gnn.off.n_params : 0;
}

int mgrit_set_coarse_weights(void* hp, const float* w, int64_t n) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::set_weights_impl(*h, w, n); });
}

int mgrit_get_coarse_weights(void* hp, float* w, int64_t n) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] {
    if (!h->has_gnn) mg::fail(MGRIT_UNSUPPORTED, "no learned coarse propagator on this hierarchy");
    if (!w || n != h->gnn.off.n_params) mg::fail(MGRIT_INVALID_ARGUMENT, "weight vector size");
    MG_HIP(hipMemcpyAsync(w, h->gnn.w32, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream));
    MG_HIP(hipStreamSynchronize(h->stream));
  });
}

int mgrit_coarse_apply(void* hp, int32_t B, const int64_t* k, const double* amp, const double* dphi,
                       const double* u, const double* p, double* psi) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] {
    if (!psi) mg::fail(MGRIT_INVALID_ARGUMENT, "psi is null");
    mg::coarse_eval_impl(*h, B, k, amp, dphi, u, p, nullptr, psi, nullptr, nullptr);
  });
}

int mgrit_coarse_gradient(void* hp, int32_t B, const int64_t* k, const double* amp,
                          const double* dphi, const double* u, const double* p, const double* y,
                          double* loss, float* grad) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] {
    if (!y || !loss || !grad) mg::fail(MGRIT_INVALID_ARGUMENT, "y, loss and grad are required");
    mg::coarse_eval_impl(*h, B, k, amp, dphi, u, p, y, nullptr, loss, grad);
  });
}

int mgrit_coarse_adam(void* hp, const float* grad, double lr) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return MGRIT_INVALID_ARGUMENT;
  return guarded(h, [&] { mg::coarse_adam_impl(*h, grad, lr); });
}

void mgrit_destroy(void* hp) {
  auto* h = static_cast<mg::Handle*>(hp);
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (auto e : h->ev) (void)hipEventDestroy(e);
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  delete h;
}

const char* mgrit_strerror(int status) {
  switch (status) {
    case MGRIT_OK: return "ok";
    case MGRIT_INVALID_ARGUMENT: return "invalid argument";
    case MGRIT_NOT_NESTED: return "meshes are not nested";
    case MGRIT_OUT_OF_MEMORY: return "out of memory";
    case MGRIT_HIP_ERROR: return "HIP runtime error";
    case MGRIT_PCG_NOT_CONVERGED: return "PCG did not converge";
    case MGRIT_NEWTON_NOT_CONVERGED: return "Newton did not converge";
    case MGRIT_NOT_CONVERGED: return "MGRIT did not converge";
    case MGRIT_NONFINITE: return "non-finite value";
    case MGRIT_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* mgrit_last_error(void* hp) {
  auto* h = static_cast<mg::Handle*>(hp);
  return h ? h->last_error.c_str() : g_setup_error.c_str();
}

}  // extern "C"
