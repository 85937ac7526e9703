// Field-circuit coupling of the linear model (Sec. 3.1, the stator coil and
// rotor bar circuit equations): kernels of the coupled step.
//
// A coupled step solves, for the vector potential a' and the k circuit
// unknowns w = (stator currents i_1..3, bar voltages v_1..nb),
//   A a' - B^T w = (M/dt) a                       (field rows)
//   (l_z/dt) E B (a' - a) + D w = (v(t'); 0)      (circuit rows)
// with B = [X; Y'/l_z] (k x n), E = diag(1, 1, 1, -1, ..., -1) and
// D = diag(r_phase I_3, C).  Eliminating a' = y + Z w with y = A^-1 (M/dt) a
// (the level's ordinary source-free step) and Z = A^-1 B^T (set-up):
//   w = S^-1 (v; 0) - S^-1 (l_z/dt) E B (y - a),  S = (l_z/dt) E B Z + D,
// so after the step's linear solve a batched column needs only k dot
// products with y - a, a k x k product and a' = y + Z w.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mg {

constexpr int kCircMax = 35;          // 3 phase currents + at most 32 bar voltages
constexpr int kCircRowsPerWave = 256; // rows of one wave's partial dot products

// CG start for A x = b with a dense right-hand side b (column c of row i at
// B[i * ldb + c]): x = 0, r^ = S b, partials r^.r^, b.b, b.b in the layout
// the reduce expects; block 0 clears the active-column counter.
void launch_circ_rhs_init(hipStream_t s, const DevLevel& L, PcgWork& w, const double* B, int64_t ldb,
                          int ncols);
// Number of per-wave partial sums of launch_circ_dots for n rows.
int circ_parts(int n);
// part[p][j][c] = sum over the rows of wave partial p of Bt[i][j] (y[i][c] - a[i][c]),
// Bt row-major [n][k]; ldp >= ncols.
void launch_circ_dots(hipStream_t s, int n, int k, int ncols, const double* Bt, CView y, CView a,
                      double* part, int64_t ldp);
// The same partials plus those of Z^T r, r = (M/dt) a - A y the residual of an
// inexact solve for y (L's rows, Z row-major [n][k]): the circuit rows of the
// exact step, whatever the solve left.
void launch_circ_dots_res(hipStream_t s, const DevLevel& L, int k, int ncols, const double* Bt,
                          const double* Z, CView y, CView a, double* part, int64_t ldp);
// d[j][c] = sum over p in order of part[p][j][c].
void launch_circ_sum(hipStream_t s, int k, int ncols, int nparts, const double* part, int64_t ldp,
                     double* d, int64_t ldd);
// w[j][c] = sum_q Sv[j][q] v_q(c) - sum_l Q[j][l] d[l][c]; cS row-major [k][3 + k]
// (Sv = S^-1 columns 0..2, Q = S^-1 (l_z/dt) E); v_q(c) = src[q * lds + c].
void launch_circ_solve(hipStream_t s, int k, int ncols, const double* d, int64_t ldd,
                       const double* src, int64_t lds, const double* cS, double* w, int64_t ldw);
// x[i][c] += sum_j Z[i][j] w[j][c], Z row-major [n][k].
void launch_circ_apply(hipStream_t s, int n, int k, int ncols, const double* Z, const double* w,
                       int64_t ldw, double* x, int64_t ldx);
// Per-time-point store wt [k][nt] of the circuit unknowns (i = t_list[c], or
// t_base + c t_stride without a list; points outside [0, nt) are skipped):
// recall writes w[j][c] = -wt[j][i] (so that launch_circ_apply subtracts
// Z w), keep writes wt[j][i] = w[j][c].
void launch_circ_recall(hipStream_t s, int k, int ncols, const int64_t* t_list, int64_t t_base,
                        int64_t t_stride, const double* wt, int64_t nt, double* w, int64_t ldw);
void launch_circ_keep(hipStream_t s, int k, int ncols, const int64_t* t_list, int64_t t_base,
                      int64_t t_stride, const double* w, int64_t ldw, double* wt, int64_t nt);

}  // namespace mg
