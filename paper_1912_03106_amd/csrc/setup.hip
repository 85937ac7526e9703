// Setup of the level hierarchy: sparsity patterns, element -> entry
// contribution lists, device assembly of the operators (eq. 7, 8) and the
// spatial transfers between nested polar meshes (Sec. 3.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "setup.h"

namespace mg {

void fail(int code, const std::string& msg) { throw Fail{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? MGRIT_OUT_OF_MEMORY
                                                                                : MGRIT_HIP_ERROR;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

void DeviceArena::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  for (void* p : host_ptrs) (void)hipHostFree(p);
  host_ptrs.clear();
}

void* DeviceArena::alloc_bytes(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  MG_HIP(hipMalloc(&p, bytes));
  ptrs.push_back(p);
  return p;
}

void* DeviceArena::alloc_host(size_t bytes) {
  void* p = nullptr;
  MG_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  host_ptrs.push_back(p);
  return p;
}

void validate_mesh(const mgrit_mesh& m, int n_materials) {
  if (m.n_nodes <= 0 || m.n_tri <= 0 || !m.xy || !m.tri || !m.cell_mat || !m.cell_phase ||
      !m.cell_sign || !m.dirichlet)
    fail(MGRIT_INVALID_ARGUMENT, "mesh: missing array or empty mesh");
  for (int64_t k = 0; k < 3LL * m.n_tri; ++k)
    if (m.tri[k] < 0 || m.tri[k] >= m.n_nodes) fail(MGRIT_INVALID_ARGUMENT, "mesh: node id out of range");
  for (int e = 0; e < m.n_tri; ++e) {
    if (m.cell_mat[e] < 0 || m.cell_mat[e] >= n_materials)
      fail(MGRIT_INVALID_ARGUMENT, "mesh: material index out of range");
    if (m.cell_phase[e] < -1 || m.cell_phase[e] > 2) fail(MGRIT_INVALID_ARGUMENT, "mesh: phase out of range");
    const int* t = m.tri + 3 * e;
    const double* a = m.xy + 2 * t[0];
    const double* b = m.xy + 2 * t[1];
    const double* c = m.xy + 2 * t[2];
    const double det = (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]);
    if (!(det > 0.0)) fail(MGRIT_INVALID_ARGUMENT, "mesh: triangle not counter-clockwise or degenerate");
  }
  for (int64_t k = 0; k < 2LL * m.n_nodes; ++k)
    if (!std::isfinite(m.xy[k])) fail(MGRIT_NONFINITE, "mesh: non-finite coordinate");
  if (m.n_r > 0 && m.n_theta > 0 && (int64_t)(m.n_r + 1) * m.n_theta != m.n_nodes)
    fail(MGRIT_INVALID_ARGUMENT, "mesh: n_r, n_theta do not match the node count");
}

// Pattern of the interior-node operator with fixed row width and, for every
// stored entry, the list of (element, a, b) local-matrix contributions.
HostPattern build_pattern(const mgrit_mesh& m) {
  HostPattern P;
  P.index.assign(m.n_nodes, -1);
  int n = 0;
  if (m.n_r > 0 && m.n_theta > 0) {
    // Polar mesh: number the unknowns angle-major (radial index fastest), so
    // a row's neighbours lie within about n_r rows of it instead of n_theta;
    // the batched kernels then find them in L2 (see the layout note in
    // kernels.hip).  The user-facing order stays the node-id order.
    for (int j = 0; j < m.n_theta; ++j)
      for (int i = 0; i <= m.n_r; ++i) {
        const int v = i * m.n_theta + j;
        if (!m.dirichlet[v]) P.index[v] = n++;
      }
  } else {
    for (int v = 0; v < m.n_nodes; ++v)
      if (!m.dirichlet[v]) P.index[v] = n++;
  }
  if (n == 0) fail(MGRIT_INVALID_ARGUMENT, "mesh: no unknowns");
  P.n = n;
  P.nat.assign(n, 0);
  for (int v = 0, k = 0; v < m.n_nodes; ++v)
    if (!m.dirichlet[v]) P.nat[P.index[v]] = k++;
  // node -> incident (element, local index)
  std::vector<int> start(m.n_nodes + 1, 0);
  for (int64_t k = 0; k < 3LL * m.n_tri; ++k) start[m.tri[k] + 1]++;
  for (int v = 0; v < m.n_nodes; ++v) start[v + 1] += start[v];
  std::vector<int> inc(3LL * m.n_tri), fillp(start.begin(), start.end() - 1);
  for (int e = 0; e < m.n_tri; ++e)
    for (int a = 0; a < 3; ++a) inc[fillp[m.tri[3 * e + a]]++] = e * 3 + a;

  std::vector<std::vector<std::pair<int, int>>> rows(n);  // (column, code)
  int wmax = 0;
  for (int v = 0; v < m.n_nodes; ++v) {
    const int r = P.index[v];
    if (r < 0) continue;
    auto& lst = rows[r];
    for (int k = start[v]; k < start[v + 1]; ++k) {
      const int e = inc[k] / 3, a = inc[k] % 3;
      for (int b = 0; b < 3; ++b) {
        const int c = P.index[m.tri[3 * e + b]];
        if (c < 0) continue;
        lst.emplace_back(c, e * 9 + a * 3 + b);
      }
    }
    std::sort(lst.begin(), lst.end());
    int ucols = 0;
    for (size_t k = 0; k < lst.size(); ++k)
      if (k == 0 || lst[k].first != lst[k - 1].first) ++ucols;
    wmax = std::max(wmax, ucols);
  }
  if (wmax <= 8) P.W = 8;
  else if (wmax <= 16) P.W = 16;
  else fail(MGRIT_UNSUPPORTED, "mesh: a node has more than 15 neighbours");
  const int W = P.W;
  P.col.assign(static_cast<size_t>(n) * W, 0);
  P.cptr.assign(static_cast<size_t>(n) * W + 1, 0);
  P.diag.assign(n, -1);
  P.contrib.clear();
  for (int r = 0; r < n; ++r) {
    const auto& lst = rows[r];
    int slot = -1, prev = -1;
    size_t k = 0;
    for (int s = 0; s < W; ++s) {
      const size_t idx = static_cast<size_t>(r) * W + s;
      P.cptr[idx] = static_cast<int>(P.contrib.size());
      if (k < lst.size()) {
        const int c = lst[k].first;
        P.col[idx] = c;
        if (c == r) P.diag[r] = s;
        while (k < lst.size() && lst[k].first == c) P.contrib.push_back(lst[k++].second);
      } else {
        P.col[idx] = r;  // padding: zero entry on the diagonal column
      }
    }
    (void)slot;
    (void)prev;
  }
  P.cptr[static_cast<size_t>(n) * W] = static_cast<int>(P.contrib.size());
  for (int r = 0; r < n; ++r)
    if (P.diag[r] < 0) fail(MGRIT_INVALID_ARGUMENT, "mesh: unknown without element");
  return P;
}

static bool coords_match(const mgrit_mesh& f, int vf, const mgrit_mesh& c, int vc) {
  const double dx = f.xy[2 * vf] - c.xy[2 * vc], dy = f.xy[2 * vf + 1] - c.xy[2 * vc + 1];
  const double scale = 1.0 + std::fabs(c.xy[2 * vc]) + std::fabs(c.xy[2 * vc + 1]);
  return std::sqrt(dx * dx + dy * dy) <= 1e-12 * scale;
}

bool same_mesh(const mgrit_mesh& a, const mgrit_mesh& b) {
  if (&a == &b) return true;
  if (a.n_nodes != b.n_nodes || a.n_tri != b.n_tri) return false;
  if (std::memcmp(a.tri, b.tri, sizeof(int32_t) * 3 * a.n_tri) != 0) return false;
  for (int v = 0; v < a.n_nodes; ++v)
    if (!coords_match(a, v, b, v) || a.dirichlet[v] != b.dirichlet[v]) return false;
  return true;
}

// Nodal interpolation from the coarse to the fine polar mesh in logical
// coordinates: fine (2i,2j) takes coarse (i,j); a fine node at the midpoint of
// a coarse edge -- radial (2i+1, 2j), angular (2i, 2j+1) or the cell diagonal
// (2i+1, 2j+1) -- takes half of each end point.  Dirichlet coarse nodes carry 0
// and are dropped.  Rows are fine unknowns, columns coarse unknowns.
HostSparse build_prolongation(const mgrit_mesh& f, const mgrit_mesh& c, const HostPattern& pf,
                              const HostPattern& pc) {
  if (f.n_r <= 0 || c.n_r <= 0 || f.n_r != 2 * c.n_r || f.n_theta != 2 * c.n_theta)
    fail(MGRIT_NOT_NESTED, "spatial coarsening needs polar meshes with n_r and n_theta doubled");
  for (int i = 0; i <= c.n_r; ++i)
    for (int j = 0; j < c.n_theta; ++j)
      if (!coords_match(f, (2 * i) * f.n_theta + 2 * j, c, i * c.n_theta + j))
        fail(MGRIT_NOT_NESTED, "coarse node does not coincide with its fine node");
  HostSparse P;
  P.n_out = pf.n;
  P.n_in = pc.n;
  P.W = 2;
  P.col.assign(static_cast<size_t>(pf.n) * 2, 0);
  P.val.assign(static_cast<size_t>(pf.n) * 2, 0.0);
  const int ntc = c.n_theta;
  auto cidx = [&](int i, int j) { return pc.index[i * ntc + ((j % ntc) + ntc) % ntc]; };
  for (int v = 0; v < f.n_nodes; ++v) {
    const int row = pf.index[v];
    if (row < 0) continue;
    const int I = v / f.n_theta, J = v % f.n_theta;
    int ids[2] = {-1, -1};
    double w[2] = {0.0, 0.0};
    if (I % 2 == 0 && J % 2 == 0) {
      ids[0] = cidx(I / 2, J / 2); w[0] = 1.0;
    } else if (I % 2 == 1 && J % 2 == 0) {
      ids[0] = cidx((I - 1) / 2, J / 2); ids[1] = cidx((I + 1) / 2, J / 2); w[0] = w[1] = 0.5;
    } else if (I % 2 == 0) {
      ids[0] = cidx(I / 2, (J - 1) / 2); ids[1] = cidx(I / 2, (J + 1) / 2); w[0] = w[1] = 0.5;
    } else {
      ids[0] = cidx((I - 1) / 2, (J - 1) / 2); ids[1] = cidx((I + 1) / 2, (J + 1) / 2);
      w[0] = w[1] = 0.5;
    }
    int k = 0;
    for (int t = 0; t < 2; ++t) {
      if (ids[t] < 0 || w[t] == 0.0) continue;
      P.col[static_cast<size_t>(row) * 2 + k] = ids[t];
      P.val[static_cast<size_t>(row) * 2 + k] = w[t];
      ++k;
    }
    for (; k < 2; ++k) P.col[static_cast<size_t>(row) * 2 + k] = 0;  // zero-weight padding
  }
  return P;
}

// R_s from P_s: transpose (kind 1), its row-normalised form D^{-1} P^T
// (kind 0), or injection of the coincident fine node (kind 2).
HostSparse build_restriction(const HostSparse& P, int kind, const mgrit_mesh& f,
                             const mgrit_mesh& c, const HostPattern& pf, const HostPattern& pc) {
  HostSparse R;
  R.n_out = P.n_in;
  R.n_in = P.n_out;
  std::vector<std::vector<std::pair<int, double>>> rows(R.n_out);
  if (kind == MGRIT_R_INJECTION) {
    for (int v = 0; v < c.n_nodes; ++v) {
      const int r = pc.index[v];
      if (r < 0) continue;
      const int i = v / c.n_theta, j = v % c.n_theta;
      rows[r].emplace_back(pf.index[(2 * i) * f.n_theta + 2 * j], 1.0);
    }
  } else {
    for (int fr = 0; fr < P.n_out; ++fr)
      for (int k = 0; k < P.W; ++k) {
        const double w = P.val[static_cast<size_t>(fr) * P.W + k];
        if (w != 0.0) rows[P.col[static_cast<size_t>(fr) * P.W + k]].emplace_back(fr, w);
      }
  }
  int wmax = 1;
  for (auto& r : rows) {
    std::sort(r.begin(), r.end());
    wmax = std::max<int>(wmax, static_cast<int>(r.size()));
  }
  R.W = wmax <= 2 ? 2 : wmax <= 4 ? 4 : wmax <= 8 ? 8 : 16;
  if (wmax > 16) fail(MGRIT_UNSUPPORTED, "restriction row wider than 16");
  R.col.assign(static_cast<size_t>(R.n_out) * R.W, 0);
  R.val.assign(static_cast<size_t>(R.n_out) * R.W, 0.0);
  for (int r = 0; r < R.n_out; ++r) {
    double d = 0.0;
    for (auto& e : rows[r]) d += e.second;
    if (kind == MGRIT_R_NORMALIZED && !(d > 0.0)) fail(MGRIT_NOT_NESTED, "empty restriction row");
    const double s = (kind == MGRIT_R_NORMALIZED) ? 1.0 / d : 1.0;
    for (size_t k = 0; k < rows[r].size(); ++k) {
      R.col[static_cast<size_t>(r) * R.W + k] = rows[r][k].first;
      R.val[static_cast<size_t>(r) * R.W + k] = rows[r][k].second * s;
    }
  }
  return R;
}

template <class T>
static T* upload(DeviceArena& A, hipStream_t s, const std::vector<T>& v) {
  T* d = A.alloc<T>(v.size());
  if (!v.empty()) MG_HIP(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  return d;
}

template <class T>
static T* upload_raw(DeviceArena& A, hipStream_t s, const T* p, size_t n) {
  T* d = A.alloc<T>(n);
  MG_HIP(hipMemcpyAsync(d, p, sizeof(T) * n, hipMemcpyHostToDevice, s));
  return d;
}

template <class T>
T* upload_vec(DeviceArena& A, hipStream_t s, const std::vector<T>& v) {
  return upload(A, s, v);
}
template int* upload_vec<int>(DeviceArena&, hipStream_t, const std::vector<int>&);

DevTransfer upload_transfer(DeviceArena& A, hipStream_t s, const HostSparse& T) {
  DevTransfer d;
  d.n_out = T.n_out;
  d.n_in = T.n_in;
  d.W = T.W;
  d.col = upload(A, s, T.col);
  d.val = upload(A, s, T.val);
  return d;
}

// Assemble A = M/dt + K, M/dt, diag(A)^{-1} and the phase load vectors of one
// level on the device.  `keep` receives the per-element data reused by the
// nonlinear model.
DevLevel assemble_level(DeviceArena& A, hipStream_t s, const mgrit_mesh& m, const HostPattern& P,
                        const mgrit_physics& ph, double dt, ElementData* keep) {
  DevLevel L;
  L.n = P.n;
  L.W = P.W;
  L.dt = dt;
  const size_t slots = static_cast<size_t>(P.n) * P.W;
  L.col = upload(A, s, P.col);
  L.a64 = A.alloc<double>(slots);
  L.a32 = A.alloc<float>(slots);
  L.m64 = A.alloc<double>(slots);
  L.has_mass = A.alloc<uint8_t>(P.n);
  L.dinv64 = A.alloc<double>(P.n);
  L.dinv32 = A.alloc<float>(P.n);
  L.F = A.alloc<double>(3 * static_cast<size_t>(P.n));
  L.s64 = A.alloc<double>(P.n);
  L.s32 = A.alloc<float>(P.n);
  L.d64 = A.alloc<double>(P.n);
  L.ah64 = A.alloc<double>(slots);
  L.ah32 = A.alloc<float>(slots);
  int* cptr = upload(A, s, P.cptr);
  int* contrib = upload(A, s, P.contrib);
  int* diag = upload(A, s, P.diag);
  double* xy = upload_raw(A, s, m.xy, 2 * static_cast<size_t>(m.n_nodes));
  int* tri = upload_raw(A, s, m.tri, 3 * static_cast<size_t>(m.n_tri));
  int* phase = upload_raw(A, s, m.cell_phase, m.n_tri);
  int* sign = upload_raw(A, s, m.cell_sign, m.n_tri);
  std::vector<double> nu_e(m.n_tri), sig_e(m.n_tri);
  std::vector<uint8_t> iron_e(m.n_tri);
  for (int e = 0; e < m.n_tri; ++e) {
    nu_e[e] = ph.nu[m.cell_mat[e]];
    sig_e[e] = ph.sigma[m.cell_mat[e]];
    iron_e[e] = static_cast<uint8_t>(ph.iron ? (ph.iron[m.cell_mat[e]] != 0) : 0);
  }
  double* dnu = upload(A, s, nu_e);
  double* dsig = upload(A, s, sig_e);
  double* area = A.alloc<double>(m.n_tri);
  double* grad = A.alloc<double>(6 * static_cast<size_t>(m.n_tri));
  launch_elem_geometry(s, m.n_tri, xy, tri, area, grad);
  launch_assemble_linear(s, L, cptr, contrib, area, grad, dnu, dsig);
  launch_diag_inverse(s, L, diag);
  launch_load_vectors(s, L, cptr, contrib, diag, area, phase, sign);
  launch_scale_matrix(s, L, diag);
  // Polar mesh numbered angle-major with both radii Dirichlet: the operator
  // is the periodic 7-diagonal stencil with R = n_r - 1 unknowns per ray.
  if (m.n_r > 2 && m.n_theta > 2 && P.n == (m.n_r - 1) * m.n_theta &&
      2 * (m.n_r - 1) + 2 < P.n) {
    L.dia_R = m.n_r - 1;
    L.dv64 = A.alloc<double>(static_cast<size_t>(P.n) * 8);
    L.dv32 = A.alloc<float>(static_cast<size_t>(P.n) * 8);
    int* bad = A.alloc<int>(1);
    MG_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    launch_build_dia(s, L, bad);
    int hbad = 0;
    MG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (hbad != 0) L.dia_R = 0;
  }
  if (keep) {
    keep->n_tri = m.n_tri;
    keep->area = area;
    keep->grad = grad;
    keep->tri = tri;
    keep->nu = dnu;
    keep->sigma = dsig;
    keep->iron = upload(A, s, iron_e);
    keep->cptr = cptr;
    keep->contrib = contrib;
    keep->diag = diag;
    std::vector<int> tu(3 * static_cast<size_t>(m.n_tri));
    for (int64_t k = 0; k < 3LL * m.n_tri; ++k) tu[k] = P.index[m.tri[k]];
    keep->tri_u = upload(A, s, tu);
  }
  return L;
}

}  // namespace mg
