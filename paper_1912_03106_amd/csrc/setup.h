// Host-side setup helpers (patterns, transfers, device memory arena).
#pragma once

#include <vector>

#include "internal.h"

namespace mg {

struct DeviceArena {
  std::vector<void*> ptrs;
  std::vector<void*> host_ptrs;
  void* alloc_bytes(size_t bytes);
  void* alloc_host(size_t bytes);
  template <class T>
  T* alloc(size_t n) {
    return static_cast<T*>(alloc_bytes(sizeof(T) * n));
  }
  void release();
  ~DeviceArena() { release(); }
};

// Interior-node operator pattern with fixed row width W.
struct HostPattern {
  int n = 0, W = 0;
  std::vector<int> index;    // node -> internal unknown index or -1 (Dirichlet)
  std::vector<int> nat;      // internal unknown -> user-facing (node-id order) index
  std::vector<int> col;      // [n*W]
  std::vector<int> cptr;     // [n*W + 1] contribution list per stored entry
  std::vector<int> contrib;  // element*9 + a*3 + b
  std::vector<int> diag;     // [n] slot of the diagonal entry
};

struct HostSparse {
  int n_out = 0, n_in = 0, W = 0;
  std::vector<int> col;
  std::vector<double> val;
};

template <class T>
T* upload_vec(DeviceArena& A, hipStream_t s, const std::vector<T>& v);

// Per-element device data kept for the nonlinear model.
struct ElementData {
  int n_tri = 0;
  double* area = nullptr;
  double* grad = nullptr;   // [n_tri][3][2]
  int* tri = nullptr;
  double* nu = nullptr;     // linear reluctivity per element
  double* sigma = nullptr;
  uint8_t* iron = nullptr;
  int* cptr = nullptr;
  int* contrib = nullptr;
  int* diag = nullptr;
  int* tri_u = nullptr;     // [n_tri][3] unknown index per vertex (-1 = Dirichlet)
};

void validate_mesh(const mgrit_mesh& m, int n_materials);
HostPattern build_pattern(const mgrit_mesh& m);
bool same_mesh(const mgrit_mesh& a, const mgrit_mesh& b);
HostSparse build_prolongation(const mgrit_mesh& f, const mgrit_mesh& c, const HostPattern& pf,
                              const HostPattern& pc);
HostSparse build_restriction(const HostSparse& P, int kind, const mgrit_mesh& f,
                             const mgrit_mesh& c, const HostPattern& pf, const HostPattern& pc);
DevTransfer upload_transfer(DeviceArena& A, hipStream_t s, const HostSparse& T);
DevLevel assemble_level(DeviceArena& A, hipStream_t s, const mgrit_mesh& m, const HostPattern& P,
                        const mgrit_physics& ph, double dt, ElementData* keep);

}  // namespace mg
