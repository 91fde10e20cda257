// Internal state behind the opaque ipdg_mesh handle.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ipdg.h"
#include "kernels.hpp"
#include "mesh_host.hpp"

namespace ipdg {

// Error carrying an ABI status; thrown inside the library, caught at the ABI.
struct Error : std::runtime_error {
  ipdg_status status;
  Error(ipdg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define IPDG_HIP(call)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::ipdg::Error(IPDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Device buffer owned by the library (hipMalloc / hipFree).
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  void alloc(size_t bytes);
  void ensure(size_t bytes) { if (bytes > n_) { release(); alloc(bytes); } }
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t size() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// Reference operators of degree N in the precision of `kind` (F32_IN64 uses
// FP32 tables), resident on the current device for the process lifetime.
const void* device_ops(int N, Kind kind);
// The same table if it is already resident on the current device, else null
// (never uploads).
const void* device_ops_resident(int N, Kind kind);
// Interpolation matrix degree Nc -> Nf (Np(Nf) x Np(Nc)), FP64 or FP32.
const void* device_interp(int Nc, int Nf, bool fp32);

struct SolverWork;   // solver workspaces (solver.cpp)

}  // namespace ipdg

struct ipdg_mesh_s {
  ipdg::HostMesh host;
  int device = 0;
  int Np = 0;
  bool has_kappa = false;
  std::vector<double> kappa;      // host copy (K) when has_kappa
  unsigned kappa_version = 0;     // changes whenever the coefficient values change
  ipdg::DevBuf geo64, geo32, conn, kap64, kap32;
  ipdg::DevBuf ones64;            // kappa = 1 for the coefficient gradient of a plain mesh
  ipdg::DevBuf sub_work;          // Runge-Kutta registers of the subcycle (4 K Np doubles)
  std::unique_ptr<ipdg::SolverWork> work;
  ~ipdg_mesh_s();
};

namespace ipdg {

inline const void* geo_for(const ipdg_mesh_s* m, Kind k) {
  return k == Kind::F64 ? m->geo64.get() : m->geo32.get();
}
inline const void* kap_for(const ipdg_mesh_s* m, Kind k) {
  if (!m->has_kappa) return nullptr;
  return k == Kind::F64 ? m->kap64.get() : m->kap32.get();
}
// Penalty constant: c_tau <= 0 selects (N+1)^2.
inline double ctau_of(int N, double tau) { return tau > 0.0 ? tau : double((N + 1) * (N + 1)); }

ElemArgs elem_args(const ipdg_mesh_s* m, int N, Kind kind, double lambda, double ctau);

}  // namespace ipdg
