// Preconditioned CG that allocates no device memory (ipdg_pcg_solve_noalloc).
//
// The same iteration as ipdg_pcg_solve with the Jacobi, identity or block
// inverse-mass preconditioner (Sec. 3), in FP64, launched directly on the
// caller's stream (no internal stream, no graph).  Its work vectors, block
// partial sums and device scalars live in one file-scope device array of
// fixed size instead of buffers the library allocates: every call on a GPU
// shares that GPU's copy, so calls that overlap on one GPU race.
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>

#include "blas.hpp"
#include "handle.hpp"
#include "noalloc.hpp"

namespace ipdg {
namespace {

// Layout of the scratch array for n = K Np <= kNoAllocMaxDofs:
//   5 FP64 vectors of kNoAllocMaxDofs values (r, p, A p, z, A x), the
//   inverse diagonal (kNoAllocMaxDofs values), 3 x kMaxPartials partial
//   sums, and the CG scalars.
constexpr size_t kVec = kNoAllocMaxDofs * sizeof(double);
constexpr size_t kPartialsOff = 6 * kVec;
constexpr size_t kScalOff = kPartialsOff + 3 * (size_t)kMaxPartials * sizeof(double);
constexpr size_t kScratchBytes = kScalOff + 256;
static_assert(sizeof(CGScal) <= 256, "CG scalars exceed their scratch slot");

}  // namespace

// Every GPU that runs this library holds one copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

// Device address of this device's scratch array, looked up once per device
// (the array's name in host code is a host-side stand-in, not a device
// address).
unsigned char* scratch_on_current_device() {
  int dev = 0;
  IPDG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(IPDG_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    IPDG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(IPDG_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch[dev]);
}

struct Bufs {
  double *r, *p, *Ap, *z, *t, *dinv, *partials;
  CGScal* sc;
};

Bufs carve(unsigned char* base) {
  Bufs b;
  b.r = reinterpret_cast<double*>(base + 0 * kVec);
  b.p = reinterpret_cast<double*>(base + 1 * kVec);
  b.Ap = reinterpret_cast<double*>(base + 2 * kVec);
  b.z = reinterpret_cast<double*>(base + 3 * kVec);
  b.t = reinterpret_cast<double*>(base + 4 * kVec);
  b.dinv = reinterpret_cast<double*>(base + 5 * kVec);
  b.partials = reinterpret_cast<double*>(base + kPartialsOff);
  b.sc = reinterpret_cast<CGScal*>(base + kScalOff);
  return b;
}

CGScal read_scal(const CGScal* sc, hipStream_t s) {
  CGScal h{};
  IPDG_HIP(hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
  IPDG_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

void noalloc_prepare() { (void)scratch_on_current_device(); }

ipdg_status pcg_solve_noalloc(ipdg_mesh_s* m, double lambda, double tau, const double* b, double* x,
                              double tol, const ipdg_solve_opts& o, ipdg_solve_info* info,
                              hipStream_t s) {
  const int N = m->host.N, K = m->host.K;
  const size_t n = (size_t)K * m->Np;
  if (o.pc != IPDG_PC_NONE && o.pc != IPDG_PC_JACOBI && o.pc != IPDG_PC_BLOCK_MASS)
    throw Error(IPDG_EUNSUPPORTED, "the allocation-free solve takes the identity, Jacobi or block "
                                   "inverse-mass preconditioner");
  if (o.prec != IPDG_PREC_FP64) throw Error(IPDG_EUNSUPPORTED, "the allocation-free solve runs in FP64 only");
  if (o.max_iters < 0) throw Error(IPDG_EINVAL, "max_iters < 0");
  if (o.reliable_drop > 0.0)
    throw Error(IPDG_EUNSUPPORTED, "the allocation-free solve replaces the residual only when the "
                                   "recurrence stops (reliable_drop must be 0)");
  if (n > kNoAllocMaxDofs)
    throw Error(IPDG_EINVAL, "K*Np = " + std::to_string(n) + " exceeds the allocation-free solve's limit of " +
                                 std::to_string(kNoAllocMaxDofs) + " values");
  if (!(tol > 0.0)) throw Error(IPDG_EINVAL, "tol must be positive");
  if (info) *info = ipdg_solve_info{};
  if (K == 0) return IPDG_OK;
  if (!b || !x) throw Error(IPDG_EINVAL, "null vector");
  const double ctau = ctau_of(N, tau);
  const void* ops = device_ops_resident(N, Kind::F64);
  if (!ops) throw Error(IPDG_EUNSUPPORTED, "the degree's operator tables are not resident on this device");
  const Bufs B = carve(scratch_on_current_device());
  const auto t0 = std::chrono::steady_clock::now();

  ElemArgs a;
  a.geo = geo_for(m, Kind::F64);
  a.conn = m->conn.as<Conn>();
  a.kap = kap_for(m, Kind::F64);
  a.ops = ops;
  a.lambda = lambda;
  a.ctau = ctau;
  a.K = K;
  const bool flexible = o.flexible > 0;
  const bool jac = o.pc != IPDG_PC_BLOCK_MASS;
  const int nf = flat_grid(n);

  // preconditioner set-up: the inverse diagonal (or ones)
  if (o.pc == IPDG_PC_JACOBI) {
    ElemArgs d = a;
    d.y = B.dinv;
    IPDG_HIP(diag(N, Kind::F64, d, s));
    IPDG_HIP(recip(B.dinv, nullptr, n, s));
  } else if (o.pc == IPDG_PC_NONE) {
    IPDG_HIP(fill(B.dinv, 1.0, n, s));
  }
  CGScal init{};
  init.tol = tol;
  init.max_iters = o.max_iters;
  init.flexible = flexible;
  IPDG_HIP(set_scal(B.sc, init, s));

  auto true_residual = [&]() {
    ElemArgs t = a;
    t.x = x;
    t.y = B.t;
    IPDG_HIP(ax(N, Kind::F64, t, s));
    IPDG_HIP(residual(b, B.t, B.r, n, B.partials, s));
    IPDG_HIP(finalize(B.partials, nf, 2, B.sc, kFinResidual, s));
  };
  auto restart = [&]() {   // z = B r, (r, z), p = z
    if (jac) {
      IPDG_HIP(jacobi(false, B.r, B.dinv, B.z, n, s));
    } else {
      ElemArgs mi = a;
      mi.x = B.r;
      mi.y = B.z;
      IPDG_HIP(minv(N, Kind::F64, mi, s));
    }
    IPDG_HIP(dots_rz(false, B.r, B.z, nullptr, B.sc, n, B.partials, s));
    IPDG_HIP(finalize(B.partials, nf, 3, B.sc, kFinInit, s));
    IPDG_HIP(hipMemcpyAsync(B.p, B.z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  };
  auto iteration = [&]() {
    ElemArgs t = a;
    t.x = B.p;
    t.y = B.Ap;
    t.partials = B.partials;
    t.skip = &B.sc->done;
    IPDG_HIP(ax(N, Kind::F64, t, s));
    IPDG_HIP(finalize(B.partials, ax_partials(N, false, K), 1, B.sc, kFinAlpha, s));
    IPDG_HIP(cg_update(false, jac, x, B.r, B.p, B.Ap, B.dinv, B.z, B.sc, n, B.partials, s));
    if (!jac) {
      ElemArgs mi = a;
      mi.x = B.r;
      mi.y = B.z;
      mi.skip = &B.sc->done;
      IPDG_HIP(minv(N, Kind::F64, mi, s));
      IPDG_HIP(dots_rz(false, B.r, B.z, B.Ap, B.sc, n, B.partials, s));
    }
    IPDG_HIP(finalize(B.partials, nf, 3, B.sc, kFinBeta, s));
    IPDG_HIP(pupdate(false, B.p, B.z, B.sc, n, s));
  };

  true_residual();
  CGScal h = read_scal(B.sc, s);
  const double bb = h.bb;
  int restarts = 0, iters = 0;
  double relres = 0.0;
  ipdg_status st = IPDG_OK;
  if (bb == 0.0) {
    IPDG_HIP(fill(x, 0.0, n, s));
    IPDG_HIP(hipStreamSynchronize(s));
  } else {
    relres = std::sqrt(h.rr / bb);
    restart();
    const int every = o.check_every > 0 ? o.check_every : 1;
    for (;;) {
      for (int k = 0; k < every; ++k) iteration();
      h = read_scal(B.sc, s);
      iters = h.iters;
      if (h.breakdown) {
        st = IPDG_EBREAKDOWN;
        relres = NAN;
        break;
      }
      if (!h.done) continue;
      // the recurrence stopped: accept only on the true FP64 residual
      true_residual();
      const CGScal t = read_scal(B.sc, s);
      relres = std::sqrt(t.rr / bb);
      if (!(t.rr == t.rr)) { st = IPDG_EBREAKDOWN; break; }
      if (t.rr <= tol * tol * bb) { st = IPDG_OK; break; }
      if (iters >= o.max_iters) { st = IPDG_NOT_CONVERGED; break; }
      ++restarts;
      // residual replacement: continue from the true residual (the scalar
      // record keeps its iteration count)
      restart();
    }
  }
  if (info) {
    info->iters = iters;
    info->relres = relres;
    info->restarts = restarts;
    info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (st == IPDG_EBREAKDOWN) throw Error(IPDG_EBREAKDOWN, "CG breakdown (p^T A p <= 0 or not finite)");
  return st;
}

}  // namespace ipdg
