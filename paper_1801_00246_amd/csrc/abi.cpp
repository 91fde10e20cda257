// C ABI entry points (include/ipdg.h).  Every call catches library errors and
// maps them to an ipdg_status; the message is kept per thread.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "gradiv.hpp"
#include "handle.hpp"
#include "ins.hpp"
#include "noalloc.hpp"
#include "probe.hpp"
#include "refelem.hpp"
#include "solver.hpp"
#include "subcycle.hpp"

namespace {

thread_local std::string g_last_error;

ipdg_status fail(ipdg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

template <typename F>
ipdg_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const ipdg::Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(IPDG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(IPDG_EINVAL, e.what());
  }
}

ipdg::Kind kind_of(ipdg_dtype d) { return d == IPDG_F32 ? ipdg::Kind::F32 : ipdg::Kind::F64; }

// Makes the mesh's device current for the duration of a call (device
// buffers, operator tables and streams of a mesh live on the device that was
// current when it was created) and restores the caller's device.
class DeviceGuard {
 public:
  explicit DeviceGuard(const ipdg_mesh_s* m) {
    IPDG_HIP(hipGetDevice(&prev_));
    if (prev_ != m->device) IPDG_HIP(hipSetDevice(m->device));
    else prev_ = -1;
  }
  ~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;

 private:
  int prev_ = -1;
};

void upload_kappa(ipdg_mesh_s* m, const double* kappa) {
  const int K = m->host.K;
  if (!kappa) {
    if (m->has_kappa) ++m->kappa_version;
    m->has_kappa = false;
    m->kappa.clear();
    return;
  }
  for (int e = 0; e < K; ++e)
    if (!(kappa[e] > 0.0)) throw ipdg::Error(IPDG_EINVAL, "kappa must be positive");
  // the same values again: nothing to upload, solver set-ups stay valid
  if (m->has_kappa && (int)m->kappa.size() == K && std::equal(kappa, kappa + K, m->kappa.begin())) return;
  ++m->kappa_version;
  m->kappa.assign(kappa, kappa + K);
  std::vector<float> k32(kappa, kappa + K);
  m->kap64.ensure(K * sizeof(double));
  m->kap32.ensure(K * sizeof(float));
  if (K) {
    IPDG_HIP(hipMemcpy(m->kap64.get(), kappa, K * sizeof(double), hipMemcpyHostToDevice));
    IPDG_HIP(hipMemcpy(m->kap32.get(), k32.data(), K * sizeof(float), hipMemcpyHostToDevice));
  }
  m->has_kappa = true;
}

}  // namespace

extern "C" {

void ipdg_default_opts(ipdg_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->pc = IPDG_PC_JACOBI;
  o->prec = IPDG_PREC_FP64;
  o->max_iters = 10000;
  o->check_every = 10;
  o->flexible = -1;
  o->n_levels = 0;
  o->cheb_degree = 2;
  o->cheb_lo = 0.1;
  o->cheb_hi = 1.1;
  o->rho_steps = 20;
  o->coarse_tol = 1e-2;
  o->coarse_max_iters = -1;
  o->reliable_drop = 0.0;
  o->coarse_persistent = 0;
  o->coarse_amg = 0;
  o->amg_coarse_size = 512;
  o->amg_cycles = 1;
  o->amg_kcycle_levels = 2;
  o->amg_top_krylov = 0;
}

const char* ipdg_last_error(void) { return g_last_error.c_str(); }

ipdg_status ipdg_mesh_create(int N, int Nv, const double* VX, const double* VY, int K,
                             const int32_t* EToV, const int8_t* EToB, const double* kappa,
                             ipdg_mesh* out) {
  return guarded([&]() -> ipdg_status {
    if (!out) return fail(IPDG_EINVAL, "out is null");
    *out = nullptr;
    if (N < 1 || N > ipdg::kMaxN) return fail(IPDG_EUNSUPPORTED, "degree outside 1..8");
    auto m = std::make_unique<ipdg_mesh_s>();
    std::string err = ipdg::build_host_mesh(N, Nv, VX, VY, K, EToV, EToB, m->host);
    if (!err.empty()) return fail(IPDG_EMESH, err);
    IPDG_HIP(hipGetDevice(&m->device));
    m->Np = ipdg::np_of(N);
    (void)ipdg::ref_ops(N);
    std::vector<float> g32(m->host.geo.begin(), m->host.geo.end());
    if (K > 0) {
      m->geo64.alloc(m->host.geo.size() * sizeof(double));
      m->geo32.alloc(g32.size() * sizeof(float));
      m->conn.alloc(K * sizeof(ipdg::Conn));
      IPDG_HIP(hipMemcpy(m->geo64.get(), m->host.geo.data(), m->host.geo.size() * sizeof(double),
                         hipMemcpyHostToDevice));
      IPDG_HIP(hipMemcpy(m->geo32.get(), g32.data(), g32.size() * sizeof(float), hipMemcpyHostToDevice));
      IPDG_HIP(hipMemcpy(m->conn.get(), m->host.conn.data(), K * sizeof(ipdg::Conn),
                         hipMemcpyHostToDevice));
    }
    upload_kappa(m.get(), kappa);
    // the degree's operator tables are resident from here on (calls that
    // must not allocate rely on that)
    (void)ipdg::device_ops(N, ipdg::Kind::F64);
    (void)ipdg::device_ops(N, ipdg::Kind::F32);
    ipdg::noalloc_prepare();
    *out = m.release();
    return IPDG_OK;
  });
}

ipdg_status ipdg_mesh_destroy(ipdg_mesh mesh) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return IPDG_OK;
    DeviceGuard dg(mesh);
    delete mesh;
    return IPDG_OK;
  });
}

ipdg_status ipdg_mesh_info(ipdg_mesh mesh, int* N, int* Np, int* K) {
  if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
  if (N) *N = mesh->host.N;
  if (Np) *Np = mesh->Np;
  if (K) *K = mesh->host.K;
  return IPDG_OK;
}

ipdg_status ipdg_node_coords(ipdg_mesh mesh, double* x, double* y) {
  return guarded([&]() -> ipdg_status {
    if (!mesh || !x || !y) return fail(IPDG_EINVAL, "null argument");
    std::vector<double> vx, vy;
    ipdg::host_node_coords(mesh->host, vx, vy);
    std::memcpy(x, vx.data(), vx.size() * sizeof(double));
    std::memcpy(y, vy.data(), vy.size() * sizeof(double));
    return IPDG_OK;
  });
}

ipdg_status ipdg_set_kappa(ipdg_mesh mesh, const double* kappa) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    DeviceGuard dg(mesh);
    upload_kappa(mesh, kappa);
    return IPDG_OK;
  });
}

ipdg_status ipdg_apply(ipdg_mesh mesh, double lambda, double tau, ipdg_dtype dtype, const void* x,
                       void* y, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!x || !y) return fail(IPDG_EINVAL, "null vector");
    if (x == y) return fail(IPDG_EINVAL, "x and y must not overlap");
    DeviceGuard dg(mesh);
    const int N = mesh->host.N;
    const ipdg::Kind k = kind_of(dtype);
    ipdg::ElemArgs a = ipdg::elem_args(mesh, N, k, lambda, ipdg::ctau_of(N, tau));
    a.x = x;
    a.y = y;
    IPDG_HIP(ipdg::ax(N, k, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_ax_variant_get(int N, ipdg_dtype dtype, int* variant) {
  return guarded([&]() -> ipdg_status {
    if (N < 1 || N > 8) return fail(IPDG_EINVAL, "degree must be 1..8");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    if (!variant) return fail(IPDG_EINVAL, "variant is null");
    *variant = ipdg::ax_variant(N, dtype == IPDG_F32);
    return IPDG_OK;
  });
}

ipdg_status ipdg_ax_variant_set(int N, ipdg_dtype dtype, int variant) {
  return guarded([&]() -> ipdg_status {
    if (N < 1 || N > 8) return fail(IPDG_EINVAL, "degree must be 1..8");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    if (!ipdg::ax_variant_exists(N, variant))
      return fail(IPDG_EINVAL, "degree " + std::to_string(N) + " has no operator variant " +
                                   std::to_string(variant));
    ipdg::set_ax_variant(N, dtype == IPDG_F32, variant);
    return IPDG_OK;
  });
}

ipdg_status ipdg_autotune_apply(ipdg_mesh mesh, double lambda, double tau, ipdg_dtype dtype, int reps,
                                int* chosen, double* times_ms, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    if (!chosen) return fail(IPDG_EINVAL, "chosen is null");
    const int N = mesh->host.N;
    const bool fp32 = dtype == IPDG_F32;
    const int prev = ipdg::ax_variant(N, fp32);
    constexpr int nvar = 5;
    if (times_ms)
      for (int v = 0; v < nvar; ++v) times_ms[v] = -1.0;
    *chosen = prev;
    if (mesh->host.K == 0) return IPDG_OK;
    if (reps <= 0) reps = 20;
    DeviceGuard dg(mesh);
    const ipdg::Kind k = kind_of(dtype);
    const size_t n = (size_t)mesh->host.K * mesh->Np;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ipdg::DevBuf x(n * (fp32 ? 4 : 8)), y(n * (fp32 ? 4 : 8));
    // operand: every value about 1 (any finite data times the same)
    IPDG_HIP(hipMemsetD32Async(x.get(), fp32 ? 0x3F800000 : 0x3FF00000, n * (fp32 ? 1 : 2), s));
    ipdg::ElemArgs a = ipdg::elem_args(mesh, N, k, lambda, ipdg::ctau_of(N, tau));
    a.x = x.get();
    a.y = y.get();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    IPDG_HIP(hipEventCreate(&e0));
    IPDG_HIP(hipEventCreate(&e1));
    int best = prev;
    double best_ms = 0.0;
    try {
      bool first = true;
      for (int v = 0; v < nvar; ++v) {
        if (!ipdg::ax_variant_exists(N, v)) continue;
        ipdg::set_ax_variant(N, fp32, v);
        IPDG_HIP(ipdg::ax(N, k, a, s));
        IPDG_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) IPDG_HIP(ipdg::ax(N, k, a, s));
        IPDG_HIP(hipEventRecord(e1, s));
        IPDG_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        IPDG_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double t = double(ms) / reps;
        if (times_ms) times_ms[v] = t;
        if (first || t < best_ms) best = v, best_ms = t;
        first = false;
      }
    } catch (...) {
      ipdg::set_ax_variant(N, fp32, prev);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ipdg::set_ax_variant(N, fp32, best);
    *chosen = best;
    return IPDG_OK;
  });
}

ipdg_status ipdg_probe_copy(size_t bytes, int sets, int reps, double* gbs, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!gbs) return fail(IPDG_EINVAL, "gbs is null");
    *gbs = ipdg::probe_copy_gbs(bytes, sets, reps, static_cast<hipStream_t>(hip_stream));
    return IPDG_OK;
  });
}

ipdg_status ipdg_probe_fma(ipdg_dtype dtype, int reps, double* tflops, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!tflops) return fail(IPDG_EINVAL, "tflops is null");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    *tflops = ipdg::probe_fma_tflops(dtype == IPDG_F32, reps, static_cast<hipStream_t>(hip_stream));
    return IPDG_OK;
  });
}

ipdg_status ipdg_mass_apply(ipdg_mesh mesh, ipdg_dtype dtype, const void* x, void* y,
                            void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (dtype != IPDG_F64 && dtype != IPDG_F32) return fail(IPDG_EINVAL, "bad dtype");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!x || !y) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    const int N = mesh->host.N;
    const ipdg::Kind k = kind_of(dtype);
    ipdg::ElemArgs a = ipdg::elem_args(mesh, N, k, 0.0, 0.0);
    a.x = x;
    a.y = y;
    IPDG_HIP(ipdg::mass(N, k, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_pcg_solve(ipdg_mesh mesh, double lambda, double tau, const double* b, double* x,
                           double tol, const ipdg_solve_opts* opts, ipdg_solve_info* info,
                           void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    DeviceGuard dg(mesh);
    ipdg_solve_opts o;
    if (opts) o = *opts;
    else ipdg_default_opts(&o);
    return ipdg::pcg_solve(mesh, lambda, tau, b, x, tol, o, info,
                           static_cast<hipStream_t>(hip_stream));
  });
}

ipdg_status ipdg_pcg_solve_noalloc(ipdg_mesh mesh, double lambda, double tau, const double* b,
                                   double* x, double tol, const ipdg_solve_opts* opts,
                                   ipdg_solve_info* info, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    DeviceGuard dg(mesh);
    ipdg_solve_opts o;
    if (opts) o = *opts;
    else ipdg_default_opts(&o);
    return ipdg::pcg_solve_noalloc(mesh, lambda, tau, b, x, tol, o, info,
                                   static_cast<hipStream_t>(hip_stream));
  });
}

ipdg_status ipdg_precond_apply(ipdg_mesh mesh, double lambda, double tau,
                               const ipdg_solve_opts* opts, const double* r, double* z,
                               ipdg_solve_info* info, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    DeviceGuard dg(mesh);
    ipdg_solve_opts o;
    if (opts) o = *opts;
    else ipdg_default_opts(&o);
    return ipdg::precond_apply(mesh, lambda, tau, o, r, z, info,
                               static_cast<hipStream_t>(hip_stream));
  });
}

ipdg_status ipdg_helmholtz_solve_batch(int nb, const ipdg_mesh* meshes, const double* lambdas,
                                       double tau, const double* const* b, double* const* x,
                                       double tol, const ipdg_solve_opts* opts, int* iters,
                                       double* relres, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (nb < 0) return fail(IPDG_EINVAL, "nb < 0");
    if (nb == 0) return IPDG_OK;
    if (!meshes || !lambdas || !b || !x) return fail(IPDG_EINVAL, "null argument");
    for (int i = 0; i < nb; ++i) {
      if (!meshes[i]) return fail(IPDG_EINVAL, "null mesh in batch");
      if (meshes[i]->device != meshes[0]->device)
        return fail(IPDG_EINVAL, "all meshes of a batch must live on one device");
    }
    DeviceGuard dg(meshes[0]);
    ipdg_solve_opts o;
    if (opts) o = *opts;
    else {
      ipdg_default_opts(&o);
      o.pc = IPDG_PC_BLOCK_MASS;
    }
    return ipdg::solve_batch(nb, meshes, lambdas, tau, b, x, tol, o, iters, relres,
                             static_cast<hipStream_t>(hip_stream));
  });
}

namespace {

ipdg::GradArgs grad_args(ipdg_mesh mesh) {
  ipdg::GradArgs a;
  a.geo = mesh->geo64.as<double>();
  a.conn = mesh->conn.as<ipdg::Conn>();
  a.ops = static_cast<const double*>(ipdg::device_ops(mesh->host.N, ipdg::Kind::F64));
  a.K = mesh->host.K;
  return a;
}

ipdg::DivArgs div_args(ipdg_mesh mesh) {
  ipdg::DivArgs a;
  a.geo = mesh->geo64.as<double>();
  a.conn = mesh->conn.as<ipdg::Conn>();
  a.ops = static_cast<const double*>(ipdg::device_ops(mesh->host.N, ipdg::Kind::F64));
  a.K = mesh->host.K;
  return a;
}

}  // namespace

ipdg_status ipdg_grad(ipdg_mesh mesh, const double* p, double* gx, double* gy, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!p || !gx || !gy) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::GradArgs a = grad_args(mesh);
    a.p = p;
    a.out_x = gx;
    a.out_y = gy;
    IPDG_HIP(ipdg::grad_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_div(ipdg_mesh mesh, const double* u, const double* v, const double* gu,
                     const double* gv, double* out, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u || !v || !out) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::DivArgs a = div_args(mesh);
    a.u = u;
    a.v = v;
    a.gu = gu;
    a.gv = gv;
    a.out = out;
    IPDG_HIP(ipdg::div_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_advect(ipdg_mesh mesh, const double* u, const double* v, const double* gu, const double* gv,
                        double* nu, double* nv, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u || !v || !nu || !nv) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::AdvectArgs a;
    a.u = u;
    a.v = v;
    a.gu = gu;
    a.gv = gv;
    a.out_u = nu;
    a.out_v = nv;
    a.geo = mesh->geo64.as<double>();
    a.conn = mesh->conn.as<ipdg::Conn>();
    a.ops = static_cast<const double*>(ipdg::device_ops(mesh->host.N, ipdg::Kind::F64));
    a.K = mesh->host.K;
    IPDG_HIP(ipdg::advect_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_dirichlet_rhs(ipdg_mesh mesh, double tau, const double* g, double* b, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!g || !b) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::DirichletArgs a;
    a.g = g;
    a.b = b;
    a.kap = mesh->has_kappa ? mesh->kap64.as<double>() : nullptr;
    a.ctau = ipdg::ctau_of(mesh->host.N, tau);
    a.geo = mesh->geo64.as<double>();
    a.conn = mesh->conn.as<ipdg::Conn>();
    a.ops = static_cast<const double*>(ipdg::device_ops(mesh->host.N, ipdg::Kind::F64));
    a.K = mesh->host.K;
    IPDG_HIP(ipdg::dirichlet_rhs(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_ins_velocity_rhs(ipdg_mesh mesh, double nu, double dt, const double* uhat,
                                  const double* vhat, const double* sigma_p, double* bu, double* bv,
                                  void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (!(nu > 0.0) || !(dt > 0.0)) return fail(IPDG_EINVAL, "nu and dt must be positive");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!uhat || !vhat || !sigma_p || !bu || !bv) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::GradArgs a = grad_args(mesh);
    a.p = sigma_p;
    a.base_x = uhat;
    a.base_y = vhat;
    a.a_base = 1.0 / (nu * dt);
    a.a_grad = -1.0 / nu;
    a.mass = true;
    a.out_x = bu;
    a.out_y = bv;
    IPDG_HIP(ipdg::grad_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_ins_pressure_rhs(ipdg_mesh mesh, double gamma, double dt, const double* u,
                                  const double* v, const double* gu, const double* gv, double* b,
                                  void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (!(gamma > 0.0) || !(dt > 0.0)) return fail(IPDG_EINVAL, "gamma and dt must be positive");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u || !v || !b) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::DivArgs a = div_args(mesh);
    a.u = u;
    a.v = v;
    a.gu = gu;
    a.gv = gv;
    a.out = b;
    a.scale = -gamma / dt;
    a.mass = true;
    IPDG_HIP(ipdg::div_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

ipdg_status ipdg_ins_correct(ipdg_mesh mesh, double gamma, double dt, const double* u, const double* v,
                             const double* dp, const double* sigma_p, double* u_out, double* v_out,
                             double* p_out, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (!(gamma > 0.0) || !(dt > 0.0)) return fail(IPDG_EINVAL, "gamma and dt must be positive");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u || !v || !dp || !sigma_p || !u_out || !v_out || !p_out) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::GradArgs a = grad_args(mesh);
    a.p = dp;
    a.base_x = u;
    a.base_y = v;
    a.a_base = 1.0;
    a.a_grad = -dt / gamma;
    a.out_x = u_out;
    a.out_y = v_out;
    a.add_p = sigma_p;
    a.p_out = p_out;
    IPDG_HIP(ipdg::grad_apply(mesh->host.N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

namespace {

ipdg_status ins_step_entry(ipdg_mesh mesh, ipdg_mesh pmesh, double nu, double dt, double tau, int subcycles,
                           const double* u_n, const double* v_n, const double* p_n, const double* p_nm1,
                           const double* gu_n, const double* gv_n, const double* gu_1, const double* gv_1,
                           double* u_1, double* v_1, double* p_1, double tol, const ipdg_solve_opts* vel_opts,
                           const ipdg_solve_opts* pres_opts, int* iters, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh || !pmesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->device != pmesh->device) return fail(IPDG_EINVAL, "the two meshes live on different devices");
    if (subcycles < 0) return fail(IPDG_EINVAL, "subcycles must not be negative");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u_n || !v_n || !p_n || !p_nm1 || !u_1 || !v_1 || !p_1) return fail(IPDG_EINVAL, "null vector");
    if (!(tol > 0.0)) return fail(IPDG_EINVAL, "tol must be positive");
    DeviceGuard dg(mesh);
    ipdg_solve_opts vo, po;
    if (vel_opts) vo = *vel_opts;
    else ipdg_default_opts(&vo);
    if (pres_opts) po = *pres_opts;
    else ipdg_default_opts(&po);
    ipdg::InsState in;
    in.u = u_n;
    in.v = v_n;
    in.p = p_n;
    in.p_prev = p_nm1;
    in.gu = gu_n;
    in.gv = gv_n;
    in.subcycles = subcycles;
    ipdg::InsOut out;
    out.u = u_1;
    out.v = v_1;
    out.p = p_1;
    out.gu = gu_1;
    out.gv = gv_1;
    return ipdg::ins_step(mesh, pmesh, nu, dt, tau, in, out, tol, vo, po, iters,
                          static_cast<hipStream_t>(hip_stream));
  });
}

}  // namespace

ipdg_status ipdg_ins_step(ipdg_mesh mesh, ipdg_mesh pmesh, double nu, double dt, double tau,
                          const double* u_n, const double* v_n, const double* p_n, const double* p_nm1,
                          const double* gu_n, const double* gv_n, const double* gu_1, const double* gv_1,
                          double* u_1, double* v_1, double* p_1, double tol, const ipdg_solve_opts* vel_opts,
                          const ipdg_solve_opts* pres_opts, int* iters, void* hip_stream) {
  return ins_step_entry(mesh, pmesh, nu, dt, tau, 0, u_n, v_n, p_n, p_nm1, gu_n, gv_n, gu_1, gv_1, u_1, v_1, p_1,
                        tol, vel_opts, pres_opts, iters, hip_stream);
}

ipdg_status ipdg_ins_step_subcycled(ipdg_mesh mesh, ipdg_mesh pmesh, double nu, double dt, double tau,
                                    int subcycles, const double* u_n, const double* v_n, const double* p_n,
                                    const double* p_nm1, const double* gu_n, const double* gv_n,
                                    const double* gu_1, const double* gv_1, double* u_1, double* v_1,
                                    double* p_1, double tol, const ipdg_solve_opts* vel_opts,
                                    const ipdg_solve_opts* pres_opts, int* iters, void* hip_stream) {
  if (subcycles < 1) return fail(IPDG_EINVAL, "subcycles must be at least 1");
  return ins_step_entry(mesh, pmesh, nu, dt, tau, subcycles, u_n, v_n, p_n, p_nm1, gu_n, gv_n, gu_1, gv_1, u_1,
                        v_1, p_1, tol, vel_opts, pres_opts, iters, hip_stream);
}

ipdg_status ipdg_subcycle_rhs(ipdg_mesh mesh, const double* ubar, const double* vbar, const double* u,
                              const double* v, const double* gu, const double* gv, int parts, double* nu,
                              double* nv, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (parts < 1 || parts > 3) return fail(IPDG_EINVAL, "parts must be 1, 2 or 3");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!ubar || !vbar || !u || !v || !nu || !nv) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    ipdg::SubArgs a;
    a.ub0 = ubar;
    a.vb0 = vbar;
    a.u = u;
    a.v = v;
    a.gu0 = gu;
    a.gv0 = gv;
    ipdg::subcycle_rhs(mesh, a, parts, nu, nv, static_cast<hipStream_t>(hip_stream));
    return IPDG_OK;
  });
}

ipdg_status ipdg_subcycle(ipdg_mesh mesh, const double* ubar0, const double* vbar0, const double* ubar1,
                          const double* vbar1, const double* gu0, const double* gv0, const double* gu1,
                          const double* gv1, double T, int Ns, double* u, double* v, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (Ns < 1) return fail(IPDG_EINVAL, "Ns must be at least 1");
    if (!std::isfinite(T)) return fail(IPDG_EINVAL, "T must be finite");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!ubar0 || !vbar0 || !u || !v) return fail(IPDG_EINVAL, "null vector");
    if ((ubar1 == nullptr) != (vbar1 == nullptr)) return fail(IPDG_EINVAL, "give both ubar1 and vbar1 or neither");
    if ((gu1 || gv1) && (!gu0 || !gv0)) return fail(IPDG_EINVAL, "data rates need the data gu0, gv0");
    DeviceGuard dg(mesh);
    ipdg::SubArgs a;
    a.ub0 = ubar0;
    a.vb0 = vbar0;
    a.ub1 = ubar1;
    a.vb1 = vbar1;
    a.gu0 = gu0;
    a.gv0 = gv0;
    a.gu1 = gu1;
    a.gv1 = gv1;
    ipdg::subcycle_advect(mesh, a, T, Ns, u, v, static_cast<hipStream_t>(hip_stream));
    return IPDG_OK;
  });
}

ipdg_status ipdg_kappa_grad(ipdg_mesh mesh, double tau, const double* u, const double* w,
                            double* dLdkappa, void* hip_stream) {
  return guarded([&]() -> ipdg_status {
    if (!mesh) return fail(IPDG_EINVAL, "mesh is null");
    if (mesh->host.K == 0) return IPDG_OK;
    if (!u || !w || !dLdkappa) return fail(IPDG_EINVAL, "null vector");
    DeviceGuard dg(mesh);
    const int N = mesh->host.N;
    const double* kap = mesh->kap64.as<double>();
    if (!mesh->has_kappa) {
      // kappa = 1: a device array of ones kept with the mesh (the mesh's
      // operator stays the coefficient-free one)
      if (!mesh->ones64.get()) {
        std::vector<double> ones(mesh->host.K, 1.0);
        mesh->ones64.ensure(mesh->host.K * sizeof(double));
        IPDG_HIP(hipMemcpy(mesh->ones64.get(), ones.data(), mesh->host.K * sizeof(double),
                           hipMemcpyHostToDevice));
      }
      kap = mesh->ones64.as<double>();
    }
    ipdg::KgradArgs a{u, w, dLdkappa, mesh->geo64.as<double>(), mesh->conn.as<ipdg::Conn>(), kap,
                      static_cast<const double*>(ipdg::device_ops(N, ipdg::Kind::F64)),
                      ipdg::ctau_of(N, tau), mesh->host.K};
    IPDG_HIP(ipdg::kgrad(N, a, static_cast<hipStream_t>(hip_stream)));
    return IPDG_OK;
  });
}

/* Host-only check of a mesh (no device use): connectivity and validation as
 * in ipdg_mesh_create.  EToE / EToF are HOST arrays of K*3 (may be NULL). */
ipdg_status ipdg_mesh_check(int N, int Nv, const double* VX, const double* VY, int K,
                            const int32_t* EToV, const int8_t* EToB, int32_t* EToE, int8_t* EToF) {
  return guarded([&]() -> ipdg_status {
    ipdg::HostMesh h;
    std::string err = ipdg::build_host_mesh(N, Nv, VX, VY, K, EToV, EToB, h);
    if (!err.empty()) return fail(N < 1 || N > ipdg::kMaxN ? IPDG_EUNSUPPORTED : IPDG_EMESH, err);
    if (EToE) std::memcpy(EToE, h.EToE.data(), h.EToE.size() * sizeof(int32_t));
    if (EToF) std::memcpy(EToF, h.EToF.data(), h.EToF.size() * sizeof(int8_t));
    return IPDG_OK;
  });
}

/* Host-only: reference nodes (r, s; Np each) and operators D_r, D_s, M
 * (Np x Np, row-major) and LIFT (Np x 3 Nfp) of degree N.  Any pointer may
 * be NULL. */
ipdg_status ipdg_reference_element(int N, double* r, double* s, double* Dr, double* Ds,
                                   double* M, double* LIFT) {
  return guarded([&]() -> ipdg_status {
    if (N < 1 || N > ipdg::kMaxN) return fail(IPDG_EUNSUPPORTED, "degree outside 1..8");
    const ipdg::RefOps& R = ipdg::ref_ops(N);
    auto cp = [](double* dst, const std::vector<double>& v) {
      if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
    };
    cp(r, R.r);
    cp(s, R.s);
    cp(Dr, R.Dr);
    cp(Ds, R.Ds);
    cp(M, R.M);
    cp(LIFT, R.LIFT);
    return IPDG_OK;
  });
}

}  // extern "C"
