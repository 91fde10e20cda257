"""Python binding of libipdg.so (the C ABI in include/ipdg.h).

Argument marshalling only: every operation runs in the library's HIP kernels.
PyTorch supplies device memory and the current HIP stream.  The binding
raises if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipdg.so")

IPDG_OK, IPDG_NOT_CONVERGED = 0, 1
STATUS = {0: "IPDG_OK", 1: "IPDG_NOT_CONVERGED", -1: "IPDG_EINVAL", -2: "IPDG_EMESH",
          -3: "IPDG_EHIP", -4: "IPDG_ENOMEM", -5: "IPDG_EUNSUPPORTED", -6: "IPDG_EBREAKDOWN"}
F64, F32 = 0, 1
BC_INTERIOR, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2
PC_NONE, PC_JACOBI, PC_BLOCK_MASS, PC_PMG = 0, 1, 2, 3
PREC_FP64, PREC_MIXED, PREC_FP32_OPERATOR = 0, 1, 2
MAX_LEVELS = 8
AMG_MAX_LEVELS = 12


class IpdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveOpts(C.Structure):
    _fields_ = [("pc", C.c_int), ("prec", C.c_int), ("max_iters", C.c_int),
                ("check_every", C.c_int), ("flexible", C.c_int), ("n_levels", C.c_int),
                ("degrees", C.c_int * MAX_LEVELS), ("cheb_degree", C.c_int),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("rho", C.c_double * MAX_LEVELS), ("rho_steps", C.c_int),
                ("coarse_tol", C.c_double), ("coarse_max_iters", C.c_int),
                ("reliable_drop", C.c_double), ("coarse_persistent", C.c_int),
                ("coarse_amg", C.c_int), ("amg_coarse_size", C.c_int), ("amg_cycles", C.c_int),
                ("amg_kcycle_levels", C.c_int), ("amg_top_krylov", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("relres", C.c_double), ("restarts", C.c_int),
                ("rho_used", C.c_double * MAX_LEVELS), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("coarse_iters", C.c_int),
                ("amg_levels", C.c_int), ("amg_n", C.c_int * AMG_MAX_LEVELS),
                ("precond_bytes", C.c_int64)]

    def as_dict(self):
        return {"iters": self.iters, "relres": self.relres, "restarts": self.restarts,
                "rho_used": list(self.rho_used), "setup_ms": self.setup_ms,
                "solve_ms": self.solve_ms, "coarse_iters": self.coarse_iters,
                "amg_sizes": list(self.amg_n)[:self.amg_levels], "precond_bytes": self.precond_bytes}


_lib = None

_P = C.c_void_p
_SIGS = {
    "ipdg_default_opts": (None, [C.POINTER(SolveOpts)]),
    "ipdg_last_error": (C.c_char_p, []),
    "ipdg_mesh_create": (C.c_int, [C.c_int, C.c_int, _P, _P, C.c_int, _P, _P, _P, C.POINTER(_P)]),
    "ipdg_mesh_destroy": (C.c_int, [_P]),
    "ipdg_mesh_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ipdg_node_coords": (C.c_int, [_P, _P, _P]),
    "ipdg_set_kappa": (C.c_int, [_P, _P]),
    "ipdg_apply": (C.c_int, [_P, C.c_double, C.c_double, C.c_int, _P, _P, _P]),
    "ipdg_mass_apply": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "ipdg_pcg_solve": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, C.c_double,
                                 C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "ipdg_pcg_solve_noalloc": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, C.c_double,
                                         C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "ipdg_precond_apply": (C.c_int, [_P, C.c_double, C.c_double, C.POINTER(SolveOpts), _P, _P,
                                     C.POINTER(SolveInfo), _P]),
    "ipdg_helmholtz_solve_batch": (C.c_int, [C.c_int, _P, _P, C.c_double, _P, _P, C.c_double,
                                             C.POINTER(SolveOpts), _P, _P, _P]),
    "ipdg_kappa_grad": (C.c_int, [_P, C.c_double, _P, _P, _P, _P]),
    "ipdg_grad": (C.c_int, [_P, _P, _P, _P, _P]),
    "ipdg_dirichlet_rhs": (C.c_int, [_P, C.c_double, _P, _P, _P]),
    "ipdg_ins_step": (C.c_int, [_P, _P, C.c_double, C.c_double, C.c_double] + [_P] * 11 + [C.c_double, _P, _P, _P, _P]),
    "ipdg_ins_step_subcycled": (C.c_int, [_P, _P, C.c_double, C.c_double, C.c_double, C.c_int] + [_P] * 11
                                + [C.c_double, _P, _P, _P, _P]),
    "ipdg_div": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "ipdg_advect": (C.c_int, [_P] * 8),
    "ipdg_subcycle_rhs": (C.c_int, [_P] * 7 + [C.c_int, _P, _P, _P]),
    "ipdg_subcycle": (C.c_int, [_P] * 9 + [C.c_double, C.c_int, _P, _P, _P]),
    "ipdg_ins_velocity_rhs": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, _P, _P, _P, _P]),
    "ipdg_ins_pressure_rhs": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, _P, _P, _P, _P]),
    "ipdg_ins_correct": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ipdg_mesh_check": (C.c_int, [C.c_int, C.c_int, _P, _P, C.c_int, _P, _P, _P, _P]),
    "ipdg_reference_element": (C.c_int, [C.c_int, _P, _P, _P, _P, _P, _P]),
    "ipdg_ax_variant_get": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "ipdg_ax_variant_set": (C.c_int, [C.c_int, C.c_int, C.c_int]),
    "ipdg_probe_copy": (C.c_int, [C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_double), _P]),
    "ipdg_probe_fma": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double), _P]),
    "ipdg_autotune_apply": (C.c_int, [_P, C.c_double, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                                      _P, _P]),
}


def lib():
    """Load libipdg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch's device runtime is initialised first: once the library has
        # brought up HIP on its own, torch no longer finds the GPU
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(status: int):
    if status not in (IPDG_OK, IPDG_NOT_CONVERGED):
        raise IpdgError(status, lib().ipdg_last_error().decode())
    return status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().ipdg_default_opts(C.byref(o))
    known = {f[0] for f in SolveOpts._fields_}
    for k in kw:
        if k not in known:
            raise TypeError(f"unknown solve option {k!r} (known: {sorted(known)})")
    for k, v in kw.items():
        if k in ("degrees", "rho"):
            arr = getattr(o, k)
            for i in range(MAX_LEVELS):
                arr[i] = v[i] if i < len(v) else 0
            if k == "degrees":
                o.n_levels = len(v)
        else:
            setattr(o, k, v)
    return o


def ax_variant(N, dtype="f64"):
    """Operator-kernel variant in use at degree N for dtype ("f64"/"f32")."""
    v = C.c_int(-1)
    check(lib().ipdg_ax_variant_get(int(N), F64 if dtype in ("f64", F64) else F32, C.byref(v)))
    return v.value


def set_ax_variant(N, dtype, variant):
    """Select the operator-kernel variant for degree N and dtype, process-wide."""
    check(lib().ipdg_ax_variant_set(int(N), F64 if dtype in ("f64", F64) else F32, int(variant)))


def probe_copy(nbytes, sets=8, reps=50, stream=None):
    """GB/s (read + write) of the library's vectorised copy kernel."""
    v = C.c_double(0.0)
    check(lib().ipdg_probe_copy(int(nbytes), int(sets), int(reps), C.byref(v), _stream(stream)))
    return v.value


def probe_fma(dtype="f64", reps=5, stream=None):
    """TFLOP/s of independent multiply-add chains in dtype ("f64"/"f32")."""
    v = C.c_double(0.0)
    check(lib().ipdg_probe_fma(F64 if dtype in ("f64", F64) else F32, int(reps), C.byref(v), _stream(stream)))
    return v.value


def _np_ptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_P)


def mesh_check(N, VX, VY, EToV, EToB):
    """Host-only validation and face matching; returns (EToE, EToF)."""
    K = int(np.asarray(EToV).shape[0])
    VX, pvx = _np_ptr(VX, np.float64)
    VY, pvy = _np_ptr(VY, np.float64)
    EToV, pv = _np_ptr(EToV, np.int32)
    EToB, pb = _np_ptr(EToB, np.int8)
    EToE = np.empty((K, 3), np.int32)
    EToF = np.empty((K, 3), np.int8)
    check(lib().ipdg_mesh_check(N, VX.size, pvx, pvy, K, pv, pb, EToE.ctypes.data_as(_P),
                                EToF.ctypes.data_as(_P)))
    return EToE, EToF


def reference_element(N):
    """Host-only reference nodes and operators of degree N."""
    Np = (N + 1) * (N + 2) // 2
    Nfp = N + 1
    out = {k: np.empty(n) for k, n in
           (("r", Np), ("s", Np), ("Dr", Np * Np), ("Ds", Np * Np), ("M", Np * Np),
            ("LIFT", Np * 3 * Nfp))}
    check(lib().ipdg_reference_element(N, *(out[k].ctypes.data_as(_P) for k in
                                            ("r", "s", "Dr", "Ds", "M", "LIFT"))))
    for k in ("Dr", "Ds", "M"):
        out[k] = out[k].reshape(Np, Np)
    out["LIFT"] = out["LIFT"].reshape(Np, 3 * Nfp)
    return out


def _stream(stream):
    if stream is not None:
        return _P(int(stream))
    import torch
    return _P(torch.cuda.current_stream().cuda_stream)


def _dev_vec(t, n, dtypes=None, name="vector"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return _P(t.data_ptr())


class Mesh:
    """A degree-N SIPDG operator on a triangle mesh (device-resident)."""

    def __init__(self, N, VX, VY, EToV, EToB, kappa=None):
        self.N = int(N)
        VX, pvx = _np_ptr(VX, np.float64)
        VY, pvy = _np_ptr(VY, np.float64)
        EToV, pv = _np_ptr(EToV, np.int32)
        EToB, pb = _np_ptr(EToB, np.int8)
        self.K = int(EToV.shape[0])
        self.Np = (self.N + 1) * (self.N + 2) // 2
        pk = None
        if kappa is not None:
            kappa, pk = _np_ptr(kappa, np.float64)
        h = _P()
        check(lib().ipdg_mesh_create(self.N, VX.size, pvx, pvy, self.K, pv, pb, pk, C.byref(h)))
        self._h = h

    @classmethod
    def from_synth(cls, N, msh, kappa=None):
        return cls(N, msh.VX, msh.VY, msh.EToV, msh.EToB, kappa)

    @property
    def handle(self):
        return self._h

    @property
    def ndof(self):
        return self.K * self.Np

    def close(self):
        if getattr(self, "_h", None):
            lib().ipdg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_coords(self):
        x = np.empty(self.ndof)
        y = np.empty(self.ndof)
        check(lib().ipdg_node_coords(self._h, x.ctypes.data_as(_P), y.ctypes.data_as(_P)))
        return x, y

    def set_kappa(self, kappa):
        pk = None
        if kappa is not None:
            kappa, pk = _np_ptr(kappa, np.float64)
        check(lib().ipdg_set_kappa(self._h, pk))

    def apply(self, x, lam=0.0, tau=0.0, out=None, stream=None):
        """y = (lam M - Lap_IPDG) x; x is a float64 or float32 device tensor."""
        import torch
        dt = F64 if x.dtype == torch.float64 else F32
        px = _dev_vec(x, self.ndof, (torch.float64, torch.float32), "x")
        if out is None:
            out = torch.empty_like(x)
        py = _dev_vec(out, self.ndof, (x.dtype,), "out")
        check(lib().ipdg_apply(self._h, float(lam), float(tau), dt, px, py, _stream(stream)))
        return out

    def autotune(self, lam=0.0, tau=0.0, dtype="f64", reps=20, stream=None):
        """Time the operator variants of this degree on this mesh and select the
        fastest for (N, dtype).  Returns (chosen, [ms per apply of variants 0..4],
        -1 where the degree has no such variant)."""
        dt = F64 if dtype in ("f64", F64) else F32
        chosen = C.c_int(-1)
        times = (C.c_double * 5)()
        check(lib().ipdg_autotune_apply(self._h, float(lam), float(tau), dt, int(reps), C.byref(chosen),
                                        C.cast(times, _P), _stream(stream)))
        return chosen.value, list(times)

    def mass(self, x, out=None, stream=None):
        import torch
        dt = F64 if x.dtype == torch.float64 else F32
        px = _dev_vec(x, self.ndof, (torch.float64, torch.float32), "x")
        if out is None:
            out = torch.empty_like(x)
        py = _dev_vec(out, self.ndof, (x.dtype,), "out")
        check(lib().ipdg_mass_apply(self._h, dt, px, py, _stream(stream)))
        return out

    def pcg(self, b, x0=None, lam=0.0, tau=0.0, tol=1e-8, opts=None, stream=None):
        """Solve A x = b (float64 device tensors).  Returns (x, info dict,
        status)."""
        import torch
        pb = _dev_vec(b, self.ndof, (torch.float64,), "b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        px = _dev_vec(x, self.ndof, (torch.float64,), "x")
        o = opts if opts is not None else default_opts()
        info = SolveInfo()
        st = check(lib().ipdg_pcg_solve(self._h, float(lam), float(tau), pb, px, float(tol),
                                        C.byref(o), C.byref(info), _stream(stream)))
        return x, info.as_dict(), st

    def pcg_noalloc(self, b, x, lam=0.0, tau=0.0, tol=1e-8, opts=None, stream=None):
        """ipdg_pcg_solve_noalloc: solve A x = b in place in x (float64 device
        tensors; x holds x0 on entry).  Returns (info dict, status)."""
        import torch
        pb = _dev_vec(b, self.ndof, (torch.float64,), "b")
        px = _dev_vec(x, self.ndof, (torch.float64,), "x")
        o = opts if opts is not None else default_opts()
        info = SolveInfo()
        st = check(lib().ipdg_pcg_solve_noalloc(self._h, float(lam), float(tau), pb, px, float(tol),
                                                C.byref(o), C.byref(info), _stream(stream)))
        return info.as_dict(), st

    def precond(self, r, lam=0.0, tau=0.0, opts=None, stream=None):
        import torch
        pr = _dev_vec(r, self.ndof, (torch.float64,), "r")
        z = torch.empty_like(r)
        pz = _dev_vec(z, self.ndof, (torch.float64,), "z")
        o = opts if opts is not None else default_opts()
        info = SolveInfo()
        check(lib().ipdg_precond_apply(self._h, float(lam), float(tau), C.byref(o), pr, pz,
                                       C.byref(info), _stream(stream)))
        return z, info.as_dict()

    # ---- around the elliptic solves of the splitting scheme (FP64) ----
    def _vec(self, t, name):
        import torch
        return _dev_vec(t, self.ndof, (torch.float64,), name)

    def _opt(self, t, name):
        return self._vec(t, name) if t is not None else None

    def grad(self, p, stream=None):
        """(G_x p, G_y p), central fluxes (Eq. INS_SD_4_1)."""
        import torch
        gx, gy = torch.empty_like(p), torch.empty_like(p)
        check(lib().ipdg_grad(self._h, self._vec(p, "p"), self._vec(gx, "gx"), self._vec(gy, "gy"),
                              _stream(stream)))
        return gx, gy

    def div(self, u, v, gu=None, gv=None, stream=None):
        """D (u, v), central fluxes, Dirichlet data gu, gv (Eq. INS_SD_4_2)."""
        import torch
        out = torch.empty_like(u)
        check(lib().ipdg_div(self._h, self._vec(u, "u"), self._vec(v, "v"), self._opt(gu, "gu"),
                             self._opt(gv, "gv"), self._vec(out, "out"), _stream(stream)))
        return out

    def advect(self, u, v, gu=None, gv=None, stream=None):
        """N(u, v): the nodal Lax-Friedrichs advection term (Eq. INS_SD_2/3)."""
        import torch
        nu, nv = torch.empty_like(u), torch.empty_like(v)
        check(lib().ipdg_advect(self._h, self._vec(u, "u"), self._vec(v, "v"), self._opt(gu, "gu"),
                                self._opt(gv, "gv"), self._vec(nu, "nu"), self._vec(nv, "nv"), _stream(stream)))
        return nu, nv

    def dirichlet_rhs(self, g, b, tau=0.0, stream=None):
        """b += the Dirichlet-data terms of the nodal field g (in place)."""
        check(lib().ipdg_dirichlet_rhs(self._h, float(tau), self._vec(g, "g"), self._vec(b, "b"), _stream(stream)))
        return b

    def ins_velocity_rhs(self, nu, dt, uhat, vhat, sigma_p, stream=None):
        import torch
        bu, bv = torch.empty_like(uhat), torch.empty_like(vhat)
        check(lib().ipdg_ins_velocity_rhs(self._h, float(nu), float(dt), self._vec(uhat, "uhat"),
                                          self._vec(vhat, "vhat"), self._vec(sigma_p, "sigma_p"),
                                          self._vec(bu, "bu"), self._vec(bv, "bv"), _stream(stream)))
        return bu, bv

    def ins_pressure_rhs(self, gamma, dt, u, v, gu=None, gv=None, stream=None):
        import torch
        b = torch.empty_like(u)
        check(lib().ipdg_ins_pressure_rhs(self._h, float(gamma), float(dt), self._vec(u, "u"), self._vec(v, "v"),
                                          self._opt(gu, "gu"), self._opt(gv, "gv"), self._vec(b, "b"),
                                          _stream(stream)))
        return b

    def ins_correct(self, gamma, dt, u, v, dp, sigma_p, stream=None):
        import torch
        uo, vo, po = torch.empty_like(u), torch.empty_like(v), torch.empty_like(dp)
        check(lib().ipdg_ins_correct(self._h, float(gamma), float(dt), self._vec(u, "u"), self._vec(v, "v"),
                                     self._vec(dp, "dp"), self._vec(sigma_p, "sigma_p"), self._vec(uo, "u_out"),
                                     self._vec(vo, "v_out"), self._vec(po, "p_out"), _stream(stream)))
        return uo, vo, po

    def ins_step(self, pmesh, nu, dt, u, v, p, p_prev, gu_n=None, gv_n=None, gu_1=None, gv_1=None, tau=0.0,
                 tol=1e-10, vel_opts=None, pres_opts=None, subcycles=0, stream=None):
        """One first-order step of the splitting scheme (ipdg_ins_step, or
        ipdg_ins_step_subcycled when subcycles > 0); returns (u, v, p) at
        t^{n+1} and the three solves' iteration counts."""
        import torch
        u1, v1, p1 = torch.empty_like(u), torch.empty_like(v), torch.empty_like(p)
        it = (C.c_int * 3)()
        vo = C.byref(vel_opts) if vel_opts is not None else None
        po = C.byref(pres_opts) if pres_opts is not None else None
        vecs = (self._vec(u, "u"), self._vec(v, "v"), self._vec(p, "p"), self._vec(p_prev, "p_prev"),
                self._opt(gu_n, "gu_n"), self._opt(gv_n, "gv_n"), self._opt(gu_1, "gu_1"), self._opt(gv_1, "gv_1"),
                self._vec(u1, "u_1"), self._vec(v1, "v_1"), self._vec(p1, "p_1"))
        if subcycles:
            check(lib().ipdg_ins_step_subcycled(self._h, pmesh.handle, float(nu), float(dt), float(tau),
                                                int(subcycles), *vecs, float(tol), vo, po, it, _stream(stream)))
        else:
            check(lib().ipdg_ins_step(self._h, pmesh.handle, float(nu), float(dt), float(tau), *vecs, float(tol),
                                      vo, po, it, _stream(stream)))
        return u1, v1, p1, list(it)

    def subcycle_rhs(self, ubar, vbar, u, v, gu=None, gv=None, parts=3, stream=None):
        """N~(Ubar, U~) of the subcycling advection with cubature (Eq. KSS_3):
        parts 1 the volume term, 2 the surface term, 3 both."""
        import torch
        nu, nv = torch.empty_like(u), torch.empty_like(v)
        check(lib().ipdg_subcycle_rhs(self._h, self._vec(ubar, "ubar"), self._vec(vbar, "vbar"), self._vec(u, "u"),
                                      self._vec(v, "v"), self._opt(gu, "gu"), self._opt(gv, "gv"), int(parts),
                                      self._vec(nu, "nu"), self._vec(nv, "nv"), _stream(stream)))
        return nu, nv

    def subcycle(self, ubar0, vbar0, u, v, T, Ns, ubar1=None, vbar1=None, gu0=None, gv0=None, gu1=None, gv1=None,
                 stream=None):
        """Ns low-storage RK4 steps over [0, T] of dU~/dt = -N~(Ubar(t), U~),
        Ubar(t) = Ubar0 + t Ubar1, Dirichlet data g0 + t g1 (Eq. SS_3).
        Returns new tensors (the inputs are left unchanged)."""
        uo, vo = u.clone(), v.clone()
        check(lib().ipdg_subcycle(self._h, self._vec(ubar0, "ubar0"), self._vec(vbar0, "vbar0"),
                                  self._opt(ubar1, "ubar1"), self._opt(vbar1, "vbar1"), self._opt(gu0, "gu0"),
                                  self._opt(gv0, "gv0"), self._opt(gu1, "gu1"), self._opt(gv1, "gv1"), float(T),
                                  int(Ns), self._vec(uo, "u"), self._vec(vo, "v"), _stream(stream)))
        return uo, vo

    def kappa_grad(self, u, w, tau=0.0, stream=None):
        import torch
        pu = _dev_vec(u, self.ndof, (torch.float64,), "u")
        pw = _dev_vec(w, self.ndof, (torch.float64,), "w")
        g = torch.empty(self.K, dtype=torch.float64, device=u.device)
        check(lib().ipdg_kappa_grad(self._h, float(tau), pu, pw, _P(g.data_ptr()),
                                    _stream(stream)))
        return g


def solve_batch(meshes, lambdas, bs, tol=1e-8, tau=0.0, opts=None, stream=None):
    """Independent solves (lambda_i M - Lap) x_i = b_i, advanced together."""
    import torch
    nb = len(meshes)
    xs = [torch.zeros_like(b) for b in bs]
    H = (_P * nb)(*[m.handle for m in meshes])
    lam = (C.c_double * nb)(*[float(v) for v in lambdas])
    Bp = (_P * nb)(*[_dev_vec(b, m.ndof, (torch.float64,), "b") for b, m in zip(bs, meshes)])
    Xp = (_P * nb)(*[_dev_vec(x, m.ndof, (torch.float64,), "x") for x, m in zip(xs, meshes)])
    iters = (C.c_int * nb)()
    rel = (C.c_double * nb)()
    o = opts if opts is not None else default_opts(pc=PC_BLOCK_MASS)
    st = check(lib().ipdg_helmholtz_solve_batch(nb, C.cast(H, _P), C.cast(lam, _P), float(tau),
                                                C.cast(Bp, _P), C.cast(Xp, _P), float(tol),
                                                C.byref(o), C.cast(iters, _P), C.cast(rel, _P),
                                                _stream(stream)))
    return xs, list(iters), list(rel), st
