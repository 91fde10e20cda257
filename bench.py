#!/usr/bin/env python3
"""Benchmark of the SIPDG elliptic operator and solvers on one MI355X.

Workload (the operator-throughput sweep): a 512 x 512-square triangulation of
the unit square (524,288 triangles), interior vertices jittered by +-0.2 h,
all faces Dirichlet, x ~ N(0,1) per node, c_tau = (N+1)^2.

A step is one application y = (lambda M - Lap_IPDG) x of the headline
configuration (default N = 3, FP64, lambda = 100).  Inputs are resident in
device memory; the timed loop rotates over enough independent copies of the
mesh data and vectors (> 1.2 GB) that the 256 MB last-level cache cannot hold
them, and is bracketed by HIP events on the stream the kernels run on.  Before
the warm-up steps, every copy is applied once and the device runs the
operator for about 0.1 s (untimed set-up), so that the timed steps see
mapped pages and working clocks rather than the state the host-side mesh
set-up left the device in.

One JSON line is printed with the headline throughput, the roofline of the
operator kernel, the CPU oracle baseline, the per-degree sweep and (when
built) the PCG + p-multigrid time-to-solution comparison.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6           # vector FP64, published
FP32_PEAK_TFS = 157.3          # vector FP32, published


# HBM bytes of one operator launch of the headline configuration, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE), each scaled by the
# counter's reading for a device-to-device copy of known size.  Valid only for
# the kernel sources it was measured on (their SHA-256), else reported null.
MEASURED_TRAFFIC = {"N": 3, "dtype": "f64", "lambda": 100.0, "variant": 4, "bytes": 111073404,
                    "sources_sha256": "901241b4655e18fb6030ea9cbdadb70cd6fa3aafea58299de02bbb73355439c2",
                    "profile": "profiles/k_axc_N3_f64_524288.md"}

KERNEL_SOURCES = ("elem_inst.hip", "sipdg_core.hpp", "sipdg_coop.hpp", "tri.hpp", "device_common.hpp",
                  "kernels.hpp", "ops_table.cpp", "ops_table.hpp", "refelem.cpp", "refelem.hpp", "dispatch.cpp")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1801_00246_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(N, dtype, lam, variant):
    t = MEASURED_TRAFFIC
    if not t or (t["N"], t["dtype"], t["lambda"], t["variant"]) != (N, dtype, lam, variant):
        return None
    return t["bytes"] if t["sources_sha256"] == kernel_sources_sha() else None


def np_of(N):
    return (N + 1) * (N + 2) // 2


def alg_bytes(N, w):
    """Minimum bytes per element: x and y (Np each), 5 metric terms, 3
    neighbour ids."""
    return (2 * np_of(N) + 5) * w + 12


def alg_flops(N):
    """Flops per element of the operator in its local-gradient + SIPDG form
    with the lift done once per face: 10 Np^2 + 12 Np Nfp."""
    Np = np_of(N)
    return 10 * Np * Np + 12 * Np * (N + 1)


def time_applies(P, torch, msh, N, dtype, lam, steps, warmup, rotate_bytes):
    """Time `steps` applications rotating over independent data sets."""
    import synth
    w = 8 if dtype == torch.float64 else 4
    K = msh.K
    Np = np_of(N)
    set_bytes = K * (2 * Np * w + 4 * w + 16)
    R = max(1, math.ceil(rotate_bytes / set_bytes))
    meshes = [P.Mesh.from_synth(N, msh) for _ in range(R)]
    x0 = torch.from_numpy(synth.nodal_normal(K, Np, seed=1)).to("cuda", dtype)
    xs = [x0.clone() for _ in range(R)]
    ys = [torch.empty_like(x0) for _ in range(R)]
    # set-up (untimed): every rotation set is applied once (first touch of its
    # pages), then the device runs the operator for about 0.1 s so that its
    # clocks have left the idle state the host-side mesh set-up left it in
    for i in range(R):
        meshes[i].apply(xs[i], lam=lam, out=ys[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < 0.1:
        for _ in range(R):
            meshes[i % R].apply(xs[i % R], lam=lam, out=ys[i % R])
            i += 1
        torch.cuda.synchronize()
    for i in range(warmup):
        meshes[i % R].apply(xs[i % R], lam=lam, out=ys[i % R])
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(steps):
        meshes[i % R].apply(xs[i % R], lam=lam, out=ys[i % R])
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for m in meshes:
        m.close()
    return ms / steps, R


def roofline(N, dtype_bytes, ms):
    t = ms * 1e-3
    K = 524288
    nbytes = K * alg_bytes(N, dtype_bytes)
    flops = K * alg_flops(N)
    peak_f = FP64_PEAK_TFS if dtype_bytes == 8 else FP32_PEAK_TFS
    ai = flops / nbytes
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai < ridge:
        ach = nbytes / t / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "alg_bytes_per_launch": nbytes, "alg_flops_per_launch": flops}
    ach = flops / t / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": peak_f, "unit": "TFLOP/s",
            "frac": round(ach / peak_f, 4), "traffic": None,
            "alg_bytes_per_launch": nbytes, "alg_flops_per_launch": flops}


def copy_probe(P, nbytes, reps=40):
    """Device-to-device copy bandwidth (the paper's empirical roof): GB/s of
    read + write traffic of the library's vectorised HIP copy kernel copying
    nbytes, rotating over source/destination pairs totalling > 1.2 GB (so
    that the 256 MB last-level cache cannot hold them)."""
    sets = max(2, math.ceil(1.2e9 / (2 * nbytes)))
    return P.probe_copy(int(nbytes), sets, reps)


_MF = {}


def _mf_init(N, n):
    """Worker set-up (spawned process): the oracle's matrix-free operator on
    the workload mesh, one BLAS thread."""
    from threadpoolctl import threadpool_limits
    import synth
    from oracle.assemble import OracleMesh
    from oracle.matfree import MatFree
    threadpool_limits(1)
    msh = synth.ax_sweep_mesh(n, seed=0)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    _MF["mf"] = MatFree(m)
    _MF["x"] = synth.nodal_normal(msh.K, m.Np, seed=1)


def _mf_rows(args):
    """Rows of the elements [lo, hi), `reps` times; returns the seconds."""
    import numpy as np
    lo, hi, lam, ctau, reps = args
    mf = _MF["mf"]
    el = np.arange(lo, hi)
    t0 = time.perf_counter()
    for _ in range(reps):
        mf.apply(lam, ctau, _MF["x"], elems=el)
    return time.perf_counter() - t0


def cpu_baseline(N, lam, target_s=6.0):
    """The FP64 oracle timed on the host's cores, on the operator workload.

    Leg 1 (the reported value): the oracle's matrix-free operator (Alg. AxG +
    Alg. AxKernel) over all 524,288 elements, split into contiguous element
    ranges over a pool of spawned worker processes (one BLAS thread each),
    repeated until about target_s seconds have passed.  Leg 2: the same on one
    core.  Leg 3: the oracle's assembled block rows of the first 32,768
    elements multiplied by scipy's CSR product (single-threaded)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits
    import synth
    from oracle.assemble import OracleMesh, block_rows
    n = 512
    K = 2 * n * n
    Np = np_of(N)
    ctau = float((N + 1) ** 2)
    nproc = os.cpu_count() or 1
    workers = max(1, min(16, nproc))
    out = {"unit": "GDOF/s", "kind": "oracle"}
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx, initializer=_mf_init,
                                initargs=(N, n)) as ex:
        bounds = np.linspace(0, K, workers + 1).astype(int)
        # warm-up round (also makes every worker finish its set-up)
        list(ex.map(_mf_rows, [(int(bounds[i]), int(bounds[i + 1]), lam, ctau, 1) for i in range(workers)]))
        t0 = time.perf_counter()
        t1 = max(ex.map(_mf_rows, [(int(bounds[i]), int(bounds[i + 1]), lam, ctau, 1)
                                   for i in range(workers)]))
        reps = max(1, int(target_s / max(t1, 1e-3)))
        t0 = time.perf_counter()
        list(ex.map(_mf_rows, [(int(bounds[i]), int(bounds[i + 1]), lam, ctau, reps)
                               for i in range(workers)]))
        dt_all = time.perf_counter() - t0
    out["value"] = reps * K * Np / dt_all / 1e9
    out["cores"] = workers
    out["host_cpus"] = nproc
    out["sample"] = (f"matrix-free oracle (Alg. AxG + AxKernel, numpy FP64) over all {K} elements "
                     f"at N={N}, lambda={lam}, {reps} applies in {dt_all:.1f}s, element ranges over "
                     f"{workers} spawned processes of 1 BLAS thread each (set-up excluded)")
    # one core, in this process
    _mf_init(N, n)
    with threadpool_limits(1):
        S = 65536
        _mf_rows((0, S, lam, ctau, 1))
        r1 = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < target_s:
            _mf_rows((0, S, lam, ctau, 1))
            r1 += 1
        dt1 = time.perf_counter() - t0
        out["one_core"] = {"value": r1 * S * Np / dt1 / 1e9, "cores": 1,
                           "sample": f"elements 0..{S - 1}, {r1} applies in {dt1:.1f}s"}
        _MF.clear()
        # assembled CSR rows of a sample, scipy's single-threaded product
        msh = synth.ax_sweep_mesh(n, seed=0)
        m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        S = 32768
        r, c, b = block_rows(m, lam, ctau, elems=np.arange(S))
        ii = np.broadcast_to(r[:, None, None] * Np + np.arange(Np)[None, :, None], b.shape).ravel()
        jj = np.broadcast_to(c[:, None, None] * Np + np.arange(Np)[None, None, :], b.shape).ravel()
        A = sp.csr_matrix((b.ravel(), (ii, jj)), shape=(S * Np, K * Np))
        x = synth.nodal_normal(K, Np, seed=1)
        r2 = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < target_s / 2:
            A @ x
            r2 += 1
        dt2 = time.perf_counter() - t0
        out["assembled_spmv_one_core"] = {"value": r2 * S * Np / dt2 / 1e9, "cores": 1,
                                          "sample": f"CSR block rows of elements 0..{S - 1}, "
                                                    f"{r2} products in {dt2:.1f}s (assembly excluded)"}
    return out


def run_pcg_compare(P, torch, coarse_caps=(150, 300)):
    """PCG + p-multigrid (7 -> 3 -> 1) on 256 x 256 squares, N = 7, FP64 vs
    mixed precision, time to a true relative residual of 1e-8."""
    import numpy as np
    import synth
    msh = synth.square_mesh(256)
    N = 7
    g = P.Mesh.from_synth(N, msh)
    x, y = g.node_coords()
    f = torch.from_numpy(2 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y)).to("cuda")
    b = g.mass(f)
    out = {"workload": "256x256 squares (131,072 triangles), N=7, f from sin(pi x) sin(pi y), "
                       "Dirichlet, lambda=0, tol 1e-8, pMG 7->3->1, Chebyshev(2), coarse Jacobi-PCG"}
    for cmax in coarse_caps:
        precs = [("fp64", P.PREC_FP64), ("mixed", P.PREC_MIXED)]
        if cmax == coarse_caps[0]:
            # FP32 outer operator as well (reliable updates after every 1e3 fall)
            precs.append(("fp32op", P.PREC_FP32_OPERATOR))
        for name, prec in precs:
            o = P.default_opts(pc=P.PC_PMG, prec=prec, degrees=[7, 3, 1], coarse_max_iters=cmax)
            g.pcg(b, tol=1e-8, opts=o)                 # setup + warm-up
            torch.cuda.synchronize()
            t0 = time.time()
            xs, info, st = g.pcg(b, tol=1e-8, opts=o)
            torch.cuda.synchronize()
            key = f"{name}_coarse{cmax}"
            out[key] = {"time_to_solution_ms": round((time.time() - t0) * 1e3, 2),
                        "coarse_iters_last": info["coarse_iters"],
                        "precond_bytes_per_element": round(info["precond_bytes"] / msh.K),
                        "iters": info["iters"], "true_relres": info["relres"],
                        "restarts": info["restarts"], "setup_ms": round(info["setup_ms"], 2)}
            print(f"# pcg {key}: {out[key]}", file=sys.stderr, flush=True)
    # pMG-AMG: the degree-1 level by one cycle of the aggregation AMG below it
    # (K-cycle on its two finest levels); "amg_top": the degree-1 level by two
    # flexible-CG steps, each preconditioned by one such cycle
    for name, prec, top in (("fp64", P.PREC_FP64, 0), ("mixed", P.PREC_MIXED, 0), ("fp64", P.PREC_FP64, 1),
                            ("mixed", P.PREC_MIXED, 1)):
        o = P.default_opts(pc=P.PC_PMG, prec=prec, degrees=[7, 3, 1], coarse_amg=1, amg_top_krylov=top)
        g.pcg(b, tol=1e-8, opts=o)                     # setup + warm-up
        torch.cuda.synchronize()
        t0 = time.time()
        xs, info, st = g.pcg(b, tol=1e-8, opts=o)
        torch.cuda.synchronize()
        key = f"{name}_amg" + ("_top" if top else "")
        out[key] = {"time_to_solution_ms": round((time.time() - t0) * 1e3, 2), "iters": info["iters"],
                    "true_relres": info["relres"], "amg_sizes": info["amg_sizes"],
                    "precond_bytes_per_element": round(info["precond_bytes"] / msh.K),
                    "setup_ms": round(info["setup_ms"], 2)}
        print(f"# pcg {key}: {out[key]}", file=sys.stderr, flush=True)
    return out


def run_gradiv(P, torch, msh, orders=(3, 7), steps=50, rotate_bytes=1.2e9):
    """DG gradient and divergence (central fluxes) and the nodal advection
    term on the 524,288-triangle mesh, FP64: microseconds per launch (HIP
    events over `steps` launches rotating over independent data sets) and
    algorithmic bandwidth, each launch reading one (G) or two (D, advection)
    nodal fields, writing two (G, advection) or one (D), plus the metric
    (32 B) and connectivity (16 B) per element."""
    import ctypes as C
    import synth
    out = {}
    K = msh.K
    for N in orders:
        Np = np_of(N)
        nbytes = K * (3 * Np * 8 + 48)
        R = max(1, math.ceil(rotate_bytes / nbytes))
        g = P.Mesh.from_synth(N, msh)
        x0 = torch.from_numpy(synth.nodal_normal(K, Np, seed=3)).to("cuda")
        ins = [(x0.clone(), x0.clone()) for _ in range(R)]
        outs = [(torch.empty_like(x0), torch.empty_like(x0)) for _ in range(R)]
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        ptr = lambda t: C.c_void_p(t.data_ptr())
        lib = P.lib()

        def grad(i):
            a, (o1, o2) = ins[i % R][0], outs[i % R]
            return lib.ipdg_grad(g.handle, ptr(a), ptr(o1), ptr(o2), st)

        def div(i):
            (a, b), o = ins[i % R], outs[i % R][0]
            return lib.ipdg_div(g.handle, ptr(a), ptr(b), None, None, ptr(o), st)

        def advect(i):
            (a, b), (o1, o2) = ins[i % R], outs[i % R]
            return lib.ipdg_advect(g.handle, ptr(a), ptr(b), None, None, ptr(o1), ptr(o2), st)

        res = {}
        for name, fn in (("grad", grad), ("div", div), ("advect", advect)):
            for i in range(R + 5):
                assert fn(i) == 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                fn(i)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / steps
            nb = nbytes if name != "advect" else K * (4 * Np * 8 + 48)
            gbs = nb / (us * 1e-6) / 1e9
            res[name] = {"us": round(us, 2), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / 8000.0, 4)}
        out[f"N{N}"] = res
        print(f"# gradiv N={N}: {res}", file=sys.stderr, flush=True)
        g.close()
    return out


def sub_dims(N):
    """Cubature sizes of the subcycling operator: q = floor(3N/2) + 1 Gauss
    points per direction (volume q^2, faces q)."""
    q = 3 * N // 2 + 1
    return q * q, q


def sub_flops(N):
    """Algorithmic FP64 flops per element of the subcycling operator as the
    kernel evaluates it: volume = interpolation of four fields (8 Nc Np),
    contravariant fluxes (10 Nc), projection with P_r, P_s for two components
    (8 Np Nc); surface = interpolation of eight traces on three faces
    (48 Nfc Nfp), the Lax-Friedrichs flux (20 per face point), the lift of two
    components (12 Np Nfc).  Also the matrix-core flops issued (16 x 16 x 4
    blocks of 2048 flops, padding included) per element."""
    Np, Nfp = np_of(N), N + 1
    Nc, Nfc = sub_dims(N)
    vol = 16 * Np * Nc + 10 * Nc
    surf = 48 * Nfc * Nfp + 60 * Nfc + 12 * Np * Nfc
    TC, KB, RB = -(-Nc // 16), -(-Np // 4), -(-Np // 16)
    KF, KT = -(-Nfp // 4), -(-Nfc // 4)
    mf_vol = (TC * KB * 4 + TC * 4 * RB * 4) * 2048 / 16
    mf_surf = 3 * (KF * 8 + KT * RB * 2) * 2048 / 16
    return vol, surf, mf_vol, mf_surf


def run_subcycle(P, torch, msh, orders=(3, 5, 7), steps=20, Ns=4):
    """Subcycling advection with cubature (Eq. KSS_3) on the 524,288-triangle
    mesh, FP64: microseconds per launch of the volume term (Alg. SSV), the
    surface term (Alg. SSS) and the fused operator (HIP events over `steps`
    launches on torch's stream), algorithmic TFLOP/s against the FP64 dense
    matrix-core peak, and the whole subcycle call (Ns five-stage substeps,
    one fused operator-and-update launch per stage; HIP events around the
    call on the same stream) per substep."""
    import ctypes as C
    import synth
    out = {"workload": "512x512-square jittered triangulation (524,288 triangles), all Dirichlet, "
                       "fields ~ N(0,1), FP64"}
    K = msh.K
    for N in orders:
        Np = np_of(N)
        g = P.Mesh.from_synth(N, msh)
        f = [torch.from_numpy(synth.nodal_normal(K, Np, seed=20 + i)).to("cuda") for i in range(6)]
        nu, nv = torch.empty_like(f[0]), torch.empty_like(f[0])
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        ptr = lambda t: C.c_void_p(t.data_ptr())
        lib = P.lib()
        vol, surf, mf_vol, mf_surf = sub_flops(N)
        res = {"Nc": sub_dims(N)[0], "Nfc": sub_dims(N)[1]}
        for name, parts, fl, mf in (("volume", 1, vol, mf_vol), ("surface", 2, surf, mf_surf),
                                    ("both", 3, vol + surf, mf_vol + mf_surf)):
            def run():
                return lib.ipdg_subcycle_rhs(g.handle, ptr(f[0]), ptr(f[1]), ptr(f[2]), ptr(f[3]), ptr(f[4]),
                                             ptr(f[5]), parts, ptr(nu), ptr(nv), st)
            for _ in range(3):
                assert run() == 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                run()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / steps
            tf = K * fl / (us * 1e-6) / 1e12
            res[name] = {"us": round(us, 2), "alg_TFLOP/s": round(tf, 2), "frac_fp64_peak": round(tf / 78.6, 4),
                         "mfma_TFLOP/s_issued": round(K * mf / (us * 1e-6) / 1e12, 2),
                         "alg_flops_per_element": fl}
        u, v = f[2].clone(), f[3].clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        assert lib.ipdg_subcycle(g.handle, ptr(f[0]), ptr(f[1]), None, None, ptr(f[4]), ptr(f[5]), None, None,
                                 C.c_double(1e-4), Ns, ptr(u), ptr(v), st) == 0
        e0.record()
        assert lib.ipdg_subcycle(g.handle, ptr(f[0]), ptr(f[1]), None, None, ptr(f[4]), ptr(f[5]), None, None,
                                 C.c_double(1e-4), Ns, ptr(u), ptr(v), st) == 0
        e1.record()
        torch.cuda.synchronize()
        res["subcycle_ms_per_substep"] = round(e0.elapsed_time(e1) / Ns, 4)
        out[f"N{N}"] = res
        print(f"# subcycle N={N}: {res}", file=sys.stderr, flush=True)
        del f, nu, nv, u, v
        g.close()
    return out


def run_ins_step(P, torch, n=64, N=5, nu=0.01, dt=1e-3, steps=5, subcycles=0):
    """Splitting steps (ipdg_ins_step, first order; ipdg_ins_step_subcycled
    when subcycles > 0) of the Taylor vortex on n x n squares at degree N,
    Dirichlet velocity data from the exact field, p-multigrid PCG to 1e-8 for
    the three solves: ms per step, solver iterations, and the velocity error
    after the timed steps."""
    import numpy as np
    import synth
    msh = synth.square_mesh(n, jitter=0.1, seed=60)
    flags = np.where(msh.EToB == P.BC_DIRICHLET, P.BC_NEUMANN,
                     np.where(msh.EToB == P.BC_NEUMANN, P.BC_DIRICHLET, msh.EToB))
    g = P.Mesh.from_synth(N, msh)
    gp = P.Mesh(N, msh.VX, msh.VY, msh.EToV, flags)
    x, y = (np.asarray(a).ravel() for a in g.node_coords())

    def taylor(t):
        f = np.exp(-2 * np.pi ** 2 * nu * t)
        return [torch.from_numpy(a).to("cuda") for a in
                (-np.cos(np.pi * x) * np.sin(np.pi * y) * f, np.sin(np.pi * x) * np.cos(np.pi * y) * f,
                 -0.25 * (np.cos(2 * np.pi * x) + np.cos(2 * np.pi * y)) * f * f)]

    o = P.default_opts(pc=P.PC_PMG)
    t = 0.0
    u, v, p = taylor(t)
    pm1 = taylor(t - dt)[2]
    data = [taylor(t + k * dt) for k in range(steps + 2)]
    times, its = [], []
    for k in range(steps + 1):                          # the first step sets up the solvers (untimed)
        torch.cuda.synchronize()
        t0 = time.time()
        u1, v1, p1, it = g.ins_step(gp, nu, dt, u, v, p, pm1, data[k][0], data[k][1], data[k + 1][0],
                                    data[k + 1][1], tol=1e-8, vel_opts=o, pres_opts=o, subcycles=subcycles)
        torch.cuda.synchronize()
        if k:
            times.append((time.time() - t0) * 1e3)
            its.append(it)
        pm1, u, v, p = p, u1, v1, p1
    ue, ve = data[steps + 1][0], data[steps + 1][1]
    err = float(torch.sqrt(((u - ue) ** 2).sum() + ((v - ve) ** 2).sum()) / torch.sqrt((ue ** 2).sum() + (ve ** 2).sum()))
    g.close()
    gp.close()
    adv = (f"advection subcycled ({subcycles} low-storage RK4 substeps, cubature operator)" if subcycles
           else "explicit nodal advection")
    return {"workload": f"Taylor vortex, {n}x{n} squares ({msh.K} triangles), N={N}, nu={nu}, dt={dt}, "
                        f"first-order splitting, {adv}, pMG-PCG to 1e-8 for the u, v and pressure solves",
            "ms_per_step": round(sum(times) / len(times), 2), "solver_iters_per_step": its[-1],
            "velocity_rel_error_nodal": err}


def run_batch_compare(P, torch, nb=64, prec=None, tol=1e-8):
    """Batched Helmholtz: nb independent (lambda_i M - Lap) u_i = M f_i on
    n_i x n_i squares (n_i ~ U{32..128}), N_i ~ U{4..8}, lambda_i = 10^U(0,3),
    f ~ N(0,1) nodal, Dirichlet, PCG with p-multigrid on halved degrees
    (N_i -> N_i/2 -> ... -> 1) to 1e-8; one batched call (one graph launch
    per check interval) vs nb serial solves."""
    import synth
    ns, Ns, lams, fseeds = synth.batch_draws(nb, seed=4)
    meshes, bs = [], []
    for n, N, fs in zip(ns, Ns, fseeds):
        msh = synth.square_mesh(int(n))
        g = P.Mesh.from_synth(int(N), msh)
        f = torch.from_numpy(synth.nodal_normal(msh.K, g.Np, seed=int(fs))).to("cuda")
        meshes.append(g)
        bs.append(g.mass(f))
    o = P.default_opts(pc=P.PC_PMG, prec=P.PREC_FP64 if prec is None else prec)

    def batched():
        torch.cuda.synchronize()
        t0 = time.time()
        out = P.solve_batch(meshes, lams, bs, tol=tol, opts=o)
        torch.cuda.synchronize()
        return time.time() - t0, out

    def serial():
        its = []
        torch.cuda.synchronize()
        t0 = time.time()
        for g, lam, b in zip(meshes, lams, bs):
            _, info, _ = g.pcg(b, lam=float(lam), tol=tol, opts=o)
            its.append(info["iters"])
        torch.cuda.synchronize()
        return time.time() - t0, its

    # warm-up (set-up of every mesh: spectral estimates, captured graphs);
    # serial solves run back to back so that each keeps its captured graph
    batched()
    serial()
    t_serial, serial_iters = serial()
    t_batch, (xs, iters, rel, st) = batched()
    dofs = sum(g.ndof for g in meshes)
    out = {"workload": f"{nb} solves, n~U{{32..128}}, N~U{{4..8}}, lambda=10^U(0,3), "
                       "PCG + p-multigrid on halved degrees, tol 1e-8",
           "total_dofs": dofs, "batched_s": round(t_batch, 3), "serial_s": round(t_serial, 3),
           "speedup": round(t_serial / t_batch, 2), "iters_max": max(iters), "iters_sum": sum(iters),
           "serial_iters_sum": sum(serial_iters),
           "max_relres": max(rel), "status": st}
    if prec is None:
        # the same batch with the FP32 preconditioner (FP64 CG), batched only
        o = P.default_opts(pc=P.PC_PMG, prec=P.PREC_MIXED)
        batched()
        t_m, (_, it_m, rel_m, st_m) = batched()
        out["mixed"] = {"batched_s": round(t_m, 3), "iters_sum": sum(it_m), "max_relres": max(rel_m),
                        "status": st_m}
    return out


def run_grad_compare(P, torch, n=128, N=5, lam=1.0, tol=1e-8, reps=3):
    """Differentiable solve: n x n squares (jittered), N = 5, kappa_e =
    exp(0.5 N(0,1)), f ~ N(0,1) nodal, L = (u - u_t)^T M (u - u_t) with u_t a
    smooth sine series; dL/df and dL/dkappa through forward PCG + adjoint PCG
    + the kappa-gradient kernel, p-multigrid 5 -> 2 -> 1, FP64 vs mixed."""
    import numpy as np
    import synth
    from paper_1801_00246_amd.autograd import helmholtz_solve, mass
    msh = synth.square_mesh(n, jitter=0.2, seed=0)
    kap = synth.kappa_draw(msh.K, seed=2)
    g = P.Mesh.from_synth(N, msh, kappa=kap)
    x, y = g.node_coords()
    ut = torch.from_numpy(synth.smooth_field(x.ravel(), y.ravel(), synth.smooth_coeffs(seed=3))).to("cuda")
    f0 = torch.from_numpy(synth.nodal_normal(msh.K, g.Np, seed=5)).to("cuda")
    kap0 = torch.from_numpy(kap).to("cuda")
    out = {"workload": f"{n}x{n} squares ({msh.K} triangles), N={N}, kappa lognormal(0,0.5), "
                       f"lambda={lam}, tol {tol}, pMG {N}->{N // 2}->...->1; forward + adjoint"}
    grads = {}
    for name, prec in (("fp64", P.PREC_FP64), ("mixed", P.PREC_MIXED)):
        o = P.default_opts(pc=P.PC_PMG, prec=prec)
        times = []
        for r in range(reps + 1):
            kap_t = kap0.clone().requires_grad_(True)
            f_t = f0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.time()
            u = helmholtz_solve(f_t, kap_t, g, lam=lam, tol=tol, opts=o)
            d = u - ut
            L = torch.dot(d, mass(d, g))
            L.backward()
            torch.cuda.synchronize()
            if r > 0:                  # the first run includes the set-up
                times.append(time.time() - t0)
        grads[name] = (kap_t.grad.detach().cpu().numpy(), f_t.grad.detach().cpu().numpy())
        out[name] = {"ms_forward_backward": round(1e3 * min(times), 2), "loss": float(L)}
        print(f"# grad {name}: {out[name]}", file=sys.stderr, flush=True)
    gk64, gf64 = grads["fp64"]
    gk32, gf32 = grads["mixed"]
    out["mixed_vs_fp64_rel"] = {"dL/dkappa": float(np.linalg.norm(gk32 - gk64) / np.linalg.norm(gk64)),
                                "dL/df": float(np.linalg.norm(gf32 - gf64) / np.linalg.norm(gf64))}
    # the coefficient-gradient kernel alone (one launch over all elements)
    u = torch.randn(msh.K * g.Np, dtype=torch.float64, device="cuda")
    w = torch.randn_like(u)
    g.kappa_grad(u, w)
    s_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s_)
    for _ in range(20):
        g.kappa_grad(u, w)
    e1.record(s_)
    torch.cuda.synchronize()
    out["kappa_grad_kernel_us"] = round(1e3 * e0.elapsed_time(e1) / 20, 2)
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--lam", type=float, default=100.0)
    ap.add_argument("--rotate-gb", type=float, default=1.2)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-solve batched Helmholtz leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the differentiable-solve leg")
    ap.add_argument("--no-gradiv", action="store_true", help="skip the gradient/divergence leg")
    ap.add_argument("--no-subcycle", action="store_true", help="skip the subcycling advection leg")
    ap.add_argument("--sweep-orders", default="1,2,3,4,5,6,7,8")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the headline with the default operator variant instead of the tuned one")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1801_00246_amd as P
    import synth

    msh = synth.ax_sweep_mesh(512, seed=0)
    dt = torch.float64 if args.dtype == "f64" else torch.float32
    w = 8 if args.dtype == "f64" else 4
    N = args.order
    tuned = None
    if not args.no_autotune:
        # pick the operator variant for the headline degree and precision on this GPU
        # (set-up, outside the timed region)
        g = P.Mesh.from_synth(N, msh)
        chosen, times = g.autotune(lam=args.lam, tau=0.0, dtype=args.dtype, reps=20)
        del g
        tuned = {"chosen": chosen, "ms_per_apply": [round(t, 5) for t in times]}
        print(f"# autotune N={N} {args.dtype}: {tuned}", file=sys.stderr, flush=True)
    variant = P.ax_variant(N, args.dtype)
    ms, R = time_applies(P, torch, msh, N, dt, args.lam, args.steps, args.warmup,
                         args.rotate_gb * 1e9)
    gdofs = msh.K * np_of(N) / (ms * 1e-3) / 1e9
    line = {
        "metric": "IPDG Ax GDOF/s and PCG+pMG time-to-1e-8 (FP64 vs mixed), % HBM roofline",
        "value": round(gdofs, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "Ax throughput: 512x512-square jittered triangulation "
                               "(524,288 triangles), all Dirichlet, x ~ N(0,1)",
                   "N": N, "Np": np_of(N), "lambda": args.lam, "c_tau": (N + 1) ** 2,
                   "rotation_sets": R, "ax_variant": variant, "parallelism": "single GPU"},
    }
    if tuned is not None:
        line["autotune"] = tuned
    line["roofline"] = roofline(N, w, ms)
    line["roofline"]["traffic"] = measured_traffic(N, args.dtype, args.lam, variant)
    # measured roofs (context for the fractions, which use the published peaks)
    line["copy_roof_gbs"] = round(copy_probe(P, msh.K * alg_bytes(N, w) / 2), 1)
    line["fma_peak_tflops"] = {"f64": round(P.probe_fma("f64"), 2), "f32": round(P.probe_fma("f32"), 2)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(N, args.lam)
    if not args.no_sweep:
        sweep = []
        for Ns in [int(v) for v in args.sweep_orders.split(",")]:
            for dname, dts, ws in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
                for lam in (0.0, 100.0):
                    msw, _ = time_applies(P, torch, msh, Ns, dts, lam, 100, 5, args.rotate_gb * 1e9)
                    rf = roofline(Ns, ws, msw)
                    sweep.append({"N": Ns, "dtype": dname, "lambda": lam, "ms": round(msw, 5),
                                  "GDOF/s": round(msh.K * np_of(Ns) / (msw * 1e-3) / 1e9, 3),
                                  "bound": rf["bound"], "frac": rf["frac"],
                                  "achieved": rf["achieved"], "unit": rf["unit"]})
                    print(f"# sweep N={Ns} {dname} lam={lam}: {sweep[-1]}", file=sys.stderr, flush=True)
        line["sweep"] = sweep
    if not args.no_pcg:
        try:
            line["pcg"] = run_pcg_compare(P, torch)
        except P.IpdgError as e:
            line["pcg"] = {"error": str(e)}
    if not args.no_gradiv:
        line["gradiv"] = run_gradiv(P, torch, msh)
        line["ins_step"] = run_ins_step(P, torch)
        print(f"# ins_step: {line['ins_step']}", file=sys.stderr, flush=True)
        # the subcycled step at the same dt, and at four times the step with four substeps
        line["ins_step_subcycled"] = [run_ins_step(P, torch, subcycles=1),
                                      run_ins_step(P, torch, dt=4e-3, subcycles=4)]
        print(f"# ins_step_subcycled: {line['ins_step_subcycled']}", file=sys.stderr, flush=True)
    if not args.no_subcycle:
        line["subcycle"] = run_subcycle(P, torch, msh)
    if not args.no_grad:
        line["grad"] = run_grad_compare(P, torch)
    if not args.no_batch:
        line["batch"] = run_batch_compare(P, torch)
        print(f"# batch: {line['batch']}", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
