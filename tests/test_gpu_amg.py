"""GPU parity of the algebraic levels below degree 1 (pMG-AMG, Sec. 3)
against the oracle's aggregation AMG (V-cycle, and K-cycle on the finest
levels), through the C ABI.

The hierarchy sizes must equal the oracle's (the aggregation depends on the
element graph only); one preconditioner application (a p-multigrid V-cycle
whose degree-1 level runs AMG cycles) is compared element by element with
the oracle's, given the same spectral estimates of the p-levels (1e-11 in
FP64, the FP32 error printed and bounded); PCG solves reach the oracle's
tolerance under the oracle's matrix with the oracle's iteration count.
"""
import numpy as np
import pytest

import synth
from oracle import solvers as S
from oracle.assemble import OracleMesh, assemble, mass_apply

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1801_00246_amd")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def amg_opts(degrees, rho, cs, cycles=1, prec=None, kcyc=2, **kw):
    return P.default_opts(pc=P.PC_PMG, prec=P.PREC_FP64 if prec is None else prec, degrees=list(degrees),
                          rho=list(rho), coarse_amg=1, amg_coarse_size=cs, amg_cycles=cycles,
                          amg_kcycle_levels=kcyc, **kw)


CASES = [
    # n, degrees, bc, lambda, kappa, coarse size, cycles
    (12, (3, 1), "dirichlet", 2.0, False, 16, 1),
    (20, (2, 1), "mixed", 0.5, True, 32, 2),
    (30, (4, 2, 1), "neumann", 1.0, False, 64, 1),
    (9, (1,), "dirichlet", 10.0, False, 8, 1),
]


@pytest.mark.parametrize("kcyc", [0, 2, 3], ids=["vcycle", "kcycle2", "kcycle3"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}-{'-'.join(map(str, c[1]))}-{c[2]}")
def test_amg_cycle_matches_oracle(case, kcyc):
    n, degrees, bc, lam, use_kappa, cs, cycles = case
    N = degrees[0]
    msh = synth.permuted(synth.square_mesh(n, jitter=0.2, seed=11, bc=bc), seed=12)
    kv = synth.kappa_draw(msh.K, seed=13) if use_kappa else None
    ctau = float((N + 1) ** 2)
    rho = [1.7 + 0.1 * l for l in range(len(degrees))]
    B = S.PMG(msh, degrees, lam, ctau, rho, coarse_amg=True, amg_cycles=cycles, amg_coarse_size=cs, kappa=kv,
              amg_kcycle_levels=kcyc)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    r = synth.nodal_normal(msh.K, m.Np, seed=14)
    zo = B(r)
    g = P.Mesh.from_synth(N, msh, kappa=kv)
    z, info = g.precond(dev(r), lam=lam, tau=ctau, opts=amg_opts(degrees, rho, cs, cycles, kcyc=kcyc))
    rel = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
    z32, _ = g.precond(dev(r), lam=lam, tau=ctau,
                       opts=amg_opts(degrees, rho, cs, cycles, prec=P.PREC_MIXED, kcyc=kcyc))
    rel32 = np.linalg.norm(host(z32) - zo) / np.linalg.norm(zo)
    print(f"K={msh.K} levels {info['amg_sizes']} (oracle {B.amg.sizes}): FP64 rel {rel:.2e}, FP32 rel {rel32:.2e}")
    assert info["amg_sizes"] == B.amg.sizes
    assert len(B.amg.sizes) >= 3
    assert rel <= 1e-11
    assert rel32 <= 1e-4
    g.close()


@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"n{c[0]}-{'-'.join(map(str, c[1]))}-{c[2]}")
def test_amg_top_krylov_matches_oracle(case):
    """The degree-1 level solved by two flexible-CG steps, each preconditioned
    by one AMG cycle (K-cycle on two levels below)."""
    n, degrees, bc, lam, use_kappa, cs, _ = case
    N = degrees[0]
    msh = synth.permuted(synth.square_mesh(n, jitter=0.2, seed=11, bc=bc), seed=12)
    kv = synth.kappa_draw(msh.K, seed=13) if use_kappa else None
    ctau = float((N + 1) ** 2)
    rho = [1.7 + 0.1 * l for l in range(len(degrees))]
    B = S.PMG(msh, degrees, lam, ctau, rho, coarse_amg=True, amg_coarse_size=cs, kappa=kv, amg_top_krylov=True)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    r = synth.nodal_normal(msh.K, m.Np, seed=14)
    zo = B(r)
    g = P.Mesh.from_synth(N, msh, kappa=kv)
    z, info = g.precond(dev(r), lam=lam, tau=ctau, opts=amg_opts(degrees, rho, cs, amg_top_krylov=1))
    rel = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
    z32, _ = g.precond(dev(r), lam=lam, tau=ctau, opts=amg_opts(degrees, rho, cs, prec=P.PREC_MIXED, amg_top_krylov=1))
    rel32 = np.linalg.norm(host(z32) - zo) / np.linalg.norm(zo)
    print(f"K={msh.K} top Krylov: FP64 rel {rel:.2e}, FP32 rel {rel32:.2e}")
    assert rel <= 1e-11
    assert rel32 <= 1e-4
    g.close()


@pytest.mark.parametrize("kcyc", [0, 2])
def test_amg_cycle_large_mesh_matches_oracle(kcyc):
    """182 x 182 jittered squares, permuted (66,248 triangles), degrees 2 -> 1
    and the default coarse size: four algebraic levels below degree 1."""
    degrees = (2, 1)
    msh = synth.permuted(synth.square_mesh(182, jitter=0.2, seed=4), seed=5)
    ctau, lam, rho = 9.0, 2.0, [1.8, 1.6]
    B = S.PMG(msh, degrees, lam, ctau, rho, coarse_amg=True, amg_coarse_size=512, amg_kcycle_levels=kcyc)
    r = synth.nodal_normal(msh.K, 6, seed=9)
    zo = B(r)
    g = P.Mesh.from_synth(2, msh)
    z, info = g.precond(dev(r), lam=lam, tau=ctau, opts=amg_opts(degrees, rho, 512, kcyc=kcyc))
    rel = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
    print(f"K={msh.K} kcycle {kcyc} levels {info['amg_sizes']}: FP64 rel {rel:.2e}")
    assert info["amg_sizes"] == B.amg.sizes
    assert rel <= 1e-11
    g.close()


@pytest.mark.parametrize("top", [0, 1], ids=["cycle", "top_krylov"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pcg_with_amg_coarse_levels(prec, top):
    """p-multigrid 5 -> 2 -> 1 with the algebraic levels: the true residual
    under the oracle's matrix and the oracle's PCG iteration count."""
    msh = synth.square_mesh(24, jitter=0.15, seed=21)
    N, lam = 5, 1.0
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    ctau = 36.0
    A = assemble(m, lam, ctau)
    b = mass_apply(m, synth.nodal_normal(msh.K, m.Np, seed=22))
    degrees = (5, 2, 1)
    rho = []
    for l, Nl in enumerate(degrees):
        ml = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, Nl)
        rho.append(S.lanczos_rho(assemble(ml, lam, ctau * ((Nl + 1) / (N + 1)) ** 2)))
    B = S.PMG(msh, degrees, lam, ctau, rho, coarse_amg=True, amg_coarse_size=64,   # K-cycle on two levels
              amg_top_krylov=bool(top))
    _, it_o, rel_o, _ = S.pcg(A, b, B, tol=1e-8, flexible=True)
    g = P.Mesh.from_synth(N, msh)
    pr = P.PREC_FP64 if prec == "fp64" else P.PREC_MIXED
    x, info, st = g.pcg(dev(b), lam=lam, tau=ctau, tol=1e-8, opts=amg_opts(degrees, rho, 64, prec=pr,
                                                                              amg_top_krylov=top))
    xh = host(x)
    rr = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    print(f"{prec}: {info['iters']} iterations (oracle {it_o}), true relres {rr:.2e}, levels {info['amg_sizes']}, "
          f"preconditioner {info['precond_bytes'] / msh.K:.0f} B per element")
    assert info["precond_bytes"] > 0
    assert st == 0
    assert rr <= 1e-8
    assert abs(info["iters"] - it_o) <= 1
    g.close()


def test_batch_with_amg_coarse_levels():
    """A batch with the algebraic levels keeps per-solve launches and
    converges every solve."""
    draws = [(10, 3, 1.0), (14, 5, 30.0), (9, 4, 300.0)]
    o = P.default_opts(pc=P.PC_PMG, coarse_amg=1, amg_coarse_size=32)
    meshes, bs, As, lams = [], [], [], []
    for i, (n, N, lam) in enumerate(draws):
        msh = synth.square_mesh(n, jitter=0.1, seed=30 + i)
        m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        b = mass_apply(m, synth.nodal_normal(msh.K, m.Np, seed=40 + i))
        As.append(assemble(m, lam, float((N + 1) ** 2)))
        meshes.append(P.Mesh.from_synth(N, msh))
        bs.append(dev(b))
        lams.append(lam)
    xs, iters, rel, st = P.solve_batch(meshes, lams, bs, tol=1e-8, opts=o)
    assert st == 0
    for A, b, x in zip(As, bs, xs):
        hb = host(b)
        assert np.linalg.norm(hb - A @ host(x)) <= 1e-8 * np.linalg.norm(hb)
    for g in meshes:
        g.close()


def test_amg_option_errors():
    msh = synth.square_mesh(6)
    g = P.Mesh.from_synth(4, msh)
    b = dev(np.ones(msh.K * g.Np))
    with pytest.raises(P.IpdgError):   # the last p-level must be degree 1
        g.pcg(b, opts=P.default_opts(pc=P.PC_PMG, degrees=[4, 2], coarse_amg=1))
    with pytest.raises(P.IpdgError):
        g.pcg(b, opts=P.default_opts(pc=P.PC_PMG, coarse_amg=1, amg_coarse_size=0))
    with pytest.raises(P.IpdgError):
        g.pcg(b, opts=P.default_opts(pc=P.PC_PMG, coarse_amg=1, amg_cycles=0))
    with pytest.raises(P.IpdgError):
        g.pcg(b, opts=P.default_opts(pc=P.PC_PMG, coarse_amg=1, amg_kcycle_levels=-1))
    with pytest.raises(P.IpdgError):
        g.pcg(b, opts=P.default_opts(pc=P.PC_PMG, coarse_amg=1, amg_top_krylov=1, amg_cycles=2))
    g.close()
    # pure Neumann with lambda = 0: the coarsest algebraic level is singular
    msh = synth.square_mesh(6, bc="neumann")
    g = P.Mesh.from_synth(2, msh)
    with pytest.raises(P.IpdgError):
        g.pcg(dev(np.ones(msh.K * g.Np)), lam=0.0, opts=P.default_opts(pc=P.PC_PMG, coarse_amg=1))
    g.close()
