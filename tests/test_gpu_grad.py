"""GPU parity of the differentiable solve: the per-element coefficient
gradient kernel against the oracle's, the autograd gradients against the
oracle's FP64 adjoint, and against central finite differences of the GPU
solve itself (FP64 and mixed precision)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.assemble import OracleMesh, assemble, kappa_grad, mass_matrix

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1801_00246_amd")
from paper_1801_00246_amd.autograd import helmholtz_solve, mass  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("N,bc", [(1, "dirichlet"), (3, "mixed"), (5, "dirichlet"), (8, "mixed")])
def test_kappa_grad_kernel_matches_oracle(N, bc):
    msh = synth.permuted(synth.square_mesh(17, jitter=0.2, seed=N, bc=bc), seed=N)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    kap = synth.kappa_draw(msh.K, seed=2)
    u = synth.nodal_normal(msh.K, m.Np, 11)
    w = synth.nodal_normal(msh.K, m.Np, 12)
    go = kappa_grad(m, float((N + 1) ** 2), kap, u, w)
    g = P.Mesh.from_synth(N, msh, kappa=kap)
    gg = host(g.kappa_grad(dev(u), dev(w)))
    assert np.linalg.norm(gg - go) <= 1e-11 * np.linalg.norm(go)


def setup_problem(n=10, N=3, seed=0):
    msh = synth.square_mesh(n, jitter=0.2, seed=seed)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    kap = synth.kappa_draw(msh.K, seed=2)
    f = synth.nodal_normal(msh.K, m.Np, seed=5)
    x, y = m.node_coords()
    ut = synth.smooth_field(x.ravel(), y.ravel(), synth.smooth_coeffs(seed=3))
    return msh, m, kap, f, ut


def oracle_grads(m, kap, f, ut, lam, ctau):
    A = assemble(m, lam, ctau, kappa=kap).tocsc()
    M = mass_matrix(m)
    u = spla.spsolve(A, M @ f)
    w = spla.spsolve(A, 2 * (M @ (u - ut)))
    return kappa_grad(m, ctau, kap, u, w), M @ w


def gpu_loss(g, kap_t, f_t, ut_t, lam, tol, opts):
    u = helmholtz_solve(f_t, kap_t, g, lam=lam, tol=tol, opts=opts)
    d = u - ut_t
    return torch.dot(d, mass(d, g))


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_MIXED] if P else [])
def test_autograd_matches_oracle_adjoint(prec):
    msh, m, kap, f, ut = setup_problem()
    lam, ctau = 1.0, 16.0
    gk_o, gf_o = oracle_grads(m, kap, f, ut, lam, ctau)
    g = P.Mesh.from_synth(3, msh)
    kap_t = dev(kap).requires_grad_(True)
    f_t = dev(f).requires_grad_(True)
    opts = P.default_opts(pc=P.PC_BLOCK_MASS, prec=prec)
    L = gpu_loss(g, kap_t, f_t, dev(ut), lam, 1e-12 if prec == P.PREC_FP64 else 1e-10, opts)
    L.backward()
    ek = np.linalg.norm(host(kap_t.grad) - gk_o) / np.linalg.norm(gk_o)
    ef = np.linalg.norm(host(f_t.grad) - gf_o) / np.linalg.norm(gf_o)
    print(f"prec={prec}: dL/dkappa rel err {ek:.2e}, dL/df rel err {ef:.2e}")
    bound = 1e-8 if prec == P.PREC_FP64 else 1e-6
    assert ek <= bound and ef <= bound


def test_autograd_matches_central_differences():
    msh, m, kap, f, ut = setup_problem(n=8, N=4, seed=1)
    g = P.Mesh.from_synth(4, msh)
    opts = P.default_opts(pc=P.PC_BLOCK_MASS)
    lam, tol = 1.0, 1e-12
    kap_t = dev(kap).requires_grad_(True)
    f_t = dev(f).requires_grad_(True)
    ut_t = dev(ut)
    L = gpu_loss(g, kap_t, f_t, ut_t, lam, tol, opts)
    L.backward()
    gk = host(kap_t.grad)
    gf = host(f_t.grad)
    h = 1e-6
    rng = np.random.default_rng(8)
    with torch.no_grad():
        for d in [np.eye(msh.K)[3], rng.standard_normal(msh.K), rng.standard_normal(msh.K)]:
            Lp = float(gpu_loss(g, dev(kap + h * d), dev(f), ut_t, lam, tol, opts))
            Lm = float(gpu_loss(g, dev(kap - h * d), dev(f), ut_t, lam, tol, opts))
            fd = (Lp - Lm) / (2 * h)
            assert gk @ d == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(float(L)))
        df = rng.standard_normal(f.size)
        Lp = float(gpu_loss(g, dev(kap), dev(f + h * df), ut_t, lam, tol, opts))
        Lm = float(gpu_loss(g, dev(kap), dev(f - h * df), ut_t, lam, tol, opts))
        assert gf @ df == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5)


def test_kappa_grad_on_a_plain_mesh_leaves_it_plain():
    """The coefficient gradient of a mesh without coefficient is taken at
    kappa = 1 and does not turn the mesh into a coefficient mesh."""
    N = 3
    msh = synth.square_mesh(9, jitter=0.2, seed=41)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    u = synth.nodal_normal(msh.K, m.Np, 42)
    w = synth.nodal_normal(msh.K, m.Np, 43)
    go = kappa_grad(m, float((N + 1) ** 2), np.ones(msh.K), u, w)
    g = P.Mesh.from_synth(N, msh)
    y0 = host(g.apply(dev(u), lam=2.0))
    gg = host(g.kappa_grad(dev(u), dev(w)))
    assert np.linalg.norm(gg - go) <= 1e-11 * np.linalg.norm(go)
    y1 = host(g.apply(dev(u), lam=2.0))
    assert np.array_equal(y0, y1)
