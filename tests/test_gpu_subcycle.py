"""GPU parity of the subcycling advection (Sec. 2.3, Eq. SS_3 and INS_CUB_N;
Sec. 5.3, Eq. KSS_3, Alg. SSV and SSS) against the oracle, through the C ABI:
the volume term, the surface term and both, for every degree and a mix of
boundary rules on meshes of several 16-element wave tiles with a ragged tail;
the five-stage Runge-Kutta subcycle with an advecting field and Dirichlet data
linear in time; exact translation of a polynomial on a larger mesh; and the
operator at the benchmark's size (524,288 triangles) on sampled elements
(the oracle computes those rows one by one) and through a property that holds
at any size (exact advection of a polynomial by a linear divergence-free
field)."""
import numpy as np
import pytest

import synth
from oracle.assemble import OracleMesh
from oracle.subcycle import advection_operator, subcycle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1801_00246_amd")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_operator_matches_oracle(N):
    # 7 x 7 squares: 98 triangles = 6 full 16-element tiles and a tail of 2
    msh = synth.permuted(synth.square_mesh(7, jitter=0.2, seed=60 + N, bc="mixed"), seed=61 + N)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    rng = np.random.default_rng(N)
    n = m.K * m.Np
    ub, vb, u, v, gu, gv = (rng.standard_normal(n) for _ in range(6))
    g = P.Mesh.from_synth(N, msh)
    errs = []
    for parts in (1, 2, 3):
        nu, nv = g.subcycle_rhs(dev(ub), dev(vb), dev(u), dev(v), dev(gu), dev(gv), parts=parts)
        ou, ov = advection_operator(m, ub, vb, u, v, gu, gv, parts=parts)
        errs += [rel(host(nu), ou), rel(host(nv), ov)]
    nu, nv = g.subcycle_rhs(dev(ub), dev(vb), dev(u), dev(v))
    ou, ov = advection_operator(m, ub, vb, u, v)
    errs += [rel(host(nu), ou), rel(host(nv), ov)]
    print(f"N={N}: rel errors volume {errs[0]:.1e} {errs[1]:.1e}, surface {errs[2]:.1e} {errs[3]:.1e}, "
          f"both {errs[4]:.1e} {errs[5]:.1e}, zero data {errs[6]:.1e} {errs[7]:.1e}")
    assert max(errs) <= 1e-12
    g.close()


@pytest.mark.parametrize("N", [2, 5])
def test_subcycle_matches_oracle(N):
    msh = synth.permuted(synth.square_mesh(5, jitter=0.2, seed=70 + N, bc="mixed"), seed=71 + N)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = (c.ravel() for c in m.node_coords())
    rng = np.random.default_rng(72)
    n = m.K * m.Np
    # a smooth advecting field with a rate, smooth data with a rate, rough U~
    ub0, vb0 = 0.6 + 0.2 * np.sin(3 * y), -0.3 + 0.2 * np.cos(2 * x)
    ub1, vb1 = 0.1 * np.cos(x), 0.1 * np.sin(y)
    gu0, gv0 = np.sin(x + y), np.cos(x - y)
    gu1, gv1 = 0.2 * x, -0.1 * y
    u0, v0 = (rng.standard_normal(n) for _ in range(2))
    T, Ns = 0.02, 3
    ou, ov = subcycle(m, ub0, vb0, u0, v0, T, Ns, ub1, vb1, gu0, gv0, gu1, gv1)
    g = P.Mesh.from_synth(N, msh)
    gu_, gv_ = g.subcycle(dev(ub0), dev(vb0), dev(u0), dev(v0), T, Ns, dev(ub1), dev(vb1), dev(gu0), dev(gv0),
                          dev(gu1), dev(gv1))
    e = (rel(host(gu_), ou), rel(host(gv_), ov))
    print(f"N={N}: subcycle rel errors {e[0]:.1e} {e[1]:.1e}")
    assert max(e) <= 1e-12
    # constant advecting field and no data (the optional fields absent)
    ou, ov = subcycle(m, ub0, vb0, u0, v0, T, 2)
    gu_, gv_ = g.subcycle(dev(ub0), dev(vb0), dev(u0), dev(v0), T, 2)
    assert max(rel(host(gu_), ou), rel(host(gv_), ov)) <= 1e-12
    g.close()


def poly(x, y, N, seed):
    c = np.random.default_rng(seed).standard_normal((N + 1, N + 1))
    f = np.zeros_like(x)
    fx = np.zeros_like(x)
    fy = np.zeros_like(x)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f += c[a, b] * x ** a * y ** b
            if a:
                fx += c[a, b] * a * x ** (a - 1) * y ** b
            if b:
                fy += c[a, b] * b * x ** a * y ** (b - 1)
    return f, fx, fy


def test_subcycle_translates_a_polynomial_exactly():
    N = 4
    msh = synth.permuted(synth.square_mesh(48, jitter=0.2, seed=80, bc="neumann"), seed=81)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    a, b = 0.7, -0.4
    u0, _, _ = poly(x, y, N, seed=82)
    v0, _, _ = poly(x, y, N, seed=83)
    T, Ns = 0.01, 4                       # inside the stability region at h = 1/48
    g = P.Mesh.from_synth(N, msh)
    one = np.ones(x.size)
    U, V = g.subcycle(dev(a * one), dev(b * one), dev(u0.ravel()), dev(v0.ravel()), T, Ns)
    eu, _, _ = poly(x - a * T, y - b * T, N, seed=82)
    ev, _, _ = poly(x - a * T, y - b * T, N, seed=83)
    e = (rel(host(U), eu.ravel()), rel(host(V), ev.ravel()))
    print(f"K={m.K}: translation rel errors {e[0]:.1e} {e[1]:.1e}")
    assert max(e) <= 1e-11
    g.close()


@pytest.mark.parametrize("N", [3, 5, 7])
def test_operator_at_full_size(N):
    msh = synth.ax_sweep_mesh(512, seed=0)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    rng = np.random.default_rng(90 + N)
    n = m.K * m.Np
    g = P.Mesh.from_synth(N, msh)
    # sampled rows against the oracle, random fields
    ub, vb, u, v, gd = (rng.standard_normal(n) for _ in range(5))
    nu, nv = g.subcycle_rhs(dev(ub), dev(vb), dev(u), dev(v), dev(gd), dev(-gd))
    E = np.sort(rng.choice(m.K, 64, replace=False))
    E = np.concatenate([[0, m.K - 1], E])
    ou, ov = advection_operator(m, ub, vb, u, v, gd, -gd, elems=E)
    rows = (E[:, None] * m.Np + np.arange(m.Np)[None, :]).ravel()
    hu, hv = host(nu), host(nv)
    e = (rel(hu[rows], ou), rel(hv[rows], ov))
    # property: a linear divergence-free field advects a degree-N polynomial
    # exactly (Dirichlet data = the polynomial)
    c = np.random.default_rng(91).standard_normal(5)
    ubl, vbl = c[0] + c[1] * x + c[2] * y, c[3] + c[4] * x - c[1] * y
    p, px, py = poly(x, y, N, seed=92)
    q, qx, qy = poly(x, y, N, seed=93)
    nu, nv = g.subcycle_rhs(dev(ubl.ravel()), dev(vbl.ravel()), dev(p.ravel()), dev(q.ravel()), dev(p.ravel()),
                            dev(q.ravel()))
    eu, ev = (ubl * px + vbl * py).ravel(), (ubl * qx + vbl * qy).ravel()
    e2 = (rel(host(nu), eu), rel(host(nv), ev))
    print(f"N={N} K={m.K}: sampled rel errors {e[0]:.1e} {e[1]:.1e}; polynomial {e2[0]:.1e} {e2[1]:.1e}")
    assert max(e) <= 1e-12
    # rounding of the nodal data is amplified by the operator's norm, about
    # N^2 / h (h = 1 / 512): allow 5e-14 N^2 / h relative (measured 1.0-1.1e-14)
    assert max(e2) <= 5e-14 * N * N * 512
    g.close()


def test_errors():
    msh = synth.square_mesh(3)
    g = P.Mesh.from_synth(3, msh)
    z = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(P.IpdgError):
        g.subcycle_rhs(z, z, z, z, parts=0)
    with pytest.raises(P.IpdgError):
        g.subcycle(z, z, z, z, 0.1, 0)
    with pytest.raises(P.IpdgError):
        g.subcycle(z, z, z, z, float("nan"), 2)
    g.close()


def test_single_element_and_empty_mesh():
    # one triangle: one wave whose other 15 columns read the same element and
    # store nothing; Dirichlet and Neumann faces
    VX = np.array([0.0, 1.0, 0.2])
    VY = np.array([0.0, 0.1, 0.9])
    EToV = np.array([[0, 1, 2]])
    EToB = np.array([[P.BC_DIRICHLET, P.BC_NEUMANN, P.BC_DIRICHLET]], np.int8)
    for N in (1, 8):
        m = OracleMesh(VX, VY, EToV, EToB, N)
        rng = np.random.default_rng(N)
        ub, vb, u, v, gu, gv = (rng.standard_normal(m.Np) for _ in range(6))
        g = P.Mesh(N, VX, VY, EToV, EToB)
        nu, nv = g.subcycle_rhs(dev(ub), dev(vb), dev(u), dev(v), dev(gu), dev(gv))
        ou, ov = advection_operator(m, ub, vb, u, v, gu, gv)
        assert max(rel(host(nu), ou), rel(host(nv), ov)) <= 1e-12
        su, sv = g.subcycle(dev(ub), dev(vb), dev(u), dev(v), 1e-3, 3, gu0=dev(gu), gv0=dev(gv))
        tu, tv = subcycle(m, ub, vb, u, v, 1e-3, 3, gu0=gu, gv0=gv)
        assert max(rel(host(su), tu), rel(host(sv), tv)) <= 1e-12
        g.close()
    # an empty mesh: both calls are no-ops
    g0 = P.Mesh(3, np.zeros(0), np.zeros(0), np.zeros((0, 3), np.int32), np.zeros((0, 3), np.int8))
    assert g0.K == 0
    P.ipdg.check(P.lib().ipdg_subcycle_rhs(g0.handle, None, None, None, None, None, None, 3, None, None, None))
    P.ipdg.check(P.lib().ipdg_subcycle(g0.handle, None, None, None, None, None, None, None, None, 0.1, 2, None, None,
                                       None))
    # a vector of the wrong length is refused by the binding
    msh = synth.square_mesh(3)
    g = P.Mesh.from_synth(2, msh)
    z = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        g.subcycle_rhs(z[:-1], z, z, z)
    g.close()
