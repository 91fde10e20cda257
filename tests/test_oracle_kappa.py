"""Pins of the oracle's kappa-weighted operator and of its coefficient
gradient (the differentiable Helmholtz solve): closed forms, scaling and
central finite differences of the oracle's own solve."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.assemble import OracleMesh, assemble, kappa_grad, mass_apply, mass_matrix


def omesh(msh, N):
    return OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)


def test_constant_kappa_scales_the_laplacian():
    msh = synth.square_mesh(4, jitter=0.2, seed=1, bc="mixed")
    m = omesh(msh, 3)
    A1 = assemble(m, 0.0, 16.0)
    Ac = assemble(m, 0.0, 16.0, kappa=np.full(msh.K, 2.5))
    assert abs(Ac - 2.5 * A1).max() < 1e-12 * abs(A1).max()
    A1l = assemble(m, 7.0, 16.0, kappa=np.ones(msh.K))
    assert abs(A1l - assemble(m, 7.0, 16.0)).max() == 0.0


def test_kappa_penalty_closed_form():
    """1_e^T A 1_e = sum over interior faces of c_tau max(k_e |F|/|E|,
    k_nb |F|/|E_nb|) |F| (all-Neumann boundary, lambda = 0)."""
    msh = synth.square_mesh(3, jitter=0.25, seed=2, bc="neumann")
    N = 2
    m = omesh(msh, N)
    kap = synth.kappa_draw(msh.K, seed=3)
    ctau = 4.0
    A = assemble(m, 0.0, ctau, kappa=kap)
    Np = m.Np
    for e in range(msh.K):
        exp = 0.0
        for f in range(3):
            nb = m.EToE[e, f]
            if nb < 0:
                continue
            L = m.face_geometry(np.array([e]), f)[4][0]
            exp += ctau * max(kap[e] * L / m.area[e], kap[nb] * L / m.area[nb]) * L
        v = np.zeros(msh.K * Np)
        v[e * Np:(e + 1) * Np] = 1
        assert v @ A @ v == pytest.approx(exp, rel=1e-12)


def loss_and_grads(m, lam, ctau, kap, f, ut):
    A = assemble(m, lam, ctau, kappa=kap).tocsc()
    M = mass_matrix(m)
    b = M @ f
    u = spla.spsolve(A, b)
    d = u - ut
    L = d @ (M @ d)
    w = spla.spsolve(A, 2 * (M @ d))
    return L, kappa_grad(m, ctau, kap, u, w), M @ w


@pytest.mark.parametrize("bc", ["dirichlet", "mixed"])
def test_kappa_gradient_matches_central_differences(bc):
    N = 3
    msh = synth.square_mesh(4, jitter=0.2, seed=4, bc=bc)
    m = omesh(msh, N)
    kap = synth.kappa_draw(msh.K, seed=2)
    f = synth.nodal_normal(msh.K, m.Np, seed=5)
    x, y = m.node_coords()
    ut = synth.smooth_field(x.ravel(), y.ravel(), synth.smooth_coeffs(seed=3))
    lam, ctau = 1.0, 16.0
    L0, gk, gf = loss_and_grads(m, lam, ctau, kap, f, ut)
    h = 1e-6
    rng = np.random.default_rng(0)
    dirs = [np.eye(msh.K)[k] for k in (0, 7, 19)] + [rng.standard_normal(msh.K) for _ in range(3)]
    for d in dirs:
        Lp = loss_and_grads(m, lam, ctau, kap + h * d, f, ut)[0]
        Lm = loss_and_grads(m, lam, ctau, kap - h * d, f, ut)[0]
        fd = (Lp - Lm) / (2 * h)
        assert gk @ d == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(L0))
    df = rng.standard_normal(f.size)
    Lp = loss_and_grads(m, lam, ctau, kap, f + h * df, ut)[0]
    Lm = loss_and_grads(m, lam, ctau, kap, f - h * df, ut)[0]
    assert gf @ df == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5)
