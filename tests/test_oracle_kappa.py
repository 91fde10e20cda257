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


def two_material_problem(n, N, k1, k2):
    """n x n unjittered squares (n even, so x = 1/2 is a mesh line), kappa =
    k1 left of x = 1/2 and k2 right of it, Dirichlet faces on x = 0 and
    x = 1, Neumann faces on y = 0 and y = 1; u continuous, piecewise linear
    in x with the continuous flux kappa du/dx = 1."""
    msh = synth.square_mesh(n, bc="dirichlet")
    EToB = msh.EToB.copy()
    for f in range(3):
        a, b = msh.EToV[:, f], msh.EToV[:, (f + 1) % 3]
        horiz = np.abs(msh.VY[a] - msh.VY[b]) < 1e-14
        EToB[(EToB[:, f] != 0) & horiz, f] = 2
    msh = synth.Mesh(msh.VX, msh.VY, msh.EToV, EToB, n=n)
    m = omesh(msh, N)
    cx = msh.VX[msh.EToV].mean(1)
    kap = np.where(cx < 0.5, k1, k2)
    x, _ = m.node_coords()
    left = (cx < 0.5)[:, None]
    u = np.where(left, x / k1, 0.5 / k1 + (x - 0.5) / k2).ravel()
    inner = ~(m.EToB == 1).any(1)          # elements without a Dirichlet face
    return m, kap, u, inner


@pytest.mark.parametrize("N", [1, 2, 4])
def test_kappa_flux_continuity_closed_form(N):
    """For u with a continuous flux kappa grad u and no jump, the kappa-weighted
    form reduces, on every element without a Dirichlet face, to the volume
    flux balance, which vanishes: (A u)_i = lambda (M u)_i.  This pins the
    flux average {kappa d_n u} (an average of kappa times an average of
    d_n u would leave a residual at x = 1/2)."""
    from oracle.matfree import MatFree
    m, kap, u, inner = two_material_problem(8, N, 1.0, 5.0)
    rows = np.repeat(inner, m.Np)
    for lam in (0.0, 3.0):
        A = assemble(m, lam, 16.0, kappa=kap)
        Au = A @ u
        Mu = (mass_matrix(m) @ u)
        scale = (abs(A) @ np.abs(u)).max()
        assert np.abs(Au - lam * Mu)[rows].max() <= 1e-12 * scale
        y = MatFree(m).apply(lam, 16.0, u, kappa=kap)
        assert np.abs(y - lam * Mu)[rows].max() <= 1e-12 * scale
    # the check is sensitive: u = x (a flux jump of 4 at x = 1/2) leaves a
    # residual on the rows of the elements at the interface
    x, _ = m.node_coords()
    A = assemble(m, 0.0, 16.0, kappa=kap)
    r = (A @ x.ravel()).reshape(m.K, m.Np)
    cx = m.VX[m.EToV].mean(1)
    at = np.abs(cx - 0.5) < 1.0 / 8
    assert np.abs(r[at & inner]).max() > 1e-6 * (abs(A) @ np.abs(x.ravel())).max()
