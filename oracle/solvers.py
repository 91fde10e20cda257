"""Krylov solvers and preconditioners of the oracle (TEST INFRASTRUCTURE ONLY).

Sec. 3 of the paper: the SIPDG systems are symmetric positive-definite, so
they are solved by preconditioned conjugate gradients; the screened Poisson
(Helmholtz) solve uses the element-wise scaled inverse mass matrix as
preconditioner; the Poisson solve uses a multigrid preconditioner whose fine
levels coarsen the polynomial degree (N -> ... -> 1) matrix-free, smoothed by a
degree-2 Chebyshev iteration.

Readings where the paper is silent (shared with the GPU library, each
implemented there independently):
  * PCG starts from x0 (default 0) and stops when ||r||_2 <= tol ||b||_2;
    the recurrence residual is replaced by the true residual b - A x before
    a stop is accepted.
  * When the preconditioner is not a fixed symmetric operator (the
    multigrid cycle with an inexact Krylov coarse solve) the flexible variant
    beta_k = -(z_{k+1}, A p_k) / (p_k, A p_k) is used (Notay 2000); for a fixed
    SPD preconditioner it equals the textbook (z_{k+1}, r_{k+1})/(z_k, r_k).
  * Level l of the p-multigrid hierarchy rediscretises the operator at degree
    N_l with penalty constant c_tau ((N_l+1)/(N_0+1))^2; prolongation P is the
    interpolation of the coarse Lagrange basis at the fine nodes, restriction
    is P^T.
  * Chebyshev smoothing acts on D^{-1} A (D = diag A) over
    [lo * rho, hi * rho] (default lo = 0.1, hi = 1.1), the semi-iteration of
    Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1; rho is an
    estimate of the largest eigenvalue of D^{-1} A passed in by the caller.
  * The same smoother runs before and after the coarse correction; the
    coarsest level is solved by Jacobi-PCG from zero to a relative residual
    coarse_tol or coarse_max iterations.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import assemble as asm
from .refelem import RefTriangle


class Breakdown(RuntimeError):
    pass


def pcg(A, b, precond=None, tol=1e-8, max_iters=10000, x0=None, flexible=False,
        keep_iterates=False):
    """Preconditioned CG on the SPD matrix (or callable) A.

    Returns (x, iters, relres, info) where relres is the true relative
    residual ||b - A x|| / ||b|| of the returned x, and info holds the
    recurrence residual history (and the iterates if requested)."""
    Aop = A if callable(A) else (lambda v: A @ v)
    B = precond if precond is not None else (lambda v: v.copy())
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = {"res": [], "iterates": []}
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0, info
    r = b - Aop(x)
    z = B(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while True:
        rn = np.linalg.norm(r)
        info["res"].append(rn / bnorm)
        if rn <= tol * bnorm:
            rt = b - Aop(x)
            if np.linalg.norm(rt) <= tol * bnorm or it >= max_iters:
                break
            r = rt                               # reliable restart
            z = B(r)
            p = z.copy()
            rz = r @ z
        if it >= max_iters:
            break
        Ap = Aop(p)
        pAp = p @ Ap
        if not (pAp > 0.0) or not np.isfinite(pAp):
            raise Breakdown(f"p^T A p = {pAp} at iteration {it}")
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        if keep_iterates:
            info["iterates"].append(x.copy())
        z = B(r)
        rz_new = r @ z
        if flexible:
            beta = -(z @ Ap) / pAp
        else:
            beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    relres = np.linalg.norm(b - Aop(x)) / bnorm
    return x, it, relres, info


def jacobi(A):
    d = A.diagonal()
    inv = 1.0 / d
    return lambda v: inv * v


def block_mass_inverse(m: "asm.OracleMesh"):
    """z_e = (J_e M)^{-1} r_e (Sec. 3, scaled inverse mass on each element)."""
    ref = m.ref
    Mref = (ref.qL * ref.qw[:, None]).T @ ref.qL
    Minv = np.linalg.inv(Mref)

    def apply(v):
        V = v.reshape(m.K, m.Np)
        return ((V @ Minv.T) / m.J[:, None]).ravel()

    return apply


def lanczos_rho(A, steps=20, seed=0):
    """Largest Ritz value of D^{-1} A after ``steps`` Jacobi-PCG (Lanczos)
    steps from a seeded N(0,1) right-hand side."""
    n = A.shape[0]
    b = np.random.default_rng(seed).standard_normal(n)
    dinv = 1.0 / A.diagonal()
    x = np.zeros(n)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(steps):
        Ap = A @ p
        a = rz / (p @ Ap)
        r = r - a * Ap
        z = dinv * r
        rz_new = r @ z
        bta = rz_new / rz
        alphas.append(a)
        betas.append(bta)
        p = z + bta * p
        rz = rz_new
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return float(np.linalg.eigvalsh(T).max())


def chebyshev(A, dinv, f, x0, lo, hi, degree):
    """Chebyshev semi-iteration (Saad Alg. 12.1) on D^{-1} A x = D^{-1} f over
    the eigenvalue interval [lo, hi], ``degree`` steps starting at x0."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(f) if x0 is None else x0.copy()
    r = f - A @ x if x0 is not None else f.copy()
    d = (dinv * r) / theta
    for k in range(degree):
        x = x + d
        if k + 1 == degree:
            break
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x


def interpolation(Nc: int, Nf: int) -> np.ndarray:
    """Np(Nf) x Np(Nc): coarse Lagrange basis evaluated at the fine nodes."""
    rc = RefTriangle(Nc)
    rf = RefTriangle(Nf)
    L, _, _ = rc.lagrange(rf.r, rf.s)
    return L


class PMG:
    """p-multigrid V-cycle on degrees ``degrees`` (fine first), Sec. 3."""

    def __init__(self, mesh, degrees, lam, ctau, rho, cheb_lo=0.1, cheb_hi=1.1,
                 cheb_degree=2, coarse_tol=1e-2, coarse_max=200, coarse_exact=False,
                 coarse_amg=False, amg_cycles=1, amg_coarse_size=1024, kappa=None, amg_kcycle_levels=2,
                 amg_top_krylov=False):
        self.degrees = list(degrees)
        N0 = self.degrees[0]
        self.levels = []
        for l, Nl in enumerate(self.degrees):
            m = asm.OracleMesh(mesh.VX, mesh.VY, mesh.EToV, mesh.EToB, Nl)
            ct = ctau * ((Nl + 1) / (N0 + 1)) ** 2
            A = asm.assemble(m, lam, ct, kappa=kappa)
            self.levels.append({"m": m, "A": A, "dinv": 1.0 / A.diagonal(), "ctau": ct})
        self.P = []
        for l in range(len(self.degrees) - 1):
            I = interpolation(self.degrees[l + 1], self.degrees[l])
            K = self.levels[l]["m"].K
            self.P.append(sp.kron(sp.identity(K, format="csr"), sp.csr_matrix(I), format="csr"))
        self.rho = list(rho)
        self.lo, self.hi, self.deg = cheb_lo, cheb_hi, cheb_degree
        self.coarse_tol, self.coarse_max = coarse_tol, coarse_max
        self.coarse_exact = coarse_exact
        self.coarse_iters = []
        self.amg = None
        self.amg_cycles = amg_cycles
        # the degree-1 level solved by the K-cycle's two flexible-CG steps on
        # it, each preconditioned by one AMG cycle, instead of plain cycles
        self.amg_top_krylov = amg_top_krylov
        if coarse_amg:
            # the algebraic levels below the degree-1 level (pMG-AMG, Sec. 3)
            from .amg import AMG
            L = self.levels[-1]
            self.amg = AMG(L["m"], L["A"], self.rho[-1], cheb_lo, cheb_hi, cheb_degree,
                           coarse_size=amg_coarse_size, kcycle_levels=amg_kcycle_levels)

    def smooth(self, l, f, x0):
        L = self.levels[l]
        return chebyshev(L["A"], L["dinv"], f, x0, self.lo * self.rho[l], self.hi * self.rho[l], self.deg)

    def vcycle(self, l, r):
        L = self.levels[l]
        if l == len(self.levels) - 1:
            if self.amg is not None:
                if self.amg_top_krylov:
                    return self.amg.krylov_correction(0, r)
                return self.amg.solve(r, self.amg_cycles)
            if self.coarse_exact:
                import scipy.sparse.linalg as spla
                return spla.spsolve(L["A"].tocsc(), r)
            x, it, _, _ = pcg(L["A"], r, precond=jacobi(L["A"]), tol=self.coarse_tol,
                              max_iters=self.coarse_max)
            self.coarse_iters.append(it)
            return x
        z = self.smooth(l, r, None)
        res = r - L["A"] @ z
        zc = self.vcycle(l + 1, self.P[l].T @ res)
        z = z + self.P[l] @ zc
        return self.smooth(l, r, z)

    def __call__(self, r):
        return self.vcycle(0, r)
