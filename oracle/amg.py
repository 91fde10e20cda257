"""Aggregation algebraic multigrid of the oracle for the degree-1 level
(TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg).

Sec. 3 (the pMG-AMG hybrid): below degree 1 the multigrid continues with
algebraic levels built from unsmoothed aggregates of maximal independent node
sets, smoothed by a degree-2 Chebyshev iteration.  Readings where the paper
is silent (each implemented independently in the GPU library):
  * The first coarsening merges the nodal values of each element: P_0 maps
    one value per element to all its nodes (degree 1 -> piecewise constant).
  * Further levels aggregate the graph of the current level, whose edges are
    the shared faces on the element level and, above it, the union of the
    members' edges.  Pass 1 visits the nodes in index order; a free node whose
    neighbours are all free starts an aggregate holding it and them.  Pass 2
    puts every node still free into the aggregate that pass 1 gave to its
    lowest-index aggregated neighbour (there is one: that neighbour is why
    the node did not start an aggregate).  Aggregates are numbered in order
    of creation.
    The choices depend on the graph only, never on matrix values.
  * Coarse operators are Galerkin products A_{l+1} = P_l^T A_l P_l, with P_l
    the 0/1 aggregate map (unsmoothed aggregation).
  * Levels are added while more than ``coarse_size`` unknowns remain; the
    coarsest system is solved exactly.
  * Smoothing: Chebyshev of degree ``cheb_degree`` on D^{-1} A over
    [lo rho, hi rho]; on the algebraic levels rho is the Gershgorin bound
    max_i sum_j |A_ij| / A_ii, on the degree-1 level it is given.
  * One cycle starts from a zero initial guess, with the same smoother
    before and after the coarse correction.  On the first ``kcycle_levels``
    levels (the paper's K-cycle on the two finest levels, default 2) the
    coarse correction is two steps of flexible CG on the next level,
    preconditioned by that level's cycle (Notay and Vassilevski's K-cycle,
    with their early exit: one step only when it already reduced the coarse
    residual norm to ``kcycle_t`` = 0.25 of its start or less); where the next
    level is the coarsest it is solved exactly instead.  Below them the
    cycle is a V-cycle (``vcycle`` is the V-cycle on every level).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .solvers import chebyshev


def element_graph(m):
    """Adjacency lists of the elements through interior faces."""
    return [sorted(int(n) for n in m.EToE[e] if n >= 0 and n != e) for e in range(m.K)]


def aggregate(adj):
    """Greedy aggregation of a graph given as adjacency lists (see the
    module notes).  Returns (agg, n_aggregates)."""
    n = len(adj)
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j in adj[i]):
            agg[i] = na
            for j in adj[i]:
                agg[j] = na
            na += 1
    first = agg.copy()
    for i in range(n):
        if agg[i] < 0:
            agg[i] = first[min(j for j in adj[i] if first[j] >= 0)]
    return agg, na


def coarse_graph(adj, agg, na):
    nbr = [set() for _ in range(na)]
    for i, js in enumerate(adj):
        for j in js:
            if agg[j] != agg[i]:
                nbr[agg[i]].add(int(agg[j]))
    return [sorted(s) for s in nbr]


def gershgorin_rho(A):
    A = sp.csr_matrix(A)
    d = A.diagonal()
    rows = np.asarray(abs(A).sum(axis=1)).ravel()
    return float((rows / d).max())


class AMG:
    """Aggregation hierarchy below the degree-1 level of mesh ``m`` (the
    oracle mesh at degree 1) with operator ``A1`` (assembled, degree 1)."""

    def __init__(self, m, A1, rho0, cheb_lo=0.1, cheb_hi=1.1, cheb_degree=2, coarse_size=1024,
                 max_levels=12, kcycle_levels=2, kcycle_t=0.25):
        if m.N != 1:
            raise ValueError("the algebraic levels start from degree 1")
        self.lo, self.hi, self.deg = cheb_lo, cheb_hi, cheb_degree
        self.kcycle_levels, self.kcycle_t = kcycle_levels, kcycle_t
        A1 = sp.csr_matrix(A1)
        K = m.K
        P0 = sp.csr_matrix((np.ones(3 * K), (np.arange(3 * K), np.repeat(np.arange(K), 3))),
                           shape=(3 * K, K))
        self.A = [A1]
        self.P = [P0]
        self.rho = [float(rho0)]
        adj = element_graph(m)
        A = (P0.T @ A1 @ P0).tocsr()
        self.aggs = []
        while True:
            self.A.append(A)
            self.rho.append(gershgorin_rho(A))
            n = A.shape[0]
            if n <= coarse_size or len(self.A) >= max_levels:
                break
            agg, na = aggregate(adj)
            if na == n:
                break
            self.aggs.append(agg)
            P = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, na))
            self.P.append(P)
            adj = coarse_graph(adj, agg, na)
            A = (P.T @ A @ P).tocsr()
        self.dinv = [1.0 / Al.diagonal() for Al in self.A]
        self.coarse = np.linalg.inv(self.A[-1].toarray())

    @property
    def sizes(self):
        return [Al.shape[0] for Al in self.A]

    def smooth(self, l, f, x0):
        return chebyshev(self.A[l], self.dinv[l], f, x0, self.lo * self.rho[l], self.hi * self.rho[l],
                         self.deg)

    def vcycle(self, l, r):
        if l == len(self.A) - 1:
            return self.coarse @ r
        z = self.smooth(l, r, None)
        res = r - self.A[l] @ z
        zc = self.vcycle(l + 1, self.P[l].T @ res)
        z = z + self.P[l] @ zc
        return self.smooth(l, r, z)

    def krylov_correction(self, l, rc):
        """Approximate solution of A_l e = rc by at most two flexible-CG steps
        from zero, each preconditioned by one cycle on level l."""
        A = self.A[l]
        v1 = self.cycle(l, rc)
        w1 = A @ v1
        rho1, alpha1 = v1 @ rc, v1 @ w1
        r2 = rc - (rho1 / alpha1) * w1
        if np.linalg.norm(r2) <= self.kcycle_t * np.linalg.norm(rc):
            return (rho1 / alpha1) * v1
        v2 = self.cycle(l, r2)
        w2 = A @ v2
        gamma, beta, rho2 = v2 @ w1, v2 @ w2, v2 @ r2
        # second direction made A-orthogonal to the first: v2 - (gamma/alpha1) v1
        alpha2 = beta - gamma * gamma / alpha1
        return (rho1 / alpha1 - gamma * rho2 / (alpha1 * alpha2)) * v1 + (rho2 / alpha2) * v2

    def cycle(self, l, r):
        """One preconditioner cycle from zero on level l: K-cycle on the first
        kcycle_levels levels, V-cycle below."""
        last = len(self.A) - 1
        if l == last:
            return self.coarse @ r
        z = self.smooth(l, r, None)
        rc = self.P[l].T @ (r - self.A[l] @ z)
        if l < self.kcycle_levels and l + 1 < last:
            zc = self.krylov_correction(l + 1, rc)
        else:
            zc = self.cycle(l + 1, rc)
        z = z + self.P[l] @ zc
        return self.smooth(l, r, z)

    def solve(self, r, cycles=1):
        """``cycles`` cycles from zero (iterative refinement)."""
        x = self.cycle(0, r)
        for _ in range(cycles - 1):
            x = x + self.cycle(0, r - self.A[0] @ x)
        return x
