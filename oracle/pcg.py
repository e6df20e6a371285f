"""FP64 preconditioned conjugate gradient, following the paper's listing.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring): imported by
tests, the smoke check and the benchmark's CPU-baseline leg, never by the
library path.

Section 2.2 gives the preconditioned CG iteration; section 2.4 takes the
preconditioner M as the main diagonal of A (Jacobi). With M = I the same
steps are plain CG. (The unpreconditioned listing of section 2.2 prints
beta with the wrong sign; the preconditioned listing is the one followed.)

Stopping rule: ||r_l|| / ||b|| < delta with a strict "<", tested before each
iteration, so delta >= 1 gives zero iterations. The potential starts at zero
unless an initial guess is passed (section 2.7 initialises it to zero).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float        # recurrence residual ||r_l|| / ||b||
    converged: bool
    breakdown: bool = False


def pcg(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
        m_diag: Optional[np.ndarray], tol: float, maxiter: int,
        x0: Optional[np.ndarray] = None,
        callback: Optional[Callable[[int, np.ndarray], None]] = None) -> PCGResult:
    """Solve A x = b. `m_diag` is the Jacobi preconditioner diag(A) (section
    2.4); None means M = I (plain CG)."""
    minv = None if m_diag is None else 1.0 / np.asarray(m_diag, np.float64).ravel()
    solve_m = (lambda r: r * minv) if minv is not None else (lambda r: r.copy())
    return _pcg(apply_A, b, solve_m, tol, maxiter, x0, callback)


def pcg_general(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
                apply_Minv: Callable[[np.ndarray], np.ndarray], tol: float, maxiter: int,
                x0: Optional[np.ndarray] = None) -> PCGResult:
    """The same listing with z = M^-1 r given by a function of r (a fixed
    symmetric positive definite preconditioner, e.g. a multigrid cycle)."""
    shape = b.shape
    return _pcg(apply_A, b, lambda r: np.asarray(apply_Minv(r.reshape(shape)), np.float64).ravel(),
                tol, maxiter, x0, None)


def _pcg(apply_A, b, solve_m, tol, maxiter, x0, callback) -> PCGResult:
    shape = b.shape
    b = np.asarray(b, np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return PCGResult(np.zeros(shape), 0, 0.0, True)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64).ravel()
    Ax = lambda v: np.asarray(apply_A(v.reshape(shape)), np.float64).ravel()

    # step 1: l = 0, r_0 = b - A x_0
    r = b - Ax(x) if x0 is not None else b.copy()
    # step 2: solve M z_0 = r_0, p_0 = z_0
    z = solve_m(r)
    p = z.copy()
    rz = float(np.dot(r, z))
    l = 0
    if callback is not None:
        callback(l, x)
    while True:
        # step 3: stop when ||r_l|| / ||b|| < delta
        relres = float(np.linalg.norm(r)) / bnorm
        if relres < tol:
            return PCGResult(x.reshape(shape), l, relres, True)
        if l >= maxiter:
            return PCGResult(x.reshape(shape), l, relres, False)
        # step 4
        l += 1
        # step 5: alpha, x and r updates
        q = Ax(p)
        pq = float(np.dot(p, q))
        if not (pq > 0.0) or not np.isfinite(pq):
            return PCGResult(x.reshape(shape), l - 1, relres, False, breakdown=True)
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        # step 6: solve M z_l = r_l
        z = solve_m(r)
        # step 7: beta and the new direction
        rz_new = float(np.dot(r, z))
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        if callback is not None:
            callback(l, x)


def jpcg(system, tol: float, maxiter: Optional[int] = None, x0=None,
         callback=None) -> PCGResult:
    """Jacobi-preconditioned CG on an assembled `fdpb.System`."""
    from . import fdpb
    if maxiter is None:
        maxiter = 10 * max(system.dims)
    return pcg(lambda v: fdpb.apply(system, v), system.b, fdpb.diagonal(system),
               tol, maxiter, x0=x0, callback=callback)


def refine(system, tol_outer: float, tol_inner: float = 1e-4,
           max_outer: int = 20, inner_solver=None, with_status: bool = False):
    """Iterative refinement: r = b - A x in FP64, inner solve A d = r to a
    tolerance relative to ||r|| from d = 0, x += d; stops when ||r||/||b|| <
    tol_outer (converged), after max_outer corrections, or when an outer step
    reduced ||r|| by less than a factor 2 (stagnation: the inner solver's own
    rounding floor has been reached). `inner_solver(rhs, tol)` defaults to the
    FP64 Jacobi PCG. Returns (x, outer_steps, inner_iterations_list, relres),
    and with `with_status` also one of "converged", "max_outer",
    "stagnated", "breakdown"."""
    from . import fdpb
    b = system.b
    bn = float(np.linalg.norm(b.ravel()))
    x = np.zeros(system.shape)
    inner = []

    def done(outer, rel, status):
        return (x, outer, inner, rel, status) if with_status else (x, outer, inner, rel)

    if bn == 0.0:
        return done(0, 0.0, "converged")
    if inner_solver is None:
        d = fdpb.diagonal(system)
        inner_solver = lambda rhs, t: pcg(lambda v: fdpb.apply(system, v), rhs, d, t,
                                          10 * max(system.dims))
    rel_prev = None
    for outer in range(max_outer + 1):
        r = b - fdpb.apply(system, x)
        rel = float(np.linalg.norm(r.ravel())) / bn
        if rel < tol_outer:
            return done(outer, rel, "converged")
        if outer == max_outer:
            return done(outer, rel, "max_outer")
        if rel_prev is not None and rel > 0.5 * rel_prev:
            return done(outer, rel, "stagnated")
        rel_prev = rel
        res = inner_solver(r, tol_inner)
        inner.append(res.iters)
        if res.breakdown:
            return done(outer, rel, "breakdown")
        x = x + res.x
    return done(max_outer, rel, "max_outer")
