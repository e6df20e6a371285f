"""FP64 CPU oracle of geometric-multigrid-preconditioned CG.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.

The paper names geometric multigrid as the next step for these systems
(sections 3.2 and 4) without fixing a scheme; this module states one plainly
(every choice below is a reading, listed in the design notes):

* Levels: vertex coarsening by two in each axis. Coarse node I of a level
  with n nodes sits at fine node 2I+1, so a level has floor(n/2) nodes per
  axis and spacing 2h; its Dirichlet ghosts sit at fine -1 and 2*nc+1.
  Coarsening stops when an axis would drop below 3 nodes or the level has at
  most `min_nodes` nodes.
* Coarse coefficients: the edge between coarse nodes E-1 and E along x is
  the series (harmonic) combination of the two fine edges it spans, fine
  edges 2E and 2E+1 (a missing second edge past the fine ghost repeats the
  first), averaged across the edge over the fine lines 2J+1+a, 2K+1+b
  (a, b in -1..1) with weights (1,2,1)x(1,2,1)/16 over the lines inside the
  grid. kbar^2 is the full-weighting (1,2,1)^3/64 average over the fine
  nodes inside the grid. The level operator is Eq. 3 at spacing 2^l h.
* Transfer: P is trilinear interpolation (coarse ghosts are zero),
  R = P^T / 8 (full weighting).
* V-cycle (the preconditioner z = M r): from z = 0, nu damped-Jacobi sweeps
  z += omega D^-1 (r - A z), residual, restriction, the coarse V-cycle,
  prolongation, nu more sweeps; on the coarsest level `coarse_sweeps`
  sweeps. Equal pre- and post-smoothing makes M symmetric; with a convergent
  smoother it is positive definite, as CG requires.
* Outer iteration: the preconditioned CG listing of section 2.2 with that M.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import fdpb, pcg

W3 = np.array([0.25, 0.5, 0.25])


@dataclasses.dataclass
class Level:
    sys: fdpb.System      # b unused on coarse levels
    d: np.ndarray         # diagonal


def _series(e1, e2):
    return 2.0 * e1 * e2 / (e1 + e2)


def coarsen_system(s: fdpb.System) -> fdpb.System:
    """The next coarser level's edge arrays and kbar^2 (module docstring)."""
    nz, ny, nx = s.shape
    ncx, ncy, ncz = nx // 2, ny // 2, nz // 2
    ex, ey, ez, k2 = s.eps_x, s.eps_y, s.eps_z, s.kappa2

    def line_avg(get, trans_a, trans_b, na, nb):
        """Weighted average over fine lines (2A+1+a, 2B+1+b) inside the grid."""
        acc = 0.0
        wsum = 0.0
        for a in (-1, 0, 1):
            ia = 2 * trans_a + 1 + a
            if ia < 0 or ia >= na:
                continue
            for b in (-1, 0, 1):
                ib = 2 * trans_b + 1 + b
                if ib < 0 or ib >= nb:
                    continue
                w = W3[a + 1] * W3[b + 1]
                acc += w * get(ia, ib)
                wsum += w
        return acc / wsum

    def along(e, n_fine, E):
        e1 = e(2 * E)
        e2 = e(2 * E + 1) if 2 * E + 1 <= n_fine else e1
        return _series(e1, e2)

    cex = np.empty((ncz, ncy, ncx + 1))
    for K in range(ncz):
        for J in range(ncy):
            for E in range(ncx + 1):
                cex[K, J, E] = line_avg(lambda j, k: along(lambda e: ex[k, j, e], nx, E), J, K, ny, nz)
    cey = np.empty((ncz, ncy + 1, ncx))
    for K in range(ncz):
        for E in range(ncy + 1):
            for I in range(ncx):
                cey[K, E, I] = line_avg(lambda i, k: along(lambda e: ey[k, e, i], ny, E), I, K, nx, nz)
    cez = np.empty((ncz + 1, ncy, ncx))
    for E in range(ncz + 1):
        for J in range(ncy):
            for I in range(ncx):
                cez[E, J, I] = line_avg(lambda i, j: along(lambda e: ez[e, j, i], nz, E), I, J, nx, ny)
    ck2 = np.empty((ncz, ncy, ncx))
    for K in range(ncz):
        for J in range(ncy):
            for I in range(ncx):
                acc = wsum = 0.0
                for c in (-1, 0, 1):
                    k = 2 * K + 1 + c
                    if not 0 <= k < nz:
                        continue
                    for b in (-1, 0, 1):
                        j = 2 * J + 1 + b
                        if not 0 <= j < ny:
                            continue
                        for a in (-1, 0, 1):
                            i = 2 * I + 1 + a
                            if not 0 <= i < nx:
                                continue
                            w = W3[a + 1] * W3[b + 1] * W3[c + 1]
                            acc += w * k2[k, j, i]
                            wsum += w
                ck2[K, J, I] = acc / wsum
    return fdpb.System(h=2.0 * s.h, eps_x=cex, eps_y=cey, eps_z=cez, kappa2=ck2, b=np.zeros((ncz, ncy, ncx)))


def hierarchy(s: fdpb.System, min_nodes: int = 512) -> List[Level]:
    levels = [Level(s, fdpb.diagonal(s))]
    cur = s
    while True:
        nx, ny, nz = cur.dims
        if min(nx, ny, nz) // 2 < 3 or nx * ny * nz <= min_nodes:
            break
        cur = coarsen_system(cur)
        levels.append(Level(cur, fdpb.diagonal(cur)))
    return levels


def prolong(xc: np.ndarray, fine_shape) -> np.ndarray:
    """Trilinear interpolation to the fine level: fine i odd takes coarse
    (i-1)/2; fine i even averages coarse i/2-1 and i/2 (zero ghosts)."""
    out = xc
    for axis, n in ((0, fine_shape[0]), (1, fine_shape[1]), (2, fine_shape[2])):
        nc = out.shape[axis]
        pad = [(0, 0)] * 3
        pad[axis] = (1, 1)
        op = np.pad(out, pad)                # op index c+1 holds coarse c; ghosts zero
        i = np.arange(n)
        odd = (i % 2) == 1
        take_a = np.where(odd, (i - 1) // 2 + 1, i // 2)      # coarse i/2-1 -> padded i/2
        take_b = np.where(odd, (i - 1) // 2 + 1, i // 2 + 1)
        wa = np.where(odd, 1.0, 0.5)
        wb = np.where(odd, 0.0, 0.5)
        A = np.take(op, take_a, axis=axis)
        B = np.take(op, take_b, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = n
        out = wa.reshape(shape) * A + wb.reshape(shape) * B
    return out


def restrict(rf: np.ndarray, coarse_shape) -> np.ndarray:
    """R = P^T / 8, written as the transpose of `prolong`'s weights."""
    out = rf
    for axis, nc in ((0, coarse_shape[0]), (1, coarse_shape[1]), (2, coarse_shape[2])):
        n = out.shape[axis]
        pad = [(0, 0)] * 3
        pad[axis] = (1, 1)
        op = np.pad(out, pad)               # op index i+1 holds fine i; outside zero
        C = np.arange(nc)
        # coarse C collects fine 2C+1 (weight 1) and fine 2C, 2C+2 (weight 1/2)
        mid = np.take(op, 2 * C + 2, axis=axis)
        lo = np.take(op, 2 * C + 1, axis=axis)
        hi = np.take(op, np.minimum(2 * C + 3, n + 1), axis=axis)
        out = (mid + 0.5 * lo + 0.5 * hi) / 2.0
    return out


def jacobi_sweep(lv: Level, b, z, omega):
    return z + omega * (b - fdpb.apply(lv.sys, z)) / lv.d


def vcycle(levels: List[Level], l: int, b, nu=2, omega=0.8, coarse_sweeps=40):
    lv = levels[l]
    if l == len(levels) - 1:
        z = np.zeros_like(b)
        for _ in range(coarse_sweeps):
            z = jacobi_sweep(lv, b, z, omega)
        return z
    z = np.zeros_like(b)
    for _ in range(nu):
        z = jacobi_sweep(lv, b, z, omega)
    r = b - fdpb.apply(lv.sys, z)
    nxt = levels[l + 1]
    bc = restrict(r, nxt.sys.shape)
    zc = vcycle(levels, l + 1, bc, nu, omega, coarse_sweeps)
    z = z + prolong(zc, lv.sys.shape)
    for _ in range(nu):
        z = jacobi_sweep(lv, b, z, omega)
    return z


def mgpcg(s: fdpb.System, tol: float, maxiter: int = 500, nu=2, omega=0.8, coarse_sweeps=40,
          min_nodes=512):
    """The section 2.2 PCG listing with M^-1 = one V-cycle."""
    levels = hierarchy(s, min_nodes)
    res = pcg.pcg_general(lambda v: fdpb.apply(s, v), s.b,
                          lambda r: vcycle(levels, 0, r, nu, omega, coarse_sweeps), tol, maxiter)
    return res, levels
