"""FP64 CPU oracle for the periodic boundary condition.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.

Section 2.7 of the paper mentions a periodic boundary as the alternative to
the free-space one. Readings (listed with the others in the design notes):

* The box holds nx*ny*nz nodes and repeats with period (nx h, ny h, nz h):
  node i+nx is node i. There is no ghost layer and no boundary term in b.
* Classification: a node is inside iff it lies strictly inside some periodic
  image of some atom sphere. Each atom's sphere is tested against the node
  positions origin + h*iu of an unwrapped index window around it, and the
  wrapped node iu mod n is marked: the same FP64 expression as the
  free-space case, so no division or rounding of coordinates enters.
* Edges: the two-point harmonic mean of the endpoint node values, the edge
  between node n-1 and node 0 included; in the staggered arrays entries 0
  and n both hold that wrap edge.
* Charges: trilinear spreading with g = (c - o)/h, i0 = floor(g), f = g - i0
  and nodes i0 mod n, i0+1 mod n (atoms may lie anywhere).
* Singular case: with kbar^2 = 0 at every node the operator annihilates
  constants. Then b has its mean removed (a uniform neutralising background)
  and the potential is reported with zero mean.
"""
from __future__ import annotations

import math

import numpy as np

from . import fdpb


def classify(nx, ny, nz, h, origin, xyz, radius) -> np.ndarray:
    """Inside mask (nz, ny, nx): 1 where the node is strictly inside some
    periodic image of some sphere."""
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    n3 = (nx, ny, nz)
    for c, r in zip(np.asarray(xyz, np.float64), np.asarray(radius, np.float64)):
        rr = r * r
        lo = [int(math.floor((c[d] - r - origin[d]) / h)) - 1 for d in range(3)]
        hi = [int(math.ceil((c[d] + r - origin[d]) / h)) + 1 for d in range(3)]
        iu = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
        dx = (origin[0] + h * iu[0].astype(np.float64)) - c[0]
        dy = (origin[1] + h * iu[1].astype(np.float64)) - c[1]
        dz = (origin[2] + h * iu[2].astype(np.float64)) - c[2]
        d2 = (dx * dx)[None, None, :] + (dy * dy)[None, :, None]
        d2 = d2 + (dz * dz)[:, None, None]
        kk, jj, ii = np.nonzero(d2 < rr)
        mask[np.mod(iu[2][kk], n3[2]), np.mod(iu[1][jj], n3[1]), np.mod(iu[0][ii], n3[0])] = 1
    return mask


def padded_mask(mask: np.ndarray) -> np.ndarray:
    """The (nz+2, ny+2, nx+2) layout of the free-space mask, ghost entries
    holding the wrapped node's value."""
    return np.pad(mask, 1, mode="wrap")


def dielectric_edges(mask: np.ndarray, eps_in: float, eps_out: float):
    """Staggered edge arrays (entries 0 and n are the wrap edge)."""
    e = np.where(mask != 0, eps_in, eps_out).astype(np.float64)
    ep = np.pad(e, 1, mode="wrap")
    eps_x = fdpb.harmonic(ep[1:-1, 1:-1, :-1], ep[1:-1, 1:-1, 1:])
    eps_y = fdpb.harmonic(ep[1:-1, :-1, 1:-1], ep[1:-1, 1:, 1:-1])
    eps_z = fdpb.harmonic(ep[:-1, 1:-1, 1:-1], ep[1:, 1:-1, 1:-1])
    return eps_x, eps_y, eps_z


def salt_term(mask: np.ndarray, eps_out: float, kappa_d2: float) -> np.ndarray:
    return np.where(mask != 0, 0.0, eps_out * kappa_d2).astype(np.float64)


def spread_weights(nx, ny, nz, h, origin, xyz):
    """Per atom: 8 wrapped node flat indices and trilinear weights."""
    xyz = np.asarray(xyz, np.float64)
    g = (xyz - np.asarray(origin, np.float64)[None, :]) / h
    i0 = np.floor(g).astype(np.int64)
    f = g - i0
    dims = (nx, ny, nz)
    idx = np.empty((xyz.shape[0], 8), dtype=np.int64)
    w = np.empty((xyz.shape[0], 8, 3), dtype=np.float64)
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        ii = np.mod(i0[:, 0] + cx, dims[0])
        jj = np.mod(i0[:, 1] + cy, dims[1])
        kk = np.mod(i0[:, 2] + cz, dims[2])
        idx[:, c] = ii + nx * (jj + ny * kk)
        w[:, c, 0] = f[:, 0] if cx else 1.0 - f[:, 0]
        w[:, c, 1] = f[:, 1] if cy else 1.0 - f[:, 1]
        w[:, c, 2] = f[:, 2] if cz else 1.0 - f[:, 2]
    return idx, w


def spread_charges(nx, ny, nz, h, origin, xyz, charge) -> np.ndarray:
    idx, w = spread_weights(nx, ny, nz, h, origin, xyz)
    q = np.asarray(charge, np.float64)
    vals = q[:, None] * w[:, :, 0] * w[:, :, 1] * w[:, :, 2]
    out = np.zeros(nx * ny * nz, dtype=np.float64)
    np.add.at(out, idx.ravel(), vals.ravel())
    return out.reshape(nz, ny, nx)


def is_singular(kappa2: np.ndarray) -> bool:
    return not (np.asarray(kappa2) > 0.0).any()


def assemble(nx, ny, nz, h, origin, xyz, radius, charge, eps_in, eps_out, kappa_d2, with_parts=False):
    """Periodic setup: classification, edges, salt, charges; b = 4 pi q / h^3,
    with its mean removed in the singular case."""
    mask = classify(nx, ny, nz, h, origin, xyz, radius)
    ex, ey, ez = dielectric_edges(mask, eps_in, eps_out)
    k2 = salt_term(mask, eps_out, kappa_d2)
    q = spread_charges(nx, ny, nz, h, origin, xyz, charge)
    b = fdpb.FOUR_PI * q / h ** 3
    if is_singular(k2):
        b = b - b.mean()
    s = fdpb.System(h=h, eps_x=ex, eps_y=ey, eps_z=ez, kappa2=k2, b=b)
    if with_parts:
        return s, dict(mask=mask, qgrid=q)
    return s


def diagonal(s: fdpb.System) -> np.ndarray:
    """Same as the free-space diagonal: the six edges of each node plus kbar^2."""
    return fdpb.diagonal(s)


def apply(s: fdpb.System, phi: np.ndarray) -> np.ndarray:
    """(A phi) with wraparound neighbours (the edge arrays' entry e couples
    node e-1 and node e, entry 0 and n both the wrap edge)."""
    phi = np.asarray(phi, np.float64).reshape(s.shape)
    ex, ey, ez = s.eps_x, s.eps_y, s.eps_z
    nb = (ex[:, :, :-1] * np.roll(phi, 1, axis=2) + ex[:, :, 1:] * np.roll(phi, -1, axis=2)
          + ey[:, :-1, :] * np.roll(phi, 1, axis=1) + ey[:, 1:, :] * np.roll(phi, -1, axis=1)
          + ez[:-1] * np.roll(phi, 1, axis=0) + ez[1:] * np.roll(phi, -1, axis=0))
    return diagonal(s) * phi - nb / (s.h * s.h)


def true_relres(s: fdpb.System, phi: np.ndarray) -> float:
    bn = float(np.linalg.norm(s.b.ravel()))
    r = s.b - apply(s, phi)
    return float(np.linalg.norm(r.ravel())) / bn if bn > 0 else float(np.linalg.norm(phi) != 0)


def dense_matrix(s: fdpb.System) -> np.ndarray:
    """Dense A from explicit index arithmetic (tiny grids; n >= 3 per axis)."""
    nz, ny, nx = s.shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    h2 = s.h * s.h
    d = diagonal(s).ravel()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                m = i + nx * (j + ny * k)
                A[m, m] = d[m]
                nbrs = [((i + 1) % nx, j, k, s.eps_x[k, j, i + 1]), ((i - 1) % nx, j, k, s.eps_x[k, j, i]),
                        (i, (j + 1) % ny, k, s.eps_y[k, j + 1, i]), (i, (j - 1) % ny, k, s.eps_y[k, j, i]),
                        (i, j, (k + 1) % nz, s.eps_z[k + 1, j, i]), (i, j, (k - 1) % nz, s.eps_z[k, j, i])]
                for a, b_, c, e in nbrs:
                    A[m, a + nx * (b_ + ny * c)] -= e / h2
    return A


def jpcg(s: fdpb.System, tol: float, maxiter=None, x0=None):
    """The section 2.2 listing with M = diag(A) on the periodic operator; in
    the singular case the result is shifted to zero mean."""
    from . import pcg
    if maxiter is None:
        maxiter = 10 * max(s.dims)
    res = pcg.pcg(lambda v: apply(s, v), s.b, diagonal(s), tol, maxiter, x0=x0)
    if is_singular(s.kappa2):
        res.x = res.x - res.x.mean()
    return res


def interpolate(nx, ny, nz, h, origin, xyz, phi) -> np.ndarray:
    idx, w = spread_weights(nx, ny, nz, h, origin, xyz)
    flat = np.asarray(phi, np.float64).ravel()
    return (w[:, :, 0] * w[:, :, 1] * w[:, :, 2] * flat[idx]).sum(axis=1)


def energy(nx, ny, nz, h, origin, xyz, charge, phi) -> float:
    pa = interpolate(nx, ny, nz, h, origin, xyz, phi)
    return 0.5 * float(np.dot(np.asarray(charge, np.float64), pa)) * fdpb.COULOMB_KCAL


def fft_solve(b: np.ndarray, h: float, eps: float, kbar2: float) -> np.ndarray:
    """Exact solution for a uniform dielectric and uniform kbar^2 by the
    discrete Fourier transform, which diagonalises the periodic 7-point
    operator: lambda(k) = (eps/h^2) sum_d (2 - 2 cos(2 pi k_d / n_d)) + kbar^2;
    the k = 0 mode is set to zero when lambda(0) = 0."""
    nz, ny, nx = b.shape
    lam = np.zeros(b.shape)
    for axis, n in ((2, nx), (1, ny), (0, nz)):
        m = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
        shape = [1, 1, 1]
        shape[axis] = n
        lam = lam + m.reshape(shape)
    lam = eps / (h * h) * lam + kbar2
    bh = np.fft.fftn(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        xh = np.where(lam > 0, bh / np.where(lam > 0, lam, 1.0), 0.0)
    return np.real(np.fft.ifftn(xh))
