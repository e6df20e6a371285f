"""FP64 CPU oracle for the linear finite-difference Poisson-Boltzmann system.

TEST INFRASTRUCTURE ONLY. This module is a plain, slow, obviously-correct
reference. It may be imported only by tests, by the smoke check and by the
benchmark's CPU-baseline leg; the library path never imports or calls it.
It shares no code with the GPU path (only the seeded input generator in
`synth` serves both).

What it computes (paper: "Acceleration of Linear Finite-Difference
Poisson-Boltzmann Methods on GPUs"):

* Eq. 2 / Eq. 3 (section 2.1): the 7-point FD operator with edge dielectrics
  eps_i, eps_j, eps_k between neighbouring nodes and a diagonal salt term
  kappa^2, right-hand side h^-3 q(i,j,k).
* Section 2.7: solute/solvent dielectrics 1/80, harmonic averaging on the
  boundary edges, free-space (Dirichlet) boundary, zero initial potential.

Readings where the paper is silent (each is listed in the design notes):

* Units: Gaussian form  -div(eps grad phi) + kbar^2 phi = 4 pi rho, so the
  right-hand side is 4 pi q_node / h^3 and phi is in e/A; energies are
  multiplied by 332.0637133 kcal A / (mol e^2).
* Grid: all nx*ny*nz nodes are unknowns; Dirichlet values live on a ghost
  layer one h outside the box. Node (i,j,k) sits at origin + h*(i,j,k).
* Classification: node inside iff dx*dx+dy*dy+dz*dz < R*R for some atom,
  evaluated in FP64 in that order (a node exactly on a surface is outside).
  Ghost nodes are classified too.
* Edge dielectric: two-point harmonic mean 2 e_a e_b / (e_a + e_b) of the two
  endpoint node values.
* Salt: kbar^2 = eps_out * kappa_D^2 at outside nodes, 0 inside (no Stern
  margin).
* Charges: trilinear spreading; g = (c - o)/h, i0 = clamp(floor(g), 0, n-2),
  f = g - i0, weights (1-f) and f per axis.
* Boundary: screened Coulomb sum phi(r) = sum_a q_a exp(-kappa_D d)/(eps_out d)
  evaluated on the face ghosts and folded into b through the ghost-side edge.

Array convention: numpy arrays indexed [k, j, i] (C order), so the flat index
is i + nx*(j + ny*k), x fastest. Staggered edge arrays:
  eps_x[k, j, e], e = 0..nx : edge between nodes (e-1, j, k) and (e, j, k)
  eps_y[k, e, i], e = 0..ny : edge between nodes (i, e-1, k) and (i, e, k)
  eps_z[e, j, i], e = 0..nz : edge between nodes (i, j, e-1) and (i, j, e)
(index -1 and n are ghost nodes).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FOUR_PI = 4.0 * math.pi
COULOMB_KCAL = 332.0637133  # e^2 / (4 pi eps0) in kcal A / mol


@dataclasses.dataclass
class System:
    """The assembled linear system A phi = b of Eq. 4 (matrix-free form)."""
    h: float
    eps_x: np.ndarray   # (nz, ny, nx+1)
    eps_y: np.ndarray   # (nz, ny+1, nx)
    eps_z: np.ndarray   # (nz+1, ny, nx)
    kappa2: np.ndarray  # (nz, ny, nx)  kbar^2 per node
    b: np.ndarray       # (nz, ny, nx)

    @property
    def shape(self):
        return self.kappa2.shape

    @property
    def dims(self):
        nz, ny, nx = self.kappa2.shape
        return nx, ny, nz


# --------------------------------------------------------------------------
# Setup (section 2.7 and Eq. 3)
# --------------------------------------------------------------------------

def padded_axis(origin: float, h: float, n: int) -> np.ndarray:
    """Coordinates of nodes -1..n along one axis: origin + h*i."""
    return origin + h * np.arange(-1, n + 1, dtype=np.float64)


def classify(nx, ny, nz, h, origin, xyz, radius) -> np.ndarray:
    """Inside mask over the padded (nz+2, ny+2, nx+2) node set, ghosts
    included. mask[k+1, j+1, i+1] == 1 iff node (i,j,k) lies strictly inside
    at least one atom sphere."""
    xs = padded_axis(origin[0], h, nx)
    ys = padded_axis(origin[1], h, ny)
    zs = padded_axis(origin[2], h, nz)
    mask = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.uint8)
    for c, r in zip(np.asarray(xyz, np.float64), np.asarray(radius, np.float64)):
        rr = r * r
        # padded-index window that certainly contains every candidate node
        lo = [int(math.floor((c[d] - r - origin[d]) / h)) for d in range(3)]
        hi = [int(math.ceil((c[d] + r - origin[d]) / h)) for d in range(3)]
        n3 = (nx, ny, nz)
        a = [min(max(lo[d] - 1, -1), n3[d]) + 1 for d in range(3)]
        b = [min(max(hi[d] + 1, -1), n3[d]) + 2 for d in range(3)]
        if any(a[d] >= b[d] for d in range(3)):
            continue
        dx = xs[a[0]:b[0]] - c[0]
        dy = ys[a[1]:b[1]] - c[1]
        dz = zs[a[2]:b[2]] - c[2]
        d2 = (dx * dx)[None, None, :] + (dy * dy)[None, :, None]
        d2 = d2 + (dz * dz)[:, None, None]
        mask[a[2]:b[2], a[1]:b[1], a[0]:b[0]] |= (d2 < rr).astype(np.uint8)
    return mask


def harmonic(ea: np.ndarray, eb: np.ndarray) -> np.ndarray:
    return 2.0 * ea * eb / (ea + eb)


def dielectric_edges(mask: np.ndarray, eps_in: float, eps_out: float):
    """Staggered edge dielectrics from the padded node mask."""
    e = np.where(mask != 0, eps_in, eps_out).astype(np.float64)
    eps_x = harmonic(e[1:-1, 1:-1, :-1], e[1:-1, 1:-1, 1:])
    eps_y = harmonic(e[1:-1, :-1, 1:-1], e[1:-1, 1:, 1:-1])
    eps_z = harmonic(e[:-1, 1:-1, 1:-1], e[1:, 1:-1, 1:-1])
    return eps_x, eps_y, eps_z


def edge_inside_fraction(nx, ny, nz, h, origin, xyz, radius, axis):
    """Fraction of each staggered edge of direction `axis` (0 x, 1 y, 2 z)
    that lies inside the union of the atom spheres, edges indexed as the
    staggered arrays (entry e joins nodes e-1 and e along the axis; -1 and n
    are ghosts). For a sphere (c, R) and the edge's line, d2 = sum of the
    squared offsets across the line (in axis order); if d2 < R*R the sphere
    covers the line parameter t in [((c_a - w) - x0)/h, ((c_a + w) - x0)/h],
    w = sqrt(R*R - d2), x0 the edge's first node coordinate along the axis.
    The intervals clipped to [0, 1] are sorted by start, merged, and their
    lengths summed in that order."""
    o = np.asarray(origin, np.float64)
    dims = (nx, ny, nz)
    shape = [nz, ny, nx]
    shape[2 - axis] += 1
    frac = np.zeros(shape)
    recs = {}
    for c, R in zip(np.asarray(xyz, np.float64), np.asarray(radius, np.float64)):
        RR = R * R
        rng = []
        for d in range(3):
            lo = int(math.floor((c[d] - R - o[d]) / h)) - 1
            hi = int(math.ceil((c[d] + R - o[d]) / h)) + 1
            if d == axis:   # edge index e: first node e-1 in [-1, n-1]
                rng.append(range(max(lo + 1, 0), min(hi + 1, dims[d]) + 1))
            else:           # node index in [0, n-1]
                rng.append(range(max(lo, 0), min(hi, dims[d] - 1) + 1))
        for k in rng[2]:
            for j in rng[1]:
                for i in rng[0]:
                    idx = [i, j, k]
                    node = [float(v) for v in idx]
                    node[axis] -= 1.0     # the edge's first node
                    p = [o[d] + h * node[d] for d in range(3)]
                    d2 = 0.0
                    for d in range(3):
                        if d != axis:
                            dd = p[d] - c[d]
                            d2 = d2 + dd * dd
                    if not d2 < RR:
                        continue
                    w = math.sqrt(RR - d2)
                    t0 = ((c[axis] - w) - p[axis]) / h
                    t1 = ((c[axis] + w) - p[axis]) / h
                    t0 = max(t0, 0.0)
                    t1 = min(t1, 1.0)
                    if t1 > t0:
                        recs.setdefault((k, j, i), []).append((t0, t1))
    for key, iv in recs.items():
        iv.sort()
        total = 0.0
        s0, s1 = iv[0]
        for a, b in iv[1:]:
            if a > s1:
                total = total + (s1 - s0)
                s0, s1 = a, b
            elif b > s1:
                s1 = b
        total = total + (s1 - s0)
        frac[key] = total
    return frac


def fractional_edges(nx, ny, nz, h, origin, xyz, radius, eps_in, eps_out):
    """Weighted harmonic edge dielectric (the fractional-edge reading of
    section 2.7): 1 / (f/eps_in + (1-f)/eps_out) with f the inside fraction
    of the edge; exactly eps_out at f = 0 and eps_in at f = 1."""
    out = []
    for axis in range(3):
        f = edge_inside_fraction(nx, ny, nz, h, origin, xyz, radius, axis)
        e = 1.0 / (f / eps_in + (1.0 - f) / eps_out)
        e = np.where(f == 0.0, eps_out, np.where(f == 1.0, eps_in, e))
        out.append(e)
    return tuple(out)


def salt_term(mask: np.ndarray, eps_out: float, kappa_d2: float) -> np.ndarray:
    """kbar^2 per node: eps_out * kappa_D^2 outside the solute, 0 inside."""
    inner = mask[1:-1, 1:-1, 1:-1]
    return np.where(inner != 0, 0.0, eps_out * kappa_d2).astype(np.float64)


def spread_weights(nx, ny, nz, h, origin, xyz):
    """Per atom: the 8 node flat indices and trilinear weights (atom, corner),
    corner = cx + 2 cy + 4 cz."""
    xyz = np.asarray(xyz, np.float64)
    dims = np.array([nx, ny, nz])
    if (dims < 2).any():
        raise ValueError("trilinear spreading needs at least 2 nodes per axis")
    g = (xyz - np.asarray(origin, np.float64)[None, :]) / h
    if (g < 0.0).any() or (g > (dims - 1)[None, :]).any():
        raise ValueError("atom centre outside the node box")
    i0 = np.clip(np.floor(g).astype(np.int64), 0, dims[None, :] - 2)
    f = g - i0
    idx = np.empty((xyz.shape[0], 8), dtype=np.int64)
    w = np.empty((xyz.shape[0], 8, 3), dtype=np.float64)
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        ii, jj, kk = i0[:, 0] + cx, i0[:, 1] + cy, i0[:, 2] + cz
        idx[:, c] = ii + nx * (jj + ny * kk)
        w[:, c, 0] = f[:, 0] if cx else 1.0 - f[:, 0]
        w[:, c, 1] = f[:, 1] if cy else 1.0 - f[:, 1]
        w[:, c, 2] = f[:, 2] if cz else 1.0 - f[:, 2]
    return idx, w


def spread_charges(nx, ny, nz, h, origin, xyz, charge) -> np.ndarray:
    """q(i,j,k) of Eq. 3: the charge each node receives by trilinear
    spreading. Contributions are added in atom order."""
    idx, w = spread_weights(nx, ny, nz, h, origin, xyz)
    q = np.asarray(charge, np.float64)
    vals = q[:, None] * w[:, :, 0] * w[:, :, 1] * w[:, :, 2]
    out = np.zeros(nx * ny * nz, dtype=np.float64)
    np.add.at(out, idx.ravel(), vals.ravel())
    return out.reshape(nz, ny, nx)


def dh_potential(points, xyz, charge, eps_out, kappa_d2, chunk=1 << 22):
    """phi(r) = sum_a q_a exp(-kappa_D d) / (eps_out d) at each point."""
    points = np.asarray(points, np.float64).reshape(-1, 3)
    xyz = np.asarray(xyz, np.float64)
    q = np.asarray(charge, np.float64)
    kd = math.sqrt(kappa_d2)
    out = np.zeros(points.shape[0])
    step = max(1, chunk // max(1, xyz.shape[0]))
    for s in range(0, points.shape[0], step):
        p = points[s:s + step]
        dx = p[:, None, 0] - xyz[None, :, 0]
        dy = p[:, None, 1] - xyz[None, :, 1]
        dz = p[:, None, 2] - xyz[None, :, 2]
        d = np.sqrt(dx * dx + dy * dy + dz * dz)
        out[s:s + step] = (q[None, :] * np.exp(-kd * d) / (eps_out * d)).sum(axis=1)
    return out


def face_ghost_points(nx, ny, nz, h, origin):
    """Coordinates of the six faces of ghost nodes, as (nz, ny)/(nz, nx)/(ny, nx)
    grids: returns dict face -> (points array (..., 3))."""
    o = np.asarray(origin, np.float64)
    xi = o[0] + h * np.arange(nx, dtype=np.float64)
    yj = o[1] + h * np.arange(ny, dtype=np.float64)
    zk = o[2] + h * np.arange(nz, dtype=np.float64)
    xm, xp = o[0] + h * -1.0, o[0] + h * float(nx)
    ym, yp = o[1] + h * -1.0, o[1] + h * float(ny)
    zm, zp = o[2] + h * -1.0, o[2] + h * float(nz)
    Z, Y = np.meshgrid(zk, yj, indexing="ij")            # (nz, ny)
    Zx, X = np.meshgrid(zk, xi, indexing="ij")           # (nz, nx)
    Yz, Xz = np.meshgrid(yj, xi, indexing="ij")          # (ny, nx)
    faces = {
        "x-": np.stack([np.full_like(Z, xm), Y, Z], axis=-1),
        "x+": np.stack([np.full_like(Z, xp), Y, Z], axis=-1),
        "y-": np.stack([X, np.full_like(X, ym), Zx], axis=-1),
        "y+": np.stack([X, np.full_like(X, yp), Zx], axis=-1),
        "z-": np.stack([Xz, Yz, np.full_like(Xz, zm)], axis=-1),
        "z+": np.stack([Xz, Yz, np.full_like(Xz, zp)], axis=-1),
    }
    return faces


def boundary_fold(h, eps_x, eps_y, eps_z, ghost):
    """Dirichlet values on the face ghosts moved to the right-hand side:
    node next to a ghost gets + eps_edge/h^2 * phi_ghost (Eq. 3 with the ghost
    potential known). `ghost` maps face -> values of shape (nz,ny)/(nz,nx)/(ny,nx)."""
    nz, ny, nxp1 = eps_x.shape
    nx = nxp1 - 1
    out = np.zeros((nz, ny, nx))
    ih2 = 1.0 / (h * h)
    out[:, :, 0] += eps_x[:, :, 0] * ih2 * ghost["x-"]
    out[:, :, nx - 1] += eps_x[:, :, nx] * ih2 * ghost["x+"]
    out[:, 0, :] += eps_y[:, 0, :] * ih2 * ghost["y-"]
    out[:, ny - 1, :] += eps_y[:, ny, :] * ih2 * ghost["y+"]
    out[0, :, :] += eps_z[0, :, :] * ih2 * ghost["z-"]
    out[nz - 1, :, :] += eps_z[nz, :, :] * ih2 * ghost["z+"]
    return out


def debye_huckel_ghosts(nx, ny, nz, h, origin, xyz, charge, eps_out, kappa_d2):
    faces = face_ghost_points(nx, ny, nz, h, origin)
    return {f: dh_potential(p, xyz, charge, eps_out, kappa_d2).reshape(p.shape[:-1])
            for f, p in faces.items()}


def assemble(nx, ny, nz, h, origin, xyz, radius, charge, eps_in, eps_out,
             kappa_d2, with_parts=False, edge_model="node"):
    """Full setup: classification, edges, salt, charges, boundary -> System.
    edge_model "node": two-point harmonic mean of the node values;
    "fraction": the fractional-edge weighted harmonic mean."""
    mask = classify(nx, ny, nz, h, origin, xyz, radius)
    if edge_model == "fraction":
        ex, ey, ez = fractional_edges(nx, ny, nz, h, origin, xyz, radius, eps_in, eps_out)
    else:
        ex, ey, ez = dielectric_edges(mask, eps_in, eps_out)
    k2 = salt_term(mask, eps_out, kappa_d2)
    q = spread_charges(nx, ny, nz, h, origin, xyz, charge)
    ghost = debye_huckel_ghosts(nx, ny, nz, h, origin, xyz, charge, eps_out, kappa_d2)
    b = FOUR_PI * q / h ** 3 + boundary_fold(h, ex, ey, ez, ghost)
    sysm = System(h=h, eps_x=ex, eps_y=ey, eps_z=ez, kappa2=k2, b=b)
    if with_parts:
        return sysm, dict(mask=mask, qgrid=q, ghost=ghost)
    return sysm


def assemble_problem(prob, with_parts=False):
    g = prob.grid
    return assemble(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius,
                    prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                    with_parts=with_parts)


# --------------------------------------------------------------------------
# Operator (Eq. 3) and energy
# --------------------------------------------------------------------------

def diagonal(s: System) -> np.ndarray:
    """A_nn = (sum of the six edge dielectrics)/h^2 + kbar^2."""
    ex, ey, ez = s.eps_x, s.eps_y, s.eps_z
    tot = ex[:, :, :-1] + ex[:, :, 1:] + ey[:, :-1, :] + ey[:, 1:, :] + ez[:-1] + ez[1:]
    return tot / (s.h * s.h) + s.kappa2


def apply(s: System, phi: np.ndarray) -> np.ndarray:
    """(A phi) of Eq. 3 with zero potential on the ghost layer."""
    phi = np.asarray(phi, np.float64).reshape(s.shape)
    nz, ny, nx = s.shape
    P = np.zeros((nz + 2, ny + 2, nx + 2))
    P[1:-1, 1:-1, 1:-1] = phi
    ex, ey, ez = s.eps_x, s.eps_y, s.eps_z
    nb = (ex[:, :, :-1] * P[1:-1, 1:-1, :-2] + ex[:, :, 1:] * P[1:-1, 1:-1, 2:]
          + ey[:, :-1, :] * P[1:-1, :-2, 1:-1] + ey[:, 1:, :] * P[1:-1, 2:, 1:-1]
          + ez[:-1] * P[:-2, 1:-1, 1:-1] + ez[1:] * P[2:, 1:-1, 1:-1])
    return diagonal(s) * phi - nb / (s.h * s.h)


def true_relres(s: System, phi: np.ndarray) -> float:
    """||b - A phi||_2 / ||b||_2 in FP64."""
    bn = float(np.linalg.norm(s.b.ravel()))
    if bn == 0.0:
        return float(np.linalg.norm(np.asarray(phi).ravel()) != 0.0)
    r = s.b - apply(s, phi)
    return float(np.linalg.norm(r.ravel())) / bn


def interpolate(nx, ny, nz, h, origin, xyz, phi) -> np.ndarray:
    """phi at each atom centre by the trilinear weights used for spreading."""
    idx, w = spread_weights(nx, ny, nz, h, origin, xyz)
    flat = np.asarray(phi, np.float64).ravel()
    return (w[:, :, 0] * w[:, :, 1] * w[:, :, 2] * flat[idx]).sum(axis=1)


def energy(nx, ny, nz, h, origin, xyz, charge, phi) -> float:
    """Electrostatic energy 1/2 sum_a q_a phi(c_a) in kcal/mol."""
    pa = interpolate(nx, ny, nz, h, origin, xyz, phi)
    return 0.5 * float(np.dot(np.asarray(charge, np.float64), pa)) * COULOMB_KCAL


# --------------------------------------------------------------------------
# Dense form (tiny grids only): independent index arithmetic
# --------------------------------------------------------------------------

def dense_matrix(s: System) -> np.ndarray:
    """Assemble A explicitly, row by row, from the edge arrays (Eq. 3)."""
    nx, ny, nz = s.dims
    n = nx * ny * nz
    if n > 4096:
        raise ValueError("dense assembly is for tiny grids only")
    A = np.zeros((n, n))
    ih2 = 1.0 / (s.h * s.h)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                row = i + nx * (j + ny * k)
                # (edge value, neighbour (i,j,k) or None for a ghost)
                edges = [
                    (s.eps_x[k, j, i], (i - 1, j, k)),
                    (s.eps_x[k, j, i + 1], (i + 1, j, k)),
                    (s.eps_y[k, j, i], (i, j - 1, k)),
                    (s.eps_y[k, j + 1, i], (i, j + 1, k)),
                    (s.eps_z[k, j, i], (i, j, k - 1)),
                    (s.eps_z[k + 1, j, i], (i, j, k + 1)),
                ]
                d = s.kappa2[k, j, i]
                for e, (a, bb, c) in edges:
                    d += e * ih2
                    if 0 <= a < nx and 0 <= bb < ny and 0 <= c < nz:
                        A[row, a + nx * (bb + ny * c)] -= e * ih2
                A[row, row] += d
    return A
