"""Seeded synthetic inputs for the linear FDPB solve (protein-like stand-ins).

This module only *draws inputs*: atom centres, radii, charges, grid edge and
origin. It holds none of the method's arithmetic (no classification, no
dielectric, no charge spreading, no boundary values, no solve), so both the
FP64 oracle and the GPU path may import it.

The paper measures on 573 Amber benchmark structures (247-8,254 atoms, Cornell
charges, modified bond radii; section 2.7). Those structures are not available
here, so seeded random-walk chains confined to a sphere stand in for them, with
the paper's grid spacing (0.5 A), dielectrics (1 inside, 80 outside), initial
guess (zero) and tolerances (1e-3 / 1e-6) from section 2.7. Grid sizes follow
the 0.74-2.6M-node range of Table 2.

Readings of the workload definitions (where the stated sizes do not fit the
stated boxes) are documented next to each config below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

H = 0.5                 # grid spacing, A (section 2.7)
EPS_IN = 1.0            # solute dielectric (section 2.7)
EPS_OUT = 80.0          # solvent dielectric (section 2.7)
BOND = 1.5              # random-walk step, A
RADIUS_RANGE = (1.2, 2.0)
CHARGE_RANGE = (-0.8, 0.8)

# Debye screening constant of a 1:1 salt (input construction, not solver math).
_NA = 6.02214076e23
_E = 1.602176634e-19
_EPS0 = 8.8541878128e-12
_KB = 1.380649e-23


def debye_kappa2(ionic_strength_molar: float, eps_out: float = EPS_OUT,
                 temperature: float = 298.15) -> float:
    """kappa_D^2 in A^-2 for a 1:1 electrolyte: 2 N_A e^2 (1000 I) / (eps0 eps kT)."""
    si = 2.0 * _NA * _E ** 2 * (1000.0 * ionic_strength_molar) / (
        _EPS0 * eps_out * _KB * temperature)
    return si * 1e-20


KAPPA_D2_150MM = debye_kappa2(0.15)   # ~0.0159051 A^-2 (Debye length ~7.93 A)


@dataclasses.dataclass
class Molecule:
    xyz: np.ndarray      # (natoms, 3) float64, A
    radius: np.ndarray   # (natoms,) float64, A
    charge: np.ndarray   # (natoms,) float64, e; sums to ~0

    @property
    def natoms(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    h: float
    origin: np.ndarray   # (3,) float64; node (i,j,k) sits at origin + h*(i,j,k)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Problem:
    name: str
    mol: Molecule
    grid: Grid
    eps_in: float = EPS_IN
    eps_out: float = EPS_OUT
    kappa_d2: float = KAPPA_D2_150MM
    tol: float = 1e-6
    precision: str = "f32"          # "f64" | "f32" | "f32_refine64"
    seed: int = 0


def random_walk(natoms: int, r_conf: float, rng: np.random.Generator,
                step: float = BOND) -> np.ndarray:
    """Chain a_0 = 0, a_{k+1} = a_k + step * u, u a normalised Gaussian draw,
    redrawn while the new point would leave the sphere |a| <= r_conf."""
    if r_conf < step:
        raise ValueError("confinement radius must exceed the bond length")
    out = np.zeros((natoms, 3))
    cur = np.zeros(3)
    for a in range(1, natoms):
        for _ in range(10000):
            u = rng.standard_normal(3)
            nrm = math.sqrt(float(u @ u))
            if nrm == 0.0:
                continue
            cand = cur + step * (u / nrm)
            if float(cand @ cand) <= r_conf * r_conf:
                break
        else:  # pragma: no cover - practically unreachable for r_conf >= step
            cand = cur - step * cur / max(math.sqrt(float(cur @ cur)), 1e-30)
        cur = cand
        out[a] = cur
    return out


def molecule(natoms: int, r_conf: float, seed: int) -> Molecule:
    rng = np.random.default_rng(seed)
    xyz = random_walk(natoms, r_conf, rng)
    radius = rng.uniform(RADIUS_RANGE[0], RADIUS_RANGE[1], natoms)
    charge = rng.uniform(CHARGE_RANGE[0], CHARGE_RANGE[1], natoms)
    charge = charge - charge.mean()
    return Molecule(xyz=xyz, radius=radius, charge=charge)


def centred_grid(xyz: np.ndarray, nx: int, ny: Optional[int] = None,
                 nz: Optional[int] = None, h: float = H) -> Grid:
    """Grid whose centre is the bounding-box midpoint of the atom centres."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    mid = 0.5 * (xyz.min(axis=0) + xyz.max(axis=0))
    half = 0.5 * h * (np.array([nx, ny, nz], dtype=np.float64) - 1.0)
    return Grid(nx, ny, nz, h, (mid - half).astype(np.float64))


def fits(mol: Molecule, grid: Grid, margin_nodes: float = 1.0) -> bool:
    """Every sphere stays at least `margin_nodes`*h inside the node box."""
    lo = grid.origin
    hi = grid.origin + grid.h * (np.array([grid.nx, grid.ny, grid.nz]) - 1.0)
    m = margin_nodes * grid.h
    ok_lo = (mol.xyz - mol.radius[:, None] >= lo + m).all()
    ok_hi = (mol.xyz + mol.radius[:, None] <= hi - m).all()
    return bool(ok_lo and ok_hi)


def extent(mol: Molecule) -> float:
    """Largest edge of the bounding box of the spheres, A."""
    lo = (mol.xyz - mol.radius[:, None]).min(axis=0)
    hi = (mol.xyz + mol.radius[:, None]).max(axis=0)
    return float((hi - lo).max())


# --------------------------------------------------------------------------
# The five workloads. Seeds are 1000*config + snapshot.
# --------------------------------------------------------------------------

def config0() -> Problem:
    """33^3, 50-atom chain, FP64, tol 1e-6. A free 50-step walk does not fit
    the 16 A box, so the walk is confined to R0 = 0.5(n-1)h - r_max - h = 5.5 A."""
    n = 33
    r0 = 0.5 * (n - 1) * H - RADIUS_RANGE[1] - H
    mol = molecule(50, r0, seed=0)
    return Problem("c0_33", mol, centred_grid(mol.xyz, n), tol=1e-6,
                   precision="f64", seed=0)


def config1() -> Problem:
    """129^3, 2,000-atom chain confined to a 24 A sphere, FP32, tol 1e-6."""
    mol = molecule(2000, 24.0, seed=1000)
    return Problem("c1_129", mol, centred_grid(mol.xyz, 129), tol=1e-6,
                   precision="f32", seed=1000)


def config2() -> Problem:
    """257^3, 20,000-atom chain confined to 24*10^(1/3) = 51.7 A (same atom
    density as config 1); FP32 inner 1e-4 inside an FP64 outer loop to 1e-9."""
    mol = molecule(20000, 24.0 * 10.0 ** (1.0 / 3.0), seed=2000)
    return Problem("c2_257", mol, centred_grid(mol.xyz, 257), tol=1e-9,
                   precision="f32_refine64", seed=2000)


C3_EDGES = (65, 97, 129, 161)


def c3_radius(n: int) -> float:
    """A 24 A, 2,000-atom globule does not fit 65^3 or 97^3 at h = 0.5, so the
    globule for edge n is compacted to R_n = 0.5(n-1)h/1.5 - 2 A, keeping the
    paper's grid/solute ratio of 1.5 (section 2.7)."""
    return 0.5 * (n - 1) * H / 1.5 - 2.0


def config3(nsnap: int = 256, natoms: int = 2000, sigma: float = 0.3) -> List[Problem]:
    """Snapshots with a seeded grid edge from {65,97,129,161}; each is one of
    four base globules (one per edge) perturbed by Gaussian noise sigma."""
    rng = np.random.default_rng(3000)
    edges = rng.choice(np.array(C3_EDGES), size=nsnap)
    base = {n: molecule(natoms, c3_radius(n), seed=3900 + n) for n in C3_EDGES}
    out = []
    for s in range(nsnap):
        n = int(edges[s])
        b = base[n]
        srng = np.random.default_rng(3000 + s + 1)
        xyz = b.xyz + sigma * srng.standard_normal(b.xyz.shape)
        mol = Molecule(xyz=xyz, radius=b.radius.copy(), charge=b.charge.copy())
        out.append(Problem(f"c3_{s}_{n}", mol, centred_grid(xyz, n), tol=1e-6,
                           precision="f32", seed=3000 + s + 1))
    return out


C4_TOLS = (1e-4, 1e-6, 1e-8)


def config4_request(idx: int) -> Problem:
    """One serving request: atom count log-uniform in [500, 30000], chain
    confined to R(N) = 22 A (N/30000)^(1/3), edge n = clamp(2 ceil(E/h)+1, 49,
    193) for the sphere extent E (box >= 2E), tol from {1e-4, 1e-6, 1e-8}
    (1e-8 solved with FP64 refinement)."""
    rng = np.random.default_rng(4000 + idx)
    natoms = int(round(math.exp(rng.uniform(math.log(500.0), math.log(30000.0)))))
    tol = float(C4_TOLS[int(rng.integers(0, 3))])
    mol = molecule(natoms, 22.0 * (natoms / 30000.0) ** (1.0 / 3.0), seed=4000 + idx)
    e = extent(mol)
    n = int(min(max(2 * math.ceil(e / H) + 1, 49), 193))
    prec = "f32_refine64" if tol < 1e-6 else "f32"
    return Problem(f"c4_{idx}_{n}", mol, centred_grid(mol.xyz, n), tol=tol,
                   precision=prec, seed=4000 + idx)


_C4_BASE = {}


def config4_molecule(idx: int, pool: int = 64, sigma: float = 0.3) -> Problem:
    """A distinct molecule for serving request `idx`: request idx % pool of
    config 4 (its atom count, radii, charges, grid and tolerance) with every
    atom moved by seeded Gaussian noise of sigma A, as config 3 perturbs its
    snapshots. Drawing whole new chains for thousands of requests would cost
    minutes of host time; the perturbation keeps each request's coordinates
    its own. The config-4 box (at least twice the extent) keeps every sphere
    inside the node box."""
    key = idx % pool
    if key not in _C4_BASE:
        _C4_BASE[key] = config4_request(key)
    base = _C4_BASE[key]
    rng = np.random.default_rng(4000 + 100000 + idx)
    xyz = base.mol.xyz + sigma * rng.standard_normal(base.mol.xyz.shape)
    mol = Molecule(xyz=xyz, radius=base.mol.radius.copy(), charge=base.mol.charge.copy())
    return Problem(f"c4m_{idx}_{base.grid.nx}", mol, base.grid, tol=base.tol, precision=base.precision,
                   seed=4000 + 100000 + idx)


def config4_arrivals(nreq: int, rate: float = 200.0, seed: int = 4999) -> np.ndarray:
    """Poisson arrival times (s) at `rate` requests/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=nreq))


def small_problem(nx: int, ny: int, nz: int, natoms: int, seed: int,
                  kappa_d2: float = KAPPA_D2_150MM, precision: str = "f64",
                  tol: float = 1e-6) -> Problem:
    """A ragged test problem: chain confined so every sphere keeps a 1h margin."""
    half = 0.5 * H * (min(nx, ny, nz) - 1)
    r_conf = max(half - RADIUS_RANGE[1] - H, BOND)
    mol = molecule(natoms, r_conf, seed)
    return Problem(f"small_{nx}x{ny}x{nz}_{seed}", mol,
                   centred_grid(mol.xyz, nx, ny, nz), kappa_d2=kappa_d2,
                   tol=tol, precision=precision, seed=seed)


def config(i: int):
    return {0: config0, 1: config1, 2: config2, 3: config3}[i]()
