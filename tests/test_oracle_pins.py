"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against mathematics the paper's system must obey:
a dense direct solve, closed-form eigenpairs, the lattice Green's function of
a point charge, the Debye-Hueckel potential, the Born solvation energy,
symmetry / definiteness, conservation laws, an energy identity and scaling
invariances. They are chosen so that a dropped term, a wrong sign, a wrong
index or a transposed axis in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import fdpb, pcg, solvation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_system(nx, ny, nz, seed, h=0.5, kappa=True):
    """Random positive edge dielectrics, random salt, random right-hand side."""
    rng = np.random.default_rng(seed)
    ex = rng.uniform(1.0, 80.0, (nz, ny, nx + 1))
    ey = rng.uniform(1.0, 80.0, (nz, ny + 1, nx))
    ez = rng.uniform(1.0, 80.0, (nz + 1, ny, nx))
    k2 = rng.uniform(0.0, 2.0, (nz, ny, nx)) if kappa else np.zeros((nz, ny, nx))
    b = rng.standard_normal((nz, ny, nx))
    return fdpb.System(h=h, eps_x=ex, eps_y=ey, eps_z=ez, kappa2=k2, b=b)


def _uniform_system(nx, ny, nz, eps, k2, h):
    return fdpb.System(h=h, eps_x=np.full((nz, ny, nx + 1), eps),
                       eps_y=np.full((nz, ny + 1, nx), eps),
                       eps_z=np.full((nz + 1, ny, nx), eps),
                       kappa2=np.full((nz, ny, nx), k2), b=np.zeros((nz, ny, nx)))


# ---------------------------------------------------------------- V1 dense

@pytest.mark.parametrize("dims,seed", [((5, 7, 9), 1), ((4, 4, 4), 2), ((9, 3, 6), 3)])
def test_v1_dense_direct_solve(dims, seed):
    nx, ny, nz = dims
    s = _rand_system(nx, ny, nz, seed)
    A = fdpb.dense_matrix(s)
    # symmetric, exactly
    assert np.array_equal(A, A.T)
    # positive definite (Cholesky succeeds)
    np.linalg.cholesky(A)
    # Jacobi-scaled spectrum inside (0, 2)
    dinv = 1.0 / np.sqrt(np.diag(A))
    ev = np.linalg.eigvalsh(dinv[:, None] * A * dinv[None, :])
    assert ev.min() > 0.0 and ev.max() < 2.0
    # matrix-free apply == dense product
    v = np.random.default_rng(seed + 10).standard_normal(nx * ny * nz)
    assert np.allclose(fdpb.apply(s, v.reshape(s.shape)).ravel(), A @ v, rtol=0, atol=1e-12 * np.abs(A).max() * np.abs(v).max() * 7)
    # diagonal used by the preconditioner == dense diagonal
    assert np.allclose(fdpb.diagonal(s).ravel(), np.diag(A), rtol=1e-14, atol=0)
    # PCG to 1e-13 == direct solve
    xd = np.linalg.solve(A, s.b.ravel())
    errs = []
    res = pcg.jpcg(s, 1e-13, maxiter=5000,
                   callback=lambda l, x: errs.append(float((x.ravel() - xd) @ A @ (x.ravel() - xd))))
    assert res.converged
    assert np.abs(res.x.ravel() - xd).max() <= 1e-10 * np.abs(xd).max()
    # CG minimises the A-norm error: it never increases
    e = np.array(errs)
    assert (np.diff(e) <= 1e-12 * e[0]).all()


def test_v1_dense_on_molecule_setup():
    """The full setup path (classification, edges, salt, charges, boundary) on
    a 9x8x7 grid, solved densely and by Jacobi PCG."""
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-0.6, 0.6, (3, 3))
    rad = np.array([1.1, 0.9, 1.3])
    q = np.array([0.5, -0.2, -0.3])
    g = synth.centred_grid(xyz, 9, 8, 7)
    s = fdpb.assemble(9, 8, 7, g.h, g.origin, xyz, rad, q, 1.0, 80.0, synth.KAPPA_D2_150MM)
    A = fdpb.dense_matrix(s)
    xd = np.linalg.solve(A, s.b.ravel())
    res = pcg.jpcg(s, 1e-13)
    assert res.converged
    assert np.abs(res.x.ravel() - xd).max() <= 1e-10 * np.abs(xd).max()
    # the system has both dielectrics and the salt term somewhere
    assert set(np.unique(s.eps_x).round(6)) >= {1.0, 80.0, round(160.0 / 81.0, 6)}
    assert (s.kappa2 == 0).any() and (s.kappa2 > 0).any()


# ---------------------------------------------------------------- V2 manufactured

@pytest.mark.parametrize("dims,modes", [((11, 13, 17), (1, 2, 3)), ((16, 9, 12), (3, 1, 2))])
def test_v2_sin_mode_is_exact_eigenvector(dims, modes):
    nx, ny, nz = dims
    eps, k2, h = 3.5, 0.7, 0.5
    s = _uniform_system(nx, ny, nz, eps, k2, h)
    ax = [np.sin(math.pi * m * (np.arange(n) + 1) / (n + 1)) for m, n in zip(modes, dims)]
    v = ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :]
    lam = eps / h ** 2 * sum(4 * math.sin(math.pi * m / (2 * (n + 1))) ** 2
                             for m, n in zip(modes, dims)) + k2
    assert np.allclose(fdpb.apply(s, v), lam * v, rtol=0, atol=1e-12 * lam)
    s.b = lam * v
    res = pcg.jpcg(s, 1e-13)
    assert res.converged and res.iters <= 2
    assert np.abs(res.x - v).max() <= 1e-12


def test_v2_two_modes_and_plain_cg():
    nx, ny, nz = 10, 12, 14
    eps, k2, h = 2.0, 0.0, 0.25
    s = _uniform_system(nx, ny, nz, eps, k2, h)
    def mode(m):
        ax = [np.sin(math.pi * mm * (np.arange(n) + 1) / (n + 1)) for mm, n in zip(m, (nx, ny, nz))]
        lam = eps / h ** 2 * sum(4 * math.sin(math.pi * mm / (2 * (n + 1))) ** 2
                                 for mm, n in zip(m, (nx, ny, nz)))
        return ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :], lam
    v1, l1 = mode((1, 1, 1))
    v2, l2 = mode((2, 3, 1))
    s.b = l1 * v1 + 0.5 * l2 * v2
    for m in (fdpb.diagonal(s), None):   # Jacobi and plain CG (M = I)
        res = pcg.pcg(lambda v: fdpb.apply(s, v), s.b, m, 1e-13, 100)
        assert res.converged and res.iters <= 3
        assert np.abs(res.x - (v1 + 0.5 * v2)).max() <= 1e-11


def test_v2_linear_field_reproduced_through_boundary_fold():
    """kappa = 0, no charge, uniform eps: phi = a x + b y + c z is discrete
    harmonic, so Dirichlet data from it must be reproduced to solver accuracy.
    This pins the ghost positions, the fold into b and its 1/h^2 scale."""
    nx, ny, nz, h = 9, 12, 7, 0.4
    origin = np.array([1.0, -2.0, 0.5])
    s = _uniform_system(nx, ny, nz, 5.0, 0.0, h)
    a = np.array([0.3, -1.1, 0.7])
    lin = lambda p: p[..., 0] * a[0] + p[..., 1] * a[1] + p[..., 2] * a[2]
    faces = fdpb.face_ghost_points(nx, ny, nz, h, origin)
    ghost = {f: lin(p) for f, p in faces.items()}
    s.b = fdpb.boundary_fold(h, s.eps_x, s.eps_y, s.eps_z, ghost)
    res = pcg.jpcg(s, 1e-14, maxiter=2000)
    zz, yy, xx = np.meshgrid(origin[2] + h * np.arange(nz), origin[1] + h * np.arange(ny),
                             origin[0] + h * np.arange(nx), indexing="ij")
    exact = xx * a[0] + yy * a[1] + zz * a[2]
    assert np.abs(res.x - exact).max() <= 1e-10 * np.abs(exact).max()


# ---------------------------------------------------------------- V3 point charge

def _watson():
    for line in open(os.path.join(GOLDEN, "watson.txt")):
        if line.startswith("W "):
            return float(line.split()[1])
    raise AssertionError


def test_golden_watson_closed_form():
    w = math.sqrt(6) / (32 * math.pi ** 3) * math.gamma(1 / 24) * math.gamma(5 / 24) \
        * math.gamma(7 / 24) * math.gamma(11 / 24)
    assert abs(w - _watson()) < 1e-14


@pytest.fixture(scope="module")
def point_charge_65():
    n, h, eps = 65, 0.5, 80.0
    org = np.full(3, -(n - 1) / 2 * h)
    xyz = np.zeros((1, 3))
    s = fdpb.assemble(n, n, n, h, org, xyz, np.array([0.1]), np.array([1.0]), eps, eps, 0.0)
    res = pcg.jpcg(s, 1e-11)
    assert res.converged
    return res.x, n, h, eps


def test_v3_point_charge_lattice_green_function(point_charge_65):
    phi, n, h, eps = point_charge_65
    c = (n - 1) // 2
    target = 4.0 * math.pi * _watson() / 6.0       # 3.1759115...
    assert abs(phi[c, c, c] * eps * h / target - 1.0) < 1e-5


def test_v3_point_charge_far_field_is_coulomb(point_charge_65):
    phi, n, h, eps = point_charge_65
    c = (n - 1) // 2
    for m in (8, 12, 16, 24):
        for idx in ((c, c, c + m), (c, c + m, c), (c + m, c, c), (c - m, c, c)):
            assert abs(phi[idx] * eps * (m * h) - 1.0) <= 5e-3


def test_v3_debye_huckel_point_charge():
    n, h, eps = 65, 0.5, 80.0
    k2 = synth.KAPPA_D2_150MM
    org = np.full(3, -(n - 1) / 2 * h)
    s = fdpb.assemble(n, n, n, h, org, np.zeros((1, 3)), np.array([0.1]), np.array([1.0]),
                      eps, eps, k2)
    res = pcg.jpcg(s, 1e-11)
    c = (n - 1) // 2
    kd = math.sqrt(k2)
    for m in (8, 12, 16, 24):
        r = m * h
        exact = math.exp(-kd * r) / (eps * r)
        for idx in ((c, c, c + m), (c, c + m, c), (c + m, c, c)):
            assert abs(res.x[idx] / exact - 1.0) <= 1e-2
    # screening really acts: beyond a Debye length the potential is well below Coulomb
    assert res.x[c, c, c + 24] < 0.4 * 1.0 / (eps * 12.0)


# ---------------------------------------------------------------- V4 Born

def _born(h, n):
    a = 2.1
    org = np.full(3, -(n - 1) / 2 * h)
    xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
    sol = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10, maxiter=20000)
    return sol.dG, solvation.born_energy(1.0, a, 1.0, 80.0)


def test_v4_born_sphere_energy():
    dg1, exact = _born(0.5, 33)
    dg2, _ = _born(0.25, 49)
    assert abs(exact - (-78.0745)) < 1e-3
    assert abs(exact - (-fdpb.COULOMB_KCAL / (2 * 2.1) * (1 - 1 / 80.0))) < 1e-12
    e1, e2 = abs(dg1 / exact - 1), abs(dg2 / exact - 1)
    assert e1 <= 0.05
    assert e2 <= 0.01
    assert e2 < e1


def test_v4_solvation_limits():
    """dG vanishes when the solvent dielectric equals the solute's and there
    is no salt; it is negative and grows in magnitude with eps_out; two ions
    of opposite charge far apart (separation >> radii) solvate like two Born
    ions, each at its own Born value (within the h = 0.5 grid error); a
    neutral (zero-charge) set has dG = 0 exactly."""
    n, h, a = 33, 0.5, 2.1
    org = np.full(3, -(n - 1) / 2 * h)
    xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
    same = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 1.0, 0.0, tol=1e-10)
    assert abs(same.dG) <= 1e-9 * abs(same.e_ref)
    d4 = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 4.0, 0.0, tol=1e-10).dG
    d80 = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10).dG
    assert d80 < d4 < 0.0
    # the continuum ratio (1 - 1/4)/(1 - 1/80) holds up to the grid error
    assert abs((d4 / d80) / (0.75 / (1 - 1 / 80.0)) - 1) < 0.03
    zero = solvation.solvation_energy(n, n, n, h, org, xyz, R, np.zeros(1), 1.0, 80.0, 0.0, tol=1e-10)
    assert zero.dG == 0.0 and zero.iters_solv == 0 and zero.iters_ref == 0
    # two opposite unit ions 10 A apart: in the continuum picture dG is twice the
    # single-ion value plus the change of their pair energy, +q^2/d (1 - 1/eps_out);
    # each ion's field polarising the other's cavity adds a few percent
    n2 = 49
    org2 = np.full(3, -(n2 - 1) / 2 * h)
    single = solvation.solvation_energy(n2, n2, n2, h, org2, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10).dG
    xyz2 = np.array([[-5.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    pair = solvation.solvation_energy(n2, n2, n2, h, org2, xyz2, np.array([a, a]), np.array([1.0, -1.0]),
                                      1.0, 80.0, 0.0, tol=1e-10).dG
    cross = fdpb.COULOMB_KCAL * (1.0 - 1.0 / 80.0) / 10.0
    assert abs(pair - (2 * single + cross)) <= 0.05 * abs(2 * single)


# ---------------------------------------------------------------- V5 SPD at scale

def test_v5_symmetry_definiteness_dominance_config0():
    p = synth.config0()
    s = fdpb.assemble_problem(p)
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal(s.shape), rng.standard_normal(s.shape)
    xay, yax = float((x * fdpb.apply(s, y)).sum()), float((y * fdpb.apply(s, x)).sum())
    assert abs(xay - yax) <= 1e-14 * abs(xay) * 10
    assert float((x * fdpb.apply(s, x)).sum()) > 0
    # diagonal >= sum |off-diagonal|; strictly where a ghost edge or salt exists
    d = fdpb.diagonal(s)
    ex, ey, ez, ih2 = s.eps_x, s.eps_y, s.eps_z, 1 / s.h ** 2
    off = np.zeros(s.shape)
    off[:, :, 1:] += ex[:, :, 1:-1] * ih2
    off[:, :, :-1] += ex[:, :, 1:-1] * ih2
    off[:, 1:, :] += ey[:, 1:-1, :] * ih2
    off[:, :-1, :] += ey[:, 1:-1, :] * ih2
    off[1:] += ez[1:-1] * ih2
    off[:-1] += ez[1:-1] * ih2
    assert (d >= off * (1 - 1e-15)).all()
    assert (d[0] > off[0]).all() and (d[:, :, -1] > off[:, :, -1]).all()
    # p^T A p > 0 along the whole Jacobi PCG run (no breakdown)
    res = pcg.jpcg(s, 1e-8)
    assert res.converged and not res.breakdown


# ---------------------------------------------------------------- V6 charges

def test_v6_charge_and_dipole_conservation():
    p = synth.config0()
    g = p.grid
    q = fdpb.spread_charges(g.nx, g.ny, g.nz, g.h, g.origin, p.mol.xyz, p.mol.charge)
    qa = p.mol.charge
    scale = np.abs(qa).sum()
    assert abs(q.sum() - qa.sum()) <= 1e-12 * scale
    zz, yy, xx = np.meshgrid(g.origin[2] + g.h * np.arange(g.nz), g.origin[1] + g.h * np.arange(g.ny),
                             g.origin[0] + g.h * np.arange(g.nx), indexing="ij")
    for coord, d in ((xx, 0), (yy, 1), (zz, 2)):
        assert abs((q * coord).sum() - (qa * p.mol.xyz[:, d]).sum()) <= 1e-12 * scale * 20


def test_spreading_on_node_and_top_edge():
    org = np.zeros(3)
    xyz = np.array([[1.0, 1.5, 0.5], [2.0, 2.0, 2.0]])    # a node; the top corner node
    q = fdpb.spread_charges(5, 5, 5, 0.5, org, xyz, np.array([0.3, -0.7]))
    assert q[1, 3, 2] == 0.3 and q[4, 4, 4] == -0.7
    assert np.count_nonzero(q) == 2
    with pytest.raises(ValueError):
        fdpb.spread_charges(5, 5, 5, 0.5, org, np.array([[2.01, 1.0, 1.0]]), np.array([1.0]))


# ---------------------------------------------------------------- V7 energy identity

def test_v7_energy_identity():
    p = synth.config0()
    g = p.grid
    s, parts = fdpb.assemble_problem(p, with_parts=True)
    phi = pcg.jpcg(s, 1e-8).x
    e_atoms = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, p.mol.xyz, p.mol.charge, phi)
    e_nodes = 0.5 * float((parts["qgrid"] * phi).sum()) * fdpb.COULOMB_KCAL
    assert abs(e_atoms - e_nodes) <= 1e-13 * abs(e_nodes) * 10


# ---------------------------------------------------------------- V8 scaling

def test_v8_scaling_is_bitwise_and_linear():
    s = fdpb.assemble_problem(synth.small_problem(13, 11, 9, 6, seed=11))
    r1 = pcg.jpcg(s, 1e-8)
    s2 = fdpb.System(h=s.h, eps_x=s.eps_x * 8, eps_y=s.eps_y * 8, eps_z=s.eps_z * 8,
                     kappa2=s.kappa2 * 8, b=s.b * 8)
    r2 = pcg.jpcg(s2, 1e-8)
    assert r1.iters == r2.iters and np.array_equal(r1.x, r2.x)
    s3 = fdpb.System(h=s.h, eps_x=s.eps_x, eps_y=s.eps_y, eps_z=s.eps_z, kappa2=s.kappa2, b=s.b * 3.0)
    r3 = pcg.jpcg(s3, 1e-10)
    r1b = pcg.jpcg(s, 1e-10)
    assert np.abs(r3.x - 3.0 * r1b.x).max() <= 1e-8 * np.abs(r3.x).max()


def test_v8_mirror_symmetry():
    p = synth.small_problem(15, 13, 11, 8, seed=12)
    g = p.grid
    s = fdpb.assemble_problem(p)
    # mirror x about the grid centre: node i -> nx-1-i
    cx = g.origin[0] + 0.5 * g.h * (g.nx - 1)
    xyz = p.mol.xyz.copy()
    xyz[:, 0] = 2 * cx - xyz[:, 0]
    sm = fdpb.assemble(g.nx, g.ny, g.nz, g.h, g.origin, xyz, p.mol.radius, p.mol.charge,
                       p.eps_in, p.eps_out, p.kappa_d2)
    a = pcg.jpcg(s, 1e-11).x
    b = pcg.jpcg(sm, 1e-11).x
    assert np.abs(a[:, :, ::-1] - b).max() <= 1e-8 * np.abs(a).max()


# ---------------------------------------------------------------- setup pieces

def test_classification_brute_force_and_ties():
    # radius 2.0 A at h = 0.5 centred on a node: nodes at distance exactly
    # 2.0 (4 h) are on the surface and count as outside (strict test).
    n, h = 13, 0.5
    org = np.full(3, -3.0)
    m = fdpb.classify(n, n, n, h, org, np.zeros((1, 3)), np.array([2.0]))
    brute = 0
    for k in range(-1, n + 1):
        for j in range(-1, n + 1):
            for i in range(-1, n + 1):
                x, y, z = org[0] + h * i, org[1] + h * j, org[2] + h * k
                brute += (x * x + y * y + z * z) < 4.0
    assert int(m.sum()) == brute
    # integer points with i^2+j^2+k^2 < 16: count by hand-free enumeration
    pts = sum(1 for i in range(-4, 5) for j in range(-4, 5) for k in range(-4, 5)
              if i * i + j * j + k * k < 16)
    assert int(m.sum()) == pts
    assert m[7, 7, 6 + 4 + 1] == 0   # node (4,0,0)*h from the centre is outside


def test_dielectric_edge_values():
    mask = np.zeros((3, 3, 4), np.uint8)
    mask[1, 1, 1] = 1    # one inside node in a 2x1x1 interior
    ex, ey, ez = fdpb.dielectric_edges(mask, 1.0, 80.0)
    assert ex.shape == (1, 1, 3)
    assert ex[0, 0, 0] == 2 * 80.0 / 81.0 and ex[0, 0, 1] == 2 * 80.0 / 81.0 and ex[0, 0, 2] == 80.0
    assert ey[0, 0, 0] == 2 * 80.0 / 81.0 and ey[0, 0, 1] == 80.0


def test_dh_reduces_to_coulomb_and_superposes():
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-2, 2, (5, 3))
    q = rng.uniform(-1, 1, 5)
    pts = rng.uniform(5, 9, (7, 3))
    d = np.linalg.norm(pts[:, None, :] - xyz[None, :, :], axis=-1)
    assert np.allclose(fdpb.dh_potential(pts, xyz, q, 4.0, 0.0), (q / (4.0 * d)).sum(1), rtol=1e-14)
    k2 = 0.02
    both = fdpb.dh_potential(pts, xyz, q, 80.0, k2)
    parts = fdpb.dh_potential(pts, xyz[:2], q[:2], 80.0, k2) + fdpb.dh_potential(pts, xyz[2:], q[2:], 80.0, k2)
    assert np.allclose(both, parts, rtol=1e-13)


# ---------------------------------------------------------------- PCG edge cases

def test_pcg_edge_cases():
    s = _rand_system(6, 5, 4, 21)
    assert pcg.jpcg(s, 1.5).iters == 0            # tol > 1: no iteration
    assert pcg.jpcg(s, 1.0).iters == 1            # strict "<": 1/1 is not below 1
    s0 = _rand_system(6, 5, 4, 21)
    s0.b[:] = 0
    r0 = pcg.jpcg(s0, 1e-6)
    assert r0.iters == 0 and not r0.x.any()       # zero rhs: x = 0
    r1 = pcg.jpcg(s, 1e-12, maxiter=3)
    assert not r1.converged and r1.iters == 3
    # warm start from the converged solution stops immediately
    r2 = pcg.jpcg(s, 1e-8)
    r3 = pcg.jpcg(s, 1e-8, x0=r2.x)
    assert r3.iters <= 1


def test_refinement_reaches_tight_tolerance():
    s = fdpb.assemble_problem(synth.small_problem(17, 15, 13, 10, seed=4))
    x, outer, inner, rel = pcg.refine(s, 1e-12, 1e-4)
    assert rel < 1e-12 and 2 <= outer <= 6
    assert fdpb.true_relres(s, x) < 1e-12


def test_refinement_stop_rules():
    """Refinement's outer stop rules, driven by inner solvers of known
    contraction: a correction c * A^-1 r leaves the residual (1 - c) r, so
    c = 0.4 (residual falls 1.67x) stagnates at the first check, c = 0.6
    (2.5x) keeps going until max_outer, an exact inner solve converges after
    one correction, and an FP32-rounded inner solve (a 2^-24 relative
    floor per step) converges geometrically."""
    s = fdpb.assemble_problem(synth.small_problem(7, 6, 5, 4, seed=12))
    A = fdpb.dense_matrix(s)
    exact = lambda rhs: np.linalg.solve(A, rhs.ravel()).reshape(s.shape)

    def scaled(c):
        return lambda rhs, t: pcg.PCGResult(c * exact(rhs), 1, 0.0, True)

    x, outer, inner, rel, st = pcg.refine(s, 1e-12, inner_solver=scaled(0.4), with_status=True)
    assert st == "stagnated" and outer == 1 and len(inner) == 1
    bn = np.linalg.norm(s.b)
    assert abs(rel - 0.6) <= 1e-12 and abs(np.linalg.norm(s.b - fdpb.apply(s, x)) / bn - 0.6) <= 1e-12
    x, outer, inner, rel, st = pcg.refine(s, 1e-12, inner_solver=scaled(0.6), max_outer=7, with_status=True)
    assert st == "max_outer" and outer == 7 and len(inner) == 7
    assert abs(rel / 0.4 ** 7 - 1.0) <= 1e-9
    x, outer, inner, rel, st = pcg.refine(s, 1e-12, inner_solver=scaled(1.0), with_status=True)
    assert st == "converged" and outer == 1 and rel < 1e-13

    def fp32_inner(rhs, t):
        d = exact(rhs.astype(np.float32).astype(np.float64)).astype(np.float32).astype(np.float64)
        return pcg.PCGResult(d, 1, 0.0, True)

    x, outer, inner, rel, st = pcg.refine(s, 1e-13, inner_solver=fp32_inner, with_status=True)
    assert st == "converged" and 2 <= outer <= 4, (outer, rel)

    def broken(rhs, t):
        return pcg.PCGResult(np.zeros(s.shape), 0, 1.0, False, breakdown=True)

    x, outer, inner, rel, st = pcg.refine(s, 1e-12, inner_solver=broken, with_status=True)
    assert st == "breakdown" and outer == 0 and not x.any()
    # the default return shape is unchanged
    assert len(pcg.refine(s, 1e-10)) == 4
