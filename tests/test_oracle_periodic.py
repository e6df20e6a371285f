"""Pins of the periodic-boundary oracle against mathematics (CPU only).

- the matrix-free operator equals a dense matrix built by explicit wrapped
  index arithmetic, which is symmetric, annihilates constants without salt,
  and is positive definite with salt;
- for a uniform dielectric and salt term the discrete Fourier transform
  diagonalises the operator: the JPCG solution equals the FFT solution
  (with and without salt, zero-mean convention in the singular case);
- classification equals a brute-force test of every node against every
  periodic image of every sphere;
- spreading conserves charge and dipole (modulo the period) and wraps;
- a molecule moved by one period gives the same system.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import fdpb, periodic


def _rand_system(nx, ny, nz, seed, kbar2):
    rng = np.random.default_rng(seed)
    e = rng.choice([1.0, 80.0], size=(nz, ny, nx))
    ep = np.pad(e, 1, mode="wrap")
    ex = fdpb.harmonic(ep[1:-1, 1:-1, :-1], ep[1:-1, 1:-1, 1:])
    ey = fdpb.harmonic(ep[1:-1, :-1, 1:-1], ep[1:-1, 1:, 1:-1])
    ez = fdpb.harmonic(ep[:-1, 1:-1, 1:-1], ep[1:, 1:-1, 1:-1])
    k2 = np.where(e > 1.0, kbar2, 0.0)
    b = rng.standard_normal((nz, ny, nx))
    return fdpb.System(h=0.5, eps_x=ex, eps_y=ey, eps_z=ez, kappa2=k2, b=b)


@pytest.mark.parametrize("dims,seed", [((3, 4, 5), 0), ((5, 3, 4), 1), ((4, 4, 3), 2)])
def test_operator_equals_dense_wrapped_matrix(dims, seed):
    s = _rand_system(*dims, seed, 1.27)
    A = periodic.dense_matrix(s)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    v = np.random.default_rng(seed + 10).standard_normal(s.shape)
    assert np.allclose(periodic.apply(s, v).ravel(), A @ v.ravel(), rtol=0, atol=1e-10 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0.0            # salt outside: definite
    s0 = _rand_system(*dims, seed, 0.0)
    A0 = periodic.dense_matrix(s0)
    one = np.ones(A0.shape[0])
    assert np.abs(A0 @ one).max() <= 1e-12 * np.abs(A0).max()
    ev = np.linalg.eigvalsh(A0)
    assert abs(ev[0]) <= 1e-10 * ev[-1] and ev[1] > 1e-6 * ev[-1]   # one-dimensional null space


@pytest.mark.parametrize("kbar2", [1.272407, 0.0])
def test_uniform_medium_matches_fft(kbar2):
    nx, ny, nz, h, eps = 12, 10, 9, 0.5, 80.0
    rng = np.random.default_rng(3)
    b = rng.standard_normal((nz, ny, nx))
    if kbar2 == 0.0:
        b -= b.mean()
    ex = np.full((nz, ny, nx + 1), eps)
    ey = np.full((nz, ny + 1, nx), eps)
    ez = np.full((nz + 1, ny, nx), eps)
    s = fdpb.System(h=h, eps_x=ex, eps_y=ey, eps_z=ez, kappa2=np.full((nz, ny, nx), kbar2), b=b)
    res = periodic.jpcg(s, 1e-13, maxiter=5000)
    assert res.converged
    ref = periodic.fft_solve(b, h, eps, kbar2)
    if kbar2 == 0.0:
        assert abs(res.x.mean()) <= 1e-14 * np.abs(ref).max() + 1e-300
    assert np.abs(res.x - ref).max() <= 1e-10 * np.abs(ref).max()
    # the FFT solution satisfies the periodic operator itself
    assert np.abs(periodic.apply(s, ref) - b).max() <= 1e-10 * np.abs(b).max()


def test_classification_matches_brute_force_over_images():
    nx, ny, nz, h = 9, 8, 7, 0.5
    origin = np.array([0.1, -0.3, 0.2])
    L = np.array([nx, ny, nz]) * h
    xyz = np.array([[0.2, 0.0, 0.3], [4.3, 3.6, 3.2], [2.0, 1.9, -0.4], [9.0, -2.0, 7.5]])
    rad = np.array([1.3, 1.1, 1.7, 0.9])
    mask = periodic.classify(nx, ny, nz, h, origin, xyz, rad)
    brute = np.zeros_like(mask)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        x = origin + h * np.array([i, j, k], dtype=np.float64)
        for c, r in zip(xyz, rad):
            for m in itertools.product((-2, -1, 0, 1, 2), repeat=3):
                d = x - (c + np.array(m) * L)
                if float(d @ d) < r * r:
                    brute[k, j, i] = 1
    assert (mask == brute).all(), np.argwhere(mask != brute)
    assert mask.sum() > 0 and mask[0].any() and mask[-1].any()   # spheres wrap across the z faces


def test_spreading_wraps_and_conserves():
    nx, ny, nz, h = 8, 9, 10, 0.5
    origin = np.zeros(3)
    xyz = np.array([[3.9, 0.05, 4.95], [-0.2, 2.0, 1.0], [1.0, 1.0, 1.0]])
    q = np.array([0.7, -0.4, 0.25])
    g = periodic.spread_charges(nx, ny, nz, h, origin, xyz, q)
    assert abs(g.sum() - q.sum()) <= 1e-15
    # the first atom sits in the last cell along x and z: weight reaches node 0
    assert g[0, :, :].any() and g[:, :, 0].any()
    # moving an atom by one period leaves the grid unchanged up to rounding
    g2 = periodic.spread_charges(nx, ny, nz, h, origin, xyz + np.array([nx * h, 0.0, -nz * h]), q)
    assert np.abs(g2 - g).max() <= 1e-12


def test_assembled_system_shift_by_period_and_singular_mean():
    nx, ny, nz, h = 12, 11, 10, 0.5
    origin = np.array([-2.7, -2.5, -2.2])
    rng = np.random.default_rng(7)
    xyz = rng.uniform(-2.0, 2.0, size=(6, 3))
    rad = rng.uniform(1.2, 1.8, size=6)
    q = rng.uniform(-0.8, 0.8, size=6)
    s = periodic.assemble(nx, ny, nz, h, origin, xyz, rad, q, 1.0, 80.0, 0.0)
    assert abs(s.b.mean()) <= 1e-14 * np.abs(s.b).max()          # neutralising background
    s2 = periodic.assemble(nx, ny, nz, h, origin, xyz + np.array([0.0, ny * h, 0.0]), rad, q, 1.0, 80.0, 0.0)
    assert np.abs(s2.b - s.b).max() <= 1e-10 * np.abs(s.b).max()
    salty = periodic.assemble(nx, ny, nz, h, origin, xyz, rad, q, 1.0, 80.0, 0.0159051)
    assert not periodic.is_singular(salty.kappa2)
    r0 = periodic.jpcg(s, 1e-10)
    r1 = periodic.jpcg(salty, 1e-10)
    assert r0.converged and r1.converged
    assert abs(r0.x.mean()) <= 1e-12 * np.abs(r0.x).max()
    assert periodic.true_relres(s, r0.x) < 1e-9 and periodic.true_relres(salty, r1.x) < 1e-9


def test_interpolation_matches_library_on_tiled_field():
    """periodic.interpolate equals scipy's trilinear interpolation of the
    periodically tiled field (3 copies per axis), for atoms inside the box,
    in its last cell (between node n-1 and node 0), below the origin and
    beyond the far face."""
    from scipy.interpolate import RegularGridInterpolator
    nx, ny, nz, h = 7, 6, 5, 0.5
    origin = np.array([0.3, -0.2, 0.1])
    rng = np.random.default_rng(21)
    phi = rng.standard_normal((nz, ny, nx))
    tiled = np.tile(phi, (3, 3, 3))                  # nodes -n .. 2n-1 on each axis
    axes = [origin[d] + h * np.arange(-n, 2 * n, dtype=np.float64) for d, n in enumerate((nx, ny, nz))]
    f = RegularGridInterpolator((axes[2], axes[1], axes[0]), tiled, method="linear")
    L = np.array([nx, ny, nz]) * h
    xyz = np.concatenate([origin + rng.uniform(0, 1, size=(20, 3)) * L,
                          origin + (np.array([nx, ny, nz]) - 0.5) * h + rng.uniform(-0.2, 0.2, size=(5, 3)),
                          origin + rng.uniform(-0.9, -0.01, size=(5, 3)) * L,
                          origin + rng.uniform(1.01, 1.75, size=(5, 3)) * L])
    got = periodic.interpolate(nx, ny, nz, h, origin, xyz, phi)
    want = f(xyz[:, ::-1])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(phi).max()


def test_energy_identity_and_period_shift():
    """1/2 sum_a q_a phi(c_a) equals 1/2 sum_nodes q_node phi_node with the
    wrapped spreading (the same trilinear weights used as a scatter instead of
    a gather), and moving every atom by whole periods leaves it unchanged."""
    nx, ny, nz, h = 9, 8, 10, 0.5
    origin = np.array([-2.0, -1.7, -2.4])
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-4.0, 4.0, size=(12, 3))
    q = rng.uniform(-0.8, 0.8, size=12)
    phi = rng.standard_normal((nz, ny, nx))
    e = periodic.energy(nx, ny, nz, h, origin, xyz, q, phi)
    qn = periodic.spread_charges(nx, ny, nz, h, origin, xyz, q)
    e_nodes = 0.5 * float(np.sum(qn * phi)) * fdpb.COULOMB_KCAL
    assert abs(e - e_nodes) <= 1e-13 * abs(e_nodes)
    shift = np.array([nx, -2 * ny, 3 * nz]) * h
    assert abs(periodic.energy(nx, ny, nz, h, origin, xyz + shift, q, phi) - e) <= 1e-11 * abs(e)


def test_solvation_zero_for_uniform_dielectric():
    """With eps_out = eps_in and no salt the solvent and reference systems of
    the periodic solvation energy are the same system: dG = 0 exactly."""
    from oracle import solvation
    prob = synth.small_problem(15, 13, 14, 6, seed=3)
    g, m = prob.grid, prob.mol
    r = solvation.solvation_energy(g.nx, g.ny, g.nz, g.h, g.origin, m.xyz, m.radius, m.charge, 2.0, 2.0, 0.0,
                                   tol=1e-10, boundary="periodic")
    assert r.dG == 0.0 and r.e_solv != 0.0


def _wigner_constant():
    """xi of a unit charge in a cubic periodic box (side 1) with a uniform
    neutralising background: minus the Ewald sum of the potential its images
    and the background create at the charge (real-space erfc terms,
    reciprocal-space Gaussian terms, the self term and the background
    term, splitting parameter 5)."""
    from math import erfc, exp, pi, sqrt
    a = 5.0
    real = sum(erfc(a * sqrt(i * i + j * j + k * k)) / sqrt(i * i + j * j + k * k)
               for i in range(-4, 5) for j in range(-4, 5) for k in range(-4, 5) if (i, j, k) != (0, 0, 0))
    recip = 0.0
    for i in range(-8, 9):
        for j in range(-8, 9):
            for k in range(-8, 9):
                if (i, j, k) != (0, 0, 0):
                    k2 = (2 * pi) ** 2 * (i * i + j * j + k * k)
                    recip += 4 * pi / k2 * exp(-k2 / (4 * a * a))
    return -(real + recip - 2 * a / sqrt(pi) - pi / (a * a))


def test_periodic_born_ion_finite_size_correction():
    """A Born ion (radius 2.1 A, eps 1 inside / 80 outside, no salt) in a
    periodic box of side L: each system's energy carries the lattice
    self-energy -q^2 xi / (2 eps L) of its medium, so the periodic dG equals
    the free-space dG on the same grid plus 332.06 q^2 xi / (2L) (1 - 1/80)
    (28 kcal/mol at L = 16.5 A), up to an O(L^-3) remainder. Checked at
    n = 33 and 41: the remainder stays below 1.2% and falls like L^-3."""
    from oracle import solvation
    xi = _wigner_constant()
    assert abs(xi - 2.837297) < 1e-6
    rel = {}
    for n in (33, 41):
        h, a = 0.5, 2.1
        org = np.full(3, -(n - 1) / 2 * h)
        xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
        per = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10, boundary="periodic")
        free = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10)
        corr = fdpb.COULOMB_KCAL * xi / (2 * n * h) * (1.0 - 1.0 / 80.0)
        rel[n] = (per.dG - (free.dG + corr)) / abs(free.dG)
    assert abs(rel[33]) < 0.012 and abs(rel[41]) < 0.006
    ratio = rel[41] / rel[33]
    assert 0.8 * (33 / 41) ** 3 < ratio < 1.2 * (33 / 41) ** 3, rel
