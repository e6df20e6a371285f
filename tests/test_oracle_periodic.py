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
