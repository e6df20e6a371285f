"""Pins of the multigrid oracle (CPU only).

- restriction is exactly the transpose of trilinear prolongation over 8
  (dense matrices from unit vectors), for odd and even grid sizes;
- a uniform medium coarsens to itself (coarse edges = eps, kbar^2 kept), a
  medium layered along x coarsens along x by the series (harmonic) rule;
- one V-cycle is a symmetric positive definite operator (u.Mv = v.Mu,
  v.Mv > 0) on a molecular system with 1/80 dielectric jumps and salt;
- MG-PCG iteration counts for the uniform Laplacian stay flat as n doubles,
  while Jacobi-PCG's grow about linearly;
- MG-PCG reaches the same solution as Jacobi-PCG on a molecular system.
"""
import numpy as np
import pytest

import synth
from oracle import fdpb, multigrid as mg, pcg


def _dense(fn, in_shape):
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(fn(e.reshape(in_shape))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("fine", [(7, 6, 5), (5, 5, 5), (8, 7, 6)])
def test_restriction_is_transpose_of_prolongation(fine):
    nz, ny, nx = fine
    coarse = (nz // 2, ny // 2, nx // 2)
    P = _dense(lambda v: mg.prolong(v, fine), coarse)
    R = _dense(lambda v: mg.restrict(v, coarse), fine)
    assert np.abs(R - P.T / 8.0).max() <= 1e-15
    # prolongation reproduces constants away from the Dirichlet ghosts (odd fine nodes)
    ones = mg.prolong(np.ones(coarse), fine)
    assert np.allclose(ones[1:2 * coarse[0]:2, 1:2 * coarse[1]:2, 1:2 * coarse[2]:2], 1.0)


def test_uniform_and_layered_media_coarsen_exactly():
    nx, ny, nz = 9, 8, 7
    s = fdpb.System(h=0.5, eps_x=np.full((nz, ny, nx + 1), 80.0), eps_y=np.full((nz, ny + 1, nx), 80.0),
                    eps_z=np.full((nz + 1, ny, nx), 80.0), kappa2=np.full((nz, ny, nx), 1.27),
                    b=np.zeros((nz, ny, nx)))
    c = mg.coarsen_system(s)
    assert c.h == 1.0 and c.dims == (4, 4, 3)
    for arr in (c.eps_x, c.eps_y, c.eps_z):
        assert np.abs(arr - 80.0).max() <= 1e-12
    assert np.abs(c.kappa2 - 1.27).max() <= 1e-12
    # layers along x: every fine x-edge e has dielectric eps_e on every line
    rng = np.random.default_rng(2)
    layer = rng.choice([1.0, 80.0], size=nx + 1)
    ex = np.broadcast_to(layer, (nz, ny, nx + 1)).copy()
    s2 = fdpb.System(h=0.5, eps_x=ex, eps_y=s.eps_y, eps_z=s.eps_z, kappa2=s.kappa2, b=s.b)
    c2 = mg.coarsen_system(s2)
    for E in range(c2.dims[0] + 1):
        e1 = layer[2 * E]
        e2 = layer[2 * E + 1] if 2 * E + 1 <= nx else e1
        assert abs(c2.eps_x[0, 0, E] - 2 * e1 * e2 / (e1 + e2)) <= 1e-12


def test_vcycle_is_symmetric_positive_definite():
    prob = synth.small_problem(21, 19, 17, 25, seed=4)
    s = fdpb.assemble_problem(prob)
    levels = mg.hierarchy(s, min_nodes=64)
    assert len(levels) >= 3
    rng = np.random.default_rng(5)
    for _ in range(3):
        u, v = rng.standard_normal(s.shape), rng.standard_normal(s.shape)
        Mu, Mv = mg.vcycle(levels, 0, u), mg.vcycle(levels, 0, v)
        assert abs(float((u * Mv).sum()) - float((v * Mu).sum())) <= 1e-12 * abs(float((u * Mu).sum()))
        assert float((v * Mv).sum()) > 0.0


def test_iterations_flat_in_n_for_uniform_laplacian():
    its_mg, its_j = [], []
    for n in (15, 31, 63):
        rng = np.random.default_rng(n)
        s = fdpb.System(h=0.5, eps_x=np.ones((n, n, n + 1)), eps_y=np.ones((n, n + 1, n)),
                        eps_z=np.ones((n + 1, n, n)), kappa2=np.zeros((n, n, n)), b=rng.standard_normal((n, n, n)))
        res, levels = mg.mgpcg(s, 1e-8)
        assert res.converged and len(levels) == {15: 2, 31: 3, 63: 4}[n]
        its_mg.append(res.iters)
        its_j.append(pcg.jpcg(s, 1e-8, maxiter=5000).iters)
    assert max(its_mg) <= 10 and max(its_mg) - min(its_mg) <= 2
    assert its_j[2] > 3 * its_j[0]


def test_mgpcg_matches_jacobi_pcg_on_molecule():
    prob = synth.config0()
    s = fdpb.assemble_problem(prob)
    res, levels = mg.mgpcg(s, 1e-10)
    ref = pcg.jpcg(s, 1e-12, maxiter=5000)
    assert res.converged and res.iters <= 25
    assert np.abs(res.x - ref.x).max() <= 1e-8 * np.abs(ref.x).max()
    assert fdpb.true_relres(s, res.x) < 1e-9
