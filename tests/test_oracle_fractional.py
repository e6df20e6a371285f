"""Pins of the fractional-edge (weighted harmonic) dielectric of the oracle (CPU only).

- analytic chord fractions for one sphere on its centre line and off axis;
- overlapping spheres count their union, not the sum;
- the inside fraction agrees with dense midpoint sampling of random edges;
- eps is eps_out at f = 0, eps_in at f = 1, the weighted harmonic mean between;
- consistency with node classification (f = 1 edges have inside or surface
  endpoints, f = 0 edges have outside endpoints unless they only touch);
- the Born ion: the fractional edges cut the h = 0.5 finite-difference error
  below 1% where the two-point rule has 3.8% (a = 2.1) and 5.4% (a = 2.0, the
  radius with exact node ties), and the error falls with h.
"""
import math

import numpy as np
import pytest

from oracle import fdpb, pcg, solvation


def test_single_sphere_chords():
    n, h = 9, 0.5
    o = np.full(3, -(n - 1) / 2 * h)
    f = fdpb.edge_inside_fraction(n, n, n, h, o, np.zeros((1, 3)), np.array([1.3]), 0)
    # centre line: x-edges from -2.5+0.5e .. : [-1.5,-1.0] covers [-1.3,-1.0] -> 0.6
    assert np.allclose(f[4, 4, :], [0, 0, 0.6, 1, 1, 1, 1, 0.6, 0, 0], atol=1e-12)
    # off axis by 0.5 (j = 5): half chord sqrt(1.69 - 0.25) = 1.2
    w = math.sqrt(1.3 * 1.3 - 0.25)
    expect = []
    for e in range(n + 1):
        x0 = -2.0 + 0.5 * (e - 1)
        lo, hi = max(-w, x0), min(w, x0 + 0.5)
        expect.append(max(0.0, hi - lo) / 0.5)
    assert np.allclose(f[4, 5, :], expect, atol=1e-12)
    fy = fdpb.edge_inside_fraction(n, n, n, h, o, np.zeros((1, 3)), np.array([1.3]), 1)
    fz = fdpb.edge_inside_fraction(n, n, n, h, o, np.zeros((1, 3)), np.array([1.3]), 2)
    assert np.allclose(fy[4, :, 4], f[4, 4, :]) and np.allclose(fz[:, 4, 4], f[4, 4, :])


def test_union_not_sum():
    n, h = 11, 0.5
    o = np.full(3, -(n - 1) / 2 * h)
    xyz = np.array([[-0.9, 0.0, 0.0], [0.9, 0.0, 0.0]])
    R = np.array([1.0, 1.0])
    f = fdpb.edge_inside_fraction(n, n, n, h, o, xyz, R, 0)
    # centre line covered from -1.9 to 1.9 as one piece; the edge [-0.5, 0] is covered once
    assert abs(f[5, 5, 5] - 1.0) <= 1e-15 and f.max() <= 1.0
    line = f[5, 5, :]
    assert abs(line.sum() * 0.5 - 3.8) <= 1e-12


def test_fraction_matches_dense_sampling():
    rng = np.random.default_rng(3)
    n, h = 8, 0.5
    o = np.zeros(3)
    xyz = rng.uniform(0.5, 3.0, size=(5, 3))
    R = rng.uniform(0.6, 1.4, size=5)
    for axis in range(3):
        f = fdpb.edge_inside_fraction(n, n, n, h, o, xyz, R, axis)
        for _ in range(40):
            idx = [rng.integers(0, n), rng.integers(0, n), rng.integers(0, n)]
            idx[axis] = rng.integers(0, n + 1)
            k, j, i = idx[2], idx[1], idx[0]
            p0 = o + h * np.array([i, j, k], dtype=float)
            p0[axis] -= h
            ts = (np.arange(20000) + 0.5) / 20000
            pts = p0[None, :] + np.outer(ts, np.eye(3)[axis]) * h
            inside = np.zeros(len(ts), bool)
            for c, r in zip(xyz, R):
                inside |= ((pts - c) ** 2).sum(1) < r * r
            assert abs(f[k, j, i] - inside.mean()) <= 1e-4


def test_eps_limits_and_classification_consistency():
    rng = np.random.default_rng(9)
    n, h = 14, 0.5
    o = np.zeros(3)
    xyz = rng.uniform(1.5, 5.0, size=(8, 3))
    R = rng.uniform(1.2, 2.0, size=8)
    ex, ey, ez = fdpb.fractional_edges(n, n, n, h, o, xyz, R, 1.0, 80.0)
    mask = fdpb.classify(n, n, n, h, o, xyz, R)
    for axis, e in enumerate((ex, ey, ez)):
        f = fdpb.edge_inside_fraction(n, n, n, h, o, xyz, R, axis)
        assert np.all(e[f == 0.0] == 80.0) and np.all(e[f == 1.0] == 1.0)
        mid = (f > 0) & (f < 1)
        assert np.allclose(e[mid], 1.0 / (f[mid] + (1 - f[mid]) / 80.0))
        assert np.all((e >= 1.0) & (e <= 80.0))
        # endpoints of each edge in the padded mask
        m = mask.astype(bool)
        if axis == 0:
            a, b = m[1:-1, 1:-1, :-1], m[1:-1, 1:-1, 1:]
        elif axis == 1:
            a, b = m[1:-1, :-1, 1:-1], m[1:-1, 1:, 1:-1]
        else:
            a, b = m[:-1, 1:-1, 1:-1], m[1:, 1:-1, 1:-1]
        assert not np.any(a & b & (f == 0.0))     # both ends inside: the edge is (partly) covered
        assert not np.any(~a & ~b & (f == 1.0))   # fully covered: both ends inside (no exact ties here)


def _born(h, n, a, model):
    org = np.full(3, -(n - 1) / 2 * h)
    xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
    es = []
    for eo in (80.0, 1.0):
        s = fdpb.assemble(n, n, n, h, org, xyz, R, q, 1.0, eo, 0.0, edge_model=model)
        r = pcg.jpcg(s, 1e-10, maxiter=20000)
        es.append(fdpb.energy(n, n, n, h, org, xyz, q, r.x))
    return (es[0] - es[1]) / solvation.born_energy(1.0, a, 1.0, 80.0) - 1.0


def test_born_error_with_fractional_edges():
    e_node = abs(_born(0.5, 33, 2.1, "node"))
    e_frac = abs(_born(0.5, 33, 2.1, "fraction"))
    e_frac_fine = abs(_born(0.25, 49, 2.1, "fraction"))
    assert e_node > 0.03 and e_frac < 0.01 and e_frac_fine < e_frac
    assert abs(_born(0.5, 33, 2.0, "fraction")) < 0.01 < abs(_born(0.5, 33, 2.0, "node"))
