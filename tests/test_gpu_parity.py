"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars (stated here, derived in the design notes):
  * setup integer/byte outputs (mask) and the edge dielectrics, salt term and
    spread charges: bitwise equal (same FP64 operations, no contraction);
  * right-hand side: max-norm relative difference <= 1e-12 (the boundary sum
    over atoms runs in a different order);
  * FP64 solves: true relative residual < 1e-6 at tol 1e-6 and the potential
    within 1e-8 (relative to max|phi|) of the oracle's own iterate, and within
    1e-12 of the oracle's iterate after the same number of iterations;
  * FP32 solves: true relative residual <= 1e-5 and max|phi - phi*| /
    max|phi*| <= 1e-5 against the oracle solved to 1e-12;
  * refinement: true relative residual below the requested 1e-10 and
    potential error <= 1e-9;
  * iteration counts within max(2, 2%) of the oracle's Jacobi PCG.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import fdpb, pcg, solvation

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pb():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1704_02745_amd as m
    return m


def gpu_setup(pb, prob, **kw):
    g = prob.grid
    return pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out,
                    prob.kappa_d2, device=DEV, **kw)


def to_system(pb, s: fdpb.System, origin=(0.0, 0.0, 0.0)):
    nx, ny, nz = s.dims
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    return pb.System(pb.make_grid(nx, ny, nz, s.h, origin), t(s.eps_x), t(s.eps_y), t(s.eps_z),
                     t(s.kappa2), t(s.b))


def rand_system(nx, ny, nz, seed, h=0.5):
    rng = np.random.default_rng(seed)
    return fdpb.System(h=h, eps_x=rng.uniform(1, 80, (nz, ny, nx + 1)),
                       eps_y=rng.uniform(1, 80, (nz, ny + 1, nx)),
                       eps_z=rng.uniform(1, 80, (nz + 1, ny, nx)),
                       kappa2=rng.uniform(0, 2, (nz, ny, nx)), b=rng.standard_normal((nz, ny, nx)))


def iters_close(a, b):
    return abs(a - b) <= max(2, math.ceil(0.02 * b))


# ------------------------------------------------------------------ setup

SETUP_CASES = [
    ("c0", synth.config0),
    ("ragged", lambda: synth.small_problem(37, 29, 23, 20, seed=5)),
    ("ragged_nosalt", lambda: synth.small_problem(26, 41, 19, 9, seed=6, kappa_d2=0.0)),
]


@pytest.mark.parametrize("name,make", SETUP_CASES, ids=[c[0] for c in SETUP_CASES])
def test_setup_matches_oracle(pb, name, make):
    prob = make()
    print(f"case {name} dims {prob.grid.nx}x{prob.grid.ny}x{prob.grid.nz}", flush=True)
    sysm = gpu_setup(pb, prob, want_q=True, want_mask=True)
    ref, parts = fdpb.assemble_problem(prob, with_parts=True)
    assert np.array_equal(sysm.mask.cpu().numpy(), parts["mask"])
    assert np.array_equal(sysm.eps_x.cpu().numpy(), ref.eps_x)
    assert np.array_equal(sysm.eps_y.cpu().numpy(), ref.eps_y)
    assert np.array_equal(sysm.eps_z.cpu().numpy(), ref.eps_z)
    assert np.array_equal(sysm.kappa2.cpu().numpy(), ref.kappa2)
    assert np.array_equal(sysm.qgrid.cpu().numpy(), parts["qgrid"])
    b = sysm.rhs.cpu().numpy()
    assert np.abs(b - ref.b).max() <= 1e-12 * np.abs(ref.b).max()
    # interior nodes carry no boundary term: bitwise equal there
    assert np.array_equal(b[1:-1, 1:-1, 1:-1], ref.b[1:-1, 1:-1, 1:-1])


def test_setup_full_size_129(pb):
    """Config-1 sizes (129^3, 2,000 atoms): everything but the boundary sum
    compared in full; the boundary nodes on a seeded sample."""
    prob = synth.config1()
    g = prob.grid
    sysm = gpu_setup(pb, prob, want_q=True, want_mask=True)
    mask = fdpb.classify(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius)
    assert np.array_equal(sysm.mask.cpu().numpy(), mask)
    ex, ey, ez = fdpb.dielectric_edges(mask, prob.eps_in, prob.eps_out)
    assert np.array_equal(sysm.eps_x.cpu().numpy(), ex)
    assert np.array_equal(sysm.eps_z.cpu().numpy(), ez)
    assert np.array_equal(sysm.kappa2.cpu().numpy(), fdpb.salt_term(mask, prob.eps_out, prob.kappa_d2))
    q = fdpb.spread_charges(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.charge)
    assert np.array_equal(sysm.qgrid.cpu().numpy(), q)
    b = sysm.rhs.cpu().numpy()
    interior = fdpb.FOUR_PI * q / g.h ** 3
    assert np.array_equal(b[1:-1, 1:-1, 1:-1], interior[1:-1, 1:-1, 1:-1])
    # sampled x- face nodes: b = 4 pi q/h^3 + eps_x(edge 0)/h^2 * phi_DH(ghost)
    rng = np.random.default_rng(1)
    js, ks = rng.integers(1, g.ny - 1, 64), rng.integers(1, g.nz - 1, 64)   # face interior only
    pts = np.stack([np.full(64, g.origin[0] + g.h * -1.0), g.origin[1] + g.h * js, g.origin[2] + g.h * ks], -1)
    phi = fdpb.dh_potential(pts, prob.mol.xyz, prob.mol.charge, prob.eps_out, prob.kappa_d2)
    expect = interior[ks, js, 0] + ex[ks, js, 0] * (1.0 / (g.h * g.h)) * phi
    got = b[ks, js, 0]
    assert np.abs(got - expect).max() <= 1e-12 * np.abs(b).max()


# ------------------------------------------------------------------ solves

@pytest.fixture(scope="module")
def c0(pb):
    prob = synth.config0()
    ref = fdpb.assemble_problem(prob)
    return prob, ref, gpu_setup(pb, prob)


@pytest.mark.parametrize("op", ["stencil", "dia"])
def test_fp64_solve_config0(pb, c0, op):
    prob, ref, sysm = c0
    o = pcg.jpcg(ref, 1e-6)
    x, info = pb.solve(sysm, tol=1e-6, precision="f64", op=op)
    xg = x.cpu().numpy()
    print(f"c0 f64 {op}: gpu iters {info['iters']} oracle {o.iters}", flush=True)
    assert info["status"] == pb.PB_OK
    assert iters_close(info["iters"], o.iters)
    assert info["relres_recur"] < 1e-6
    rel = fdpb.true_relres(ref, xg)
    assert rel < 1e-6 and abs(info["relres_true"] - rel) <= 1e-3 * rel
    scale = np.abs(o.x).max()
    assert np.abs(xg - o.x).max() <= 1e-8 * scale
    exact = pcg.jpcg(ref, 1e-12).x
    assert np.abs(xg - exact).max() <= 1e-5 * scale
    # the oracle's iterate after the same number of iterations: equal up to the
    # order of the sums (FP64 rounding, ~1e-16 relative per operation)
    same = pcg.jpcg(ref, 1e-300, maxiter=info["iters"]).x
    d = np.abs(xg - same).max() / scale
    print(f"c0 f64 {op}: against the oracle's iterate {info['iters']}: {d:.3e}", flush=True)
    assert d <= 1e-12


@pytest.fixture(scope="module")
def ragged(pb):
    prob = synth.small_problem(61, 53, 47, 300, seed=9, precision="f32")
    ref = fdpb.assemble_problem(prob)
    exact = pcg.jpcg(ref, 1e-13, maxiter=20000).x
    o6 = pcg.jpcg(ref, 1e-6)
    return prob, ref, gpu_setup(pb, prob), exact, o6


@pytest.mark.parametrize("op", ["stencil", "dia"])
def test_fp32_solve_ragged(pb, ragged, op):
    prob, ref, sysm, exact, o6 = ragged
    x, info = pb.solve(sysm, tol=1e-6, precision="f32", op=op)
    xg = x.cpu().numpy()
    print(f"ragged f32 {op}: gpu iters {info['iters']} oracle {o6.iters} "
          f"relres_true {info['relres_true']:.3e}", flush=True)
    assert info["status"] == pb.PB_OK
    assert iters_close(info["iters"], o6.iters)
    assert fdpb.true_relres(ref, xg) <= 1e-5
    assert np.abs(xg - exact).max() <= 1e-5 * np.abs(exact).max()


@pytest.mark.parametrize("op", ["stencil", "dia"])
def test_refinement_ragged(pb, ragged, op):
    prob, ref, sysm, exact, _ = ragged
    x, info = pb.solve(sysm, tol=1e-10, precision="f32_refine64", op=op)
    xg = x.cpu().numpy()
    print(f"ragged refine {op}: outer {info['outer_iters']} inner {info['iters']} "
          f"relres_true {info['relres_true']:.3e}", flush=True)
    assert info["status"] == pb.PB_OK and 2 <= info["outer_iters"] <= 8
    rel = fdpb.true_relres(ref, xg)
    assert rel < 1e-10
    assert np.abs(xg - exact).max() <= 1e-9 * np.abs(exact).max()


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 1), (1, 5, 7), (7, 1, 1), (9, 4, 3), (70, 3, 5),
                                  (3, 67, 2), (130, 2, 9)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_degenerate_and_thin_grids(pb, dims, prec):
    s = rand_system(*dims, seed=sum(dims))
    o = pcg.jpcg(s, 1e-8, maxiter=5000)
    x, info = pb.solve(to_system(pb, s), tol=1e-8 if prec == "f64" else 1e-5, precision=prec,
                       maxiter=5000)
    xg = x.cpu().numpy()
    bound = 1e-7 if prec == "f64" else 1e-4
    assert np.abs(xg - o.x).max() <= bound * np.abs(o.x).max()


def test_energy_matches_oracle(pb, c0):
    prob, ref, sysm = c0
    g = prob.grid
    x, _ = pb.solve(sysm, tol=1e-8, precision="f64")
    atom_phi = torch.empty(prob.mol.natoms, dtype=torch.float64, device=DEV)
    e = pb.energy(g, prob.mol.xyz, prob.mol.charge, x, atom_phi=atom_phi)
    xs = x.cpu().numpy()
    e_ref = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.charge, xs)
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    pa = fdpb.interpolate(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, xs)
    assert np.abs(atom_phi.cpu().numpy() - pa).max() <= 1e-14 * np.abs(pa).max()


# ------------------------------------------------------------------ edge cases

def test_zero_rhs_and_loose_tolerance(pb, c0):
    prob, ref, sysm = c0
    z = pb.System(sysm.grid, sysm.eps_x, sysm.eps_y, sysm.eps_z, sysm.kappa2, torch.zeros_like(sysm.rhs))
    for prec in ("f64", "f32", "f32_refine64"):
        x0 = torch.ones_like(sysm.rhs)
        x, info = pb.solve(z, tol=1e-6, precision=prec, x0=x0)
        assert info["iters"] == 0 and not x.any(), prec
    x, info = pb.solve(sysm, tol=2.0, precision="f32")
    assert info["iters"] == 0 and not x.any()


def test_maxiter_and_warm_start(pb, c0):
    prob, ref, sysm = c0
    x, info = pb.solve(sysm, tol=1e-6, precision="f64", maxiter=1, check=False)
    assert info["status"] == pb.PB_NOT_CONVERGED and info["iters"] == 1
    o1 = pcg.jpcg(ref, 1e-6, maxiter=1)
    assert np.abs(x.cpu().numpy() - o1.x).max() <= 1e-10 * np.abs(o1.x).max()
    xc, _ = pb.solve(sysm, tol=1e-7, precision="f64")
    x2, info2 = pb.solve(sysm, tol=1e-6, precision="f64", x0=xc)
    assert info2["iters"] == 0
    # a warm start from a partly converged iterate continues
    xw, _ = pb.solve(sysm, tol=1e-2, precision="f64")
    x3, info3 = pb.solve(sysm, tol=1e-6, precision="f64", x0=xw)
    o3 = pcg.jpcg(ref, 1e-6, x0=xw.cpu().numpy())
    assert iters_close(info3["iters"], o3.iters)


def test_bad_inputs(pb, c0):
    prob, ref, sysm = c0
    bad = pb.System(sysm.grid, -sysm.eps_x, sysm.eps_y, sysm.eps_z, sysm.kappa2, sysm.rhs)
    with pytest.raises(pb.PBError) as e:
        pb.solve(bad, tol=1e-6)
    assert e.value.status == pb.PB_ERR_ARG
    nanb = sysm.rhs.clone()
    nanb[3, 4, 5] = float("nan")
    with pytest.raises(pb.PBError) as e:
        pb.solve(pb.System(sysm.grid, sysm.eps_x, sysm.eps_y, sysm.eps_z, sysm.kappa2, nanb), tol=1e-6)
    assert e.value.status == pb.PB_ERR_NONFINITE
    # the binding replaces too-small workspaces, so call the ABI directly
    import ctypes
    o = pb.SolveOpts()
    o.tol, o.precision = 1e-6, 1
    ws = torch.empty(4096, dtype=torch.uint8, device=DEV)
    x = torch.empty_like(sysm.rhs)
    st = pb.lib.pb_solve(33, 33, 33, 0.5, pb._ptr(sysm.eps_x), pb._ptr(sysm.eps_y), pb._ptr(sysm.eps_z),
                         pb._ptr(sysm.kappa2), pb._ptr(sysm.rhs), pb._ptr(x), ctypes.byref(o), pb._ptr(ws),
                         4096, pb._stream(), None)
    assert st == pb.PB_ERR_NOMEM
    # an atom outside the box
    g = prob.grid
    xyz = prob.mol.xyz.copy()
    xyz[0, 0] = g.origin[0] - 3.0
    with pytest.raises(pb.PBError) as e:
        pb.setup(g, xyz, prob.mol.radius, prob.mol.charge, device=DEV)
    assert e.value.status == pb.PB_ERR_ARG


def test_determinism(pb, ragged):
    prob, ref, sysm, exact, _ = ragged
    for prec in ("f32", "f64"):
        a, ia = pb.solve(sysm, tol=1e-6, precision=prec)
        b, ib = pb.solve(sysm, tol=1e-6, precision=prec)
        assert ia["iters"] == ib["iters"] and torch.equal(a, b), prec
    s1 = gpu_setup(pb, prob)
    s2 = gpu_setup(pb, prob)
    assert torch.equal(s1.rhs, s2.rhs)


# ------------------------------------------------------------------ full sizes

def test_full_size_129_stencil_and_dia(pb):
    """Config 1: 129^3 FP32 at tol 1e-6 in both forms; the oracle checks the
    FP64 true residual of each result."""
    prob = synth.config1()
    sysm = gpu_setup(pb, prob)
    s = fdpb.System(h=prob.grid.h, eps_x=sysm.eps_x.cpu().numpy(), eps_y=sysm.eps_y.cpu().numpy(),
                    eps_z=sysm.eps_z.cpu().numpy(), kappa2=sysm.kappa2.cpu().numpy(), b=sysm.rhs.cpu().numpy())
    its = {}
    for op in ("stencil", "dia"):
        x, info = pb.solve(sysm, tol=1e-6, precision="f32", op=op)
        rel = fdpb.true_relres(s, x.cpu().numpy())
        print(f"c1 {op}: iters {info['iters']} relres_true {rel:.3e} ({info['seconds']*1e3:.1f} ms)", flush=True)
        assert info["status"] == pb.PB_OK and rel <= 1e-5
        its[op] = info["iters"]
    assert iters_close(its["stencil"], its["dia"])


def test_full_size_257_refinement(pb):
    """Config 2: 257^3, 20,000 atoms, FP32 inner 1e-4 / FP64 outer to 1e-9."""
    prob = synth.config2()
    g = prob.grid
    sysm = gpu_setup(pb, prob)
    x, info = pb.solve(sysm, tol=1e-9, precision="f32_refine64", inner_tol=1e-4)
    s = fdpb.System(h=g.h, eps_x=sysm.eps_x.cpu().numpy(), eps_y=sysm.eps_y.cpu().numpy(),
                    eps_z=sysm.eps_z.cpu().numpy(), kappa2=sysm.kappa2.cpu().numpy(), b=sysm.rhs.cpu().numpy())
    xs = x.cpu().numpy()
    rel = fdpb.true_relres(s, xs)
    print(f"c2 refine: outer {info['outer_iters']} inner {info['iters']} relres_true {rel:.3e} "
          f"({info['seconds']*1e3:.1f} ms)", flush=True)
    assert info["status"] == pb.PB_OK and rel < 1e-9
    e = pb.energy(g, prob.mol.xyz, prob.mol.charge, x)
    e_ref = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.charge, xs)
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)


def test_autotune_then_solve(pb, ragged):
    """The autotuner times every feasible tiling; the recorded winner is used
    by later solves, which must still match the oracle."""
    prob, ref, sysm, exact, o6 = ragged
    for prec in ("f32", "f64"):
        best = pb.autotune(sysm, precision=prec, iters_per_trial=5)
        print(f"autotune {prec}: {best}", flush=True)
        assert best["candidates"] >= 1 and best["us_per_iter"] > 0
        x, info = pb.solve(sysm, tol=1e-6, precision=prec)
        assert iters_close(info["iters"], o6.iters)
        assert np.abs(x.cpu().numpy() - exact).max() <= 1e-5 * np.abs(exact).max()
        nx, ny, nz = sysm.dims
        pb.set_tuning(nx, ny, nz, prec, best["block"], best["groups"], best["zchunk"], best["grid"], best["scheme"],
                      best["streaming"], best["segments"])
    with pytest.raises(pb.PBError):
        pb.set_tuning(61, 53, 47, "f32", 256, 1, 1, 3)   # infeasible grid size


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_tiling_and_pass_form(pb, ragged, prec):
    """Every feasible launch shape of the fused kernel, both pass forms (the
    pass that stores A.p and the 40-byte pass that recomputes it) and both
    access kinds (cached, streaming), solves the ragged system to the oracle's
    exact solution in the oracle's iteration count; the two forms give the same
    iterates up to rounding, and the two access kinds of one launch shape give
    bitwise the same result."""
    prob, ref, sysm, exact, o6 = ragged
    nx, ny, nz = sysm.dims
    cands = pb.tiling_candidates(nx, ny, nz, prec)
    assert {c["scheme"] for c in cands} == {0, 1}, cands
    assert {c["streaming"] for c in cands} == {0, 1}, cands
    xs = {}
    by_shape = {}
    try:
        for c in cands:
            pb.set_tuning(nx, ny, nz, prec, c["block"], c["groups"], c["zchunk"], c["grid"], c["scheme"],
                          c["streaming"], c["segments"])
            print(f"tiling {prec} {c}", flush=True)
            x, info = pb.solve(sysm, tol=1e-6, precision=prec)
            assert info["status"] == pb.PB_OK
            assert iters_close(info["iters"], o6.iters), (c, info["iters"], o6.iters)
            xv = x.cpu().numpy()
            assert np.abs(xv - exact).max() <= 1e-5 * np.abs(exact).max(), c
            xs.setdefault(c["scheme"], []).append(xv)
            shape = (c["block"], c["groups"], c["zchunk"], c["grid"], c["scheme"], c["segments"])
            if shape in by_shape:
                assert np.array_equal(by_shape[shape], xv), c
            by_shape[shape] = xv
    finally:
        best = pb.autotune(sysm, precision=prec, iters_per_trial=3)   # leave a recorded winner behind
    a, b = xs[0][0], xs[1][0]
    assert np.abs(a - b).max() <= 1e-6 * np.abs(exact).max()


# ------------------------------------------------------------------ solvation energy

@pytest.fixture(scope="module")
def born_case():
    n, h, a = 33, 0.5, 2.1
    org = np.full(3, -(n - 1) / 2 * h)
    xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
    sol = solvation.solvation_energy(n, n, n, h, org, xyz, R, q, 1.0, 80.0, 0.0, tol=1e-10)
    return n, h, org, xyz, R, q, sol


@pytest.mark.parametrize("prec,tol,rel", [("f64", 1e-10, 1e-7), ("f32_refine64", 1e-10, 1e-7),
                                          ("f32", 1e-6, 1e-3)])
def test_solvation_born_ion(pb, born_case, prec, tol, rel):
    """One unit ion: the two-solve dG equals the oracle's discrete value and
    lies within the h = 0.5 grid error of Born's formula."""
    n, h, org, xyz, R, q, sol = born_case
    g = pb.make_grid(n, n, n, h, org)
    r = pb.solvation_energy(g, xyz, R, q, 1.0, 80.0, 0.0, tol=tol, precision=prec)
    print(f"born {prec}: gpu {r['dG']:.9f} oracle {sol.dG:.9f} "
          f"iters {r['info_solv']['iters']}/{r['info_ref']['iters']}", flush=True)
    assert r["status"] == pb.PB_OK
    assert abs(r["dG"] - sol.dG) <= rel * abs(sol.dG)
    assert abs(r["dG"] / solvation.born_energy(1.0, 2.1, 1.0, 80.0) - 1) <= 0.05
    assert abs(r["e_solv"] - r["e_ref"] - r["dG"]) <= 1e-12 * abs(r["e_ref"])


def test_solvation_molecule_with_salt(pb, c0):
    """Config-0 molecule (50 atoms, salt): dG from the GPU matches the
    oracle's two FP64 solves; the returned potentials give the same energies
    through pb_energy."""
    prob = c0[0]
    g = prob.grid
    sol = solvation.solvation_energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius,
                                     prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2, tol=1e-10)
    r = pb.solvation_energy(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out,
                            prob.kappa_d2, tol=1e-10, precision="f64", want_phi=True)
    print(f"c0 dG gpu {r['dG']:.9f} oracle {sol.dG:.9f}", flush=True)
    assert abs(r["dG"] - sol.dG) <= 1e-7 * abs(sol.dG)
    assert iters_close(r["info_solv"]["iters"], sol.iters_solv)
    assert iters_close(r["info_ref"]["iters"], sol.iters_ref)
    e_s = pb.energy(g, prob.mol.xyz, prob.mol.charge, r["phi_solv"])
    assert e_s == r["e_solv"]
    assert np.abs(r["phi_ref"].cpu().numpy() - sol.phi_ref).max() <= 1e-8 * np.abs(sol.phi_ref).max()


@pytest.mark.parametrize("prec,tol,bar", [("f64", 1e-10, 1e-7), ("f32_refine64", 1e-10, 1e-7)])
def test_solvation_molecule_multigrid(pb, c0, prec, tol, bar):
    """The same dG with both solves preconditioned by the multigrid V-cycle:
    within the bar of the oracle's two Jacobi-PCG solves, with far fewer
    iterations for the uniform reference."""
    prob = c0[0]
    g = prob.grid
    sol = solvation.solvation_energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius,
                                     prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2, tol=1e-10)
    r = pb.solvation_energy(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out,
                            prob.kappa_d2, tol=tol, precision=prec, op="mg")
    print(f"c0 dG mg {prec}: gpu {r['dG']:.9f} oracle {sol.dG:.9f} iters {r['info_solv']['iters']}/"
          f"{r['info_ref']['iters']} (oracle JPCG {sol.iters_solv}/{sol.iters_ref})", flush=True)
    assert r["status"] == pb.PB_OK
    assert abs(r["dG"] - sol.dG) <= bar * abs(sol.dG)
    assert r["info_ref"]["iters"] * 5 < sol.iters_ref


# ------------------------------------------------------------------ batched form

BATCH_SHAPES = [(37, 29, 23, 20), (45, 45, 45, 60), (21, 30, 17, 8), (64, 9, 33, 12), (33, 33, 65, 40)]


@pytest.fixture(scope="module")
def batch_set(pb):
    probs = [synth.small_problem(nx, ny, nz, na, seed=100 + i) for i, (nx, ny, nz, na) in enumerate(BATCH_SHAPES)]
    refs = [fdpb.assemble_problem(p) for p in probs]
    exact = [pcg.jpcg(r, 1e-13, maxiter=20000).x for r in refs]
    o6 = [pcg.jpcg(r, 1e-6) for r in refs]
    systems = [gpu_setup(pb, p) for p in probs]
    return probs, refs, exact, o6, systems


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_oracle_and_is_mix_independent(pb, batch_set, prec):
    probs, refs, exact, o6, systems = batch_set
    xs, infos = pb.solve_batch(systems, tol=1e-6, precision=prec)
    for i in range(len(systems)):
        xg = xs[i].cpu().numpy()
        print(f"batch {prec} #{i} {BATCH_SHAPES[i][:3]}: iters {infos[i]['iters']} oracle {o6[i].iters} "
              f"relres_true {infos[i]['relres_true']:.2e}", flush=True)
        assert infos[i]["status"] == pb.PB_OK
        assert iters_close(infos[i]["iters"], o6[i].iters)
        assert fdpb.true_relres(refs[i], xg) <= 1e-5
        assert np.abs(xg - exact[i]).max() <= 1e-5 * np.abs(exact[i]).max()
    # each problem alone gives bitwise the same result as in the mix
    for i in (0, 3):
        xa, ia = pb.solve_batch([systems[i]], tol=1e-6, precision=prec)
        assert ia[0]["iters"] == infos[i]["iters"] and torch.equal(xa[0], xs[i])
    # a different mix (reversed order, a subset) changes nothing either
    sub = [systems[4], systems[1], systems[2]]
    xb, ib = pb.solve_batch(sub, tol=1e-6, precision=prec)
    for j, i in enumerate((4, 1, 2)):
        assert torch.equal(xb[j], xs[i])


def test_batch_per_problem_tolerance_and_status(pb, batch_set):
    probs, refs, exact, o6, systems = batch_set
    tols = [1e-3, 1e-6, 2.0, 1e-4, 1e-6]
    xs, infos = pb.solve_batch(systems, tol=tols, precision="f32")
    assert infos[2]["iters"] == 0 and not xs[2].any()
    for i, t in enumerate(tols):
        if t < 1:
            assert infos[i]["relres_recur"] < t
    xs, infos = pb.solve_batch(systems[:2], tol=1e-6, precision="f32", maxiter=3, check=False)
    assert all(i["status"] == pb.PB_NOT_CONVERGED and i["iters"] == 3 for i in infos)


def test_batch_autotune(pb, batch_set):
    """The batch autotuner times its candidate z-chunks on the batch and makes
    the fastest the device's setting without writing the systems' arrays;
    solves afterwards match the oracle and stay mix independent, and so do
    solves under any other z-chunk."""
    probs, refs, exact, o6, systems = batch_set
    z0 = pb.get_batch_zchunk()
    saved = [(s.rhs.clone(), s.eps_x.clone()) for s in systems]
    try:
        r = pb.batch_autotune(systems, precision="f32", iters_per_trial=10)
        print(f"batch autotune: {r}", flush=True)
        assert r["zchunk"] in (16, 24, 32, 48, 64) and r["seconds"] > 0
        assert pb.get_batch_zchunk() == r["zchunk"]
        for s, (b, e) in zip(systems, saved):
            assert torch.equal(s.rhs, b) and torch.equal(s.eps_x, e)
        for z in (r["zchunk"], 7):
            pb.set_batch_zchunk(z)
            xs, infos = pb.solve_batch(systems, tol=1e-6, precision="f32")
            for i in range(len(systems)):
                assert infos[i]["status"] == pb.PB_OK
                assert np.abs(xs[i].cpu().numpy() - exact[i]).max() <= 1e-5 * np.abs(exact[i]).max(), (z, i)
            xa, ia = pb.solve_batch([systems[1]], tol=1e-6, precision="f32")
            assert ia[0]["iters"] == infos[1]["iters"] and torch.equal(xa[0], xs[1]), z
        for bad in (0, 5000):
            with pytest.raises(pb.PBError):
                pb.set_batch_zchunk(bad)
    finally:
        pb.set_batch_zchunk(z0)


def test_batch_graph_replay(pb, batch_set):
    probs, refs, exact, o6, systems = batch_set
    ref_x, ref_info = pb.solve_batch(systems, tol=1e-6, precision="f32")
    g = pb.BatchGraph(systems, tol=1e-6, precision="f32")
    print(f"graph cooperative={g.cooperative}", flush=True)
    for rep in range(3):
        g.launch()
        infos = g.results()
        for i in range(len(systems)):
            assert infos[i]["iters"] == ref_info[i]["iters"]
            assert torch.equal(g.outs[i], ref_x[i]), (rep, i)
        torch.cuda.synchronize()
    # new contents in the same buffers: doubling every rhs doubles every potential exactly
    saved = [s.rhs.clone() for s in systems]
    for s in systems:
        s.rhs.mul_(2.0)
    g.launch()
    infos = g.results()
    for s, r in zip(systems, saved):
        s.rhs.copy_(r)
    for i in range(len(systems)):
        assert torch.equal(g.outs[i], 2.0 * ref_x[i])
    g.close()


# ------------------------------------------------------------------ serving

SERVE_SET = [((37, 29, 23, 20), 1e-6, "f32"), ((45, 45, 45, 60), 1e-8, "f32_refine64"),
             ((21, 30, 17, 8), 1e-4, "f32"), ((64, 9, 33, 12), 1e-6, "f32"),
             ((33, 33, 65, 40), 1e-8, "f32_refine64"), ((29, 29, 29, 15), 1e-6, "f32")]


@pytest.fixture(scope="module")
def serve_set(pb):
    probs = [synth.small_problem(nx, ny, nz, na, seed=200 + i) for i, ((nx, ny, nz, na), _, _) in enumerate(SERVE_SET)]
    refs = [fdpb.assemble_problem(p) for p in probs]
    exact = [pcg.jpcg(r, 1e-13, maxiter=20000).x for r in refs]
    systems = [gpu_setup(pb, p) for p in probs]
    return probs, refs, exact, systems


def _serve(pb, systems, order, arena, chunk=16):
    srv = pb.Server(arena, max_slots=8)
    ids = {}
    for i in order:
        _, tol, prec = SERVE_SET[i]
        ids[srv.submit(systems[i], tol=tol, precision=prec)] = i
    results, trace = {}, []
    for _ in range(2000):
        st = srv.stats()
        assert st["arena_used"] <= st["arena_bytes"]
        trace.append((st["active"], st["pending"]))
        for rid, info in srv.step(chunk=chunk):
            results[ids[rid]] = (srv.outputs[rid].clone(), info)
        if len(results) == len(order):
            break
    srv.close()
    return results, trace


def test_server_continuous_batching(pb, serve_set):
    probs, refs, exact, systems = serve_set
    sizes = [pb.Server.request_bytes(s) for s in systems]
    arena = int(sum(sorted(sizes)[-3:]) * 1.05) + (1 << 20)      # room for about three requests at once
    mixed, trace = _serve(pb, systems, list(range(len(systems))), arena)
    assert len(mixed) == len(systems)
    # the budget limited admission at some point, and requests were backfilled
    assert any(a > 0 and p > 0 for a, p in trace)
    assert max(a for a, _ in trace) >= 2
    for i, (x, info) in mixed.items():
        _, tol, prec = SERVE_SET[i]
        xg = x.cpu().numpy()
        rel = fdpb.true_relres(refs[i], xg)
        print(f"serve #{i} {prec} tol {tol}: iters {info['iters']} outer {info['outer_iters']} relres_true {rel:.2e}",
              flush=True)
        assert info["status"] == pb.PB_OK
        if prec == "f32_refine64":
            assert rel < tol and np.abs(xg - exact[i]).max() <= 1e-7 * np.abs(exact[i]).max()
        else:
            assert rel <= max(10 * tol, 1e-5)
    # every result is the same alone, and in a different arrival order
    for i in (0, 1, 3):
        alone, _ = _serve(pb, [systems[k] if k == i else None for k in range(len(systems))], [i], arena)
        assert torch.equal(alone[i][0], mixed[i][0]), i
    rev, _ = _serve(pb, systems, list(reversed(range(len(systems)))), arena)
    for i in range(len(systems)):
        assert torch.equal(rev[i][0], mixed[i][0]), i
