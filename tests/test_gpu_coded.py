"""Coded coefficients in the 40-byte FP32 pass (pb_set_coded_coefficients).

The operator of Eq. 3 built from the two-point dielectric model holds few
distinct FP32 values, so its solves read one word of dictionary codes per node
instead of the four coefficient arrays. The decoded values are the
coefficients themselves, so:

- every coded solve gives bitwise the potential and the iteration count of
  the uncoded pass with the same tiling (every feasible 40-byte tiling:
  256/512 threads, cached and streaming accesses);
- it reaches the oracle's solution within the FP32 bound, also under FP64
  refinement and at the benchmark's 257^3 size;
- operators with more than 256 distinct values, and grids too small for the
  dictionary's scratch, run the uncoded pass (pb_info.coded_launches = 0).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fdpb, pcg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pb():
    import paper_1704_02745_amd as m
    m.set_coded_coefficients(True)
    yield m
    m.set_coded_coefficients(True)


def gpu_setup(pb, prob):
    g = prob.grid
    return pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                    device=DEV)


def forty_byte_tilings(pb, dims, prec="f32"):
    return [c for c in pb.tiling_candidates(*dims, prec) if c["scheme"] == 1]


def pin(pb, dims, prec, c):
    pb.set_tuning(*dims, prec, c["block"], c["groups"], c["zchunk"], c["grid"], c["scheme"], c["streaming"],
                  c["segments"])


def coded_and_uncoded(pb, sysm, **kw):
    pb.set_coded_coefficients(True)
    x1, i1 = pb.solve(sysm, **kw)
    pb.set_coded_coefficients(False)
    try:
        x0, i0 = pb.solve(sysm, **kw)
    finally:
        pb.set_coded_coefficients(True)
    return x1, i1, x0, i0


def restore_default(pb, sysm, prec="f32"):
    best = pb.autotune(sysm, precision=prec, iters_per_trial=3)
    assert best["grid"] > 0


@pytest.mark.parametrize("dims,natoms,seed", [((61, 53, 47), 300, 9), ((65, 65, 65), 500, 3),
                                              ((97, 37, 29), 200, 5)])
def test_coded_equals_uncoded_every_tiling(pb, dims, natoms, seed):
    prob = synth.small_problem(*dims, natoms, seed=seed, precision="f32")
    ref = fdpb.assemble_problem(prob)
    exact = pcg.jpcg(ref, 1e-13, maxiter=20000).x
    sysm = gpu_setup(pb, prob)
    cands = forty_byte_tilings(pb, dims)
    assert cands and {c["streaming"] for c in cands} == {0, 1}, cands
    try:
        for c in cands:
            pin(pb, dims, "f32", c)
            print(f"coded {dims} {c}", flush=True)
            x1, i1, x0, i0 = coded_and_uncoded(pb, sysm, tol=1e-6, precision="f32")
            assert i1["status"] == pb.PB_OK and i0["status"] == pb.PB_OK, (i1, i0)
            assert i1["coded_launches"] == i1["kernel_launches"] == 1, i1
            assert i0["coded_launches"] == 0, i0
            assert i1["iters"] == i0["iters"], (i1, i0)
            assert torch.equal(x1, x0), c
            xv = x1.cpu().numpy()
            assert fdpb.true_relres(ref, xv) <= 1e-5
            assert np.abs(xv - exact).max() <= 1e-5 * np.abs(exact).max(), c
    finally:
        restore_default(pb, sysm)


def test_coded_refinement(pb):
    dims = (61, 53, 47)
    prob = synth.small_problem(*dims, 300, seed=9, precision="f32")
    ref = fdpb.assemble_problem(prob)
    exact = pcg.jpcg(ref, 1e-13, maxiter=20000).x
    sysm = gpu_setup(pb, prob)
    cands = forty_byte_tilings(pb, dims, "f32_refine64")
    assert cands
    try:
        pin(pb, dims, "f32_refine64", cands[-1])
        x1, i1, x0, i0 = coded_and_uncoded(pb, sysm, tol=1e-10, precision="f32_refine64", inner_tol=1e-4)
        print(f"refine: coded {i1} uncoded {i0}", flush=True)
        assert i1["status"] == pb.PB_OK and i1["outer_iters"] >= 2
        assert i1["coded_launches"] == i1["kernel_launches"] >= 2, i1
        assert i0["coded_launches"] == 0
        assert i1["iters"] == i0["iters"] and i1["outer_iters"] == i0["outer_iters"]
        assert torch.equal(x1, x0)
        xv = x1.cpu().numpy()
        assert fdpb.true_relres(ref, xv) < 1e-10
        assert np.abs(xv - exact).max() <= 1e-9 * np.abs(exact).max()
    finally:
        restore_default(pb, sysm, "f32_refine64")


def test_many_distinct_values_run_uncoded(pb):
    """Random coefficient arrays hold millions of distinct values: the
    dictionary overflows and the uncoded pass runs, to the oracle's solution."""
    dims = (48, 40, 36)
    rng = np.random.default_rng(17)
    nx, ny, nz = dims
    s = fdpb.System(h=0.5, eps_x=rng.uniform(1, 80, (nz, ny, nx + 1)), eps_y=rng.uniform(1, 80, (nz, ny + 1, nx)),
                    eps_z=rng.uniform(1, 80, (nz + 1, ny, nx)), kappa2=rng.uniform(0, 2, (nz, ny, nx)),
                    b=rng.standard_normal((nz, ny, nx)))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    sysm = pb.System(pb.make_grid(nx, ny, nz, s.h, (0.0, 0.0, 0.0)), t(s.eps_x), t(s.eps_y), t(s.eps_z),
                     t(s.kappa2), t(s.b))
    exact = pcg.jpcg(s, 1e-12, maxiter=20000).x
    cands = forty_byte_tilings(pb, dims)
    assert cands
    try:
        pin(pb, dims, "f32", cands[0])
        x1, i1, x0, i0 = coded_and_uncoded(pb, sysm, tol=1e-6, precision="f32")
        assert i1["status"] == pb.PB_OK
        assert i1["coded_launches"] == 0 and i0["coded_launches"] == 0
        assert torch.equal(x1, x0) and i1["iters"] == i0["iters"]
        assert np.abs(x1.cpu().numpy() - exact).max() <= 1e-5 * np.abs(exact).max()
    finally:
        restore_default(pb, sysm)


def test_small_grid_runs_uncoded(pb):
    """15^3 has 3,840 padded positions, fewer than the dictionary's scratch
    needs: the uncoded pass runs, and matches the oracle."""
    dims = (15, 15, 15)
    prob = synth.small_problem(*dims, 10, seed=2, precision="f32")
    ref = fdpb.assemble_problem(prob)
    exact = pcg.jpcg(ref, 1e-13, maxiter=20000).x
    sysm = gpu_setup(pb, prob)
    cands = forty_byte_tilings(pb, dims)
    assert cands
    try:
        pin(pb, dims, "f32", cands[0])
        x, info = pb.solve(sysm, tol=1e-6, precision="f32")
        assert info["status"] == pb.PB_OK and info["coded_launches"] == 0
        assert np.abs(x.cpu().numpy() - exact).max() <= 1e-5 * np.abs(exact).max()
    finally:
        restore_default(pb, sysm)


def test_coded_config2_257(pb):
    """The benchmark's system (257^3, 20,000 atoms) with the 512-thread
    streaming 40-byte tiling: coded and uncoded solves to 1e-6 agree bitwise,
    and the oracle's FP64 operator gives the true residual."""
    prob = synth.config2()
    dims = (prob.grid.nx, prob.grid.ny, prob.grid.nz)
    sysm = gpu_setup(pb, prob)
    cands = [c for c in forty_byte_tilings(pb, dims) if c["block"] == 512 and c["streaming"] == 1]
    assert cands
    try:
        pin(pb, dims, "f32", cands[0])
        x1, i1, x0, i0 = coded_and_uncoded(pb, sysm, tol=1e-6, precision="f32")
        print(f"257: coded iters {i1['iters']} {1e3 * i1['kernel_seconds']:.2f} ms, uncoded "
              f"{1e3 * i0['kernel_seconds']:.2f} ms", flush=True)
        assert i1["status"] == pb.PB_OK and i1["coded_launches"] == 1
        assert i1["iters"] == i0["iters"] and torch.equal(x1, x0)
        host = fdpb.System(h=prob.grid.h, eps_x=sysm.eps_x.cpu().numpy(), eps_y=sysm.eps_y.cpu().numpy(),
                           eps_z=sysm.eps_z.cpu().numpy(), kappa2=sysm.kappa2.cpu().numpy(),
                           b=sysm.rhs.cpu().numpy())
        assert fdpb.true_relres(host, x1.cpu().numpy()) <= 1e-5
    finally:
        restore_default(pb, sysm)
        del sysm
        torch.cuda.empty_cache()


def test_coded_batch_and_server(pb):
    """The batched and served forms: coded and uncoded launches give bitwise the
    same potentials and iteration counts (FP32 and FP64-refined requests); a
    batch holding a grid too small for the dictionary runs uncoded, with the
    other problems' results unchanged."""
    shapes = [(61, 53, 47, 300), (65, 65, 65, 500), (33, 41, 29, 60), (49, 49, 49, 120)]
    probs = [synth.small_problem(*sh[:3], sh[3], seed=300 + i, precision="f32") for i, sh in enumerate(shapes)]
    refs = [fdpb.assemble_problem(p) for p in probs]
    systems = [gpu_setup(pb, p) for p in probs]

    pb.set_coded_coefficients(True)
    x1, i1 = pb.solve_batch(systems, tol=1e-6, precision="f32")
    pb.set_coded_coefficients(False)
    try:
        x0, i0 = pb.solve_batch(systems, tol=1e-6, precision="f32")
    finally:
        pb.set_coded_coefficients(True)
    assert all(i["coded_launches"] == 1 for i in i1), i1
    assert all(i["coded_launches"] == 0 for i in i0), i0
    for j in range(len(systems)):
        assert i1[j]["status"] == pb.PB_OK
        assert i1[j]["iters"] == i0[j]["iters"] and torch.equal(x1[j], x0[j]), j
        assert fdpb.true_relres(refs[j], x1[j].cpu().numpy()) <= 1e-5

    small = gpu_setup(pb, synth.small_problem(15, 15, 15, 10, seed=2, precision="f32"))
    x2, i2 = pb.solve_batch(systems[:2] + [small], tol=1e-6, precision="f32")
    assert all(i["coded_launches"] == 0 for i in i2), i2
    assert torch.equal(x2[0], x1[0]) and torch.equal(x2[1], x1[1])

    def serve(on):
        pb.set_coded_coefficients(on)
        try:
            arena = sum(pb.Server.request_bytes(s) for s in systems) + (64 << 20)
            srv = pb.Server(arena, max_slots=8, device=DEV)
            ids = {}
            for i, s in enumerate(systems):
                tol, prec = (1e-6, "f32") if i % 2 == 0 else (1e-9, "f32_refine64")
                ids[srv.submit(s, tol=tol, precision=prec)] = i
            out = {}
            for _ in range(10000):
                for rid, info in srv.step(chunk=32):
                    out[ids[rid]] = (srv.outputs[rid].clone(), info)
                if len(out) == len(systems):
                    break
            stats = srv.stats()
            srv.close()
            return out, stats
        finally:
            pb.set_coded_coefficients(True)

    (s1, st1), (s0, st0) = serve(True), serve(False)
    print(f"server: coded launches {st1['coded_launches']} of {st1['launches']}; uncoded run "
          f"{st0['coded_launches']} of {st0['launches']}", flush=True)
    assert st1["coded_launches"] == st1["launches"] > 0 and st0["coded_launches"] == 0
    for i in range(len(systems)):
        assert s1[i][1]["status"] == pb.PB_OK, s1[i][1]
        assert s1[i][1]["iters"] == s0[i][1]["iters"] and torch.equal(s1[i][0], s0[i][0]), i
        rel = fdpb.true_relres(refs[i], s1[i][0].cpu().numpy())
        assert rel <= (1e-5 if i % 2 == 0 else 1e-9), (i, rel)


@pytest.mark.parametrize("nsalt,coded", [(254, True), (255, False)])
def test_dictionary_capacity_boundary(pb, nsalt, coded):
    """Uniform eps = 1 at h = 0.5 gives couplings {4, 0} and diagonals 24 + kbar^2;
    a 40 x 32 plane is a multiple of the 64-position padding, so no pad slots
    add a value. With K distinct salt values the operator holds exactly K + 2
    FP32 values: K = 254 (256 values) runs coded, K = 255 (257 values)
    uncoded; both solve to the oracle's solution."""
    nx, ny, nz = 40, 32, 30
    rng = np.random.default_rng(nsalt)
    salt = (np.arange(nsalt) + 1) * 1e-3
    k2 = salt[np.arange(nx * ny * nz) % nsalt].reshape(nz, ny, nx)
    s = fdpb.System(h=0.5, eps_x=np.ones((nz, ny, nx + 1)), eps_y=np.ones((nz, ny + 1, nx)),
                    eps_z=np.ones((nz + 1, ny, nx)), kappa2=k2, b=rng.standard_normal((nz, ny, nx)))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    sysm = pb.System(pb.make_grid(nx, ny, nz, s.h, (0.0, 0.0, 0.0)), t(s.eps_x), t(s.eps_y), t(s.eps_z),
                     t(s.kappa2), t(s.b))
    exact = pcg.jpcg(s, 1e-12, maxiter=20000).x
    dims = (nx, ny, nz)
    cands = forty_byte_tilings(pb, dims)
    assert cands
    try:
        pin(pb, dims, "f32", cands[0])
        x1, i1, x0, i0 = coded_and_uncoded(pb, sysm, tol=1e-6, precision="f32")
        assert i1["status"] == pb.PB_OK
        assert i1["coded_launches"] == (1 if coded else 0), i1
        assert torch.equal(x1, x0) and i1["iters"] == i0["iters"]
        assert np.abs(x1.cpu().numpy() - exact).max() <= 1e-5 * np.abs(exact).max()
    finally:
        restore_default(pb, sysm)


def test_coded_graph_decides_per_replay(pb):
    """A recorded batch rebuilds every problem's dictionary at each replay: after
    one problem's edge dielectrics are overwritten in place with random values
    (far more than 256 distinct), that problem runs uncoded and the others
    coded, and every replay equals direct solves of the same contents."""
    shapes = [(49, 45, 41, 100), (57, 49, 43, 150), (41, 41, 41, 60)]
    probs = [synth.small_problem(*sh[:3], sh[3], seed=400 + i, precision="f32") for i, sh in enumerate(shapes)]
    systems = [gpu_setup(pb, p) for p in probs]
    g = pb.BatchGraph(systems, tol=1e-6, precision="f32")
    try:
        g.launch()
        i1 = g.results()
        assert [i["coded_launches"] for i in i1] == [1, 1, 1], i1
        xd, _ = pb.solve_batch(systems, tol=1e-6, precision="f32")
        assert all(torch.equal(g.outs[j], xd[j]) for j in range(3))

        s = systems[1]
        saved = [a.clone() for a in (s.eps_x, s.eps_y, s.eps_z)]
        rng = np.random.default_rng(5)
        for a in (s.eps_x, s.eps_y, s.eps_z):
            a.copy_(torch.as_tensor(rng.uniform(1, 80, tuple(a.shape)), dtype=torch.float64, device=DEV))
        g.launch()
        i2 = g.results()
        assert [i["coded_launches"] for i in i2] == [1, 0, 1], i2
        assert all(i["status"] == pb.PB_OK for i in i2)
        xd2, id2 = pb.solve_batch(systems, tol=1e-6, precision="f32")
        assert all(i["coded_launches"] == 0 for i in id2)   # the direct batch codes all problems or none
        assert all(torch.equal(g.outs[j], xd2[j]) for j in range(3))
        ref = fdpb.System(h=s.grid.h, eps_x=s.eps_x.cpu().numpy(), eps_y=s.eps_y.cpu().numpy(),
                          eps_z=s.eps_z.cpu().numpy(), kappa2=s.kappa2.cpu().numpy(), b=s.rhs.cpu().numpy())
        assert fdpb.true_relres(ref, g.outs[1].cpu().numpy()) <= 1e-5

        for a, b in zip((s.eps_x, s.eps_y, s.eps_z), saved):
            a.copy_(b)
        g.launch()
        i3 = g.results()
        assert [i["coded_launches"] for i in i3] == [1, 1, 1], i3
        assert all(torch.equal(g.outs[j], xd[j]) for j in range(3))
    finally:
        g.close()


@pytest.mark.parametrize("nz,coded", [(132, False), (133, True)])
def test_scratch_size_threshold(pb, nz, coded):
    """The dictionary's scratch lives in the 40-byte form's unused q array, so
    a grid needs 8,450 padded positions for the coded pass: a 16 x 4 plane (64
    positions, no padding) gives 8,448 at nz = 132 (uncoded) and 8,512 at
    nz = 133 (coded). Uniform eps and three salt values keep the operator's
    values few; both solve to the oracle's solution."""
    nx, ny = 16, 4
    rng = np.random.default_rng(nz)
    k2 = np.array([0.0, 0.5, 1.25])[rng.integers(0, 3, (nz, ny, nx))]
    s = fdpb.System(h=0.5, eps_x=np.ones((nz, ny, nx + 1)), eps_y=np.ones((nz, ny + 1, nx)),
                    eps_z=np.ones((nz + 1, ny, nx)), kappa2=k2, b=rng.standard_normal((nz, ny, nx)))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    sysm = pb.System(pb.make_grid(nx, ny, nz, s.h, (0.0, 0.0, 0.0)), t(s.eps_x), t(s.eps_y), t(s.eps_z),
                     t(s.kappa2), t(s.b))
    exact = pcg.jpcg(s, 1e-12, maxiter=20000).x
    dims = (nx, ny, nz)
    cands = forty_byte_tilings(pb, dims)
    assert cands
    try:
        pin(pb, dims, "f32", cands[0])
        x, info = pb.solve(sysm, tol=1e-6, precision="f32")
        assert info["status"] == pb.PB_OK
        assert info["coded_launches"] == (1 if coded else 0), info
        assert np.abs(x.cpu().numpy() - exact).max() <= 1e-5 * np.abs(exact).max()
    finally:
        restore_default(pb, sysm)
