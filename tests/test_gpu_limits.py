"""Row-width limits of the fused and batched kernels.

A tile's in-plane halo is one grid row on each side, handled by one
16-byte vector group per thread, so a block of B threads takes rows of at
most B * VEC / 2 nodes (VEC = 4 in FP32, 2 in FP64). The fused kernel's
widest block (512 threads) gives nx <= 1024 in FP32 and 512 in FP64; the
batched and served kernel (256 threads) gives 512 and 256. At each limit
every feasible tiling solves a random system to the oracle's solution; one
node wider is rejected with PB_ERR_ARG before any launch.
"""
import numpy as np
import pytest
import torch

from oracle import fdpb, pcg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
LIMITS = [("f32", 1024, 512), ("f64", 512, 256)]   # precision, fused max nx, batched max nx
NY, NZ = 3, 4


@pytest.fixture(scope="module")
def pb():
    import paper_1704_02745_amd as m
    return m


def rand_system(nx, ny, nz, seed, h=0.5):
    rng = np.random.default_rng(seed)
    return fdpb.System(h=h, eps_x=rng.uniform(1, 80, (nz, ny, nx + 1)), eps_y=rng.uniform(1, 80, (nz, ny + 1, nx)),
                       eps_z=rng.uniform(1, 80, (nz + 1, ny, nx)), kappa2=rng.uniform(0, 2, (nz, ny, nx)),
                       b=rng.standard_normal((nz, ny, nx)))


def to_system(pb, s):
    nx, ny, nz = s.dims
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    return pb.System(pb.make_grid(nx, ny, nz, s.h, (0.0, 0.0, 0.0)), t(s.eps_x), t(s.eps_y), t(s.eps_z),
                     t(s.kappa2), t(s.b))


def _bars(prec):
    return (1e-8, 1e-7) if prec == "f64" else (1e-5, 1e-4)   # solve tolerance, max-norm error bound


@pytest.mark.parametrize("prec,fmax,bmax", LIMITS)
def test_widest_fused_rows(pb, prec, fmax, bmax):
    tol, bound = _bars(prec)
    s = rand_system(fmax, NY, NZ, seed=fmax)
    o = pcg.jpcg(s, 1e-10, maxiter=5000)
    sysm = to_system(pb, s)
    cands = pb.tiling_candidates(fmax, NY, NZ, prec)
    print(f"{prec} nx={fmax}: {len(cands)} tilings", flush=True)
    assert cands
    for c in cands:
        pb.set_tuning(fmax, NY, NZ, prec, c["block"], c["groups"], c["zchunk"], c["grid"], c["scheme"],
                      c["streaming"], c["segments"])
        x, info = pb.solve(sysm, tol=tol, precision=prec, maxiter=5000)
        assert info["status"] == pb.PB_OK, c
        assert np.abs(x.cpu().numpy() - o.x).max() <= bound * np.abs(o.x).max(), c
    wide = to_system(pb, rand_system(fmax + 1, NY, NZ, seed=1))
    assert pb.tiling_candidates(fmax + 1, NY, NZ, prec) == []
    with pytest.raises(pb.PBError) as e:
        pb.solve(wide, tol=tol, precision=prec)
    assert e.value.status == pb.PB_ERR_ARG


@pytest.mark.parametrize("prec,fmax,bmax", LIMITS)
def test_widest_batched_rows(pb, prec, fmax, bmax):
    tol, bound = _bars(prec)
    s = rand_system(bmax, NY, NZ, seed=bmax + 1)
    o = pcg.jpcg(s, 1e-10, maxiter=5000)
    xs, infos = pb.solve_batch([to_system(pb, s)], tol=tol, precision=prec, maxiter=5000)
    assert infos[0]["status"] == pb.PB_OK
    assert np.abs(xs[0].cpu().numpy() - o.x).max() <= bound * np.abs(o.x).max()
    wide = to_system(pb, rand_system(bmax + 1, NY, NZ, seed=2))
    with pytest.raises(pb.PBError) as e:
        pb.solve_batch([wide], tol=tol, precision=prec)
    assert e.value.status == pb.PB_ERR_ARG
