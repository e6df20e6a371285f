"""pb_solve_noalloc: the solve in the library's per-GPU scratch array (no
workspace, no device allocation), through the C ABI.

Two calls in a row, the second on a smaller grid, each checked against
pb_solve on the same system: the same kernels run on the same tiling, so the
potential and the iteration counts must be bitwise those of pb_solve, and the
potential must meet the FP32 bar (max |phi - phi_oracle| / max |phi_oracle|
<= 1e-5 at tol 1e-6, 1e-9 after FP64 refinement) against the oracle's
solution. A grid beyond the scratch is refused before any launch.
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
    return m


def _case(pb, prob):
    g = prob.grid
    sysm = pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                    device=DEV)
    exact = pcg.jpcg(fdpb.assemble_problem(prob), 1e-12, maxiter=20000).x
    return sysm, exact


def test_noalloc_matches_pb_solve_twice_shrinking(pb):
    big = synth.small_problem(65, 61, 57, 120, seed=21, precision="f32")
    small = synth.config0()
    runs = [(big, "f32", 1e-6, 1e-5), (small, "f32_refine64", 1e-10, 1e-9)]
    for prob, prec, tol, bar in runs:
        sysm, exact = _case(pb, prob)
        g = prob.grid
        x_ref, i_ref = pb.solve(sysm, tol=tol, precision=prec)
        out = torch.full((g.nz, g.ny, g.nx), float("nan"), dtype=torch.float64, device=DEV)
        info = pb.solve_noalloc(sysm, out, tol=tol, precision=prec)
        torch.cuda.synchronize()
        err = float(np.abs(out.cpu().numpy() - exact).max() / np.abs(exact).max())
        print(f"noalloc {prob.name} {prec}: iters {info['iters']} (pb_solve {i_ref['iters']}) "
              f"outer {info['outer_iters']} relres {info['relres_true']:.2e} phi err {err:.2e}", flush=True)
        assert info["status"] == pb.PB_OK
        assert info["iters"] == i_ref["iters"] and info["outer_iters"] == i_ref["outer_iters"]
        assert info["kernel_seconds"] == 0.0
        assert torch.equal(out, x_ref)
        assert err <= bar


def test_noalloc_refuses_grid_beyond_scratch(pb):
    n = 161   # 161^3 needs about 423 MiB of scratch
    opt = dict(dtype=torch.float64, device=DEV)
    g = pb.make_grid(n, n, n, 0.5, (0.0, 0.0, 0.0))
    tiny = torch.zeros(1, **opt)
    sysm = pb.System(g, tiny, tiny, tiny, tiny, tiny)
    out = torch.zeros(1, **opt)
    with pytest.raises(pb.PBError) as ei:
        pb.solve_noalloc(sysm, out, tol=1e-6, precision="f32")
    assert ei.value.status == pb.PB_ERR_NOMEM
    assert "scratch" in str(ei.value)
