"""Fractional-edge weighted harmonic dielectric (PB_EDGE_FRACTION) on the GPU,
through the C ABI, against the oracle's fractional_edges.

The device path is switched off (pb_setup_ex refuses PB_EDGE_FRACTION): its
first device run ended in a memory fault with no cause found yet, so the
parity tests below stay skipped until one is; the kernel text itself is
checked on the host (test_frac_kernel_host.py)."""
import numpy as np
import pytest
import torch

import synth
from oracle import fdpb, pcg, solvation

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pb():
    import paper_1704_02745_amd as m
    return m


OFF = pytest.mark.skip(reason="PB_EDGE_FRACTION device path switched off: its first device run faulted, "
                              "cause not found yet")

CASES = [("c0", lambda: synth.config0()),
         ("ragged", lambda: synth.small_problem(61, 53, 47, 80, seed=7)),
         ("thin", lambda: synth.small_problem(40, 9, 23, 6, seed=8)),
         ("nosalt", lambda: synth.small_problem(29, 31, 27, 30, seed=9, kappa_d2=0.0))]


@OFF
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fractional_setup_matches_oracle(pb, name, make):
    prob = make()
    g = prob.grid
    sm = pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                  device=DEV, want_q=True, want_mask=True, edge_model="fraction")
    ref, parts = fdpb.assemble(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius, prob.mol.charge,
                               prob.eps_in, prob.eps_out, prob.kappa_d2, with_parts=True, edge_model="fraction")
    for a, b in ((sm.eps_x, ref.eps_x), (sm.eps_y, ref.eps_y), (sm.eps_z, ref.eps_z)):
        a = a.cpu().numpy()
        assert np.array_equal(a, b), (name, np.argwhere(a != b)[:5])
    assert ((ref.eps_x > 1.0) & (ref.eps_x < 80.0)).any()        # some edges really are fractional
    assert np.array_equal(sm.mask.cpu().numpy(), parts["mask"])
    assert np.array_equal(sm.kappa2.cpu().numpy(), ref.kappa2)
    assert np.array_equal(sm.qgrid.cpu().numpy(), parts["qgrid"])
    b = sm.rhs.cpu().numpy()
    assert np.abs(b - ref.b).max() <= 1e-12 * np.abs(ref.b).max()


@OFF
def test_fractional_solve_and_energy(pb):
    prob = synth.config0()
    g = prob.grid
    sm = pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                  device=DEV, edge_model="fraction")
    ref = fdpb.assemble(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius, prob.mol.charge,
                        prob.eps_in, prob.eps_out, prob.kappa_d2, edge_model="fraction")
    exact = pcg.jpcg(ref, 1e-13, maxiter=5000).x
    for op in ("stencil", "mg"):
        x, info = pb.solve(sm, tol=1e-10, precision="f64", op=op)
        assert np.abs(x.cpu().numpy() - exact).max() <= 1e-8 * np.abs(exact).max(), op
    e = pb.energy(g, prob.mol.xyz, prob.mol.charge, x)
    e_ref = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.charge, x.cpu().numpy())
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)


@OFF
def test_fractional_born_ion(pb):
    """The Born ion's h = 0.5 error drops below 1% with fractional edges (3.8% with the two-point rule)."""
    n, h, a = 33, 0.5, 2.1
    org = np.full(3, -(n - 1) / 2 * h)
    grid = synth.Grid(n, n, n, h, org)
    xyz, R, q = np.zeros((1, 3)), np.array([a]), np.array([1.0])
    es = {}
    for model in ("node", "fraction"):
        e2 = []
        for eo in (80.0, 1.0):
            sm = pb.setup(grid, xyz, R, q, 1.0, eo, 0.0, device=DEV, edge_model=model)
            x, _ = pb.solve(sm, tol=1e-10, precision="f64", op="mg")
            e2.append(pb.energy(grid, xyz, q, x))
        es[model] = (e2[0] - e2[1]) / solvation.born_energy(1.0, a, 1.0, 80.0) - 1.0
    print("Born relative error", es, flush=True)
    assert abs(es["fraction"]) < 0.01 < abs(es["node"])


def test_fractional_rejections(pb):
    """Both refusals happen on the host before any launch."""
    prob = synth.config0()
    g = prob.grid
    for kw in (dict(boundary="periodic"), dict()):
        with pytest.raises(pb.PBError) as ei:
            pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, device=DEV, edge_model="fraction", **kw)
        assert ei.value.status == pb.PB_ERR_ARG
    assert "switched off" in str(ei.value)
    # the two-point model still works after the refusals
    sm = pb.setup(g, prob.mol.xyz, prob.mol.radius, prob.mol.charge, prob.eps_in, prob.eps_out, prob.kappa_d2,
                  device=DEV, edge_model="node")
    torch.cuda.synchronize()
    assert torch.isfinite(sm.rhs).all()
