"""Served requests given as molecules (pb_server_submit_atoms): the server
runs the setup of section 2.7 at admission and the energy when a request
finishes, through the C ABI.

- Each result solves the oracle's own assembled system (its FP64 true
  residual) and, on the small grids, matches the oracle's solution within the
  FP32 bar (1e-5; 1e-7 refined to tol 1e-8); the energy equals the oracle's
  energy of the returned potential.
- Potentials and energies are bitwise the same alone, in the mix and in
  reversed arrival order.
- A molecule with an atom outside its node box finishes with PB_ERR_ARG and
  leaves the other requests untouched.
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


def _requests():
    out = []
    for k, (n, natoms, tol, prec) in enumerate([(33, 40, 1e-6, "f32"), (41, 90, 1e-8, "f32_refine64"),
                                                 (37, 60, 1e-4, "f32"), (45, 120, 1e-6, "f32"),
                                                 (29, 25, 1e-8, "f32_refine64")]):
        p = synth.small_problem(n, n, n, natoms, seed=700 + k, precision=prec, tol=tol)
        out.append(p)
    return out


def _serve(pb, reqs, order, chunk=16):
    arena = sum(pb.Server.request_bytes_atoms(p.grid, p.mol.natoms) for p in reqs) + (64 << 20)
    srv = pb.Server(arena, max_slots=32, device=DEV)
    ids = {}
    for i in order:
        p = reqs[i]
        rid = srv.submit_atoms(p.grid, p.mol.xyz, p.mol.radius, p.mol.charge, p.eps_in, p.eps_out, p.kappa_d2,
                               tol=p.tol, precision=p.precision)
        ids[rid] = i
    out = {}
    for _ in range(100000):
        for rid, info in srv.step(chunk=chunk):
            out[ids[rid]] = (srv.outputs[rid].clone(), srv.energies.get(rid), info)
        if len(out) == len(order):
            break
    srv.close()
    return out


def test_served_molecules_match_oracle_and_are_mix_independent(pb):
    reqs = _requests()
    order = list(range(len(reqs)))
    mix = _serve(pb, reqs, order)
    rev = _serve(pb, reqs, order[::-1])
    for i, p in enumerate(reqs):
        x, e, info = mix[i]
        g = p.grid
        s = fdpb.assemble_problem(p)
        xg = x.cpu().numpy()
        rel = fdpb.true_relres(s, xg)
        e_ref = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, p.mol.xyz, p.mol.charge, xg)
        exact = pcg.jpcg(s, 1e-12, maxiter=20000).x
        err = np.abs(xg - exact).max() / np.abs(exact).max()
        print(f"molecule {i} ({g.nx}^3, {p.mol.natoms} atoms, tol {p.tol}, {p.precision}): iters {info['iters']} "
              f"outer {info['outer_iters']} relres_true {rel:.2e} phi err {err:.2e} energy {e:.6f}", flush=True)
        assert info["status"] == pb.PB_OK
        if p.precision == "f32_refine64":
            assert rel < p.tol and err <= 1e-7
        else:
            assert rel <= max(10 * p.tol, 1e-5)
            if p.tol <= 1e-6:
                assert err <= 1e-5
        assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
        alone = _serve(pb, reqs, [i])
        for other in (alone, rev):
            assert torch.equal(other[i][0], x), i
            assert other[i][1] == e, i
            assert other[i][2]["iters"] == info["iters"], i


def test_served_molecule_outside_box_fails_alone(pb):
    reqs = _requests()[:3]
    bad = synth.small_problem(33, 33, 33, 30, seed=799, precision="f32")
    bad.mol.xyz = bad.mol.xyz.copy()
    bad.mol.xyz[0] = bad.grid.origin - 3.0          # one atom centre outside the node box
    reqs.append(bad)
    out = _serve(pb, reqs, list(range(len(reqs))))
    assert out[3][2]["status"] == pb.PB_ERR_ARG
    good = _serve(pb, reqs[:3], [0, 1, 2])
    for i in range(3):
        assert out[i][2]["status"] == pb.PB_OK
        assert torch.equal(out[i][0], good[i][0])


def test_served_molecules_admitted_while_others_run(pb):
    """Molecules submitted while earlier requests are mid-solve: their setup
    runs on the server's admission stream beside the running launch, and they
    join the following launches. Every result is bitwise the one it gets
    alone."""
    reqs = _requests()
    alone = {i: _serve(pb, reqs, [i])[i] for i in range(len(reqs))}
    arena = sum(pb.Server.request_bytes_atoms(p.grid, p.mol.natoms) for p in reqs) + (64 << 20)
    srv = pb.Server(arena, max_slots=32, device=DEV)
    ids, out = {}, {}

    def submit(i):
        p = reqs[i]
        rid = srv.submit_atoms(p.grid, p.mol.xyz, p.mol.radius, p.mol.charge, p.eps_in, p.eps_out, p.kappa_d2,
                               tol=p.tol, precision=p.precision)
        ids[rid] = i

    def step():
        for rid, info in srv.step(chunk=8):
            out[ids[rid]] = (srv.outputs[rid].clone(), srv.energies.get(rid), info)

    submit(1)
    submit(3)
    step()
    step()
    assert srv.stats()["active"] == 2          # both still running
    for i in (0, 2, 4):
        submit(i)
        step()
    for _ in range(100000):
        if len(out) == len(reqs):
            break
        step()
    srv.close()
    for i in range(len(reqs)):
        x, e, info = out[i]
        print(f"molecule {i}: iters {info['iters']} status {info['status']}", flush=True)
        assert info["status"] == pb.PB_OK
        assert torch.equal(x, alone[i][0]), i
        assert e == alone[i][1] and info["iters"] == alone[i][2]["iters"], i
