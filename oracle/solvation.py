"""FP64 CPU oracle of the solvation (reaction-field) energy.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: imported by tests, the
smoke check and the benchmark's CPU-baseline leg, never by the library path.

Section 3.1 of the paper judges accuracy by electrostatic solvation energies
computed from the FD potential. The energy of a charge set on a grid contains
a large grid self-energy; it cancels in the difference of two solves on the
same grid with the same charges:

    dG = E(eps_in inside, eps_out and salt outside) - E(uniform eps_in, no salt)

with E = 1/2 sum_a q_a phi(c_a) (kcal/mol, fdpb.energy). The reference system
is the same setup with eps_out = eps_in and kappa_D^2 = 0 (its Dirichlet
values are then plain Coulomb in eps_in). For one ion of charge q and radius
a the continuum value is Born's -332.06 q^2/(2a) (1/eps_in - 1/eps_out).
"""
from __future__ import annotations

import dataclasses

from . import fdpb, pcg, periodic


@dataclasses.dataclass
class Solvation:
    dG: float            # kcal/mol
    e_solv: float        # energy in the solvent system
    e_ref: float         # energy in the uniform reference
    iters_solv: int
    iters_ref: int
    phi_solv: object     # (nz, ny, nx) potentials
    phi_ref: object


def solvation_energy(nx, ny, nz, h, origin, xyz, radius, charge, eps_in, eps_out, kappa_d2,
                     tol=1e-10, maxiter=None, boundary="free") -> Solvation:
    """Two full setups and JPCG solves on the same grid, then the energy
    difference (section 3.1 energies; systems of Eq. 3 as in fdpb, or the
    periodic box of oracle.periodic)."""
    out = []
    for eo, k2 in ((eps_out, kappa_d2), (eps_in, 0.0)):
        if boundary == "periodic":
            s = periodic.assemble(nx, ny, nz, h, origin, xyz, radius, charge, eps_in, eo, k2)
            res = periodic.jpcg(s, tol, maxiter=maxiter)
            e = periodic.energy(nx, ny, nz, h, origin, xyz, charge, res.x) if res.converged else None
        else:
            s = fdpb.assemble(nx, ny, nz, h, origin, xyz, radius, charge, eps_in, eo, k2)
            res = pcg.jpcg(s, tol, maxiter=maxiter)
            e = fdpb.energy(nx, ny, nz, h, origin, xyz, charge, res.x) if res.converged else None
        if not res.converged:
            raise RuntimeError(f"oracle solve did not converge (eps_out={eo})")
        out.append((e, res.iters, res.x))
    (es, its, xs), (er, itr, xr) = out
    return Solvation(dG=es - er, e_solv=es, e_ref=er, iters_solv=its, iters_ref=itr, phi_solv=xs, phi_ref=xr)


def born_energy(q, a, eps_in, eps_out) -> float:
    """Born's continuum solvation energy of one ion, kcal/mol."""
    return -fdpb.COULOMB_KCAL * q * q / (2.0 * a) * (1.0 / eps_in - 1.0 / eps_out)
