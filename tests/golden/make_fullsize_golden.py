"""Write the oracle's reference solutions of the 129^3 and 257^3 workloads.

Calls only `oracle/` (and the seeded input generators in `synth/`): the FP64
setup of section 2.7 (classification, two-point harmonic edges, salt,
trilinear charges, Debye-Hueckel boundary), the Jacobi-preconditioned CG of
sections 2.2/2.4 solved to a recurrence residual of 1e-12, the FP64 true
residual, and the energy 1/2 sum_a q_a phi(c_a). Full potentials are too large
to store, so each file keeps:

  - the oracle's iteration count to 1e-6 (FP64, x0 = 0);
  - max |phi|, the energy (kcal/mol) and the true relative residual;
  - phi at a seeded sample of nodes: uniform random nodes, the node nearest
    to each of a seeded subset of atom centres (where |phi| peaks), and the
    full central x-line.

Usage:  python tests/golden/make_fullsize_golden.py c1|c2
Runtime on one host core: about 2 minutes (c1) and 40 minutes (c2).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fdpb, pcg  # noqa: E402

N_UNIFORM = 2048
N_ATOM_NODES = 512


def sample_nodes(prob, seed):
    g = prob.grid
    rng = np.random.default_rng(seed)
    n = g.nx * g.ny * g.nz
    uni = rng.choice(n, size=N_UNIFORM, replace=False)
    pick = rng.choice(prob.mol.natoms, size=min(N_ATOM_NODES, prob.mol.natoms), replace=False)
    ijk = np.rint((prob.mol.xyz[pick] - g.origin) / g.h).astype(np.int64)
    ijk = np.clip(ijk, 0, np.array([g.nx, g.ny, g.nz]) - 1)
    near = ijk[:, 0] + g.nx * (ijk[:, 1] + g.ny * ijk[:, 2])
    jc, kc = g.ny // 2, g.nz // 2
    line = np.arange(g.nx) + g.nx * (jc + g.ny * kc)
    return np.unique(np.concatenate([uni, near, line]))


def main(which: str) -> None:
    prob = {"c1": synth.config1, "c2": synth.config2}[which]()
    g = prob.grid
    t0 = time.time()
    sysm = fdpb.assemble_problem(prob)
    print(f"{which}: setup {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    r6 = pcg.jpcg(sysm, 1e-6)
    print(f"{which}: {r6.iters} iterations to 1e-6 ({time.time() - t0:.1f} s)", flush=True)
    t0 = time.time()
    r12 = pcg.jpcg(sysm, 1e-12, maxiter=20 * max(sysm.dims), x0=r6.x)
    print(f"{which}: +{r12.iters} iterations to 1e-12 ({time.time() - t0:.1f} s)", flush=True)
    if not r12.converged:
        raise SystemExit(f"{which}: oracle did not reach 1e-12")
    x = r12.x
    rel = fdpb.true_relres(sysm, x)
    e = fdpb.energy(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.charge, x)
    nodes = sample_nodes(prob, seed=prob.seed + 17)
    flat = x.ravel()
    out = {
        "workload": prob.name,
        "dims": [g.nx, g.ny, g.nz],
        "h": g.h,
        "natoms": prob.mol.natoms,
        "generator_seed": prob.seed,
        "oracle": "FP64 Jacobi-PCG (oracle.pcg.jpcg), x0 = 0 to 1e-6, then warm-started to 1e-12",
        "iters_to_1e-6": int(r6.iters),
        "true_relres": rel,
        "max_abs_phi": float(np.abs(flat).max()),
        "energy_kcal": e,
        "sample_nodes": [int(v) for v in nodes],
        "sample_phi": [float(flat[v]) for v in nodes],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{prob.name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{which}: wrote {path}: relres {rel:.3e}, energy {e:.6f}, {len(nodes)} nodes", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
