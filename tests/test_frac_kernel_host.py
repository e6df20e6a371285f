"""The fractional-edge device kernels (k_cell_keys, k_bitonic_step,
k_cell_bounds, k_edges_fraction), their source text compiled for the host
with g++ under AddressSanitizer and UBSan and run through pb_setup_ex's host
steps: every access stays inside its exactly sized buffer, and the edge
dielectrics equal the oracle's weighted harmonic edges (section 2.7, read as
the inside fraction of each edge) bit for bit. No GPU involved."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import fdpb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SETUP = os.path.join(ROOT, "paper_1704_02745_amd", "csrc", "setup.hip")
HARNESS = os.path.join(ROOT, "tests", "host_kernels", "frac_edges_host.cpp")
KERNELS = ["int padded_cell(", "void k_cell_keys(", "void k_cell_bounds(", "void k_edges_fraction(",
           "void k_bitonic_step("]


def _extract(src, name):
    i = src.index(name)
    i = src.rfind("\n", 0, i) + 1
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return src[i:k + 1] + "\n"
    raise ValueError(name)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("frac_host")
    src = open(SETUP).read()
    seg = src[src.index("constexpr int kMaxSegments"):]
    seg = seg[:seg.index("\n") + 1]
    with open(d / "kernels.inc", "w") as f:
        f.write(seg + "".join(_extract(src, n) for n in KERNELS))
    exe = d / "frac_edges_host"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", str(d), HARNESS, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return d, exe


CASES = {"c0": lambda: synth.config0(),
         "thin": lambda: synth.small_problem(40, 9, 23, 6, seed=8),
         "ragged": lambda: synth.small_problem(61, 53, 47, 80, seed=7),
         "dense": lambda: synth.small_problem(24, 22, 20, 60, seed=3)}


@pytest.mark.parametrize("name", list(CASES))
def test_device_kernel_text_matches_oracle_in_bounds(harness, name):
    d, exe = harness
    prob = CASES[name]()
    g = prob.grid
    ex, ey, ez = fdpb.fractional_edges(g.nx, g.ny, g.nz, g.h, g.origin, prob.mol.xyz, prob.mol.radius,
                                       prob.eps_in, prob.eps_out)
    assert ((ex > prob.eps_in) & (ex < prob.eps_out)).any()
    path = d / (name + ".bin")
    with open(path, "wb") as f:
        np.array([g.nx, g.ny, g.nz], np.int32).tofile(f)
        np.array([g.h, *g.origin, prob.eps_in, prob.eps_out], np.float64).tofile(f)
        np.array([len(prob.mol.radius)], np.int64).tofile(f)
        for a in (prob.mol.xyz, prob.mol.radius, ex, ey, ez):
            np.ascontiguousarray(a, np.float64).tofile(f)
    r = subprocess.run([str(exe), str(path)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert " mismatching 0 " in r.stdout, r.stdout
