"""The charge-key sort (setup.hip: bitonic_sort with k_bitonic_local and
k_bitonic_step), its source text compiled for the host with g++ and run on
seeded distinct 64-bit keys of every power-of-two size from 2 to 2^18: the
result is the ascending order. The LDS kernel runs with one thread per block
on the host (its steps pair disjoint positions, so any block size gives the
same result), the global steps thread by thread. No GPU involved."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SETUP = os.path.join(ROOT, "paper_1704_02745_amd", "csrc", "setup.hip")

DRIVER = r"""
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>
using std::min;
struct D3 { unsigned x = 1, y = 1, z = 1; D3() {} D3(unsigned a) : x(a) {} };
using dim3 = D3;
static D3 blockIdx, threadIdx, blockDim, gridDim;
typedef void* hipStream_t;
typedef int pb_status;
enum { PB_OK = 0 };
static int hipGetLastError() { return 0; }
#define PB_HIP(x) (void)(x)
#define __global__
#define __launch_bounds__(n)
#define __restrict__
#define __shared__ static
static void __syncthreads() {}
#include "sort.inc"
int main() {
    int n;
    while (std::scanf("%d", &n) == 1) {
        std::vector<uint64_t> a(n);
        for (auto& v : a) std::scanf("%llu", (unsigned long long*)&v);
        bitonic_sort(a.data(), n, nullptr);
        for (auto v : a) std::printf("%llu ", (unsigned long long)v);
        std::printf("\n");
    }
    return 0;
}
"""

LAUNCH = r"""
template <class F, class... A>
static void host_launch(F* f, D3 grid, D3 block, A... args) {
    // the LDS kernel with one thread per block (its steps are then taken in
    // order within the block); the global steps thread by thread
    const bool local = (void*)f == (void*)&k_bitonic_local;
    gridDim = grid;
    blockDim = local ? D3(1) : block;
    for (unsigned b = 0; b < grid.x; ++b)
        for (unsigned t = 0; t < blockDim.x; ++t) {
            blockIdx.x = b;
            threadIdx.x = t;
            f(args...);
        }
}
#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) host_launch(K, G, B, __VA_ARGS__)
"""


def _block(src, start):
    i = src.index(start)
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return src[i:k + 1] + "\n"
    raise ValueError(start)


@pytest.fixture(scope="module")
def sorter(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sort_host")
    src = open(SETUP).read()
    inc = (_block(src, "__global__ void k_bitonic_step(") + "constexpr int kSortChunk = " +
           src.split("constexpr int kSortChunk = ")[1].split(";")[0] + ";\n" +
           _block(src, "__global__ __launch_bounds__(1024) void k_bitonic_local(") + LAUNCH +
           _block(src, "inline unsigned blocks_for(") + _block(src, "pb_status bitonic_sort("))
    (d / "sort.inc").write_text(inc)
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    r = subprocess.run(["g++", "-std=c++17", "-O2", str(d / "drv.cpp"), "-o", str(exe)], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_bitonic_sort_orders_keys(sorter):
    rng = np.random.default_rng(4242)
    sizes = [1 << e for e in range(1, 19)]
    keys = []
    for n in sizes:
        k = rng.choice(np.uint64(1) << np.uint64(40), size=n, replace=False).astype(np.uint64)
        keys.append(k)
    stdin = "".join(f"{len(k)}\n" + " ".join(str(int(v)) for v in k) + "\n" for k in keys)
    out = subprocess.run([str(sorter)], input=stdin, capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().split("\n")
    assert len(lines) == len(keys)
    for k, line in zip(keys, lines):
        got = np.array([int(v) for v in line.split()], dtype=np.uint64)
        assert np.array_equal(got, np.sort(k)), len(k)
