"""The served form's launch sharing (server.hip: share_launch), its source text
compiled for the host with g++ and run on seeded mixes of request tilings.
Checked: every request gets at least one workgroup and at most its tile count;
the workgroups stay within the co-resident capacity; no request can take a
workgroup step that would shorten the slowest iteration while capacity is
left; the slowest request runs exactly `chunk` iterations and every other one
between `chunk` and 16x `chunk`, in proportion to how much cheaper its
iteration is; the offsets are the running sums. No GPU involved."""
import os
import random
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SERVER = os.path.join(ROOT, "paper_1704_02745_amd", "csrc", "server.hip")

DRIVER = r"""
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>
struct Tiling { int ntiles, seglen, zchunk; };
#include "share.inc"
int main() {
    int n, cap, chunk;
    while (std::scanf("%d %d %d", &n, &cap, &chunk) == 3) {
        std::vector<Tiling> T(n);
        for (auto& t : T) std::scanf("%d %d %d", &t.ntiles, &t.seglen, &t.zchunk);
        std::vector<int> first(n + 1, 0), chunks(n, chunk);
        share_launch(T, cap, chunk, first, chunks);
        for (int i = 0; i <= n; ++i) std::printf("%d ", first[i]);
        for (int i = 0; i < n; ++i) std::printf("%d ", chunks[i]);
        std::printf("\n");
    }
    return 0;
}
"""


def _extract(src):
    a = src.index("constexpr double kBarrierNodes")
    b = src.index("void share_launch(")
    b = src.index("\n}\n", b) + 3
    return src[a:b]


def _cost(t, g, barrier):
    per = (t[0] + g - 1) // g
    return per * t[1] * (t[2] + 2) + barrier


@pytest.fixture(scope="module")
def share(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("share_host")
    src = open(SERVER).read()
    (d / "share.inc").write_text(_extract(src))
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    r = subprocess.run(["g++", "-std=c++17", "-O1", str(d / "drv.cpp"), "-o", str(exe)], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr
    barrier = float(re.search(r"kBarrierNodes = ([0-9.]+)", src).group(1))
    scale = int(re.search(r"kMaxChunkScale = (\d+)", src).group(1))
    return exe, barrier, scale


def test_share_launch_properties(share):
    exe, barrier, max_scale = share
    rng = random.Random(1234)
    cases = []
    for _ in range(300):
        n = rng.randint(1, 24)
        tilings = []
        for _ in range(n):
            seg = rng.randint(2, 40)
            nzc = rng.randint(1, 16)
            tilings.append((seg * nzc, rng.choice([1024, 512, 1536]), rng.choice([8, 12, 16, 32])))
        cap = rng.randint(n, 600)
        chunk = rng.choice([1, 8, 32])
        cases.append((n, cap, chunk, tilings))
    stdin = "".join(f"{n} {cap} {chunk}\n" + "".join(f"{a} {b} {c}\n" for a, b, c in t) for n, cap, chunk, t in cases)
    out = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for (n, cap, chunk, t), line in zip(cases, lines):
        v = [int(x) for x in line.split()]
        first, chunks = v[:n + 1], v[n + 1:]
        g = [first[i + 1] - first[i] for i in range(n)]
        assert first[0] == 0 and first[-1] <= cap
        assert all(1 <= g[i] <= t[i][0] for i in range(n))
        cost = [_cost(t[i], g[i], barrier) for i in range(n)]
        cmax = max(cost)
        left = cap - first[-1]
        # the slowest request could not have been sped up within the capacity left
        for i in range(n):
            if cost[i] == cmax and g[i] < t[i][0]:
                per = (t[i][0] + g[i] - 1) // g[i]
                want = (t[i][0] + per - 2) // (per - 1)
                assert want - g[i] > left
        for i in range(n):
            expect = max(chunk, min(int(chunk * min(max_scale, cmax / cost[i])), 2_000_000_000))
            assert chunks[i] == expect
            assert chunk <= chunks[i] <= max_scale * chunk
            if cost[i] == cmax:
                assert chunks[i] == chunk
