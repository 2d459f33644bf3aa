"""The label harness of the learned switch plans the levels after a forced
direction on the host with the search kernel's own alpha/beta rule
(paper_2012_10026_amd/csrc/switch.h, compiled here for the host with g++).
Level by level, that rule gives the oracle's alpha/beta schedule (Alg 2's
switch in the integer form the library uses)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r"""
#include <cstdio>
#include "switch.h"
int main() {
  long long n, alpha, beta;
  int levels;
  while (std::scanf("%lld %lld %lld %d", &n, &alpha, &beta, &levels) == 4) {
    long long nf[64], mf[64], mu[64];
    for (int i = 0; i < levels; ++i) std::scanf("%lld %lld %lld", &nf[i], &mf[i], &mu[i]);
    int dir = 0;
    std::printf("0");
    for (int e = 1; e < levels; ++e) {
      dir = rbfs::heuristic_dir(dir, nf[e], mf[e], mu[e], nf[e - 1], n, (int)alpha, (int)beta);
      std::printf(" %d", dir);
    }
    std::printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def host_rule(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("switch_host")
    src, exe = d / "rule.cpp", d / "rule"
    src.write_text(SRC)
    subprocess.run(["g++", "-O1", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_2012_10026_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


def test_host_rule_gives_the_oracle_schedule(host_rule):
    rng = np.random.default_rng(11)
    cases, lines = [], []
    for _ in range(400):
        levels = int(rng.integers(1, 24))
        n = int(rng.integers(10, 10 ** 9))
        nf = rng.integers(1, max(2, n // 4), size=levels)
        mf = nf * rng.integers(1, 64, size=levels)
        mu = np.sort(rng.integers(0, 2 ** 40, size=levels))[::-1]
        alpha, beta = int(rng.integers(1, 129)), int(rng.integers(1, 33))
        cases.append((nf, mf, mu, n, alpha, beta))
        lines.append("%d %d %d %d %s" % (n, alpha, beta, levels, " ".join(
            "%d %d %d" % (a, b, c) for a, b, c in zip(nf, mf, mu))))
    out = subprocess.run([host_rule], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    switches = 0
    for (nf, mf, mu, n, alpha, beta), got in zip(cases, out):
        want = oracle.heuristic_schedule(nf, mf, mu, n, alpha, beta).tolist()
        assert [int(x) for x in got.split()] == want
        switches += sum(a != b for a, b in zip(want, want[1:]))
    assert switches > 100  # both switches of the rule occur many times
