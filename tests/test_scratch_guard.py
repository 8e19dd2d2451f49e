"""Guard against kernels whose private (scratch) memory could exhaust the
per-queue scratch reservation of the HIP runtime (it reserves bytes per lane
x 64 lanes x 32 waves x 256 CUs for every hardware queue a process uses and
keeps it): every kernel the library launches unconditionally stays within
kMaxLaneScratch bytes per lane, and only the lane forms of the Fock and
gradient class kernels, which the engine checks against that bound at run
time, may exceed it.  Reads the compiler's resource remarks that the build
writes next to each object file."""

import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENGINE = os.path.join(ROOT, "paper_1601_02713_amd", "csrc", "engine.cpp")


def _records():
    recs = []
    for f in glob.glob(os.path.join(ROOT, "_build", "obj", "*.resources.txt")):
        name = None
        for ln in open(f):
            ln = ln.strip()
            if ln.startswith("Function Name:"):
                name = ln.split(":", 1)[1].strip()
            elif ln.startswith("ScratchSize") and name:
                recs.append((int(ln.split(":")[1]), name))
    return recs


def test_scratch_bound_and_unconditional_kernels():
    src = open(ENGINE).read()
    kmax = int(re.search(r"constexpr int kMaxLaneScratch = (\d+);", src).group(1))
    # the reservation of one hardware queue at full occupancy stays within 2 GiB
    assert kmax * 64 * 32 * 256 <= 2 ** 31
    # every lane-form selection tests the context's bound: Fock (FP64 and
    # mixed) and gradient at context creation, the Fock autotuner and the
    # gradient's; the environment can only lower that bound
    assert len(re.findall(r"private_bytes\[q\]\[[0-2]\] <= c->lane_scratch_max", src)) >= 5
    assert "int lane_scratch_max = lane_scratch_bound();" in src
    assert "std::min(kMaxLaneScratch, atoi(v))" in src
    recs = _records()
    if not recs:
        pytest.skip("no resource records: build the library first")
    lane = re.compile(r"^_ZN4bscf16(fock_unit_kernel|grad_unit_kernel)")
    over = [(s, n) for s, n in recs if s > kmax and not lane.match(n)]
    assert not over, over
