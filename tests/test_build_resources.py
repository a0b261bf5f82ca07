"""Kernel resource usage of the gfx950 build (CPU only: hipcc cross-compiles).

The walk is bound by instruction issue, so a per-lane array that the compiler
moves to scratch memory, or promotes to LDS, slows every step several-fold
without changing a single result; the parity tests cannot see it.  This
compiles the kernels with resource remarks and checks that no kernel uses
scratch and that the walk kernels use only the LDS they declare.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2603_15780_amd import build as B

# LDS each walk kernel declares itself (bytes per block)
WALK_LDS = {"k_walk": 0, "k_walk2": 0, "k_walk_bwd": 0, "k_exp_plain": 0, "k_walk_gx": 4 * 4097}


@pytest.fixture(scope="module")
def remarks(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    kernels = {}
    for src in (s for s in B.SOURCES if s.endswith(".hip")):
        out = tmp_path_factory.mktemp("res") / (src + ".o")
        cmd = [B.HIPCC, *B.HIP_FLAGS, "--cuda-device-only", "-c", "-Rpass-analysis=kernel-resource-usage",
               "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC, os.path.join(B.CSRC, src), "-o", str(out)]
        r = subprocess.run(cmd, capture_output=True, text=True, check=True)
        for block in r.stderr.split("Function Name: ")[1:]:
            name = block.split()[0]
            sc = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", block)
            lds = re.search(r"LDS Size \[bytes/block\]: (\d+)", block)
            if sc and lds:
                kernels[name] = (int(sc.group(1)), int(lds.group(1)))
    assert kernels, "no resource remarks parsed"
    return kernels


def test_no_kernel_uses_scratch(remarks):
    bad = {k: v for k, v in remarks.items() if v[0] > 0}
    assert not bad, bad


def test_walk_kernels_use_only_their_declared_lds(remarks):
    seen = set()
    for name, (_, lds) in remarks.items():
        m = re.match(r"_ZN2sg12_GLOBAL__N_1\d+(k_[a-z0-9_]+?)(I|E)", name)
        if not m or m.group(1) not in WALK_LDS:
            continue
        seen.add(m.group(1))
        assert lds == WALK_LDS[m.group(1)], (name, lds)
    assert seen == set(WALK_LDS), seen
