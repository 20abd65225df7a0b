"""The C ABI called from plain C (paper_2409_02294_amd/examples/solve_c.c,
built by the package build): impulse responses in FP64 and FP32 against the
kernel values at every cell, a batched call against single solves, and a
rejected size.  No torch is involved in that process."""
import os
import subprocess

import pytest

from conftest import ROOT

pytestmark = pytest.mark.gpu

EXAMPLE = os.path.join(ROOT, "paper_2409_02294_amd", "examples", "solve_c")


def test_c_program_solves():
    assert os.path.exists(EXAMPLE), "examples/solve_c is not built: run python -m paper_2409_02294_amd.build"
    r = subprocess.run([EXAMPLE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().endswith("ok")
