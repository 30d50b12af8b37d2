"""The library called from plain C (tests/c_abi/check_build.c): no Python, no
torch, device memory allocated by the caller.  The program checks its grid
against the contract's invariants and the host-recomputed cell boxes."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_abi", "check_build")


def test_c_caller_builds_a_valid_grid():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(BIN):
        pytest.skip("tests/c_abi/check_build is not built (python -m paper_2403_10647_amd.build)")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok ") and int(r.stdout.split()[1]) > 5000
