"""The C ABI used from plain C: tests/c_abi/abi_check.c (built by build())
drives the library through include/scprop.h alone, without Python or torch,
and checks norms, a finite gradient, the two LCAM entry points' bitwise
agreement and the refusal of bad arguments."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi", "abi_check")


def test_c_program_through_the_abi():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/c_abi/abi_check not built: run __graft_entry__.build()"
    print("[c abi] running tests/c_abi/abi_check", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "c abi ok" in r.stdout
