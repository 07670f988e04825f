"""The library used from plain C: tests/abi_client/abi_client.c (built by the
repository's build entry point with gcc, linking libspc3d.so, the oracle and
the HIP runtime) runs setup, both gathers, the fused SDDMM+SpMM pass and the
scatter-reduce through the C entry points on a small block with global ids,
checks them against the oracle's C functions (integer and data-movement
results bit for bit, SDDMM and SpMM within 1e-5 of the magnitude sum) and
three error paths, and exits 0 only if all hold."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abi_client", "abi_client")


def test_c_client_runs_the_step_and_matches_the_oracle():
    if not os.path.exists(BIN):
        pytest.fail("tests/abi_client/abi_client is not built (run __graft_entry__.build())")
    print("c abi client", BIN, file=sys.stderr, flush=True)
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, file=sys.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "abi_client: ok" in r.stdout
