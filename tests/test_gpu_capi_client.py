"""The plain-C client of the C ABI (tests/capi_client.c, built by the package build next to the
library) run on the GPU: a float32 fixed point and a batched bf16 closed form, checked by the
client itself without Python or torch."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "_build", "capi_client")


def test_c_client_runs_on_the_gpu():
    assert os.path.exists(CLIENT), "tests/_build/capi_client is built by __graft_entry__.build()"
    r = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
