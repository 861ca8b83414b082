"""The C ABI from plain C: tests/helpers/abi_c_client.c (built by
__graft_entry__.build() with gcc against include/shaken.h and the HIP
runtime, no PyTorch) runs chains on the grid and single-workgroup kernels,
checks records against sd_observe and the resume identity, and checks that
argument errors come back as SD_EINVAL with a message."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "helpers", "abi_c_client.out")


def test_c_client_through_the_abi():
    if not os.path.exists(CLIENT):
        pytest.fail("the C ABI client is not built: run __graft_entry__.build()")
    print("C ABI client", flush=True)
    r = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi c client: ok" in r.stdout
