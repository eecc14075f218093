"""The library through its C ABI alone: a C program (tests/c_abi) that
allocates with hipMalloc, calls gls_factor / gls_whiten_fixed /
gls_solve_block / gls_free and checks b_i against Eq. (1) computed on the
host with its own Cholesky factor."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c_program_through_the_abi():
    exe = os.path.join(HERE, "c_abi", "gls_c_check")
    assert os.path.exists(exe), "not built: run python -m paper_1210_7325_amd.build"
    print("c-abi program", file=sys.stderr, flush=True)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    print(r.stdout, file=sys.stderr, flush=True)
    assert r.returncode == 0, r.stdout
    assert "max rel err" in r.stdout
