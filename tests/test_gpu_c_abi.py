"""The C ABI from plain C: paper_2302_10083_amd/examples/c_primes (built by
build()) uses hipMalloc buffers and the system HIP runtime, without Python or
torch in its process.  Its list and count must equal the oracle's, and its
dqmc_primes_batch call on a device job array must agree with them."""
import os
import subprocess

import numpy as np
import pytest

from paper_2302_10083_amd import build as hip_build
from paper_2302_10083_amd import inputs

from _gpu_common import log, make_tt, oracle_primes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,kind", [(0, "const1"), (3, "parity"), (9, "bern0.7"), (14, "dnf40"), (18, "bern0.9")])
def test_c_program_matches_oracle(n, kind, tmp_path):
    if not os.path.exists(hip_build.EXAMPLE_BIN):
        pytest.fail("the C example is not built (run build())")
    tt = make_tt(n, kind, 9300 + n)
    ttf, outf = tmp_path / "tt.bin", tmp_path / "out.bin"
    np.asarray(tt, dtype="<u4").tofile(ttf)
    log("c_primes n=%d %s" % (n, kind))
    r = subprocess.run([hip_build.EXAMPLE_BIN, str(n), str(ttf), str(outf)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(outf, dtype="<u8")
    count = int(out[0])
    _, _, ref = oracle_primes(n, tt)
    assert count == len(ref)
    assert np.array_equal(out[1:1 + count], ref)
    assert np.array_equal(out[1 + count:1 + 2 * count], ref)  # dqmc_extract on the same bitmap
    if n <= 16:
        # dqmc_primes_batch on a device-resident job array, checked by the program
        assert "batch ok" in r.stdout, r.stdout


def test_c_program_rejects_bad_n(tmp_path):
    r = subprocess.run([hip_build.EXAMPLE_BIN, "26", str(tmp_path / "x"), str(tmp_path / "y")], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 1 and "out of range" in r.stderr
