"""The command line (python -m paper_2302_10083_amd): argument handling on
the CPU, and on the GPU the paper's majority example and a file-based table
against the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2302_10083_amd import inputs
from paper_2302_10083_amd.__main__ import cube_string, read_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cli(*args):
    return subprocess.run([sys.executable, "-m", "paper_2302_10083_amd"] + [str(a) for a in args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_cube_string_digit_order():
    # s_1 is the least significant ternary digit (Sec. 4.2), printed leftmost
    assert cube_string(3, 14) == "*11"
    assert cube_string(3, 16) == "1*1"
    assert cube_string(3, 22) == "11*"
    assert cube_string(0, 0) == ""


def test_read_table_hex_and_file(tmp_path):
    assert read_table(3, "0xE8").tolist() == [0xE8]
    assert read_table(6, "0x1" + "0" * 15).tolist() == [0, 0x10000000]
    with pytest.raises(SystemExit):
        read_table(3, "0x1" + "0" * 8)  # needs a second word; n = 3 has one
    tt = inputs.bernoulli(9, 0.5, 3)
    f = tmp_path / "t.bin"
    np.asarray(tt, dtype="<u4").tofile(f)
    assert np.array_equal(read_table(9, str(f)), tt)
    with pytest.raises(SystemExit):
        read_table(10, str(f))


@pytest.mark.gpu
def test_cli_majority_example():
    r = _cli(3, "0xE8")
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["3", "*11", "1*1", "11*"]
    r = _cli(3, "0xE8", "--cnf")  # NOT maj: the cubes with two zeros
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["3", "*00", "0*0", "00*"]  # increasing index: 2, 6, 18


@pytest.mark.gpu
def test_cli_file_matches_oracle(tmp_path):
    from _gpu_common import oracle_primes

    n = 14
    tt = inputs.bernoulli(n, 0.8, 41)
    f = tmp_path / "t.bin"
    np.asarray(tt, dtype="<u4").tofile(f)
    _, _, ref = oracle_primes(n, tt)
    r = _cli(n, f, "--rho")
    assert r.returncode == 0, r.stderr
    out = [int(x) for x in r.stdout.split()]
    assert out[0] == len(ref) and out[1:] == ref.tolist()
    r = _cli(n, f, "--sliced", 2, "--limit", 5)
    assert r.returncode == 0, r.stderr
    out = r.stdout.split()
    assert int(out[0]) == len(ref) and out[1:] == [cube_string(n, int(x)) for x in ref[:5]]
    r = _cli(n, f, "--count-only")
    assert r.returncode == 0 and r.stdout.split() == [str(len(ref))]
