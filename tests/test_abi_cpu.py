"""Host-only checks of the C ABI: the library loads, exports every function
that include/dqmc.h declares, and its pure size functions and argument checks
behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2302_10083_amd import dqmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(dqmc_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    lib = dqmc.load()
    names = _declared_functions()
    assert {"dqmc_create", "dqmc_primes", "dqmc_implicants", "dqmc_extract", "dqmc_primes_batch"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), name
        ctypes.cast(getattr(lib, name), ctypes.c_void_p)  # resolvable symbol


@pytest.mark.parametrize("n", list(range(0, 26)))
def test_sizes(n):
    assert dqmc.dqmc_num_cubes(n) == 3**n
    assert dqmc.dqmc_tt_words(n) == max(1, 2 ** (n - 5)) if n >= 5 else dqmc.dqmc_tt_words(n) == 1
    # one tile of 8-word blocks up to n = 12, then 3^(n-12) slots of the tile
    # (17,496 words) and 8 zero words
    assert dqmc.dqmc_state_words(n) == (17504 * 3 ** (n - 12) if n > 12 else 8 * 3 ** max(n - 5, 0))
    if n > 12:
        assert dqmc.dqmc_state_words(n) * 4 % 128 == 0  # slots start on 128-byte lines
    assert dqmc.dqmc_dense_words(n) == (3**n + 63) // 64
    # every cube has a place: 243 per 8-word block (or all of them in one block)
    blocks = 2187 * 3 ** (n - 12) if n > 12 else dqmc.dqmc_state_words(n) // 8
    assert blocks * 243 >= 3**n


@pytest.mark.parametrize("n", [-1, 26, 100])
def test_sizes_out_of_range(n):
    assert dqmc.dqmc_num_cubes(n) == 0
    assert dqmc.dqmc_state_words(n) == 0


def test_null_context_is_einval():
    lib = dqmc.load()
    assert lib.dqmc_primes(None, 4, None, None, None, 0, None, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_implicants(None, 4, None, None, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_extract(None, 4, None, None, 0, None, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_primes_batch(None, None, 0, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_primes_sliced(None, 26, 1, None, 0, None, None, None, 0, None, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_primes_sliced_multi(None, 26, 1, None, 0, None, None, 0, None, 0, None, None) == dqmc.DQMC_EINVAL
    assert lib.dqmc_last_error(None) == b"no context"
    lib.dqmc_destroy(None)  # ignored


def test_create_without_device_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = dqmc.load()
    out = ctypes.c_void_p(1)
    rc = lib.dqmc_create(0, ctypes.byref(out))
    assert rc in (dqmc.DQMC_EDEVICE, dqmc.DQMC_ENOMEM)
    assert not out.value


def test_binding_shares_torchs_hip_runtime():
    """Loading the library before torch is imported must not bring up a
    second HIP runtime next to torch's own copy."""
    import subprocess
    import sys

    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2302_10083_amd import dqmc\n"
            "dqmc.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys

    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout.strip() == ""
