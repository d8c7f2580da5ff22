"""The host build's thread helpers (host_par.hpp) on the CPU: a counting
sort is stable and drops negative keys, results do not depend on the
thread count (BA_THREADS 1, 3, 16), per-index work lands at its index, and a
worker's exception reaches the caller.  The check program is built with g++
(no GPU, no HIP)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "host_par_check.cpp")


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host_par") / "host_par_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", SRC, "-o", exe], check=True)
    return exe


def _run(exe, threads, n, n_keys):
    env = dict(os.environ, BA_THREADS=str(threads))
    out = subprocess.run([exe, str(n), str(n_keys)], env=env, capture_output=True, text=True, check=True).stdout
    lines = {}
    for line in out.strip().splitlines():
        name, _, rest = line.partition(" ")
        lines[name] = rest
    return (int(lines["threads"]), np.array(lines["ptr"].split(), np.int64),
            np.array(lines["out"].split(), np.int64), int(lines["sum"]), lines["caught"] == "1")


def _keys(n, n_keys):
    """The program's xorshift keys, formed the same way in Python."""
    x = 88172645463325252
    mask = (1 << 64) - 1
    keys = np.empty(n, np.int64)
    for i in range(n):
        x ^= (x << 13) & mask
        x ^= x >> 7
        x ^= (x << 17) & mask
        keys[i] = x % (n_keys + 3) - 3
    return keys


@pytest.mark.parametrize("n,n_keys", [(1, 5), (1000, 7), (300000, 97)])
def test_counting_sort_and_threads(prog, n, n_keys):
    keys = _keys(n, n_keys)
    ref_out = np.concatenate([np.flatnonzero(keys == k) for k in range(n_keys)]) if n else np.zeros(0, np.int64)
    ref_ptr = np.concatenate([[0], np.cumsum([np.count_nonzero(keys == k) for k in range(n_keys)])])
    ref_sum = int((keys * keys + np.arange(n)).sum())
    runs = [_run(prog, t, n, n_keys) for t in (1, 3, 16)]
    assert [r[0] for r in runs] == [1, 3, 16]
    for _, ptr, out, s, caught in runs:
        assert np.array_equal(ptr, ref_ptr)
        assert np.array_equal(out, ref_out)   # stable: ascending index inside each key
        assert s == ref_sum
        assert caught
