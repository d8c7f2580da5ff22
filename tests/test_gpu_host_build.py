"""The host build of a context (internal order, pattern, couples, FSAI and
network index structures) does not depend on its thread count (needs a
GPU): contexts built with 1 and with 7 host threads (BA_THREADS, read once
per process, so each count runs in a child process) give bit-identical
patterns, RCS, PCG iterates with block-Jacobi, FSAI and the learned factor,
and LM steps, on the aerial grid, the long-track scene and a shared-
intrinsics scene with long tracks.  Also: a non-finite pixel, found on the
device, is reported with the caller's index of its observation."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")

CHILD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "host_build_child.py")


def _run(threads):
    env = dict(os.environ, BA_THREADS=str(threads))
    print(f"host build with {threads} threads", flush=True)
    out = subprocess.run([sys.executable, CHILD, "aerial", "long", "shared_long"], env=env, capture_output=True,
                         text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


@pytest.mark.timeout(600)
def test_host_build_independent_of_thread_count():
    a, b = _run(1), _run(7)
    assert a.keys() == b.keys()
    for scene in a:
        assert a[scene] == b[scene], scene


@pytest.mark.parametrize("k", [0, 3, 1234])
def test_non_finite_pixel_reported(k):
    s = scenegen.aerial_grid_scene(seed=3, nx=10, ny=8, n_pts=500, with_stats=False)
    uv = orc.observations(s)
    uv[1, k] = np.inf
    uv[0, k + 7] = np.nan
    with pytest.raises(ba.BAError) as ei:
        create(s, uv)
    assert ei.value.status == ba.BA_ERR_INVALID_ARG
    assert f"observation {k} is not finite" in str(ei.value)
