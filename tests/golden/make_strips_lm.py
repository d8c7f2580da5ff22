"""Writes strips20000_lm_oracle.json: the oracle's fixed-budget LM run on
the 20,000-camera strip scene (seed 1: 5 flight strips plus cross strips,
5M points, ~20M observations), the scene the mixed-precision path is
reported on.

The run starts far from the optimum: the first step lowers F about 200-fold
and the second overshoots (rejected), so at the benchmark's PCG tolerance
(rel 1e-6) two correct runs part ways (a 3e-5 difference of the first
step's F', which that tolerance allows, becomes 8% after the rejection).
The stored run therefore solves every step to rel 1e-12 (at most 20000 PCG
iterations, which no step reaches), where the LM path is reproducible: a
solve stopped by an iteration cap is not (its iterate depends on the
rounding of thousands of CG steps).

Calls only the scene generator (random draws) and the oracle, through the
same run as make_partition_lm.py: observations = the oracle's projection of
the true parameters plus the scene's noise; 10 LM iterations from the
perturbed start, lambda0 = 1e-4, block-Jacobi PCG.  The oracle holds about
8 GB of host memory on this scene and takes 20-30 minutes on 8 cores.

Usage: python tests/golden/make_strips_lm.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import make_partition_lm  # noqa: E402
from paper_2307_08383_amd import scenegen  # noqa: E402

OUT = os.path.join(HERE, "strips20000_lm_oracle.json")
PCG_TOL = 1e-12
PCG_MAX_ITER = 20000

if __name__ == "__main__":
    make_partition_lm.run(
        scenegen.strips_scene(seed=1, with_stats=False), OUT,
        "Oracle (FP64, CPU) LM run on the 20,000-camera strip scene (seed 1): 10 iterations from the "
        "perturbed start, lambda0 1e-4, block-Jacobi PCG to rel 1e-12, cap 20000. Written by "
        "tests/golden/make_strips_lm.py from the oracle only.", pcg_tol=PCG_TOL, pcg_max_iter=PCG_MAX_ITER)
