"""Full-size parity in tolerance mode: the benchmark workloads' converged
time steps (test (I) every sweep, warm start, tree descent between
repartitions) against the oracle with the same partition and order
(Sec. 2.1, 3.1, 3.2).  The oracle spreads each sweep's domains over OpenMP
threads (the results do not depend on it)."""
import os

import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import both, compare_step

pytestmark = pytest.mark.gpu


def _threads():
    from oracle import cdref
    cdref.set_threads(max(1, min(16, os.cpu_count() or 1)))


def test_disks_262k_2048_domains_three_tolerance_steps():
    """512x512 disks at 2,048 domains with the benchmark's parameters
    (alpha = 1e-6, test (I), at most 2,000 sweeps, warm start, repartition
    every 10 steps): step 0 from rest reaches the sweep cap, steps 1 and 2
    are warm-started and descend the tree of step 0."""
    _threads()
    pk = inputs.config("disks_262k")
    kw = dict(mu=0.3, alpha=1e-6, criterion=0, max_iter=2000, n_domains=2048,
              repartition_every=10, warm_start=1)
    sim, ctx = both(pk, **kw)
    for s in range(3):
        compare_step(sim, ctx, f"262k tol step {s}")


def test_spheres_1m_16384_domains_two_tolerance_steps():
    """128x128x64 spheres at 16,384 domains with the benchmark's parameters
    except the sweep cap, lowered to 400 so that the oracle's two steps take
    about a minute: step 0 from rest stops at the cap, step 1 is
    warm-started from it and descends the tree."""
    _threads()
    pk = inputs.config("spheres_1m")
    kw = dict(mu=0.5, alpha=1e-6, criterion=0, max_iter=400, n_domains=16384,
              repartition_every=10, warm_start=1)
    sim, ctx = both(pk, **kw)
    for s in range(2):
        compare_step(sim, ctx, f"1m spheres tol step {s}")
