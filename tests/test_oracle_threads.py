"""The oracle's domains spread over OpenMP threads (the paper's domain-wise
scheme on shared memory, used for the multi-core CPU timing) give the same
simulation, bit for bit, as the serial loop: the domains of a sweep share
only the exchanged velocities, which they read, and write disjoint forces."""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs


def _run(oracle, pk, threads, steps, setup=None, **kw):
    oracle.set_threads(threads)
    try:
        sim = oracle.Sim(oracle.make_params(pk.dim, pk.n_walls, **kw), pk)
        if setup:
            setup(sim)
        its = [sim.step().iterations for _ in range(steps)]
        return its, sim.state(), sim.contacts()["R"]
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("case", ["plain", "random", "mixed", "3d"])
def test_threads_do_not_change_the_simulation(oracle, case):
    setup = None
    if case == "3d":
        pk = inputs.lattice_3d(8, 8, 6, 21, gravity=1.0)
        kw = dict(mu=0.5, n_domains=16, repartition_every=2)
    else:
        pk = inputs.lattice_2d(40, 40, 22)
        kw = dict(mu=0.3, n_domains=32, repartition_every=2)
        if case == "random":
            setup = lambda s: s.set_random(True, 4)
        if case == "mixed":
            setup = lambda s: s.set_mixed(0.02, 4)
    a = _run(oracle, pk, 1, 3, setup, **kw)
    b = _run(oracle, pk, 4, 3, setup, **kw)
    assert a[0] == b[0]
    for u, v in zip(a[1], b[1]):
        np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(a[2], b[2])
