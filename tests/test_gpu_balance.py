"""Adaptive load balancing (Sec. 3.3) on the GPU against the oracle.

With the same per-domain capacities on both sides every tree rebuild must
give the same cuts, domains, order and forces.  Measured capacities are
checked end to end: after a measured step the test forms n_i / T_i from
the reported times and the step's contacts per domain, hands them to the
oracle, and the next rebuild must agree with the library's own.
"""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import both, compare_step

pytestmark = pytest.mark.gpu


def _capacities(P, seed):
    cap = np.random.default_rng(seed).uniform(0.5, 2.0, P)
    cap[3] = 0.0            # no measurement: counts as the mean
    cap[5] = float("nan")
    return cap


def test_given_capacities_2d():
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = both(pk, mu=0.3, n_domains=64, repartition_every=2)
    cap = _capacities(64, 11)
    sim.set_capacity(cap)
    ctx.set_domain_capacity(cap)
    for s in range(3):   # rebuild, descend, rebuild
        compare_step(sim, ctx, f"capacities 2D step{s}")


def test_given_capacities_3d():
    pk = inputs.lattice_3d(16, 16, 12, 5, gravity=1.0)
    sim, ctx = both(pk, mu=0.5, n_domains=16, repartition_every=2)
    cap = _capacities(16, 12)
    sim.set_capacity(cap)
    ctx.set_domain_capacity(cap)
    for s in range(3):
        compare_step(sim, ctx, f"capacities 3D step{s}")


def test_measured_capacities_drive_the_next_rebuild():
    """64x64 disks, 64 domains, rebuild every second step, threshold 0:
    step 1's measured times decide step 2's tree."""
    from paper_1104_3516_amd import binding
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = both(pk, mu=0.3, n_domains=64, repartition_every=2)
    with pytest.raises(binding.CDError):
        ctx.domain_times()
    ctx.set_load_balance(0.0)
    for s in range(2):
        compare_step(sim, ctx, f"measured step{s}")
        T, sig = ctx.domain_times()
        dom = ctx.contacts()["dom"].cpu().numpy()
        n = np.bincount(dom, minlength=64)
        print(f"[measured step{s}] T min/mean/max {T.min():.2f}/{T.mean():.2f}/{T.max():.2f} us "
              f"sigma_T {sig:.4f}", flush=True)
        assert np.all(T[n > 0] > 0.0)
        mean, mean2 = T.mean(), (T * T).mean()
        assert sig == pytest.approx(np.sqrt(max(mean2 - mean * mean, 0.0)) / mean, rel=1e-9)
    cap = np.where((n > 0) & (T > 0.0), n / np.where(T > 0.0, T, 1.0), 0.0)
    sim.set_capacity(cap)
    compare_step(sim, ctx, "measured rebuild")
    # the cuts moved away from the leaf-count cuts
    from oracle import cdref
    sim0 = cdref.Sim(cdref.make_params(2, pk.n_walls, mu=0.3, n_domains=64, repartition_every=2),
                     pk)
    for s in range(3):
        sim0.step()
    assert not np.array_equal(sim0.tree().cut, ctx.tree()["cut"])
