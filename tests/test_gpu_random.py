"""Random sequential order (Sec. 2.1) on the GPU against the oracle: the same
SplitMix64 draws order every domain's contacts in every sweep on both sides,
and the forces, states and sweep counts must agree (bit for bit up to the
stop decision's rounding) in each sweep form: contact data staged in LDS,
read ahead into registers (solve mode 2), and particle records in global
memory (a domain too large for LDS)."""
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import both, compare_step

pytestmark = pytest.mark.gpu


def _random_pair(pk, seed, solve_mode=1, **kw):
    sim, ctx = both(pk, solve_mode=solve_mode, **kw)
    sim.set_random(True, seed)
    ctx.set_random_order(True, seed)
    return sim, ctx


@pytest.mark.parametrize("solve_mode", [1, 2])
def test_random_2d_several_domains(solve_mode):
    """64x64 disks, 16 domains, three steps to the tolerance (the draws of
    each step use its index)."""
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = _random_pair(pk, 11, solve_mode, mu=0.3, n_domains=16, repartition_every=2)
    for s in range(3):
        compare_step(sim, ctx, f"random mode{solve_mode} step{s}")


def test_random_single_domain_global_records():
    """80x80 disks in one domain: its particle records live in global memory,
    the draws and ranks (about 120 KB) in LDS; 20 sweeps."""
    pk = inputs.lattice_2d(80, 80, 1000)
    sim, ctx = _random_pair(pk, 12, mu=0.3, n_domains=1, fixed_iters=20)
    compare_step(sim, ctx, "random one domain")
    assert ctx.timing().global_records == 1


def test_random_single_domain_records_move_to_global_memory():
    """64x64 disks in one domain: the particle records (about 150 KB) fit in
    LDS alone but not beside the draws and ranks, so the random order keeps
    them in global memory; 10 sweeps."""
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = _random_pair(pk, 15, mu=0.3, n_domains=1, fixed_iters=10)
    compare_step(sim, ctx, "random one domain 64x64")
    assert ctx.timing().global_records == 1


def test_random_3d():
    pk = inputs.lattice_3d(12, 12, 10, 13, gravity=1.0, top_velocity=1e-3)
    sim, ctx = _random_pair(pk, 13, mu=0.5, n_domains=16, repartition_every=2, fixed_iters=40)
    for s in range(2):
        compare_step(sim, ctx, f"random 3D step{s}")


def test_random_full_size_spheres_folded_decision():
    """128x128x64 spheres, 16,384 domains: more workgroups than fit at once,
    so the stop decision is folded into workgroup 0 beside the random
    order's serial walk; 3 sweeps."""
    pk = inputs.config("spheres_1m")
    sim, ctx = _random_pair(pk, 16, mu=0.5, n_domains=16384, repartition_every=10,
                            fixed_iters=3)
    compare_step(sim, ctx, "random 1m spheres fixed3")
    assert ctx.timing().staged == 2


@pytest.mark.parametrize("P", [1, 4])
def test_random_chain_to_the_tolerance(P):
    """The compressed chain of Fig. 13(a), 128 disks: the same sweep count."""
    pk = inputs.chain_2d(128, 1.0)
    sim, ctx = _random_pair(pk, 14, mu=0.3, n_domains=P, max_iter=100000)
    io, ig = compare_step(sim, ctx, f"random chain P={P}")
    assert ig.status == 0


def test_random_order_is_refused_where_unsupported():
    from paper_1104_3516_amd import binding
    pk = inputs.lattice_2d(16, 16, 1000)
    _, ctx = both(pk, solve_mode=0, mu=0.3, n_domains=4)
    ctx.set_random_order(True, 1)
    with pytest.raises(binding.CDError):
        ctx.step()
    _, ctx = both(pk, mu=0.3, n_domains=4)
    ctx.set_adjoint(4)
    with pytest.raises(binding.CDError):
        ctx.set_random_order(True, 1)
    _, ctx = both(pk, mu=0.3, n_domains=4)
    ctx.set_random_order(True, 1)
    with pytest.raises(binding.CDError):
        ctx.set_mixed_update(0.2, 1)
    with pytest.raises(binding.CDError):
        ctx.set_load_balance(0.1)
    with pytest.raises(binding.CDError):
        binding.Batch([ctx]).step()


def test_random_order_needs_lds_for_its_ranks():
    """120x120 disks in one domain: 16.5k contacts need more than 160 KiB of
    draws and ranks; the step reports the capacity error."""
    from paper_1104_3516_amd import binding
    pk = inputs.lattice_2d(120, 120, 1000)
    _, ctx = both(pk, mu=0.3, n_domains=1, fixed_iters=2)
    ctx.set_random_order(True, 1)
    with pytest.raises(binding.CDError) as e:
        ctx.step()
    assert e.value.code == binding.ECAPACITY
