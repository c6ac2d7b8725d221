"""Mixed sequential/parallel update (Sec. 2.3) on the GPU against the oracle:
the same pair numbers select the parallel contacts on both sides, and the
colours, order, forces and iteration counts must agree bit for bit.

These lattice piles lose convergence at a small parallel share (between
0.03 and 0.05 for 64 x 64 disks), so the cases that run to the tolerance
use p = 0.02, and larger shares run a fixed number of sweeps of one step,
where the forces grow but stay finite and comparable."""
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import both, compare_step

pytestmark = pytest.mark.gpu


def _mixed_pair(pk, p, seed, solve_mode=1, **kw):
    sim, ctx = both(pk, solve_mode=solve_mode, **kw)
    sim.set_mixed(p, seed)
    ctx.set_mixed_update(p, seed)
    return sim, ctx


@pytest.mark.parametrize("solve_mode", [1, 2])
def test_mixed_2d_several_domains(solve_mode):
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = _mixed_pair(pk, 0.02, 5, solve_mode, mu=0.3, n_domains=16, repartition_every=2)
    for s in range(3):
        compare_step(sim, ctx, f"mixed p=0.02 mode{solve_mode} step{s}")


@pytest.mark.parametrize("solve_mode", [1, 2])
def test_mixed_2d_large_share_fixed_sweeps(solve_mode):
    pk = inputs.lattice_2d(64, 64, 1000)
    sim, ctx = _mixed_pair(pk, 0.3, 5, solve_mode, mu=0.3, n_domains=16, fixed_iters=40)
    compare_step(sim, ctx, f"mixed p=0.3 fixed 40 mode{solve_mode}")


def test_mixed_single_domain_global_records():
    pk = inputs.lattice_2d(96, 96, 1000)
    sim, ctx = _mixed_pair(pk, 0.02, 6, mu=0.3, n_domains=1, max_iter=3000)
    compare_step(sim, ctx, "mixed p=0.02 one domain")
    assert ctx.timing().global_records == 1


def test_mixed_3d():
    pk = inputs.lattice_3d(12, 12, 10, 13, gravity=1.0, top_velocity=1e-3)
    sim, ctx = _mixed_pair(pk, 0.05, 7, mu=0.5, n_domains=16, repartition_every=2,
                           fixed_iters=40)
    for s in range(2):
        compare_step(sim, ctx, f"mixed 3D step{s}")


def test_all_parallel_is_the_jacobi_scheme():
    pk = inputs.lattice_2d(32, 32, 1000)
    sim, ctx = _mixed_pair(pk, 1.0, 8, mu=0.3, n_domains=4, fixed_iters=50)
    compare_step(sim, ctx, "p=1 Jacobi")


def test_mixed_update_is_refused_where_unsupported():
    from paper_1104_3516_amd import binding
    pk = inputs.lattice_2d(16, 16, 1000)
    _, ctx = both(pk, solve_mode=0, mu=0.3, n_domains=4)
    ctx.set_mixed_update(0.2, 1)
    with pytest.raises(binding.CDError):
        ctx.step()
    _, ctx = both(pk, mu=0.3, n_domains=4)
    ctx.set_adjoint(4)
    with pytest.raises(binding.CDError):
        ctx.set_mixed_update(0.2, 1)
