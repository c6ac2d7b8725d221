"""The benchmark boundary conditions on the GPU (Sec. 4.1, Fig. 10; Sec. 4.4):
periodic x, confining walls of finite mass under a constant force (pressure),
walls sliding in opposite directions (shear), against the oracle's steps on
the same inputs: lists, forces, positions, velocities and walls bit for bit
(the tests allow 1e-10 relative), sweep counts equal."""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import _torch

pytestmark = pytest.mark.gpu


def run_both(oracle, pk, steps, **kw):
    from paper_1104_3516_amd import binding
    _torch()
    ctx = binding.Context(binding.make_params(pk.dim, pk.n_walls, **kw), pk, timing=0)
    sim = oracle.Sim(oracle.make_params(pk.dim, pk.n_walls, **kw), pk)
    for s in range(steps):
        rg = ctx.step()
        ro = sim.step()
        assert (rg.n_contacts, rg.iterations, rg.status) == (ro.n_contacts, ro.iterations,
                                                             ro.status), (s, rg, ro)
        cg = {k: v.cpu().numpy() for k, v in ctx.contacts().items()}
        co = sim.contacts()
        for k in ("ci", "cj", "dom", "slot"):
            np.testing.assert_array_equal(cg[k], co[k], err_msg=f"step {s} {k}")
        scale = max(np.abs(co["R"]).max(), 1e-300)
        assert np.abs(cg["R"] - co["R"]).max() <= 1e-10 * scale, s
        xg, vg, wg = (t.cpu().numpy() for t in ctx.state())
        xo, vo, wo, offo = sim.state()
        np.testing.assert_allclose(xg, xo, rtol=0, atol=1e-10 * np.abs(xo).max())
        np.testing.assert_allclose(vg, vo, rtol=0, atol=1e-10 * max(np.abs(vo).max(), 1e-300))
        np.testing.assert_allclose(ctx.wall_offsets(), offo, rtol=0, atol=1e-12)
        np.testing.assert_allclose(ctx.wall_velocities(), sim.wall_velocities(), rtol=0,
                                   atol=1e-14)
    return ctx, sim


@pytest.mark.parametrize("P", [1, 7, 24])
def test_sheared_periodic_box_under_pressure(oracle, P):
    pk = inputs.sheared_box_2d(24, 18, 81, pressure=0.25, shear_velocity=0.01)
    ctx, sim = run_both(oracle, pk, 4, mu=0.4, n_domains=P, repartition_every=2,
                        max_iter=3000)
    # the walls moved and some contact crosses the periodic boundary
    U = ctx.wall_velocities()
    assert U[1, 1] != 0.0 and U[0, 0] == -0.01 and U[1, 0] == 0.01
    c = sim.contacts()
    x = sim.state()[0]
    pp = c["cj"] < pk.n
    L = pk.box_hi[0] - pk.box_lo[0]
    assert np.any(np.abs(x[0, c["ci"][pp]] - x[0, c["cj"][pp]]) > L / 2)


def test_periodic_box_with_fixed_walls_under_gravity(oracle):
    pk = inputs.sheared_box_2d(30, 12, 82)
    pk.wall_inv_mass = None
    pk.wall_force = None
    pk.f[1] = -pk.m                      # gravity 1, walls at rest
    run_both(oracle, pk, 3, mu=0.3, n_domains=9, repartition_every=2, max_iter=3000)


def test_fixed_sweeps_and_global_test_with_pressure_walls(oracle):
    pk = inputs.sheared_box_2d(20, 14, 83, pressure=1.0, shear_velocity=0.0)
    run_both(oracle, pk, 3, mu=0.2, n_domains=5, fixed_iters=40)
    run_both(oracle, pk, 2, mu=0.2, n_domains=5, criterion=1, max_iter=3000)


def test_3d_box_with_a_pressure_lid(oracle):
    """3D: a lattice periodic in x and y under a top wall of finite mass
    pushed down (the compression of the 3D workload driven by a force)."""
    pk = inputs.lattice_3d(8, 8, 6, 84)
    # periodic x and y: drop those walls, wrap the box to the lattice period
    keep = [4, 5]
    pk.wall_normal = pk.wall_normal[keep].copy()
    pk.wall_offset = pk.wall_offset[keep].copy()
    pk.wall_velocity = pk.wall_velocity[keep].copy()
    pk.box_lo = np.array([-1.025, -1.025, pk.box_lo[2]])
    pk.box_hi = np.array([-1.025 + 8 * 2.05, -1.025 + 8 * 2.05, pk.box_hi[2]])
    pk.periodic = 3
    pk.wall_inv_mass = np.array([0.0, 1.0 / 50.0])
    pk.wall_force = np.array([0.0, 20.0])
    run_both(oracle, pk, 3, mu=0.5, n_domains=6, repartition_every=2, max_iter=3000)


def test_mid_size_sheared_box(oracle):
    """16,384 disks (128 x 128), 64 domains, 3 steps (at 256 domains of 64 disks the
    domain-wise update of this packing diverges, in the oracle as well)."""
    pk = inputs.sheared_box_2d(128, 128, 85, pressure=0.25, shear_velocity=0.005)
    run_both(oracle, pk, 3, mu=0.5, n_domains=64, repartition_every=2, max_iter=2000)


def test_boundary_refusals():
    from paper_1104_3516_amd import binding
    _torch()
    pk = inputs.sheared_box_2d(16, 10, 86)
    ctx = binding.Context(binding.make_params(2, pk.n_walls, n_domains=2), pk, timing=0)
    with pytest.raises(binding.CDError):
        ctx.set_mixed_update(0.1, 0)
    with pytest.raises(binding.CDError):
        ctx.set_random_order(True, 0)
    with pytest.raises(binding.CDError):
        ctx.set_adjoint(5)
    with pytest.raises(binding.CDError):
        binding.Batch([ctx])
    # a wall on a periodic axis
    bad = inputs.lattice_2d(10, 8, 87)
    bad.periodic = 1
    with pytest.raises(binding.CDError):
        binding.Context(binding.make_params(2, bad.n_walls), bad, timing=0)
    # a periodic axis of fewer than three cells
    thin = inputs.sheared_box_2d(2, 6, 88)
    c2 = binding.Context(binding.make_params(2, thin.n_walls), thin, timing=0)
    with pytest.raises(binding.CDError):
        c2.step()
    # wall masses and forces need one value per wall
    short = inputs.sheared_box_2d(16, 10, 89)
    short.wall_inv_mass = short.wall_inv_mass[:1]
    with pytest.raises(ValueError):
        binding.Context(binding.make_params(2, short.n_walls), short, timing=0)
