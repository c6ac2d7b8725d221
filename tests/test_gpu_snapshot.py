"""Checkpoint and resume: a context loaded from a snapshot of another one
steps bitwise as the other one does (the state a step depends on: positions,
velocities, walls, step counter, previous contact list and forces for the
warm start, bisection tree, Sec. 3.2)."""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs

pytestmark = pytest.mark.gpu


def _binding():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    from paper_1104_3516_amd import binding
    return binding


def _ctx(binding, pk, **kw):
    return binding.Context(binding.make_params(pk.dim, pk.n_walls, **kw), pk, timing=0)


def _state(ctx):
    x, v, w = (t.cpu().numpy() for t in ctx.state())
    c = {k: t.cpu().numpy() for k, t in ctx.contacts().items()}
    return dict(x=x, v=v, w=w, ci=c["ci"], cj=c["cj"], R=c["R"], dom=c["dom"],
                off=ctx.wall_offsets(), U=ctx.wall_velocities())


CASES = {
    # periodic in x, pressure walls sliding apart (walls of finite mass)
    "sheared_2d": (lambda: inputs.sheared_box_2d(24, 18, 91, pressure=0.25, shear_velocity=0.01),
                   dict(mu=0.4, n_domains=7, repartition_every=3, max_iter=3000)),
    # 3D, top wall driven down, staged sweeps with the foreign forces in LDS
    "spheres_3d": (lambda: inputs.lattice_3d(16, 16, 12, 92, gravity=0.0, top_velocity=1e-3),
                   dict(mu=0.5, n_domains=16, repartition_every=3)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_resumed_context_steps_bitwise(case):
    binding = _binding()
    make, kw = CASES[case]
    pk = make()
    a = _ctx(binding, pk, **kw)
    b = _ctx(binding, pk, **kw)
    for _ in range(3):
        a.step()
        b.step()
    snap = b.snapshot()
    b.close()
    c = _ctx(binding, pk, **kw)
    c.restore(snap)
    # the list's geometry comes with the next step
    with pytest.raises(binding.CDError) as err:
        c.contacts()
    assert err.value.code == binding.ENOTREADY
    # steps 3..6: a tree rebuild at 3 and 6, the tree descent at 4 and 5
    for s in range(4):
        ra, rc = a.step(), c.step()
        assert (ra.iterations, ra.n_contacts, ra.status) == (rc.iterations, rc.n_contacts,
                                                             rc.status), (case, s)
        sa, sc = _state(a), _state(c)
        for k in sa:
            assert np.array_equal(sa[k], sc[k]), (case, s, k)
    a.close()
    c.close()


def test_snapshot_refusals():
    binding = _binding()
    pk = inputs.lattice_2d(16, 16, 93)
    a = _ctx(binding, pk, mu=0.3, n_domains=4)
    a.step()
    snap = a.snapshot()
    # another domain count
    other = _ctx(binding, pk, mu=0.3, n_domains=8)
    with pytest.raises(binding.CDError):
        other.restore(snap)
    # not a snapshot, or cut short
    with pytest.raises(binding.CDError):
        a.restore(b"x" * len(snap))
    with pytest.raises(binding.CDError):
        a.restore(snap[:-8])
    # a split axis that is no coordinate (the root's, the first of the 2P-1
    # axes that precede the cuts at the end of the snapshot)
    nodes = 2 * 4 - 1
    bad = bytearray(snap)
    at = len(bad) - 12 * nodes
    bad[at:at + 4] = (7).to_bytes(4, "little", signed=True)
    with pytest.raises(binding.CDError) as err:
        a.restore(bytes(bad))
    assert err.value.code == binding.EINVAL
    # between the phases of a step
    a.prepare()
    with pytest.raises(binding.CDError):
        a.snapshot()
    a.close()
    other.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_shadow_mode_finds_the_step_deterministic(case):
    """Shadow mode runs every step twice from a snapshot and compares the
    runs bitwise; the results equal those of a context stepping once."""
    binding = _binding()
    make, kw = CASES[case]
    pk = make()
    a = _ctx(binding, pk, **kw)
    s = _ctx(binding, pk, **kw)
    s.set_shadow(1)
    for step in range(4):
        ra, rs = a.step(), s.step()
        assert (ra.iterations, ra.n_contacts, ra.status) == (rs.iterations, rs.n_contacts,
                                                             rs.status), (case, step)
        sa, ss = _state(a), _state(s)
        for k in sa:
            assert np.array_equal(sa[k], ss[k]), (case, step, k)
    a.close()
    s.close()


def test_shadow_mode_self_test_reports_a_difference():
    """mode 2 starts the second run with one velocity 1e-9 away from the
    snapshot's: the comparison must report it (the failure path, forced from
    the host)."""
    binding = _binding()
    pk = inputs.lattice_2d(16, 16, 94)
    s = _ctx(binding, pk, mu=0.3, n_domains=4)
    s.set_shadow(2)
    with pytest.raises(binding.CDError) as err:
        s.step()
    assert err.value.code == binding.ESHADOW
    s.close()


@pytest.mark.parametrize("P", [16, 64])
def test_workgroup_width_does_not_change_results_3d(P):
    """The same 3D steps with 64-, 128- and 256-thread domain workgroups
    (different passes over the staged data and the foreign incidences, and
    the shared LDS layout only from 128 threads on) are bitwise equal."""
    binding = _binding()
    pk = inputs.lattice_3d(16, 16, 12, 96, gravity=0.0, top_velocity=1e-3)
    ref = None
    for width in (64, 128, 256):
        ctx = binding.Context(binding.make_params(3, pk.n_walls, mu=0.5, n_domains=P,
                                                  repartition_every=2), pk, timing=0,
                              block_threads=width)
        states = []
        for _ in range(3):
            r = ctx.step()
            states.append((r.iterations, r.status, _state(ctx)))
        assert ctx.timing().block_threads == width
        ctx.close()
        if ref is None:
            ref = states
            continue
        for (ia, sa_, a), (ib, sb_, b) in zip(ref, states):
            assert (ia, sa_) == (ib, sb_), (P, width)
            for k in a:
                assert np.array_equal(a[k], b[k]), (P, width, k)
