"""Batches of independent packings (cd_batch_*): every packing's results
must equal the oracle's run of that packing alone with the same partition
and order, and the HIP path's own single-packing run bit for bit."""
import math

import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import _torch, compare_results

pytestmark = pytest.mark.gpu


def domains_for(pk, target=150):
    """Domain count of a packing for about `target` contacts per domain
    (about 1.15 contacts per particle in these packings)."""
    return max(1, int(round(1.15 * pk.n / target)))


def make_set(packs, mus, over=None):
    from oracle import cdref
    from paper_1104_3516_amd import binding
    _torch()
    sims, ctxs = [], []
    for b, (pk, mu) in enumerate(zip(packs, mus)):
        kw = dict(mu=float(mu), n_domains=domains_for(pk), repartition_every=2)
        kw.update((over or {}).get(b, {}))
        sims.append(cdref.Sim(cdref.make_params(pk.dim, pk.n_walls, **kw), pk))
        ctxs.append(binding.Context(binding.make_params(pk.dim, pk.n_walls, **kw), pk))
    return sims, ctxs


def spread(pk):
    """The packing pulled apart so that it has no contacts."""
    pk.x = pk.x * 3.0
    pk.box_lo = pk.box_lo * 3.0 - 5.0
    pk.box_hi = pk.box_hi * 3.0 + 5.0
    pk.wall_offset = np.array([pk.box_lo[0], -pk.box_hi[0], pk.box_lo[1], -pk.box_hi[1]])
    return pk


def test_batch_matches_oracle_per_packing():
    """Six uneven packings (N log-uniform in [64, 4096], mu uniform in
    [0.1, 0.6]), domain counts by contact count, three steps; one packing
    runs a fixed sweep count, one hits a small sweep cap, one is a single
    domain."""
    from paper_1104_3516_amd import binding
    packs, mus = inputs.uneven_batch(6, seed=5, n_lo=64, n_hi=4096)
    over = {1: dict(fixed_iters=17), 2: dict(max_iter=6), 3: dict(n_domains=1)}
    sims, ctxs = make_set(packs, mus, over)
    batch = binding.Batch(ctxs)
    for s in range(3):
        res = batch.step()
        tm = batch.timing()
        print(f"[batch step {s}] launches={tm.sweep_launches} executed={tm.sweeps_executed} "
              f"workgroups={tm.workgroups}", flush=True)
        for b in range(len(packs)):
            io = sims[b].step()
            compare_results(sims[b], ctxs[b], io, res[b], f"batch s{s} p{b} N={packs[b].n}")
    assert res[1].iterations == 17
    assert res[2].status == binding.MAXITER and res[2].iterations == 6
    batch.close()


def test_batch_equals_single_runs_bitwise():
    """The batch against each packing stepped alone on the GPU: identical
    contact lists, forces, iteration counts and states, including a packing
    without contacts."""
    from paper_1104_3516_amd import binding
    packs, mus = inputs.uneven_batch(5, seed=9, n_lo=128, n_hi=8192)
    packs[3] = spread(packs[3])
    _, ctx_b = make_set(packs, mus)
    _, ctx_s = make_set(packs, mus)
    batch = binding.Batch(ctx_b)
    for s in range(2):
        res = batch.step()
        for b in range(len(packs)):
            r1 = ctx_s[b].step()
            assert res[b].iterations == r1.iterations and res[b].status == r1.status
            assert res[b].n_contacts == r1.n_contacts
            cb = {k: v.cpu().numpy() for k, v in ctx_b[b].contacts().items()}
            cs = {k: v.cpu().numpy() for k, v in ctx_s[b].contacts().items()}
            for k in ("ci", "cj", "dom", "color", "slot"):
                np.testing.assert_array_equal(cb[k], cs[k])
            np.testing.assert_array_equal(cb["R"], cs["R"])
            for tb, ts in zip(ctx_b[b].state(), ctx_s[b].state()):
                np.testing.assert_array_equal(tb.cpu().numpy(), ts.cpu().numpy())
    assert res[3].n_contacts == 0 and res[3].iterations == 0
    batch.close()


def test_batch_rejects_mixed_dimensions():
    from paper_1104_3516_amd import binding
    _torch()
    p2 = inputs.lattice_2d(6, 6, 1)
    p3 = inputs.lattice_3d(4, 4, 4, 2)
    c2 = binding.Context(binding.make_params(2, p2.n_walls), p2)
    c3 = binding.Context(binding.make_params(3, p3.n_walls), p3)
    with pytest.raises(binding.CDError):
        binding.Batch([c2, c3])


def test_full_size_batch512_one_step():
    """The 512-packing workload (N log-uniform in [256, 65536], 5.58M disks,
    mu uniform in [0.1, 0.6]) at about 300 contacts per domain, one step:
    the batch against every packing stepped alone on the GPU, bit for bit;
    and eight packings, the largest among them, against the oracle."""
    import os
    from oracle import cdref
    from paper_1104_3516_amd import binding
    _torch()
    cdref.set_threads(max(1, min(16, os.cpu_count() or 1)))
    packs, mus = inputs.uneven_batch(512)
    kw = lambda pk, mu: dict(mu=float(mu), alpha=1e-6, criterion=0, max_iter=2000,
                             n_domains=domains_for(pk, 300), repartition_every=10, warm_start=1)
    ctx_b = [binding.Context(binding.make_params(2, pk.n_walls, **kw(pk, mu)), pk, timing=0)
             for pk, mu in zip(packs, mus)]
    batch = binding.Batch(ctx_b, timing=0)
    res = batch.step()
    sizes = np.array([pk.n for pk in packs])
    print(f"[batch512] N total {sizes.sum()}, contacts {sum(r.n_contacts for r in res)}, "
          f"largest N {sizes.max()}, sweeps max {max(r.iterations for r in res)}, "
          f"at the cap {sum(r.status == binding.MAXITER for r in res)}", flush=True)
    for b, (pk, mu) in enumerate(zip(packs, mus)):
        single = binding.Context(binding.make_params(2, pk.n_walls, **kw(pk, mu)), pk, timing=0)
        r1 = single.step()
        assert res[b].iterations == r1.iterations and res[b].status == r1.status, b
        assert res[b].n_contacts == r1.n_contacts, b
        cb = {k: v.cpu().numpy() for k, v in ctx_b[b].contacts().items()}
        cs = {k: v.cpu().numpy() for k, v in single.contacts().items()}
        for k in ("ci", "cj", "dom", "color", "slot", "R"):
            np.testing.assert_array_equal(cb[k], cs[k], err_msg=f"packing {b} {k}")
        for tb, ts in zip(ctx_b[b].state(), single.state()):
            np.testing.assert_array_equal(tb.cpu().numpy(), ts.cpu().numpy())
        single.close()
    order = np.argsort(sizes)
    pick = sorted(set([int(order[-1])] + [int(order[q]) for q in np.linspace(0, 510, 7).astype(int)]))
    for b in pick:
        pk, mu = packs[b], mus[b]
        sim = cdref.Sim(cdref.make_params(2, pk.n_walls, **kw(pk, mu)), pk)
        io = sim.step()
        compare_results(sim, ctx_b[b], io, res[b], f"batch512 p{b} N={pk.n}")
    batch.close()
