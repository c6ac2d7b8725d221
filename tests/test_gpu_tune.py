"""Autotuning: the workgroup width (library) and the batch domain size (tune.py)."""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_gpu_parity import _torch

pytestmark = pytest.mark.gpu


def test_width_tuning_keeps_results_and_caches_choice():
    """A context tuning its width (-1) steps like one at a fixed width, picks
    one of the candidates after four timed steps, and a later context of the
    same kind starts with the cached width."""
    from paper_1104_3516_amd import binding
    _torch()
    pk = inputs.lattice_2d(64, 64, 21)
    kw = dict(mu=0.3, n_domains=24, repartition_every=3)
    tuned = binding.Context(binding.make_params(2, pk.n_walls, **kw), pk, timing=1,
                            block_threads=-1)
    fixed = binding.Context(binding.make_params(2, pk.n_walls, **kw), pk, timing=1,
                            block_threads=128)
    widths = []
    for s in range(6):
        rt, rf = tuned.step(), fixed.step()
        widths.append(tuned.timing().block_threads)
        assert rt.n_contacts == rf.n_contacts
        ct = {k: v.cpu().numpy() for k, v in tuned.contacts().items()}
        cf = {k: v.cpu().numpy() for k, v in fixed.contacts().items()}
        np.testing.assert_array_equal(ct["ci"], cf["ci"])
        if rt.iterations == rf.iterations:
            np.testing.assert_array_equal(ct["R"], cf["R"])
    print("widths per step:", widths, flush=True)
    assert widths[:4] == [64, 128, 192, 256]
    assert widths[4] == widths[5] and widths[4] in (64, 128, 192, 256)
    again = binding.Context(binding.make_params(2, pk.n_walls, **kw), pk, timing=1,
                            block_threads=-1)
    again.step()
    assert again.timing().block_threads == widths[4]


def test_batch_domain_size_tuner_picks_a_stable_candidate():
    from paper_1104_3516_amd import binding, tune
    _torch()
    packs, mus = inputs.uneven_batch(4, seed=13, n_lo=256, n_hi=4096)
    mk = lambda pk, mu, p: binding.make_params(2, pk.n_walls, mu=float(mu), n_domains=p,
                                               repartition_every=10)
    out = tune.tune_batch_target(packs, mus, mk, binding, steps=1, candidates=(150, 600),
                                 use_cache=False)
    print(out, flush=True)
    assert out["target"] in (150, 600)
    assert len(out["trials"]) == 2
    best = [t for t in out["trials"] if t["target"] == out["target"]][0]
    assert not best["diverged"] or all(t["diverged"] for t in out["trials"])


def test_domain_count_tuner_stops_at_divergence_and_matches_oracle(tmp_path, monkeypatch):
    """Single context: candidates in increasing order until the first that
    diverges (a 64x64 lattice at 512 domains, eight particles each), its
    boundary share recorded as the critical share, the fastest converging
    candidate kept; the tuned decomposition steps exactly as the oracle at
    the same domain count; a later tuning of the same kind is cached."""
    from oracle import cdref
    from paper_1104_3516_amd import binding, tune
    from tests.test_gpu_parity import compare_step
    _torch()
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    pk = inputs.lattice_2d(64, 64, 7)
    kw = dict(mu=0.3, repartition_every=10)
    mk = lambda P: binding.make_params(2, pk.n_walls, n_domains=P, **kw)
    out = tune.tune_domains(pk, mk, binding, candidates=(64, 128, 256, 512), steps=3)
    print({k: v for k, v in out.items() if k != "trials"}, flush=True)
    trials = out["trials"]
    for t in trials:
        print(t, flush=True)
    assert [t["n_domains"] for t in trials] == [64, 128, 256, 512]
    assert trials[-1]["diverged"] and not any(t["diverged"] for t in trials[:-1])
    fbs = [t["boundary_fraction"] for t in trials]
    assert fbs == sorted(fbs)
    assert out["critical_boundary_fraction"] == fbs[-1]
    P = out["n_domains"]
    assert P in (64, 128, 256)
    assert P == min(trials[:-1], key=lambda t: t["ms_per_step"])["n_domains"]
    # the tuned decomposition against the oracle at the same domain count
    sim = cdref.Sim(cdref.make_params(2, pk.n_walls, n_domains=P, **kw), pk)
    ctx = binding.Context(mk(P), pk)
    for s in range(3):
        compare_step(sim, ctx, f"tuned P={P} step {s}")
    again = tune.tune_domains(pk, mk, binding, candidates=(64, 128, 256, 512), steps=3)
    assert again["cached"] and again["n_domains"] == P
    # another packing of the same dimension: the cached critical share stops
    # the candidates at or above it after their first step
    pk2 = inputs.lattice_2d(90, 90, 8)
    mk2 = lambda P: binding.make_params(2, pk2.n_walls, n_domains=P, **kw)
    out2 = tune.tune_domains(pk2, mk2, binding, candidates=(128, 1024, 4096), steps=2)
    print(out2, flush=True)
    last = out2["trials"][-1]
    assert last["rejected"] or last["diverged"] or last["n_domains"] == 4096
    for t in out2["trials"]:
        if t["rejected"]:
            assert t["boundary_fraction"] >= out["critical_boundary_fraction"]
            assert len(t["sweeps"]) == 1
