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
