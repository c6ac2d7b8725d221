"""Autotuning of the batched solve's domain size.

A batch of packings is split into domains of about `target` contacts each
(the domain count of a packing is round(1.15 N / target), at least 1).  The
domain size sets how much of each packing is swept in parallel: small
domains fill the GPU but put more contacts on domain borders, where the
mixed parallel/sequential update needs more sweeps and can diverge
(Sec. 2.3); large domains lengthen each workgroup's sequential chain.  The
tuner runs a few time steps of the batch for every candidate target on
throwaway contexts, rejects targets under which any packing diverges,
and keeps the one with the shortest time per step.  The choice is cached
per (dimension, packing-count bucket, total-N bucket, device name) in a JSON
file, so a later run of the same kind skips the trials.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

CANDIDATES = (150, 300, 600, 1200)


def domains_for(n: int, target: int) -> int:
    """Domains of a packing of n particles for about `target` contacts each
    (about 1.15 contacts per particle in these packings)."""
    return max(1, int(round(1.15 * n / target)))


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1104_3516_amd", "tune.json")


def _key(dim: int, count: int, total_n: int, device: str) -> str:
    return f"dim{dim}-b{int(math.log2(max(count, 1)))}-n{int(math.log2(max(total_n, 1)))}-{device}"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune_batch_target(packs: Sequence, mus: Sequence[float], make_params, binding,
                      steps: int = 3, candidates: Sequence[int] = CANDIDATES,
                      use_cache: bool = True, log=None) -> Dict:
    """Pick the contacts-per-domain target for a batch.

    make_params(pk, mu, n_domains) -> binding.Params for one packing.
    Returns {"target": t, "trials": [...], "cached": bool}; every trial holds
    the target, the ms per step over `steps` steps (the first included), the
    packings that diverged and the sweeps of the slowest packing."""
    import torch
    device = torch.cuda.get_device_name(0).replace(" ", "_")
    total_n = int(sum(pk.n for pk in packs))
    key = _key(packs[0].dim, len(packs), total_n, device)
    path = _cache_path()
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            return dict(hit, cached=True)
    trials: List[Dict] = []
    for t in candidates:
        ctxs = [binding.Context(make_params(pk, mu, domains_for(pk.n, t)), pk, timing=0)
                for pk, mu in zip(packs, mus)]
        bt = binding.Batch(ctxs, timing=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        failed = set()
        slow = 0
        for _ in range(steps):
            res = bt.step()
            for b, r in enumerate(res):
                if r.status < 0:
                    failed.add(b)
            slow = max(slow, max(r.iterations for r in res))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        bt.close()
        del bt, ctxs
        trial = {"target": t, "ms_per_step": ms, "diverged": sorted(failed), "slowest_sweeps": slow}
        trials.append(trial)
        if log:
            log(f"tune: {trial}")
    ok = [x for x in trials if not x["diverged"]]
    pool = ok if ok else trials
    best = min(pool, key=lambda x: (len(x["diverged"]), x["ms_per_step"]))
    out = {"target": best["target"], "trials": trials, "key": key}
    if use_cache:
        data = _load(path)
        data[key] = out
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(data, f, indent=1)
        except OSError:
            pass
    return dict(out, cached=False)
