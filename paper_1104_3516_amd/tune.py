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


# ---------------------------------------------------------------------------
# Domain count of one context
#
# A context's domain count sets the same trade-off for a single packing.  The
# boundary share f_b of a decomposition (contacts with a body that also has
# contacts in another domain: their neighbours' forces reach them only
# through the exchange, as the parallel contacts of Sec. 2.3 see the others
# only at the next exchange) grows with the domain count, and past a
# critical share the domain-wise solve stops converging (the domain
# analogue of the paper's p_c).  The tuner tries domain counts in increasing
# order on throwaway contexts, stops at the first one whose solve diverges
# and records that decomposition's boundary share as the measured critical
# share: a later tuning of the same kind (cached) rejects any candidate at or
# above it after its first step.  Among the candidates that converged it
# keeps the one with the shortest time per warm-started step.

def boundary_fraction(ci, cj, dom, n: int) -> float:
    """Share of the contacts with a particle that also has contacts in
    another domain (walls, cj >= n, belong to no domain)."""
    import numpy as np
    ci = np.asarray(ci, dtype=np.int64)
    cj = np.asarray(cj, dtype=np.int64)
    dom = np.asarray(dom, dtype=np.int64)
    if ci.size == 0:
        return 0.0
    P = int(dom.max()) + 1
    body = np.concatenate([ci, cj[cj < n]])
    bdom = np.concatenate([dom, dom[cj < n]])
    pairs = np.unique(body * P + bdom)
    multi = np.bincount(pairs // P, minlength=n) > 1
    touch = multi[ci] | np.where(cj < n, multi[np.minimum(cj, n - 1)], False)
    return float(touch.mean())


def domain_candidates(n: int, lo: int = 12, hi: int = 1024):
    """Powers of two P with n / P particles per domain in [lo, hi]."""
    out = []
    p = 1
    while n / p >= lo:
        if n / p <= hi:
            out.append(p)
        p *= 2
    return out


def _diverged(res) -> bool:
    """A step diverged: non-finite forces (an error status), or the sweep
    cap reached with the mean force of the last sweep still changing by more
    than 1e-5 (test (II)'s measure; slow but converging solves stopped by the
    cap were measured below 1e-6, diverging ones above 5e-4)."""
    if res.status < 0:
        return True
    return res.status != 0 and res.rel_change_last > 1e-5


def tune_domains(pk, make_params, binding, candidates: Optional[Sequence[int]] = None,
                 steps: int = 3, use_cache: bool = True, log=None) -> Dict:
    """Pick the domain count of one packing.

    make_params(P) -> binding.Params.  Each candidate runs `steps` steps from
    the packing's initial state on a throwaway context; it is ranked by the
    mean time of its steps after the first.  Returns {"n_domains": P,
    "trials": [...], "critical_boundary_fraction": f or None, "cached": bool};
    a trial holds P, that mean, each step's time, status and sweeps, the
    boundary share of its first step's decomposition, and whether it
    diverged or was rejected by the critical share after its first step."""
    import torch
    device = torch.cuda.get_device_name(0).replace(" ", "_")
    key = f"domains-dim{pk.dim}-n{int(math.log2(max(pk.n, 1)))}-{device}"
    path = _cache_path()
    data = _load(path) if use_cache else {}
    if use_cache and key in data and "n_domains" in data[key]:
        return dict(data[key], cached=True)
    f_crit = data.get(f"fcrit-dim{pk.dim}") if use_cache else None
    cands = sorted(candidates) if candidates else domain_candidates(pk.n)
    trials: List[Dict] = []
    for P in cands:
        ctx = binding.Context(make_params(P), pk, timing=0)
        sweeps, status, change, times, div, fb = [], [], [], [], False, None
        try:
            for s in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.step()
                torch.cuda.synchronize()
                times.append(1e3 * (time.perf_counter() - t0))
                sweeps.append(res.iterations)
                status.append(res.status)
                change.append(res.rel_change_last)
                if s == 0:
                    c = ctx.contacts()
                    fb = boundary_fraction(c["ci"].cpu().numpy(), c["cj"].cpu().numpy(),
                                           c["dom"].cpu().numpy(), pk.n)
                    if f_crit is not None and fb >= f_crit:
                        break
                if _diverged(res):
                    div = True
                    break
        except binding.CDError:
            div = True
        # the first step starts from the packing's initial forces and is
        # timed but not ranked when later ones exist (it is no guide to the
        # warm-started steps that follow)
        ranked = times[1:] if len(times) > 1 else times
        ms = sum(ranked) / len(ranked) if ranked else float("inf")
        ctx.close()
        rejected = f_crit is not None and fb is not None and fb >= f_crit and not div
        trial = {"n_domains": P, "ms_per_step": ms, "ms_steps": times, "sweeps": sweeps,
                 "status": status,
                 "rel_change_last": change, "boundary_fraction": fb, "diverged": div,
                 "rejected": rejected}
        trials.append(trial)
        if log:
            log(f"tune domains: {trial}")
        if div and fb is not None:
            f_crit = fb if f_crit is None else min(f_crit, fb)
        if div or rejected:
            break
    ok = [t for t in trials if not t["diverged"] and not t["rejected"]]
    best = min(ok, key=lambda t: t["ms_per_step"]) if ok else trials[0]
    out = {"n_domains": best["n_domains"], "trials": trials,
           "critical_boundary_fraction": f_crit, "key": key}
    if use_cache:
        data = _load(path)
        data[key] = out
        if f_crit is not None:
            data[f"fcrit-dim{pk.dim}"] = f_crit
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(data, f, indent=1)
        except OSError:
            pass
    return dict(out, cached=False)
