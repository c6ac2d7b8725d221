"""Benchmark of the contact-force solve on one MI355X.

Headline workload (`--workload spheres_1m`, the default): 3D spheres,
N = 1,048,576 on a 128x128x64 jittered simple-cubic lattice (spacing 2.05,
radii U[0.8, 1.2], jitter +-0.05), mass ~ r^3, Coulomb cone mu = 0.5,
dt = 1e-3, no gravity, top wall driven down at 1e-3 (uniaxial compression),
initial velocities N(0, 0.01^2), hierarchical bisection balanced by contact
count into 16,384 domains, repartition every 10 steps, tolerance
alpha = 1e-6 on the local test (I), at most 2,000 sweeps per step.

With the headline the line also carries `other_workloads`: the 2D
workload of 262,144 disks (512x512 jittered triangular lattice, gravity 1,
mu = 0.3) timed at 2,048 domains, and the outcome of the same packing at
the 4,096 domains of its stated configuration, where the domain-wise update
diverges (the instability of Sec. 2.3; the CPU oracle diverges identically).
`--workload disks_262k`, `batch512` and `adjoint65k` time those workloads
on their own.  A "step" is one full time step: detection, warm start,
partition, order, the sweeps to convergence and the Euler update.

The JSON line reports whole-step contact updates/s (sum over steps of sweeps
x contacts, divided by the timed wall-clock), the milliseconds per step, the
roofline of the sweep kernel (algorithmic bytes per sweep over the summed
durations of the sweep launches that did work, from HIP events on the
library's stream) and the CPU oracle on a bounded sample.  For the 2D
workloads it also solves the final state once more from zero forces with the
workload's domains and with one domain (`sequential_comparison`: the extra
sweeps of Sec. 4.3 and the observables of Sec. 4.4; `--sequential 0` skips
it, outside the timed region either way).  Optional legs:
`--mixed-experiment` (the mixed sequential/parallel update of Sec. 2.3:
sweeps N_I(p) and the critical share p_c on a settled pile),
`--order-experiment` (sweeps in colour-major, random sequential and Jacobi
order on the chain of Fig. 13(a) and a pile, Sec. 4.3), `--random-order
SEED` (the timed steps in the random sequential order of Sec. 2.1, which
then no longer measure the headline configuration) and
`--balance SIGMA` (adaptive load balancing of Sec. 3.3 in the timed steps,
which then no longer measure the headline configuration).
"""
from __future__ import annotations

import argparse
import json
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contact updates/sec and ms per converged time step at tol 1e-6 (FP64), % HBM peak"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes a streaming sweep must move: per contact the pair
# indices, normal, gap, force read and force write; per particle the base
# velocities and the mass, inertia and radius terms (2D: 64 and 48 B; 3D:
# 88 and 72 B)
BYTES = {2: (64, 48), 3: (88, 72)}

# name -> (generator config, dim, mu, domains, default steps, traffic record, description)
WORKLOADS = {
    "disks_262k": dict(
        config="disks_262k", dim=2, mu=0.3, domains=2048, steps=100, cpu_sweeps=600,
        traffic="sweep_disks_262k_traffic.json", tune=(512, 1024, 2048, 4096), tune_use=True,
        text=("disks_262k: 2D disks N=262144 (512x512 jittered triangular lattice), mu=0.3, "
              "dt=1e-3, gravity 1, contact-count-balanced bisection domains, their count "
              "picked by the domain-count tuner among 512-4096 (the stated 4096 diverges; "
              "2048 without tuning), repartition every 10 steps, alpha=1e-6 local test, max "
              "2000 sweeps, gravity settling")),
    "spheres_1m": dict(
        config="spheres_1m", dim=3, mu=0.5, domains=16384, steps=50, cpu_sweeps=60,
        traffic="sweep_spheres_1m_traffic.json", tune=(4096, 8192, 16384, 32768),
        tune_use=False,
        text=("spheres_1m: 3D spheres N=1048576 (128x128x64 jittered simple-cubic lattice), "
              "mu=0.5, dt=1e-3, no gravity, top wall driven down at 1e-3, 16384 "
              "contact-count-balanced bisection domains, repartition every 10 steps, "
              "alpha=1e-6 local test, max 2000 sweeps")),
    "batch512": dict(
        config="batch512", dim=2, mu=None, domains=None, steps=20, cpu_sweeps=600,
        traffic="sweep_batch512_traffic.json",
        text=("batch512: 512 independent 2D disk packings (generator of the 1k case), N "
              "log-uniform in [256, 65536] (sum 5,580,310), mu uniform in [0.1, 0.6] per "
              "packing, autotuned contacts per domain, repartition every 10 steps, alpha=1e-6 "
              "local test, max 2000 sweeps, one sweep launch over all packings per sweep")),
    "adjoint65k": dict(
        config="disks_65k", dim=2, mu=None, domains=256, steps=5, cpu_sweeps=0,
        traffic="sweep_adjoint65k_traffic.json", sweeps=200, every=10, window=20,
        text=("adjoint65k: 2D disks N=65536 (256x256 jittered triangular lattice), friction per "
              "pair uniform in [0.2, 0.4] (hash of the pair), 256 domains, contact list of gap <= "
              "0.2 r_max built at the first step and kept, 20 time steps of exactly 200 sweeps, "
              "checkpoints every 10 sweeps; each timed pass is the 20 steps from the initial "
              "state followed by their adjoint (dL/dmu, dL/dv, dL/dw of the bottom-wall normal "
              "forces after the last step)")),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(path, n_domains=None):
    """HBM bytes per sweep launch from the committed counter measurement, or
    None when the sweep kernel's sources changed since it was taken or it
    was taken at another domain count."""
    import hashlib
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if n_domains is not None and rec.get("n_domains") not in (None, n_domains):
        return None
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_core.h", "cd_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1104_3516_amd", "csrc", f), "rb").read())
    return rec.get("bytes_per_launch") if rec.get("kernel_sources_sha256") == h.hexdigest() else None


def make_ctx(wl, pk, binding, timing=1, solve_mode=1, block=0, n_domains=None, max_iter=2000,
             alpha=1e-6):
    params = binding.make_params(wl["dim"], pk.n_walls, mu=wl["mu"], dt=1e-3, alpha=alpha,
                                 criterion=0, max_iter=max_iter,
                                 n_domains=wl["domains"] if n_domains is None else n_domains,
                                 repartition_every=10, warm_start=1)
    return binding.Context(params, pk, timing=timing, solve_mode=solve_mode, block_threads=block)


def boundary_fraction(n, c):
    """Fraction of contacts with a body that also has contacts in another
    domain (walls excluded): the share of the update that sees frozen
    foreign forces, the parallel fraction p of Sec. 2.3."""
    from paper_1104_3516_amd import tune
    return tune.boundary_fraction(c["ci"], c["cj"], c["dom"], n)


def tuned_domains(wl, pk, binding, candidates):
    """The domain-count tuner on this workload's parameters: candidates in
    increasing order until one diverges, the fastest converging one kept
    (three steps each on throwaway contexts, no cache)."""
    from paper_1104_3516_amd import tune
    mk = lambda P: binding.make_params(wl["dim"], pk.n_walls, mu=wl["mu"], dt=1e-3, alpha=1e-6,
                                       criterion=0, max_iter=2000, n_domains=P,
                                       repartition_every=10, warm_start=1)
    out = tune.tune_domains(pk, mk, binding, candidates=candidates, steps=3, use_cache=False,
                            log=log)
    keep = ("n_domains", "ms_per_step", "sweeps", "boundary_fraction", "diverged")
    return {"n_domains": out["n_domains"],
            "critical_boundary_fraction": out["critical_boundary_fraction"],
            "trials": [{k: t[k] for k in keep} for t in out["trials"]]}


def mixed_experiment(torch, binding, inputs, cap=3000, settle=50, seed=2023):
    """The mixed-update experiment of Sec. 2.3: a packing of 128 x 128 disks
    settled for `settle` steps, then one step solved from zero forces on that
    geometry with a single domain and a share p of the contacts (by pair
    number) updated in parallel; the sweeps to convergence N_I(p), and p_c,
    the smallest p that does not converge within `cap` sweeps."""
    wl = dict(WORKLOADS["disks_262k"], domains=64)
    pk = inputs.lattice_2d(128, 128, 1005)
    ctx = make_ctx(wl, pk, binding, timing=0)
    for s in range(settle):
        ctx.step()
    q = pk.copy()
    x, v, w = (t.cpu().numpy() for t in ctx.state())
    q.x, q.v, q.w = x, v, w
    q.wall_offset = ctx.wall_offsets()
    nc = ctx.num_contacts()
    ctx.close()
    rows = []
    for p in (0.0, 0.01, 0.02, 0.03, 0.04, 0.05, 0.07, 0.1, 0.2, 0.5, 1.0):
        c = make_ctx(wl, q, binding, timing=0, n_domains=1, max_iter=cap)
        c.set_mixed_update(p, seed)
        t0 = time.perf_counter()
        try:
            r = c.step()
            status, sweeps = int(r.status), int(r.iterations)
        except binding.CDError as err:
            status, sweeps = int(err.code), None
        torch.cuda.synchronize()
        rows.append({"p": p, "sweeps": sweeps, "status": status,
                     "converged": status == 0, "seconds": time.perf_counter() - t0})
        log(f"mixed update p={p:.2f}: {sweeps} sweeps, status {status}")
        c.close()
    failing = [row["p"] for row in rows if not row["converged"]]
    return {"packing": f"128x128 disks settled for {settle} steps, {nc} contacts, mu=0.3",
            "procedure": "one step from zero forces, one domain, alpha=1e-6, at most "
                         f"{cap} sweeps; parallel contacts by pair number (seed {seed})",
            "rows": rows, "p_c": min(failing) if failing else None}


def strict_tolerance(wl, pk, torch, binding, steps):
    """The same workload with alpha = 1e-12 instead of 1e-6: the tolerance
    is applied to squared ratios (reading C12), so 1e-6 asks for about 1e-3
    relative change per force and 1e-12 for about 1e-6; `steps` steps from
    the initial state, timed as a whole."""
    ctx = make_ctx(wl, pk, binding, timing=0, alpha=1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps, capped, updates = [], 0, 0
    for s in range(steps):
        r = ctx.step()
        sweeps.append(int(r.iterations))
        capped += int(r.status == binding.MAXITER)
        updates += r.iterations * r.n_contacts
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    log(f"alpha 1e-12: sweeps per step {sweeps}")
    return {"alpha": 1e-12, "steps": steps, "sweeps_per_step": sweeps,
            "steps_at_sweep_cap": capped, "ms_per_step": 1e3 * el / steps,
            "contact_updates_per_s": updates / el}


def confined_pc_experiment(torch, binding, inputs, nx=40, steps=3000, dt=1e-2, pressure=1.0,
                           cap=20000, seed=7):
    """The protocol of Sec. 2.3 on a confined packing: nx x nx disks without
    gravity compressed between two walls of finite mass pushed with
    `pressure` per unit width (periodic in x) for `steps` steps, then the
    walls held at their positions, the forces reset, and one step solved with
    one domain and a share p of the contacts updated in parallel; N_I(p), the
    closed-contact coordination Z of the compressed packing, and p_c, the
    smallest p that does not converge within `cap` sweeps."""
    import numpy as np
    pk = inputs.sheared_box_2d(nx, nx, 2023, pressure=pressure)
    prm = binding.make_params(2, pk.n_walls, mu=0.3, dt=dt, n_domains=1, max_iter=3000)
    ctx = binding.Context(prm, pk, timing=0)
    t0 = time.perf_counter()
    for s in range(steps):
        ctx.step()
    x, v, w = (t.cpu().numpy() for t in ctx.state())
    wo = ctx.wall_offsets()
    c = {k: t.cpu().numpy() for k, t in ctx.contacts().items()}
    z = 2.0 * float((c["R"][0] > 0).sum()) / pk.n
    vw = ctx.wall_velocities()
    ctx.close()
    log(f"confined packing: {steps} steps in {time.perf_counter() - t0:.1f} s, Z = {z:.2f}, "
        f"wall speeds {np.abs(vw).max():.2e}")
    q = pk.copy()
    q.x, q.v, q.w = x, v, w
    q.wall_offset = wo.copy()
    q.wall_inv_mass = None
    q.wall_force = None
    q.wall_velocity = np.zeros_like(q.wall_velocity)
    q.box_lo = np.array([pk.box_lo[0], wo[0]])
    q.box_hi = np.array([pk.box_hi[0], -wo[1]])
    rows = []
    for p in (0.0, 0.02, 0.05, 0.1, 0.2, 0.3, 0.5, 0.65, 1.0):
        prm = binding.make_params(2, q.n_walls, mu=0.3, dt=dt, n_domains=1, max_iter=cap,
                                  warm_start=0)
        cq = binding.Context(prm, q, timing=0)
        cq.set_mixed_update(p, seed)
        try:
            r = cq.step()
            status, sweeps = int(r.status), int(r.iterations)
        except binding.CDError as err:
            status, sweeps = int(err.code), None
        cq.close()
        rows.append({"p": p, "sweeps": sweeps, "status": status, "converged": status == 0})
        log(f"confined mixed update p={p:.2f}: {sweeps} sweeps, status {status}")
    failing = [row["p"] for row in rows if not row["converged"]]
    return {"packing": f"{nx}x{nx} disks, no gravity, periodic in x, compressed for {steps} "
                       f"steps (dt {dt}) between walls of finite mass under pressure {pressure}; "
                       f"Z of closed contacts {z:.2f}",
            "procedure": "walls then held, forces reset, one step with one domain, alpha=1e-6, "
                         f"at most {cap} sweeps; parallel contacts by pair number (seed {seed})",
            "rows": rows, "p_c": min(failing) if failing else None}


def order_experiment(torch, binding, inputs, seeds=8):
    """Sweeps of one cold-started time step in three update orders (Sec. 2.1,
    Sec. 4.3): colour-major, random sequential (mean over `seeds` draws) and
    parallel (Jacobi, the mixed update with p = 1).  On the compressed chain
    of Fig. 13(a) (128 disks) at 1 to 16 domains: N_I(Jacobi) / N_I(random)
    estimates D_s / D_p, and N_I(P) / N_I(1) of each order is set beside the
    diffusion model 1 / (1 - (P/n)(1 - D_p/D_s)) with the paper's 1.53.  On a
    64 x 64 disk pile (mu = 0.3): one domain and 16."""
    import numpy as np

    def sweeps(pk, P, order, seed=0, max_iter=200000):
        prm = binding.make_params(2, pk.n_walls, mu=0.3, n_domains=P, max_iter=max_iter)
        c = binding.Context(prm, pk, timing=0)
        if order == "random":
            c.set_random_order(True, seed)
        elif order == "jacobi":
            c.set_mixed_update(1.0, 0)
        r = c.step()
        c.close()
        return int(r.iterations), int(r.status)

    def mean_random(pk, P):
        runs = [sweeps(pk, P, "random", s) for s in range(seeds)]
        return float(np.mean([r[0] for r in runs])), max(r[1] for r in runs)

    n = 128
    chain = inputs.chain_2d(n, 1.0)
    rows = []
    for P in (1, 2, 4, 8, 16):
        cm, st_cm = sweeps(chain, P, "colour")
        rd, st_rd = mean_random(chain, P)
        rows.append({"domains": P, "colour_major": cm, "random_mean": rd,
                     "status": max(st_cm, st_rd),
                     "model_ratio": 1.0 / (1.0 - (P / n) * (1.0 - 1.0 / 1.53))})
        log(f"order experiment, chain P={P}: colour-major {cm}, random {rd:.1f}")
    for r in rows:
        r["colour_major_ratio"] = r["colour_major"] / rows[0]["colour_major"]
        r["random_ratio"] = r["random_mean"] / rows[0]["random_mean"]
    jac, st_j = sweeps(chain, 1, "jacobi")
    pile = inputs.lattice_2d(64, 64, 1000)
    pile_rows = []
    for P in (1, 16):
        cm, st_cm = sweeps(pile, P, "colour", max_iter=20000)
        # one domain: a single thread per sweep walks all 4,800 contacts
        runs = [sweeps(pile, P, "random", s, max_iter=20000) for s in range(2 if P == 1 else seeds)]
        rd, st_rd = float(np.mean([r[0] for r in runs])), max(r[1] for r in runs)
        pile_rows.append({"domains": P, "colour_major": cm, "random_mean": rd,
                          "status": max(st_cm, st_rd)})
        log(f"order experiment, 64x64 pile P={P}: colour-major {cm}, random {rd:.1f}")
    return {
        "chain": {"disks": n, "rows": rows, "jacobi_one_domain": jac, "jacobi_status": st_j,
                  "ds_over_dp_estimate": jac / rows[0]["random_mean"],
                  "ds_over_dp_paper": 1.53, "q_s_over_q_p_theory": 0.797 / 0.5},
        "pile_64x64": pile_rows,
        "procedure": "one step from zero forces, mu=0.3, alpha=1e-6; random order mean over "
                     f"{seeds} seeds (2 on the one-domain pile)",
    }


def sequential_comparison(wl, pk, ctx, torch, binding, max_iter):
    """One time step solved from scratch (cold start) on the state the timed
    steps ended in, with the workload's domains and with a single domain
    (the plain sequential solve): the extra sweeps of the domain-wise solve,
    N_I(P) / N_I(1) (Sec. 4.3), and the macroscopic observables of Sec. 4.4."""
    from paper_1104_3516_amd import analysis
    q = pk.copy()
    x, v, w = (t.cpu().numpy() for t in ctx.state())
    q.x, q.v, q.w = x, v, w
    q.wall_offset = ctx.wall_offsets()
    runs = {}
    for P in (wl["domains"], 1):
        log(f"sequential comparison: one cold-started step with {P} domain(s) ...")
        c = make_ctx(wl, q, binding, timing=0, n_domains=P, max_iter=max_iter)
        t0 = time.perf_counter()
        r = c.step()
        torch.cuda.synchronize()
        hc = analysis.host_contacts(c.contacts())
        runs[P] = dict(x=q.x, c=hc, it=r.iterations, status=r.status,
                       seconds=time.perf_counter() - t0, glob=c.timing().global_records)
        log(f"  {r.iterations} sweeps, status {r.status}, {runs[P]['seconds']:.1f} s")
        c.close()
    P = wl["domains"]
    d = analysis.compare(q, runs[1], runs[P])
    frac = boundary_fraction(q.n, runs[P]["c"])
    # Sec. 4.3: N_I ~ 1 / D with D = D_p p + D_s (1 - p), D_s / D_p = 1.53
    model = 1.0 / (1.0 - frac * (1.0 - 1.0 / 1.53))
    return {
        "state": "the positions and velocities after the timed steps, forces from zero",
        "n_domains": P, "sweeps": runs[P]["it"], "sweeps_one_domain": runs[1]["it"],
        "status": runs[P]["status"], "status_one_domain": runs[1]["status"],
        "extra_sweep_factor": runs[P]["it"] / max(runs[1]["it"], 1),
        "boundary_contact_fraction": frac,
        "model_extra_sweep_factor": model,
        "model": "1 / (1 - p (1 - D_p / D_s)), D_s / D_p = 1.53 fitted in Sec. 4.3, p the "
                 "boundary contact fraction",
        "mean_stress_rel_diff": d["mean_stress"], "sigma_yy_strips_rel_diff": d["strips"],
        "orientation_tv_distance": d["orientation_tv"],
        "max_force_rel_diff": d.get("forces"),
        "one_domain_seconds": runs[1]["seconds"],
        "one_domain_global_records": bool(runs[1]["glob"]),
    }


def batch_domains(pk, target):
    """Domains of a packing for about `target` contacts per domain."""
    from paper_1104_3516_amd.tune import domains_for
    return domains_for(pk.n, target)


def batch_params_p(binding, pk, mu, n_domains):
    return binding.make_params(2, pk.n_walls, mu=float(mu), dt=1e-3, alpha=1e-6, criterion=0,
                               max_iter=2000, n_domains=n_domains, repartition_every=10,
                               warm_start=1)


def batch_params(binding, pk, mu, target):
    return batch_params_p(binding, pk, mu, batch_domains(pk, target))


def run_batch(args, wl, torch, binding, inputs) -> dict:
    """The batched workload: value over the timed steps of the batch, and the
    same packings stepped one at a time (cd_step) on the same GPU for two
    steps as the plain comparison."""
    packs, mus = inputs.uneven_batch(512)
    tuning = None
    if args.target > 0:
        target = args.target
    else:
        from paper_1104_3516_amd import tune
        tuning = tune.tune_batch_target(
            packs, mus, lambda pk, mu, p: batch_params_p(binding, pk, mu, p), binding, log=log)
        target = tuning["target"]
        log(f"tuned contacts per domain: {target} (cached: {tuning['cached']})")
    if args.warmup > 0:
        ctxs = [binding.Context(batch_params(binding, pk, mu, target), pk, timing=0)
                for pk, mu in zip(packs, mus)]
        bt = binding.Batch(ctxs)
        for s in range(args.warmup):
            bt.step()
            log(f"warmup step {s}")
        bt.close()
        del bt, ctxs
    ctxs = [binding.Context(batch_params(binding, pk, mu, target), pk, timing=0)
            for pk, mu in zip(packs, mus)]
    bt = binding.Batch(ctxs, timing=args.time_every)
    torch.cuda.synchronize()
    updates = sweeps_max = 0
    kernel_ms = solve_ms = prepare_ms = finish_ms = 0.0
    bytes_all = 0.0
    executed = timed = 0
    n_maxiter = 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = bt.step()
        tm = bt.timing()
        for pk, r in zip(packs, res):
            updates += r.iterations * r.n_contacts
            n_maxiter += int(r.status == binding.MAXITER)
            bytes_all += r.iterations * (BYTES[2][0] * r.n_contacts + BYTES[2][1] * pk.n)
        sweeps_max += max(r.iterations for r in res)
        kernel_ms += tm.sweep_kernel_ms
        solve_ms += tm.solve_ms
        prepare_ms += tm.prepare_ms
        finish_ms += tm.finish_ms
        executed += tm.sweeps_executed
        timed += tm.sweeps_timed
        log(f"step {s}: sweep launches {tm.sweep_launches}, slowest packing "
            f"{max(r.iterations for r in res)} sweeps, prepare {tm.prepare_ms:.1f} ms, solve "
            f"{tm.solve_ms:.1f} ms, finish {tm.finish_ms:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    bt.close()
    # the plain comparison: every packing on its own, two steps
    plain_steps = 2
    ctxs_p = [binding.Context(batch_params(binding, pk, mu, target), pk, timing=0)
              for pk, mu in zip(packs, mus)]
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plain_updates = 0
    for s in range(plain_steps):
        for c in ctxs_p:
            r = c.step()
            plain_updates += r.iterations * r.n_contacts
    torch.cuda.synchronize()
    plain_elapsed = time.perf_counter() - tp
    achieved = bytes_all / (kernel_ms / 1e3) / 1e9 if kernel_ms > 0 else None
    return {
        "value": updates / elapsed, "elapsed": elapsed, "updates": updates,
        "sweeps_per_step": sweeps_max / args.steps, "steps_at_sweep_cap": n_maxiter,
        "solve_ms_per_step": solve_ms / args.steps, "prepare_ms_per_step": prepare_ms / args.steps,
        "finish_ms_per_step": finish_ms / args.steps,
        "sweep_kernel_us": 1e3 * kernel_ms / max(executed, 1),
        "sweeps_executed": executed, "sweeps_timed": timed,
        "contacts_per_domain_target": target,
        "tuning": tuning,
        "packings_failed": int(sum(1 for r in res if r.status < 0)),
        "plain": {"steps": plain_steps, "ms_per_step": 1e3 * plain_elapsed / plain_steps,
                  "contact_updates_per_s": plain_updates / plain_elapsed,
                  "note": "the same 512 packings stepped one at a time with cd_step"},
        "achieved": achieved, "bytes_per_sweep": bytes_all / max(executed, 1),
        "n_particles": int(sum(pk.n for pk in packs)),
    }


def cpu_baseline(wl, pk, sweeps: int) -> dict:
    """The oracle as it is, single-threaded, on the first time step of the
    same workload with the sweep count capped."""
    from oracle import cdref
    cdref.build(force=False)
    p = cdref.make_params(wl["dim"], pk.n_walls, mu=wl["mu"], dt=1e-3, alpha=1e-6, criterion=0,
                          max_iter=sweeps, n_domains=wl["domains"], repartition_every=10)
    sim = cdref.Sim(p, pk)
    t0 = time.perf_counter()
    info = sim.step()
    dt = time.perf_counter() - t0
    updates = info.iterations * info.n_contacts
    return {"value": updates / dt, "unit": "contact updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"first time step of the same workload (N={pk.n}, {wl['domains']} domains), "
                       f"sweeps capped at {sweeps} ({info.iterations} run, "
                       f"{info.n_contacts} contacts), whole step incl. detection and "
                       f"partition, {dt:.1f} s single-threaded")}


def cpu_parallel(wl, pk, sweeps: int) -> dict:
    """The same sample with the oracle's domains spread over the host's
    threads (OpenMP over the domains of each sweep: the paper's domain-wise
    scheme on shared memory); results are bit-identical to the serial run."""
    from oracle import cdref
    cdref.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    p = cdref.make_params(wl["dim"], pk.n_walls, mu=wl["mu"], dt=1e-3, alpha=1e-6, criterion=0,
                          max_iter=sweeps, n_domains=wl["domains"], repartition_every=10)
    cdref.set_threads(threads)
    try:
        sim = cdref.Sim(p, pk)
        t0 = time.perf_counter()
        info = sim.step()
        dt = time.perf_counter() - t0
    finally:
        cdref.set_threads(1)
    updates = info.iterations * info.n_contacts
    return {"value": updates / dt, "unit": "contact updates/s", "cores": threads,
            "kind": "oracle, domains over OpenMP threads",
            "sample": (f"first time step of the same workload, sweeps capped at {sweeps} "
                       f"({info.iterations} run), whole step, {dt:.1f} s on {threads} threads "
                       "(detection, partition and the exchange stay serial)")}


def run_adjoint(args, wl, torch, binding, inputs) -> dict:
    """Windows of wl["window"] time steps (200 sweeps each) on the kept
    contact list and the adjoint of each window, timed separately."""
    pk = inputs.config(wl["config"])
    skin = 0.2 * pk.r.max()
    T = wl["window"]
    ctx = binding.Context(binding.make_params(2, pk.n_walls, fixed_iters=wl["sweeps"],
                                              n_domains=wl["domains"], skin=skin), pk,
                          timing=args.time_every)
    ctx.set_adjoint(wl["every"])
    ctx.prepare()
    c = {k: v.cpu().numpy() for k, v in ctx.contacts().items()}
    mu = torch.as_tensor(inputs.pair_mu(1004, c["ci"], c["cj"]), device="cuda")
    nc = len(c["ci"])
    seed = torch.zeros((2, nc), dtype=torch.float64, device="cuda")
    seed[0] = torch.as_tensor(c["cj"] == pk.n + 2, device="cuda").double()
    ctx.set_frozen_list(True)
    acc = {"kernel_ms": 0.0, "executed": 0}

    def primal(count):
        ctx.reset()
        for t in range(T):
            ctx.prepare()
            if t == 0:
                ctx.set_contact_mu(mu)
            ctx.solve()
            if count:
                tm = ctx.timing()
                acc["kernel_ms"] += tm.sweep_kernel_ms
                acc["executed"] += tm.sweeps_executed

    for _ in range(max(args.warmup, 1)):
        primal(False)
        ctx.adjoint(seed)
    torch.cuda.synchronize()
    t_primal = t_adj = 0.0
    for _ in range(args.steps):
        t0 = time.perf_counter()
        primal(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.adjoint(seed)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_primal += t1 - t0
        t_adj += t2 - t1
    updates = args.steps * T * wl["sweeps"] * nc
    avg = (acc["kernel_ms"] / 1e3) / max(acc["executed"], 1)
    bps = BYTES[2][0] * nc + BYTES[2][1] * pk.n
    achieved = bps / avg / 1e9 if avg > 0 else None
    return {"value": updates / t_primal, "primal_ms": 1e3 * t_primal / args.steps,
            "adjoint_ms": 1e3 * t_adj / args.steps, "adjoint_over_primal": t_adj / t_primal,
            "n_contacts": nc, "n_particles": pk.n, "sweep_kernel_us": 1e6 * avg if avg > 0 else None,
            "achieved": achieved, "bytes_per_sweep": bps, "sweeps": wl["sweeps"], "window": T}


def cpu_baseline_batch(packs, mus, target, sweeps: int) -> dict:
    """The oracle, single-threaded, on the first step of the first packings of
    the batch (about 20 s of work), sweeps capped."""
    from oracle import cdref
    cdref.build(force=False)
    updates, spent, used = 0, 0.0, 0
    for pk, mu in zip(packs, mus):
        p = cdref.make_params(2, pk.n_walls, mu=float(mu), dt=1e-3, alpha=1e-6, criterion=0,
                              max_iter=sweeps, n_domains=batch_domains(pk, target),
                              repartition_every=10)
        sim = cdref.Sim(p, pk)
        t0 = time.perf_counter()
        info = sim.step()
        spent += time.perf_counter() - t0
        updates += info.iterations * info.n_contacts
        used += 1
        if spent > 20.0:
            break
    return {"value": updates / spent, "unit": "contact updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"first time step of the first {used} of the 512 packings, sweeps capped "
                       f"at {sweeps}, {spent:.1f} s single-threaded")}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="spheres_1m", choices=sorted(WORKLOADS),
                    help="spheres_1m (the headline: 3D, 1,048,576 spheres, 16,384 domains), "
                         "disks_262k, batch512 or adjoint65k")
    ap.add_argument("--extra", type=int, default=1,
                    help="with the headline workload also time disks_262k (2,048 domains) and "
                         "report the 4,096-domain configuration's divergence (0: skip)")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--steps", type=int, default=0, help="time steps (0: the workload's own)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sweeps", type=int, default=-1,
                    help="sweep cap of the CPU-oracle sample (0 skips it; default: about "
                         "20 s of oracle work for the workload)")
    ap.add_argument("--solve-mode", type=int, default=1,
                    help="1: one launch per sweep; 0: all sweeps of a step in one launch")
    ap.add_argument("--time-every", type=int, default=8,
                    help="time sweep launches in event-bracketed groups of this size (0: none)")
    ap.add_argument("--block", type=int, default=0,
                    help="threads per domain workgroup (0: chosen from the domain sizes)")
    ap.add_argument("--copy-mib", type=int, default=1024, metavar="MIB",
                    help="size of the copy whose bandwidth the line reports beside the "
                         "roofline (0 skips it)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), the reference "
                         "for scaling hardware byte counters, and exit")
    ap.add_argument("--target", type=int, default=0,
                    help="batch512: contacts per domain (0: the workload's default)")
    ap.add_argument("--balance", type=float, default=-1.0, metavar="SIGMA",
                    help="adaptive load balancing (Sec. 3.3) with this threshold on sigma_T "
                         "(negative: off, the headline configuration)")
    ap.add_argument("--random-order", type=int, default=-1, metavar="SEED",
                    help="timed steps in the random sequential order (Sec. 2.1) instead of "
                         "colour-major; the headline configuration is colour-major")
    ap.add_argument("--order-experiment", action="store_true",
                    help="sweeps in colour-major, random sequential and Jacobi order (Sec. 4.3)")
    ap.add_argument("--mixed-experiment", action="store_true",
                    help="also run the mixed-update experiment of Sec. 2.3 (N_I(p), p_c)")
    ap.add_argument("--sequential", type=int, default=1,
                    help="after the timed steps, solve one step from scratch with the "
                         "workload's domains and with one domain (2D workloads)")
    ap.add_argument("--sequential-max-iter", type=int, default=20000)
    ap.add_argument("--strict-steps", type=int, default=5,
                    help="steps of the workload at alpha = 1e-12 reported beside the line (0: none)")
    ap.add_argument("--domains", type=int, default=0,
                    help="domain count of the workload (0: its own, or the tuner's where it tunes)")
    ap.add_argument("--tune-domains", type=int, default=1,
                    help="run the domain-count tuner (disks_262k uses its choice; spheres_1m "
                         "keeps the stated 16384 and reports the tuner's trials)")
    ap.add_argument("--traffic-json", default=None,
                    help="counter record of the sweep kernel (default: the workload's)")
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    if args.steps <= 0:
        args.steps = wl["steps"]
    if args.cpu_sweeps < 0:
        args.cpu_sweeps = wl["cpu_sweeps"]
    if args.traffic_json is None:
        args.traffic_json = os.path.join(ROOT, "profiles", wl["traffic"])
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the solver "
              f"runs on one GPU (over several it would shard by subtrees of the bisection "
              f"tree, exchanging boundary forces after every sweep)", file=sys.stderr)
        return 2

    import torch

    from paper_1104_3516_amd import binding, inputs
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "repeats": 5}))
        return 0
    if args.workload == "adjoint65k":
        ra = run_adjoint(args, wl, torch, binding, inputs)
        traffic = measured_traffic(args.traffic_json)
        out = {
            "metric": METRIC, "value": ra["value"], "unit": "contact updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ra["primal_ms"] + ra["adjoint_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": wl["text"], "n_particles": ra["n_particles"],
                       "n_domains": wl["domains"], "passes": args.steps,
                       "time_steps_per_pass": ra["window"]},
            "primal_ms_per_pass": ra["primal_ms"], "adjoint_ms_per_pass": ra["adjoint_ms"],
            "primal_ms_per_time_step": ra["primal_ms"] / ra["window"],
            "adjoint_over_primal": ra["adjoint_over_primal"],
            "n_contacts": ra["n_contacts"], "sweeps_per_step": ra["sweeps"],
            "sweep_kernel_us": ra["sweep_kernel_us"],
            "roofline": {"bound": "hbm", "achieved": ra["achieved"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s",
                         "frac": ra["achieved"] / HBM_PEAK_GBS if ra["achieved"] else None,
                         "traffic": traffic, "kernel": "k_sweep<2>",
                         "bytes_per_sweep": ra["bytes_per_sweep"]},
        }
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "batch512":
        rb = run_batch(args, wl, torch, binding, inputs)
        traffic = measured_traffic(args.traffic_json)
        out = {
            "metric": METRIC, "value": rb["value"], "unit": "contact updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * rb["elapsed"] / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl["text"], "n_particles": rb["n_particles"],
                       "n_packings": 512, "time_steps": args.steps},
            "sweeps_per_step": rb["sweeps_per_step"],
            "steps_at_sweep_cap": rb["steps_at_sweep_cap"],
            "solve_ms_per_step": rb["solve_ms_per_step"],
            "prepare_ms_per_step": rb["prepare_ms_per_step"],
            "finish_ms_per_step": rb["finish_ms_per_step"],
            "sweep_kernel_us": rb["sweep_kernel_us"], "sweeps_executed": rb["sweeps_executed"],
            "sweeps_timed": rb["sweeps_timed"],
            "contacts_per_domain_target": rb["contacts_per_domain_target"],
            "domain_size_tuning": rb["tuning"],
            "packings_failed": rb["packings_failed"],
            "plain_comparison": rb["plain"],
            "roofline": {"bound": "hbm", "achieved": rb["achieved"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s",
                         "frac": rb["achieved"] / HBM_PEAK_GBS if rb["achieved"] else None,
                         "traffic": traffic, "kernel": "k_sweep_batch<2>",
                         "bytes_per_sweep": rb["bytes_per_sweep"]},
        }
        if args.cpu_sweeps > 0:
            log("cpu baseline (oracle) ...")
            packs, mus = inputs.uneven_batch(512)
            out["cpu_baseline"] = cpu_baseline_batch(packs, mus, rb["contacts_per_domain_target"],
                                                     args.cpu_sweeps)
        print(json.dumps(out), flush=True)
        return 0
    pk = inputs.config(wl["config"])
    tuning = None
    if args.domains > 0:
        wl = dict(wl, domains=args.domains)
    elif args.tune_domains and wl.get("tune"):
        log(f"domain-count tuning on {args.workload} ...")
        tuning = tuned_domains(wl, pk, binding, wl["tune"])
        tuning["used"] = bool(wl["tune_use"])
        if wl["tune_use"]:
            wl = dict(wl, domains=tuning["n_domains"])
    out = run_single(args, wl, pk, torch, binding, inputs, steps=args.steps,
                     warmup=args.warmup, time_every=args.time_every,
                     traffic_json=args.traffic_json, random_order=args.random_order,
                     balance=args.balance)
    if args.mixed_experiment:
        out["mixed_parallelness"] = mixed_experiment(torch, binding, inputs)
        out["mixed_parallelness_confined"] = confined_pc_experiment(torch, binding, inputs)
    if args.order_experiment:
        out["update_orders"] = order_experiment(torch, binding, inputs)
    if tuning is not None:
        out["domain_count_tuning"] = tuning
    if args.strict_steps > 0:
        log(f"{args.workload} at alpha 1e-12 ...")
        out["strict_tolerance"] = strict_tolerance(wl, pk, torch, binding, args.strict_steps)
    ctx = out.pop("_ctx")
    if args.sequential and wl["dim"] == 2:
        out["sequential_comparison"] = sequential_comparison(wl, pk, ctx, torch, binding,
                                                             args.sequential_max_iter)
    ctx.close()
    if args.workload == "spheres_1m" and args.extra:
        out["other_workloads"] = extra_workloads(args, torch, binding, inputs)
    if args.copy_mib > 0:
        out["copy_bandwidth"] = copy_bandwidth(torch, args.copy_mib)
    if args.cpu_sweeps > 0:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, pk, args.cpu_sweeps)
        out["cpu_parallel"] = cpu_parallel(wl, pk, args.cpu_sweeps)
    print(json.dumps(out), flush=True)
    return 0


def copy_bandwidth(torch, mib: int, reps: int = 10) -> dict:
    """What the HBM gives a plain streaming kernel on this GPU: a
    device-to-device copy of `mib` MiB, timed with events over `reps` copies
    after two untimed ones (bytes read plus bytes written over the time),
    beside the 8 TB/s peak the roofline fraction uses."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    sec = t0.elapsed_time(t1) / 1e3
    gbs = 2.0 * n * 8 * reps / sec / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"GB/s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes_per_copy": 2 * n * 8,
            "copies": reps, "note": "device-to-device copy (torch copy_), read + written bytes"}


def run_single(args, wl, pk, torch, binding, inputs, steps, warmup, time_every, traffic_json,
               random_order=-1, balance=-1.0, n_domains=None, quiet=False) -> dict:
    """Time `steps` whole time steps of one context after `warmup` steps on a
    throwaway context; returns the JSON fields of the line (the context of
    the timed steps under "_ctx", still open)."""
    dim = wl["dim"]
    P = wl["domains"] if n_domains is None else n_domains
    # warm-up on a throwaway context (kernels loaded, allocations made)
    if warmup > 0:
        ctx = make_ctx(wl, pk, binding, solve_mode=args.solve_mode, block=args.block,
                       n_domains=P)
        for s in range(warmup):
            r = ctx.step()
            log(f"warmup step {s}: {r.iterations} sweeps, {r.n_contacts} contacts")
        ctx.close()
        del ctx

    ctx = make_ctx(wl, pk, binding, timing=time_every, solve_mode=args.solve_mode,
                   block=args.block, n_domains=P)
    if balance >= 0.0:
        ctx.set_load_balance(balance)
    if random_order >= 0:
        ctx.set_random_order(True, random_order)
    sigmas = []
    torch.cuda.synchronize()
    sweeps = 0
    updates = 0
    sweep_kernel_ms = 0.0
    solve_ms = 0.0
    bytes_sweeps = 0.0
    maxiter_steps = 0
    executed = 0
    timed = 0
    step_ms, solve_ms_steps, phase_ms = [], [], []
    t0 = time.perf_counter()
    for s in range(steps):
        r = ctx.step()
        tm = ctx.timing()
        # device time of the step's stages (events on the library's stream)
        step_ms.append(tm.detect_ms + tm.partition_ms + tm.order_ms + tm.solve_ms + tm.update_ms)
        solve_ms_steps.append(tm.solve_ms)
        phase_ms.append((tm.detect_ms, tm.partition_ms, tm.order_ms, tm.solve_ms, tm.update_ms))
        sweeps += r.iterations
        updates += r.iterations * r.n_contacts
        sweep_kernel_ms += tm.sweep_kernel_ms
        solve_ms += tm.solve_ms
        executed += tm.sweeps_executed
        timed += tm.sweeps_timed
        bytes_sweeps += tm.sweeps_executed * (BYTES[dim][0] * r.n_contacts +
                                              BYTES[dim][1] * pk.n)
        maxiter_steps += int(r.status == binding.MAXITER)
        if balance >= 0.0:
            sigmas.append(ctx.domain_times()[1])
        if s % 10 == 0 or s == steps - 1:
            log(f"step {s}: {r.iterations} sweeps, {r.n_contacts} contacts, status {r.status}, "
                f"solve {tm.solve_ms:.2f} ms, sweep kernels {tm.sweep_kernel_ms:.2f} ms "
                f"({tm.sweep_launches} launches)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per executed sweep (the one-launch solve computes one sweep past the stop)
    avg_sweep_s = (sweep_kernel_ms / 1e3) / max(executed, 1)
    bytes_per_sweep = bytes_sweeps / max(executed, 1)
    # no per-sweep events (--time-every 0): no kernel duration, no roofline
    achieved = bytes_per_sweep / avg_sweep_s / 1e9 if sweeps and avg_sweep_s > 0 else None
    # the counters were taken on the colour-major sweep
    traffic = measured_traffic(traffic_json, P) if random_order < 0 else None
    out = {
        "metric": METRIC,
        "value": updates / elapsed,
        "unit": "contact updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["text"], "n_particles": pk.n, "n_domains": P,
                   "time_steps": steps},
        "sweeps_total": sweeps,
        "sweeps_per_step": sweeps / steps,
        "steps_at_sweep_cap": maxiter_steps,
        "solve_ms_per_step": solve_ms / steps,
        "median_step_ms": statistics.median(step_ms) if step_ms else None,
        "median_solve_ms": statistics.median(solve_ms_steps) if solve_ms_steps else None,
        # medians over the timed steps of each stage's device time (events)
        "median_phase_ms": ({name: statistics.median(p[k] for p in phase_ms) for k, name in
                             enumerate(("detect", "partition", "order", "solve", "update"))}
                            if phase_ms else None),
        "solve_contact_updates_per_s": updates / (solve_ms / 1e3) if solve_ms > 0 else None,
        "sweep_kernel_us": 1e6 * avg_sweep_s if avg_sweep_s > 0 else None,
        "contact_states_last_step": {"open": r.n_contacts - r.n_active,
                                     "stick": r.n_active - r.n_sliding,
                                     "slide": r.n_sliding},
        "sweeps_executed": executed,
        "sweeps_timed": timed,
        "solve_mode": args.solve_mode,
        "block_threads": tm.block_threads, "contact_data_in_lds": bool(tm.staged),
        "decision_in_workgroup0": tm.staged == 2,
        "foreign_forces_in_lds": bool(tm.foreign_in_lds),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
                     "traffic": traffic,
                     "kernel": (f"k_sweep<{dim}>, one launch per step" if args.solve_mode == 0
                                else f"k_sweep<{dim}, {'staged' if tm.staged else 'register'}"
                                f"{', random order' if random_order >= 0 else ''}>"),
                     "bytes_per_sweep": bytes_per_sweep},
        "_ctx": ctx,
    }
    if random_order >= 0:
        out["update_order"] = (f"random sequential (Sec. 2.1), seed {random_order}: one "
                               "thread per domain walks its contacts in a fresh draw each sweep")
    if balance >= 0.0:
        out["load_balance"] = {
            "threshold": balance,
            "sigma_t_first_step": sigmas[0] if sigmas else None,
            "sigma_t_last_step": sigmas[-1] if sigmas else None,
            "sigma_t_mean": sum(sigmas) / len(sigmas) if sigmas else None,
            "note": "per-domain sweep times measured in the timed steps; capacities n_i / T_i "
                    "place the cuts of every later rebuild (Sec. 3.3)"}
    return out


def extra_workloads(args, torch, binding, inputs) -> dict:
    """Beside the 3D headline: the 2D 262,144-disk workload at the domain
    count its tuner picks (timed like the headline, fewer steps); the
    tuner's trials include the 4,096 domains of its stated configuration,
    which diverge."""
    wl = WORKLOADS["disks_262k"]
    pk = inputs.config(wl["config"])
    res = {}
    tuning = None
    if args.tune_domains:
        log("extra workload: disks_262k domain-count tuning ...")
        tuning = tuned_domains(wl, pk, binding, wl["tune"])
        wl = dict(wl, domains=tuning["n_domains"])
    log(f"extra workload: disks_262k at {wl['domains']} domains ...")
    o = run_single(args, wl, pk, torch, binding, inputs, steps=args.extra_steps, warmup=2,
                   time_every=args.time_every,
                   traffic_json=os.path.join(ROOT, "profiles", wl["traffic"]))
    o.pop("_ctx").close()
    keep = ("value", "unit", "ms_per_step", "steps", "sweeps_per_step", "steps_at_sweep_cap",
            "sweep_kernel_us", "roofline", "config")
    res["disks_262k"] = {k: o[k] for k in keep}
    if tuning is not None:
        res["disks_262k"]["domain_count_tuning"] = tuning
    return res


if __name__ == "__main__":
    sys.exit(main())
