"""Pins of the oracle's mixed sequential/parallel update (Sec. 2.3) on the CPU.

A contact updated in parallel takes its new force from the velocities of
the sweep's start (all other forces at their previous values) and its
change reaches the other contacts only through the next exchange.  That is
exactly what the domain-wise solve does to a contact alone in its own
domain, a semantics pinned elsewhere; so the mixed solve of one domain with
flagged contacts F must equal, bit for bit, the domain-wise solve in which
every contact of F is a domain of its own and the rest one domain.
"""
import numpy as np
import pytest

from paper_1104_3516_amd import inputs


def _geometry(oracle, pk):
    ci, cj = oracle.detect(pk, 0.0, use_cells=True)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    return ci, cj, normal, gap


def _mixed(oracle, pk, ci, cj, normal, gap, flags, **kw):
    params = oracle.make_params(pk.dim, pk.n_walls, n_domains=1, **kw)
    dom = np.zeros(len(ci), np.int32)
    color, slot, ds = oracle.order(pk.n, ci, cj, 1, dom, parallel=flags)
    R, info, _ = oracle.solve(params, pk, ci, cj, normal, gap, 1, ds, slot, parallel=flags)
    return R, info, color, slot


def _own_domains(oracle, pk, ci, cj, normal, gap, flags, **kw):
    dom = np.zeros(len(ci), np.int32)
    idx = np.flatnonzero(flags)
    dom[idx] = 1 + np.arange(len(idx), dtype=np.int32)
    P = 1 + len(idx)
    params = oracle.make_params(pk.dim, pk.n_walls, n_domains=P, **kw)
    color, slot, ds = oracle.order(pk.n, ci, cj, P, dom)
    R, info, _ = oracle.solve(params, pk, ci, cj, normal, gap, P, ds, slot)
    return R, info


def test_pair_numbers_are_the_input_generators(oracle):
    rng = np.random.default_rng(3)
    ci = rng.integers(0, 10**6, 500).astype(np.int32)
    cj = rng.integers(0, 10**6, 500).astype(np.int32)
    for seed in (0, 17, 2**40 + 5):
        u = inputs.pair_mu(seed, ci, cj, 0.0, 1.0)
        got = np.array([oracle.pair_uniform(seed, int(a), int(b)) for a, b in zip(ci, cj)])
        np.testing.assert_array_equal(got, u)
        np.testing.assert_array_equal(oracle.parallel_flags(ci, cj, 0.4, seed), u < 0.4)


@pytest.mark.parametrize("dim,p,kw", [
    (2, 0.3, dict(mu=0.3, fixed_iters=40)),
    (2, 0.3, dict(mu=0.3)),
    (2, 1.0, dict(mu=0.3, fixed_iters=25)),
    (3, 0.4, dict(mu=0.5, fixed_iters=30)),
])
def test_parallel_contacts_act_as_domains_of_their_own(oracle, dim, p, kw):
    if dim == 2:
        pk = inputs.lattice_2d(16, 16, 21)
    else:
        pk = inputs.lattice_3d(7, 7, 6, 22, gravity=1.0)
    ci, cj, normal, gap = _geometry(oracle, pk)
    flags = oracle.parallel_flags(ci, cj, p, 9)
    assert 0 < flags.sum() <= len(ci)
    Rm, im, color, slot = _mixed(oracle, pk, ci, cj, normal, gap, flags, **kw)
    Rd, idm = _own_domains(oracle, pk, ci, cj, normal, gap, flags, **kw)
    assert im.iterations == idm.iterations and im.status == idm.status
    np.testing.assert_array_equal(Rm, Rd)
    # parallel contacts carry colour 0 and open the order; the rest start at 1
    assert np.all(color[flags == 1] == 0) and np.all(color[flags == 0] >= 1)
    assert np.all(flags[slot[:int(flags.sum())]] == 1)


def test_no_parallel_contacts_is_the_plain_solve(oracle):
    pk = inputs.lattice_2d(16, 16, 21)
    ci, cj, normal, gap = _geometry(oracle, pk)
    flags = np.zeros(len(ci), np.uint8)
    Rm, im, color, _ = _mixed(oracle, pk, ci, cj, normal, gap, flags, mu=0.3)
    params = oracle.make_params(2, pk.n_walls, n_domains=1, mu=0.3)
    c0, s0, d0 = oracle.order(pk.n, ci, cj, 1, np.zeros(len(ci), np.int32))
    R0, i0, _ = oracle.solve(params, pk, ci, cj, normal, gap, 1, d0, s0)
    np.testing.assert_array_equal(Rm, R0)
    assert im.iterations == i0.iterations
    np.testing.assert_array_equal(color, c0 + 1)   # colours shifted past the parallel block


@pytest.mark.parametrize("n", [64, 128])
def test_chain_sweeps_follow_the_diffusion_model(oracle, n):
    """Sec. 4.3, Fig. 13(a, b): a chain of n touching disks compressed by a
    force, cut into P domains, needs N_I(P) / N_I(1) = D_s / D_eff sweeps
    with D_eff = D_p p + D_s (1 - p), p = P / n and the fitted
    D_s / D_p = 1.53; within 2 %."""
    pk = inputs.chain_2d(n, 1.0)
    base = None
    for P in (1, 2, 4, 8, 16):
        sim = oracle.Sim(oracle.make_params(2, pk.n_walls, mu=0.3, n_domains=P, max_iter=100000),
                         pk)
        info = sim.step()
        assert info.status == 0
        base = base or info.iterations
        model = 1.0 / (1.0 - (P / n) * (1.0 - 1.0 / 1.53))
        assert info.iterations / base == pytest.approx(model, rel=0.02)
