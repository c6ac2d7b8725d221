"""Pins of the oracle's adaptive load balancing (Sec. 3.3) on the CPU.

The capacity of a branch is the sum over its leaves of V_i / T_i; each
inner node is cut so that its left branch receives the share
nu_L / (nu_L + nu_R) of the node's contacts (reading C25: contacts take the
place of the volume, as in the contact-count bisection).  Pinned against
the paper's worked example, against brute-force sums over the leaves below
each node, against the leaf-count shares for equal capacities, and against
counts of contacts sent left.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _leaves_below(child, node):
    if child[2 * node] < 0:
        return [node]
    return _leaves_below(child, child[2 * node]) + _leaves_below(child, child[2 * node + 1])


def _shape(oracle, P):
    pk_x = np.zeros((2, 1))
    t, _ = oracle.orb(2, P, [0.0, 0.0], [1.0, 1.0], pk_x[:, :0])
    return t


def test_worked_example_of_the_paper(oracle):
    """Fig. 8's 14 leaves: equal times give 8/14 at the root and 4/6 on its
    right; processors 12 and 13 at half speed give 8/13 and 4/5."""
    g = json.load(open(os.path.join(GOLDEN, "load_balance_p14.json")))
    P = g["P"]
    t = _shape(oracle, P)
    right = t.child[1]
    # the right branch of the root holds the slow leaves, below its right child
    leaf_ids = [t.leaf[n] for n in _leaves_below(t.child, t.child[2 * right + 1])]
    assert sorted(leaf_ids) == g["slow_leaves"]
    T = np.ones(P)
    f = oracle.balance_fractions(P, 1.0 / T)
    a, b = g["equal_times"]["root_left_share"]
    assert f[0] == a / b
    a, b = g["equal_times"]["right_node_left_share"]
    assert f[right] == a / b
    T[g["slow_leaves"]] = g["slow_time_factor"]
    f = oracle.balance_fractions(P, 1.0 / T)
    a, b = g["slowed"]["root_left_share"]
    assert f[0] == a / b
    a, b = g["slowed"]["right_node_left_share"]
    assert f[right] == a / b


@pytest.mark.parametrize("P", list(range(1, 41)))
def test_equal_capacities_give_leaf_count_shares(oracle, P):
    t = _shape(oracle, P)
    f = oracle.balance_fractions(P, np.full(P, 3.7))
    for node in range(2 * P - 1):
        if t.child[2 * node] < 0:
            assert f[node] == 0.0
        else:
            L, R = t.leaves[t.child[2 * node]], t.leaves[t.child[2 * node + 1]]
            assert f[node] == pytest.approx(L / (L + R), rel=1e-15)


def test_shares_are_capacity_sums_over_the_leaves_below(oracle):
    P = 23
    rng = np.random.default_rng(7)
    cap = rng.uniform(0.2, 5.0, P)
    t = _shape(oracle, P)
    f = oracle.balance_fractions(P, cap)
    for node in range(2 * P - 1):
        if t.child[2 * node] < 0:
            continue
        left = sum(cap[t.leaf[n]] for n in _leaves_below(t.child, t.child[2 * node]))
        right = sum(cap[t.leaf[n]] for n in _leaves_below(t.child, t.child[2 * node + 1]))
        assert f[node] == pytest.approx(left / (left + right), rel=1e-13)


def test_capacities_without_a_measurement_count_as_the_mean(oracle):
    """P = 4 (two pairs): capacities (1, 0, 3, NaN) act as (1, 2, 3, 2)."""
    f = oracle.balance_fractions(4, [1.0, 0.0, 3.0, float("nan")])
    assert f[0] == pytest.approx(3.0 / 8.0, rel=1e-15)
    f_none = oracle.balance_fractions(4, [0.0, -1.0, float("inf"), 0.0])
    assert f_none[0] == 0.5


def test_sigma_t(oracle):
    assert oracle.sigma_t([2.0, 2.0, 2.0]) == 0.0
    assert oracle.sigma_t([1.0, 1.0, 1.0, 3.0]) == pytest.approx(1.0 / math.sqrt(3.0), rel=1e-15)
    # two equal halves at T and 3T: mean 2T, deviation T
    assert oracle.sigma_t([1.0, 3.0] * 5) == pytest.approx(0.5, rel=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cuts_send_the_capacity_share_of_contacts_left(oracle, seed):
    """With distinct contact positions every inner node sends exactly
    floor(n share) of its contacts to its left branch."""
    rng = np.random.default_rng(seed)
    P, nc = 11, 997
    xmid = rng.uniform(0.0, 10.0, (2, nc))
    cap = rng.uniform(0.5, 2.0, P)
    t, dom = oracle.orb(2, P, [0.0, 0.0], [10.0, 10.0], xmid, capacity=cap)
    f = oracle.balance_fractions(P, cap)
    count = np.bincount(dom, minlength=P)
    for node in range(2 * P - 1):
        if t.child[2 * node] < 0:
            continue
        below = lambda n: sum(count[t.leaf[m]] for m in _leaves_below(t.child, n))
        n_node = below(node)
        k = min(max(math.floor(float(n_node) * f[node]), 0), n_node - 1) if n_node else 0
        assert below(t.child[2 * node]) == k
    # no capacities: leaf-count shares in integer arithmetic
    t0, dom0 = oracle.orb(2, P, [0.0, 0.0], [10.0, 10.0], xmid)
    count0 = np.bincount(dom0, minlength=P)
    assert sum(count0[:t0.leaves[t0.child[0]]]) == (nc * t0.leaves[t0.child[0]]) // P
