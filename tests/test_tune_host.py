"""Host logic of the domain-count tuner: the boundary share of a
decomposition and the candidate domain counts (no GPU)."""
import numpy as np

from paper_1104_3516_amd import tune


def test_boundary_fraction_hand_case():
    # particles 0..3, one wall (id 4): particle 1 has contacts in domains 0
    # and 1, so the two contacts touching it are boundary contacts
    ci = np.array([0, 1, 2, 3])
    cj = np.array([1, 2, 3, 4])
    dom = np.array([0, 1, 1, 1])
    assert tune.boundary_fraction(ci, cj, dom, 4) == 0.5
    assert tune.boundary_fraction(ci, cj, np.zeros(4, int), 4) == 0.0
    assert tune.boundary_fraction(ci[:0], cj[:0], dom[:0], 4) == 0.0


def test_boundary_fraction_against_brute_force():
    rng = np.random.default_rng(3)
    n, nc, P = 60, 200, 7
    ci = rng.integers(0, n, nc)
    cj = rng.integers(0, n + 3, nc)
    dom = rng.integers(0, P, nc)
    doms = {p: set() for p in range(n)}
    for a, b, d in zip(ci, cj, dom):
        doms[a].add(d)
        if b < n:
            doms[b].add(d)
    want = np.mean([len(doms[a]) > 1 or (b < n and len(doms[b]) > 1) for a, b in zip(ci, cj)])
    assert tune.boundary_fraction(ci, cj, dom, n) == want


def test_domain_candidates():
    assert tune.domain_candidates(262144) == [256, 512, 1024, 2048, 4096, 8192, 16384]
    assert tune.domain_candidates(100, lo=10, hi=50) == [2, 4, 8]
    assert tune.domain_candidates(5) == []
