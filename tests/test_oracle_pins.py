"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Every test here runs on the CPU.  None of them re-types the oracle's own
formulas: they use closed forms derived by hand, hand-computed sweep
sequences, static equilibria, conservation laws, brute-force enumeration of
contact states, the frictionless reduction to a textbook LCP, and the
paper's worked tree example.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests import physics_pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_packing(dim, x, v, r, w=None, walls=(), gravity=0.0, force=None, lo=None, hi=None):
    x = np.asarray(x, dtype=np.float64).T.copy()
    v = np.asarray(v, dtype=np.float64).T.copy()
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    dr = 1 if dim == 2 else 3
    if dim == 2:
        m = math.pi * r * r
        inertia = 0.5 * m * r * r
    else:
        m = 4.0 / 3.0 * math.pi * r ** 3
        inertia = 0.4 * m * r * r
    w = np.zeros((dr, n)) if w is None else np.asarray(w, dtype=np.float64).reshape(dr, n)
    f = np.zeros((dim, n))
    f[dim - 1] = -m * gravity
    if force is not None:
        f += np.asarray(force, dtype=np.float64).T
    wn = np.array([wl[0] for wl in walls], dtype=np.float64).reshape(len(walls), dim)
    wo = np.array([wl[1] for wl in walls], dtype=np.float64)
    wv = np.array([wl[2] if len(wl) > 2 else np.zeros(dim) for wl in walls],
                  dtype=np.float64).reshape(len(walls), dim)
    lo = np.full(dim, -10.0) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.full(dim, 10.0) if hi is None else np.asarray(hi, dtype=np.float64)
    return inputs.Packing(dim, x, v, w, r, m, inertia, f, np.zeros((dr, n)), wn, wo, wv, lo, hi)


def solve_all(oracle, pk, mu=0.3, P=1, fixed=0, alpha=1e-6, max_iter=2000, skin=0.0, mu_c=None,
              history=False, criterion=0):
    ci, cj = oracle.detect(pk, skin, use_cells=False)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    tree, dom = oracle.orb(pk.dim, P, pk.box_lo, pk.box_hi, xmid)
    color, slot, ds = oracle.order(pk.n, ci, cj, P, dom)
    params = oracle.make_params(pk.dim, pk.n_walls, mu=mu, n_domains=P, fixed_iters=fixed,
                                alpha=alpha, max_iter=max_iter, criterion=criterion)
    R, info, hist = oracle.solve(params, pk, ci, cj, normal, gap, P, ds, slot, mu_c=mu_c,
                                 history=history)
    return dict(ci=ci, cj=cj, normal=normal, gap=gap, xmid=xmid, dom=dom, color=color,
                slot=slot, ds=ds, R=R, info=info, hist=hist, params=params)


# --------------------------------------------------------------------------
# single contact: closed forms of Sec. 2.1 (Eqs. 3-9)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gap0", [0.0, 2e-4])
def test_head_on_two_disks(oracle, gap0):
    """Closing speed U along the normal: R_n = m_red (U - g/dt)/dt, R_t = 0,
    post-step normal relative velocity -g/dt; momentum is conserved and the
    second sweep changes nothing."""
    U, dt = 0.5, 1e-3
    pk = make_packing(2, [[0.0, 0.0], [2.0 + gap0, 0.0]], [[U / 2, 0.0], [-U / 2, 0.0]],
                      [1.0, 1.0])
    out = solve_all(oracle, pk, skin=1e-3, fixed=2)
    m = pk.m[0]
    mred = m / 2
    expect = mred * (U - gap0 / dt) / dt
    assert len(out["ci"]) == 1
    assert out["R"][0, 0] == pytest.approx(expect, rel=1e-12)
    assert out["R"][1, 0] == 0.0
    V, W = oracle.velocities(pk, dt, out["ci"], out["cj"], out["normal"], out["R"])
    rel_normal = V[0, 1] - V[0, 0]
    assert rel_normal == pytest.approx(-gap0 / dt, abs=1e-12)
    assert (pk.m * V[0]).sum() == pytest.approx(0.0, abs=1e-12)
    # converged after the second sweep: D = 0 for the only contact
    out2 = solve_all(oracle, pk, skin=1e-3, max_iter=50)
    assert out2["info"].iterations == 2 and out2["info"].status == 0


def test_head_on_stays_open(oracle):
    """If the predicted gap g + dt u_n stays positive, R = 0 (Eq. 3)."""
    U, dt, gap0 = 0.1, 1e-3, 2e-4    # U dt = 1e-4 < g
    pk = make_packing(2, [[0.0, 0.0], [2.0 + gap0, 0.0]], [[U / 2, 0.0], [-U / 2, 0.0]],
                      [1.0, 1.0])
    out = solve_all(oracle, pk, skin=1e-3, fixed=1)
    assert np.all(out["R"] == 0.0)


@pytest.mark.parametrize("ut_over_un", [0.5, 1.0, 1.5])
def test_oblique_disks_stick_or_slide(oracle, ut_over_un):
    """Equal touching disks, relative normal velocity -U and tangential u_t.
    For disks w_t = 3 w_n, so the contact sticks iff |u_t| <= 3 mu U; a
    sliding contact carries R_t = -mu R_n sign(u_t).  Spins change by
    -r R_t dt / I on both disks."""
    mu, U, dt = 0.3, 1.0, 1e-3
    ut = ut_over_un * 3 * mu * U
    # n = +x, t = z x n = +y: give body 2 the tangential velocity ut
    pk = make_packing(2, [[0.0, 0.0], [2.0, 0.0]], [[0.0, 0.0], [-U, ut]], [1.0, 1.0])
    out = solve_all(oracle, pk, mu=mu, fixed=1)
    m, inertia, r = pk.m[0], pk.inertia[0], 1.0
    Rn = (m / 2) * U / dt
    assert out["R"][0, 0] == pytest.approx(Rn, rel=1e-13)
    if ut_over_un <= 1.0:
        # sticking force cancels the tangential slip: R_t = -u_t / (dt w_t)
        assert out["R"][1, 0] == pytest.approx(-ut / (dt * 6.0 / m), rel=1e-12)
    else:
        assert out["R"][1, 0] == pytest.approx(-mu * Rn, rel=1e-13)
    V, W = oracle.velocities(pk, dt, out["ci"], out["cj"], out["normal"], out["R"])
    Rt = out["R"][1, 0]
    assert W[0, 0] == pytest.approx(-r * Rt * dt / inertia, rel=1e-12)
    assert W[0, 1] == pytest.approx(-r * Rt * dt / inertia, rel=1e-12)
    # tangential slip after the step: 0 if sticking, same sign as before if sliding
    slip = (V[1, 1] - W[0, 1] * r) - (V[1, 0] + W[0, 0] * r)
    if ut_over_un < 1.0:
        assert abs(slip) < 1e-12
    elif ut_over_un > 1.0:
        assert slip > 0


@pytest.mark.parametrize("ut_over_un", [0.7, 1.3])
def test_oblique_spheres_cone(oracle, ut_over_un):
    """Spheres: w_t = 3.5 w_n, stick iff |u_t| <= 3.5 mu U; sliding force
    antiparallel to the slip with |R_t| = mu R_n (the 3D cone)."""
    mu, U, dt = 0.5, 1.0, 1e-3
    d = np.array([0.0, 0.6, 0.8])
    ut = ut_over_un * 3.5 * mu * U * d
    pk = make_packing(3, [[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]], [[0.0, 0.0, 0.0], [-U, ut[1], ut[2]]],
                      [1.0, 1.0])
    out = solve_all(oracle, pk, mu=mu, fixed=1)
    m = pk.m[0]
    Rn = (m / 2) * U / dt
    normal = out["normal"][:, 0]
    # world tangential force from the frame coefficients via the frame check below
    V, W = oracle.velocities(pk, dt, out["ci"], out["cj"], out["normal"], out["R"])
    dP = pk.m[1] * (V[:, 1] - pk.v[:, 1]) / dt      # force on body 2
    assert dP @ normal == pytest.approx(Rn, rel=1e-12)
    Rt = dP - (dP @ normal) * normal
    if ut_over_un < 1:
        np.testing.assert_allclose(Rt, -ut / (dt * 7.0 / m), rtol=1e-11, atol=1e-9)
    else:
        np.testing.assert_allclose(Rt, -mu * Rn * ut / np.linalg.norm(ut), rtol=1e-11, atol=1e-9)
    assert out["R"][0, 0] == pytest.approx(Rn, rel=1e-13)


# --------------------------------------------------------------------------
# domain-wise sweep semantics (Sec. 3.1) on a hand-computed case
# --------------------------------------------------------------------------

def test_domain_semantics_three_disks(oracle):
    gold = json.load(open(os.path.join(GOLDEN, "domain_jacobi_3disks.json")))
    U, dt = 1.0, 1e-3
    pk = make_packing(2, [[0.0, 0.0], [2.0, 0.0], [4.0, 0.0]], [[U, 0], [0, 0], [-U, 0]],
                      [1.0, 1.0, 1.0])
    ci, cj = oracle.detect(pk, 0.0, use_cells=False)
    assert list(ci) == [0, 1] and list(cj) == [1, 2]
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    unit = pk.m[0] * U / dt
    for P, key in ((1, "sequential_one_domain"), (2, "two_domains_one_contact_each")):
        if P == 1:
            ds, slot = np.array([0, 2]), np.array([0, 1])
        else:
            ds, slot = np.array([0, 1, 2]), np.array([0, 1])
        for j, (name, vals) in enumerate(sorted(gold[key].items()), start=1):
            params = oracle.make_params(2, 0, n_domains=P, fixed_iters=j)
            R, info, _ = oracle.solve(params, pk, ci, cj, normal, gap, P, ds, slot)
            np.testing.assert_allclose(R[0] / unit, vals, rtol=1e-12)
    # the ORB on this row puts one contact in each of two domains
    tree, dom = oracle.orb(2, 2, pk.box_lo, pk.box_hi, xmid)
    assert list(dom) == [0, 1]


# --------------------------------------------------------------------------
# static equilibria: the exact force network is known
# --------------------------------------------------------------------------

def test_static_column_carries_weight(oracle):
    n = 6
    pk = inputs.column_2d(n)
    out = solve_all(oracle, pk, fixed=400)
    m, g = pk.m[0], 1.0
    ci, cj, R = out["ci"], out["cj"], out["R"]
    for c in range(len(ci)):
        if cj[c] >= pk.n:
            assert R[0, c] == pytest.approx(n * m * g, rel=1e-9)   # floor carries all
        else:
            above = n - 1 - ci[c]
            assert R[0, c] == pytest.approx(above * m * g, rel=1e-9)
        assert abs(R[1, c]) < 1e-9 * m
    V, W = oracle.velocities(pk, 1e-3, ci, cj, out["normal"], R)
    assert np.abs(V).max() < 1e-10


def test_chain_end_force(oracle):
    """Fig. 13a: a chain of touching disks between two walls, pushed with F
    at one end: every contact force equals F and the near wall is unloaded."""
    n, F = 12, 3.0
    pk = inputs.chain_2d(n, F)
    for P in (1, 3):
        out = solve_all(oracle, pk, fixed=3000, P=P)
        ci, cj, R = out["ci"], out["cj"], out["R"]
        for c in range(len(ci)):
            if cj[c] == pk.n:          # wall at x = 0 (the pushed end's wall)
                assert abs(R[0, c]) < 1e-9 * F
            else:
                assert R[0, c] == pytest.approx(F, rel=1e-9)


# --------------------------------------------------------------------------
# invariants on a generated packing
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_packing_solution(oracle):
    pk = inputs.lattice_2d(16, 16, 7)
    skin = 2 * np.sqrt((pk.v ** 2).sum(0)).max() * 1e-3
    out = solve_all(oracle, pk, mu=0.3, P=4, fixed=4000, skin=skin)
    return pk, out


def test_invariants_cone_and_momentum(oracle, small_packing_solution):
    pk, out = small_packing_solution
    R, mu, dt = out["R"], 0.3, 1e-3
    assert np.all(R[0] >= 0)
    assert np.all(np.abs(R[1]) <= mu * R[0] * (1 + 1e-15))
    V, W = oracle.velocities(pk, dt, out["ci"], out["cj"], out["normal"], R)
    n = out["normal"]
    t = np.stack([-n[1], n[0]])
    world = R[0] * n + R[1] * t
    wall = out["cj"] >= pk.n
    lhs = (pk.m * (V - pk.v)).sum(axis=1)
    rhs = dt * (pk.f.sum(axis=1) - world[:, wall].sum(axis=1))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-12 * np.abs(dt * pk.f).sum())


def test_converged_complementarity(oracle, small_packing_solution):
    pk, out = small_packing_solution
    R, mu, dt = out["R"], 0.3, 1e-3
    V, W = oracle.velocities(pk, dt, out["ci"], out["cj"], out["normal"], R)
    J = pins.jacobian_2d(pk, out["ci"], out["cj"], out["normal"])
    q = np.zeros(3 * pk.n)
    q[0::3], q[1::3], q[2::3] = V[0], V[1], W[0]
    u = J @ q + pins.wall_velocity_terms_2d(pk, out["ci"], out["cj"], out["normal"])
    un, ut = u[0::2], u[1::2]
    pred = np.maximum(out["gap"], 0.0) / dt + un     # predicted gap / dt
    vs = np.abs(pk.v).max() + 1.0
    fs = R[0].max()
    assert np.all(pred >= -1e-8 * vs)
    assert np.all(np.abs(R[0] * pred) <= 1e-8 * vs * fs)
    stick = np.abs(R[1]) < mu * R[0] * (1 - 1e-9)
    assert np.all(np.abs(ut[stick & (R[0] > 0)]) <= 1e-8 * vs)
    slide = (R[0] > 0) & ~stick
    assert np.all(R[1, slide] * ut[slide] <= 1e-8 * vs * fs)


# --------------------------------------------------------------------------
# brute force: every open/stick/slide assignment of a 3-contact system
# --------------------------------------------------------------------------

def _case_corner():
    s3 = math.sqrt(3.0)
    return make_packing(2, [[1.0, 1.0], [2.0, 1.0 + s3]], [[-0.3, 0.1], [0.2, -0.5]], [1.0, 1.0],
                        w=[[0.4, -0.2]], walls=[([1.0, 0.0], 0.0), ([0.0, 1.0], 0.0)],
                        gravity=1.0)


def _case_between_walls():
    return make_packing(2, [[1.0, 5.0], [3.0, 5.0]], [[0.5, 0.05], [-0.5, -0.1]], [1.0, 1.0],
                        w=[[0.0, 0.3]], walls=[([1.0, 0.0], 0.0), ([-1.0, 0.0], -4.0)],
                        gravity=1.0)


def _case_floor_two_neighbours():
    s3 = math.sqrt(3.0)
    return make_packing(2, [[0.0, 1.0], [-s3, 2.0], [s3, 2.0]],
                        [[0.01, -0.2], [0.3, -0.1], [-0.1, -0.4]], [1.0, 1.0, 1.0],
                        walls=[([0.0, 1.0], 0.0)], gravity=1.0)


@pytest.mark.parametrize("case", [_case_corner, _case_between_walls, _case_floor_two_neighbours])
@pytest.mark.parametrize("mu", [0.1, 0.3, 0.8])
def test_brute_force_three_contacts(oracle, case, mu):
    pk = case()
    dt = 1e-3
    out = solve_all(oracle, pk, mu=mu, fixed=6000, skin=1e-9)
    assert len(out["ci"]) == 3
    args = (pk, out["ci"], out["cj"], out["normal"], out["gap"], dt, mu)
    # the converged forces satisfy the whole one-step problem for some
    # assignment of contact states ...
    accepted = pins.consistent_states_2d(*args, out["R"])
    assert accepted, "converged forces satisfy no open/stick/slide assignment"
    # ... and where that assignment has an isolated solution, they are it
    sols = pins.enumerate_states_2d(*args)
    scale = 1.0 + np.abs(out["R"]).max()
    if sols:
        err = min(np.abs(out["R"] - s).max() for s in sols) / scale
        A = pins.delassus_2d(pk, out["ci"], out["cj"], out["normal"], dt)[0]
        if np.linalg.eigvalsh(A).min() > 1e-12 * np.abs(A).max():
            assert err < 1e-8


# --------------------------------------------------------------------------
# textbook reduction: mu = 0 is a symmetric positive definite LCP
# --------------------------------------------------------------------------

def test_frictionless_matches_lcp(oracle):
    pk = inputs.lattice_2d(10, 10, 11)
    skin = 2 * np.sqrt((pk.v ** 2).sum(0)).max() * 1e-3
    for P in (1, 4):
        out = solve_all(oracle, pk, mu=0.0, P=P, fixed=6000, skin=skin)
        Rn = pins.frictionless_lcp_2d(pk, out["ci"], out["cj"], out["normal"], out["gap"], 1e-3)
        assert np.all(out["R"][1] == 0.0)
        np.testing.assert_allclose(out["R"][0], Rn, rtol=0, atol=1e-8 * Rn.max())


# --------------------------------------------------------------------------
# hierarchical tree (Sec. 3.2, Fig. 8) and the contact-count bisection
# --------------------------------------------------------------------------

def test_tree_p14_matches_paper(oracle):
    gold = json.load(open(os.path.join(GOLDEN, "tree_p14.json")))
    P = gold["P"]
    rng = np.random.default_rng(0)
    xmid = rng.uniform(0, 1, size=(2, 1000))
    tree, dom = oracle.orb(2, P, [0, 0], [1, 1], xmid)
    leaves = tree.leaves
    assert leaves[0] == P
    l, r = tree.child[0], tree.child[1]
    assert [leaves[l], leaves[r]] == gold["root_split_leaves"]
    assert [leaves[tree.child[2 * r]], leaves[tree.child[2 * r + 1]]] == gold["right_child_split_leaves"]


@pytest.mark.parametrize("P", [1, 2, 3, 5, 7, 8, 14, 100, 4096])
def test_tree_shape(oracle, P):
    leaves = oracle.tree_leaves(P)
    assert leaves[0] == P
    assert (leaves == 1).sum() == P
    # leaves differ in depth by at most one (Fig. 8)
    tree, _ = oracle.orb(2, P, [0, 0], [1, 1], np.zeros((2, 0)))
    depth = np.zeros(2 * P - 1, int)
    for k in range(2 * P - 1):
        if tree.child[2 * k] >= 0:
            depth[tree.child[2 * k]] = depth[k] + 1
            depth[tree.child[2 * k + 1]] = depth[k] + 1
    ld = depth[tree.leaf >= 0]
    assert ld.max() - ld.min() <= 1
    assert sorted(tree.leaf[tree.leaf >= 0]) == list(range(P))


@pytest.mark.parametrize("P", [2, 14, 64, 333])
def test_orb_balances_contacts(oracle, P):
    pk = inputs.lattice_2d(40, 30, 5)
    ci, cj = oracle.detect(pk, 1e-4)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    tree, dom = oracle.orb(2, P, pk.box_lo, pk.box_hi, xmid)
    counts = np.bincount(dom, minlength=P)
    # each cut splits in proportion to leaf counts (floor), so domains differ
    # by at most one contact per tree level plus ties at the cut
    assert counts.max() - counts.min() <= int(math.ceil(math.log2(P))) + 2
    np.testing.assert_array_equal(oracle.descend(2, P, tree, xmid), dom)
    # every contact lies inside its domain's region on each cut axis
    lo, hi = pk.box_lo.copy(), pk.box_hi.copy()

    def walk(node, lo, hi, members):
        if tree.leaf[node] >= 0:
            assert np.all(dom[members] == tree.leaf[node])
            return
        a, cut = tree.axis[node], tree.cut[node]
        left = members[xmid[a, members] < cut]
        right = members[xmid[a, members] >= cut]
        walk(tree.child[2 * node], lo, hi, left)
        walk(tree.child[2 * node + 1], lo, hi, right)

    walk(0, lo, hi, np.arange(len(ci)))


# --------------------------------------------------------------------------
# detection: cell method == brute force; colouring validity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,skin", [((32, 32), 1e-4), ((31, 17), 0.2), ((8, 8, 8), 1e-4),
                                        ((7, 9, 5), 0.2)])
def test_detect_cells_equals_brute_force(oracle, shape, skin):
    pk = inputs.lattice_2d(*shape, 3) if len(shape) == 2 else inputs.lattice_3d(*shape, 3)
    a = oracle.detect(pk, skin, use_cells=True)
    b = oracle.detect(pk, skin, use_cells=False)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    # canonical order, and every listed pair really is within the skin
    key = a[0].astype(np.int64) * (pk.n + pk.n_walls) + a[1]
    assert np.all(np.diff(key) > 0)
    normal, gap, _ = oracle.geometry(pk, a[0], a[1])
    assert np.all(gap <= skin)
    np.testing.assert_allclose(np.linalg.norm(normal, axis=0), 1.0, rtol=1e-15)


def test_colouring_is_first_fit_and_conflict_free(oracle):
    pk = inputs.lattice_2d(24, 24, 9)
    ci, cj = oracle.detect(pk, 1e-4)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    P = 9
    tree, dom = oracle.orb(2, P, pk.box_lo, pk.box_hi, xmid)
    color, slot, ds = oracle.order(pk.n, ci, cj, P, dom)
    for d in range(P):
        members = np.flatnonzero(dom == d)
        used = {}
        for c in members:                       # canonical order
            ends = [ci[c]] + ([cj[c]] if cj[c] < pk.n else [])
            taken = set()
            for e in ends:
                taken |= used.get(e, set())
            first_free = next(k for k in range(1000) if k not in taken)
            assert color[c] == first_free
            for e in ends:
                used.setdefault(e, set()).add(color[c])
        s = slot[ds[d]:ds[d + 1]]
        assert sorted(s) == list(members)
        keys = list(zip(color[s], s))
        assert keys == sorted(keys)


# --------------------------------------------------------------------------
# convergence criteria on hand-made force sequences (Sec. 2.1)
# --------------------------------------------------------------------------

def test_criterion_zero_over_zero_passes(oracle):
    R = np.zeros((2, 5))
    conv, npass, maxd, ravg, fin = oracle.criterion(R, R, 0.0, 1e-6, 0)
    assert conv and npass == 5 and ravg == 0.0


def test_criterion_ninety_percent_boundary(oracle):
    nc = 20
    Rprev = np.ones((2, nc))
    R = Rprev.copy()
    # two contacts (10%) change by a relative 1e-2 (squared ratio 2.5e-5 > alpha)
    R[0, :2] = 1.0 + 1e-2 * 2
    conv, npass, maxd, ravg, _ = oracle.criterion(Rprev, R, math.sqrt(2), 1e-6, 0)
    assert npass == 18
    # the rest test: |dR|^2 = 4e-4 < alpha * R_avg^2 needs R_avg^2 > 400
    assert not conv
    conv, *_ = oracle.criterion(Rprev, R, 30.0, 1e-6, 0)
    assert conv
    # three failing contacts (85% pass) never converge
    R[0, :3] = 1.02
    conv, npass, *_ = oracle.criterion(Rprev, R, 1e6, 1e-6, 0)
    assert npass == 17 and not conv


def test_criterion_strict_threshold(oracle):
    # D / S exactly alpha does not pass (strict inequality)
    alpha = 0.25
    Rprev = np.array([[1.0], [0.0]])
    R = np.array([[3.0], [0.0]])          # D = 4, S = 16, D/S = 0.25
    conv, npass, *_ = oracle.criterion(Rprev, R, 1.0, alpha, 0)
    assert npass == 0
    conv, npass, *_ = oracle.criterion(Rprev, R, 1.0, 0.2500001, 0)
    assert npass == 1


def test_criterion_global(oracle):
    R0 = np.full((2, 4), 1.0)
    R1 = R0 * 1.0001
    conv, _, _, ravg, _ = oracle.criterion(R0, R1, math.sqrt(2), 1e-6, 1)
    # (dRavg)^2 / (sum)^2 = (1e-4)^2/(2.0001)^2 ~ 2.5e-9 < 1e-6
    assert conv and ravg == pytest.approx(math.sqrt(2) * 1.0001, rel=1e-14)
    conv, *_ = oracle.criterion(R0, R0 * 1.01, math.sqrt(2), 1e-6, 1)
    assert not conv


# --------------------------------------------------------------------------
# time stepping (Eqs. 1-2) and the 3D contact frame
# --------------------------------------------------------------------------

def test_euler_step_and_warm_start(oracle):
    pk = inputs.lattice_2d(12, 10, 21)
    params = oracle.make_params(2, pk.n_walls, n_domains=3, repartition_every=2)
    sim = oracle.Sim(params, pk)
    info = sim.step()
    c = sim.contacts()
    x, v, w, wo = sim.state()
    V, W = oracle.velocities(pk, 1e-3, c["ci"], c["cj"], c["normal"], c["R"])
    np.testing.assert_array_equal(v, V)
    np.testing.assert_array_equal(w, W)
    np.testing.assert_array_equal(x, pk.x + V * 1e-3)
    # the next step starts from the forces of the same pairs
    info2 = sim.step()
    assert info2.iterations < info.iterations


def test_tangent_basis_right_handed(oracle):
    rng = np.random.default_rng(3)
    pts = rng.normal(size=(3, 200))
    pts /= np.linalg.norm(pts, axis=0)
    pts[:, 0] = [0, 0, -1.0]
    pts[:, 1] = [0, 0, 1.0]
    # two spheres touching along each direction; the oracle's frame shows up
    # in the forces: a sticking force of a purely tangential slip must be
    # antiparallel to the slip whatever the basis
    for k in range(5):
        n = pts[:, k]
        slip = np.cross(n, [0.3, -0.2, 0.5])
        pk = make_packing(3, [[0, 0, 0], list(2.0 * n)], [[0, 0, 0], list(-n + 0.01 * slip)],
                          [1.0, 1.0])
        out = solve_all(oracle, pk, mu=10.0, fixed=1, skin=1e-9)
        V, W = oracle.velocities(pk, 1e-3, out["ci"], out["cj"], out["normal"], out["R"])
        force = pk.m[1] * (V[:, 1] - pk.v[:, 1]) / 1e-3
        ft = force - (force @ n) * n
        if np.linalg.norm(slip) > 0:
            cosang = ft @ slip / (np.linalg.norm(ft) * np.linalg.norm(slip))
            assert cosang == pytest.approx(-1.0, abs=1e-12)


def test_contact_position_mid_gap(oracle):
    """The contact position is the middle of the gap (Sec. 3.1, Fig. 1)."""
    pk = make_packing(2, [[0.0, 0.0], [3.0, 0.0], [0.0, 5.0]], [[0, 0]] * 3, [1.0, 1.5, 1.0],
                      walls=[([0.0, 1.0], -0.5)])
    ci, cj = oracle.detect(pk, 1.0, use_cells=False)
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    got = {(int(a), int(b)): (g, xmid[:, k]) for k, (a, b, g) in enumerate(zip(ci, cj, gap))}
    # disks 0 and 1: surfaces at x = 1 and x = 1.5
    g, p = got[(0, 1)]
    assert g == pytest.approx(0.5) and p == pytest.approx([1.25, 0.0])
    # disk 0 and the floor y = -0.5: surface at y = -1, gap 0.5... overlap of 0.5
    g, p = got[(0, 3)]
    assert g == pytest.approx(-0.5) and p == pytest.approx([0.0, -0.75])
