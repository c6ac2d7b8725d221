"""Pins of the oracle's rotation, wall motion, boundary width, warm start and
update orders.

Every expected value here comes from a closed form of rigid-body mechanics,
an independent matrix formulation of the one-step problem (tests/physics_pins
.py) or plain bookkeeping done in Python from the oracle's outputs; none
re-types the oracle's formulas.

  * 3D contact frame: the force and torque that a unit frame component
    produces on a body give t1, t2 and n x t1 explicitly (Sec. 2.1, Fig. 1).
  * Rolling and sliding spheres (Sec. 2.1, Eqs. 3-9 with rotation): a sphere
    spinning on a floor, and a disk or sphere at rest on a floor that moves
    tangentially (a shear wall), end the step at the classical sticking or
    sliding velocities.
  * Walls translate with their normal velocity and drag the box face they lie
    on (walls as bodies with prescribed motion, Sec. 2.1).
  * The boundary width is 2 v_max dt with wall speeds included, and a width
    above 0.2 r_max is refused (Sec. 3.1).
  * Warm start: a step starts from the previous step's forces of the same
    pairs (paper silent; reading C16).
  * Update orders (Sec. 2.3): the sequential, the fully parallel (Jacobi) and
    the mixed sweep equal projected Gauss-Seidel / projected Jacobi written on
    the Delassus matrix of the frictionless problem.
"""
import math

import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests import physics_pins as pins
from tests.test_oracle_pins import make_packing, solve_all

DT = 1e-3


def sim_of(oracle, pk, **kw):
    params = oracle.make_params(pk.dim, pk.n_walls, **kw)
    return oracle.Sim(params, pk)


# --------------------------------------------------------------------------
# the 3D contact frame, read off the forces and torques the oracle applies
# --------------------------------------------------------------------------

def _frame_from_forces(oracle, n):
    """World force and torque on body 2 of a sphere pair touching along n for
    unit frame components (1,0,0), (0,1,0), (0,0,1)."""
    pk = make_packing(3, [[0, 0, 0], list(2.0 * n)], [[0, 0, 0], [0, 0, 0]], [1.0, 1.0])
    ci, cj = oracle.detect(pk, 1e-9, use_cells=False)
    normal, gap, _ = oracle.geometry(pk, ci, cj)
    assert len(ci) == 1
    out = []
    for k in range(3):
        R = np.zeros((3, 1))
        R[k, 0] = 1.0
        V, W = oracle.velocities(pk, DT, ci, cj, normal, R)
        force = pk.m[1] * V[:, 1] / DT            # impulse on body 2 / dt
        torque = pk.inertia[1] * W[:, 1] / DT
        torque1 = pk.inertia[0] * W[:, 0] / DT
        out.append((force, torque, torque1))
    return normal[:, 0], out


@pytest.mark.parametrize("k", range(8))
def test_frame_is_right_handed_orthonormal(oracle, k):
    rng = np.random.default_rng(100 + k)
    special = [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, -1.0, 0]]
    n = np.array(special[k]) if k < 4 else rng.normal(size=3)
    n = n / np.linalg.norm(n)
    nn, parts = _frame_from_forces(oracle, n)
    (fn, qn, qn1), (f1, q1, q11), (f2, q2, q21) = parts
    np.testing.assert_allclose(fn, nn, rtol=0, atol=1e-13)     # R_n acts along n
    for a, b in ((f1, f2), (f1, fn), (f2, fn)):
        assert abs(a @ b) < 1e-13
    for v in (f1, f2):
        assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-13)
    # t1 x t2 = n, the right-handed frame
    np.testing.assert_allclose(np.cross(f1, f2), nn, rtol=0, atol=1e-13)
    # torque on body 2 (lever -r n) is -r n x F; on body 1 (lever +r n, force -F) too
    np.testing.assert_allclose(q1, -np.cross(nn, f1), rtol=0, atol=1e-13)
    np.testing.assert_allclose(q2, -np.cross(nn, f2), rtol=0, atol=1e-13)
    np.testing.assert_allclose(q11, -np.cross(nn, f1), rtol=0, atol=1e-13)
    np.testing.assert_allclose(qn, 0.0, atol=1e-13)


# --------------------------------------------------------------------------
# rotation: a spinning sphere set on a floor (3D), a body on a moving floor
# --------------------------------------------------------------------------

def _sphere_on_floor(w0, gravity=1.0, floor_velocity=(0.0, 0.0, 0.0)):
    return make_packing(3, [[0.0, 0.0, 1.0]], [[0.0, 0.0, 0.0]], [1.0], w=np.asarray(w0),
                        walls=[([0.0, 0.0, 1.0], 0.0, np.asarray(floor_velocity))],
                        gravity=gravity)


@pytest.mark.parametrize("axis", [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.6, -0.8, 0.0)])
def test_spinning_sphere_sticks_and_rolls(oracle, axis):
    """omega0 about a horizontal axis a, touching a floor under gravity g:
    the contact point slips at s = -r omega0 (a x z).  If the friction needed
    is below mu m g the contact sticks: angular momentum about the contact
    point is conserved, so the sphere ends the step rolling with
    omega' = 2/7 omega0 a and v' = -2/7 s; the normal force is m g."""
    a = np.array(axis)
    w0, mu, g, r = 1e-3, 0.5, 1.0, 1.0          # needs 2 r w0 / 7 <= mu g dt
    assert 2 * r * w0 / 7 <= mu * g * DT
    pk = _sphere_on_floor(w0 * a, gravity=g)
    sim = sim_of(oracle, pk, mu=mu, fixed_iters=3, skin=0.0)
    sim.step()
    x, v, w, _ = sim.state()
    s = -r * w0 * np.cross(a, [0.0, 0.0, 1.0])
    np.testing.assert_allclose(v[:, 0], -2.0 / 7.0 * s, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w[:, 0], 2.0 / 7.0 * w0 * a, rtol=0, atol=1e-15)
    c = sim.contacts()
    assert c["R"][0, 0] == pytest.approx(pk.m[0] * g, rel=1e-13)
    # the contact point is at rest after the step
    cp = v[:, 0] + np.cross(w[:, 0], [0.0, 0.0, -r])
    np.testing.assert_allclose(cp, 0.0, atol=1e-16)


@pytest.mark.parametrize("axis", [(1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.8, 0.6, 0.0)])
def test_spinning_sphere_slides(oracle, axis):
    """Fast spin: the contact slides, the friction force mu m g opposes the
    slip s, v' = -mu g dt s/|s| and omega' = (omega0 - 5 mu g dt / (2 r)) a
    (torque r mu m g about -a, moment of inertia 2/5 m r^2)."""
    a = np.array(axis)
    w0, mu, g, r = 0.1, 0.5, 1.0, 1.0
    pk = _sphere_on_floor(w0 * a, gravity=g)
    sim = sim_of(oracle, pk, mu=mu, fixed_iters=3, skin=0.0)
    sim.step()
    x, v, w, _ = sim.state()
    s = -r * w0 * np.cross(a, [0.0, 0.0, 1.0])
    shat = s / np.linalg.norm(s)
    np.testing.assert_allclose(v[:, 0], -mu * g * DT * shat, rtol=0, atol=1e-16)
    np.testing.assert_allclose(w[:, 0], (w0 - 2.5 * mu * g * DT / r) * a, rtol=0, atol=1e-16)
    R = sim.contacts()["R"][:, 0]
    assert math.hypot(R[1], R[2]) == pytest.approx(mu * R[0], rel=1e-13)


def test_disk_on_moving_floor_sticks(oracle):
    """A disk at rest on a floor moving tangentially at U (a shear wall):
    sticking drags it to v' = U/3, omega' = 2U/(3r) (disk I = m r^2/2), so
    the contact point moves with the floor; the floor does not move along
    its normal, so its offset stays."""
    U, mu, g, r = 5e-4, 0.3, 1.0, 1.0              # needs m U / 3 <= mu m g dt
    pk = make_packing(2, [[0.0, 1.0]], [[0.0, 0.0]], [r],
                      walls=[([0.0, 1.0], 0.0, np.array([U, 0.0]))], gravity=g)
    sim = sim_of(oracle, pk, mu=mu, fixed_iters=3)
    info = sim.step()
    x, v, w, wo = sim.state()
    assert info.skin == pytest.approx(2 * U * DT, rel=1e-15)
    assert v[0, 0] == pytest.approx(U / 3, rel=1e-12) and abs(v[1, 0]) < 1e-18
    assert w[0, 0] == pytest.approx(2 * U / (3 * r), rel=1e-12)
    assert v[0, 0] + w[0, 0] * r == pytest.approx(U, rel=1e-12)
    assert wo[0] == 0.0


def test_sphere_on_moving_floor_sticks_and_slides(oracle):
    """3D: stick gives v' = 2U/7 along the floor velocity and omega' = 5U/(7r)
    about z x u (sphere I = 2/5 m r^2); above 7 mu g dt / 2 the contact slides
    and v' = mu g dt along the floor velocity."""
    mu, g, r = 0.5, 1.0, 1.0
    for U, stick in ((1e-3, True), (0.05, False)):
        u = U * np.array([0.6, 0.8, 0.0])
        pk = _sphere_on_floor([0.0, 0.0, 0.0], gravity=g, floor_velocity=u)
        sim = sim_of(oracle, pk, mu=mu, fixed_iters=3)
        sim.step()
        x, v, w, _ = sim.state()
        uhat = u / U
        spin_axis = np.cross([0.0, 0.0, 1.0], uhat)
        if stick:
            np.testing.assert_allclose(v[:, 0], 2.0 / 7.0 * u, rtol=0, atol=1e-15)
            np.testing.assert_allclose(w[:, 0], -5.0 / 7.0 * U / r * spin_axis, rtol=0,
                                       atol=1e-15)
        else:
            np.testing.assert_allclose(v[:, 0], mu * g * DT * uhat, rtol=0, atol=1e-15)
            np.testing.assert_allclose(w[:, 0], -2.5 * mu * g * DT / r * spin_axis, rtol=0,
                                       atol=1e-15)


# --------------------------------------------------------------------------
# walls: translation, box faces, boundary width
# --------------------------------------------------------------------------

def test_walls_translate_and_drag_box_faces(oracle):
    """After k steps a wall {nu.x = o} moving with u has o = o0 + k dt (nu.u);
    tangential motion leaves it in place; an axis-aligned wall carries the box
    face it lies on, an oblique wall none."""
    s2 = math.sqrt(0.5)
    walls = [([0.0, 1.0], -1.0, np.array([0.3e-3, 0.0])),          # floor, tangential only
             ([0.0, -1.0], -9.0, np.array([0.0, -2e-3])),          # top, moving down
             ([1.0, 0.0], -1.0, np.array([1e-3, 0.0])),            # left, moving right
             ([-s2, -s2], -20.0, np.array([0.0, -1e-3]))]          # oblique, approaching
    pk = make_packing(2, [[3.0, 3.0]], [[0.0, 0.0]], [1.0], walls=walls,
                      lo=[-1.0, -1.0], hi=[12.0, 9.0])
    sim = sim_of(oracle, pk, fixed_iters=2)
    k = 7
    for _ in range(k):
        sim.step()
    _, _, _, wo = sim.state()
    lo, hi = sim.box()
    expect = [-1.0, -9.0 + k * DT * 2e-3, -1.0 + k * DT * 1e-3, -20.0 + k * DT * s2 * 1e-3]
    np.testing.assert_allclose(wo, expect, rtol=1e-14, atol=1e-15)
    assert lo[1] == -1.0                      # the floor did not move
    assert hi[1] == pytest.approx(9.0 - k * DT * 2e-3, rel=1e-14)
    assert lo[0] == pytest.approx(-1.0 + k * DT * 1e-3, abs=1e-15)
    assert hi[0] == 12.0                      # no wall on this face


def test_boundary_width_counts_wall_speed(oracle):
    """skin = 2 v_max dt with v_max over particles and walls: two disks 1.5e-4
    apart are listed when a far wall moves at 0.1 (skin 2e-4), not at 0.05
    (skin 1e-4); a particle faster than every wall sets the width."""
    gap0 = 1.5e-4
    x = [[0.0, 0.0], [2.0 + gap0, 0.0]]
    for speed, listed in ((0.1, True), (0.05, False)):
        walls = [([0.0, 1.0], -50.0, np.array([0.0, speed]))]
        pk = make_packing(2, x, [[0.0, 0.0], [0.0, 0.0]], [1.0, 1.0], walls=walls,
                          lo=[-10, -50], hi=[10, 10])
        sim = sim_of(oracle, pk, fixed_iters=1)
        info = sim.step()
        assert info.skin == pytest.approx(2 * speed * DT, rel=1e-15)
        c = sim.contacts()
        assert (len(c["ci"]) == 1) == listed
    pk = make_packing(2, x, [[0.0, 0.3], [0.0, 0.0]], [1.0, 1.0],
                      walls=[([0.0, 1.0], -50.0, np.array([0.0, 0.05]))], lo=[-10, -50],
                      hi=[10, 10])
    info = sim_of(oracle, pk, fixed_iters=1).step()
    assert info.skin == pytest.approx(2 * 0.3 * DT, rel=1e-15)


def test_boundary_width_above_bound_is_refused(oracle):
    """A width above 0.2 r_max (the displacement bound of the cell method) is
    refused; just below it is accepted."""
    r = 1.0
    vlim = 0.2 * r / (2 * DT)
    for v, ok in ((vlim * 0.999, True), (vlim * 1.001, False)):
        pk = make_packing(2, [[0.0, 0.0]], [[v, 0.0]], [r])
        sim = sim_of(oracle, pk, fixed_iters=1)
        if ok:
            sim.step()
        else:
            with pytest.raises(RuntimeError, match="-1"):
                sim.step()
    # a fixed width is checked the same way
    pk = make_packing(2, [[0.0, 0.0]], [[0.0, 0.0]], [r])
    with pytest.raises(RuntimeError, match="-1"):
        sim_of(oracle, pk, fixed_iters=1, skin=0.21 * r).step()


# --------------------------------------------------------------------------
# warm start: the forces a step starts from
# --------------------------------------------------------------------------

@pytest.mark.parametrize("warm", [1, 0])
def test_warm_start_is_previous_forces_by_pair(oracle, warm):
    """Step 2 of a simulation equals a standalone solve of step 2's list
    started from step 1's forces looked up by pair (i, j) in Python (zero
    for new pairs), or from zero without warm start; a tolerance solve, so
    any other starting forces end elsewhere."""
    pk = inputs.lattice_2d(14, 12, 31)
    pk.v = pk.v * 60.0           # fast enough for pairs to enter and leave the list
    kw = dict(mu=0.3, n_domains=4, repartition_every=1, warm_start=warm, alpha=1e-6,
              max_iter=3000)
    sim = sim_of(oracle, pk, **kw)
    sim.step()
    c1 = sim.contacts()
    x, v, w, wo = sim.state()
    info2 = sim.step()
    c2 = sim.contacts()
    pk2 = pk.copy()
    pk2.x, pk2.v, pk2.w = x, v, w
    ci, cj = oracle.detect(pk2, info2.skin)
    np.testing.assert_array_equal(ci, c2["ci"])
    np.testing.assert_array_equal(cj, c2["cj"])
    normal, gap, xmid = oracle.geometry(pk2, ci, cj)
    tree, dom = oracle.orb(2, 4, pk.box_lo, pk.box_hi, xmid)
    color, slot, ds = oracle.order(pk.n, ci, cj, 4, dom)
    prev = {(int(a), int(b)): c1["R"][:, k] for k, (a, b) in enumerate(zip(c1["ci"], c1["cj"]))}
    R0 = np.zeros((2, len(ci)))
    survived = 0
    if warm:
        for k, (a, b) in enumerate(zip(ci, cj)):
            if (int(a), int(b)) in prev:
                R0[:, k] = prev[(int(a), int(b))]
                survived += 1
        assert 0 < survived < len(ci)
    assert len(c1["ci"]) != len(ci)
    params = oracle.make_params(2, pk.n_walls, **kw)
    R, info, _ = oracle.solve(params, pk2, ci, cj, normal, gap, 4, ds, slot, R0=R0)
    assert info.iterations == info2.iterations
    np.testing.assert_array_equal(R, c2["R"])
    if warm:
        # and the cold start of the same step ends elsewhere
        Rc, infoc, _ = oracle.solve(params, pk2, ci, cj, normal, gap, 4, ds, slot)
        assert infoc.iterations != info2.iterations or np.abs(Rc - c2["R"]).max() > 0


# --------------------------------------------------------------------------
# update orders on the Delassus matrix (Sec. 2.1, Sec. 2.3)
# --------------------------------------------------------------------------

def _chain_between_walls():
    """Three touching disks between two walls, pushed together."""
    return make_packing(2, [[1.0, 0.0], [3.0, 0.0], [5.0, 0.0]],
                        [[0.4, 0.0], [0.0, 0.0], [-0.7, 0.0]], [1.0, 1.0, 1.0],
                        walls=[([1.0, 0.0], 0.0), ([-1.0, 0.0], -6.0)], lo=[0, -5], hi=[6, 5])


def _triangle_on_floor():
    """Two disks on a floor with a third resting on both, falling."""
    s3 = math.sqrt(3.0)
    return make_packing(2, [[0.0, 1.0], [2.0, 1.0], [1.0, 1.0 + s3]],
                        [[0.05, -0.3], [-0.1, -0.2], [0.02, -0.5]], [1.0, 1.0, 1.0],
                        walls=[([0.0, 1.0], 0.0)], gravity=1.0, lo=[-5, 0], hi=[7, 8])


def _delassus_sweeps(pk, out, parallel, sweeps):
    """Frictionless projected Gauss-Seidel / Jacobi on A_nn: contact c takes
    R_c <- max(0, R_c - (q_c + (A R)_c) / A_cc), q = g_e/dt + u0_n.  Flagged
    contacts use the forces at the start of the sweep and their new values
    are substituted at its end; the others run in slot order on the current
    forces, seeing the flagged ones at their start-of-sweep values."""
    A, u0, _, _, _ = pins.delassus_2d(pk, out["ci"], out["cj"], out["normal"], DT)
    Ann = A[0::2, 0::2]
    q = np.maximum(out["gap"], 0.0) / DT + u0[0::2]
    R = np.zeros(len(q))
    hist = []
    order = list(out["slot"])
    for _ in range(sweeps):
        start = R.copy()
        new_par = {}
        for c in order:
            if parallel[c]:
                new_par[c] = max(0.0, start[c] - (q[c] + Ann[c] @ start) / Ann[c, c])
        for c in order:
            if not parallel[c]:
                R[c] = max(0.0, R[c] - (q[c] + Ann[c] @ R) / Ann[c, c])
        for c, val in new_par.items():
            R[c] = val
        hist.append(R.copy())
    return hist


@pytest.mark.parametrize("case", [_chain_between_walls, _triangle_on_floor])
@pytest.mark.parametrize("mode", ["sequential", "jacobi", "mixed"])
def test_update_orders_equal_projected_iterations(oracle, case, mode):
    pk = case()
    out = solve_all(oracle, pk, mu=0.0, fixed=1, skin=1e-9)
    nc = len(out["ci"])
    assert nc >= 4
    if mode == "sequential":
        par = np.zeros(nc, np.uint8)
    elif mode == "jacobi":
        par = np.ones(nc, np.uint8)
    else:
        par = (np.arange(nc) % 2).astype(np.uint8)
    # the oracle's order with these flags (flagged contacts first: colour 0)
    color, slot, ds = oracle.order(pk.n, out["ci"], out["cj"], 1, np.zeros(nc, np.int32),
                                   parallel=par)
    want = _delassus_sweeps(pk, dict(out, slot=slot), par.astype(bool), 8)
    scale = max(np.abs(w).max() for w in want)
    for k in range(1, 9):
        params = oracle.make_params(2, pk.n_walls, mu=0.0, fixed_iters=k)
        R, info, _ = oracle.solve(params, pk, out["ci"], out["cj"], out["normal"], out["gap"], 1,
                                  ds, slot, parallel=par)
        np.testing.assert_allclose(R[0], want[k - 1], rtol=0, atol=1e-12 * scale)
        assert np.all(R[1] == 0.0)
    if mode == "jacobi":
        # the Jacobi iterates differ from Gauss-Seidel's after the first sweep
        gs = _delassus_sweeps(pk, dict(out, slot=slot), np.zeros(nc, bool), 2)
        assert np.abs(gs[1] - want[1]).max() > 1e-6 * scale


def _sphere_pair_on_floor():
    """Two spinning spheres on a floor, pressed together: contacts (A, B),
    (A, floor), (B, floor); the floor contacts follow the pair contact in the
    sweep and see its change of both spins."""
    h = math.sqrt(1.8 ** 2 - 0.2 ** 2)          # radii 1 and 0.8, both on the floor
    return make_packing(3, [[0.0, 0.0, 1.0], [0.6 * h, 0.8 * h, 0.8]],
                        [[0.3, 0.05, -0.2], [-0.25, -0.1, -0.1]], [1.0, 0.8],
                        w=np.array([[0.4, -1.0], [1.2, 0.3], [-0.5, 0.8]]),
                        walls=[([0.0, 0.0, 1.0], 0.0)], gravity=1.0)


def _law_3d(uc0, a_n, a_t, ge_dt, mu):
    """Contact force from the relative velocity without the contact's own
    force: closed if g_e/dt + u_n < 0, sticking force cancelling the slip,
    else radial return onto the cone at fixed R_n."""
    s = ge_dt + uc0[0]
    if s >= 0.0:
        return np.zeros(3)
    rn = -s / a_n
    T = -uc0[1:] / a_t
    tn = np.linalg.norm(T)
    if tn > mu * rn:
        T = T * (mu * rn / tn)
    return np.array([rn, T[0], T[1]])


@pytest.mark.parametrize("mu", [0.05, 0.3, 2.0])
def test_3d_sweeps_equal_delassus_gauss_seidel(oracle, mu):
    """The 3D sequential sweep with rotation equals Gauss-Seidel on the
    Delassus matrix of an independent 3D Jacobian (spins enter through
    rho x e), sweep by sweep; compared in body velocities, which do not
    depend on the tangent basis.  The block of each contact is diagonal with
    dt (w_n, w_t, w_t), w_t = w_n + sum r^2/I."""
    pk = _sphere_pair_on_floor()
    out = solve_all(oracle, pk, mu=mu, fixed=1, skin=1e-9)
    ci, cj = out["ci"], out["cj"]
    assert len(ci) == 3
    frames = pins.orthonormal_frames_3d(out["normal"])
    A, u0, J, minv, q0 = pins.delassus_3d(pk, ci, cj, frames, DT)
    for c in range(3):
        blk = A[3 * c:3 * c + 3, 3 * c:3 * c + 3]
        a, b = int(ci[c]), int(cj[c])
        wn = 1 / pk.m[a] + (1 / pk.m[b] if b < pk.n else 0.0)
        wt = wn + pk.r[a] ** 2 / pk.inertia[a] + (pk.r[b] ** 2 / pk.inertia[b] if b < pk.n else 0)
        np.testing.assert_allclose(blk, DT * np.diag([wn, wt, wt]), rtol=1e-14, atol=1e-18)
    ge = np.maximum(out["gap"], 0.0)
    R = np.zeros(9)
    order = list(out["slot"])
    for k in range(1, 5):
        for c in order:
            sl = slice(3 * c, 3 * c + 3)
            uc0 = u0[sl] + A[sl] @ R - A[sl, sl] @ R[sl]
            R[sl] = _law_3d(uc0, A[3 * c, 3 * c], A[3 * c + 1, 3 * c + 1], ge[c] / DT, mu)
        q = q0 + DT * minv * (J.T @ R)
        params = oracle.make_params(3, pk.n_walls, mu=mu, fixed_iters=k)
        Ro, info, _ = oracle.solve(params, pk, ci, cj, out["normal"], out["gap"], 1, out["ds"],
                                   out["slot"])
        V, W = oracle.velocities(pk, DT, ci, cj, out["normal"], Ro)
        scale = np.abs(q).max()
        for body in range(pk.n):
            np.testing.assert_allclose(V[:, body], q[6 * body:6 * body + 3], rtol=0,
                                       atol=1e-13 * scale)
            np.testing.assert_allclose(W[:, body], q[6 * body + 3:6 * body + 6], rtol=0,
                                       atol=1e-13 * scale)
        np.testing.assert_allclose(Ro[0], R[0::3], rtol=1e-12)
