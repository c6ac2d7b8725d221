"""Pins of the oracle's benchmark boundary conditions (Sec. 4.1, Fig. 10;
Sec. 4.4): a box periodic in x, confining walls of finite mass pushed with a
constant force (pressure-controlled walls) and walls sliding along
themselves (shear).

Expected values come from brute force over periodic images, closed forms
of small systems and an independent Delassus-matrix formulation in which a
wall of finite mass is one more generalized coordinate (its position along
its normal); none re-types the oracle's formulas."""
import math

import numpy as np
import pytest

from paper_1104_3516_amd import inputs
from tests.test_oracle_pins import make_packing

DT = 1e-3


def periodic(pk, mask=1, inv_mass=None, force=None):
    pk.periodic = mask
    if inv_mass is not None:
        pk.wall_inv_mass = np.asarray(inv_mass, dtype=np.float64)
        pk.wall_force = np.asarray(force, dtype=np.float64)
    return pk


def sim_of(oracle, pk, **kw):
    return oracle.Sim(oracle.make_params(pk.dim, pk.n_walls, **kw), pk)


# --------------------------------------------------------------------------
# periodic x: detection, geometry, wrap
# --------------------------------------------------------------------------

@pytest.mark.parametrize("skin", [1e-4, 0.2])
def test_periodic_detection_equals_brute_force_over_images(oracle, skin):
    pk = inputs.sheared_box_2d(20, 14, 71)
    L = pk.box_hi[0] - pk.box_lo[0]
    ci, cj = oracle.detect(pk, skin, use_cells=True)
    # brute force: every pair at the nearest of its images x + k L, k = -1, 0, 1
    x, r, n = pk.x, pk.r, pk.n
    want = []
    for i in range(n):
        for j in range(i + 1, n):
            g = min(math.hypot(x[0, j] + k * L - x[0, i], x[1, j] - x[1, i])
                    for k in (-1, 0, 1)) - r[i] - r[j]
            if g <= skin:
                want.append((i, j))
        for w in range(pk.n_walls):
            g = pk.wall_normal[w] @ x[:, i] - pk.wall_offset[w] - r[i]
            if g <= skin:
                want.append((i, n + w))
    assert list(zip(ci.tolist(), cj.tolist())) == want
    crossing = sum(1 for i, j in want if j < n and abs(x[0, j] - x[0, i]) > L / 2)
    assert crossing > 0        # some pairs touch across the periodic boundary
    np.testing.assert_array_equal(oracle.detect(pk, skin, use_cells=False)[0], ci)


def test_periodic_geometry_across_the_boundary(oracle):
    """Disks at x = 0.5 and x = L - 1.25 touch across x = 0: the normal from
    the first to the second points along -x, the gap is the image distance
    minus the radii, and the mid-gap position is taken back into [0, L)."""
    L = 10.0
    pk = periodic(make_packing(2, [[0.5, 3.0], [L - 1.25, 3.0]], [[0, 0], [0, 0]], [0.8, 0.9],
                               lo=[0.0, 0.0], hi=[L, 6.0]))
    ci, cj = oracle.detect(pk, 0.1, use_cells=False)
    assert list(ci) == [0] and list(cj) == [1]
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    np.testing.assert_allclose(normal[:, 0], [-1.0, 0.0], atol=1e-15)
    assert gap[0] == pytest.approx(1.75 - 1.7, abs=1e-14)
    # mid-gap: 0.5 - (0.8 + 0.025) = -0.325 -> L - 0.325
    assert xmid[0, 0] == pytest.approx(L - 0.325, abs=1e-14) and xmid[1, 0] == 3.0


def test_periodic_cells_need_three_along_the_axis(oracle):
    pk = periodic(make_packing(2, [[0.5, 1.0], [2.5, 1.0]], [[0, 0], [0, 0]], [1.0, 1.0],
                               lo=[0.0, 0.0], hi=[4.0, 8.0]))
    with pytest.raises(RuntimeError):
        oracle.detect(pk, 0.1, use_cells=True)


def test_particle_leaving_the_box_reenters(oracle):
    L = 12.0
    pk = periodic(make_packing(2, [[L - 0.001, 3.0], [5.0, 3.0]], [[2.0, 0.0], [-1.5, 0.0]],
                               [1.0, 1.0], lo=[0.0, 0.0], hi=[L, 6.0]))
    sim = sim_of(oracle, pk, fixed_iters=1)
    sim.step()
    x = sim.state()[0]
    assert x[0, 0] == pytest.approx(0.001, abs=1e-12)
    assert x[0, 1] == pytest.approx(5.0 - 1.5e-3, abs=1e-12)


# --------------------------------------------------------------------------
# walls of finite mass under a constant force
# --------------------------------------------------------------------------

def _column_under_wall(k, F, M, U=0.0, gravity=0.0):
    """k touching unit disks stacked on a fixed floor (y = 0), a wall of mass
    M on top (normal -y) pushed down with F, moving down at U."""
    x = [[0.0, 1.0 + 2.0 * q] for q in range(k)]
    top = 2.0 * k
    walls = [([0.0, 1.0], 0.0), ([0.0, -1.0], -top, np.array([0.0, -U]))]
    pk = make_packing(2, x, [[0.0, 0.0]] * k, [1.0] * k, walls=walls, gravity=gravity,
                      lo=[-3.0, 0.0], hi=[3.0, top])
    pk.wall_inv_mass = np.array([0.0, 1.0 / M])
    pk.wall_force = np.array([0.0, F])
    return pk


@pytest.mark.parametrize("k", [1, 4])
def test_static_pressure_wall_is_balanced(oracle, k):
    """At rest, the wall's force F runs through the column: every contact
    carries F, the wall's reaction equals F and it stays at rest."""
    F, M = 0.25 * 6.0, 17.0
    pk = _column_under_wall(k, F, M)
    sim = sim_of(oracle, pk, fixed_iters=20000, mu=0.3)
    sim.step()
    c = sim.contacts()
    assert len(c["ci"]) == k + 1
    np.testing.assert_allclose(c["R"][0], F, rtol=1e-12)
    np.testing.assert_allclose(c["R"][1], 0.0, atol=1e-12 * F)
    U = sim.wall_velocities()
    assert abs(U[1, 1]) < 1e-14 and U[1, 0] == 0.0
    # the wall's reaction is the sum of its contacts' normal forces
    top = c["cj"] == pk.n + 1
    assert c["R"][0, top].sum() == pytest.approx(F, rel=1e-12)
    # and the oracle's wall velocity function agrees with the bookkeeping
    Uf = oracle.wall_velocities(pk, DT, c["cj"], c["R"])
    np.testing.assert_array_equal(Uf, U)


def test_moving_pressure_wall_is_stopped(oracle):
    """A wall of mass M coming down at U onto a disk that rests on a fixed
    floor stops within the step: its contact force is F + M U / dt and the
    floor carries the same (no gravity)."""
    F, M, U = 2.0, 5.0, 0.03
    pk = _column_under_wall(1, F, M, U=U)
    sim = sim_of(oracle, pk, fixed_iters=20000, mu=0.3)
    sim.step()
    c = sim.contacts()
    want = F + M * U / DT
    np.testing.assert_allclose(c["R"][0], want, rtol=1e-9)
    assert abs(sim.wall_velocities()[1, 1]) < 1e-9 * U
    # the wall moved by dt u_n of the step's final velocity
    wo = sim.state()[3]
    assert wo[1] == pytest.approx(-2.0, abs=1e-12)


def test_free_wall_accelerates_under_its_force(oracle):
    """Without contacts a wall of mass M under F gains F dt / M along its
    normal per step and moves by dt times that velocity."""
    F, M = 3.0, 6.0
    pk = make_packing(2, [[0.0, 1.0]], [[0.0, 0.0]], [1.0],
                      walls=[([0.0, 1.0], 0.0), ([0.0, -1.0], -20.0, np.array([0.4, 0.0]))],
                      lo=[-5.0, 0.0], hi=[5.0, 20.0])
    pk.wall_inv_mass = np.array([0.0, 1.0 / M])
    pk.wall_force = np.array([0.0, F])
    sim = sim_of(oracle, pk, fixed_iters=2)
    steps = 5
    for _ in range(steps):
        sim.step()
    U = sim.wall_velocities()
    # normal -y: the wall moves down at steps F dt / M, its x velocity stays
    assert U[1, 1] == pytest.approx(-steps * F * DT / M, rel=1e-12)
    assert U[1, 0] == 0.4
    wo = sim.state()[3]
    expect = -20.0 + sum(k * F * DT / M * DT for k in range(1, steps + 1))
    assert wo[1] == pytest.approx(expect, rel=1e-12)
    lo, hi = sim.box()
    assert hi[1] == pytest.approx(-expect, rel=1e-12)


# --------------------------------------------------------------------------
# independent formulation: Delassus matrix with the wall as a coordinate
# --------------------------------------------------------------------------

def _delassus_with_walls(pk, ci, cj, normal, dt):
    """Generalized coordinates: (vx, vy, w) per disk, then the normal speed
    u_n of each wall of finite mass (position along its normal nu).  Contact
    rows (u_n, u_t) of the relative velocity of the contact points; a wall
    contributes u_n nu + its prescribed tangential velocity."""
    N = pk.n
    mob = [w for w in range(pk.n_walls) if pk.wall_inv_mass[w] != 0.0]
    col = {w: 3 * N + q for q, w in enumerate(mob)}
    nq = 3 * N + len(mob)
    nc = len(ci)
    J = np.zeros((2 * nc, nq))
    u_presc = np.zeros(2 * nc)
    z = np.array([0.0, 0.0, 1.0])
    for c in range(nc):
        a, b = int(ci[c]), int(cj[c])
        n = np.array([normal[0, c], normal[1, c], 0.0])
        t = np.cross(z, n)
        for row, e in ((2 * c, n), (2 * c + 1, t)):
            J[row, 3 * a:3 * a + 2] -= e[:2]
            J[row, 3 * a + 2] -= np.cross(z, pk.r[a] * n) @ e
            if b < N:
                J[row, 3 * b:3 * b + 2] += e[:2]
                J[row, 3 * b + 2] += np.cross(z, -pk.r[b] * n) @ e
            else:
                w = b - N
                nu = np.array([pk.wall_normal[w][0], pk.wall_normal[w][1], 0.0])
                u = np.array([pk.wall_velocity[w][0], pk.wall_velocity[w][1], 0.0])
                if w in col:
                    J[row, col[w]] += nu @ e
                    u_presc[row] += (u - (u @ nu) * nu) @ e     # tangential part prescribed
                else:
                    u_presc[row] += u @ e
    minv = np.zeros(nq)
    minv[0:3 * N:3] = 1.0 / pk.m
    minv[1:3 * N:3] = 1.0 / pk.m
    minv[2:3 * N:3] = 1.0 / pk.inertia
    q0 = np.zeros(nq)
    q0[0:3 * N:3] = pk.v[0] + dt * pk.f[0] / pk.m
    q0[1:3 * N:3] = pk.v[1] + dt * pk.f[1] / pk.m
    q0[2:3 * N:3] = pk.w[0] + dt * pk.t[0] / pk.inertia
    for w, k in col.items():
        minv[k] = pk.wall_inv_mass[w]
        u_n = pk.wall_velocity[w] @ pk.wall_normal[w]
        q0[k] = u_n + dt * pk.wall_inv_mass[w] * pk.wall_force[w]
    A = dt * (J * minv) @ J.T
    return A, J @ q0 + u_presc, J, minv, q0


def _law_2d(uc0, a_n, a_t, ge_dt, mu):
    s = ge_dt + uc0[0]
    if s >= 0.0:
        return np.zeros(2)
    rn = -s / a_n
    T = -uc0[1] / a_t
    return np.array([rn, max(-mu * rn, min(mu * rn, T))])


def _sheared_stack():
    """Three disks on a fixed floor sliding at -0.002, two more resting on
    them, and a top wall of finite mass on those two, pushed down and sliding
    at +0.003: the wall carries two contacts."""
    s3 = math.sqrt(3.0)
    x = [[0.0, 1.0], [2.0, 1.0], [4.0, 1.0], [1.0, 1.0 + s3], [3.0, 1.0 + s3]]
    top = 2.0 + s3
    walls = [([0.0, 1.0], 0.0, np.array([-0.002, 0.0])),
             ([0.0, -1.0], -top, np.array([0.003, -0.05]))]
    pk = make_packing(2, x, [[0.02, 0.01], [-0.03, 0.0], [0.01, 0.02], [0.01, -0.04],
                             [-0.02, -0.01]], [1.0] * 5,
                      w=[[0.1, -0.2, 0.05, 0.0, 0.03]], walls=walls, gravity=0.5,
                      lo=[-4.0, 0.0], hi=[8.0, top])
    pk.wall_inv_mass = np.array([0.0, 1.0 / 4.0])
    pk.wall_force = np.array([0.0, 3.0])
    return pk


@pytest.mark.parametrize("mu", [0.05, 0.4])
@pytest.mark.parametrize("domains", [None, "alternate", "halves"])
def test_sweeps_with_a_wall_of_finite_mass_equal_delassus(oracle, mu, domains):
    """Sequential sweeps (and the domain-wise sweep: Jacobi across domains,
    Gauss-Seidel inside, the wall a body shared by both) equal the same
    iteration written on the Delassus matrix in which the wall's normal speed
    is a coordinate of inverse mass 1/M; compared sweep by sweep in the body
    and wall velocities."""
    pk = _sheared_stack()
    ci, cj = oracle.detect(pk, 1e-9, use_cells=False)
    nc = len(ci)
    assert int((cj == pk.n + 1).sum()) == 2
    normal, gap, xmid = oracle.geometry(pk, ci, cj)
    if domains is None:
        dom = np.zeros(nc, np.int32)
    elif domains == "alternate":
        dom = (np.arange(nc) % 2).astype(np.int32)
    else:
        dom = (np.arange(nc) >= nc // 2).astype(np.int32)
    P = int(dom.max()) + 1
    color, slot, ds = oracle.order(pk.n, ci, cj, P, dom)
    A, u0, J, minv, q0 = _delassus_with_walls(pk, ci, cj, normal, DT)
    ge = np.maximum(gap, 0.0)
    R = np.zeros(2 * nc)
    for k in range(1, 7):
        Rprev = R.copy()
        new = Rprev.copy()
        for d in range(P):
            Rd = Rprev.copy()            # the domain sees foreign contacts frozen
            for c in slot[ds[d]:ds[d + 1]]:
                sl = slice(2 * c, 2 * c + 2)
                uc0 = u0[sl] + A[sl] @ Rd - A[sl, sl] @ Rd[sl]
                Rd[sl] = _law_2d(uc0, A[2 * c, 2 * c], A[2 * c + 1, 2 * c + 1], ge[c] / DT, mu)
                new[sl] = Rd[sl]
        R = new
        params = oracle.make_params(2, pk.n_walls, mu=mu, fixed_iters=k, n_domains=P)
        Ro, info, _ = oracle.solve(params, pk, ci, cj, normal, gap, P, ds, slot)
        np.testing.assert_allclose(Ro[0], R[0::2], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Ro[1], R[1::2], rtol=1e-12, atol=1e-12)
        q = q0 + DT * minv * (J.T @ R)
        V, W = oracle.velocities(pk, DT, ci, cj, normal, Ro)
        N3 = 3 * pk.n
        np.testing.assert_allclose(V, np.stack([q[0:N3:3], q[1:N3:3]]), rtol=0, atol=1e-13)
        U = oracle.wall_velocities(pk, DT, cj, Ro)
        assert U[1, 1] == pytest.approx(-q[N3], rel=1e-12)        # u_n along nu = -y
        assert U[1, 0] == 0.003 and U[0, 0] == -0.002


def test_shear_drives_the_packing_and_conserves_momentum(oracle):
    """A sheared periodic box: the x momentum gained by the particles in a
    step equals dt times the tangential forces of the walls on them, and the
    walls drag the rows next to them in their own direction."""
    pk = inputs.sheared_box_2d(16, 10, 72, pressure=0.25, shear_velocity=0.02)
    sim = sim_of(oracle, pk, mu=0.5, max_iter=3000, n_domains=4, repartition_every=5)
    for _ in range(3):
        v0 = sim.state()[1].copy()
        sim.step()
        c = sim.contacts()
        x, v, w, wo = sim.state()
        n = c["normal"]
        t = np.stack([-n[1], n[0]])
        world = c["R"][0] * n + c["R"][1] * t           # force on body 2 (the wall)
        wall = c["cj"] >= pk.n
        lhs = (pk.m * (v - v0)).sum(axis=1)
        rhs = -DT * world[:, wall].sum(axis=1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-12)
    top = x[1] > np.median(x[1])
    assert v[0, top].mean() > 0 > v[0, ~top].mean()
    assert np.all((x[0] >= pk.box_lo[0]) & (x[0] < pk.box_hi[0]))
