"""Independent rigid-body formulation of the one-step contact problem.

Used only to pin the oracle.  It shares nothing with the oracle's code: the
contact problem of Sec. 2.1 is written here in generalized coordinates,
u = J V with V = v + dt M^-1 (F + J^T R), so that the post-step relative
contact velocity is u = u0 + A R with the Delassus matrix A = dt J M^-1 J^T.
Kinematics are built from 3D cross products (2D embedded in the xy plane).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg
import scipy.optimize


def contact_frames_2d(normal: np.ndarray):
    """t = z x n for every contact (2D)."""
    n = normal.T
    t = np.stack([-n[:, 1], n[:, 0]], axis=1)
    return n, t


def jacobian_2d(pk, ci, cj, normal):
    """J maps generalized velocities q = (vx_0, vy_0, w_0, vx_1, ...) to the
    contact-frame relative velocities (u_n0, u_t0, u_n1, u_t1, ...)."""
    N = pk.n
    nc = len(ci)
    J = np.zeros((2 * nc, 3 * N))
    n, t = contact_frames_2d(normal)
    z = np.array([0.0, 0.0, 1.0])
    for c in range(nc):
        a, b = int(ci[c]), int(cj[c])
        n3 = np.array([n[c, 0], n[c, 1], 0.0])
        t3 = np.array([t[c, 0], t[c, 1], 0.0])
        for row, e in ((2 * c, n3), (2 * c + 1, t3)):
            # body 1 contact point velocity: V_a + w_a z x (r_a n); enters with -
            lever_a = pk.r[a] * n3
            J[row, 3 * a + 0] -= e[0]
            J[row, 3 * a + 1] -= e[1]
            J[row, 3 * a + 2] -= np.dot(np.cross(z, lever_a), e)
            if b < N:
                lever_b = -pk.r[b] * n3
                J[row, 3 * b + 0] += e[0]
                J[row, 3 * b + 1] += e[1]
                J[row, 3 * b + 2] += np.dot(np.cross(z, lever_b), e)
    return J


def wall_velocity_terms_2d(pk, ci, cj, normal):
    """Contribution of moving walls to the relative velocities."""
    N = pk.n
    nc = len(ci)
    n, t = contact_frames_2d(normal)
    u = np.zeros(2 * nc)
    for c in range(nc):
        b = int(cj[c])
        if b >= N:
            uw = pk.wall_velocity[b - N]
            u[2 * c] = uw @ n[c]
            u[2 * c + 1] = uw @ t[c]
    return u


def delassus_2d(pk, ci, cj, normal, dt):
    N = pk.n
    J = jacobian_2d(pk, ci, cj, normal)
    minv = np.zeros(3 * N)
    minv[0::3] = 1.0 / pk.m
    minv[1::3] = 1.0 / pk.m
    minv[2::3] = 1.0 / pk.inertia
    q0 = np.zeros(3 * N)
    q0[0::3] = pk.v[0] + dt * pk.f[0] / pk.m
    q0[1::3] = pk.v[1] + dt * pk.f[1] / pk.m
    q0[2::3] = pk.w[0] + dt * pk.t[0] / pk.inertia
    u0 = J @ q0 + wall_velocity_terms_2d(pk, ci, cj, normal)
    A = dt * (J * minv) @ J.T
    return A, u0, J, minv, q0


def enumerate_states_2d(pk, ci, cj, normal, gap, dt, mu, tol=1e-9):
    """All solutions of the one-step frictional contact problem, found by
    trying every assignment of open / stick / slide+ / slide- to the
    contacts.  Returns a list of force arrays (2 x nc) in the contact frame."""
    A, u0, _, _, _ = delassus_2d(pk, ci, cj, normal, dt)
    nc = len(ci)
    ge = np.maximum(gap, 0.0)
    sols = []
    for states in itertools.product(range(4), repeat=nc):
        M = np.zeros((2 * nc, 2 * nc))
        rhs = np.zeros(2 * nc)
        for c, s in enumerate(states):
            rn, rt = 2 * c, 2 * c + 1
            if s == 0:          # open: R = 0
                M[rn, rn] = 1.0
                M[rt, rt] = 1.0
                continue
            # closed: ge/dt + u_n = 0
            M[rn] = A[rn]
            rhs[rn] = -(ge[c] / dt + u0[rn])
            if s == 1:          # stick: u_t = 0
                M[rt] = A[rt]
                rhs[rt] = -u0[rt]
            elif s == 2:        # slide with R_t = +mu R_n
                M[rt, rt] = 1.0
                M[rt, rn] = -mu
            else:               # slide with R_t = -mu R_n
                M[rt, rt] = 1.0
                M[rt, rn] = mu
        try:
            x = np.linalg.solve(M, rhs)
        except np.linalg.LinAlgError:
            continue
        if not np.allclose(M @ x, rhs, rtol=0, atol=1e-9 * (1 + np.abs(rhs).max())):
            continue
        u = u0 + A @ x
        scale = 1.0 + np.abs(x).max()
        vscale = 1.0 + np.abs(u).max() + np.abs(ge / dt).max()
        ok = True
        for c, s in enumerate(states):
            Rn, Rt = x[2 * c], x[2 * c + 1]
            un, ut = u[2 * c], u[2 * c + 1]
            if s == 0:
                ok &= ge[c] / dt + un >= -tol * vscale
            else:
                ok &= Rn >= -tol * scale
                if s == 1:
                    ok &= abs(Rt) <= mu * Rn + tol * scale
                elif s == 2:
                    ok &= ut <= tol * vscale
                else:
                    ok &= ut >= -tol * vscale
        if ok:
            sols.append(np.stack([x[0::2], x[1::2]]))
    return sols


def consistent_states_2d(pk, ci, cj, normal, gap, dt, mu, R, tol=1e-9):
    """Assignments of open / stick / slide+ / slide- under which the contact
    forces R (2 x nc, contact frame) satisfy every equation and inequality of
    the one-step problem.  Unlike enumerate_states_2d this also accepts
    forces of statically indeterminate systems, where a state's equations
    have a family of solutions."""
    A, u0, _, _, _ = delassus_2d(pk, ci, cj, normal, dt)
    nc = len(ci)
    ge = np.maximum(gap, 0.0)
    x = np.empty(2 * nc)
    x[0::2], x[1::2] = R[0], R[1]
    u = u0 + A @ x
    scale = 1.0 + np.abs(x).max()
    vscale = 1.0 + np.abs(u0).max() + np.abs(ge / dt).max()
    accepted = []
    for states in itertools.product(range(4), repeat=nc):
        ok = True
        for c, s in enumerate(states):
            Rn, Rt = x[2 * c], x[2 * c + 1]
            pred, ut = ge[c] / dt + u[2 * c], u[2 * c + 1]
            if s == 0:
                ok &= abs(Rn) <= tol * scale and abs(Rt) <= tol * scale and pred >= -tol * vscale
            else:
                ok &= abs(pred) <= tol * vscale and Rn >= -tol * scale
                if s == 1:
                    ok &= abs(ut) <= tol * vscale and abs(Rt) <= mu * Rn + tol * scale
                elif s == 2:
                    ok &= abs(Rt - mu * Rn) <= tol * scale and ut <= tol * vscale
                else:
                    ok &= abs(Rt + mu * Rn) <= tol * scale and ut >= -tol * vscale
            if not ok:
                break
        if ok:
            accepted.append(states)
    return accepted


def frictionless_lcp_2d(pk, ci, cj, normal, gap, dt):
    """mu = 0: the normal forces solve the LCP  w = q + A_nn R_n >= 0,
    R_n >= 0, R_n . w = 0 with q = g_e/dt + u0_n.  With A_nn symmetric
    positive definite this is min 1/2 R A R + q R over R >= 0, solved as a
    non-negative least-squares problem through the Cholesky factor."""
    A, u0, _, _, _ = delassus_2d(pk, ci, cj, normal, dt)
    Ann = A[0::2, 0::2]
    q = np.maximum(gap, 0.0) / dt + u0[0::2]
    L = scipy.linalg.cholesky(Ann, lower=True)
    # 1/2 R^T L L^T R + q^T R = 1/2 |L^T R + L^-1 q|^2 + const
    b = -scipy.linalg.solve_triangular(L, q, lower=True)
    Rn, _ = scipy.optimize.nnls(L.T, b, maxiter=100 * len(q))
    return Rn


def orthonormal_frames_3d(normal: np.ndarray):
    """A right-handed orthonormal frame (n, t1, t2) per contact by
    Gram-Schmidt from the coordinate axis least aligned with n (any
    tangent basis serves: the force law is isotropic in the tangent plane)."""
    n = normal.T
    frames = []
    for c in range(n.shape[0]):
        e = np.zeros(3)
        e[np.argmin(np.abs(n[c]))] = 1.0
        t1 = e - (e @ n[c]) * n[c]
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(n[c], t1)
        frames.append((n[c].copy(), t1, t2))
    return frames


def delassus_3d(pk, ci, cj, frames, dt):
    """3D analogue of delassus_2d: generalized velocities per body
    (vx, vy, vz, wx, wy, wz); contact rows (u_n, u_t1, u_t2) of the relative
    velocity of the contact points, body 2 minus body 1, with lever arms
    r_a n on body 1 and -r_b n on body 2: (W x rho) . e = W . (rho x e)."""
    N = pk.n
    nc = len(ci)
    J = np.zeros((3 * nc, 6 * N))
    uw = np.zeros(3 * nc)
    for c in range(nc):
        a, b = int(ci[c]), int(cj[c])
        n = frames[c][0]
        for k, e in enumerate(frames[c]):
            row = 3 * c + k
            J[row, 6 * a:6 * a + 3] -= e
            J[row, 6 * a + 3:6 * a + 6] -= np.cross(pk.r[a] * n, e)
            if b < N:
                J[row, 6 * b:6 * b + 3] += e
                J[row, 6 * b + 3:6 * b + 6] += np.cross(-pk.r[b] * n, e)
            else:
                uw[row] = pk.wall_velocity[b - N] @ e
    minv = np.zeros(6 * N)
    for k in range(3):
        minv[k::6] = 1.0 / pk.m
        minv[3 + k::6] = 1.0 / pk.inertia
    q0 = np.zeros(6 * N)
    for k in range(3):
        q0[k::6] = pk.v[k] + dt * pk.f[k] / pk.m
        q0[3 + k::6] = pk.w[k] + dt * pk.t[k] / pk.inertia
    A = dt * (J * minv) @ J.T
    return A, J @ q0 + uw, J, minv, q0
