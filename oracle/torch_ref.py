"""FP64 PyTorch (CPU) reference of a fixed-count domain-wise force solve in
2D, differentiable with autograd.

TEST INFRASTRUCTURE ONLY: it checks the gradients of the HIP library's
adjoint (cd_adjoint).  It shares no code with the HIP library; the contact
list, bisection tree and colouring come from the C oracle (cdref).

What it computes, for one time step from the given velocities (Sec. 2.1
and 3.1):
  * per contact (Sec. 2.1, Fig. 1): normal n, tangent t = (-n_y, n_x),
    gap clamped at zero, inverse-mass terms w_n = 1/m_1 + 1/m_2 and
    w_t = w_n + r_1^2/I_1 + r_2^2/I_2 (walls contribute nothing);
  * per sweep: every particle's velocity recomputed from its base velocity,
    external force and all contact forces of the previous sweep (the
    exchange); every domain takes its own copy for the particles it touches;
    colour by colour (all domains at once, the colours of one domain in
    order) each contact solves the single-contact law (Eqs. 3-9) with the
    current velocities of its bodies in its domain's copy, and the change of
    its force is applied to those copies;
  * after K sweeps: the forces.
The colour batches make autograd see exactly the sequential order of the
domain-wise sweep.  Branches (open / stick / slide) are selected with
torch.where, so gradients follow the branch each contact takes.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from oracle import cdref


@dataclasses.dataclass
class Problem:
    n: int
    ci: np.ndarray
    cj: np.ndarray
    normal: np.ndarray
    gap: np.ndarray
    dom: np.ndarray
    color: np.ndarray
    slot: np.ndarray
    dom_start: np.ndarray
    P: int
    dt: float


def setup(pk, P: int, skin: float, dt: float = 1e-3) -> Problem:
    """Contact list (gap <= skin), tree and colouring from the C oracle."""
    ci, cj = cdref.detect(pk, skin)
    normal, gap, xmid = cdref.geometry(pk, ci, cj)
    _, dom = cdref.orb(pk.dim, P, pk.box_lo, pk.box_hi, xmid)
    color, slot, dom_start = cdref.order(pk.n, ci, cj, P, dom)
    return Problem(pk.n, ci, cj, normal, gap, dom, color, slot, dom_start, P, dt)


class _Setup:
    """Per-contact and per-particle constants, entries and colour batches."""

    def __init__(self, pb: Problem, pk):
        f64 = torch.float64
        N, nc, dt = pb.n, len(pb.ci), pb.dt
        ci, cj = pb.ci.astype(np.int64), pb.cj.astype(np.int64)
        wall = cj >= N
        jj = np.where(wall, 0, cj)
        m, r, I = pk.m, pk.r, pk.inertia
        # per-contact constants, in the oracle's order of operations
        inv_m, inv_I = 1.0 / m, 1.0 / I
        wn = inv_m[ci] + np.where(wall, 0.0, inv_m[jj])
        wt = wn + (r[ci] * r[ci]) * inv_I[ci]
        wt = wt + np.where(wall, 0.0, (r[jj] * r[jj]) * inv_I[jj])
        dwn, dwt = dt * wn, dt * wt
        T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=f64)
        self.N, self.nc, self.dt = N, nc, dt
        self.ci, self.cj, self.jj, self.wall = ci, cj, jj, wall
        self.dwn, self.dwt = T(dwn), T(dwt)
        self.kn, self.kt = T(1.0 / dwn), T(1.0 / dwt)
        self.dtim, self.dtii = T(dt * inv_m), T(dt * inv_I)
        rt = T(r)
        self.rt = rt
        self.walln = torch.as_tensor(wall)
        self.ra = rt[ci]
        self.rb = torch.where(self.walln, torch.zeros(nc, dtype=f64), rt[jj])
        self.dma, self.dia = self.dtim[ci], self.dtii[ci]
        self.dmb = torch.where(self.walln, torch.zeros(nc, dtype=f64), self.dtim[jj])
        self.dib = torch.where(self.walln, torch.zeros(nc, dtype=f64), self.dtii[jj])
        wall_u = np.zeros((2, nc))
        wid = np.where(wall, cj - N, 0)
        wall_u[:, wall] = pk.wall_velocity[wid[wall]].T
        self.uw0, self.uw1 = T(wall_u[0]), T(wall_u[1])
        self.fext, self.text = T(pk.f), T(pk.t)
        # entries: (domain, particle) pairs touched by the domain's contacts
        keys = {}
        ea = np.empty(nc, np.int64)
        eb = np.full(nc, -1, np.int64)
        ent_p = []
        for c in range(nc):
            d = int(pb.dom[c])
            for side, p in ((0, ci[c]), (1, cj[c])):
                if p >= N:
                    continue
                k = (d, int(p))
                if k not in keys:
                    keys[k] = len(ent_p)
                    ent_p.append(int(p))
                if side == 0:
                    ea[c] = keys[k]
                else:
                    eb[c] = keys[k]
        self.ea, self.eb = ea, eb
        self.ent_p = torch.as_tensor(np.array(ent_p, np.int64))
        self.colors = [np.nonzero(pb.color == k)[0]
                       for k in range(int(pb.color.max()) + 1 if nc else 0)]
        self.cit, self.cjt = torch.as_tensor(ci), torch.as_tensor(jj)
        self.nw = torch.as_tensor(~wall)
        # walls: unit normal into the box and offset
        self.wnu = T(pk.wall_normal)
        self.woff = T(pk.wall_offset)


def _exchange(S: _Setup, n0, n1, Rn, Rt, v, w):
    """Every particle's velocity from its base velocity, external force and
    all contact forces (Eq. 1): V = v + dt/m (f + sum of +-F), W = w + dt/I
    (t - sum r R_t), with F = R_n n + R_t t on body 2 and -F on body 1."""
    F0 = Rn * n0 + Rt * (-n1)
    F1 = Rn * n1 + Rt * n0
    nw = S.nw
    acc0 = S.fext[0].index_add(0, S.cit, -F0).index_add(0, S.cjt[nw], F0[nw])
    acc1 = S.fext[1].index_add(0, S.cit, -F1).index_add(0, S.cjt[nw], F1[nw])
    tacc = S.text[0].index_add(0, S.cit, -(Rt * S.ra)).index_add(0, S.cjt[nw], -(Rt * S.rb)[nw])
    return v[0] + S.dtim * acc0, v[1] + S.dtim * acc1, w[0] + S.dtii * tacc


def _solve(S: _Setup, n0, n1, gdt, mu, v, w, Rn, Rt, sweeps: int):
    f64 = torch.float64
    nc = S.nc
    for _ in range(sweeps):
        V0, V1, W = _exchange(S, n0, n1, Rn, Rt, v, w)
        E0, E1, EW = V0[S.ent_p], V1[S.ent_p], W[S.ent_p]
        Rn_new = torch.zeros(nc, dtype=f64)
        Rt_new = torch.zeros(nc, dtype=f64)
        for idx_np in S.colors:
            idx = torch.as_tensor(idx_np)
            a_e = torch.as_tensor(S.ea[idx_np])
            wl = torch.as_tensor(S.eb[idx_np] < 0)
            b_e = torch.as_tensor(np.where(S.eb[idx_np] < 0, 0, S.eb[idx_np]))
            Va0, Va1, Wa = E0[a_e], E1[a_e], EW[a_e]
            Vb0 = torch.where(wl, S.uw0[idx], E0[b_e])
            Vb1 = torch.where(wl, S.uw1[idx], E1[b_e])
            Wb = torch.where(wl, torch.zeros_like(Wa), EW[b_e])
            nn0, nn1 = n0[idx], n1[idx]
            tt0, tt1 = -nn1, nn0
            ra, rb = S.ra[idx], S.rb[idx]
            dV0, dV1 = Vb0 - Va0, Vb1 - Va1
            vn = dV0 * nn0 + dV1 * nn1
            vt = (dV0 * tt0 + dV1 * tt1) - (ra * Wa + rb * Wb)
            un = vn - S.dwn[idx] * Rn[idx]
            ut = vt - S.dwt[idx] * Rt[idx]
            s = gdt[idx] + un
            rn = -s * S.kn[idx]
            Tt = -ut * S.kt[idx]
            lim = mu[idx] * rn
            opn = s >= 0.0
            stick = torch.abs(Tt) <= lim
            rn_c = torch.where(opn, torch.zeros_like(rn), rn)
            rt_c = torch.where(opn, torch.zeros_like(rn),
                               torch.where(stick, Tt, torch.where(Tt > 0.0, lim, -lim)))
            dRn, dRt = rn_c - Rn[idx], rt_c - Rt[idx]
            dF0 = dRn * nn0 + dRt * tt0
            dF1 = dRn * nn1 + dRt * tt1
            E0 = E0.index_put((a_e,), Va0 - S.dma[idx] * dF0)
            E1 = E1.index_put((a_e,), Va1 - S.dma[idx] * dF1)
            EW = EW.index_put((a_e,), Wa - S.dia[idx] * (ra * dRt))
            keep = ~wl
            if bool(keep.any()):
                bk = b_e[keep]
                E0 = E0.index_put((bk,), (Vb0 + S.dmb[idx] * dF0)[keep])
                E1 = E1.index_put((bk,), (Vb1 + S.dmb[idx] * dF1)[keep])
                EW = EW.index_put((bk,), (Wb - S.dib[idx] * (rb * dRt))[keep])
            Rn_new = Rn_new.index_put((idx,), rn_c)
            Rt_new = Rt_new.index_put((idx,), rt_c)
        Rn, Rt = Rn_new, Rt_new
    return Rn, Rt


def forces(pb: Problem, pk, mu, v, w, sweeps: int, R0=None):
    """Forces (2 x n_c, frame components (R_n, R_t)) after `sweeps` sweeps
    from R0 (default zero), at the packing's positions.  mu: (n_c,),
    v: (2, N), w: (1, N) tensors."""
    S = _Setup(pb, pk)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
    n0, n1 = T(pb.normal[0]), T(pb.normal[1])
    gdt = T(np.maximum(pb.gap, 0.0) / pb.dt)
    Rn = torch.zeros(S.nc, dtype=torch.float64) if R0 is None else T(R0[0])
    Rt = torch.zeros(S.nc, dtype=torch.float64) if R0 is None else T(R0[1])
    Rn, Rt = _solve(S, n0, n1, gdt, mu, v, w, Rn, Rt, sweeps)
    return torch.stack([Rn, Rt])


def geometry(S: _Setup, x):
    """Normal and gap of every listed contact at positions x (2, N), as a
    differentiable function of x (Sec. 2.1, Fig. 1): particle pairs
    n = d/|d|, g = |d| - r_i - r_j with d = x_j - x_i; walls n = -nu,
    g = nu.x_i - o - r_i."""
    ci, jj, wall = S.cit, S.cjt, S.walln
    d0 = x[0][jj] - x[0][ci]
    d1 = x[1][jj] - x[1][ci]
    # wall rows pair a particle with itself here: keep their (unused) branch
    # finite so that its zero gradient does not turn into NaN
    d0 = torch.where(wall, torch.ones_like(d0), d0)
    dist = torch.sqrt(d0 * d0 + d1 * d1)
    wid = torch.as_tensor(np.where(S.wall, S.cj - S.N, 0))
    nu0, nu1 = S.wnu[wid, 0], S.wnu[wid, 1]
    proj = nu0 * x[0][ci] + nu1 * x[1][ci]
    n0 = torch.where(wall, -nu0, d0 / dist)
    n1 = torch.where(wall, -nu1, d1 / dist)
    g = torch.where(wall, (proj - S.woff[wid]) - S.rt[ci], (dist - S.rt[ci]) - S.rb)
    return n0, n1, g


def forces_steps(pb: Problem, pk, mu, v, w, steps: int, sweeps: int):
    """Forces after the last of `steps` time steps with the contact list,
    tree and colours of the first kept (frozen) for all of them: each step
    recomputes the geometry at the current positions, starts from the
    previous step's forces, runs `sweeps` sweeps and moves the particles
    (Eqs. 1-2: v <- V(R), x <- x + dt v).  Walls must not move."""
    S = _Setup(pb, pk)
    x = torch.as_tensor(pk.x, dtype=torch.float64)
    Rn = torch.zeros(S.nc, dtype=torch.float64)
    Rt = torch.zeros(S.nc, dtype=torch.float64)
    for t in range(steps):
        n0, n1, g = geometry(S, x)
        gdt = torch.clamp(g, min=0.0) / S.dt
        Rn, Rt = _solve(S, n0, n1, gdt, mu, v, w, Rn, Rt, sweeps)
        if t + 1 < steps:
            V0, V1, W = _exchange(S, n0, n1, Rn, Rt, v, w)
            v = torch.stack([V0, V1])
            w = W.unsqueeze(0)
            x = x + S.dt * v
    return torch.stack([Rn, Rt])
