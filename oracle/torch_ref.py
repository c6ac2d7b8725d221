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


def forces(pb: Problem, pk, mu, v, w, sweeps: int, R0=None):
    """Forces (2 x n_c, frame components (R_n, R_t)) after `sweeps` sweeps
    from R0 (default zero).  mu: (n_c,), v: (2, N), w: (1, N) tensors."""
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
    kn, kt = 1.0 / dwn, 1.0 / dwt
    gdt = np.maximum(pb.gap, 0.0) / dt
    n0, n1 = pb.normal[0], pb.normal[1]
    wall_u = np.zeros((2, nc))
    wid = np.where(wall, cj - N, 0)
    wall_u[:, wall] = pk.wall_velocity[wid[wall]].T
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=f64)
    n0t, n1t, gdtt = T(n0), T(n1), T(gdt)
    dwnt, dwtt, knt, ktt = T(dwn), T(dwt), T(kn), T(kt)
    dtim, dtii = T(dt * inv_m), T(dt * inv_I)
    rt = T(r)
    walln = torch.as_tensor(wall)
    ra = rt[ci]
    rb = torch.where(walln, torch.zeros(nc, dtype=f64), rt[jj])
    dma, dia = dtim[ci], dtii[ci]
    dmb = torch.where(walln, torch.zeros(nc, dtype=f64), dtim[jj])
    dib = torch.where(walln, torch.zeros(nc, dtype=f64), dtii[jj])
    uw0, uw1 = T(wall_u[0]), T(wall_u[1])
    fext, text = T(pk.f), T(pk.t)
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
    ent_p = torch.as_tensor(np.array(ent_p, np.int64))
    colors = [np.nonzero(pb.color == k)[0] for k in range(int(pb.color.max()) + 1 if nc else 0)]
    Rn = torch.zeros(nc, dtype=f64) if R0 is None else T(R0[0])
    Rt = torch.zeros(nc, dtype=f64) if R0 is None else T(R0[1])
    cit, cjt = torch.as_tensor(ci), torch.as_tensor(jj)
    nw = torch.as_tensor(~wall)
    for _ in range(sweeps):
        # exchange: velocities from the previous sweep's forces
        F0 = Rn * n0t + Rt * (-n1t)
        F1 = Rn * n1t + Rt * n0t
        acc0 = fext[0].index_add(0, cit, -F0).index_add(0, cjt[nw], F0[nw])
        acc1 = fext[1].index_add(0, cit, -F1).index_add(0, cjt[nw], F1[nw])
        tq = -(Rt * ra)
        tacc = text[0].index_add(0, cit, tq).index_add(0, cjt[nw], -(Rt * rb)[nw])
        V0 = v[0] + dtim * acc0
        V1 = v[1] + dtim * acc1
        W = w[0] + dtii * tacc
        E0, E1, EW = V0[ent_p], V1[ent_p], W[ent_p]
        Rn_new = torch.zeros(nc, dtype=f64)
        Rt_new = torch.zeros(nc, dtype=f64)
        for idx_np in colors:
            idx = torch.as_tensor(idx_np)
            a_e = torch.as_tensor(ea[idx_np])
            wl = torch.as_tensor(eb[idx_np] < 0)
            b_e = torch.as_tensor(np.where(eb[idx_np] < 0, 0, eb[idx_np]))
            Va0, Va1, Wa = E0[a_e], E1[a_e], EW[a_e]
            Vb0 = torch.where(wl, uw0[idx], E0[b_e])
            Vb1 = torch.where(wl, uw1[idx], E1[b_e])
            Wb = torch.where(wl, torch.zeros_like(Wa), EW[b_e])
            nn0, nn1 = n0t[idx], n1t[idx]
            tt0, tt1 = -nn1, nn0
            dV0, dV1 = Vb0 - Va0, Vb1 - Va1
            vn = dV0 * nn0 + dV1 * nn1
            vt = (dV0 * tt0 + dV1 * tt1) - (ra[idx] * Wa + rb[idx] * Wb)
            un = vn - dwnt[idx] * Rn[idx]
            ut = vt - dwtt[idx] * Rt[idx]
            s = gdtt[idx] + un
            rn = -s * knt[idx]
            Tt = -ut * ktt[idx]
            lim = mu[idx] * rn
            opn = s >= 0.0
            stick = torch.abs(Tt) <= lim
            rn_c = torch.where(opn, torch.zeros_like(rn), rn)
            rt_c = torch.where(opn, torch.zeros_like(rn),
                               torch.where(stick, Tt, torch.where(Tt > 0.0, lim, -lim)))
            dRn, dRt = rn_c - Rn[idx], rt_c - Rt[idx]
            dF0 = dRn * nn0 + dRt * tt0
            dF1 = dRn * nn1 + dRt * tt1
            E0 = E0.index_put((a_e,), Va0 - dma[idx] * dF0)
            E1 = E1.index_put((a_e,), Va1 - dma[idx] * dF1)
            EW = EW.index_put((a_e,), Wa - dia[idx] * (ra[idx] * dRt))
            keep = ~wl
            if bool(keep.any()):
                bk = b_e[keep]
                E0 = E0.index_put((bk,), (Vb0 + dmb[idx] * dF0)[keep])
                E1 = E1.index_put((bk,), (Vb1 + dmb[idx] * dF1)[keep])
                EW = EW.index_put((bk,), (Wb - dib[idx] * (rb[idx] * dRt))[keep])
            Rn_new = Rn_new.index_put((idx,), rn_c)
            Rt_new = Rt_new.index_put((idx,), rt_c)
        Rn, Rt = Rn_new, Rt_new
    return torch.stack([Rn, Rt])
