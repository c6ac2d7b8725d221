"""Macroscopic observables of a solved step, for comparing solves that differ
only in their domain decomposition (Sec. 4.4): the mean stress tensor, the
sigma_yy profile in horizontal strips of width 2 r_max, and the histogram of
contact force orientations over [0, pi) in 18 bins.

All functions take host (numpy) arrays: the packing's particle data and a
contact set as returned by `Context.contacts()` (moved to the host with
`host_contacts`).  Walls are bodies with index >= N.

Conventions (2D).  Contact c joins body i (ci) and body j (cj) along the
unit normal n from i to j, with gap g; the frame force (R_n, R_t) acts on
body j as F = R_n n + R_t t with t = (-n_y, n_x).  The branch vector is
l = (r_i + r_j + g) n with r_j = 0 for a wall (the wall's point is the
contact point), so that l ⊗ F summed over contacts and divided by the box
volume is the mean stress (compression positive).
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def host_contacts(contacts: Dict[str, object]) -> Dict[str, np.ndarray]:
    """Context.contacts() (device tensors) as numpy arrays."""
    return {k: v.detach().cpu().numpy() for k, v in contacts.items()}


def _branch_and_force(pk, c):
    ci, cj = c["ci"].astype(np.int64), c["cj"].astype(np.int64)
    n = c["normal"]
    R = c["R"]
    if pk.dim != 2:
        raise ValueError("the observables are defined for 2D packings")
    part = cj < pk.n
    rj = np.where(part, pk.r[np.where(part, cj, 0)], 0.0)
    L = pk.r[ci] + rj + c["gap"]
    t = np.stack([-n[1], n[0]])
    F = R[0] * n + R[1] * t
    return ci, L, n, F


def mean_stress(pk, c) -> np.ndarray:
    """(1/V) sum_c l_c ⊗ F_c over all contacts, V the box volume (2x2)."""
    _, L, n, F = _branch_and_force(pk, c)
    V = float(np.prod(np.asarray(pk.box_hi) - np.asarray(pk.box_lo)))
    return np.einsum("c,ic,jc->ij", L, n, F) / V


def stress_profile(pk, x, c, width=None) -> np.ndarray:
    """sigma_yy(y) in horizontal strips of `width` (default 2 r_max) from the
    bottom of the box: each contact counts in the strip holding the midpoint
    of its branch vector; the strip's sum of l_y F_y over its area."""
    ci, L, n, F = _branch_and_force(pk, c)
    w = 2.0 * float(pk.r.max()) if width is None else float(width)
    lo, hi = float(pk.box_lo[1]), float(pk.box_hi[1])
    nb = max(1, int(np.ceil((hi - lo) / w)))
    ymid = x[1, ci] + 0.5 * L * n[1]
    b = np.clip(np.floor((ymid - lo) / w).astype(np.int64), 0, nb - 1)
    area = w * float(pk.box_hi[0] - pk.box_lo[0])
    return np.bincount(b, weights=L * n[1] * F[1], minlength=nb) / area


def orientation_histogram(c, bins: int = 18) -> np.ndarray:
    """Counts of the orientation phi = atan(F_y / F_x) in [0, pi) of the
    forces of closed contacts (R_n > 0), in `bins` equal bins."""
    n, R = c["normal"], c["R"]
    t = np.stack([-n[1], n[0]])
    F = R[0] * n + R[1] * t
    act = R[0] > 0.0
    phi = np.mod(np.arctan2(F[1][act], F[0][act]), np.pi)
    k = np.minimum((phi / (np.pi / bins)).astype(np.int64), bins - 1)
    return np.bincount(k, minlength=bins)


def compare(pk, ref, other) -> Dict[str, float]:
    """Differences of `other` from `ref`, each a dict with the state x and
    the host contacts c: mean stress (max entry difference over the largest
    entry), sigma_yy strips (max difference over the largest strip value),
    orientation histograms (total-variation distance of the normalised
    histograms) and forces when both hold the same contact list."""
    s0, s1 = mean_stress(pk, ref["c"]), mean_stress(pk, other["c"])
    p0 = stress_profile(pk, ref["x"], ref["c"])
    p1 = stress_profile(pk, other["x"], other["c"])
    h0 = orientation_histogram(ref["c"]).astype(np.float64)
    h1 = orientation_histogram(other["c"]).astype(np.float64)
    out = dict(
        mean_stress=float(np.abs(s1 - s0).max() / max(np.abs(s0).max(), 1e-300)),
        strips=float(np.abs(p1 - p0).max() / max(np.abs(p0).max(), 1e-300)),
        orientation_tv=float(0.5 * np.abs(h1 / max(h1.sum(), 1) - h0 / max(h0.sum(), 1)).sum()),
    )
    a, b = ref["c"], other["c"]
    if (a["ci"].shape == b["ci"].shape and np.array_equal(a["ci"], b["ci"])
            and np.array_equal(a["cj"], b["cj"])):
        out["forces"] = float(np.abs(b["R"] - a["R"]).max() / max(np.abs(a["R"]).max(), 1e-300))
    return out
