"""ctypes front end of the FP64 CPU oracle (libcdref.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CDREF_LIB") or os.path.join(HERE, "libcdref.so")

OK, MAXITER, EINVAL, ENOMEM, ECAPACITY, ENONFINITE = 0, 1, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: IEEE FP64, no contraction into FMA."""
    src = os.path.join(HERE, "cdref.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-Wall", "-fPIC", "-fopenmp", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_walls", C.c_int), ("dt", C.c_double),
                ("alpha", C.c_double), ("mu", C.c_double), ("criterion", C.c_int),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("overlap_mode", C.c_int),
                ("n_domains", C.c_int), ("repartition_every", C.c_int),
                ("warm_start", C.c_int), ("skin", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("n_contacts", C.c_int64),
                ("n_pass", C.c_int64), ("max_d_fail", C.c_double), ("r_avg", C.c_double),
                ("r_avg_prev", C.c_double), ("skin", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        L.cdref_detect.argtypes = [C.c_int, i64, P, P, C.c_int, P, P, C.c_double, C.c_int, P, P,
                                   i64, P, P, C.POINTER(i64)]
        L.cdref_detect_bc.argtypes = [C.c_int, i64, P, P, C.c_int, P, P, C.c_double, C.c_int, P,
                                      P, P, i64, P, P, C.POINTER(i64)]
        L.cdref_geometry_bc.argtypes = [C.c_int, i64, P, P, C.c_int, P, P, P, P, i64, P, P, P,
                                        P, P]
        L.cdref_geometry_bc.restype = None
        L.cdref_wall_velocities.argtypes = [C.c_int, i64, C.c_double, C.c_int, P, P, i64, P, P,
                                            P]
        L.cdref_wall_velocities.restype = None
        L.cdref_solve_bc.argtypes = [C.POINTER(Params), i64, P, P, P, P, P, P, P, P, i64, P, P,
                                     P, P, P, P, C.c_int, P, P, P, P, C.POINTER(Info), P]
        L.cdref_sim_set_bc.argtypes = [P, C.c_int, P, P]
        L.cdref_order_bc.argtypes = [i64, i64, P, P, C.c_int, P, P, C.c_int, P, P, P]
        L.cdref_sim_wall_velocities.argtypes = [P, P]
        L.cdref_sim_wall_velocities.restype = None
        L.cdref_geometry.argtypes = [C.c_int, i64, P, P, C.c_int, P, P, i64, P, P, P, P, P]
        L.cdref_geometry.restype = None
        L.cdref_orb.argtypes = [C.c_int, C.c_int, P, P, i64, P, P, P, P, P, P, P]
        L.cdref_orb_capacity.argtypes = [C.c_int, C.c_int, P, P, i64, P, P, P, P, P, P, P, P]
        L.cdref_balance_fractions.argtypes = [C.c_int, P, P]
        L.cdref_sigma_t.argtypes = [C.c_int, P]
        L.cdref_sigma_t.restype = C.c_double
        L.cdref_sim_set_capacity.argtypes = [P, P]
        L.cdref_pair_uniform.argtypes = [C.c_uint64, i64, i64]
        L.cdref_pair_uniform.restype = C.c_double
        L.cdref_parallel_flags.argtypes = [i64, P, P, C.c_double, C.c_uint64, P]
        L.cdref_parallel_flags.restype = None
        L.cdref_order_mixed.argtypes = [i64, i64, P, P, C.c_int, P, P, P, P, P]
        L.cdref_solve_mixed.argtypes = [C.POINTER(Params), i64, P, P, P, P, P, P, P, P, i64, P,
                                        P, P, P, P, P, C.c_int, P, P, P, C.POINTER(Info), P]
        L.cdref_sim_set_mixed.argtypes = [P, C.c_double, C.c_uint64]
        L.cdref_sim_set_mixed.restype = None
        L.cdref_set_threads.argtypes = [C.c_int]
        L.cdref_set_threads.restype = None
        L.cdref_random_step_key.argtypes = [C.c_uint64, i64]
        L.cdref_random_step_key.restype = C.c_uint64
        L.cdref_random_slot_key.argtypes = [C.c_uint64, C.c_int, i64]
        L.cdref_random_slot_key.restype = C.c_uint64
        L.cdref_solve_random.argtypes = [C.POINTER(Params), i64, P, P, P, P, P, P, P, P, i64, P,
                                         P, P, P, P, C.c_int, P, P, C.c_uint64, i64, P,
                                         C.POINTER(Info), P]
        L.cdref_sim_set_random.argtypes = [P, C.c_int, C.c_uint64]
        L.cdref_descend.argtypes = [C.c_int, C.c_int, P, P, P, P, i64, P, P]
        L.cdref_descend.restype = None
        L.cdref_tree_leaves.argtypes = [C.c_int, P]
        L.cdref_order.argtypes = [i64, i64, P, P, C.c_int, P, P, P, P]
        L.cdref_solve.argtypes = [C.POINTER(Params), i64, P, P, P, P, P, P, P, P, i64, P, P, P,
                                  P, P, C.c_int, P, P, P, C.POINTER(Info), P]
        L.cdref_criterion.argtypes = [C.c_int, i64, P, P, C.c_double, C.c_double, C.c_int,
                                      C.POINTER(i64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.cdref_velocities.argtypes = [C.c_int, i64, C.c_double, P, P, P, P, P, P, P, i64, P, P,
                                       P, P, P, P]
        L.cdref_velocities.restype = None
        L.cdref_sim_create.argtypes = [C.POINTER(Params), i64] + [P] * 13
        L.cdref_sim_create.restype = C.c_void_p
        L.cdref_sim_destroy.argtypes = [P]
        L.cdref_sim_destroy.restype = None
        L.cdref_sim_step.argtypes = [P, C.POINTER(Info)]
        L.cdref_sim_state.argtypes = [P, P, P, P, P]
        L.cdref_sim_state.restype = None
        L.cdref_sim_contacts.argtypes = [P, i64, P, P, P, P, P, P, P, P]
        L.cdref_sim_contacts.restype = i64
        L.cdref_sim_box.argtypes = [P, P, P]
        L.cdref_sim_box.restype = None
        L.cdref_sim_tree.argtypes = [P, P, P, P, P]
        L.cdref_sim_tree.restype = None
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def make_params(dim: int, n_walls: int, *, dt=1e-3, alpha=1e-6, mu=0.3, criterion=0,
                max_iter=2000, fixed_iters=0, overlap_mode=0, n_domains=1,
                repartition_every=1, warm_start=1, skin=-1.0) -> Params:
    return Params(dim, n_walls, dt, alpha, mu, criterion, max_iter, fixed_iters, overlap_mode,
                  n_domains, repartition_every, warm_start, skin)


def period_of(pk):
    """Lengths of the periodic axes of a packing (0 for open axes), or None."""
    mask = getattr(pk, "periodic", 0) or 0
    if not mask:
        return None
    return np.array([(pk.box_hi[k] - pk.box_lo[k]) if (mask >> k) & 1 else 0.0
                     for k in range(pk.dim)], dtype=np.float64)


def detect(pk, skin: float, use_cells: bool = True):
    L = lib()
    x = _f64(pk.x)
    cap = max(16, 8 * pk.n)
    period = period_of(pk)
    while True:
        ci = np.empty(cap, np.int32)
        cj = np.empty(cap, np.int32)
        nc = C.c_int64(0)
        st = L.cdref_detect_bc(pk.dim, pk.n, _p(x), _p(_f64(pk.r)), pk.n_walls,
                               _p(_f64(pk.wall_normal)), _p(_f64(pk.wall_offset)), skin,
                               1 if use_cells else 0, _p(_f64(pk.box_lo)), _p(_f64(pk.box_hi)),
                               _p(period), cap, _p(ci), _p(cj), C.byref(nc))
        if st == ECAPACITY:
            cap = int(nc.value)
            continue
        if st != OK:
            raise RuntimeError(f"cdref_detect failed: {st}")
        return ci[:nc.value].copy(), cj[:nc.value].copy()


def geometry(pk, ci, cj):
    L = lib()
    nc = len(ci)
    normal = np.zeros((pk.dim, nc))
    gap = np.zeros(nc)
    xmid = np.zeros((pk.dim, nc))
    L.cdref_geometry_bc(pk.dim, pk.n, _p(_f64(pk.x)), _p(_f64(pk.r)), pk.n_walls,
                        _p(_f64(pk.wall_normal)), _p(_f64(pk.wall_offset)), _p(period_of(pk)),
                        _p(_f64(pk.box_lo)), nc, _p(_i32(ci)), _p(_i32(cj)), _p(normal), _p(gap),
                        _p(xmid))
    return normal, gap, xmid


class MobileWalls(C.Structure):
    _fields_ = [("normal", C.c_void_p), ("inv_mass", C.c_void_p), ("force", C.c_void_p)]


def mobile_walls(pk):
    """The cdref_mobile_walls of a packing with walls of finite mass (else
    None), and the arrays it points to (kept alive by the caller)."""
    if getattr(pk, "wall_inv_mass", None) is None or not np.any(pk.wall_inv_mass != 0):
        return None, None
    keep = (_f64(pk.wall_normal), _f64(pk.wall_inv_mass),
            _f64(pk.wall_force if pk.wall_force is not None else np.zeros(pk.n_walls)))
    return MobileWalls(*[a.ctypes.data for a in keep]), keep


def wall_velocities(pk, dt, cj, R):
    """Velocities of the walls after forces R (cdref_wall_velocities), W x dim."""
    mw, keep = mobile_walls(pk)
    U = np.zeros((max(pk.n_walls, 1), pk.dim))
    lib().cdref_wall_velocities(pk.dim, pk.n, dt, pk.n_walls, _p(_f64(pk.wall_velocity)),
                                C.byref(mw) if mw is not None else None, len(cj), _p(_i32(cj)),
                                _p(_f64(R)), _p(U))
    return U[:pk.n_walls]


@dataclasses.dataclass
class Tree:
    axis: np.ndarray
    cut: np.ndarray
    child: np.ndarray
    leaf: np.ndarray
    leaves: np.ndarray


def orb(dim: int, P: int, box_lo, box_hi, xmid, capacity=None):
    """Bisection tree and domains; `capacity` (P values) places the cuts by
    capacity share (Sec. 3.3) instead of leaf counts."""
    L = lib()
    xmid = _f64(xmid)
    nc = xmid.shape[1] if xmid.ndim == 2 else 0
    nodes = 2 * P - 1
    t = Tree(np.zeros(nodes, np.int32), np.zeros(nodes), np.zeros(2 * nodes, np.int32),
             np.zeros(nodes, np.int32), np.zeros(nodes, np.int32))
    dom = np.zeros(max(nc, 1), np.int32)
    cap = None if capacity is None else _f64(capacity)
    st = L.cdref_orb_capacity(dim, P, _p(_f64(box_lo)), _p(_f64(box_hi)), nc, _p(xmid), _p(cap),
                              _p(t.axis), _p(t.cut), _p(t.child), _p(t.leaf), _p(t.leaves),
                              _p(dom))
    if st != OK:
        raise RuntimeError(f"cdref_orb failed: {st}")
    return t, dom[:nc]


def balance_fractions(P: int, capacity) -> np.ndarray:
    """Left-branch share of every inner node for per-domain capacities
    (Sec. 3.3); 2P-1 entries in creation order, 0 for leaves."""
    out = np.zeros(2 * P - 1)
    st = lib().cdref_balance_fractions(P, _p(_f64(capacity)), _p(out))
    if st != OK:
        raise RuntimeError(st)
    return out


def sigma_t(T) -> float:
    """Load imbalance of per-domain times (Sec. 3.3)."""
    T = _f64(T)
    return float(lib().cdref_sigma_t(len(T), _p(T)))


def descend(dim: int, P: int, tree: Tree, xmid):
    L = lib()
    xmid = _f64(xmid)
    nc = xmid.shape[1]
    dom = np.zeros(max(nc, 1), np.int32)
    L.cdref_descend(dim, P, _p(tree.axis), _p(tree.cut), _p(tree.child), _p(tree.leaf), nc,
                    _p(xmid), _p(dom))
    return dom[:nc]


def tree_leaves(P: int) -> np.ndarray:
    out = np.zeros(2 * P - 1, np.int32)
    st = lib().cdref_tree_leaves(P, _p(out))
    if st != OK:
        raise RuntimeError(st)
    return out


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def pair_uniform(seed: int, i: int, j: int) -> float:
    return float(lib().cdref_pair_uniform(seed, i, j))


def parallel_flags(ci, cj, p: float, seed: int) -> np.ndarray:
    """Contacts updated in parallel in the mixed scheme (Sec. 2.3)."""
    nc = len(ci)
    out = np.zeros(max(nc, 1), np.uint8)
    lib().cdref_parallel_flags(nc, _p(_i32(ci)), _p(_i32(cj)), p, seed, _p(out))
    return out[:nc]


def order(n: int, ci, cj, P: int, dom, parallel=None, mobile_mask: int = 0):
    """Colour-major order per domain; walls in mobile_mask (bit w) conflict
    like particles (cdref_order_bc)."""
    L = lib()
    nc = len(ci)
    color = np.zeros(max(nc, 1), np.int32)
    slot = np.zeros(max(nc, 1), np.int32)
    dom_start = np.zeros(P + 1, np.int64)
    par = None if parallel is None else _u8(parallel)
    st = L.cdref_order_bc(n, nc, _p(_i32(ci)), _p(_i32(cj)), P, _p(_i32(dom)), _p(par),
                          int(mobile_mask), _p(color), _p(slot), _p(dom_start))
    if st != OK:
        raise RuntimeError(f"cdref_order failed: {st}")
    return color[:nc], slot[:nc], dom_start


def solve(params: Params, pk, ci, cj, normal, gap, P: int, dom_start, slot, R0=None,
          mu_c=None, history: bool = False, parallel=None, random_order=None):
    """One force solve.  Returns (R, info, history-or-None).  `random_order`
    = (seed, step): each domain updates its contacts in the random order of
    `random_slot_key`, drawn afresh in every sweep (Sec. 2.1)."""
    L = lib()
    nc = len(ci)
    dim = pk.dim
    R = np.zeros((dim, nc)) if R0 is None else _f64(R0).copy()
    info = Info()
    limit = params.fixed_iters if params.fixed_iters > 0 else params.max_iter
    hist = np.zeros((4, limit)) if history else None
    par = None if parallel is None else _u8(parallel)
    if random_order is not None:
        if parallel is not None:
            raise ValueError("the random order has no parallel contacts")
        seed, step = random_order
        st = L.cdref_solve_random(C.byref(params), pk.n, _p(_f64(pk.v)), _p(_f64(pk.w)),
                                  _p(_f64(pk.r)), _p(_f64(pk.m)), _p(_f64(pk.inertia)),
                                  _p(_f64(pk.f)), _p(_f64(pk.t)), _p(_f64(pk.wall_velocity)), nc,
                                  _p(_i32(ci)), _p(_i32(cj)), _p(_f64(normal)), _p(_f64(gap)),
                                  None if mu_c is None else _p(_f64(mu_c)), P,
                                  _p(np.ascontiguousarray(dom_start, np.int64)), _p(_i32(slot)),
                                  int(seed), int(step), _p(R), C.byref(info), _p(hist))
        if st < 0:
            raise RuntimeError(f"cdref_solve_random failed: {st}")
        return R, info, (hist[:, :info.iterations] if hist is not None else None)
    mw, keep_mw = mobile_walls(pk)
    st = L.cdref_solve_bc(C.byref(params), pk.n, _p(_f64(pk.v)), _p(_f64(pk.w)),
                          _p(_f64(pk.r)), _p(_f64(pk.m)), _p(_f64(pk.inertia)),
                          _p(_f64(pk.f)), _p(_f64(pk.t)), _p(_f64(pk.wall_velocity)), nc,
                          _p(_i32(ci)), _p(_i32(cj)), _p(_f64(normal)), _p(_f64(gap)),
                          None if mu_c is None else _p(_f64(mu_c)), _p(par), P,
                          _p(np.ascontiguousarray(dom_start, np.int64)), _p(_i32(slot)),
                          C.byref(mw) if mw is not None else None, _p(R), C.byref(info),
                          _p(hist))
    if st < 0:
        raise RuntimeError(f"cdref_solve failed: {st}")
    if hist is not None:
        hist = hist[:, :info.iterations]
    return R, info, hist


def set_threads(threads: int) -> None:
    """Spread the domains of each sweep over `threads` OpenMP threads."""
    lib().cdref_set_threads(int(threads))


def random_step_key(seed: int, step: int) -> int:
    """K = SplitMix64(SplitMix64(seed) ^ step) of a time step's random order."""
    return int(lib().cdref_random_step_key(seed, step))


def random_slot_key(step_key: int, j: int, s: int) -> int:
    """Draw of slot s in sweep j: SplitMix64(SplitMix64(K ^ j) ^ s)."""
    return int(lib().cdref_random_slot_key(step_key, j, s))


def criterion(Rprev, R, ravg_prev: float, alpha: float, which: int = 0):
    """Convergence tests (I)/(II) on one pair of sweeps.  Returns
    (converged, n_pass, max_d_fail, r_avg, finite)."""
    Rprev = _f64(np.atleast_2d(Rprev))
    R = _f64(np.atleast_2d(R))
    dim, nc = R.shape
    npass = C.c_int64(0)
    maxd = C.c_double(0)
    ravg = C.c_double(0)
    fin = C.c_int(0)
    conv = lib().cdref_criterion(dim, nc, _p(Rprev), _p(R), ravg_prev, alpha, which,
                                 C.byref(npass), C.byref(maxd), C.byref(ravg), C.byref(fin))
    return bool(conv), int(npass.value), float(maxd.value), float(ravg.value), bool(fin.value)


def velocities(pk, dt, ci, cj, normal, R):
    L = lib()
    dr = 1 if pk.dim == 2 else 3
    V = np.zeros((pk.dim, pk.n))
    W = np.zeros((dr, pk.n))
    L.cdref_velocities(pk.dim, pk.n, dt, _p(_f64(pk.v)), _p(_f64(pk.w)), _p(_f64(pk.m)),
                       _p(_f64(pk.inertia)), _p(_f64(pk.r)), _p(_f64(pk.f)), _p(_f64(pk.t)),
                       len(ci), _p(_i32(ci)), _p(_i32(cj)), _p(_f64(normal)), _p(_f64(R)),
                       _p(V), _p(W))
    return V, W


class Sim:
    """Whole time steps on the CPU (state carried between steps)."""

    def __init__(self, params: Params, pk):
        self.L = lib()
        self.params = params
        self.pk = pk
        self.dim = pk.dim
        self.n = pk.n
        self._keep = [_f64(a) for a in (pk.x, pk.v, pk.w, pk.r, pk.m, pk.inertia, pk.f, pk.t,
                                         pk.wall_normal, pk.wall_offset, pk.wall_velocity,
                                         pk.box_lo, pk.box_hi)]
        self.h = self.L.cdref_sim_create(C.byref(params), pk.n, *[_p(a) for a in self._keep])
        if not self.h:
            raise RuntimeError("cdref_sim_create failed")
        mask = getattr(pk, "periodic", 0) or 0
        im = getattr(pk, "wall_inv_mass", None)
        if mask or im is not None:
            self._bc = (None if im is None else _f64(im),
                        None if getattr(pk, "wall_force", None) is None else _f64(pk.wall_force))
            st = self.L.cdref_sim_set_bc(self.h, int(mask), _p(self._bc[0]), _p(self._bc[1]))
            if st != OK:
                raise RuntimeError(f"cdref_sim_set_bc failed: {st}")

    def close(self):
        if self.h:
            self.L.cdref_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self) -> Info:
        info = Info()
        st = self.L.cdref_sim_step(self.h, C.byref(info))
        if st < 0:
            raise RuntimeError(f"cdref_sim_step failed: {st}")
        return info

    def state(self):
        dr = 1 if self.dim == 2 else 3
        x = np.zeros((self.dim, self.n))
        v = np.zeros((self.dim, self.n))
        w = np.zeros((dr, self.n))
        wo = np.zeros(max(self.params.n_walls, 1))
        self.L.cdref_sim_state(self.h, _p(x), _p(v), _p(w), _p(wo))
        return x, v, w, wo[:self.params.n_walls]

    def wall_velocities(self):
        U = np.zeros((max(self.params.n_walls, 1), self.dim))
        self.L.cdref_sim_wall_velocities(self.h, _p(U))
        return U[:self.params.n_walls]

    def box(self):
        lo = np.zeros(self.dim)
        hi = np.zeros(self.dim)
        self.L.cdref_sim_box(self.h, _p(lo), _p(hi))
        return lo, hi

    def contacts(self):
        nc = self.L.cdref_sim_contacts(self.h, 0, None, None, None, None, None, None, None, None)
        cap = max(nc, 1)
        ci = np.zeros(cap, np.int32)
        cj = np.zeros(cap, np.int32)
        normal = np.zeros((self.dim, cap))
        gap = np.zeros(cap)
        R = np.zeros((self.dim, cap))
        dom = np.zeros(cap, np.int32)
        color = np.zeros(cap, np.int32)
        slot = np.zeros(cap, np.int32)
        self.L.cdref_sim_contacts(self.h, cap, _p(ci), _p(cj), _p(normal), _p(gap), _p(R),
                                  _p(dom), _p(color), _p(slot))
        return dict(ci=ci[:nc], cj=cj[:nc], normal=normal[:, :nc], gap=gap[:nc], R=R[:, :nc],
                    dom=dom[:nc], color=color[:nc], slot=slot[:nc])

    def set_mixed(self, p: float, seed: int = 0):
        """Mixed update from now on (Sec. 2.3): contacts with pair number
        below p are updated in parallel; p < 0 switches it off."""
        self.L.cdref_sim_set_mixed(self.h, float(p), int(seed))

    def set_random(self, on: bool = True, seed: int = 0):
        """Random sequential order from now on (Sec. 2.1); the draws of a
        step use the number of steps taken before it."""
        self.L.cdref_sim_set_random(self.h, 1 if on else 0, int(seed))

    def set_capacity(self, capacity=None):
        """Per-domain capacities for every later tree rebuild (None: leaf counts)."""
        self._cap = None if capacity is None else _f64(capacity)
        st = self.L.cdref_sim_set_capacity(self.h, _p(self._cap))
        if st != OK:
            raise RuntimeError(st)

    def tree(self) -> Tree:
        P = self.params.n_domains
        nodes = 2 * P - 1
        t = Tree(np.zeros(nodes, np.int32), np.zeros(nodes), np.zeros(2 * nodes, np.int32),
                 np.zeros(nodes, np.int32), tree_leaves(P))
        self.L.cdref_sim_tree(self.h, _p(t.axis), _p(t.cut), _p(t.child), _p(t.leaf))
        return t
