"""ctypes binding of libcdhip (include/cdhip.h): argument marshalling only.

PyTorch provides device memory and the stream; every step of the solve runs
in the library's HIP kernels.  There is no CPU fallback: without the built
library or without a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdhip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cdhip.h")

OK, MAXITER, EINVAL, ENOMEM, ECAPACITY, ENONFINITE, EHIP, ENOTREADY = 0, 1, -1, -2, -3, -4, -5, -6
ESHADOW = -7


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_walls", C.c_int), ("dt", C.c_double),
                ("alpha", C.c_double), ("mu", C.c_double), ("criterion", C.c_int),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("overlap_mode", C.c_int),
                ("n_domains", C.c_int), ("repartition_every", C.c_int),
                ("warm_start", C.c_int), ("skin", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("n_contacts", C.c_int64),
                ("n_pass", C.c_int64), ("max_d_fail", C.c_double), ("r_avg", C.c_double),
                ("r_avg_prev", C.c_double), ("skin", C.c_double), ("max_colors", C.c_int),
                ("max_domain_contacts", C.c_int), ("n_active", C.c_int64),
                ("crit_last", C.c_double), ("rel_change_last", C.c_double),
                ("n_sliding", C.c_int64)]


class Timing(C.Structure):
    _fields_ = [("detect_ms", C.c_double), ("partition_ms", C.c_double),
                ("order_ms", C.c_double), ("solve_ms", C.c_double), ("update_ms", C.c_double),
                ("sweep_kernel_ms", C.c_double), ("sweep_launches", C.c_int),
                ("sweeps_executed", C.c_int), ("block_threads", C.c_int),
                ("sweeps_timed", C.c_int), ("staged", C.c_int), ("global_records", C.c_int),
                ("foreign_in_lds", C.c_int)]


class BatchTiming(C.Structure):
    _fields_ = [("prepare_ms", C.c_double), ("solve_ms", C.c_double), ("finish_ms", C.c_double),
                ("sweep_kernel_ms", C.c_double), ("sweep_launches", C.c_int),
                ("sweeps_executed", C.c_int), ("sweeps_timed", C.c_int),
                ("block_threads", C.c_int), ("workgroups", C.c_int), ("staged", C.c_int)]


def make_params(dim: int, n_walls: int, *, dt=1e-3, alpha=1e-6, mu=0.3, criterion=0,
                max_iter=2000, fixed_iters=0, overlap_mode=0, n_domains=1,
                repartition_every=1, warm_start=1, skin=-1.0) -> Params:
    return Params(dim, n_walls, dt, alpha, mu, criterion, max_iter, fixed_iters, overlap_mode,
                  n_domains, repartition_every, warm_start, skin)


def declared_symbols() -> list:
    """Function names declared in include/cdhip.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(cd_\w+)\s*\(", text,
                                 re.MULTILINE)))


_lib = None


def lib():
    """Load libcdhip.so (after torch, whose HIP runtime it shares)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads libamdhip64 first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        L.cd_create.argtypes = [C.POINTER(P), C.POINTER(Params), i64, i64, P]
        L.cd_solve_contacts.argtypes = [P, i64, P, P, P, P, P, C.POINTER(Result)]
        L.cd_set_boundary.argtypes = [P, C.c_int, P, P]
        L.cd_get_wall_velocities.argtypes = [P, P]
        L.cd_destroy.argtypes = [P]
        L.cd_set_particles.argtypes = [P, P, P, P, P, P, P]
        L.cd_set_external.argtypes = [P, P, P]
        L.cd_set_walls.argtypes = [P, P, P, P]
        L.cd_set_box.argtypes = [P, P, P]
        L.cd_set_timing.argtypes = [P, C.c_int]
        L.cd_set_solve_mode.argtypes = [P, C.c_int]
        L.cd_set_launch.argtypes = [P, C.c_int]
        L.cd_step.argtypes = [P, C.POINTER(Result)]
        L.cd_get_state.argtypes = [P, P, P, P]
        L.cd_get_walls.argtypes = [P, P]
        L.cd_num_contacts.argtypes = [P]
        L.cd_num_contacts.restype = i64
        L.cd_get_contacts.argtypes = [P, i64, P, P, P, P, P, P, P, P]
        L.cd_get_tree.argtypes = [P, P, P, P, P]
        L.cd_snapshot_size.argtypes = [P, C.POINTER(i64)]
        L.cd_snapshot_save.argtypes = [P, P, i64]
        L.cd_snapshot_load.argtypes = [P, P, i64]
        L.cd_get_timing.argtypes = [P, C.POINTER(Timing)]
        L.cd_status_string.argtypes = [C.c_int]
        L.cd_status_string.restype = C.c_char_p
        L.cd_last_error.argtypes = [P]
        L.cd_last_error.restype = C.c_char_p
        L.cd_prepare.argtypes = [P]
        L.cd_set_contact_mu.argtypes = [P, P]
        L.cd_solve.argtypes = [P, C.POINTER(Result)]
        L.cd_set_adjoint.argtypes = [P, C.c_int]
        L.cd_set_frozen_list.argtypes = [P, C.c_int]
        L.cd_set_mixed_update.argtypes = [P, C.c_double, C.c_ulonglong]
        L.cd_set_random_order.argtypes = [P, C.c_int, C.c_ulonglong]
        L.cd_set_shadow.argtypes = [P, C.c_int]
        L.cd_set_load_balance.argtypes = [P, C.c_double]
        L.cd_set_domain_capacity.argtypes = [P, P]
        L.cd_get_domain_times.argtypes = [P, P, P]
        L.cd_adjoint.argtypes = [P, P, P, P, P]
        if hasattr(L, "cd_adjoint_static"):
            L.cd_adjoint_static.argtypes = [P, P, P, P, P]
        L.cd_batch_create.argtypes = [C.POINTER(P), C.POINTER(P), C.c_int]
        L.cd_batch_destroy.argtypes = [P]
        L.cd_batch_set_timing.argtypes = [P, C.c_int]
        L.cd_batch_step.argtypes = [P, C.POINTER(Result)]
        L.cd_batch_get_timing.argtypes = [P, C.POINTER(BatchTiming)]
        L.cd_batch_last_error.argtypes = [P]
        L.cd_batch_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(t) -> Optional[int]:
    return None if t is None else C.c_void_p(t.data_ptr())


class CDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libcdhip error {code}: {msg}")
        self.code = code


class Context:
    """One simulation on one GPU.  `packing` is a paper_1104_3516_amd.inputs.Packing."""

    def __init__(self, params: Params, packing, device: str = "cuda:0", timing: int = 1,
                 solve_mode: int = 1, block_threads: int = 0, contact_capacity: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libcdhip needs a ROCm GPU; none is visible")
        self.torch = torch
        self.L = lib()
        self.solves = 0     # solves started on this context (stamps autograd records)
        self.device = torch.device(device)
        self.params = params
        self.dim = packing.dim
        self.dr = 1 if self.dim == 2 else 3
        self.n = packing.n
        self.W = packing.n_walls
        if params.n_walls != self.W or params.dim != self.dim:
            raise ValueError("params do not match the packing")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            self._check(self.L.cd_create(C.byref(h), C.byref(params), self.n,
                                         int(contact_capacity),
                                         C.c_void_p(self.stream.cuda_stream)), None)
            self.h = h
            dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64),
                                            device=self.device)
            x, v, w = dev(packing.x), dev(packing.v), dev(packing.w)
            r, m, inertia = dev(packing.r), dev(packing.m), dev(packing.inertia)
            f, t = dev(packing.f), dev(packing.t)
            self._check(self.L.cd_set_particles(self.h, _ptr(x), _ptr(v), _ptr(w), _ptr(r),
                                                _ptr(m), _ptr(inertia)))
            self._x0, self._r, self._m, self._inertia = x, r, m, inertia
            self._v0, self._w0 = v, w
            self._walls = (packing.wall_normal, packing.wall_offset, packing.wall_velocity,
                           packing.box_lo, packing.box_hi)
            self._check(self.L.cd_set_external(self.h, _ptr(f), _ptr(t)))
            wn = np.ascontiguousarray(packing.wall_normal, dtype=np.float64)
            wo = np.ascontiguousarray(packing.wall_offset, dtype=np.float64)
            wv = np.ascontiguousarray(packing.wall_velocity, dtype=np.float64)
            self._check(self.L.cd_set_walls(self.h, wn.ctypes.data_as(C.c_void_p),
                                            wo.ctypes.data_as(C.c_void_p),
                                            wv.ctypes.data_as(C.c_void_p)))
            lo = np.ascontiguousarray(packing.box_lo, dtype=np.float64)
            hi = np.ascontiguousarray(packing.box_hi, dtype=np.float64)
            self._check(self.L.cd_set_box(self.h, lo.ctypes.data_as(C.c_void_p),
                                          hi.ctypes.data_as(C.c_void_p)))
            self._set_boundary(packing)
            self._check(self.L.cd_set_timing(self.h, int(timing)))
            self._check(self.L.cd_set_solve_mode(self.h, solve_mode))
            self._check(self.L.cd_set_launch(self.h, block_threads))
            torch.cuda.synchronize(self.device)

    def _set_boundary(self, packing):
        """Periodic axes and walls of finite mass of the packing (cd_set_boundary)."""
        mask = int(getattr(packing, "periodic", 0) or 0)
        im = getattr(packing, "wall_inv_mass", None)
        wf = getattr(packing, "wall_force", None)
        if not mask and im is None:
            return
        self._bc = tuple(None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                         for a in (im, wf))
        for name, arr in zip(("wall_inv_mass", "wall_force"), self._bc):
            if arr is not None and arr.shape != (self.W,):
                raise ValueError(f"{name} needs one value per wall ({self.W})")
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        self._check(self.L.cd_set_boundary(self.h, mask, ptr(self._bc[0]), ptr(self._bc[1])))

    def wall_velocities(self) -> np.ndarray:
        """The walls' velocities after the steps so far (W x dim): as given,
        with the normal part of walls of finite mass evolved."""
        out = np.zeros(max(self.W, 1) * self.dim)
        self._check(self.L.cd_get_wall_velocities(self.h, out.ctypes.data_as(C.c_void_p)))
        return out[:self.W * self.dim].reshape(self.W, self.dim)

    def _check(self, code: int, h="self"):
        if code < 0:
            msg = self.L.cd_last_error(self.h if h == "self" else None)
            raise CDError(code, (msg or b"").decode())
        return code

    def close(self):
        if getattr(self, "h", None):
            self.L.cd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self) -> Result:
        res = Result()
        self.solves += 1
        self._check(self.L.cd_step(self.h, C.byref(res)))
        return res

    def solve_contacts(self, ci, cj, R=None, dom=None, order=None) -> Result:
        """The force solve alone on a given canonical list (cd_solve_contacts):
        ci, cj (n_c), optional starting forces R (dim x n_c, default 0),
        domains dom (n_c) and update order (n_c, needs dom).  Returns the
        result; the forces are in self.last_R (dim x n_c) and in contacts()."""
        torch = self.torch
        dev = dict(device=self.device)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32, **dev)
        ci_t, cj_t = i32(ci), i32(cj)
        nc = int(ci_t.numel())
        if cj_t.numel() != nc:
            raise ValueError("ci and cj differ in length")
        if R is None:
            R_t = torch.zeros((self.dim, nc), dtype=torch.float64, **dev)
        else:
            R_t = torch.as_tensor(R, dtype=torch.float64, **dev).clone().contiguous()
            if tuple(R_t.shape) != (self.dim, nc):
                raise ValueError(f"R must be ({self.dim}, {nc})")
        dom_t = None if dom is None else i32(dom)
        order_t = None if order is None else i32(order)
        for t in (dom_t, order_t):
            if t is not None and t.numel() != nc:
                raise ValueError("dom and order need one entry per contact")
        res = Result()
        self.solves += 1
        self._check(self.L.cd_solve_contacts(self.h, nc, _ptr(ci_t), _ptr(cj_t), _ptr(dom_t),
                                             _ptr(order_t), _ptr(R_t), C.byref(res)))
        self.last_R = R_t
        return res

    def state(self):
        torch = self.torch
        x = torch.empty((self.dim, self.n), dtype=torch.float64, device=self.device)
        v = torch.empty_like(x)
        w = torch.empty((self.dr, self.n), dtype=torch.float64, device=self.device)
        self._check(self.L.cd_get_state(self.h, _ptr(x), _ptr(v), _ptr(w)))
        return x, v, w

    def wall_offsets(self) -> np.ndarray:
        out = np.zeros(max(self.W, 1))
        self._check(self.L.cd_get_walls(self.h, out.ctypes.data_as(C.c_void_p)))
        return out[:self.W]

    def num_contacts(self) -> int:
        return int(self.L.cd_num_contacts(self.h))

    def contacts(self) -> Dict[str, "object"]:
        torch = self.torch
        nc = self.num_contacts()
        cap = max(nc, 1)
        i32 = dict(dtype=torch.int32, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        out = dict(ci=torch.empty(cap, **i32), cj=torch.empty(cap, **i32),
                   normal=torch.empty((self.dim, cap), **f64), gap=torch.empty(cap, **f64),
                   R=torch.empty((self.dim, cap), **f64), dom=torch.empty(cap, **i32),
                   color=torch.empty(cap, **i32), slot=torch.empty(cap, **i32))
        if nc > 0:
            # (dim x nc) arrays are written with stride nc
            normal = torch.empty(self.dim * nc, **f64)
            R = torch.empty(self.dim * nc, **f64)
            self._check(self.L.cd_get_contacts(self.h, cap, _ptr(out["ci"]), _ptr(out["cj"]),
                                               _ptr(normal), _ptr(out["gap"]), _ptr(R),
                                               _ptr(out["dom"]), _ptr(out["color"]),
                                               _ptr(out["slot"])))
            out["normal"] = normal.view(self.dim, nc)
            out["R"] = R.view(self.dim, nc)
        return {k: (v[..., :nc] if v.dim() == 1 or k in ("normal", "R") else v)
                for k, v in out.items()}

    def tree(self):
        P = self.params.n_domains
        nodes = 2 * P - 1
        axis = np.zeros(nodes, np.int32)
        cut = np.zeros(nodes)
        child = np.zeros(2 * nodes, np.int32)
        leaf = np.zeros(nodes, np.int32)
        self._check(self.L.cd_get_tree(self.h, axis.ctypes.data_as(C.c_void_p),
                                       cut.ctypes.data_as(C.c_void_p),
                                       child.ctypes.data_as(C.c_void_p),
                                       leaf.ctypes.data_as(C.c_void_p)))
        return dict(axis=axis, cut=cut, child=child, leaf=leaf)

    def snapshot(self) -> bytes:
        """The state the next step depends on, as bytes (cd_snapshot_save)."""
        size = C.c_int64(0)
        self._check(self.L.cd_snapshot_size(self.h, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._check(self.L.cd_snapshot_save(self.h, C.cast(buf, C.c_void_p), size.value))
        return buf.raw

    def restore(self, snap: bytes) -> None:
        """Loads a snapshot of a context set up as this one (cd_snapshot_load)."""
        buf = C.create_string_buffer(bytes(snap), len(snap))
        self._check(self.L.cd_snapshot_load(self.h, C.cast(buf, C.c_void_p), len(snap)))

    def timing(self) -> Timing:
        t = Timing()
        self._check(self.L.cd_get_timing(self.h, C.byref(t)))
        return t

    # ---- a step in phases, per-contact friction, adjoint (cd_prepare ...) ----
    def reset(self, v=None, w=None):
        """Back to the initial positions and walls (cold start), with the
        given velocities (default: the packing's)."""
        torch = self.torch
        v = self._v0 if v is None else v.detach().to(self.device, torch.float64).contiguous()
        w = self._w0 if w is None else w.detach().to(self.device, torch.float64).contiguous()
        self._check(self.L.cd_set_particles(self.h, _ptr(self._x0), _ptr(v), _ptr(w),
                                            _ptr(self._r), _ptr(self._m), _ptr(self._inertia)))
        wn, wo, wv, lo, hi = (np.ascontiguousarray(a, dtype=np.float64) for a in self._walls)
        self._check(self.L.cd_set_walls(self.h, wn.ctypes.data_as(C.c_void_p),
                                        wo.ctypes.data_as(C.c_void_p),
                                        wv.ctypes.data_as(C.c_void_p)))
        self._check(self.L.cd_set_box(self.h, lo.ctypes.data_as(C.c_void_p),
                                      hi.ctypes.data_as(C.c_void_p)))

    def prepare(self) -> int:
        self._check(self.L.cd_prepare(self.h))
        return self.num_contacts()

    def set_contact_mu(self, mu):
        mu = mu.detach().to(self.device, self.torch.float64).contiguous()
        nc = self.num_contacts()
        if mu.numel() != nc:
            raise ValueError(f"one friction coefficient per contact of the prepared list: "
                             f"{mu.numel()} given, {nc} contacts")
        self._mu_keep = mu
        self._check(self.L.cd_set_contact_mu(self.h, _ptr(mu)))

    def solve(self) -> Result:
        res = Result()
        self.solves += 1
        self._check(self.L.cd_solve(self.h, C.byref(res)))
        return res

    def set_adjoint(self, checkpoint_every: int):
        self._check(self.L.cd_set_adjoint(self.h, int(checkpoint_every)))

    def set_frozen_list(self, on: bool = True):
        """Keep the next step's contact list, tree and colouring for the
        steps after it (geometry recomputed each step)."""
        self._check(self.L.cd_set_frozen_list(self.h, int(bool(on))))

    def set_mixed_update(self, p: float, seed: int = 0):
        """Mixed sequential/parallel update (Sec. 2.3): contacts with pair
        number below p are updated in parallel; p < 0 switches it off."""
        self._check(self.L.cd_set_mixed_update(self.h, float(p), int(seed)))

    def set_shadow(self, mode: int = 1):
        """Shadow mode (cd_set_shadow): 1 runs every step twice from a
        snapshot and raises CDError(ESHADOW) if the runs differ; 2 is its
        self-test (the second run starts 1e-9 away in one velocity); 0
        steps once."""
        self._check(self.L.cd_set_shadow(self.h, int(mode)))

    def set_random_order(self, on: bool = True, seed: int = 0):
        """Random sequential order (Sec. 2.1): every sweep, each domain's
        contacts one at a time in a fresh SplitMix64 draw of (seed, step,
        sweep, slot); False returns to the colour-major order."""
        self._check(self.L.cd_set_random_order(self.h, int(bool(on)), int(seed)))

    def set_load_balance(self, sigma_star: float):
        """Adaptive load balancing (Sec. 3.3) with threshold sigma_star on
        sigma_T; negative switches it off."""
        self._check(self.L.cd_set_load_balance(self.h, float(sigma_star)))

    def set_domain_capacity(self, capacity=None):
        """Per-domain capacities for the tree rebuilds (None: leaf counts)."""
        if capacity is None:
            self._check(self.L.cd_set_domain_capacity(self.h, None))
            return
        cap = np.ascontiguousarray(capacity, dtype=np.float64)
        if cap.shape != (self.params.n_domains,):
            raise ValueError("one capacity per domain")
        self._check(self.L.cd_set_domain_capacity(self.h, cap.ctypes.data_as(C.c_void_p)))

    def domain_times(self):
        """(per-domain times of the last measured step in microseconds, sigma_T)."""
        t = np.zeros(self.params.n_domains)
        sig = C.c_double(0.0)
        self._check(self.L.cd_get_domain_times(self.h, t.ctypes.data_as(C.c_void_p),
                                               C.byref(sig)))
        return t, sig.value

    def adjoint(self, dL_dR):
        """dL/dmu (n_c), dL/dv (dim x N), dL/dw (dr x N) of the last recorded solve."""
        torch = self.torch
        nc = self.num_contacts()
        if tuple(dL_dR.shape) != (self.dim, nc):
            raise ValueError(f"dL_dR must be ({self.dim}, {nc}) for the recorded solve, "
                             f"got {tuple(dL_dR.shape)}")
        g = dL_dR.detach().to(self.device, torch.float64).contiguous()
        dmu = torch.zeros(max(nc, 1), dtype=torch.float64, device=self.device)
        dv = torch.zeros((self.dim, self.n), dtype=torch.float64, device=self.device)
        dw = torch.zeros((self.dr, self.n), dtype=torch.float64, device=self.device)
        self._check(self.L.cd_adjoint(self.h, _ptr(g), _ptr(dmu), _ptr(dv), _ptr(dw)))
        return dmu[:nc], dv, dw

    def adjoint_static(self, dL_dR):
        """adjoint() through cd_adjoint_static: the reverse pass's workspace
        is the library's static per-device array (no device allocation)."""
        torch = self.torch
        nc = self.num_contacts()
        if tuple(dL_dR.shape) != (self.dim, nc):
            raise ValueError(f"dL_dR must be ({self.dim}, {nc}) for the recorded solve, "
                             f"got {tuple(dL_dR.shape)}")
        g = dL_dR.detach().to(self.device, torch.float64).contiguous()
        dmu = torch.zeros(max(nc, 1), dtype=torch.float64, device=self.device)
        dv = torch.zeros((self.dim, self.n), dtype=torch.float64, device=self.device)
        dw = torch.zeros((self.dr, self.n), dtype=torch.float64, device=self.device)
        self._check(self.L.cd_adjoint_static(self.h, _ptr(g), _ptr(dmu), _ptr(dv), _ptr(dw)))
        return dmu[:nc], dv, dw


def _forces_function():
    import torch

    class ContactForces(torch.autograd.Function):
        """R = forces after a fixed-count solve of one step from the initial
        positions, as a function of per-contact friction mu (n_c) and initial
        velocities v (dim x N), w (dr x N).  Backward: cd_adjoint.  The
        context must be set to a fixed sweep count, a fixed boundary width
        (so that the contact list does not depend on v) and cd_set_adjoint."""

        @staticmethod
        def forward(fctx, mu, v, w, context):
            if not context.params.skin >= 0.0:
                # with the width 2 v_max dt the list would depend on v
                raise ValueError("contact_forces needs a fixed boundary width (params.skin >= 0)")
            if context.params.fixed_iters <= 0:
                raise ValueError("contact_forces needs a fixed sweep count (params.fixed_iters)")
            context.reset(v, w)
            context.prepare()
            context.set_contact_mu(mu)
            context.solve()
            fctx.context = context
            fctx.solve_stamp = context.solves
            return context.contacts()["R"].clone()

        @staticmethod
        def backward(fctx, gR):
            if fctx.context.solves != fctx.solve_stamp:
                raise RuntimeError("the context has solved again since this forward; its "
                                   "adjoint would belong to the later solve")
            dmu, dv, dw = fctx.context.adjoint(gR)
            return dmu, dv, dw, None

    return ContactForces


def contact_forces(mu, v, w, context):
    """Autograd-aware forces of one fixed-count solve (see ContactForces)."""
    return _forces_function().apply(mu, v, w, context)


class Batch:
    """Independent packings stepped together (cd_batch_*): one sweep launch
    per sweep over the domains of every packing still solving.  `contexts`
    are Context objects on one device and stream; they stay owned by the
    caller and must outlive the batch."""

    def __init__(self, contexts, timing: int = 8):
        self.L = lib()
        self.contexts = list(contexts)
        handles = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        code = self.L.cd_batch_create(C.byref(h), handles, len(self.contexts))
        if code < 0:
            raise CDError(code, "cd_batch_create: contexts differ in dimension, device or stream")
        self.h = h
        self._check(self.L.cd_batch_set_timing(self.h, int(timing)))

    def _check(self, code: int):
        if code < 0:
            raise CDError(code, (self.L.cd_batch_last_error(self.h) or b"").decode())
        return code

    def step(self):
        res = (Result * len(self.contexts))()
        code = self.L.cd_batch_step(self.h, res)
        if code < 0 and code != ENONFINITE:
            self._check(code)
        # packings that diverged carry ENONFINITE or EINVAL in their status
        return list(res)

    def timing(self) -> BatchTiming:
        t = BatchTiming()
        self._check(self.L.cd_batch_get_timing(self.h, C.byref(t)))
        return t

    def close(self):
        if getattr(self, "h", None):
            self.L.cd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
