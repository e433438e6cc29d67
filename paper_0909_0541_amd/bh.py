"""Thin Python binding of libbh (the HIP C-ABI library, include/bh.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream, every step runs in the library's kernels.  There is no fallback: when
libbh.so is missing or no GPU is present, load() raises.

Method names follow the C entry points without the ``bh_`` prefix:
``Context.build_tree`` calls ``bh_build_tree`` and so on.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbh.so")

_lib = None

BH_MAX_NCRIT = 256
KIND_CELL, KIND_PARTICLE, KIND_BUCKET, KIND_EMPTY = 0, 1, 2, 3
_STATUS = {0: "BH_OK", -1: "BH_EINVAL", -2: "BH_ENOMEM", -3: "BH_EHIP", -4: "BH_ESTATE", -5: "BH_EINTERNAL"}


class BHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_systems", C.c_int32), ("n_crit", C.c_int32), ("n_cells", C.c_int64),
                ("n_slots", C.c_int64), ("n_groups", C.c_int64), ("interactions", C.c_int64),
                ("list_entries", C.c_int64), ("max_list", C.c_int64), ("max_level", C.c_int32),
                ("error_flags", C.c_int32), ("t_build_ms", C.c_double), ("t_groups_ms", C.c_double),
                ("t_walk_ms", C.c_double), ("t_force_ms", C.c_double), ("n_build_calls", C.c_int32),
                ("n_groups_calls", C.c_int32), ("n_walk_calls", C.c_int32), ("n_force_calls", C.c_int32),
                ("n_split_groups", C.c_int32), ("n_segments", C.c_int32), ("n_split_levels", C.c_int32),
                ("n_walk_attempts", C.c_int32), ("t_particle_ms", C.c_double), ("n_particle_calls", C.c_int32),
                ("n_neighbor_calls", C.c_int32), ("t_neighbor_ms", C.c_double), ("neighbor_pairs", C.c_int64),
                ("neighbor_tests", C.c_int64), ("t_theta_ms", C.c_double), ("n_theta_calls", C.c_int32),
                ("n_theta_fallback", C.c_int32), ("node_visits", C.c_int64), ("near_entries", C.c_int64)]


class _Mlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("mu", C.c_void_p), ("sigma", C.c_void_p)]


MLP_FEATURES, MLP_HIDDEN, MLP_PARAMS = 12, 64, 5057


class _Options(C.Structure):
    _fields_ = [("waves_per_cu", C.c_int32), ("timing", C.c_int32), ("split_visits", C.c_int32),
                ("quadrupole", C.c_int32), ("curve", C.c_int32), ("list_tile", C.c_int32)]


def load():
    """Load libbh.so (built by paper_0909_0541_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sigs = {
        "bh_create": ([C.POINTER(vp), vp], C.c_int),
        "bh_destroy": ([vp], None),
        "bh_last_error": ([vp], C.c_char_p),
        "bh_set_stream": ([vp, vp], C.c_int),
        "bh_get_options": ([vp, C.POINTER(_Options)], C.c_int),
        "bh_set_options": ([vp, C.POINTER(_Options)], C.c_int),
        "bh_sync": ([vp], C.c_int),
        "bh_build_tree": ([vp, i64, vp, vp], C.c_int),
        "bh_build_batch": ([vp, i32, vp, vp, vp], C.c_int),
        "bh_make_groups": ([vp, i32, C.POINTER(i64)], C.c_int),
        "bh_compute_forces": ([vp, dbl, dbl, vp, vp, vp], C.c_int),
        "bh_compute_forces_batch": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "bh_compute_forces_particle": ([vp, dbl, dbl, vp, vp], C.c_int),
        "bh_compute_forces_particle_batch": ([vp, vp, vp, vp, vp], C.c_int),
        "bh_leapfrog": ([vp, i64, vp, vp, vp, C.c_double, C.c_double, i32, C.c_double, i32, vp, vp], C.c_int),
        "bh_get_stats": ([vp, C.POINTER(_Stats)], C.c_int),
        "bh_graph_capture": ([vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp], C.c_int),
        "bh_graph_capture_learned": ([vp, i32, vp, vp, vp, i32, vp, vp, C.POINTER(_Mlp), C.c_float, vp, vp, vp],
                                     C.c_int),
        "bh_graph_launch": ([vp], C.c_int),
        "bh_group_features": ([vp, vp, vp], C.c_int),
        "bh_mlp_infer": ([vp, C.POINTER(_Mlp), i64, vp, C.c_float, vp], C.c_int),
        "bh_group_theta": ([vp, C.POINTER(_Mlp), vp, C.c_float, vp], C.c_int),
        "bh_mlp_grad": ([vp, C.POINTER(_Mlp), i32, vp, vp, vp, vp, vp], C.c_int),
        "bh_mlp_adam": ([vp, vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "bh_direct_sampled": ([vp, i64, vp, vp, dbl, i64, vp, vp, vp], C.c_int),
        "bh_direct_sampled_noalloc": ([vp, i64, vp, vp, dbl, i64, vp, vp, vp], C.c_int),
        "bh_kick": ([vp, i64, vp, vp, dbl], C.c_int),
        "bh_drift": ([vp, i64, vp, vp, dbl], C.c_int),
        "bh_energy": ([vp, i64, vp, vp, vp, vp], C.c_int),
        "bh_export_sorted": ([vp, vp, vp], C.c_int),
        "bh_export_nodes": ([vp, vp, vp], C.c_int),
        "bh_export_moments": ([vp, vp], C.c_int),
        "bh_neighbors": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "bh_export_groups": ([vp, vp, vp, vp, vp], C.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return t


@dataclass
class Stats:
    n: int
    n_systems: int
    n_crit: int
    n_cells: int
    n_slots: int
    n_groups: int
    interactions: int
    list_entries: int
    max_list: int
    max_level: int
    error_flags: int
    t_build_ms: float
    t_groups_ms: float
    t_walk_ms: float
    t_force_ms: float
    n_build_calls: int
    n_groups_calls: int
    n_walk_calls: int
    n_force_calls: int
    n_split_groups: int
    n_segments: int
    n_split_levels: int
    n_walk_attempts: int
    t_particle_ms: float
    n_particle_calls: int
    n_neighbor_calls: int
    t_neighbor_ms: float
    neighbor_pairs: int
    neighbor_tests: int
    t_theta_ms: float
    n_theta_calls: int
    n_theta_fallback: int
    node_visits: int
    near_entries: int


class Context:
    """A bh_ctx bound to a torch stream (the current stream by default)."""

    def __init__(self, stream: torch.cuda.Stream | None = None, waves_per_cu: int | None = None,
                 timing: bool = False, split_visits: int | None = None, quadrupole: bool = False,
                 curve: int = 0, list_tile: int = 0):
        self._L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: libbh runs only on the device")
        self.stream = stream or torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(self._L.bh_create(C.byref(h), C.c_void_p(self.stream.cuda_stream)), None)
        self._h = h
        self.n = 0
        self.n_systems = 0
        opt = _Options()
        self._check(self._L.bh_get_options(self._h, C.byref(opt)))
        if waves_per_cu is not None:
            opt.waves_per_cu = int(waves_per_cu)
        opt.timing = 1 if timing else 0
        if split_visits is not None:
            opt.split_visits = int(split_visits)
        opt.quadrupole = 1 if quadrupole else 0
        opt.curve = int(curve)
        opt.list_tile = int(list_tile)
        self._check(self._L.bh_set_options(self._h, C.byref(opt)))

    def _check(self, st, h=0):
        if st != 0:
            hh = self._h if h == 0 else h
            msg = self._L.bh_last_error(hh).decode() if hh else ""
            raise BHError(st, msg)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.bh_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, waves_per_cu: int | None = None, timing: bool | None = None,
                    split_visits: int | None = None, quadrupole: bool | None = None, curve: int | None = None,
                    list_tile: int | None = None):
        opt = _Options()
        self._check(self._L.bh_get_options(self._h, C.byref(opt)))
        if waves_per_cu is not None:
            opt.waves_per_cu = int(waves_per_cu)
        if timing is not None:
            opt.timing = 1 if timing else 0
        if split_visits is not None:
            opt.split_visits = int(split_visits)
        if quadrupole is not None:
            opt.quadrupole = 1 if quadrupole else 0
        if curve is not None:
            opt.curve = int(curve)
        if list_tile is not None:
            opt.list_tile = int(list_tile)
        self._check(self._L.bh_set_options(self._h, C.byref(opt)))

    def sync(self):
        self._check(self._L.bh_sync(self._h))

    # ---- tree and groups ----
    def build_tree(self, pos: torch.Tensor, mass: torch.Tensor):
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        self._check(self._L.bh_build_tree(self._h, n, _ptr(pos), _ptr(mass)))
        self.n, self.n_systems = n, 1

    def build_batch(self, offsets, pos: torch.Tensor, mass: torch.Tensor):
        import numpy as np
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        n = int(off[-1])
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        self._check(self._L.bh_build_batch(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), _ptr(pos),
                                           _ptr(mass)))
        self.n, self.n_systems = n, len(off) - 1

    def make_groups(self, n_crit: int, sync: bool = True):
        g = C.c_int64(-1)
        self._check(self._L.bh_make_groups(self._h, int(n_crit), C.byref(g) if sync else None))
        return int(g.value) if sync else None

    # ---- forces ----
    def compute_forces(self, eps: float, theta: float, theta_group=None, acc=None, pot=None):
        n = self.n
        dev = torch.device("cuda", torch.cuda.current_device())
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=dev)
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        if theta_group is not None:
            _dev(theta_group, torch.float32, None, "theta_group")
        self._check(self._L.bh_compute_forces(self._h, float(eps), float(theta), _ptr(theta_group), _ptr(acc),
                                              _ptr(pot)))
        return acc, pot

    def compute_forces_batch(self, eps_sys, theta_sys, theta_group=None, acc=None, pot=None):
        import numpy as np
        e = np.ascontiguousarray(np.asarray(eps_sys, dtype=np.float64))
        t = np.ascontiguousarray(np.asarray(theta_sys, dtype=np.float64))
        if e.shape != (self.n_systems,) or t.shape != (self.n_systems,):
            raise ValueError("eps_sys and theta_sys need one value per system")
        n = self.n
        dev = torch.device("cuda", torch.cuda.current_device())
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=dev)
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        self._check(self._L.bh_compute_forces_batch(self._h, e.ctypes.data_as(C.c_void_p),
                                                    t.ctypes.data_as(C.c_void_p), _ptr(theta_group), _ptr(acc),
                                                    _ptr(pot)))
        return acc, pot

    def compute_forces_particle(self, eps, theta, acc=None, pot=None):
        """Per-particle walk and sum (no groups, no lists); eps and theta are
        scalars or one value per system."""
        import numpy as np
        n = self.n
        dev = torch.device("cuda", torch.cuda.current_device())
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=dev)
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        if np.ndim(eps) == 0 and np.ndim(theta) == 0:
            self._check(self._L.bh_compute_forces_particle(self._h, float(eps), float(theta), _ptr(acc), _ptr(pot)))
        else:
            ns = self.n_systems
            e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (ns,)))
            t = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, dtype=np.float64), (ns,)))
            self._check(self._L.bh_compute_forces_particle_batch(self._h, e.ctypes.data_as(C.c_void_p),
                                                                 t.ctypes.data_as(C.c_void_p), _ptr(acc), _ptr(pot)))
        return acc, pot

    def graph_capture(self, offsets, pos: torch.Tensor, mass: torch.Tensor, n_crit: int, eps_sys, theta_sys,
                      theta_group=None, acc=None, pot=None):
        """Record one whole step into a HIP graph (runs it once eagerly first);
        returns (acc, pot), which every graph_launch() rewrites."""
        import numpy as np
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        ns = len(off) - 1
        n = int(off[-1])
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps_sys, dtype=np.float64), (ns,)))
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_sys, dtype=np.float64), (ns,)))
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        dev = torch.device("cuda", torch.cuda.current_device())
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=dev)
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        if theta_group is not None:
            _dev(theta_group, torch.float32, None, "theta_group")
        self._check(self._L.bh_graph_capture(self._h, ns, off.ctypes.data_as(C.c_void_p), _ptr(pos), _ptr(mass),
                                             int(n_crit), e.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                             _ptr(theta_group), _ptr(acc), _ptr(pot)))
        self.n, self.n_systems = n, ns
        self._graph_io = (pos, mass, acc, pot, theta_group)  # keep the captured buffers alive
        return acc, pot

    def graph_capture_learned(self, offsets, pos: torch.Tensor, mass: torch.Tensor, n_crit: int, eps_sys,
                              theta_sys, params, mu, sigma, shift: float = 0.0, theta_group=None, acc=None,
                              pot=None):
        """Record one whole step with the network's per-group theta (features,
        probe walk and inference inside the graph); theta_sys is the fixed
        theta of groups whose network output is NaN.  Returns (acc, pot,
        theta_group), which every graph_launch() rewrites."""
        import numpy as np
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        ns = len(off) - 1
        n = int(off[-1])
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps_sys, dtype=np.float64), (ns,)))
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_sys, dtype=np.float64), (ns,)))
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        dev = torch.device("cuda", torch.cuda.current_device())
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=dev)
        if theta_group is None:
            theta_group = torch.empty((max(n, 1),), dtype=torch.float32, device=dev)
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        _dev(theta_group, torch.float32, (max(n, 1),), "theta_group")
        net = self._net(params, mu, sigma)
        self._check(self._L.bh_graph_capture_learned(self._h, ns, off.ctypes.data_as(C.c_void_p), _ptr(pos),
                                                     _ptr(mass), int(n_crit), e.ctypes.data_as(C.c_void_p),
                                                     t.ctypes.data_as(C.c_void_p), C.byref(net), float(shift),
                                                     _ptr(theta_group), _ptr(acc), _ptr(pot)))
        self.n, self.n_systems = n, ns
        # keep the captured buffers (and the network) alive
        self._graph_io = (pos, mass, acc, pot, theta_group, params, mu, sigma)
        return acc, pot, theta_group

    def graph_launch(self):
        self._check(self._L.bh_graph_launch(self._h))

    def get_stats(self) -> Stats:
        s = _Stats()
        self._check(self._L.bh_get_stats(self._h, C.byref(s)))
        return Stats(*[getattr(s, f) for f, _ in _Stats._fields_])

    # ---- judge and integration ----
    def direct_sampled(self, pos: torch.Tensor, mass: torch.Tensor, eps: float, idx: torch.Tensor):
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        _dev(idx, torch.int64, None, "idx")
        s = idx.shape[0]
        acc = torch.empty((s, 3), dtype=torch.float64, device=pos.device)
        pot = torch.empty((s,), dtype=torch.float64, device=pos.device)
        self._check(self._L.bh_direct_sampled(self._h, n, _ptr(pos), _ptr(mass), float(eps), s, _ptr(idx),
                                              _ptr(acc), _ptr(pot)))
        return acc, pot

    def direct_sampled_noalloc(self, pos: torch.Tensor, mass: torch.Tensor, eps: float, idx: torch.Tensor,
                               acc: torch.Tensor, pot: torch.Tensor):
        """The same judge through the entry point that allocates nothing
        (partial sums in the library's static device array); the caller
        provides acc [s, 3] and pot [s] (FP64, on the device)."""
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(mass, torch.float64, (n,), "mass")
        _dev(idx, torch.int64, None, "idx")
        s = idx.shape[0]
        _dev(acc, torch.float64, (s, 3), "acc")
        _dev(pot, torch.float64, (s,), "pot")
        self._check(self._L.bh_direct_sampled_noalloc(self._h, n, _ptr(pos), _ptr(mass), float(eps), s, _ptr(idx),
                                                      _ptr(acc), _ptr(pot)))
        return acc, pot

    def kick(self, vel: torch.Tensor, acc: torch.Tensor, dt: float):
        n = vel.shape[0]
        _dev(vel, torch.float64, (n, 3), "vel")
        _dev(acc, torch.float32, (n, 3), "acc")
        self._check(self._L.bh_kick(self._h, n, _ptr(vel), _ptr(acc), float(dt)))

    def drift(self, pos: torch.Tensor, vel: torch.Tensor, dt: float):
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(vel, torch.float64, (n, 3), "vel")
        self._check(self._L.bh_drift(self._h, n, _ptr(pos), _ptr(vel), float(dt)))

    def leapfrog(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, eps: float, theta: float,
                 n_crit: int, dt: float, steps: int, acc: torch.Tensor, pot: torch.Tensor):
        """steps KDK steps in place; acc/pot must hold the forces at pos."""
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(vel, torch.float64, (n, 3), "vel")
        _dev(mass, torch.float64, (n,), "mass")
        _dev(acc, torch.float32, (n, 3), "acc")
        _dev(pot, torch.float32, (n,), "pot")
        self._check(self._L.bh_leapfrog(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), float(eps), float(theta),
                                        int(n_crit), float(dt), int(steps), _ptr(acc), _ptr(pot)))
        self.n, self.n_systems = n, 1

    def energy(self, vel: torch.Tensor, mass: torch.Tensor, pot: torch.Tensor, out: torch.Tensor | None = None):
        n = vel.shape[0]
        _dev(vel, torch.float64, (n, 3), "vel")
        _dev(mass, torch.float64, (n,), "mass")
        _dev(pot, torch.float32, (n,), "pot")
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=vel.device)
        self._check(self._L.bh_energy(self._h, n, _ptr(vel), _ptr(mass), _ptr(pot), _ptr(out)))
        return out

    # ---- learned per-group theta ----
    @staticmethod
    def _net(params, mu, sigma):
        _dev(params, torch.float32, (MLP_PARAMS,), "params")
        _dev(mu, torch.float32, (MLP_FEATURES,), "mu")
        _dev(sigma, torch.float32, (MLP_FEATURES,), "sigma")
        return _Mlp(_ptr(params), _ptr(mu), _ptr(sigma))

    def _eps_sys(self, eps):
        import numpy as np
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (self.n_systems,)))
        return e

    def group_features(self, eps, n_groups: int):
        """[n_groups, 12] FP32 features of the current groups (n_groups as
        returned by make_groups)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        feat = torch.empty((max(self.n, 1), MLP_FEATURES), dtype=torch.float32, device=dev)
        e = self._eps_sys(eps)
        self._check(self._L.bh_group_features(self._h, e.ctypes.data_as(C.c_void_p), _ptr(feat)))
        return feat[:n_groups]

    def mlp_infer(self, params, mu, sigma, feat, shift: float = 0.0, theta=None):
        rows = feat.shape[0]
        _dev(feat, torch.float32, (rows, MLP_FEATURES), "feat")
        if theta is None:
            theta = torch.empty(rows, dtype=torch.float32, device=feat.device)
        _dev(theta, torch.float32, None, "theta")
        net = self._net(params, mu, sigma)
        self._check(self._L.bh_mlp_infer(self._h, C.byref(net), rows, _ptr(feat), float(shift), _ptr(theta)))
        return theta

    def group_theta(self, params, mu, sigma, eps, shift: float = 0.0, theta=None):
        """theta of every current group (room for max(n, 1) values)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        if theta is None:
            theta = torch.empty(max(self.n, 1), dtype=torch.float32, device=dev)
        _dev(theta, torch.float32, None, "theta")
        if theta.shape[0] < max(self.n, 1):
            raise ValueError("theta needs room for max(n, 1) values")
        net = self._net(params, mu, sigma)
        e = self._eps_sys(eps)
        self._check(self._L.bh_group_theta(self._h, C.byref(net), e.ctypes.data_as(C.c_void_p), float(shift),
                                           _ptr(theta)))
        return theta

    def mlp_grad(self, params, mu, sigma, x, target, weight, grad=None, loss=None):
        B = x.shape[0]
        _dev(x, torch.float32, (B, MLP_FEATURES), "x")
        _dev(target, torch.float32, (B,), "target")
        _dev(weight, torch.float32, (B,), "weight")
        if grad is None:
            grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        net = self._net(params, mu, sigma)
        self._check(self._L.bh_mlp_grad(self._h, C.byref(net), B, _ptr(x), _ptr(target), _ptr(weight), _ptr(grad),
                                        _ptr(loss)))
        return grad, loss

    def mlp_adam(self, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        n = params.shape[0]
        for t_, name in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
            _dev(t_, torch.float32, (n,), name)
        self._check(self._L.bh_mlp_adam(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, int(step), float(lr),
                                        float(beta1), float(beta2), float(eps)))

    # ---- inspection ----
    def export_sorted(self):
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty(self.n, dtype=torch.int64, device=dev)
        perm = torch.empty(self.n, dtype=torch.int32, device=dev)
        self._check(self._L.bh_export_sorted(self._h, _ptr(keys), _ptr(perm)))
        return keys, perm

    def export_nodes(self):
        st = self.get_stats()
        dev = torch.device("cuda", torch.cuda.current_device())
        ints = torch.empty((st.n_slots, 6), dtype=torch.int32, device=dev)
        reals = torch.empty((st.n_slots, 6), dtype=torch.float64, device=dev)
        self._check(self._L.bh_export_nodes(self._h, _ptr(ints), _ptr(reals)))
        return ints, reals

    def neighbors(self, h: torch.Tensor, count: bool = True, rho: bool = False, offsets: torch.Tensor | None = None,
                  nbr: torch.Tensor | None = None):
        """Neighbour search on the current tree and groups: h FP64 [n] device
        (input order).  Returns (count int32 [n] or None, rho FP64 [n] or
        None); with offsets (int64 [n + 1]) and nbr (int32 [offsets[n]]) the
        lists are written into nbr."""
        n = self.n
        dev = torch.device("cuda", torch.cuda.current_device())
        _dev(h, torch.float64, (n,), "h")
        c = torch.empty(n, dtype=torch.int32, device=dev) if count else None
        r = torch.empty(n, dtype=torch.float64, device=dev) if rho else None
        if offsets is not None:
            _dev(offsets, torch.int64, (n + 1,), "offsets")
            _dev(nbr, torch.int32, None, "nbr")
        self._check(self._L.bh_neighbors(self._h, _ptr(h), _ptr(c), _ptr(r), _ptr(offsets), _ptr(nbr)))
        return c, r

    def neighbor_lists(self, h: torch.Tensor):
        """Counts, then CSR lists: (offsets int64 [n + 1], nbr int32 [total]),
        each row in walk order."""
        c, _ = self.neighbors(h, count=True)
        n = self.n
        off = torch.zeros(n + 1, dtype=torch.int64, device=c.device)
        off[1:] = torch.cumsum(c.to(torch.int64), 0)
        total = int(off[-1].item())
        nbr = torch.empty(max(total, 1), dtype=torch.int32, device=c.device)
        self.neighbors(h, count=False, rho=False, offsets=off, nbr=nbr)
        return off, nbr[:total]

    def export_moments(self):
        """Second mass moments about each node's centre of mass, FP64
        [n_slots, 6] (xx, yy, zz, xy, xz, yz; zero for particle leaves).
        Needs a tree built with the quadrupole option."""
        st = self.get_stats()
        dev = torch.device("cuda", torch.cuda.current_device())
        out = torch.empty((st.n_slots, 6), dtype=torch.float64, device=dev)
        self._check(self._L.bh_export_moments(self._h, _ptr(out)))
        return out

    def export_groups(self, lists: bool = False):
        st = self.get_stats()
        dev = torch.device("cuda", torch.cuda.current_device())
        G = st.n_groups
        ints = torch.empty((G, 3), dtype=torch.int32, device=dev)
        box = torch.empty((G, 6), dtype=torch.float64, device=dev)
        ll = torch.empty(G, dtype=torch.int32, device=dev) if lists else None
        lm = torch.empty(G, dtype=torch.float64, device=dev) if lists else None
        self._check(self._L.bh_export_groups(self._h, _ptr(ints), _ptr(box), _ptr(ll), _ptr(lm)))
        return ints, box, ll, lm


def tree_forces(pos: torch.Tensor, mass: torch.Tensor, eps: float, theta: float, n_crit: int,
                ctx: Context | None = None):
    """One call: build, group and evaluate (single system)."""
    c = ctx or Context()
    c.build_tree(pos, mass)
    c.make_groups(n_crit, sync=False)
    return c.compute_forces(eps, theta)
