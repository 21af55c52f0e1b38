"""ctypes binding of the MR. POP C ABI.

Functions take and return torch tensors on the context's device; host
inputs (numpy arrays) are copied to the device first.  Work is queued on
torch's current stream for that device.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libmrpop.so"

STATUS_NAMES = {
    0: "OK", 1: "E_INVALID_ARG", 2: "E_NONFINITE", 3: "E_START_INVALID", 4: "E_GOAL_INVALID",
    5: "E_NO_SOLUTION", 6: "E_CAPACITY", 7: "E_NOMEM", 8: "E_BUFFER", 9: "E_DEVICE", 10: "PENDING",
}


class MrpopError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


class _Robot(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("dh", C.c_void_p), ("q_lo", C.c_void_p), ("q_hi", C.c_void_p),
                ("base_tf", C.c_void_p), ("n_spheres", C.c_int32), ("sphere_link", C.c_void_p),
                ("sphere_xyzr", C.c_void_p)]


class _Env(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("spheres", C.c_void_p), ("n_boxes", C.c_int32), ("boxes", C.c_void_p)]


class _ValidateStats(C.Structure):
    _fields_ = [("edge_states", C.c_int64), ("states_checked", C.c_int64), ("edges_invalid", C.c_int64),
                ("nonfinite_edges", C.c_int64), ("tiles", C.c_int64), ("work", C.c_int64 * 8)]


class _KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("kernel_ms", C.c_double), ("states_checked", C.c_int64),
                ("edge_states", C.c_int64), ("work", C.c_int64 * 8), ("grid_blocks", C.c_int32),
                ("block_threads", C.c_int32), ("timed_launches", C.c_int64)]


class PlanParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("delta", C.c_float), ("n_roadmap", C.c_int32), ("candidates", C.c_int32),
                ("resolution", C.c_float), ("max_rounds", C.c_int32), ("max_iterations", C.c_int32),
                ("max_growth_rounds", C.c_int32), ("time_budget_s", C.c_double), ("max_tree_nodes", C.c_int32),
                ("max_roadmap_nodes", C.c_int32), ("stop_at_first", C.c_int32), ("warm_cost", C.c_float),
                ("direct", C.c_int32), ("step", C.c_float), ("rewire", C.c_int32)]


class _PlanStats(C.Structure):
    _fields_ = [("time_to_first_s", C.c_double), ("total_time_s", C.c_double), ("rounds", C.c_int32),
                ("iterations", C.c_int32), ("solutions", C.c_int32), ("first_round", C.c_int32),
                ("edge_states", C.c_int64), ("roadmap_edge_states", C.c_int64), ("roadmap_vertices", C.c_int32),
                ("roadmap_connected", C.c_int32), ("capacity_hit", C.c_int32), ("n_costs", C.c_int32),
                ("costs", C.c_float * 64), ("speculative_edge_states", C.c_int64), ("rewired", C.c_int64)]


class _PlanRequest(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("q_start", C.c_void_p), ("q_goal", C.c_void_p), ("params", PlanParams),
                ("path_out", C.c_void_p), ("path_cap", C.c_int32), ("status", C.c_int32), ("path_len", C.c_int32),
                ("cost", C.c_float), ("stats", _PlanStats)]


MAX_ROBOTS = 16  # MRPOP_MAX_ROBOTS


class _PlanHistory(C.Structure):
    _fields_ = [("waypoints", C.c_void_p), ("waypoint_cap", C.c_int64), ("offsets", C.c_void_p),
                ("costs", C.c_void_p), ("found_s", C.c_void_p), ("found_round", C.c_void_p),
                ("entry_cap", C.c_int32), ("n_entries", C.c_int32), ("n_written", C.c_int32),
                ("vertex_ids", C.c_void_p), ("rm_vertices", C.c_void_p), ("rm_edges", C.c_void_p),
                ("rm_vertex_cap", C.c_int32), ("rm_edge_cap", C.c_int32),
                ("rm_n_vertices", C.c_int32 * MAX_ROBOTS), ("rm_n_edges", C.c_int32 * MAX_ROBOTS)]


class _ServerConfig(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("mem_budget_bytes", C.c_int64)]


class _ServerResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("path_len", C.c_int32), ("cost", C.c_float), ("stats", _PlanStats),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("device_bytes", C.c_int64)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("queue_len", C.c_int32), ("running", C.c_int32),
                ("max_queue_len", C.c_int32), ("max_running", C.c_int32), ("reserved_bytes", C.c_int64),
                ("peak_reserved_bytes", C.c_int64), ("flushes", C.c_int64), ("launches", C.c_int64)]


class _ExtendBatch(C.Structure):
    _fields_ = [("n", C.c_int32), ("near_idx", C.c_void_p), ("q_rand", C.c_void_p), ("c_rand", C.c_void_p),
                ("tree_q", C.c_void_p), ("tree_g", C.c_void_p), ("tree_vid", C.c_void_p), ("tree_cap", C.c_int32),
                ("rm_vertices", C.c_void_p), ("rm_rowptr", C.c_void_p), ("rm_col", C.c_void_p),
                ("rm_cap", C.c_int32), ("col_cap", C.c_int32), ("resolution", C.c_float), ("q_new", C.c_void_p),
                ("vid_new", C.c_void_p), ("g_new", C.c_void_p), ("alive", C.c_void_p), ("edge_a", C.c_void_p),
                ("edge_b", C.c_void_p), ("n_states", C.c_void_p)]


class _BatchStats(C.Structure):
    _fields_ = [("wall_s", C.c_double), ("instances", C.c_int32), ("solved", C.c_int32), ("flushes", C.c_int64),
                ("launches", C.c_int64)]


@dataclass
class PlanResult:
    status: str
    path: Optional[np.ndarray]
    cost: float
    stats: dict


@dataclass
class Incumbent:
    """One entry of a plan's incumbent history (mrpop_plan_with_history)."""
    path: np.ndarray   # [len][D], start to goal
    cost: float
    found_s: float     # seconds from the call's start
    found_round: int
    vertex_ids: Optional[np.ndarray] = None  # [len][R] roadmap vertex of each arm per waypoint


WORK_NAMES = ("chains", "links", "env_tests", "box_exact", "rr_coarse", "fine_sphere", "fine_box", "fine_rr")


@dataclass
class ValidateStats:
    edge_states: int
    states_checked: int
    edges_invalid: int
    nonfinite_edges: int
    tiles: int
    work: dict


@dataclass
class KernelProfile:
    launches: int
    kernel_ms: float
    states_checked: int
    edge_states: int
    work: dict
    grid_blocks: int = 0
    block_threads: int = 0
    timed_launches: int = 0


_lib = None


def load_library():
    """Load libmrpop.so; raises ImportError when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    # torch ships its own HIP runtime (same soname); load it first so that the
    # process holds a single runtime and torch's allocations and streams are
    # valid for the library.
    _torch()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2609_30644_amd.build`")
    lib = C.CDLL(path)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    lib.mrpop_version.restype = C.c_char_p
    lib.mrpop_last_error.restype = C.c_char_p
    lib.mrpop_last_error.argtypes = [P]
    lib.mrpop_ctx_create.argtypes = [C.c_int, C.POINTER(P)]
    lib.mrpop_ctx_destroy.argtypes = [P]
    lib.mrpop_scene_create.argtypes = [P, P, I32, P, C.POINTER(P)]
    lib.mrpop_scene_destroy.argtypes = [P]
    lib.mrpop_scene_set_env.argtypes = [P, P]
    lib.mrpop_replan.argtypes = [P, P, P, P, P, P, I32, P, I32, P, P, P, P]
    lib.mrpop_scene_dof.argtypes = [P]
    lib.mrpop_scene_dof.restype = I32
    lib.mrpop_scene_total_spheres.argtypes = [P]
    lib.mrpop_scene_total_spheres.restype = I32
    lib.mrpop_scene_obstacle_clusters.argtypes = [P]
    lib.mrpop_scene_obstacle_clusters.restype = I32
    lib.mrpop_scene_set_tile_mode.argtypes = [P, I32]
    lib.mrpop_scene_set_tile_mode.restype = I32
    lib.mrpop_scene_tile_mode.argtypes = [P]
    lib.mrpop_scene_tile_mode.restype = I32
    lib.mrpop_fk_spheres.argtypes = [P, P, P, I64, P, P]
    lib.mrpop_validate_edges.argtypes = [P, P, P, P, I64, C.c_float, P, P, P, P]
    lib.mrpop_validate_edges_noalloc.argtypes = [P, P, P, P, I64, C.c_float, P, P, P, P]
    lib.mrpop_validate_counted.argtypes = [P, P, P, P, I64, P, P, P, P]
    lib.mrpop_tuner_configure.argtypes = [C.c_char_p, I32]
    lib.mrpop_tuner_entries.argtypes = []
    lib.mrpop_tuner_entries.restype = I32
    lib.mrpop_nearest.argtypes = [P, P, P, I64, I32, P, P, I64, P, P]
    lib.mrpop_sample.argtypes = [P, P, P, P, P, C.c_float, C.c_uint64, C.c_uint64, I64, I64, P, P, P]
    lib.mrpop_extend.argtypes = [P, P, P, P]
    lib.mrpop_plan_params_default.argtypes = [P]
    lib.mrpop_plan_params_default.restype = None
    lib.mrpop_plan.argtypes = [P, P, P, P, P, P, I32, P, P, P]
    lib.mrpop_plan_with_history.argtypes = [P, P, P, P, P, P, I32, P, P, P, P]
    lib.mrpop_plan_batch.argtypes = [P, P, I32, P]
    lib.mrpop_server_create.argtypes = [P, P, P]
    lib.mrpop_server_destroy.argtypes = [P]
    lib.mrpop_server_destroy.restype = None
    lib.mrpop_server_submit.argtypes = [P, P, P, P, P, P]
    lib.mrpop_server_poll.argtypes = [P, I64, P]
    lib.mrpop_server_wait.argtypes = [P, I64, C.c_double, P]
    lib.mrpop_server_path.argtypes = [P, I64, P, I32]
    lib.mrpop_server_release.argtypes = [P, I64]
    lib.mrpop_server_get_stats.argtypes = [P, P]
    lib.mrpop_server_clock.argtypes = [P]
    lib.mrpop_server_clock.restype = C.c_double
    lib.mrpop_profile_enable.argtypes = [P, C.c_int]
    lib.mrpop_profile_read.argtypes = [P, P]
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _stream_ptr(device) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """Owns a library context on one HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        h = C.c_void_p()
        self._check(self._lib.mrpop_ctx_create(device, C.byref(h)), None)
        self._h = h

    def _check(self, st: int, h) -> None:
        if st != 0:
            msg = self._lib.mrpop_last_error(h).decode()
            raise MrpopError(st, msg)

    def check(self, st: int) -> None:
        self._check(st, self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mrpop_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # tensors -----------------------------------------------------------
    def to_device(self, a, dtype=None):
        torch = _torch()
        if isinstance(a, torch.Tensor):
            t = a.to(self.device)
        else:
            t = torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        if dtype is not None:
            t = t.to(dtype)
        return t.contiguous()

    def stream(self) -> int:
        return _stream_ptr(self.device)

    def plan_batch(self, problems, path_cap: int = 4096, **common):
        """mrpop_plan_batch over problems = [(scene, q_start, q_goal, params
        dict), ...]; `common` holds parameters shared by all.  Returns
        ([PlanResult], batch stats dict)."""
        lib = self._lib
        n = len(problems)
        reqs = (_PlanRequest * max(1, n))()
        keep = []
        for i, (scene, qs, qg, prm) in enumerate(problems):
            pp = PlanParams()
            lib.mrpop_plan_params_default(C.byref(pp))
            for k, v in {**common, **(prm or {})}.items():
                if not hasattr(pp, k):
                    raise KeyError(k)
                setattr(pp, k, v)
            qs = np.ascontiguousarray(qs, np.float32).reshape(scene.dof)
            qg = np.ascontiguousarray(qg, np.float32).reshape(scene.dof)
            path = np.zeros((max(1, path_cap), scene.dof), np.float32)
            keep.append((qs, qg, path))
            reqs[i].scene = scene.handle
            reqs[i].q_start = qs.ctypes.data
            reqs[i].q_goal = qg.ctypes.data
            reqs[i].params = pp
            reqs[i].path_out = path.ctypes.data
            reqs[i].path_cap = path_cap
        bs = _BatchStats()
        self.check(lib.mrpop_plan_batch(self.handle, reqs, n, C.byref(bs)))
        out = []
        for i in range(n):
            r = reqs[i]
            stats = {k: getattr(r.stats, k) for k, _ in _PlanStats._fields_ if k != "costs"}
            stats["costs"] = list(r.stats.costs[:r.stats.n_costs])
            stats["path_len"] = r.path_len
            path = keep[i][2]
            out.append(PlanResult(STATUS_NAMES.get(r.status, str(r.status)),
                                  path[:r.path_len].copy() if r.status == 0 else None, float(r.cost), stats))
        return out, {k: getattr(bs, k) for k, _ in _BatchStats._fields_}

    def nearest(self, vertices, costs, queries, budgets=None, out=None):
        """Cost-bounded nearest vertex per query (int32, -1 when none)."""
        torch = _torch()
        Q = self.to_device(queries, torch.float32)
        dim = Q.shape[-1]
        Q = Q.reshape(-1, dim)
        V = self.to_device(vertices, torch.float32).reshape(-1, dim)
        g = None if costs is None else self.to_device(costs, torch.float32).reshape(V.shape[0])
        b = None if budgets is None else self.to_device(budgets, torch.float32).reshape(Q.shape[0])
        if out is None:
            out = torch.empty(Q.shape[0], dtype=torch.int32, device=self.device)
        self.check(self._lib.mrpop_nearest(self._h, V.data_ptr(), None if g is None else g.data_ptr(), V.shape[0],
                                           V.shape[1], Q.data_ptr(), None if b is None else b.data_ptr(), Q.shape[0],
                                           out.data_ptr(), self.stream()))
        return out

    def tuner_configure(self, cache_file: Optional[str] = None, enable: bool = True) -> None:
        """mrpop_tuner_configure: the tile-shape cache file (None: none) and
        whether unseen launch kinds are measured (process-wide)."""
        self._check(self._lib.mrpop_tuner_configure(None if cache_file is None else cache_file.encode(),
                                                     1 if enable else 0), None)

    def tuner_entries(self) -> int:
        return int(self._lib.mrpop_tuner_entries())

    def profile_enable(self, on=True) -> None:
        """True or 1: time every tile launch; k > 1: time every k-th; False: stop."""
        self.check(self._lib.mrpop_profile_enable(self._h, int(on)))

    def profile_read(self) -> "KernelProfile":
        p = _KernelProfile()
        self.check(self._lib.mrpop_profile_read(self._h, C.byref(p)))
        return KernelProfile(p.launches, p.kernel_ms, p.states_checked, p.edge_states,
                             dict(zip(WORK_NAMES, list(p.work))), p.grid_blocks, p.block_threads,
                             p.timed_launches)


class Scene:
    """Arms and obstacles uploaded to the device (``mrpop_scene_create``).

    ``scene`` is a ``workloads.Scene``-like object with ``models`` (each with
    dh, q_lo, q_hi, sphere_link, sphere_xyzr), ``base_tf`` (R x 12),
    ``env_spheres`` (N x 4) and ``env_boxes`` (N x 6)."""

    def __init__(self, ctx: Context, scene):
        self.ctx = ctx
        self.src = scene
        keep = []
        robots = (_Robot * len(scene.models))()
        for i, m in enumerate(scene.models):
            arrs = [np.ascontiguousarray(m.dh, np.float32), np.ascontiguousarray(m.q_lo, np.float32),
                    np.ascontiguousarray(m.q_hi, np.float32),
                    np.ascontiguousarray(np.asarray(scene.base_tf, np.float32).reshape(-1, 12)[i]),
                    np.ascontiguousarray(m.sphere_link, np.int32), np.ascontiguousarray(m.sphere_xyzr, np.float32)]
            keep.extend(arrs)
            robots[i] = _Robot(m.dh.shape[0], arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                               arrs[3].ctypes.data, m.sphere_xyzr.shape[0], arrs[4].ctypes.data, arrs[5].ctypes.data)
        es = np.ascontiguousarray(np.asarray(scene.env_spheres, np.float32).reshape(-1, 4))
        eb = np.ascontiguousarray(np.asarray(scene.env_boxes, np.float32).reshape(-1, 6))
        keep.extend([es, eb])
        env = _Env(es.shape[0], es.ctypes.data if es.size else None, eb.shape[0], eb.ctypes.data if eb.size else None)
        h = C.c_void_p()
        ctx.check(ctx._lib.mrpop_scene_create(ctx.handle, robots, len(scene.models), C.byref(env), C.byref(h)))
        self._h = h
        self.dof = int(ctx._lib.mrpop_scene_dof(h))
        self.total_spheres = int(ctx._lib.mrpop_scene_total_spheres(h))
        self.n_robots = len(scene.models)

    @property
    def handle(self):
        return self._h

    @property
    def obstacle_clusters(self) -> int:
        """Clusters of the two-level coarse filter (0: one level)."""
        return int(self.ctx._lib.mrpop_scene_obstacle_clusters(self._h))

    TILE_MODES = {"auto": 0, "lds": 1, "scalar": 2}

    def set_tile_mode(self, mode: str):
        """Where the validation kernel reads the coarse rows: "auto", "lds"
        or "scalar" (performance only)."""
        self.ctx.check(self.ctx._lib.mrpop_scene_set_tile_mode(self._h, self.TILE_MODES[mode]))

    @property
    def tile_mode(self) -> str:
        v = int(self.ctx._lib.mrpop_scene_tile_mode(self._h))
        return {b: a for a, b in self.TILE_MODES.items()}[v]

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.mrpop_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def fk_spheres(self, q, out=None):
        """World spheres (n_cfg, S_total, 4) float32 on the device."""
        torch = _torch()
        qd = self.ctx.to_device(q, torch.float32).reshape(-1, self.dof)
        n = qd.shape[0]
        if out is None:
            out = torch.empty((n, self.total_spheres, 4), dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(self.ctx._lib.mrpop_fk_spheres(self.ctx.handle, self._h, qd.data_ptr(), n, out.data_ptr(),
                                                      self.ctx.stream()))
        return out

    def validate_edges(self, qa, qb, resolution: float, n_states=None, out=None, stats: bool = False):
        """Edge-valid bits (uint8, 1 = free) on the device; with stats=True
        also returns a ValidateStats (the call then waits for the stream)."""
        return self._validate(self.ctx._lib.mrpop_validate_edges, qa, qb, resolution, n_states, out, stats)

    def validate_edges_noalloc(self, qa, qb, resolution: float, n_states=None, out=None, stats: bool = False):
        """As validate_edges, through mrpop_validate_edges_noalloc (the
        library's fixed device array instead of the context's scratch; at most
        MRPOP_NOALLOC_MAX_EDGES edges)."""
        return self._validate(self.ctx._lib.mrpop_validate_edges_noalloc, qa, qb, resolution, n_states, out, stats)

    def validate_counted(self, qa, qb, n_states, out=None, stats: bool = False):
        """mrpop_validate_counted: at most MRPOP_COUNTED_MAX_EDGES edges with
        the caller's state counts (n <= 0: invalid, unchecked), one launch."""
        fn = self.ctx._lib.mrpop_validate_counted
        return self._validate(lambda c, h, a, b, E, _res, ns, o, st, s: fn(c, h, a, b, E, ns, o, st, s),
                              qa, qb, 1.0, n_states, out, stats)

    def _validate(self, fn, qa, qb, resolution, n_states, out, stats):
        torch = _torch()
        a = self.ctx.to_device(qa, torch.float32).reshape(-1, self.dof)
        b = self.ctx.to_device(qb, torch.float32).reshape(-1, self.dof)
        if a.shape != b.shape:
            raise ValueError("qa and qb differ in shape")
        E = a.shape[0]
        ns = None if n_states is None else self.ctx.to_device(n_states, torch.int32).reshape(E)
        if out is None:
            out = torch.empty(E, dtype=torch.uint8, device=self.ctx.device)
        st = _ValidateStats()
        self.ctx.check(fn(
            self.ctx.handle, self._h, a.data_ptr(), b.data_ptr(), E, float(resolution),
            None if ns is None else ns.data_ptr(), out.data_ptr(), C.byref(st) if stats else None,
            self.ctx.stream()))
        if stats:
            return out, ValidateStats(st.edge_states, st.states_checked, st.edges_invalid, st.nonfinite_edges,
                                      st.tiles, dict(zip(WORK_NAMES, list(st.work))))
        return out

    def sample(self, q_start, q_goal, root, c_best: float, seed: int, round_: int, n: int, first: int = 0):
        """Candidate samples (q [n, D], c [n]) of one round on the device."""
        torch = _torch()
        qs = self.ctx.to_device(q_start, torch.float32).reshape(self.dof)
        qg = self.ctx.to_device(q_goal, torch.float32).reshape(self.dof)
        rt = self.ctx.to_device(root, torch.float32).reshape(self.dof)
        out_q = torch.empty((n, self.dof), dtype=torch.float32, device=self.ctx.device)
        out_c = torch.empty(n, dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(self.ctx._lib.mrpop_sample(self.ctx.handle, self._h, qs.data_ptr(), qg.data_ptr(), rt.data_ptr(),
                                                  float(c_best), seed & 0xFFFFFFFFFFFFFFFF, round_, first, n,
                                                  out_q.data_ptr(), out_c.data_ptr(), self.ctx.stream()))
        return out_q, out_c

    def extend(self, near_idx, q_rand, c_rand, tree_q, tree_g, tree_vid, rm_vertices, rm_rowptr, rm_col,
               resolution: float = 0.05) -> dict:
        """mrpop_extend (ORACLE_AOX of one round) on host arrays: near_idx [n],
        q_rand [n][D], c_rand [n] or None, tree_q [D][cap] (SoA), tree_g [cap],
        tree_vid [R][cap], rm_vertices [R][rm_cap][8], rm_rowptr
        [R][rm_cap + 1], rm_col [R][col_cap].  Returns host arrays q_new,
        vid_new [R][n], g_new, alive, edge_a, edge_b, n_states."""
        torch = _torch()
        dev = self.ctx.device
        f32, i32 = torch.float32, torch.int32
        near = self.ctx.to_device(np.asarray(near_idx, np.int32), i32)
        n = int(near.numel())
        qr = self.ctx.to_device(q_rand, f32).reshape(n, self.dof)
        cr = None if c_rand is None else self.ctx.to_device(c_rand, f32).reshape(n)
        tq = self.ctx.to_device(tree_q, f32)
        tg = self.ctx.to_device(tree_g, f32)
        tv = self.ctx.to_device(tree_vid, i32)
        rv = self.ctx.to_device(rm_vertices, f32)
        rp = self.ctx.to_device(rm_rowptr, i32)
        rc = self.ctx.to_device(rm_col, i32)
        R = int(tv.shape[0])
        out = dict(q_new=torch.empty((n, self.dof), dtype=f32, device=dev),
                   vid_new=torch.empty((R, n), dtype=i32, device=dev),
                   g_new=torch.empty(n, dtype=f32, device=dev),
                   alive=torch.empty(n, dtype=torch.uint8, device=dev),
                   edge_a=torch.empty((n, self.dof), dtype=f32, device=dev),
                   edge_b=torch.empty((n, self.dof), dtype=f32, device=dev),
                   n_states=torch.empty(n, dtype=i32, device=dev))
        b = _ExtendBatch(n, near.data_ptr(), qr.data_ptr(), None if cr is None else cr.data_ptr(), tq.data_ptr(),
                         tg.data_ptr(), tv.data_ptr(), int(tq.shape[1]), rv.data_ptr(), rp.data_ptr(),
                         rc.data_ptr(), int(rv.shape[1]), int(rc.shape[1]), float(resolution),
                         out["q_new"].data_ptr(), out["vid_new"].data_ptr(), out["g_new"].data_ptr(),
                         out["alive"].data_ptr(), out["edge_a"].data_ptr(), out["edge_b"].data_ptr(),
                         out["n_states"].data_ptr())
        self.ctx.check(self.ctx._lib.mrpop_extend(self.ctx.handle, self._h, C.byref(b), self.ctx.stream()))
        return {k: v.cpu().numpy() for k, v in out.items()}

    def plan(self, q_start, q_goal, path_cap: int = 4096, raise_on_error: bool = True, **params) -> "PlanResult":
        """mrpop_plan on host start/goal; keyword arguments override the
        defaults of mrpop_plan_params."""
        lib = self.ctx._lib
        pp = PlanParams()
        lib.mrpop_plan_params_default(C.byref(pp))
        for k, v in params.items():
            if not hasattr(pp, k):
                raise KeyError(k)
            setattr(pp, k, v)
        qs = np.ascontiguousarray(q_start, np.float32).reshape(self.dof)
        qg = np.ascontiguousarray(q_goal, np.float32).reshape(self.dof)
        path = np.zeros((max(1, path_cap), self.dof), np.float32)
        plen = C.c_int32(0)
        cost = C.c_float(0)
        st = _PlanStats()
        rc = lib.mrpop_plan(self.ctx.handle, self._h, qs.ctypes.data, qg.ctypes.data, C.byref(pp), path.ctypes.data,
                            path_cap, C.byref(plen), C.byref(cost), C.byref(st))
        stats = {k: getattr(st, k) for k, _ in _PlanStats._fields_ if k != "costs"}
        stats["costs"] = list(st.costs[:st.n_costs])
        stats["path_len"] = plen.value
        name = STATUS_NAMES.get(rc, str(rc))
        if rc != 0 and raise_on_error:
            raise MrpopError(rc, lib.mrpop_last_error(self.ctx.handle).decode())
        return PlanResult(name, path[:plen.value].copy() if rc == 0 else None, float(cost.value), stats)

    def set_env(self, env_spheres, env_boxes):
        """mrpop_scene_set_env: replace the obstacles (N x 4 spheres, N x 6
        boxes); the arms stay."""
        es = np.ascontiguousarray(np.asarray(env_spheres, np.float32).reshape(-1, 4))
        eb = np.ascontiguousarray(np.asarray(env_boxes, np.float32).reshape(-1, 6))
        env = _Env(es.shape[0], es.ctypes.data if es.size else None, eb.shape[0], eb.ctypes.data if eb.size else None)
        self.ctx.check(self.ctx._lib.mrpop_scene_set_env(self._h, C.byref(env)))

    def replan(self, q_start, q_goal, prev_path=None, path_cap: int = 4096, raise_on_error: bool = True, **params):
        """mrpop_replan: one replanning tick from the previous path (kept as
        the incumbent when it is still free and runs start -> goal).  Returns
        (PlanResult, kept)."""
        lib = self.ctx._lib
        pp = PlanParams()
        lib.mrpop_plan_params_default(C.byref(pp))
        for k, v in params.items():
            if not hasattr(pp, k):
                raise KeyError(k)
            setattr(pp, k, v)
        qs = np.ascontiguousarray(q_start, np.float32).reshape(self.dof)
        qg = np.ascontiguousarray(q_goal, np.float32).reshape(self.dof)
        prev = None if prev_path is None else np.ascontiguousarray(prev_path, np.float32).reshape(-1, self.dof)
        path = np.zeros((max(1, path_cap), self.dof), np.float32)
        plen = C.c_int32(0)
        cost = C.c_float(0)
        kept = C.c_int32(0)
        st = _PlanStats()
        rc = lib.mrpop_replan(self.ctx.handle, self._h, qs.ctypes.data, qg.ctypes.data, C.byref(pp),
                              prev.ctypes.data if prev is not None else None, 0 if prev is None else len(prev),
                              path.ctypes.data, path_cap, C.byref(plen), C.byref(cost), C.byref(st), C.byref(kept))
        stats = {k: getattr(st, k) for k, _ in _PlanStats._fields_ if k != "costs"}
        stats["costs"] = list(st.costs[:st.n_costs])
        stats["path_len"] = plen.value
        name = STATUS_NAMES.get(rc, str(rc))
        if rc != 0 and raise_on_error:
            raise MrpopError(rc, lib.mrpop_last_error(self.ctx.handle).decode())
        return PlanResult(name, path[:plen.value].copy() if rc == 0 else None, float(cost.value), stats), \
            bool(kept.value)

    def plan_with_history(self, q_start, q_goal, max_entries: int = 64, max_waypoints: int = 65536,
                          path_cap: int = 4096, raise_on_error: bool = True, roadmaps: bool = False, **params):
        """mrpop_plan_with_history: the plan's result and its incumbents,
        cheapest first (at most max_entries entries and max_waypoints rows),
        plus the number of incumbents found.  roadmaps=True also returns each
        waypoint's roadmap vertices (Incumbent.vertex_ids) and the arms'
        final roadmaps in stats["roadmaps"]: [(vertices [n][7], edges [m][2])]."""
        lib = self.ctx._lib
        pp = PlanParams()
        lib.mrpop_plan_params_default(C.byref(pp))
        for k, v in params.items():
            if not hasattr(pp, k):
                raise KeyError(k)
            setattr(pp, k, v)
        qs = np.ascontiguousarray(q_start, np.float32).reshape(self.dof)
        qg = np.ascontiguousarray(q_goal, np.float32).reshape(self.dof)
        path = np.zeros((max(1, path_cap), self.dof), np.float32)
        plen = C.c_int32(0)
        cost = C.c_float(0)
        st = _PlanStats()
        wp = np.zeros((max(1, max_waypoints), self.dof), np.float32)
        off = np.zeros(max_entries + 1, np.int32)
        costs = np.zeros(max(1, max_entries), np.float32)
        found_s = np.zeros(max(1, max_entries), np.float64)
        found_r = np.zeros(max(1, max_entries), np.int32)
        R = self.n_robots
        vids = np.zeros((max(1, max_waypoints), R), np.int32)
        rm_cap = int(params.get("max_roadmap_nodes", pp.max_roadmap_nodes))
        rm_v = np.zeros((R, rm_cap, 8), np.float32) if roadmaps else None
        rm_e = np.zeros((R, rm_cap * 32, 2), np.int32) if roadmaps else None
        h = _PlanHistory(wp.ctypes.data, max_waypoints, off.ctypes.data, costs.ctypes.data, found_s.ctypes.data,
                         found_r.ctypes.data, max_entries, 0, 0, vids.ctypes.data if roadmaps else None,
                         rm_v.ctypes.data if roadmaps else None, rm_e.ctypes.data if roadmaps else None,
                         rm_cap if roadmaps else 0, rm_cap * 32 if roadmaps else 0)
        rc = lib.mrpop_plan_with_history(self.ctx.handle, self._h, qs.ctypes.data, qg.ctypes.data, C.byref(pp),
                                         path.ctypes.data, path_cap, C.byref(plen), C.byref(cost), C.byref(st),
                                         C.byref(h))
        stats = {k: getattr(st, k) for k, _ in _PlanStats._fields_ if k != "costs"}
        stats["costs"] = list(st.costs[:st.n_costs])
        stats["path_len"] = plen.value
        name = STATUS_NAMES.get(rc, str(rc))
        if rc != 0 and raise_on_error:
            raise MrpopError(rc, lib.mrpop_last_error(self.ctx.handle).decode())
        hist = [Incumbent(wp[off[k]:off[k + 1]].copy(), float(costs[k]), float(found_s[k]), int(found_r[k]),
                          vids[off[k]:off[k + 1]].copy() if roadmaps else None)
                for k in range(h.n_written)]
        if roadmaps:
            stats["roadmaps"] = [(rm_v[r, :min(h.rm_n_vertices[r], rm_cap), :7].copy(),
                                  rm_e[r, :min(h.rm_n_edges[r], rm_cap * 32)].copy()) for r in range(R)]
        return PlanResult(name, path[:plen.value].copy() if rc == 0 else None, float(cost.value), stats), hist, \
            h.n_entries

    def states_free(self, q) -> np.ndarray:
        """Host bool per composite state (True = collision-free)."""
        qd = self.ctx.to_device(q, _torch().float32).reshape(-1, self.dof)
        return self.validate_edges(qd, qd, 1.0).cpu().numpy().astype(bool)


class Server:
    """Continuous-batching planning server (mrpop_server_*): requests are
    queued, admitted by slots and device memory, and run with their device
    work merged; results are kept per ticket."""

    def __init__(self, ctx: "Context", max_slots: int = 64, mem_budget_bytes: int = 0):
        self.ctx = ctx
        cfg = _ServerConfig(max_slots, mem_budget_bytes)
        h = C.c_void_p()
        ctx.check(ctx._lib.mrpop_server_create(ctx.handle, C.byref(cfg), C.byref(h)))
        self._h = h
        self._dof = {}

    def submit(self, scene: "Scene", q_start, q_goal, **params) -> int:
        lib = self.ctx._lib
        pp = PlanParams()
        lib.mrpop_plan_params_default(C.byref(pp))
        for k, v in params.items():
            if not hasattr(pp, k):
                raise KeyError(k)
            setattr(pp, k, v)
        qs = np.ascontiguousarray(q_start, np.float32).reshape(scene.dof)
        qg = np.ascontiguousarray(q_goal, np.float32).reshape(scene.dof)
        t = C.c_int64(0)
        self.ctx.check(lib.mrpop_server_submit(self._h, scene.handle, qs.ctypes.data, qg.ctypes.data,
                                               C.byref(pp), C.byref(t)))
        self._dof[t.value] = scene.dof
        return t.value

    def _result(self, ticket: int, r: "_ServerResult") -> dict:
        out = {k: getattr(r, k) for k, _ in _ServerResult._fields_ if k != "stats"}
        out["status"] = STATUS_NAMES.get(r.status, str(r.status))
        st = {k: getattr(r.stats, k) for k, _ in _PlanStats._fields_ if k != "costs"}
        st["costs"] = list(r.stats.costs[:r.stats.n_costs])
        out["stats"] = st
        out["path"] = None
        if r.status == 0:
            path = np.zeros((max(1, r.path_len), self._dof[ticket]), np.float32)
            self.ctx.check(self.ctx._lib.mrpop_server_path(self._h, ticket, path.ctypes.data, r.path_len))
            out["path"] = path[:r.path_len]
        return out

    def poll(self, ticket: int) -> dict:
        r = _ServerResult()
        self.ctx.check(self.ctx._lib.mrpop_server_poll(self._h, ticket, C.byref(r)))
        return self._result(ticket, r)

    def wait(self, ticket: int, timeout_s: float = 60.0) -> dict:
        r = _ServerResult()
        self.ctx.check(self.ctx._lib.mrpop_server_wait(self._h, ticket, timeout_s, C.byref(r)))
        return self._result(ticket, r)

    def release(self, ticket: int) -> None:
        self.ctx.check(self.ctx._lib.mrpop_server_release(self._h, ticket))
        self._dof.pop(ticket, None)

    def stats(self) -> dict:
        st = _ServerStats()
        self.ctx.check(self.ctx._lib.mrpop_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def clock(self) -> float:
        return float(self.ctx._lib.mrpop_server_clock(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.mrpop_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
