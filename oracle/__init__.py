"""Plain FP64 CPU oracle for the MR. POP hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  The arithmetic lives in
``mrpop_oracle.c`` (forward kinematics, signed margins, the coarse-to-fine
checker, NEAREST, the random stream and the informed sample) and in
``planner.py`` (the round-based planner); see those files for the paper
passages each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrpop_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")

BAND = 1e-5  # metres: |margin| below this is the boundary band


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math, no vector intrinsics)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm",
                               "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(C.Structure):
    _fields_ = [
        ("n_robots", C.c_int32),
        ("nj", C.c_void_p), ("q_off", C.c_void_p), ("dh", C.c_void_p), ("base", C.c_void_p),
        ("ns", C.c_void_p), ("s_off", C.c_void_p), ("s_link", C.c_void_p), ("s_xyzr", C.c_void_p),
        ("n_env_spheres", C.c_int32), ("env_s", C.c_void_p),
        ("n_env_boxes", C.c_int32), ("env_b", C.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        lib.orc_fk_spheres.argtypes = [P, P, I64, P]
        lib.orc_classify_edges.argtypes = [P, P, P, I64, C.c_float, P, P, P, C.c_int]
        lib.orc_validate_fast.argtypes = [P, P, P, I64, C.c_float, P, P, P, P, C.c_int, C.c_int]
        lib.orc_state_margins.argtypes = [P, P, I64, P]
        lib.orc_edge_nstates.argtypes = [P, P, C.c_int, C.c_float]
        lib.orc_edge_nstates.restype = I32
        lib.orc_nearest.argtypes = [P, P, I64, C.c_int, P, C.c_double, P]
        lib.orc_nearest.restype = I64
        lib.orc_nearest_batch.argtypes = [P, P, I64, C.c_int, P, P, I64, P]
        lib.orc_mix64.argtypes = [C.c_uint64]
        lib.orc_mix64.restype = C.c_uint64
        lib.orc_key.argtypes = [C.c_uint64] * 4
        lib.orc_key.restype = C.c_uint64
        lib.orc_u01.argtypes = [C.c_uint64, C.c_uint64]
        lib.orc_u01.restype = C.c_double
        lib.orc_u01_batch.argtypes = [C.c_uint64, I64, P]
        lib.orc_unit_ball.argtypes = [C.c_uint64, C.c_int, P]
        lib.orc_ellipsoid_map.argtypes = [C.c_int, P, P, C.c_double, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleScene:
    """Flattened copy of a ``workloads.Scene`` in the oracle's layout."""

    def __init__(self, scene):
        models = scene.models
        self.R = len(models)
        self.nj = np.array([m.n_joints for m in models], np.int32)
        self.q_off = np.concatenate([[0], np.cumsum(self.nj)[:-1]]).astype(np.int32)
        self.dh = np.ascontiguousarray(np.concatenate([m.dh for m in models]), np.float32)
        self.base = np.ascontiguousarray(scene.base_tf, np.float32).reshape(self.R, 12)
        self.ns = np.array([m.n_spheres for m in models], np.int32)
        self.s_off = np.concatenate([[0], np.cumsum(self.ns)[:-1]]).astype(np.int32)
        self.s_link = np.ascontiguousarray(np.concatenate([m.sphere_link for m in models]), np.int32)
        self.s_xyzr = np.ascontiguousarray(np.concatenate([m.sphere_xyzr for m in models]), np.float32)
        self.env_s = np.ascontiguousarray(scene.env_spheres, np.float32).reshape(-1, 4)
        self.env_b = np.ascontiguousarray(scene.env_boxes, np.float32).reshape(-1, 6)
        if self.env_s.shape[0] == 0:
            self.env_s = np.zeros((1, 4), np.float32)[:0]
        self.D = int(self.nj.sum())
        self.S = int(self.ns.sum())
        self._st = _Scene(self.R, _ptr(self.nj), _ptr(self.q_off), _ptr(self.dh), _ptr(self.base),
                          _ptr(self.ns), _ptr(self.s_off), _ptr(self.s_link), _ptr(self.s_xyzr),
                          int(scene.env_spheres.shape[0]), _ptr(self.env_s),
                          int(scene.env_boxes.shape[0]), _ptr(self.env_b))

    @property
    def ref(self):
        return C.byref(self._st)


def _scene(scene) -> OracleScene:
    return scene if isinstance(scene, OracleScene) else OracleScene(scene)


def _f32(a, D=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if D is not None:
        a = a.reshape(-1, D)
    return a


def fk_spheres(scene, q) -> np.ndarray:
    """World sphere centres and radii, shape (n_cfg, S_total, 4), float64."""
    sc = _scene(scene)
    q = _f32(q, sc.D)
    out = np.zeros((q.shape[0], sc.S, 4), np.float64)
    _load().orc_fk_spheres(sc.ref, _ptr(q), q.shape[0], _ptr(out))
    return out


def edge_nstates(qa, qb, res: float) -> np.ndarray:
    qa, qb = np.atleast_2d(_f32(qa)), np.atleast_2d(_f32(qb))
    lib = _load()
    return np.array([lib.orc_edge_nstates(_ptr(np.ascontiguousarray(qa[i])),
                                          _ptr(np.ascontiguousarray(qb[i])), qa.shape[1], res)
                     for i in range(qa.shape[0])], np.int32)


def classify_edges(scene, qa, qb, res: float, nstates=None, threads: int = 0):
    """Per edge: (n_states int32, minimum margin float64) over all pairs/states."""
    sc = _scene(scene)
    qa, qb = _f32(qa, sc.D), _f32(qb, sc.D)
    E = qa.shape[0]
    n = np.zeros(E, np.int32)
    m = np.zeros(E, np.float64)
    ns = None if nstates is None else np.ascontiguousarray(nstates, np.int32)
    th = threads or min(8, os.cpu_count() or 1)
    _load().orc_classify_edges(sc.ref, _ptr(qa), _ptr(qb), E, res, None if ns is None else _ptr(ns),
                               _ptr(n), _ptr(m), th)
    return n, m


COUNT_NAMES = ["states", "fk_robot", "coarse_env_sphere", "coarse_env_box", "coarse_rr",
               "fine_env_sphere", "fine_env_box", "fine_rr", "edges_invalid"]


def validate_fast(scene, qa, qb, res: float, nstates=None, early_exit: bool = True, threads: int = 1):
    """Coarse-to-fine checker.  Returns (valid uint8[E], n_states int32[E], counts dict)."""
    sc = _scene(scene)
    qa, qb = _f32(qa, sc.D), _f32(qb, sc.D)
    E = qa.shape[0]
    valid = np.zeros(E, np.uint8)
    n = np.zeros(E, np.int32)
    cnt = np.zeros(len(COUNT_NAMES), np.int64)
    ns = None if nstates is None else np.ascontiguousarray(nstates, np.int32)
    _load().orc_validate_fast(sc.ref, _ptr(qa), _ptr(qb), E, res, None if ns is None else _ptr(ns),
                              _ptr(valid), _ptr(n), _ptr(cnt), int(early_exit), max(1, threads))
    return valid, n, dict(zip(COUNT_NAMES, cnt.tolist()))


def state_margins(scene, q) -> np.ndarray:
    sc = _scene(scene)
    q = _f32(q, sc.D)
    out = np.zeros(q.shape[0], np.float64)
    _load().orc_state_margins(sc.ref, _ptr(q), q.shape[0], _ptr(out))
    return out


def states_free(scene, q) -> np.ndarray:
    """Checker for ``workloads.make_problem``: True where the state is free
    with margin at least the band (so that a single-precision checker agrees)."""
    return state_margins(scene, q) >= BAND


def classify(m: np.ndarray) -> np.ndarray:
    """+1 certainly free, -1 certainly colliding, 0 inside the band."""
    return np.where(m >= BAND, 1, np.where(m < -BAND, -1, 0)).astype(np.int8)


def nearest(V, g, q, c: float) -> int:
    V = np.ascontiguousarray(V, np.float32)
    g = np.ascontiguousarray(g, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    return int(_load().orc_nearest(_ptr(V), _ptr(g), V.shape[0], V.shape[1], _ptr(q), float(c), None))


def nearest_batch(V, g, Q, c) -> np.ndarray:
    V = np.ascontiguousarray(V, np.float32)
    g = np.ascontiguousarray(g, np.float32)
    Q = np.ascontiguousarray(Q, np.float32).reshape(-1, V.shape[1])
    cc = np.ascontiguousarray(np.broadcast_to(np.asarray(c, np.float64), (Q.shape[0],)))
    out = np.zeros(Q.shape[0], np.int64)
    _load().orc_nearest_batch(_ptr(V), _ptr(g), V.shape[0], V.shape[1], _ptr(Q), _ptr(cc), Q.shape[0],
                              _ptr(out))
    return out


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def key(seed: int, a: int, b: int, c: int) -> int:
    m = 0xFFFFFFFFFFFFFFFF
    return int(_load().orc_key(seed & m, a & m, b & m, c & m))


def u01(key_: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.float64)
    _load().orc_u01_batch(key_ & 0xFFFFFFFFFFFFFFFF, n, _ptr(out))
    return out


def unit_ball(key_: int, D: int) -> np.ndarray:
    out = np.zeros(D, np.float64)
    _load().orc_unit_ball(key_ & 0xFFFFFFFFFFFFFFFF, D, _ptr(out))
    return out


def ellipsoid_map(q_start, q_goal, c_best: float, x) -> np.ndarray:
    qs = np.ascontiguousarray(q_start, np.float32)
    qg = np.ascontiguousarray(q_goal, np.float32)
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(qs.shape[0], np.float64)
    _load().orc_ellipsoid_map(qs.shape[0], _ptr(qs), _ptr(qg), float(c_best), _ptr(x), _ptr(out))
    return out
