"""Seeded synthetic inputs for the MR. POP hot path.

This module builds robot models, obstacle scenes, composite edge batches and
planning problems from integer seeds.  It is shared by the HIP library's tests
and benchmark and by the CPU oracle, and it holds none of the method's
arithmetic: no kinematics, no collision predicate, no sampling rule of the
planner.  Where a planning problem needs collision-free start and goal states,
the caller passes a ``checker`` (the oracle in tests, the GPU library in the
benchmark) and this module only keeps or redraws what the checker rejects.

The paper evaluates on multi-Franka benchmark sets (Sec. Experiments,
"Methodology") that are not available here; the recipes below stand in for
them with the same robot class (7-DoF Franka-like arms), team sizes and
clutter levels.

Conventions
-----------
* A robot model is a serial chain in Craig's modified Denavit-Hartenberg
  convention: row j of ``dh`` is (a_{j-1}, d_j, alpha_{j-1}, theta_off_j).
* Link 0 is the base link (fixed to the base frame), link j >= 1 moves with
  joint j.  Each collision sphere names its link and its link-local centre.
* ``base_tf`` rows are row-major 3x4 [R | t] world-from-base transforms.
* A composite configuration concatenates the robots' joint vectors in robot
  order (Sec. Problem Setup).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

F32 = np.float32

# ---------------------------------------------------------------------------
# Robot models
# ---------------------------------------------------------------------------


@dataclass
class RobotModel:
    name: str
    dh: np.ndarray            # (nj, 4) float32 modified DH rows
    q_lo: np.ndarray          # (nj,) float32
    q_hi: np.ndarray          # (nj,) float32
    sphere_link: np.ndarray   # (S,) int32, 0..nj
    sphere_xyzr: np.ndarray   # (S, 4) float32, link-local centre + radius

    @property
    def n_joints(self) -> int:
        return int(self.dh.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_xyzr.shape[0])


# Franka Panda kinematic table (manufacturer documentation), modified DH.
PANDA_DH = np.array(
    [
        [0.0, 0.333, 0.0, 0.0],
        [0.0, 0.0, -math.pi / 2, 0.0],
        [0.0, 0.316, math.pi / 2, 0.0],
        [0.0825, 0.0, math.pi / 2, 0.0],
        [-0.0825, 0.384, -math.pi / 2, 0.0],
        [0.0, 0.0, math.pi / 2, 0.0],
        [0.088, 0.0, math.pi / 2, 0.0],
    ],
    dtype=F32,
)
PANDA_Q_LO = np.array([-2.8973, -1.7628, -2.8973, -3.0718, -2.8973, -0.0175, -2.8973], dtype=F32)
PANDA_Q_HI = np.array([2.8973, 1.7628, 2.8973, -0.0698, 2.8973, 3.7525, 2.8973], dtype=F32)

# Fixed geometric segment of each link in its own frame: from the link origin
# to the next joint's origin, written out by hand from the table above
# (link 7 runs 0.107 m to the flange plus 0.10 m of hand along its z axis).
# Links 1 and 5 have zero length; their spheres sit on the joint axis,
# spread +-0.06 m along the local z axis like a joint housing.
_PANDA_SEGMENTS = [
    ((0.0, 0.0, 0.0), (0.0, 0.0, 0.333)),
    ((0.0, 0.0, -0.06), (0.0, 0.0, 0.06)),
    ((0.0, 0.0, 0.0), (0.0, -0.316, 0.0)),
    ((0.0, 0.0, 0.0), (0.0825, 0.0, 0.0)),
    ((0.0, 0.0, 0.0), (-0.0825, 0.384, 0.0)),
    ((0.0, 0.0, -0.06), (0.0, 0.0, 0.06)),
    ((0.0, 0.0, 0.0), (0.088, 0.0, 0.0)),
    ((0.0, 0.0, 0.0), (0.0, 0.0, 0.207)),
]
PANDA_COUNTS = {20: [2, 1, 3, 2, 4, 1, 3, 4], 59: [6, 4, 8, 5, 12, 4, 8, 12]}


def panda_like(n_spheres: int = 59) -> RobotModel:
    """Procedural Franka-like arm with 20 or 59 spheres.

    Link l carries k_l spheres spaced evenly along its segment (both ends
    included when k_l >= 2, the midpoint when k_l == 1).  Radii fall linearly
    with the link index from 0.08 m (link 0) to 0.04 m (link 7).
    """
    counts = PANDA_COUNTS[n_spheres]
    links, xyzr = [], []
    for l, (k, (p0, p1)) in enumerate(zip(counts, _PANDA_SEGMENTS)):
        rad = 0.08 - 0.04 * l / 7.0
        for i in range(k):
            t = 0.5 if k == 1 else i / (k - 1)
            links.append(l)
            xyzr.append([p0[0] + t * (p1[0] - p0[0]), p0[1] + t * (p1[1] - p0[1]),
                         p0[2] + t * (p1[2] - p0[2]), rad])
    return RobotModel(
        name=f"panda_like_{n_spheres}",
        dh=PANDA_DH.copy(),
        q_lo=PANDA_Q_LO.copy(),
        q_hi=PANDA_Q_HI.copy(),
        sphere_link=np.array(links, dtype=np.int32),
        sphere_xyzr=np.array(xyzr, dtype=F32),
    )


def planar_two_link(l1: float = 0.6, l2: float = 0.4, radius: float = 0.05) -> RobotModel:
    """Planar 2R arm in the base x-y plane: joint 1 at the base origin, joint 2
    at distance l1 along link 1's x axis, one tool sphere at l2 along link 2's
    x axis and one sphere at the middle of link 1."""
    dh = np.array([[0.0, 0.0, 0.0, 0.0], [l1, 0.0, 0.0, 0.0]], dtype=F32)
    return RobotModel(
        name="planar_2link",
        dh=dh,
        q_lo=np.array([-math.pi, -math.pi], dtype=F32),
        q_hi=np.array([math.pi, math.pi], dtype=F32),
        sphere_link=np.array([1, 2], dtype=np.int32),
        sphere_xyzr=np.array([[0.5 * l1, 0.0, 0.0, radius], [l2, 0.0, 0.0, radius]], dtype=F32),
    )


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------


def base_transform(x: float, y: float, yaw: float, z: float = 0.0) -> np.ndarray:
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([c, -s, 0.0, x, s, c, 0.0, y, 0.0, 0.0, 1.0, z], dtype=F32)


@dataclass
class Scene:
    models: List[RobotModel]
    base_tf: np.ndarray                   # (R, 12) float32
    env_spheres: np.ndarray               # (Ns, 4) float32
    env_boxes: np.ndarray                 # (Nb, 6) float32: lo xyz, hi xyz
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_robots(self) -> int:
        return len(self.models)

    @property
    def joint_offsets(self) -> np.ndarray:
        return np.cumsum([0] + [m.n_joints for m in self.models]).astype(np.int64)

    @property
    def dof(self) -> int:
        return int(sum(m.n_joints for m in self.models))

    @property
    def q_lo(self) -> np.ndarray:
        return np.concatenate([m.q_lo for m in self.models]).astype(F32)

    @property
    def q_hi(self) -> np.ndarray:
        return np.concatenate([m.q_hi for m in self.models]).astype(F32)

    def with_env(self, spheres: np.ndarray, boxes: np.ndarray) -> "Scene":
        return Scene(self.models, self.base_tf, np.asarray(spheres, F32).reshape(-1, 4),
                     np.asarray(boxes, F32).reshape(-1, 6), self.name, dict(self.meta))

    def fingerprint(self) -> str:
        import hashlib
        h = hashlib.sha256()
        for m in self.models:
            for a in (m.dh, m.q_lo, m.q_hi, m.sphere_link, m.sphere_xyzr):
                h.update(np.ascontiguousarray(a).tobytes())
        for a in (self.base_tf, self.env_spheres, self.env_boxes):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def ring_bases(n_robots: int, radius: float, offset: float = 0.0) -> np.ndarray:
    """Bases evenly spaced on a circle (the first at angle `offset`), each
    yawed to face the centre."""
    out = []
    for i in range(n_robots):
        ang = offset + 2.0 * math.pi * i / n_robots
        out.append(base_transform(radius * math.cos(ang), radius * math.sin(ang), ang + math.pi))
    return np.stack(out).astype(F32)


def ring_radius_for_spacing(n_robots: int, spacing: float) -> float:
    if n_robots == 2:
        return 0.5 * spacing
    return spacing / (2.0 * math.sin(math.pi / n_robots))


def _rand_spheres(rng, n, lo, hi, rmin=0.05, rmax=0.15):
    c = rng.uniform(lo, hi, size=(n, 3))
    r = rng.uniform(rmin, rmax, size=(n, 1))
    return np.concatenate([c, r], axis=1).astype(F32)


def _rand_boxes(rng, n, lo, hi, smin=0.05, smax=0.3):
    c = rng.uniform(lo, hi, size=(n, 3))
    half = 0.5 * rng.uniform(smin, smax, size=(n, 3))
    return np.concatenate([c - half, c + half], axis=1).astype(F32)


def scene_c1(seed: int) -> Scene:
    """2 arms x 20 spheres, bases 1.0 m apart facing each other; 16 random
    obstacle spheres r ~ U(0.05, 0.15) m in a 1.5 m cube."""
    rng = np.random.default_rng([1, seed])
    m = panda_like(20)
    bases = np.stack([base_transform(-0.5, 0.0, 0.0), base_transform(0.5, 0.0, math.pi)])
    sph = _rand_spheres(rng, 16, [-0.75, -0.75, 0.0], [0.75, 0.75, 1.5])
    return Scene([m, m], bases, sph, np.zeros((0, 6), F32), name=f"c1/{seed}")


def scene_single(seed: int) -> Scene:
    """One arm x 59 spheres at the origin (the direct-mode workload: no
    roadmaps, the search in the arm's own joint space); 12 spheres and 12
    axis-aligned cuboids around it in [-0.9, 0.9]^2 x [0, 1.2]."""
    rng = np.random.default_rng([6, seed])
    lo, hi = [-0.9, -0.9, 0.0], [0.9, 0.9, 1.2]
    return Scene([panda_like(59)], base_transform(0.0, 0.0, 0.0)[None], _rand_spheres(rng, 12, lo, hi),
                 _rand_boxes(rng, 12, lo, hi), name=f"single/{seed}")


def scene_c2(seed: int) -> Scene:
    """4 arms x 59 spheres on a 1.2 m square facing the centre; 32 spheres and
    32 axis-aligned cuboids (sides U(0.05, 0.3) m)."""
    rng = np.random.default_rng([2, seed])
    m = panda_like(59)
    bases = np.stack([base_transform(x, y, math.atan2(-y, -x))
                      for x, y in ((0.6, 0.6), (-0.6, 0.6), (-0.6, -0.6), (0.6, -0.6))])
    lo, hi = [-1.2, -1.2, 0.0], [1.2, 1.2, 1.5]
    return Scene([m] * 4, bases, _rand_spheres(rng, 32, lo, hi), _rand_boxes(rng, 32, lo, hi),
                 name=f"c2/{seed}")


def shelf_grid_boxes(rng, levels=(0.2, 0.5, 0.8, 1.1), n_side=8, pitch=0.3, jitter=0.05):
    """One cuboid per cell of a levels x n_side x n_side lattice centred on the
    origin, sides U(0.05, 0.3) m, centre jittered by U(-jitter, jitter)."""
    out = []
    off = 0.5 * (n_side - 1) * pitch
    for z in levels:
        for i in range(n_side):
            for j in range(n_side):
                c = np.array([i * pitch - off, j * pitch - off, z]) + rng.uniform(-jitter, jitter, 3)
                half = 0.5 * rng.uniform(0.05, 0.3, 3)
                out.append(np.concatenate([c - half, c + half]))
    return np.array(out, dtype=F32)


def scene_c3(seed: int) -> Scene:
    """8 arms x 59 spheres on a circle of radius 1.5 m around a shared table;
    256 cuboids in a 4-level 8 x 8 shelf grid with 0.3 m pitch.  The ring
    starts at 22.5 degrees so that no base stands on a corner of the grid
    (the grid's corners lie on the circle at 45 + k 90 degrees)."""
    rng = np.random.default_rng([3, seed])
    m = panda_like(59)
    return Scene([m] * 8, ring_bases(8, 1.5, math.pi / 8), np.zeros((0, 4), F32), shelf_grid_boxes(rng),
                 name=f"c3/{seed}", meta={"grid": True})


def _mixed_obstacles(rng, n_obs, R, radius):
    span = radius + 0.9
    lo, hi = [-span, -span, 0.0], [span, span, 1.5]
    kinds = rng.random(n_obs) < 0.5
    sph = _rand_spheres(rng, int(kinds.sum()), lo, hi)
    box = _rand_boxes(rng, int((~kinds).sum()), lo, hi)
    return sph, box


def scene_c4(seed: int, index: int) -> Scene:
    """One instance of the 512-instance batch: R ~ U{2,3,4,6,8}, ring with
    about 1.1 m neighbour spacing, N_obs ~ U{16..256} spheres or cuboids."""
    rng = np.random.default_rng([4, seed, index])
    R = int(rng.choice([2, 3, 4, 6, 8]))
    n_obs = int(rng.integers(16, 257))
    radius = ring_radius_for_spacing(R, 1.0 if R == 2 else 1.1)
    m = panda_like(59)
    sph, box = _mixed_obstacles(rng, n_obs, R, radius)
    return Scene([m] * R, ring_bases(R, radius), sph, box, name=f"c4/{seed}/{index}")


def scene_c5(seed: int, index: int) -> Scene:
    """One served query: R ~ U{2..16}, N_obs ~ U{32..512} spheres or cuboids."""
    rng = np.random.default_rng([5, seed, index])
    R = int(rng.integers(2, 17))
    n_obs = int(rng.integers(32, 513))
    radius = ring_radius_for_spacing(R, 1.0 if R == 2 else 1.1)
    m = panda_like(59)
    sph, box = _mixed_obstacles(rng, n_obs, R, radius)
    return Scene([m] * R, ring_bases(R, radius), sph, box, name=f"c5/{seed}/{index}")


# ---------------------------------------------------------------------------
# Configurations and edge batches
# ---------------------------------------------------------------------------


def random_configs(scene: Scene, n: int, rng) -> np.ndarray:
    lo, hi = scene.q_lo.astype(np.float64), scene.q_hi.astype(np.float64)
    return (lo + rng.random((n, scene.dof)) * (hi - lo)).astype(F32)


def edge_batch(scene: Scene, n_edges: int, res: float, seed: int, n_min: int = 8,
               n_max: int = 64) -> tuple:
    """Random composite edges: q_a uniform in the joint limits, a direction
    with L-infinity norm 1, a target state count n ~ U{n_min..n_max}, and
    q_b = clip(q_a + (n - 1) * res * u)."""
    rng = np.random.default_rng([7, seed, scene.dof, n_edges])
    lo, hi = scene.q_lo.astype(np.float64), scene.q_hi.astype(np.float64)
    qa = lo + rng.random((n_edges, scene.dof)) * (hi - lo)
    u = rng.uniform(-1.0, 1.0, size=(n_edges, scene.dof))
    u /= np.abs(u).max(axis=1, keepdims=True)
    nt = rng.integers(n_min, n_max + 1, size=(n_edges, 1))
    qb = np.clip(qa + (nt - 1) * res * u, lo, hi)
    return qa.astype(F32), qb.astype(F32)


def edge_batch_near(scene: Scene, anchors: np.ndarray, n_edges: int, res: float, seed: int,
                    n_min: int = 8, n_max: int = 64, spread: float = 0.3) -> tuple:
    """Edges starting near given anchor configurations (e.g. known-free
    states), used to get batches with a sizeable fraction of free edges."""
    rng = np.random.default_rng([8, seed, scene.dof, n_edges])
    lo, hi = scene.q_lo.astype(np.float64), scene.q_hi.astype(np.float64)
    a = anchors[rng.integers(0, anchors.shape[0], n_edges)].astype(np.float64)
    qa = np.clip(a + rng.uniform(-spread, spread, size=a.shape), lo, hi)
    u = rng.uniform(-1.0, 1.0, size=qa.shape)
    u /= np.abs(u).max(axis=1, keepdims=True)
    nt = rng.integers(n_min, n_max + 1, size=(n_edges, 1))
    qb = np.clip(qa + (nt - 1) * res * u, lo, hi)
    return qa.astype(F32), qb.astype(F32)


# ---------------------------------------------------------------------------
# Planning problems
# ---------------------------------------------------------------------------

Checker = Callable[[Scene, np.ndarray], np.ndarray]  # (scene, qs[N, D]) -> bool[N] (True = free)


@dataclass
class Problem:
    scene: Scene
    q_start: np.ndarray
    q_goal: np.ndarray
    seed: int
    dropped_obstacles: int = 0


def make_problem(scene: Scene, seed: int, checker: Checker, max_config_tries: int = 4000,
                 max_obstacle_tries: int = 32) -> Problem:
    """Start and goal drawn uniformly in the joint limits until both are free
    of robot-robot contact; then every obstacle of ``scene`` that touches the
    start or the goal is redrawn (same kind and size law, new centre) up to
    ``max_obstacle_tries`` times, and dropped if it still does."""
    rng = np.random.default_rng([9, seed, scene.dof])
    bare = scene.with_env(np.zeros((0, 4), F32), np.zeros((0, 6), F32))
    ends = []
    for _ in range(max_config_tries):
        qs = random_configs(scene, 16, rng)
        ok = checker(bare, qs)
        ends.extend(qs[np.nonzero(ok)[0]])
        if len(ends) >= 2:
            break
    if len(ends) < 2:
        raise RuntimeError(f"no robot-robot free start/goal found for {scene.name}")
    q_start, q_goal = np.asarray(ends[0], F32), np.asarray(ends[1], F32)
    pair = np.stack([q_start, q_goal])

    spheres_out, boxes_out, dropped = [], [], 0
    sph, box = scene.env_spheres, scene.env_boxes
    none4, none6 = np.zeros((0, 4), F32), np.zeros((0, 6), F32)
    for s in sph:
        cand = s.copy()
        for t in range(max_obstacle_tries):
            if checker(scene.with_env(cand[None], none6), pair).all():
                spheres_out.append(cand)
                break
            cand = s.copy()
            cand[:3] = s[:3] + rng.uniform(-0.3, 0.3, 3).astype(F32) * (1 + t / 8)
        else:
            dropped += 1
    for b in box:
        cand = b.copy()
        for t in range(max_obstacle_tries):
            if checker(scene.with_env(none4, cand[None]), pair).all():
                boxes_out.append(cand)
                break
            shift = rng.uniform(-0.05, 0.05, 3).astype(F32) * (1 + t)
            cand = np.concatenate([b[:3] + shift, b[3:] + shift]).astype(F32)
        else:
            dropped += 1
    env_s = np.array(spheres_out, F32).reshape(-1, 4)
    env_b = np.array(boxes_out, F32).reshape(-1, 6)
    return Problem(scene.with_env(env_s, env_b), q_start, q_goal, seed, dropped)


# ---------------------------------------------------------------------------
# Served-mode arrivals
# ---------------------------------------------------------------------------


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with seeded exponential gaps."""
    rng = np.random.default_rng([11, seed])
    gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * duration_s * 1.5) + 16)
    t = np.cumsum(gaps)
    return t[t < duration_s]


CONFIGS = {
    "c1": dict(desc="plan 2x7-DoF, 20 spheres/arm, 16 spheres, res 0.05", res=0.05),
    "c2": dict(desc="validate 4096 edges, 4x7-DoF, 59 spheres/arm, 32 spheres + 32 cuboids, res 0.05",
               res=0.05),
    "c3": dict(desc="8x7-DoF, 59 spheres/arm, 256 shelf-grid cuboids, res 0.02", res=0.02),
    "c4": dict(desc="512 instances, R in {2,3,4,6,8}, 16-256 obstacles", res=None),
    "c5": dict(desc="served, Poisson 200 q/s, R in 2..16, 32-512 obstacles", res=None),
}
