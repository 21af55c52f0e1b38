#!/usr/bin/env python3
"""Benchmark of the MR. POP hot path on one MI355X.

Workload (4 arms x 7-DoF, 59 spheres per arm, 32 spheres + 32 boxes,
0.05 rad resolution): every step validates two batches of 4096 composite
edges with ``mrpop_validate_edges`` -- one whose edges are all certainly free
(every state must be fully checked) and one drawn the same way without
selection (mostly colliding, early exit applies) -- and runs one full plan
(``mrpop_plan``: roadmaps, initial dRRT solve, AO-X improvement) between the
workload's start and goal with the step's seed.  Inputs sit in device memory
before the timed region.

Printed: one JSON line with composite edge-states validated per second over
the step (both batches and the plan's search), the plans' p50 time to first
solution, the roofline of the edge-validation tile kernels (the flop model's
flops for the states and links they evaluated, with the coarse stage at its
full table of every link against every obstacle, over their HIP-event time,
against the FP32 vector peak; beside it the same pricing of only the coarse
tests the kernels ran) and the oracle's CPU rate on a sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FIXTURE = os.path.join(ROOT, "tests", "golden", "c2_bench.json")
METRIC = "composite edge-states validated/sec + p50 time-to-solution; batched vs plain"
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 flop/clk)

# Algorithmic flops per operation (FMA = 2; add, sub, mul, min, max = 1),
# the flop model the roofline is priced with: a generic modified-DH joint
# (building its 3x4 transform and composing it onto the parent frame) 63; a
# point transform R p + t 18; a sphere-sphere test (3 sub, a squared norm,
# the squared radius sum) 10; a sphere-box test (2 sub and 2 max per axis,
# then the squared norm) 17.  The kernel's own joint step is cheaper (48:
# three frame rows at 16), so executed flops sit below these counts.
F_JOINT, F_XFORM, F_SS, F_SB = 63, 18, 10, 17

# Planner settings of the benchmark step (delta: per-arm roadmap radius in
# rad; P = candidates per round; the plan stops after max_iterations outer
# iterations or max_rounds rounds).
PLAN = dict(candidates=512, n_roadmap=32, delta=3.0, max_rounds=150, max_iterations=4)
# In the timed steps, every PROFILE_STRIDE-th tile launch carries the event
# pair that times it (an event-timed launch costs several us more dispatch;
# the work counters still cover every launch).
PROFILE_STRIDE = 8

# Time to solution on the 50 two-arm problems: the plain planner with a 5 s
# budget (first solution only for the time to solution; the whole budget on
# a few problems for the cost reached).  The oracle's planner runs the same
# round parameters.
C1_FIXTURE = os.path.join(ROOT, "tests", "golden", "c1_problems.json")
C1_PLAN = dict(candidates=128, n_roadmap=32, delta=3.0, max_rounds=100000, max_iterations=100000,
               time_budget_s=5.0)
C1_PLAN_ORACLE = dict(candidates=128, n_roadmap=32, delta=3.0, max_rounds=2000, max_iterations=100)
# the oracle is far slower than the GPU planner: its wall-clock cap per problem is larger
ORACLE_PLAN_BUDGET_S = 10.0

# The 8-arm shelf workload: validation batches (4096 certainly free, 4096
# unselected; 0.02 rad) and cost-bounded replanning for 30 s.
C3_FIXTURE = os.path.join(ROOT, "tests", "golden", "c3_bench.json")
C3_PLAN = dict(candidates=512, n_roadmap=32, delta=3.0, max_rounds=1000000, max_iterations=1000000,
               max_growth_rounds=24)

# HBM traffic of the tile kernels, from hardware counters (FETCH_SIZE and
# WRITE_SIZE per dispatch, scaled by what they read for a plain copy of known
# size).  The summary records a digest of the kernel sources it was taken on;
# when the sources differ, the figure no longer applies and is reported as null.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "validate_tiles_traffic_c2.md")
KERNEL_SOURCES = ("validate.hip", "device_common.h", "mrpop_internal.h")


def kernel_digest() -> str:
    """Digest of the kernel sources' code (comments and whitespace removed,
    so that only a change of code voids the recorded counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_30644_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def recorded_counters():
    """(fields, note) from the committed counter summary: bytes per tile-kernel
    launch and the FP32 flops the hardware issued per launch; fields is None
    when the summary is missing or was taken on other kernel sources."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None, "no counter summary"
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("` ")] = v.strip("` ")
    if fields.get("kernel_digest") != kernel_digest():
        return None, "counters were taken on other kernel sources"
    try:
        out = {k: float(fields[k]) for k in ("traffic_bytes_per_launch", "valu_fp32_flops_per_launch")}
    except (KeyError, ValueError):
        return None, "counter summary lacks its fields"
    return out, "FETCH_SIZE + WRITE_SIZE per launch, copy-calibrated"


def copy_probe(mib: int):
    """A plain device copy of `mib` MiB, three times: the calibration run of
    the traffic counters (each copy reads and writes `mib` MiB)."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 3}), flush=True)


def load_workload(path=FIXTURE, scene_fn="scene_c2"):
    import workloads as W
    d = json.load(open(path))
    sc = getattr(W, scene_fn)(d["scene_seed"]).with_env(np.array(d["env_spheres"], np.float32).reshape(-1, 4),
                                                        np.array(d["env_boxes"], np.float32).reshape(-1, 6))
    anchors = W.random_configs(sc, d["anchor_draws"], np.random.default_rng([d["anchor_seed"]]))
    anchors = anchors[np.array(d["anchor_free_idx"])]
    qa, qb = W.edge_batch_near(sc, anchors, d["pool"], d["resolution"], d["pool_seed"], d["n_min"], d["n_max"],
                               spread=d["spread"])
    free = np.array(d["free_edge_idx"])
    batches = {"free": (qa[free], qb[free]), "mixed": (qa[:4096], qb[:4096])}
    return sc, batches, d


def algorithmic_flops(work: dict, scene) -> float:
    """Flops of the operations the kernel executed, priced by the model above:
    chains (arm x state) of nj joints; coarse link centres (a transform each);
    coarse link-obstacle tests, a sphere test against an environment sphere
    and a sphere-box test against a box (split by the scene's obstacle
    counts); exact link-box tests; coarse link-link tests; and the fine
    tests, each a sphere transform plus its test."""
    nj = scene.models[0].n_joints
    ns, nb = int(scene.env_spheres.shape[0]), int(scene.env_boxes.shape[0])
    env_s = work["env_tests"] * (ns / (ns + nb) if ns + nb else 0.0)
    env_b = work["env_tests"] - env_s
    return (work["chains"] * nj * F_JOINT + work["links"] * F_XFORM + env_s * F_SS + env_b * F_SB
            + work["box_exact"] * F_SB + work["rr_coarse"] * F_SS + work["fine_sphere"] * (F_XFORM + F_SS)
            + work["fine_box"] * (F_XFORM + F_SB) + work["fine_rr"] * (F_XFORM + F_SS))


def full_table_flops(work: dict, scene) -> float:
    """Algorithmic flops of the flop model: the same pricing with the coarse
    environment stage counted as every evaluated link against every obstacle
    (the model's fixed part per state), where the kernel tests only the
    obstacles within each link's reach and, in some lists, clusters first."""
    n_obs = int(scene.env_spheres.shape[0]) + int(scene.env_boxes.shape[0])
    return algorithmic_flops(dict(work, env_tests=work["links"] * n_obs), scene)


def host_info() -> dict:
    """Host cores and CPU model of the machine the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model}


def checker_rate(scene, batches, res, target_s: float, threads: int) -> dict:
    """The oracle's coarse-to-fine checker (early exit) on a bounded sample of
    the same two batches, on `threads` host threads."""
    import oracle
    sc = oracle.OracleScene(scene)

    def run(k, passes=1):
        t0 = time.perf_counter()
        states = 0
        for _ in range(passes):
            for name in ("free", "mixed"):
                qa, qb = batches[name]
                _, n, _ = oracle.validate_fast(sc, qa[:k], qb[:k], res, threads=threads)
                states += int(n.sum())
        return states, time.perf_counter() - t0

    k, passes = 64, 1
    states, dt = run(k)
    print(f"[bench]   checker, {threads} thread(s): {k} edges x {passes} in {dt:.2f} s", file=sys.stderr, flush=True)
    while dt < target_s / 2:
        if k < 4096:
            k = min(4096, int(k * max(2.0, target_s / max(dt, 1e-3) / 2)))
        else:
            passes = max(passes + 1, int(passes * target_s / max(dt, 1e-3)))
        states, dt = run(k, passes)
        print(f"[bench]   checker, {threads} thread(s): {k} edges x {passes} in {dt:.2f} s",
              file=sys.stderr, flush=True)
    return {"value": states / dt, "unit": "edge-states/s", "cores": threads,
            "sample": f"{passes} pass(es) over the first {k} edges of each batch ({states} edge-states), "
                      f"FP64 coarse-to-fine checker with early exit, {dt:.1f} s"}


def oracle_planner_tts(n_seeds: int) -> dict:
    """The oracle's planner (Python rounds over the FP64 checker, one
    thread) on the first C1 problems, first solution only, with the GPU
    leg's round parameters: time to first solution and solve rate."""
    import workloads as W
    from oracle import planner as PL
    d = json.load(open(C1_FIXTURE))
    tts, ok = [], 0
    for j, pr in enumerate(d["problems"][:n_seeds]):
        sc = W.scene_c1(pr["seed"]).with_env(np.array(pr["env_spheres"], np.float32).reshape(-1, 4),
                                             np.array(pr["env_boxes"], np.float32).reshape(-1, 6))
        prm = PL.PlanParams(**dict(C1_PLAN_ORACLE, seed=pr["seed"], stop_at_first=True,
                                   time_budget_s=ORACLE_PLAN_BUDGET_S))
        t0 = time.perf_counter()
        r = PL.plan(sc, np.array(pr["q_start"], np.float32), np.array(pr["q_goal"], np.float32), prm)
        dt = time.perf_counter() - t0
        if r.status == "OK":
            ok += 1
            tts.append(dt)
        if (j + 1) % 10 == 0:
            print(f"[bench]   oracle planner: {j + 1} problems, {ok} solved", file=sys.stderr, flush=True)
    return {"problems": n_seeds, "solved": ok, "tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
            "threads": 1, "params": C1_PLAN_ORACLE, "budget_s": ORACLE_PLAN_BUDGET_S,
            "note": "wall time of oracle.planner.plan with stop_at_first (roadmaps, then the initial search)"}


def cpu_baseline(scene, batches, res, target_s: float, planner_seeds: int) -> dict:
    """The oracle on the host cores: its checker on all cores (at most 16
    threads, the host share of one GPU) and on one thread, and its planner
    on the first C1 problems."""
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    allc = checker_rate(scene, batches, res, target_s / 2, threads)
    one = checker_rate(scene, batches, res, target_s / 2, 1)
    out = {"value": allc["value"], "unit": "edge-states/s", "cores": threads, "kind": "oracle",
           "sample": allc["sample"], "single_thread": one, "host": host_info(),
           "note": "plain FP64 C checker without SIMD intrinsics, not a vectorised state of the art"}
    if planner_seeds > 0:
        out["planner_c1"] = oracle_planner_tts(planner_seeds)
    return out


def check_bits(free_bits: np.ndarray, mixed_bits: np.ndarray, fx: dict) -> dict:
    """The timed batches' bits against the oracle's classes stored in the
    fixture: every free-batch edge is certainly free; on the unselected
    batch every edge outside the band has the oracle's verdict."""
    cls = np.array(fx["mixed_first_4096_class"])
    certain = cls != 0
    bad_mixed = int((mixed_bits[certain] != (cls[certain] == 1)).sum())
    bad_free = int((free_bits != 1).sum())
    return {"free_mismatches": bad_free, "mixed_mismatches": bad_mixed, "mixed_band": int((~certain).sum()),
            "mixed_oracle_free": int((cls == 1).sum()), "ok": bad_free == 0 and bad_mixed == 0}


def c1_leg(ctx, n_problems: int, n_full: int) -> dict:
    """Time to first solution on the two-arm problems (one plan each, seed =
    problem seed, first solution only), and the cost reached after the whole
    5 s budget on the first n_full problems."""
    import workloads as W
    import paper_2609_30644_amd as M
    d = json.load(open(C1_FIXTURE))
    res = d["resolution"]
    probs = []
    for pr in d["problems"][:n_problems]:
        sc = W.scene_c1(pr["seed"]).with_env(np.array(pr["env_spheres"], np.float32).reshape(-1, 4),
                                             np.array(pr["env_boxes"], np.float32).reshape(-1, 6))
        probs.append((pr["seed"], M.Scene(ctx, sc), np.array(pr["q_start"], np.float32),
                      np.array(pr["q_goal"], np.float32)))
    _, s0, a0, b0 = probs[0]
    s0.plan(a0, b0, raise_on_error=False, resolution=res, **dict(C1_PLAN, seed=99, stop_at_first=1))  # warm
    tts, wall, solved = [], [], 0
    for seed, s, qs, qg in probs:
        t0 = time.perf_counter()
        r = s.plan(qs, qg, raise_on_error=False, resolution=res, **dict(C1_PLAN, seed=seed, stop_at_first=1))
        wall.append(time.perf_counter() - t0)
        if r.status == "OK":
            solved += 1
            tts.append(r.stats["time_to_first_s"])
    full = []
    for seed, s, qs, qg in probs[:n_full]:
        r = s.plan(qs, qg, raise_on_error=False, resolution=res, **dict(C1_PLAN, seed=seed))
        full.append({"seed": seed, "status": r.status, "first_cost": r.stats["costs"][0] if r.stats["costs"] else None,
                     "cost_at_budget": r.cost if r.status == "OK" else None, "improvements": r.stats["solutions"],
                     "rounds": r.stats["rounds"], "iterations": r.stats["iterations"],
                     "straight_line": float(np.linalg.norm(qg.astype(np.float64) - qs))})
    return {"problems": len(probs), "solved": solved, "solve_rate": solved / len(probs),
            "tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
            "tts_p90_ms": float(np.percentile(tts, 90)) * 1e3 if tts else None,
            "tts_max_ms": float(np.max(tts)) * 1e3 if tts else None,
            "plan_call_p50_ms": float(np.median(wall)) * 1e3, "params": C1_PLAN, "full_budget": full}


def batch_rooflines(ctx, scene, batches, fx, reps: int, out: dict):
    """Both 4096-edge batches of a fixture validated `reps` times each, alone:
    edge-states/s, the tile kernel's time and its roofline (flop model and
    executed), bits checked against the fixture.  Returns the device scene."""
    import torch
    import paper_2609_30644_amd as M
    res = float(fx["resolution"])
    s = M.Scene(ctx, scene)
    dev = {k: (ctx.to_device(a), ctx.to_device(b)) for k, (a, b) in batches.items()}
    outs = {k: torch.empty(a.shape[0], dtype=torch.uint8, device=ctx.device) for k, (a, _) in dev.items()}
    for k, (a, b) in dev.items():
        _, st = s.validate_edges(a, b, res, out=outs[k], stats=True)  # warm, and the nominal states
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            s.validate_edges(a, b, res, out=outs[k])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        executed = algorithmic_flops(prof.work, scene) / (prof.kernel_ms * 1e-3) / 1e12
        model = full_table_flops(prof.work, scene) / (prof.kernel_ms * 1e-3) / 1e12
        out[k] = {"edges": int(a.shape[0]), "edge_states": st.edge_states, "reps": reps,
                  "edge_states_per_s": st.edge_states * reps / dt,
                  "kernel_us": prof.kernel_ms * 1e3 / max(1, prof.launches),
                  "achieved_tflops": model, "frac": model / PEAK_FP32_TFLOPS,
                  "executed_tflops": executed, "executed_frac": executed / PEAK_FP32_TFLOPS}
    out["bits"] = check_bits(outs["free"].cpu().numpy(), outs["mixed"].cpu().numpy(), fx)
    return s


def c2_batches_leg(ctx, reps: int) -> dict:
    """The step's two C2 batches timed alone (the certainly-free one is the
    batch whose every state must be evaluated)."""
    scene, batches, fx = load_workload()
    out = {"workload": "4 arms x 7-DoF (59 spheres/arm), 32 spheres + 32 boxes, res 0.05 rad"}
    batch_rooflines(ctx, scene, batches, fx, reps, out)
    return out


C3_COST_MARKS_S = (0.01, 0.1, 1.0, 5.0, 10.0, 30.0)


def c3_leg(ctx, reps: int, plan_s: float, plan_seeds: int = 1) -> dict:
    """The 8-arm shelf workload: both 4096-edge batches validated `reps`
    times (edge-states/s, the tile kernel's time and algorithmic flops, bits
    checked against the fixture), then plans with a wall-clock budget (time
    to first solution, cost after each improvement, cost at the end): seed 0
    in full, and with plan_seeds > 1 the time-to-solution median and the
    cost's median and quartiles at fixed times over seeds 0..plan_seeds-1."""
    scene, batches, fx = load_workload(C3_FIXTURE, "scene_c3")
    res = float(fx["resolution"])
    out = {"workload": "8 arms x 7-DoF (59 spheres/arm) on a 3 m circle, 256 shelf boxes, res 0.02 rad"}
    s = batch_rooflines(ctx, scene, batches, fx, reps, out)
    if plan_s > 0:
        qs, qg = np.array(fx["q_start"], np.float32), np.array(fx["q_goal"], np.float32)
        prm = dict(C3_PLAN, seed=0, resolution=res, time_budget_s=plan_s)
        t0 = time.perf_counter()
        r, hist, n = s.plan_with_history(qs, qg, max_entries=64, max_waypoints=65536, raise_on_error=False, **prm)
        out["plan"] = {"status": r.status, "wall_s": time.perf_counter() - t0,
                       "tts_ms": r.stats["time_to_first_s"] * 1e3 if r.stats["time_to_first_s"] >= 0 else None,
                       "cost": r.cost if r.status == "OK" else None,
                       "cost_vs_time": sorted([(h.found_s, h.cost) for h in hist]),
                       "rounds": r.stats["rounds"], "iterations": r.stats["iterations"],
                       "edge_states": r.stats["edge_states"], "roadmap_vertices": r.stats["roadmap_vertices"],
                       "straight_line": float(np.linalg.norm(qg.astype(np.float64) - qs)),
                       "params": dict(prm, time_budget_s=plan_s)}
        if plan_seeds > 1:
            runs = [(r, out["plan"]["cost_vs_time"])]
            for seed in range(1, plan_seeds):
                print(f"[bench] c3 plan seed {seed}", file=sys.stderr, flush=True)
                r2, h2, _ = s.plan_with_history(qs, qg, max_entries=64, max_waypoints=65536, raise_on_error=False,
                                                **dict(prm, seed=seed))
                runs.append((r2, sorted([(h.found_s, h.cost) for h in h2])))
            tts = [x.stats["time_to_first_s"] * 1e3 for x, _ in runs if x.stats["time_to_first_s"] >= 0]
            at = {}
            for t in C3_COST_MARKS_S:
                if t > plan_s:
                    continue
                c = [min([cost for found, cost in cv if found <= t], default=math.inf) for _, cv in runs]
                q1, q2, q3 = np.percentile(c, [25, 50, 75])
                at[str(t)] = {"median": float(q2), "q1": float(q1), "q3": float(q3),
                              "solved": int(np.isfinite(c).sum())}
            out["plan_seeds"] = {"seeds": plan_seeds, "solved": sum(x.status == "OK" for x, _ in runs),
                                 "tts_p50_ms": float(np.median(tts)) if tts else None,
                                 "tts_max_ms": float(max(tts)) if tts else None,
                                 "cost_at_s": at, "note": "same problem, planner seeds 0..seeds-1; "
                                 "cost inf before a seed's first solution"}
    return out


BATCH_FIXTURE = os.path.join(ROOT, "tests", "golden", "c4_batch.json")
# Planner settings of the batched comparison (round budgets, so that the
# batch and the plain runs compute the same paths).
BATCH_PLAN = dict(candidates=64, n_roadmap=16, delta=3.0, max_rounds=200, max_iterations=3, max_tree_nodes=8192,
                  max_roadmap_nodes=2048)


def batched_vs_plain(ctx, n_inst: int) -> dict:
    """The batched workload (independent instances with 2-8 arms, 16-256
    obstacles, uneven edge resolutions) planned once as one mrpop_plan_batch
    call and once as sequential mrpop_plan calls; both timed on the wall
    clock, results compared instance by instance."""
    import paper_2609_30644_amd as M
    import workloads as W
    d = json.load(open(BATCH_FIXTURE))
    inst = d["instances"][:n_inst]
    jobs = []
    for i, x in enumerate(inst):
        R = x["n_robots"]
        sc = W.Scene([W.panda_like(59)] * R, np.array(x["bases"], np.float32).reshape(R, 12),
                     np.array(x["env_spheres"], np.float32).reshape(-1, 4),
                     np.array(x["env_boxes"], np.float32).reshape(-1, 6))
        jobs.append((M.Scene(ctx, sc), np.array(x["q_start"], np.float32), np.array(x["q_goal"], np.float32),
                     dict(BATCH_PLAN, seed=i, resolution=x["resolution"])))
    ctx.plan_batch(jobs[:4])  # warm-up (kernel loading, buffers)
    t = time.perf_counter()
    got, bst = ctx.plan_batch(jobs)
    t_batch = time.perf_counter() - t
    plain = []
    t = time.perf_counter()
    for s, qs, qg, prm in jobs:
        plain.append(s.plan(qs, qg, raise_on_error=False, **prm))
    t_plain = time.perf_counter() - t
    same = all(g.status == p.status and g.cost == p.cost and
               (g.path is None and p.path is None or (g.path is not None and p.path is not None and
                                                      np.array_equal(g.path, p.path)))
               for g, p in zip(got, plain))
    states = sum(g.stats["edge_states"] + g.stats["roadmap_edge_states"] for g in got)
    tts_b = [g.stats["time_to_first_s"] for g in got if g.stats["time_to_first_s"] >= 0]
    tts_p = [p.stats["time_to_first_s"] for p in plain if p.stats["time_to_first_s"] >= 0]
    return {"instances": len(jobs), "arms": sorted(set(x["n_robots"] for x in inst)),
            "batched_wall_s": t_batch, "plain_wall_s": t_plain, "speedup": t_plain / t_batch,
            "identical_to_plain": bool(same), "solved": sum(g.status == "OK" for g in got),
            "edge_states": int(states), "batched_edge_states_per_s": states / t_batch,
            "plain_edge_states_per_s": states / t_plain,
            "tts_p50_ms_batched": float(np.median(tts_b)) * 1e3 if tts_b else None,
            "tts_p50_ms_plain_alone": float(np.median(tts_p)) * 1e3 if tts_p else None,
            "merged_launches": bst["launches"], "flushes": bst["flushes"], "params": BATCH_PLAN}


SERVE_FIXTURE = os.path.join(ROOT, "tests", "golden", "c5_served.json")
# Per-query settings of the served workload: first solution within a round
# budget and a 2 s deadline (counted from admission).
SERVE_PLAN = dict(candidates=64, n_roadmap=16, delta=3.0, resolution=0.05, max_rounds=200, max_iterations=4,
                  stop_at_first=1, max_tree_nodes=8192, max_roadmap_nodes=2048, time_budget_s=2.0)


# AO-X against the rewiring baseline on the 4-arm workload (the paper's
# cost-vs-time comparison): the same roadmap and round settings, a wall-clock
# budget per run, several seeds.
AODRRT_PLAN = dict(candidates=128, n_roadmap=32, delta=3.0, max_rounds=1000000, max_iterations=1000000,
                   max_tree_nodes=262144)


def aox_vs_aodrrt(s, q_start, q_goal, res: float, seconds: float, seeds: int) -> dict:
    """Incumbent cost against time for MR. POP (AO-X) and ao-dRRT (rewire=1)
    on the 4-arm problem: per seed and mode the (time, cost) of every
    incumbent; summaries at fixed times (median over seeds of the best cost
    found by then) and the first-solution times."""
    marks = [t for t in (0.05, 0.1, 0.25, 0.5, 1.0, 2.0, 5.0, 10.0, 30.0) if t <= seconds]
    out = {"seconds": seconds, "seeds": seeds, "marks_s": marks, "params": AODRRT_PLAN}
    for mode, rw in (("aox", 0), ("aodrrt", 1)):
        runs = []
        for seed in range(seeds):
            r, hist, _ = s.plan_with_history(q_start, q_goal, max_entries=64, max_waypoints=65536, raise_on_error=False,
                                             resolution=res, time_budget_s=seconds, rewire=rw,
                                             **dict(AODRRT_PLAN, seed=seed))
            curve = sorted((h.found_s, h.cost) for h in hist)
            runs.append({"seed": seed, "status": r.status, "tts_s": r.stats["time_to_first_s"],
                         "final_cost": r.cost if r.status == "OK" else None, "curve": curve,
                         "rounds": r.stats["rounds"], "iterations": r.stats["iterations"],
                         "rewired": r.stats["rewired"], "wall_s": r.stats["total_time_s"]})
        at = {}
        for t in marks:
            best = [min([c for ts, c in x["curve"] if ts <= t], default=float("inf")) for x in runs]
            at[str(t)] = float(np.median(best))
        tts = [x["tts_s"] for x in runs if x["tts_s"] >= 0]
        out[mode] = {"median_cost_at": at, "tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
                     "solved": len(tts), "runs": runs}
    return out


def history_leg(s, q_start, q_goal, res: float, n: int) -> dict:
    """Incumbent-history export: the same n plans (seeds 0..n-1) with and
    without mrpop_plan_with_history; entries found and written, and the time
    of both."""
    t_with, t_without, entries, written, same = 0.0, 0.0, [], [], True
    for seed in range(n):
        kw = dict(PLAN, seed=seed, resolution=res)
        t0 = time.perf_counter()
        a = s.plan(q_start, q_goal, raise_on_error=False, **kw)
        t1 = time.perf_counter()
        b, hist, found = s.plan_with_history(q_start, q_goal, max_entries=16, max_waypoints=4096,
                                             raise_on_error=False, **kw)
        t2 = time.perf_counter()
        t_without += t1 - t0
        t_with += t2 - t1
        entries.append(found)
        written.append(len(hist))
        same = same and a.status == b.status and a.cost == b.cost and (not hist or hist[0].cost == b.cost)
    return {"plans": n, "incumbents_mean": float(np.mean(entries)), "incumbents_max": int(np.max(entries)),
            "written_mean": float(np.mean(written)), "ms_per_plan_with": t_with * 1e3 / n,
            "ms_per_plan_without": t_without * 1e3 / n, "same_plans": bool(same),
            "buffers": {"max_entries": 16, "max_waypoints": 4096}}


def unprofiled_leg(s, q_start, q_goal, res: float, n: int) -> dict:
    """The timed region times every tile launch with a HIP event pair, which
    adds about 12-18 us of dispatch cost per launch.  The same plans (seeds
    0..n-1, as the first timed steps) without events show the planner's own
    latency."""
    ts, tts, states = [], [], 0
    for seed in range(n):
        t0 = time.perf_counter()
        r = s.plan(q_start, q_goal, raise_on_error=False, resolution=res, **dict(PLAN, seed=seed))
        ts.append(time.perf_counter() - t0)
        if r.stats["time_to_first_s"] >= 0:
            tts.append(r.stats["time_to_first_s"])
        states += r.stats["edge_states"]
    return {"plans": n, "mean_plan_ms": float(np.mean(ts)) * 1e3,
            "tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
            "plan_edge_states_per_s": states / float(np.sum(ts))}


SINGLE_FIXTURE = os.path.join(ROOT, "tests", "golden", "single_arm.json")
# Direct mode (one arm, no roadmaps): extension length `step` (rad).
DIRECT_PLAN = dict(candidates=128, max_rounds=150, max_iterations=4, direct=1, step=1.0)


def direct_leg(ctx, res: float) -> dict:
    """Direct mode on the single-arm problems (one plan each, seed = index):
    solve rate, time to first solution, final cost, edge-states/s."""
    import workloads as W
    import paper_2609_30644_amd as M
    d = json.load(open(SINGLE_FIXTURE))
    tts, costs, straight, states, wall, ok = [], [], [], 0, 0.0, 0
    for i, pr in enumerate(d["problems"]):
        sc = W.scene_single(pr["scene_seed"]).with_env(np.array(pr["env_spheres"], np.float32).reshape(-1, 4),
                                                        np.array(pr["env_boxes"], np.float32).reshape(-1, 6))
        s = M.Scene(ctx, sc)
        qs, qg = np.array(pr["q_start"], np.float32), np.array(pr["q_goal"], np.float32)
        s.plan(qs, qg, raise_on_error=False, resolution=res, **dict(DIRECT_PLAN, seed=10_000 + i))  # warm
        t0 = time.perf_counter()
        r = s.plan(qs, qg, raise_on_error=False, resolution=res, **dict(DIRECT_PLAN, seed=i))
        wall += time.perf_counter() - t0
        states += r.stats["edge_states"]
        if r.status == "OK":
            ok += 1
            tts.append(r.stats["time_to_first_s"])
            costs.append(r.cost)
            straight.append(float(np.linalg.norm(qg.astype(np.float64) - qs)))
    return {"problems": len(d["problems"]), "solved": ok,
            "tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
            "mean_plan_ms": wall * 1e3 / len(d["problems"]),
            "cost_over_straight_line_median": float(np.median(np.array(costs) / np.array(straight))) if costs else None,
            "edge_states_per_s": states / wall if wall > 0 else None, "params": DIRECT_PLAN}


REPLAN_FIXTURE = os.path.join(ROOT, "tests", "golden", "replan_ticks.json")
# One replanning tick: roadmaps regrown each tick, a short search budget.
REPLAN_PLAN = dict(candidates=128, n_roadmap=32, delta=3.0, max_rounds=40, max_iterations=2)


def replan_leg(ctx, res: float) -> dict:
    """Replanning amid a moving sphere (two arms of the C1 kind): per tick,
    mrpop_scene_set_env with the sphere's new position, then mrpop_replan
    from the previous tick's path; latency per tick, ticks whose previous
    path stayed free (kept), solved ticks and costs."""
    import workloads as W
    import paper_2609_30644_amd as M
    d = json.load(open(REPLAN_FIXTURE))
    sph0 = np.array(d["env_spheres"], np.float32).reshape(-1, 4)
    box0 = np.array(d["env_boxes"], np.float32).reshape(-1, 6)
    sc = W.scene_c1(0).with_env(sph0, box0)
    qs, qg = np.array(d["q_start"], np.float32), np.array(d["q_goal"], np.float32)
    s = M.Scene(ctx, sc)
    s.plan(qs, qg, raise_on_error=False, resolution=res, **dict(REPLAN_PLAN, seed=99))  # warm
    prev, lat, env_ms, kept_n, solved, costs = None, [], [], 0, 0, []
    for t, c in enumerate(d["ticks"]):
        t0 = time.perf_counter()
        s.set_env(np.concatenate([sph0, [[*c, d["radius"]]]]).astype(np.float32), box0)
        t1 = time.perf_counter()
        r, kept = s.replan(qs, qg, prev, raise_on_error=False, resolution=res, **dict(REPLAN_PLAN, seed=t))
        t2 = time.perf_counter()
        env_ms.append((t1 - t0) * 1e3)
        lat.append((t2 - t0) * 1e3)
        kept_n += int(kept)
        if r.status == "OK":
            solved += 1
            costs.append(r.cost)
            prev = r.path
    return {"ticks": len(d["ticks"]), "solved": solved, "kept_previous": kept_n,
            "tick_ms_p50": float(np.median(lat)), "tick_ms_p99": float(np.percentile(lat, 99)),
            "set_env_ms_p50": float(np.median(env_ms)), "mean_cost": float(np.mean(costs)) if costs else None,
            "params": REPLAN_PLAN}


def served(ctx, rate_hz: float, duration_s: float, slots: int, mem_gb: float) -> dict:
    """Poisson arrivals of queries (2-16 arms, 32-512 obstacles) submitted to
    a continuous-batching server on the wall clock; latency is arrival ->
    result on the server's clock."""
    import paper_2609_30644_amd as M
    import workloads as W
    d = json.load(open(SERVE_FIXTURE))
    probs = []
    for x in d["instances"]:
        R = x["n_robots"]
        sc = W.Scene([W.panda_like(59)] * R, np.array(x["bases"], np.float32).reshape(R, 12),
                     np.array(x["env_spheres"], np.float32).reshape(-1, 4),
                     np.array(x["env_boxes"], np.float32).reshape(-1, 6))
        probs.append((M.Scene(ctx, sc), np.array(x["q_start"], np.float32), np.array(x["q_goal"], np.float32)))
    arrivals = W.poisson_arrivals(rate_hz, duration_s, 0)
    if not len(arrivals):
        return {"rate_hz": rate_hz, "duration_s": duration_s, "queries": 0}
    srv = M.Server(ctx, max_slots=slots, mem_budget_bytes=int(mem_gb * (1 << 30)))
    # warm-up request (kernel loading), not counted
    s0, a0, b0 = probs[0]
    srv.wait(srv.submit(s0, a0, b0, **dict(SERVE_PLAN, seed=10 ** 6)), 60.0)
    t0 = srv.clock()
    tickets = []
    for i, a in enumerate(arrivals):
        while srv.clock() - t0 < a:
            time.sleep(0.0002)
        s, qs, qg = probs[i % len(probs)]
        tickets.append(srv.submit(s, qs, qg, **dict(SERVE_PLAN, seed=i)))
    res = [srv.wait(t, 600.0) for t in tickets]
    st = srv.stats()
    srv.close()
    done = [(r, a, i) for i, (r, a) in enumerate(zip(res, arrivals)) if r["status"] != "PENDING"]
    lat = np.array([r["t_done"] - (t0 + a) for r, a, _ in done])
    lat_ok = np.array([r["t_done"] - (t0 + a) for r, a, _ in done if r["status"] == "OK"])
    queue = np.array([r["t_admit"] - (t0 + a) for r, a, _ in done])
    span = max(r["t_done"] for r, _, _ in done) - t0 if done else float("nan")
    states = sum(r["stats"]["edge_states"] + r["stats"]["roadmap_edge_states"] for r, _, _ in done)
    by_arms = {}
    for r, _, i in done:
        R = probs[i % len(probs)][0].n_robots
        n, ok = by_arms.get(R, (0, 0))
        by_arms[R] = (n + 1, ok + (r["status"] == "OK"))
    pct = lambda x, q: float(np.percentile(x, q)) * 1e3 if len(x) else None
    return {"rate_hz": rate_hz, "duration_s": duration_s, "queries": len(tickets), "completed": len(done),
            "solved": int(len(lat_ok)),
            "statuses": {k: sum(r["status"] == k for r, _, _ in done) for k in sorted(set(r["status"] for r, _, _ in done))},
            "solve_rate_by_arms": {str(k): {"queries": v[0], "solved": v[1]} for k, v in sorted(by_arms.items())},
            "latency_p50_ms": pct(lat, 50), "latency_p99_ms": pct(lat, 99),
            "solved_latency_p50_ms": pct(lat_ok, 50), "solved_latency_p99_ms": pct(lat_ok, 99),
            "queue_wait_p50_ms": pct(queue, 50), "queue_wait_p99_ms": pct(queue, 99),
            "queries_per_s": len(done) / span, "edge_states_per_s": states / span,
            "sustained": bool(len(done) / span >= 0.9 * rate_hz and st["max_queue_len"] <= max(8, 0.1 * len(tickets))),
            "slots": slots, "mem_budget_gb": mem_gb, "max_running": st["max_running"],
            "max_queue_len": st["max_queue_len"], "peak_reserved_gb": st["peak_reserved_bytes"] / (1 << 30),
            "rejected": st["rejected"], "merged_launches": st["launches"], "flushes": st["flushes"],
            "params": SERVE_PLAN}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plan", action="store_true", help="validation batches only")
    ap.add_argument("--batch-instances", type=int, default=512,
                    help="instances of the batched-vs-plain comparison (0: skip)")
    ap.add_argument("--no-direct", dest="direct", action="store_false",
                    help="skip the direct-mode (single-arm, no roadmap) leg")
    ap.add_argument("--no-replan", dest="replan", action="store_false",
                    help="skip the replanning (moving obstacle) leg")
    ap.add_argument("--no-unprofiled", dest="unprofiled", action="store_false",
                    help="skip replaying the first timed plans without per-launch events")
    ap.add_argument("--history-plans", type=int, default=10,
                    help="plans timed with and without the incumbent-history export (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="arrival window of the served run (0: skip)")
    ap.add_argument("--serve-sweep", type=str, default="25,50,100",
                    help="comma-separated lower arrival rates, 2 s each, to find the rate one GPU sustains")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate of the served run")
    ap.add_argument("--serve-slots", type=int, default=128)
    ap.add_argument("--serve-mem-gb", type=float, default=96.0)
    ap.add_argument("--c1-problems", type=int, default=50,
                    help="two-arm problems of the time-to-solution leg (0: skip)")
    ap.add_argument("--c1-full", type=int, default=2, help="of those, plans run for the whole 5 s budget")
    ap.add_argument("--c3-reps", type=int, default=10, help="repetitions of each 8-arm batch (0: skip the leg)")
    ap.add_argument("--c3-plan-seconds", type=float, default=30.0, help="budget of the 8-arm plan (0: skip)")
    ap.add_argument("--c3-plan-seeds", type=int, default=1, help="8-arm plans over seeds 0..N-1 (N > 1: statistics)")
    ap.add_argument("--aodrrt-seconds", type=float, default=5.0,
                    help="budget of each AO-X and ao-dRRT run of the cost-vs-time comparison (0: skip)")
    ap.add_argument("--aodrrt-seeds", type=int, default=3)
    ap.add_argument("--oracle-planner-seeds", type=int, default=50,
                    help="two-arm problems planned by the oracle in the CPU baseline (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB on the device three times (traffic-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the hot path is measured on a single GPU; run with --gpus 1"}))
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return

    import torch

    import paper_2609_30644_amd as M

    scene, batches, fx = load_workload()
    res = float(fx["resolution"])
    print(f"[bench] workload loaded: free {batches['free'][0].shape}, mixed {batches['mixed'][0].shape}",
          file=sys.stderr, flush=True)
    ctx = M.Context(0)
    s = M.Scene(ctx, scene)
    dev = {k: (ctx.to_device(a), ctx.to_device(b)) for k, (a, b) in batches.items()}
    outs = {k: torch.empty(a.shape[0], dtype=torch.uint8, device=ctx.device) for k, (a, _) in dev.items()}
    nominal = {}
    for k, (a, b) in dev.items():
        _, st = s.validate_edges(a, b, res, out=outs[k], stats=True)
        nominal[k] = st.edge_states
    states_per_step = sum(nominal.values())

    q_start = np.array(fx["q_start"], np.float32)
    q_goal = np.array(fx["q_goal"], np.float32)
    plans = []

    def step(seed):
        for k, (a, b) in dev.items():
            s.validate_edges(a, b, res, out=outs[k])
        if not args.no_plan:
            plans.append(s.plan(q_start, q_goal, raise_on_error=False, resolution=res, **dict(PLAN, seed=seed)))

    for w in range(args.warmup):
        step(10_000 + w)
    torch.cuda.synchronize()
    plans.clear()
    ctx.profile_enable(PROFILE_STRIDE)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    bits = check_bits(outs["free"].cpu().numpy(), outs["mixed"].cpu().numpy(), fx)

    # average duration of the timed launches; flops per launch over every launch
    launch_s = prof.kernel_ms * 1e-3 / max(1, prof.timed_launches)
    flops = full_table_flops(prof.work, scene)
    achieved = flops / max(1, prof.launches) / launch_s / 1e12
    executed_flops = algorithmic_flops(prof.work, scene)
    executed = executed_flops / max(1, prof.launches) / launch_s / 1e12
    counted, traffic_note = recorded_counters()
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": counted["traffic_bytes_per_launch"] if counted else None, "traffic_unit": "bytes/launch",
                "traffic_note": traffic_note,
                "valu_fp32_flops_per_launch": counted["valu_fp32_flops_per_launch"] if counted else None,
                "kernel": "validate_tiles_kernel + validate_small_kernel + validate_segments_kernel", "launches": prof.launches,
                "avg_launch_us": launch_s * 1e6, "timed_launches": prof.timed_launches,
                "timed_every": PROFILE_STRIDE,
                "flops_per_launch": flops / max(1, prof.launches),
                "grid": [prof.grid_blocks, prof.block_threads], "work": prof.work,
                "flops_note": "flop model per evaluated state: chains, link centres, every link against every "
                              "obstacle, the masked link pairs and the executed fine tests",
                "executed": {"achieved": executed, "frac": executed / PEAK_FP32_TFLOPS,
                             "flops_per_launch": executed_flops / max(1, prof.launches),
                             "note": "the same pricing on the coarse tests the kernel ran: only the obstacles "
                                     "within each link's reach"}}
    plan_states = sum(p.stats["edge_states"] for p in plans)
    value = (states_per_step * args.steps + plan_states) / elapsed
    tts = [p.stats["time_to_first_s"] for p in plans if p.stats["time_to_first_s"] >= 0]
    line = {
        "metric": METRIC, "value": value, "unit": "edge-states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "4 arms x 7-DoF (59 spheres/arm), 32 spheres + 32 boxes, res 0.05 rad; "
                               "per step 4096 certainly-free + 4096 unselected composite edges",
                   "edge_states_per_step": states_per_step, "edges_per_step": 8192,
                   "free_batch_states": nominal["free"], "mixed_batch_states": nominal["mixed"]},
        "roofline": roofline,
        "states_checked_frac": prof.states_checked / max(1, prof.edge_states),
        "bits_vs_oracle": bits,
    }
    if plans:
        line["plan"] = {"tts_p50_ms": float(np.median(tts)) * 1e3 if tts else None,
                        "tts_p90_ms": float(np.percentile(tts, 90)) * 1e3 if tts else None,
                        "solve_rate": len(tts) / len(plans),
                        "median_cost": float(np.median([p.cost for p in plans if p.status == "OK"] or [np.nan])),
                        "mean_plan_ms": float(np.mean([p.stats["total_time_s"] for p in plans])) * 1e3,
                        "edge_states_per_plan": plan_states / len(plans),
                        "params": PLAN}
        line["config"]["plan"] = "one mrpop_plan per step, seed = step index"
        if args.unprofiled:
            n_same = min(10, len(plans))
            line["plan_unprofiled"] = unprofiled_leg(s, q_start, q_goal, res, n_same)
            line["plan_unprofiled"]["timed_mean_plan_ms_same_seeds"] = float(
                np.mean([p.stats["total_time_s"] for p in plans[:n_same]])) * 1e3
    if args.c1_problems > 0:
        print("[bench] two-arm time to solution", file=sys.stderr, flush=True)
        line["c1"] = c1_leg(ctx, args.c1_problems, args.c1_full)
    if args.c3_reps > 0:
        print("[bench] eight-arm shelf", file=sys.stderr, flush=True)
        line["c3"] = c3_leg(ctx, args.c3_reps, args.c3_plan_seconds, args.c3_plan_seeds)
    if args.c3_reps > 0:
        print("[bench] four-arm batches alone", file=sys.stderr, flush=True)
        line["c2_batches"] = c2_batches_leg(ctx, args.c3_reps)
    if args.direct:
        print("[bench] direct mode", file=sys.stderr, flush=True)
        line["direct"] = direct_leg(ctx, res)
    if args.replan:
        print("[bench] replanning", file=sys.stderr, flush=True)
        line["replan"] = replan_leg(ctx, res)
    if args.aodrrt_seconds > 0 and args.aodrrt_seeds > 0:
        print("[bench] AO-X against ao-dRRT", file=sys.stderr, flush=True)
        line["aox_vs_aodrrt"] = aox_vs_aodrrt(s, q_start, q_goal, res, args.aodrrt_seconds, args.aodrrt_seeds)
    if plans and args.history_plans > 0:
        print("[bench] incumbent history", file=sys.stderr, flush=True)
        line["history"] = history_leg(s, q_start, q_goal, res, args.history_plans)
    if args.batch_instances > 0:
        print("[bench] batched vs plain", file=sys.stderr, flush=True)
        line["batched"] = batched_vs_plain(ctx, args.batch_instances)
    if args.serve_seconds > 0:
        print("[bench] served", file=sys.stderr, flush=True)
        line["served"] = served(ctx, args.serve_rate, args.serve_seconds, args.serve_slots, args.serve_mem_gb)
        sweep = [float(x) for x in args.serve_sweep.split(",") if x.strip()]
        if sweep:
            runs = [served(ctx, r, 2.0, args.serve_slots, args.serve_mem_gb) for r in sweep]
            line["served_sweep"] = [{k: x.get(k) for k in ("rate_hz", "queries", "completed", "solved",
                                                            "queries_per_s", "latency_p50_ms", "latency_p99_ms",
                                                            "solved_latency_p50_ms", "solved_latency_p99_ms",
                                                            "queue_wait_p50_ms", "max_queue_len", "sustained")}
                                    for x in runs]
            ok = [x["rate_hz"] for x in runs + [line["served"]] if x.get("sustained")]
            line["served_max_sustained_rate_hz"] = max(ok) if ok else None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(scene, batches, res, args.cpu_seconds, args.oracle_planner_seeds)
    print(json.dumps(line), flush=True)
    if not bits["ok"] or not line.get("c3", {}).get("bits", {"ok": True})["ok"]:
        print("[bench] timed bits disagree with the oracle's classes", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
