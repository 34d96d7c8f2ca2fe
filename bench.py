"""Benchmark: batched CHIP-8 environment step on one MI355X.

Workload: 65,536 envs over 16 seed-generated ROMs mixed within every
wavefront (256-1792 instructions, draw share 5-40%, branch share 10-30%),
10 instructions per frame, frame skip 4, (4, 64, 32) uint8 observations,
geometric truncation horizons (mean 500), auto-reset.  One benchmark step is
one replay of a captured HIP graph holding one fused launch of 64
environment steps over all envs (64 x 65,536 env steps); actions for each
replay are copied into the graph's action buffer from a pool already in HBM.
The headline runs the envs in their own order, so that every wavefront holds
a mix of ROMs; the same inputs are then run with the envs sorted by ROM, and
through the plain one-env-per-lane kernel on both placements.

Prints one JSON line on stdout.  Everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
ALGO_BYTES_PER_ENV_STEP = 8192 + 4 + 1 + 4   # obs + reward + done + action
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_fused_c3_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "step_fused_c3_valu.json")
# integer vector-ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane operations per second
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
KERNEL_SOURCES = ["step_fused.hip", "octax_grouped.h", "octax_core.h", "octax_device.h", "octax_kernels.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_01764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_valu():
    """Vector-ALU lane operations per launch from the committed counter
    summary, if it was taken on the kernel source as it is now; else None."""
    try:
        with open(VALU_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("valu_lane_ops_per_launch")


def measured_active_lanes():
    """Mean fraction of the 64 lanes active per VALU instruction, from the
    same summary under the same condition; else None."""
    try:
        with open(VALU_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("active_lane_fraction")


COUNTER_FILES = {
    "fused": (os.path.join(ROOT, "profiles", "step_fused_c3_counters.json"), KERNEL_SOURCES),
    "plain": (os.path.join(ROOT, "profiles", "step_plain_c3_counters.json"),
              ["step_plain.hip", "octax_core.h", "octax_device.h", "octax_kernels.h", "octax_plain_mem.h"]),
}


def measured_counters(which):
    """LDS, VALU and active-lane figures of one kernel from its committed
    counter summary, if taken on the kernel source as it is now; else None."""
    path, sources = COUNTER_FILES[which]
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2510_01764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if d.get("kernel_source_hash") != h.hexdigest()[:16]:
        return None
    c, dv = d["per_dispatch"], d["derived"]
    return {"kernel": d["kernel"],
            "lds_insts_per_wave": dv.get("lds_per_wave"),
            "lds_bank_conflict_cycles_per_lds_active_cycle": dv.get("lds_bank_conflict_per_active_cycle"),
            "lds_wait_cycles_per_dispatch": c.get("SQ_WAIT_INST_LDS"),
            "valu_insts_per_wave": dv.get("valu_per_wave"),
            "salu_insts_per_wave": dv.get("salu_per_wave"),
            "active_lane_fraction": dv.get("active_lane_fraction"),
            "source": os.path.relpath(path, ROOT)}


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the kernel source as it is now; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(spec, sample_envs: int, sample_steps: int):
    """The CPU oracle on a bounded sample of the same workload, and what the
    workload's programs execute (the oracle's execution profile of every ROM
    over 1,000 frames, two envs per ROM, the workload's own actions)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2510_01764_amd import workload as W
    cores = min(16, len(os.sched_getaffinity(0)))
    sub = spec.subset(list(range(sample_envs)), name="cpu-sample")
    orc = O.OracleBatch(sub)
    acts = spec.actions(0, sample_steps)[:, :sample_envs]
    t0, c0 = time.perf_counter(), time.process_time()
    _, _, used = orc.run_threaded(acts, cores)
    dt, cpu_s = time.perf_counter() - t0, time.process_time() - c0
    orc.close()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    base = {"value": sample_envs * sample_steps / dt, "unit": "env steps/s", "cores": int(used),
            "kind": "oracle", "cpu_model": model,
            "sample": f"first {sample_envs} envs of the workload x {sample_steps} steps, observations "
                      f"materialised every step, {used} POSIX threads, {dt:.2f} s wall, {cpu_s:.1f} s of CPU time"}
    # executed instruction classes, per ROM and over the workload
    R = spec.num_roms
    prof_spec = spec.subset(np.concatenate([np.flatnonzero(spec.env_rom == r)[:2] for r in range(R)]),
                            name="exec-profile")
    po = O.OracleBatch(prof_spec)
    pc_hist, op_hist = po.profile_execution()
    steps = 1000 // spec.frame_skip
    pacts = spec.actions(0, steps)[:, np.concatenate([np.flatnonzero(spec.env_rom == r)[:2] for r in range(R)])]
    for k in range(steps):
        po.step(pacts[k], want_obs=False)
    po.close()
    cls = np.array([W.CLASS_NAMES.index(W.opcode_class(op)) for op in range(65536)])
    per_rom = np.stack([np.bincount(cls, weights=op_hist[r].astype(np.float64), minlength=len(W.CLASS_NAMES))
                        for r in range(R)])
    total = per_rom.sum()
    inside = sum(float(pc_hist[r, W.PROGRAM_START:W.PROGRAM_START + len(spec.roms[r])].sum()) for r in range(R))
    draw = per_rom[:, W.CLASS_NAMES.index("draw")] / per_rom.sum(axis=1)
    executed = {"classes": dict(zip(W.CLASS_NAMES, (per_rom.sum(axis=0) / total).round(4).tolist())),
                "in_program_share": round(inside / float(pc_hist.sum()), 4),
                "draw_share_by_rom": [round(float(x), 4) for x in draw],
                "how": "oracle execution profile: every ROM, 2 envs each, 1,000 frames, the workload's actions"}
    return base, executed


def time_replays(torch, stream, graph, act_buf, act_pool, n, start):
    """Launch n replays; per-replay durations (ms) from events on the engine's stream."""
    evs = []
    for i in range(n):
        with torch.cuda.stream(stream):
            act_buf.copy_(act_pool[(start + i) % act_pool.shape[0]], non_blocking=True)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            graph.launch()
            e1.record(stream)
        evs.append((e0, e1))
    return evs


def serving_run(args, log):
    """Continuous batching of Poisson-arriving groups (32 ROMs, sizes log-uniform
    in 1..4096, 200-2000 steps each) on a pool of args.serving_slots slots.
    The pool's sustained rate is measured first, on a burst of groups that
    keeps it full; then args.serving_groups groups arrive at each offered
    load (a fraction of that rate)."""
    import numpy as np
    from paper_2510_01764_amd import serving as S
    from paper_2510_01764_amd import workload as W
    from paper_2510_01764_amd import octax as X
    spec = W.make_config("c4")
    K = args.serving_steps_per_tick
    be = S.PoolBackend(spec, args.serving_slots * X.Pool.slot_bytes(), depth=args.serving_depth, steps_per_tick=K)
    # sustained rate: groups of the workload's sizes that fill the pool at
    # once, all running 400 steps (the loop's steady state at full occupancy)
    burst, used = [], 0
    for g in W.serving_groups(4000, 1.0, seed=13):
        if used + g.size <= args.serving_slots:
            burst.append(W.Group(g.gid, 0.0, g.rom, g.size, 400, g.seed))
            used += g.size
    cal = S.serve(spec, burst, be)
    capacity = cal["env_steps_per_s"]
    log(f"serving: sustained {capacity / 1e6:.1f} M env steps/s with the pool kept full, {K} steps per tick, "
        f"{args.serving_depth} ticks in flight")
    probe = W.serving_groups(args.serving_groups, 1.0, seed=3)
    mean_work = float(np.mean([g.size * g.steps for g in probe]))
    loads = {}
    for load in args.serving_loads:
        rate = load * capacity / mean_work
        groups = W.serving_groups(args.serving_groups, rate, seed=3)
        out = S.serve(spec, groups, be, log=log)
        loads[f"{load:.2f}"] = {
            "offered_groups_per_s": rate,
            "env_steps_per_s": out["env_steps_per_s"],
            "busy_env_steps_per_s": out["busy_env_steps_per_s"],
            "p50_step_latency_ms": out["p50_step_latency_ms"],
            "p99_step_latency_ms": out["p99_step_latency_ms"],
            "p50_queue_ms": out["p50_queue_ms"],
            "p99_queue_ms": out["p99_queue_ms"],
            "ticks": out["ticks"],
            "tick_ms_mean": out["tick_ms_mean"],
            "wall_s": out["wall_s"],
        }
        log(f"serving at {load:.0%}: {out['env_steps_per_s'] / 1e6:.1f} M env steps/s, step latency p50/p99 "
            f"{out['p50_step_latency_ms']:.3f}/{out['p99_step_latency_ms']:.3f} ms, queueing p99 "
            f"{out['p99_queue_ms']:.1f} ms")
    be.close()
    return {
        "workload": f"{args.serving_groups} groups per load over 32 ROMs, sizes log-uniform 1..4096, "
                    f"200-2000 steps, Poisson arrivals at the given fractions of the sustained rate",
        "pool_slots": args.serving_slots,
        "steps_per_tick": K,
        "ticks_in_flight": args.serving_depth,
        "sustained_env_steps_per_s": capacity,
        "sustained_def": "groups filling the pool admitted at once, 400 steps each: env steps over wall time",
        "loads": loads,
        "step_latency_def": "per group step: host time from enqueueing the tick that runs it to its rewards and done "
                            "flags on the host (a tick runs steps_per_tick steps of every resident group; a group "
                            "stops at its last step inside a tick)",
        "admission": "any free slots (the lowest-numbered), by memory, in arrival order",
    }


def step_latency(stamps_np, hz):
    """Per-step latency (ms) from one launch's step clock: for each step, the
    largest end minus the smallest start over the wave pairs that ran."""
    import numpy as np
    st, en = stamps_np[..., 0].astype(np.float64), stamps_np[..., 1].astype(np.float64)
    ok = (stamps_np[..., 0] != 0) & (stamps_np[..., 1] != 0)
    lat = []
    for k in range(stamps_np.shape[0]):
        if ok[k].any():
            lat.append((en[k][ok[k]].max() - st[k][ok[k]].min()) / hz * 1e3)
    return lat


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed graph replays (64 env steps each)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--envs", type=int, default=65536)
    ap.add_argument("--k", type=int, default=64, help="env steps per replay")
    ap.add_argument("--latency-replays", type=int, default=10,
                    help="replays after the timed region whose step clocks give the step latency")
    ap.add_argument("--latency-steps", type=int, default=50, help="octax_step launches for the K = 1 latency")
    ap.add_argument("--cpu-envs", type=int, default=65536)
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-by-rom", action="store_true", help="skip the legs on ROM-sorted placement")
    ap.add_argument("--no-wrappers", action="store_true",
                    help="skip the leg with sticky actions, no-op reset and start-up sequences")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the leg with every quirk flag and per-ROM game descriptors")
    ap.add_argument("--no-programs", action="store_true",
                    help="skip the leg on the Target Shooter programs")
    ap.add_argument("--no-schip", action="store_true", help="skip the SUPER-CHIP leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline leg (fused kernel, ROMs mixed in every wave): for profiler runs")
    ap.add_argument("--tune", choices=["auto", "default"], default="auto")
    ap.add_argument("--sweep", default="",
                    help="comma-separated env counts: also time the fused kernel at each (the paper's scaling "
                         "experiment), one observation slot")
    ap.add_argument("--sweep-workloads", default="mixed",
                    help="comma-separated workloads of the sweep: mixed, single-const, draw-heavy")
    ap.add_argument("--serving-groups", type=int, default=2000,
                    help="groups of the serving run (0 = skip it)")
    ap.add_argument("--serving-loads", type=lambda t: [float(x) for x in t.split(",")], default=[0.4, 0.7, 0.9],
                    help="offered loads as fractions of the pool's measured sustained rate")
    ap.add_argument("--serving-slots", type=int, default=65536)
    ap.add_argument("--serving-depth", type=int, default=2,
                    help="serving ticks in flight (more overlap of the host loop with the device, longer tick latency)")
    ap.add_argument("--serving-steps-per-tick", type=int, default=8,
                    help="env steps per serving tick (1..64, one action window)")
    args = ap.parse_args()
    if args.serving_depth < 1:
        ap.error("--serving-depth must be at least 1")
    if args.headline_only:
        args.no_cpu = args.no_plain = args.no_by_rom = args.no_wrappers = args.no_profile = True
        args.no_programs = args.no_schip = True
        args.serving_groups = 0
        args.latency_steps = 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the environment step has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only; launch it without torch.distributed", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    from paper_2510_01764_amd import autotune as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = W.make_config("c3", num_envs=args.envs)
    E, K = spec.num_envs, args.k
    stream = torch.cuda.Stream(device=dev)

    n_pool = max(1, min(args.warmup + args.steps, 8))
    act_pool = torch.from_numpy(spec.actions(0, n_pool * K).reshape(n_pool, K, E)).to(dev)
    act = torch.empty((K, E), dtype=torch.int32, device=dev)
    obs = torch.empty((K, E, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.empty((K, E), dtype=torch.float32, device=dev)
    done = torch.empty((K, E), dtype=torch.uint8, device=dev)

    # calibration: attainable write bandwidth and a copy of known size (its
    # counters scale the HBM byte counters of the step kernel)
    calib_bytes = 1 << 30
    cbuf = torch.empty(2 * calib_bytes, dtype=torch.uint8, device=dev)
    L = X.library()
    with torch.cuda.stream(stream):
        for _ in range(2):
            L.octax_calib_write(cbuf.data_ptr(), 2 * calib_bytes, 7, 0, stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            L.octax_calib_write(cbuf.data_ptr(), 2 * calib_bytes, 7, 0, stream.cuda_stream)
        e1.record(stream)
        L.octax_calib_copy(cbuf.data_ptr(), cbuf.data_ptr() + calib_bytes, calib_bytes, stream.cuda_stream)
    stream.synchronize()
    write_gbs = 5 * 2 * calib_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cbuf
    log(f"calibration: streaming write {write_gbs:.0f} GB/s")

    # fused engine on identity placement (the ROMs mixed within every
    # wavefront), tuned for this workload
    act.copy_(act_pool[0])
    tuning = (T.default_tuning() if args.tune == "default" else
              T.tune(spec, K=K, stream=stream, log=log, buffers=(act, obs, rew, done), use_cache=False,
                     placement="identity"))
    eng = X.Engine(spec, kernel="fused", placement="identity", envs_per_block=tuning["envs_per_block"],
                   rom_in_lds=tuning["rom_in_lds"], stream=stream)
    stamps = torch.zeros((K, (E + 63) // 64, 2), dtype=torch.int64, device=dev)
    clock_hz = eng.set_step_clock(stamps, K)
    graph = eng.graph(act, obs, rew, done)
    time_replays(torch, stream, graph, act, act_pool, args.warmup, 0)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = time_replays(torch, stream, graph, act, act_pool, args.steps, args.warmup)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    replay_ms = np.array([a.elapsed_time(b) for a, b in evs])
    value = E * K * args.steps / wall
    kernel_ms = float(replay_ms.mean())
    # per-step latency inside the K-step launches, from the step clock of
    # replays run after the timed region (each read back before the next)
    lat_k = []
    for i in range(args.latency_replays):
        time_replays(torch, stream, graph, act, act_pool, 1, args.warmup + args.steps + i)
        stream.synchronize()
        lat_k += step_latency(stamps.cpu().numpy(), clock_hz)
    lat_k = np.array(lat_k if lat_k else [float("nan")])
    graph.close()
    eng.set_step_clock(None, 0)
    eng.status()
    log(f"fused, identity placement: {value / 1e6:.1f} M env steps/s ({kernel_ms:.3f} ms per replay), "
        f"step latency p50 {np.percentile(lat_k, 50):.3f} ms p99 {np.percentile(lat_k, 99):.3f} ms")

    # single-step latency: octax_step (one fused launch of K = 1) over all envs
    lat1 = []
    if args.latency_steps > 0:
        a1 = act_pool[0, 0].contiguous()
        for i in range(5 + args.latency_steps):
            with torch.cuda.stream(stream):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                eng.step(a1, obs[0], rew[0], done[0])
                e1.record(stream)
            stream.synchronize()
            if i >= 5:
                lat1.append(e0.elapsed_time(e1))
        eng.status()
    lat1 = np.array(lat1 if lat1 else [float("nan")])
    eng.close()

    def timed_leg(kernel, placement, n):
        """Graph replays of the same workload on another kernel or placement."""
        kw = {}
        if kernel == "fused":
            tn = (T.default_tuning() if args.tune == "default" else
                  T.tune(spec, K=K, stream=stream, log=log, buffers=(act, obs, rew, done), use_cache=False,
                         placement=placement))
            kw = dict(envs_per_block=tn["envs_per_block"], rom_in_lds=tn["rom_in_lds"])
        e2 = X.Engine(spec, kernel=kernel, placement=placement, stream=stream, **kw)
        g2 = e2.graph(act, obs, rew, done)
        time_replays(torch, stream, g2, act, act_pool, 1, 0)
        stream.synchronize()
        t0 = time.perf_counter()
        time_replays(torch, stream, g2, act, act_pool, n, args.warmup)
        stream.synchronize()
        w2 = time.perf_counter() - t0
        g2.close()
        e2.status()
        e2.close()
        out = {"value": E * K * n / w2, "ms_per_step": w2 * 1e3 / n, "replays": n, "placement": placement}
        out.update(kw)
        log(f"{kernel}, {placement} placement: {out['value'] / 1e6:.1f} M env steps/s "
            f"({out['ms_per_step']:.2f} ms per replay)")
        return out

    fused_by_rom = None if args.no_by_rom else timed_leg("fused", "by_rom", max(2, args.steps // 2))
    plain = None
    if not args.no_plain:
        plain = {"identity": timed_leg("plain", "identity", max(2, args.steps // 4))}
        if not args.no_by_rom:
            plain["by_rom"] = timed_leg("plain", "by_rom", max(2, args.steps // 4))

    def variant_leg(vspec, pool=None, placement="identity"):
        """Graph replays of the same launch shape under another spec; (env steps/s, ms per replay, replays)."""
        pool = act_pool if pool is None else pool
        engv = X.Engine(vspec, kernel="fused", placement=placement, envs_per_block=tuning["envs_per_block"],
                        rom_in_lds=tuning["rom_in_lds"], stream=stream)
        gv = engv.graph(act, obs, rew, done)
        time_replays(torch, stream, gv, act, pool, 1, 0)
        stream.synchronize()
        n_v = max(2, args.steps // 4)
        t0 = time.perf_counter()
        time_replays(torch, stream, gv, act, pool, n_v, args.warmup)
        stream.synchronize()
        vwall = time.perf_counter() - t0
        resets = float((done != 0).float().mean().item())
        gv.close()
        engv.status()
        engv.close()
        return {"value": E * K * n_v / vwall, "ms_per_step": vwall * 1e3 / n_v, "replays": n_v,
                "resets_per_env_step": resets, "placement": placement}

    # the same workload with the environment wrappers of Section 3.2 on
    wrappers = None
    if not args.no_wrappers:
        wspec = W.with_wrappers(spec, sticky=0.25, noop_max=30, startup_max=3, seed=1)
        # envs spread over the wavefronts by horizon, so that the envs that
        # reset most often run their reset steps in different wavefronts; the
        # identity placement beside it
        wrappers = variant_leg(wspec, placement="by_horizon")
        ident = variant_leg(wspec)
        wrappers.update({"sticky_prob": 0.25, "noop_max": 30,
                         "startup_steps": [int(x) for x in wspec.startup_len],
                         "identity": {"value": ident["value"], "ms_per_step": ident["ms_per_step"]}})
        log(f"wrappers: {wrappers['value'] / 1e6:.1f} M env steps/s ({wrappers['ms_per_step']:.2f} ms per replay; "
            f"identity placement {ident['value'] / 1e6:.1f} M)")

    # ... and with the quirk flags and per-ROM game descriptors (Section 3.3).
    # Display wait stays off: it cuts the instructions run per frame, so the
    # leg would no longer time the same emulation work.
    profile = None
    if not args.no_profile:
        qspec = W.with_profile(spec, quirks=0x3F, seed=1)
        profile = variant_leg(qspec)
        profile.update({"quirks": qspec.quirks, "display_wait": False,
                        "score_mode": [int(x) for x in qspec.score_mode],
                        "term_op": [int(x) for x in qspec.term_op],
                        "term2_op": [int(x) for x in qspec.term2_op]})
        log(f"profile: {profile['value'] / 1e6:.1f} M env steps/s ({profile['ms_per_step']:.2f} ms per replay)")

    # a second workload: the three Target Shooter levels (Octo programs
    # assembled in-tree), 65,536 envs, uniform random actions over its 5 keys
    shooter = None
    if not args.no_programs and E == 65536:
        tspec = W.make_config("ts")
        tpool = torch.from_numpy(tspec.actions(0, n_pool * K).reshape(n_pool, K, E)).to(dev)
        shooter = variant_leg(tspec, tpool)
        shooter.update({"workload": "Target Shooter levels 1-3, 65,536 envs, a third each, keys 5 7 8 9 6, "
                                    "score V2, done V3 == 1, geometric horizons mean 500"})
        log(f"target shooter: {shooter['value'] / 1e6:.1f} M env steps/s ({shooter['ms_per_step']:.2f} ms per replay)")

    # SUPER-CHIP (128x64, (4, 128, 64) observations): 65,536 envs on its
    # lane-per-env kernels, Ks steps per replay so that a launch writes the
    # same observation bytes as the CHIP-8 one
    schip = None
    Ks = K * 8192 // 32768
    if not args.no_schip and E == 65536 and Ks >= 1:
        sspec = W.make_config("s1")
        Es = sspec.num_envs
        sobs = obs.view(-1)[: Ks * Es * 32768].view(Ks, Es, 4, 128, 64)
        spool = torch.from_numpy(sspec.actions(0, n_pool * Ks).reshape(n_pool, Ks, Es)).to(dev)
        sact = torch.empty((Ks, Es), dtype=torch.int32, device=dev)
        srew = torch.empty((Ks, Es), dtype=torch.float32, device=dev)
        sdone = torch.empty((Ks, Es), dtype=torch.uint8, device=dev)
        engs = X.Engine(sspec, kernel="plain", stream=stream)
        gs = engs.graph(sact, sobs, srew, sdone)
        time_replays(torch, stream, gs, sact, spool, 1, 0)
        stream.synchronize()
        n_s = max(2, args.steps // 4)
        t0 = time.perf_counter()
        time_replays(torch, stream, gs, sact, spool, n_s, args.warmup)
        stream.synchronize()
        swall = time.perf_counter() - t0
        # algorithmic bytes per env step: the 32 KB observation, reward, done and action
        s_bytes = 32768 + 4 + 1 + 4
        s_achieved = Es * Ks * n_s * s_bytes / swall / 1e9
        schip = {"value": Es * Ks * n_s / swall, "ms_per_step": swall * 1e3 / n_s, "replays": n_s,
                 "obs_GBs": Es * Ks * n_s * 32768 / swall / 1e9,
                 "roofline": {"bound": "hbm", "achieved": s_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": s_achieved / HBM_PEAK_GBS, "bytes_per_env_step": s_bytes,
                              "timing": "wall clock over the timed replays"},
                 "kernel": "emulation of step k beside the observations of step k - 1, one launch per step",
                 "workload": f"SUPER-CHIP: 65,536 envs over 8 generated programs with 12% SUPER-CHIP "
                             f"instructions, {Ks} steps per graph replay, ipf 10, frame skip 4, "
                             f"4x128x64 uint8 obs, geometric horizons mean 500"}
        log(f"schip: {schip['value'] / 1e6:.1f} M env steps/s ({schip['ms_per_step']:.2f} ms per replay)")
        gs.close()
        engs.close()

    # the paper's scaling experiment: env steps/s against the number of envs
    # (mixed: the benchmark recipe; single-const: one generated program with
    # one action held throughout, the shape of the paper's own measurement;
    # draw-heavy: 64 programs, 40 % DXYN of up to 15 rows, 20 instructions
    # per frame)
    sweep = None
    if args.sweep:
        sweep = []
        sweep_cfg = {"mixed": "c3", "single-const": "c2", "draw-heavy": "c5"}
        for label in args.sweep_workloads.split(","):
            for Ew in (int(x) for x in args.sweep.split(",")):
                wspec = W.make_config(sweep_cfg[label], num_envs=Ew)
                wact_np = wspec.actions(0, K)
                if label == "single-const":
                    wact_np[:] = 0
                wact = torch.from_numpy(wact_np).to(dev)
                wobs = torch.empty((1, Ew, 4, 64, 32), dtype=torch.uint8, device=dev)
                wrew = torch.empty((K, Ew), dtype=torch.float32, device=dev)
                wdone = torch.empty((K, Ew), dtype=torch.uint8, device=dev)
                ew = X.Engine(wspec, kernel="fused", placement="identity", stream=stream)
                gw = ew.graph(wact, wobs, wrew, wdone)
                with torch.cuda.stream(stream):
                    gw.launch()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    n_w = 6 if Ew <= 65536 else 3
                    for _ in range(n_w):
                        gw.launch()
                    e1.record(stream)
                stream.synchronize()
                ms = e0.elapsed_time(e1) / n_w
                gw.close()
                ew.status()
                ew.close()
                sweep.append({"workload": label, "envs": Ew, "ms_per_launch": ms, "env_steps_per_s": Ew * K / ms * 1e3})
                log(f"sweep: {label} {Ew} envs {ms:.3f} ms per launch, {Ew * K / ms / 1e3:.1f} M env steps/s")
                del wobs, wrew, wdone, wact
                torch.cuda.empty_cache()

    serving = None
    if args.serving_groups > 0:
        serving = serving_run(args, log)

    algo_per_launch = E * K * ALGO_BYTES_PER_ENV_STEP
    achieved = algo_per_launch / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    valu_ops = measured_valu()
    cpu, executed = (None, None) if args.no_cpu else cpu_baseline(spec, min(args.cpu_envs, E), args.cpu_steps)
    fop = None
    if plain:
        fop = {"identity": value / plain["identity"]["value"]}
        if fused_by_rom and "by_rom" in plain:
            fop["by_rom"] = fused_by_rom["value"] / plain["by_rom"]["value"]
    out = {
        "metric": "env steps/s @65,536 envs mixed-ROM (fused vs plain), p99 step latency",
        "value": value,
        "unit": "env steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic: seed-generated CHIP-8 ROMs and uniform random actions",
        "config": {
            "workload": "mixed-ROM batching: 65,536 envs over 16 seed-generated ROMs mixed within every "
                        "wavefront, 64 env steps per graph replay, ipf 10, frame skip 4, 4x64x32 uint8 obs, "
                        "geometric horizons mean 500, auto-reset",
            "envs": E, "roms": spec.num_roms, "env_steps_per_bench_step": E * K,
            "instr_per_frame": spec.instr_per_frame, "frame_skip": spec.frame_skip,
            "kernel": "fused", "envs_per_block": tuning["envs_per_block"],
            "lanes_per_env": 1, "rom_in_lds": bool(tuning["rom_in_lds"]), "placement": "identity",
            "executed": executed,
        },
        "frames_per_s": 4 * value,
        "chip8_instr_per_s": value * spec.instr_per_frame * spec.frame_skip,
        "p50_step_latency_ms": float(np.percentile(lat_k, 50)),
        "p99_step_latency_ms": float(np.percentile(lat_k, 99)),
        "step_latency_def": f"per step of the timed {K}-step graph launches: the last wave pair's end of step k "
                            f"(its last observation store issued) minus the first pair's start of step k, from "
                            f"the device wall clock ({len(lat_k)} steps over {args.latency_replays} launches)",
        "octax_step_latency_ms": {"p50": float(np.percentile(lat1, 50)), "p99": float(np.percentile(lat1, 99)),
                                  "def": "octax_step on all envs (one fused launch of K = 1), HIP events"},
        "replay_ms_p50": float(np.percentile(replay_ms, 50)),
        "replay_ms_p99": float(np.percentile(replay_ms, 99)),
        "fused_by_rom": fused_by_rom,
        "plain": plain,
        "fused_over_plain": fop,
        "wrappers": wrappers,
        "profile": profile,
        "target_shooter": shooter,
        "schip": schip,
        "sweep": sweep,
        "calib_write_GBs": write_gbs,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"step_fused_kernel<{tuning['envs_per_block']}, true, false, false>",
            "algorithmic_bytes_per_launch": algo_per_launch,
            "kernel_ms": kernel_ms,
        },
        # the other roofline of the path: integer vector ALU, from the committed
        # SQ_INSTS_VALU counter summary of the same kernel (null if stale)
        "valu": (None if valu_ops is None else {
            "achieved": valu_ops / (kernel_ms * 1e-3), "peak": VALU_PEAK_LANE_OPS, "unit": "lane ops/s",
            "frac": valu_ops / (kernel_ms * 1e-3) / VALU_PEAK_LANE_OPS, "lane_ops_per_launch": valu_ops,
            "active_lane_fraction": measured_active_lanes()}),
        # LDS instructions and bank conflicts, VALU issue and active lanes of the
        # fused and plain kernels, from the committed counter summaries (null if stale)
        "counters": {"fused": measured_counters("fused"), "plain": measured_counters("plain")},
        "context": "paper: 350,000 env steps/s (Pong, constant action, RTX 3090) - other hardware and workload",
    }
    if serving is not None:
        out["serving"] = serving
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
