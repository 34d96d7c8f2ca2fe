"""Serving loop: continuous batching of environment groups on one pool.

Requests are groups of envs of one ROM that run a fixed number of steps
(Section 3.2's functional reset/step environment, many of them at once).
They arrive over time.  Each arrival waits in a FIFO queue until enough pool
slots are free to hold it; admission is by memory (the pool has a fixed
device budget; a group takes any free slots, so the pool never fragments),
in arrival order, with later groups allowed to start while a larger one at
the head of the queue does not fit yet.  Every tick
enqueues K steps (steps_per_tick) of every resident group as one launch
over the pool, so the work of groups that arrived at different times runs
together on the device; a group whose last step falls inside a tick stops
there (a per-slot step budget of the launch).  A group leaves the pool after
its last step.

All emulation runs in liboctax (``octax.Pool``); this module only decides
which group goes where and when, builds the per-slot action vector of each
tick and collects results.  The backend is an argument so that the
scheduling logic can be checked without a device.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import workload as W


@dataclasses.dataclass
class GroupRun:
    group: W.Group
    num_actions: int
    pool_id: int = -1          # the pool's id of the group while resident
    slots: Optional[np.ndarray] = None   # its envs' slots while resident
    t0: int = -1               # tick of the group's first step
    step: int = 0              # steps run (set when the group leaves)
    t_arrival: float = 0.0
    t_admit: float = -1.0
    t_done: float = -1.0
    rewards: Optional[np.ndarray] = None   # [steps, size] when recording
    dones: Optional[np.ndarray] = None
    final_obs: Optional[np.ndarray] = None
    final_state: Optional[np.ndarray] = None
    seeds: Optional[np.ndarray] = None     # per-env RNG seeds and horizons, drawn on arrival
    horizons: Optional[np.ndarray] = None
    runs: Optional[list] = None            # runs of consecutive slots while resident
    stream: Optional[np.random.PCG64] = None   # its action stream, drawn one window after another


class PoolBackend:
    """liboctax pool on the current GPU, with `depth` ticks of `steps_per_tick`
    steps in flight.

    Actions are taken from a pinned host schedule of `rows` rows, one per
    global step (a ring indexed by step number; tick T runs steps T*K ..
    T*K + K - 1); each tick copies its K rows and the slots' step budgets to
    the device.
    """

    def __init__(self, spec, pool_bytes: int, depth: int = 2, with_obs: bool = True,
                 envs_per_block: int = 256, rows: int = 128, steps_per_tick: int = 1):
        import torch
        from . import octax as X
        self.torch = torch
        dev = torch.device("cuda")
        K = self.K = int(steps_per_tick)
        if not 1 <= K <= 255:
            raise ValueError("steps_per_tick must be in 1..255")
        rows = max(rows, WINDOW + (depth + 1) * K)
        rows = -(-rows // K) * K
        self.stream = torch.cuda.Stream(device=dev)
        self.pool = X.Pool(spec, pool_bytes, envs_per_block=envs_per_block, stream=self.stream)
        cap = self.capacity = self.pool.capacity
        self.depth = depth
        self.rows = rows
        self.h_sched = torch.zeros((rows, cap), dtype=torch.int32).pin_memory()
        self.act = [torch.zeros((K, cap), dtype=torch.int32, device=dev) for _ in range(depth)]
        self.rew = [torch.zeros((K, cap), dtype=torch.float32, device=dev) for _ in range(depth)]
        self.done = [torch.zeros((K, cap), dtype=torch.uint8, device=dev) for _ in range(depth)]
        self.h_rew = [torch.zeros((K, cap), dtype=torch.float32).pin_memory() for _ in range(depth)]
        self.h_done = [torch.zeros((K, cap), dtype=torch.uint8).pin_memory() for _ in range(depth)]
        self.h_budget = [torch.zeros(cap, dtype=torch.uint8).pin_memory() for _ in range(depth)]
        self.budget = [torch.zeros(cap, dtype=torch.uint8, device=dev) for _ in range(depth)]
        self.obs = (torch.zeros((1, cap, 4, 64, 32), dtype=torch.uint8, device=dev)
                    if with_obs else None)
        self.ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(depth)]
        self.ready = [torch.cuda.Event() for _ in range(depth)]   # results are on the host
        self.n = 0

    def admit(self, rom, seeds, horizons):
        return self.pool.admit(rom, seeds, horizons)

    def retire(self, pool_id):
        self.pool.retire(pool_id)

    def schedule(self) -> np.ndarray:
        """Host action schedule [rows, capacity] (pinned), one row per global step."""
        return self.h_sched.numpy()

    def launch(self, tick: int, budget: Optional[np.ndarray]) -> int:
        """Tick `tick`: K steps of every resident slot, slot s stopping after
        budget[s] of them (None: all K)."""
        d = self.n % self.depth
        torch = self.torch
        r0 = (tick * self.K) % self.rows
        with torch.cuda.stream(self.stream):
            self.act[d].copy_(self.h_sched[r0:r0 + self.K], non_blocking=True)
            if budget is not None:
                self.h_budget[d].numpy()[:] = budget
                self.budget[d].copy_(self.h_budget[d], non_blocking=True)
            self.ev[d][0].record(self.stream)
            self.pool.step(self.act[d], self.obs, self.rew[d], self.done[d],
                           budget=self.budget[d] if budget is not None else None)
            self.ev[d][1].record(self.stream)
            self.h_rew[d].copy_(self.rew[d], non_blocking=True)
            self.h_done[d].copy_(self.done[d], non_blocking=True)
            self.ready[d].record(self.stream)
        self.n += 1
        return self.n - 1

    def wait(self, ticket: int):
        """Rewards and done flags [K][capacity] of a tick, and its device time (ms)."""
        d = ticket % self.depth
        self.ready[d].synchronize()
        return (self.h_rew[d].numpy(), self.h_done[d].numpy(),
                self.ev[d][0].elapsed_time(self.ev[d][1]))

    def finish(self):
        self.stream.synchronize()

    def obs_of(self, slots: np.ndarray) -> np.ndarray:
        self.stream.synchronize()
        return self.obs[0].cpu().numpy()[slots]

    def state_of(self, slots: np.ndarray) -> np.ndarray:
        return self.pool.get_state(slots)

    def close(self):
        self.stream.synchronize()
        self.pool.close()


WINDOW = W.ACTION_CHUNK   # steps of a group's actions written into the schedule at a time


def _weighted_percentile(values: np.ndarray, weights: np.ndarray, q: float) -> float:
    if len(values) == 0 or weights.sum() == 0:
        return float("nan")
    o = np.argsort(values)
    cw = np.cumsum(weights[o])
    return float(values[o][np.searchsorted(cw, q / 100.0 * cw[-1])])


def serve(spec, groups: List[W.Group], backend, *, record=False,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          log: Optional[Callable[[str], None]] = None) -> Dict:
    """Run the request loop over `groups` (arrival times in seconds from the start).

    Tick T runs global steps T*K .. T*K + K - 1 (K = backend.K) and reads its
    actions from those rows of the backend's schedule ring; a group admitted
    before tick T0 takes its step k at global step T0*K + k, and its actions
    are written into the ring a window of steps ahead, so a tick costs the
    host O(1) work besides admissions, window refills, retirements and the
    groups that stop inside it.  With ``record`` (True for every group, or a
    set of group ids) every step's rewards and dones, the last observation
    and the final architectural state of the recorded groups are kept (the
    ticks in flight are drained before a finishing recorded group's slots are
    read).  Returns per-group runs and latency figures.
    """
    depth = backend.depth
    K = getattr(backend, "K", 1)
    R = backend.rows
    if K > WINDOW:
        raise ValueError(f"at most {WINDOW} steps per tick (one action window per group and tick)")
    if R % K or R < WINDOW + (depth + 1) * K:
        raise ValueError("the schedule ring must be a multiple of K rows holding a window plus the ticks in flight")
    sched = backend.schedule()
    cap = backend.capacity
    runs = [GroupRun(g, int(spec.num_actions[g.rom])) for g in groups]
    order = sorted(range(len(runs)), key=lambda i: runs[i].group.arrival)
    queue: List[GroupRun] = []
    resident: Dict[int, GroupRun] = {}
    inflight: collections.deque = collections.deque()
    refill_at: Dict[int, List] = collections.defaultdict(list)
    finish_at: Dict[int, List[GroupRun]] = collections.defaultdict(list)
    short_at: Dict[int, List[GroupRun]] = collections.defaultdict(list)   # groups that stop inside tick T
    budget = np.full(cap, K, dtype=np.uint8)
    tick_lat: List[float] = []
    tick_groups: List[int] = []
    tick_ms: List[float] = []
    nxt = 0
    T = 0
    busy_env_steps = 0
    changed = True
    t0 = clock()

    def recorded(r: GroupRun) -> bool:
        return record is True or (bool(record) and r.group.gid in record)

    def write_window(r: GroupRun, k0: int):
        """Actions of the group's steps k0 .. k0 + WINDOW - 1 into the ring,
        one block copy per run of consecutive slots and of ring rows."""
        g = r.group
        n = min(WINDOW, g.steps - k0)
        row0 = (r.t0 * K + k0) % R
        parts = [(row0, 0, min(n, R - row0))]
        if parts[0][2] < n:
            parts.append((0, parts[0][2], n - parts[0][2]))
        # windows are the group's action chunks in order (WINDOW ==
        # ACTION_CHUNK), drawn from one stream per group
        if r.stream is None:
            r.stream = W.action_stream(g)
        acts = W.actions_from_words(W.group_action_words(g, k0 // WINDOW, r.stream), r.num_actions)
        for s0, i0, m in r.runs:
            for q0, a0, c in parts:
                sched[q0:q0 + c, s0:s0 + m] = acts[a0:a0 + c, i0:i0 + m]
        if k0 + n < g.steps:
            refill_at[r.t0 + (k0 + n) // K].append((r, k0 + n))

    def collect():
        ticket, tick, n_groups, members, t_launch = inflight.popleft()
        rew, done, dev_ms = backend.wait(ticket)
        tick_lat.append(clock() - t0 - t_launch)
        tick_groups.append(n_groups)
        tick_ms.append(dev_ms)
        for r in members:
            k0 = (tick - r.t0) * K
            n = min(K, r.group.steps - k0)
            r.rewards[k0:k0 + n] = rew[:n, r.slots]
            r.dones[k0:k0 + n] = done[:n, r.slots]

    while nxt < len(order) or queue or resident or inflight:
        now = clock() - t0
        fresh = []
        while nxt < len(order) and runs[order[nxt]].group.arrival <= now:
            r = runs[order[nxt]]
            r.t_arrival = r.group.arrival
            r.seeds = W.group_env_seeds(r.group)
            r.horizons = W.group_horizons(r.group)
            queue.append(r)
            fresh.append(r)
            nxt += 1
        # admission: arrival order; a group that does not fit lets later ones
        # try.  Queued groups are retried only after a retirement.
        for r in (list(queue) if changed else fresh):
            g = r.group
            adm = backend.admit(g.rom, r.seeds, r.horizons)
            if adm is None:
                continue
            r.pool_id, r.slots = adm
            # runs of consecutive slots: (first slot, first env, length)
            brk = np.flatnonzero(np.diff(r.slots.astype(np.int64)) != 1) + 1
            starts = np.concatenate([[0], brk])
            ends = np.concatenate([brk, [len(r.slots)]])
            r.runs = [(int(r.slots[a]), int(a), int(b - a)) for a, b in zip(starts, ends)]
            r.t0 = T
            r.t_admit = clock() - t0
            if recorded(r):
                r.rewards = np.zeros((g.steps, g.size), dtype=np.float32)
                r.dones = np.zeros((g.steps, g.size), dtype=np.uint8)
            queue.remove(r)
            resident[r.pool_id] = r
            write_window(r, 0)
            last = T + (g.steps - 1) // K
            finish_at[last].append(r)
            if g.steps % K:
                short_at[last].append(r)
        changed = False
        if resident:
            if len(inflight) >= depth:
                collect()
            for r, k0 in refill_at.pop(T, ()):
                write_window(r, k0)
            # slots that stop inside this tick run only their remaining steps
            short = short_at.pop(T, ())
            for r in short:
                budget[r.slots] = r.group.steps % K
            t_launch = clock() - t0
            ticket = backend.launch(T, budget if K > 1 else None)
            for r in short:
                budget[r.slots] = K
            members = [r for r in resident.values() if recorded(r)] if record else []
            inflight.append((ticket, T, len(resident), members, t_launch))
            busy_env_steps += sum(r.group.size * min(K, r.group.steps - (T - r.t0) * K) for r in resident.values())
            finished = finish_at.pop(T, ())
            if any(recorded(r) for r in finished):
                while inflight:
                    collect()
            for r in finished:
                resident.pop(r.pool_id)
                if recorded(r):
                    r.final_obs = backend.obs_of(r.slots)
                    r.final_state = backend.state_of(r.slots)
                backend.retire(r.pool_id)
                r.step = r.group.steps
                r.t_done = clock() - t0
                changed = True
            T += 1
        elif inflight:
            collect()
        elif queue:
            raise RuntimeError("a queued group does not fit in an empty pool")
        elif nxt < len(order):
            wait = runs[order[nxt]].group.arrival - (clock() - t0)
            if wait > 0:
                sleep(wait)
    backend.finish()
    t_end = clock() - t0
    total = sum(r.group.size * r.group.steps for r in runs)
    lat = np.array(tick_lat) * 1e3
    wts = np.array(tick_groups, dtype=np.float64)
    qd = np.array([r.t_admit - r.t_arrival for r in runs]) * 1e3
    p50 = _weighted_percentile(lat, wts, 50)
    p99 = _weighted_percentile(lat, wts, 99)
    if log:
        log(f"serving: {len(runs)} groups, {total} env steps in {t_end:.2f} s, "
            f"{len(tick_ms)} ticks of {K} steps, p50/p99 tick latency {p50:.3f}/{p99:.3f} ms")
    return {
        "runs": runs,
        "wall_s": t_end,
        "env_steps": total,
        "env_steps_per_s": total / t_end if t_end > 0 else float("nan"),
        "steps_per_tick": K,
        "ticks": len(tick_ms),
        "tick_ms_mean": float(np.mean(tick_ms)) if tick_ms else float("nan"),
        "busy_env_steps_per_s": (busy_env_steps / (np.sum(tick_ms) * 1e-3)) if tick_ms else float("nan"),
        "p50_step_latency_ms": p50,
        "p99_step_latency_ms": p99,
        "p50_queue_ms": float(np.percentile(qd, 50)),
        "p99_queue_ms": float(np.percentile(qd, 99)),
    }
