"""Serving loop: continuous batching of environment groups on one pool.

Requests are groups of envs of one ROM that run a fixed number of steps
(Section 3.2's functional reset/step environment, many of them at once).
They arrive over time.  Each arrival waits in a FIFO queue until enough pool
slots are free to hold it; admission is by memory (the pool has a fixed
device budget; a group takes any free slots, so the pool never fragments),
in arrival order, with later groups allowed to start while a larger one at
the head of the queue does not fit yet.  Every tick
enqueues one step of every resident group as one launch over the pool, so
the work of groups that arrived at different times runs together on the
device.  A group leaves the pool after its last step.

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


class PoolBackend:
    """liboctax pool on the current GPU, with `depth` ticks in flight.

    Actions are taken from a pinned host schedule of `rows` tick rows (a
    ring indexed by tick number); each tick copies its row to the device.
    """

    def __init__(self, spec, pool_bytes: int, depth: int = 2, with_obs: bool = True,
                 envs_per_block: int = 256, rows: int = 128):
        import torch
        from . import octax as X
        self.torch = torch
        dev = torch.device("cuda")
        self.stream = torch.cuda.Stream(device=dev)
        self.pool = X.Pool(spec, pool_bytes, envs_per_block=envs_per_block, stream=self.stream)
        cap = self.capacity = self.pool.capacity
        self.depth = depth
        self.rows = rows
        self.h_sched = torch.zeros((rows, cap), dtype=torch.int32).pin_memory()
        self.act = [torch.zeros((1, cap), dtype=torch.int32, device=dev) for _ in range(depth)]
        self.rew = [torch.zeros((1, cap), dtype=torch.float32, device=dev) for _ in range(depth)]
        self.done = [torch.zeros((1, cap), dtype=torch.uint8, device=dev) for _ in range(depth)]
        self.h_rew = [torch.zeros((1, cap), dtype=torch.float32).pin_memory() for _ in range(depth)]
        self.h_done = [torch.zeros((1, cap), dtype=torch.uint8).pin_memory() for _ in range(depth)]
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
        """Host action schedule [rows, capacity] (pinned)."""
        return self.h_sched.numpy()

    def launch(self, row: int) -> int:
        d = self.n % self.depth
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.act[d][0].copy_(self.h_sched[row], non_blocking=True)
            self.ev[d][0].record(self.stream)
            self.pool.step(self.act[d], self.obs, self.rew[d], self.done[d])
            self.ev[d][1].record(self.stream)
            self.h_rew[d].copy_(self.rew[d], non_blocking=True)
            self.h_done[d].copy_(self.done[d], non_blocking=True)
            self.ready[d].record(self.stream)
        self.n += 1
        return self.n - 1

    def wait(self, ticket: int):
        d = ticket % self.depth
        self.ready[d].synchronize()
        return (self.h_rew[d].numpy()[0], self.h_done[d].numpy()[0],
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

    Tick T reads its actions from row T of the backend's schedule ring; a
    group admitted before tick T0 takes step k in tick T0 + k, and its
    actions are written into the ring a window of steps ahead, so a tick
    costs the host O(1) work besides admissions, window refills and
    retirements.  With ``record`` (True for every group, or a set of group
    ids) every step's rewards and dones, the last observation and the final
    architectural state of the recorded groups are kept (the ticks in flight
    are drained before a finishing recorded group's slots are read).
    Returns per-group runs and latency figures.
    """
    depth = backend.depth
    R = backend.rows
    if R < WINDOW + depth + 1:
        raise ValueError("the schedule ring must hold a window plus the ticks in flight")
    sched = backend.schedule()
    runs = [GroupRun(g, int(spec.num_actions[g.rom])) for g in groups]
    order = sorted(range(len(runs)), key=lambda i: runs[i].group.arrival)
    queue: List[GroupRun] = []
    resident: Dict[int, GroupRun] = {}
    inflight: collections.deque = collections.deque()
    refill_at: Dict[int, List[GroupRun]] = collections.defaultdict(list)
    finish_at: Dict[int, List[GroupRun]] = collections.defaultdict(list)
    tick_lat: List[float] = []
    tick_groups: List[int] = []
    tick_ms: List[float] = []
    nxt = 0
    T = 0
    resident_envs = 0
    busy_env_steps = 0
    changed = True
    t0 = clock()

    def recorded(r: GroupRun) -> bool:
        return record is True or (bool(record) and r.group.gid in record)

    def write_window(r: GroupRun, t_start: int):
        g = r.group
        k0 = t_start - r.t0
        n = min(WINDOW, g.steps - k0)
        rows = (t_start + np.arange(n)) % R
        sched[np.ix_(rows, r.slots)] = W.group_actions(g, k0, n, r.num_actions)
        if k0 + n < g.steps:
            refill_at[t_start + n].append(r)

    def collect():
        ticket, tick, n_groups, members, t_launch = inflight.popleft()
        rew, done, dev_ms = backend.wait(ticket)
        tick_lat.append(clock() - t0 - t_launch)
        tick_groups.append(n_groups)
        tick_ms.append(dev_ms)
        for r in members:
            k = tick - r.t0
            r.rewards[k] = rew[r.slots]
            r.dones[k] = done[r.slots]

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
            r.t0 = T
            r.t_admit = clock() - t0
            if recorded(r):
                r.rewards = np.zeros((g.steps, g.size), dtype=np.float32)
                r.dones = np.zeros((g.steps, g.size), dtype=np.uint8)
            queue.remove(r)
            resident[r.pool_id] = r
            resident_envs += g.size
            write_window(r, T)
            finish_at[T + g.steps - 1].append(r)
        changed = False
        if resident:
            if len(inflight) >= depth:
                collect()
            for r in refill_at.pop(T, ()):
                write_window(r, T)
            t_launch = clock() - t0
            ticket = backend.launch(T % R)
            members = [r for r in resident.values() if recorded(r)] if record else []
            inflight.append((ticket, T, len(resident), members, t_launch))
            busy_env_steps += resident_envs
            finished = finish_at.pop(T, ())
            if any(recorded(r) for r in finished):
                while inflight:
                    collect()
            for r in finished:
                resident.pop(r.pool_id)
                resident_envs -= r.group.size
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
            f"{len(tick_ms)} ticks, p50/p99 step latency {p50:.3f}/{p99:.3f} ms")
    return {
        "runs": runs,
        "wall_s": t_end,
        "env_steps": total,
        "env_steps_per_s": total / t_end if t_end > 0 else float("nan"),
        "ticks": len(tick_ms),
        "tick_ms_mean": float(np.mean(tick_ms)) if tick_ms else float("nan"),
        "busy_env_steps_per_s": (busy_env_steps / (np.sum(tick_ms) * 1e-3)) if tick_ms else float("nan"),
        "p50_step_latency_ms": p50,
        "p99_step_latency_ms": p99,
        "p50_queue_ms": float(np.percentile(qd, 50)),
        "p99_queue_ms": float(np.percentile(qd, 99)),
    }
