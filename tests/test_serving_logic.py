"""Host logic of the serving loop, on the CPU with a stand-in backend.

The stand-in keeps the pool's contract (a group takes the lowest-numbered
free slots of a fixed capacity, admission refused when too few are free;
each tick runs K steps, slot s stopping after budget[s] of them, with one
result row per step indexed by slot) and reports, as each slot's reward,
the global step number and the slot, so the tests can check which group
stepped where and when.
"""
import numpy as np
import pytest

from paper_2510_01764_amd import serving as S
from paper_2510_01764_amd import workload as W


class FakeBackend:
    def __init__(self, capacity, depth=2, rows=128, steps_per_tick=1):
        self.capacity = capacity
        self.depth = depth
        self.K = steps_per_tick
        self.rows = max(rows, S.WINDOW + (depth + 1) * self.K)
        self.rows = -(-self.rows // self.K) * self.K
        self.sched = np.zeros((self.rows, capacity), dtype=np.int32)
        self.groups = {}
        self.next_id = 0
        self.occupied = np.zeros(capacity, dtype=np.int32)
        self.ticks = []                     # per tick: (tick number, occupied map, budgets)
        self.n = 0
        self.acts = {}                      # global step -> action row sent
        self.steps_run = np.zeros(capacity, dtype=np.int64)   # steps each slot ran while occupied
        self.max_used = 0

    def admit(self, rom, seeds, horizons):
        free = np.flatnonzero(self.occupied == 0)
        if len(free) < len(seeds):
            return None
        slots = free[:len(seeds)].astype(np.uint32)
        self.occupied[slots] = 1
        self.steps_run[slots] = 0
        self.max_used = max(self.max_used, int(self.occupied.sum()))
        gid = self.next_id
        self.next_id += 1
        self.groups[gid] = slots
        return gid, slots

    def retire(self, gid):
        self.occupied[self.groups.pop(gid)] = 0

    def schedule(self):
        return self.sched

    def launch(self, tick, budget):
        b = np.full(self.capacity, self.K) if budget is None else budget.astype(np.int64).copy()
        self.ticks.append((tick, self.occupied.copy(), b))
        for i in range(self.K):
            self.acts[tick * self.K + i] = self.sched[(tick * self.K + i) % self.rows].copy()
        self.steps_run += np.where(self.occupied != 0, np.minimum(b, self.K), 0)
        self.n += 1
        return self.n - 1

    def wait(self, ticket):
        tick, occ, b = self.ticks[ticket]
        steps = tick * self.K + np.arange(self.K)
        rew = (steps[:, None] * 1000 + np.arange(self.capacity)[None, :]).astype(np.float32)   # exact below 2^24
        done = ((occ[None, :] != 0) & (np.arange(self.K)[:, None] < b[None, :])).astype(np.uint8)
        return rew, done, 0.1

    def finish(self):
        pass

    def obs_of(self, slots):
        return np.zeros((len(slots), 4, 64, 32), dtype=np.uint8)

    def state_of(self, slots):
        return self.steps_run[slots].copy()


class FakeClock:
    """Time advances 1 ms per clock read, and sleep jumps ahead."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t

    def sleep(self, dt):
        self.t += dt


def _groups(n, rate, max_size=300, steps=(5, 30), seed=11):
    gs = W.serving_groups(n, rate, seed=seed, n_roms=32, max_size=max_size,
                          min_steps=steps[0], max_steps=steps[1])
    return gs


@pytest.mark.parametrize("depth,K", [(1, 1), (2, 1), (3, 1), (2, 4), (1, 5), (3, 8)])
def test_every_group_runs_exactly_its_steps_in_its_own_slots(depth, K):
    spec = W.make_config("c4")
    groups = _groups(40, rate=400.0, steps=(5, 150))
    be = FakeBackend(capacity=700, depth=depth, steps_per_tick=K)
    clk = FakeClock()
    out = S.serve(spec, groups, be, record=True, clock=clk, sleep=clk.sleep)
    runs = out["runs"]
    assert len(runs) == len(groups)
    for r in runs:
        g = r.group
        assert r.t_admit >= r.t_arrival and r.t_done > r.t_admit
        # recorded rewards identify (global step, slot): consecutive steps, the group's own slots
        steps = (r.rewards[:, 0] // 1000).astype(int)
        slots = (r.rewards % 1000).astype(int)
        assert np.all(np.diff(steps) == 1), "a resident group steps in every step of every tick"
        assert steps[0] % K == 0, "a group starts at a tick boundary"
        assert np.all(slots == r.slots[None, :].astype(int))
        assert r.dones.all(), "every recorded step of the group ran"
        # the group's slots ran exactly its steps (the budget stops it inside its last tick)
        assert np.all(r.final_state == g.steps)
        # the actions sent in those steps are the group's own stream
        for k in sorted({0, 63, 64, 65, g.steps // 2, g.steps - 1}):
            if k >= g.steps:
                continue
            sent = be.acts[steps[k]][r.slots]
            assert np.array_equal(sent, W.group_actions(g, k, 1, int(spec.num_actions[g.rom]))[0])
    assert be.max_used <= be.capacity
    assert not be.groups, "every group was retired"
    assert out["env_steps"] == sum(g.size * g.steps for g in groups)


def test_group_waits_for_memory_and_later_groups_backfill():
    spec = W.make_config("c4")
    # two big groups that cannot be resident together, then a small one
    gs = [W.Group(0, 0.0, 1, 600, 20, 5), W.Group(1, 0.0005, 2, 600, 20, 6),
          W.Group(2, 0.0006, 3, 50, 10, 7)]
    be = FakeBackend(capacity=700, depth=2)
    clk = FakeClock()
    out = S.serve(spec, gs, be, clock=clk, sleep=clk.sleep)
    r0, r1, r2 = out["runs"]
    assert r1.t_admit >= r0.t_done, "the second big group waits until the first leaves"
    assert r2.t_admit < r0.t_done, "the small group fills the free range meanwhile"
    assert be.max_used <= 700


def test_group_larger_than_pool_is_an_error():
    spec = W.make_config("c4")
    be = FakeBackend(capacity=100)
    clk = FakeClock()
    with pytest.raises(RuntimeError):
        S.serve(spec, [W.Group(0, 0.0, 0, 101, 5, 1)], be, clock=clk, sleep=clk.sleep)


def test_idle_pool_sleeps_until_next_arrival():
    spec = W.make_config("c4")
    gs = [W.Group(0, 0.0, 0, 10, 3, 1), W.Group(1, 5.0, 1, 10, 3, 2)]
    be = FakeBackend(capacity=64)
    clk = FakeClock()
    out = S.serve(spec, gs, be, clock=clk, sleep=clk.sleep)
    assert out["runs"][1].t_admit >= 5.0
    assert be.n == 6
    # with ticks of two steps a group of three steps takes two ticks
    be2 = FakeBackend(capacity=64, steps_per_tick=2)
    clk2 = FakeClock()
    S.serve(spec, gs, be2, clock=clk2, sleep=clk2.sleep)
    assert be2.n == 4


def test_group_generators_are_slot_independent_and_windowed():
    g = W.serving_groups(5, 10.0)[3]
    a = W.group_actions(g, 0, 150, 5)
    assert np.array_equal(a[70:130], W.group_actions(g, 70, 60, 5))
    assert a.min() >= 0 and a.max() < 5
    assert np.array_equal(W.group_env_seeds(g), W.group_env_seeds(g))
    h = W.group_horizons(g)
    assert h.dtype == np.uint32 and (h >= 1).all()


def test_a_group_takes_free_slots_wherever_they_are():
    """Free slots never fragment: a group larger than any run of free slots is
    admitted as soon as enough slots are free in total."""
    spec = W.make_config("c4")
    gs = [W.Group(0, 0.0, 1, 300, 40, 5), W.Group(1, 0.0, 2, 300, 10, 6), W.Group(2, 0.0, 3, 100, 40, 7),
          W.Group(3, 0.002, 4, 350, 10, 8)]
    be = FakeBackend(capacity=750, depth=2)
    clk = FakeClock()
    out = S.serve(spec, gs, be, record={3}, clock=clk, sleep=clk.sleep)
    r0, r1, r2, r3 = out["runs"]
    # group 3 (350 envs) fits once group 1 (300) leaves: slots 300..599 and 700..749
    assert r1.t_done <= r3.t_admit < r0.t_done
    assert len(np.flatnonzero(np.diff(r3.slots.astype(int)) != 1)) == 1      # two runs of slots
    assert r3.rewards is not None and r0.rewards is None   # only the sampled group is recorded
    assert be.max_used <= 750


def test_recorded_sample_sees_its_own_slots():
    spec = W.make_config("c4")
    groups = _groups(30, rate=400.0, steps=(5, 90))
    be = FakeBackend(capacity=500, depth=2)
    clk = FakeClock()
    sample = {g.gid for g in groups[::7]}
    out = S.serve(spec, groups, be, record=sample, clock=clk, sleep=clk.sleep)
    for r in out["runs"]:
        if r.group.gid in sample:
            slots = (r.rewards % 1000).astype(int)
            assert np.all(slots == r.slots[None, :].astype(int))
        else:
            assert r.rewards is None


def test_ticks_longer_than_an_action_window_are_rejected():
    # a tick reads one window of each group's actions; a longer tick would
    # run steps whose actions were never written
    spec = W.make_config("c4")
    be = FakeBackend(capacity=64, depth=2, steps_per_tick=S.WINDOW + 1)
    with pytest.raises(ValueError):
        S.serve(spec, [W.Group(0, 0.0, 1, 8, 10, 5)], be)
