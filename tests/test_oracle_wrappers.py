"""Pins of the oracle's environment wrappers (Section 3.2: start-up sequences,
no-op reset, sticky actions).

Each wrapper is checked against the case it reduces to, run by the oracle
with the wrappers off:
  * sticky actions with probability 1 hold no key at all, so on programs
    that draw no random numbers they equal a run of no-op actions;
  * with probability p, the share of steps that keep the previous key while
    the action asks for another one is p (statistical, 2^17 samples);
  * a start-up sequence equals power-on followed by steps whose actions hold
    the listed keys, on the same RNG stream;
  * a no-op reset leaves each env in the state of power-on followed by n
    no-op steps for some n in 0..noop_max, and n is spread uniformly;
  * after a reset the frame stack holds the display four times, the score
    baseline is the score register and the step count is zero.
Programs come from the seeded generator with the random-number class
switched off wherever the comparison needs the RNG stream to be irrelevant.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import workload as W

ARCH = ("v", "i", "pc", "sp", "dt", "st", "stack", "mem", "disp")


def _spec(E, seed=11, R=4, rnd=0.0, horizon=0, keys=W.KEYS_8, misc=0.005):
    mix = W.OpcodeMix(rnd=rnd, key=0.2, misc=misc)
    roms = [W.gen_rom(seed * 100 + r, 300, mix, keys) for r in range(R)]
    return W.custom_spec(roms, E, keys=keys, horizon=horizon, seed=seed,
                         env_rom=(np.arange(E) % R).astype(np.uint16))


def _arch(b):
    return O.canonical(b.get_state(0, b.E))


def _same(a, b, fields=ARCH, where=""):
    for f in fields:
        assert np.array_equal(a[f], b[f]), f"{where}: {f} differs"


def test_always_sticky_equals_noop_actions():
    spec = _spec(256, horizon=40)
    noop = np.asarray(spec.num_actions)[spec.env_rom].astype(np.int32)   # action index K = no key
    a = O.OracleBatch(dataclasses.replace(spec, sticky_q24=1 << 24))
    b = O.OracleBatch(spec)
    for k in range(120):
        _, ra, da = a.step(spec.actions(k, 1)[0], want_obs=False)
        _, rb, db = b.step(noop, want_obs=False)
        assert np.array_equal(ra, rb) and np.array_equal(da, db), k
    _same(_arch(a), _arch(b), ARCH + ("t", "prev_score", "hist"), "after 120 steps")
    assert (a.get_state(0, a.E)["prev_key"] == 16).all()


def test_sticky_share_matches_probability():
    p = 0.25
    spec = dataclasses.replace(_spec(1024, rnd=0.02, horizon=50), sticky_q24=int(p * (1 << 24)))
    b = O.OracleBatch(spec)
    keys = np.asarray(spec.action_keys)[spec.env_rom]
    prev = b.get_state(0, b.E)["prev_key"].astype(np.int64)
    kept = asked = 0
    for k in range(128):
        act = spec.actions(k, 1)[0]
        want = keys[np.arange(b.E), act].astype(np.int64)
        _, _, done = b.step(act, want_obs=False)
        cur = b.get_state(0, b.E)["prev_key"].astype(np.int64)
        live = done == 0                      # a reset sets the previous key to none
        assert (cur[~live] == 16).all()
        differ = (want != prev) & live
        asked += int(differ.sum())
        kept += int((differ & (cur == prev)).sum())
        assert np.all(((cur == prev) | (cur == want))[live]), "the held key is neither the previous nor the asked one"
        prev = cur
    share = kept / asked
    assert asked > 60000
    assert abs(share - p) < 0.01, share


def test_startup_sequence_replays_its_keys():
    spec = _spec(64, rnd=0.05)          # the RNG stream is shared: draws must line up
    R = spec.num_roms
    rng = np.random.default_rng(5)
    lens = np.array([0, 1, 3, 5], dtype=np.uint8)[:R]
    akeys = np.asarray(spec.action_keys)
    nact = np.asarray(spec.num_actions)
    picks = rng.integers(0, nact[0] + 1, size=(R, 16))            # action index; nact = no key
    skeys = np.where(picks < nact[:, None], akeys[np.arange(R)[:, None], np.minimum(picks, 15)], 16).astype(np.uint8)
    wspec = dataclasses.replace(spec, startup_len=lens, startup_keys=skeys)
    a = O.OracleBatch(wspec)
    b = O.OracleBatch(spec)
    for i in range(int(lens.max())):
        act = np.where(i < lens[spec.env_rom], picks[spec.env_rom, i], nact[spec.env_rom]).astype(np.int32)
        # envs whose sequence is shorter must not step: run them separately
        sb = b.get_state(0, b.E)
        b.step(act, want_obs=False)
        sa = b.get_state(0, b.E)
        done_envs = i >= lens[spec.env_rom]
        sa[done_envs] = sb[done_envs]
        b.set_state(0, sa)
    ga, gb = O.canonical(a.get_state(0, a.E)), O.canonical(b.get_state(0, b.E))
    _same(ga, gb, ARCH + ("rng",), "after the start-up sequence")
    assert (ga["t"] == 0).all()
    assert np.array_equal(ga["prev_score"], ga["v"][np.arange(a.E), np.asarray(spec.score_reg)[spec.env_rom]])
    for h in range(3):
        assert np.array_equal(ga["hist"][:, h], ga["disp"])
    obs = a.reset(want_obs=True)
    assert all(np.array_equal(obs[:, f], obs[:, 3]) for f in range(3))


def test_noop_reset_lands_on_a_prefix_of_noop_steps():
    nmax = 7
    E = 2048
    # no FX0A: with no key held it waits, so a program that reaches one stops changing
    spec = _spec(E, R=1, seed=23, misc=0.0)
    a = O.OracleBatch(dataclasses.replace(spec, noop_max=nmax))
    # power-on followed by n no-op steps, n = 0..nmax (one ROM, no RNG use: the same for all envs)
    b = O.OracleBatch(spec.subset(np.arange(1)))
    noop = np.array([spec.num_actions[0]], dtype=np.int32)
    prefixes = []
    for n in range(nmax + 1):
        prefixes.append(O.canonical(b.get_state(0, 1)))
        b.step(noop, want_obs=False)
    got = O.canonical(a.get_state(0, E))
    counts = np.zeros(nmax + 1, dtype=np.int64)
    for e in range(E):
        match = [n for n in range(nmax + 1)
                 if all(np.array_equal(got[f][e], prefixes[n][f][0]) for f in ARCH)]
        assert match, f"env {e} is not in the state of any no-op prefix"
        counts[match[0]] += 1
    expected = E / (nmax + 1)
    assert counts.min() > 0.6 * expected and counts.max() < 1.4 * expected, counts


def test_wrappers_apply_at_automatic_reset():
    spec = _spec(128, R=2, seed=31, horizon=3)
    lens = np.array([2, 1], dtype=np.uint8)
    skeys = np.zeros((2, 16), dtype=np.uint8)
    skeys[0, :2] = [spec.action_keys[0][1], 16]
    skeys[1, 0] = spec.action_keys[1][2]
    wspec = dataclasses.replace(spec, startup_len=lens, startup_keys=skeys)
    a = O.OracleBatch(wspec)
    fresh = O.canonical(a.get_state(0, a.E))        # after the create-time reset
    for k in range(3):
        _, _, d = a.step(spec.actions(k, 1)[0], want_obs=False)
    assert (d == 2).all()                           # truncated at the horizon
    after = O.canonical(a.get_state(0, a.E))
    _same(after, fresh, ARCH + ("t", "prev_score", "hist"), "after the automatic reset")


def test_set_wrappers_rejects_out_of_range():
    b = O.OracleBatch(_spec(4))
    L = O.lib()
    assert L.oracle_set_wrappers(b._h, (1 << 24) + 1, 0, None, None) != 0
    assert L.oracle_set_wrappers(b._h, 0, 1001, None, None) != 0
    bad = np.array([17, 0, 0, 0], dtype=np.uint8)
    keys = np.zeros((4, 16), dtype=np.uint8)
    assert L.oracle_set_wrappers(b._h, 0, 0, bad.ctypes.data, keys.ctypes.data) != 0
