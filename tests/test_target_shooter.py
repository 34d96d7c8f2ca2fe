"""The Target Shooter programs (three levels written in Octo for this
repository from the game's description in Appendix F.2, assembled by
paper_2510_01764_amd/octo.py) played on the oracle.

The game's contract with the environment (the paper's wrapper): score in V2,
game over when V3 == 1, keys 5 7 8 9 6 (up, left, down, right, shoot).
Checked here:
  * an aiming policy that reads the target's position scores 10 in level 1
    and the episode then ends, with rewards summing to 10;
  * with no key pressed, levels 2 and 3 end after ten expired targets with
    no reward, at the same step in every env (the game's clock does not
    depend on the random target positions);
  * in level 3 the target moves, and the aiming policy still scores;
  * V3 is 1 exactly at the steps that report termination.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import workload as W

UP, LEFT, DOWN, RIGHT, SHOOT, NOOP = range(6)


def _batch(level, n=8, ipf=10, seed=0):
    roms = W.target_shooter_roms()
    spec = W.custom_spec([roms[level - 1]], n, keys=W.KEYS_5, instr_per_frame=ipf,
                         score_reg=2, term_reg=3, term_value=1, seed=seed)
    return O.OracleBatch(spec)


def _aim(v):
    """Move the reticle's centre (top-left + 2) onto the 4x4 target, then shoot."""
    act = np.full(len(v), SHOOT, np.int32)
    for e in range(len(v)):
        cx, cy, tx, ty = (int(v[e, r]) for r in (0, 1, 4, 5))
        if cx > 59 or cy > 27:          # mid-tick (wrapped, about to be clamped): wait
            act[e] = NOOP
            continue
        wx, wy = max(tx - 1, 0), max(ty - 1, 0)
        if cx < wx:
            act[e] = RIGHT
        elif cx > wx:
            act[e] = LEFT
        elif cy < wy:
            act[e] = DOWN
        elif cy > wy:
            act[e] = UP
    return act


def _play(b, policy, steps):
    total = np.zeros(b.E)
    episodes = []
    for k in range(steps):
        s = b.get_state(0, b.E)
        act = policy(s["v"])
        _, r, d = b.step(act, want_obs=False)
        total += r
        after = b.get_state(0, b.E)
        for e in np.nonzero(d)[0]:
            episodes.append((int(e), k, float(total[e]), int(d[e])))
            total[e] = 0
        # a terminated env was reset: its V3 is 0 again; a live one has V3 == 0 too
        assert (after["v"][:, 3] == 0).all()
    return episodes


def test_programs_assemble_and_start_with_a_clear():
    for rom in W.target_shooter_roms():
        assert 100 < len(rom) < 400
        assert rom[:2] == bytes([0x00, 0xE0])


def test_level1_aiming_policy_scores_ten():
    b = _batch(1)
    eps = _play(b, _aim, 1500)
    assert len({e for e, *_ in eps}) == b.E, "every env finished an episode"
    for e, k, total, d in eps:
        assert d == 1 and total == 10.0, (e, k, total)


@pytest.mark.parametrize("level", [2, 3])
def test_idle_player_misses_ten_targets(level):
    b = _batch(level, seed=level)
    eps = _play(b, lambda v: np.full(len(v), NOOP, np.int32), 700)
    firsts = {}
    for e, k, total, d in eps:
        assert d == 1 and total == 0.0
        firsts.setdefault(e, k)
    assert len(firsts) == b.E and len(set(firsts.values())) == 1, firsts


def test_level3_target_moves_and_can_be_hit():
    b = _batch(3, seed=5)
    xs = []
    for k in range(30):
        xs.append(b.get_state(0, b.E)["v"][:, 4].copy())
        b.step(np.full(b.E, NOOP, np.int32), want_obs=False)
    assert all(len(np.unique(np.array(xs)[:, e])) > 5 for e in range(b.E))
    eps = _play(b, _aim, 1500)
    assert sum(total for *_, total, _ in eps) > 0
