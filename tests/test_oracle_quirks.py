"""Pins of the oracle's quirk flags and game descriptors.

Each quirk switches one behaviour of the base profile; it is pinned against
the base profile itself (pinned by the instruction tests) on an input where
the two must agree, or against an independent definition:
  * SHIFT_VX: 8XY6 / 8XYE equal the base instruction with Y = X, for every VX,
    and VY is not read;
  * MEM_KEEP_I: FX55 / FX65 leave memory and registers as the base profile
    does, with I unchanged;
  * JUMP_VX: BXNN equals the base BNNN run with V0 set to VX;
  * NO_VF_RESET: 8XY1/2/3 give the base result in VX and leave VF alone;
  * PIXEL_WRAP: DXYN equals XOR with the sprite drawn at the origin of an
    empty 64x32 canvas and rolled by (VX, VY) with numpy.roll (wrap-around by
    definition), the collision flag being any lit pixel under a sprite pixel;
    where the sprite fits on the screen it equals the clipped draw;
  * DISPLAY_WAIT: a step equals frames run by hand on a bare machine, one
    instruction at a time, each frame ending after a DXYN; and a three-
    instruction loop gives its closed form.
Game descriptors (Section 3.3, Appendix C.3): the score modes and
termination clauses are checked against the formulas the paper prints for
Pong, Space Flight, Airplane, Shooting Stars, Deep8 and Flight Runner
(tests/golden/game_descriptors.txt), and each op over every register value.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import workload as W
from tests.golden_util import GOLDEN

BASE = 1
SHIFT_VX, MEM_KEEP_I, JUMP_VX, NO_VF_RESET, PIXEL_WRAP, DISPLAY_WAIT = (1 << 1), (1 << 2), (1 << 3), (1 << 4), (1 << 5), (1 << 6)


def _run(op, quirks, v, i=0x300, mem=None, disp=None):
    m = O.Machine(W.assemble([op]), quirks=quirks)
    s = m.state()
    s["v"] = v
    s["i"] = i
    if mem is not None:
        s["mem"][0x300:0x300 + len(mem)] = mem
    if disp is not None:
        s["disp"] = disp
    m.set_state(s)
    m.execute(1)
    return m.state()


def test_shift_vx_is_the_base_shift_with_y_equal_x():
    rng = np.random.default_rng(1)
    for n in (0x6, 0xE):
        for vx in range(256):
            v = rng.integers(0, 256, 16).astype(np.uint8)
            v[3] = vx
            q = _run(0x8350 | n, BASE | SHIFT_VX, v)
            b = _run(0x8330 | n, BASE, v)                 # base profile, 8X X n
            assert np.array_equal(q["v"], b["v"]), (n, vx)
            v2 = v.copy()
            v2[5] ^= 0xA5                                  # VY is not read
            assert np.array_equal(_run(0x8350 | n, BASE | SHIFT_VX, v2)["v"][[3, 15]], q["v"][[3, 15]])
    # and the base profile does read VY
    v = np.zeros(16, np.uint8)
    v[5] = 0x81
    assert _run(0x8356, BASE, v)["v"][3] == 0x40


@pytest.mark.parametrize("nn", [0x55, 0x65])
def test_mem_keep_i_changes_only_i(nn):
    rng = np.random.default_rng(2)
    for x in range(16):
        v = rng.integers(0, 256, 16).astype(np.uint8)
        mem = rng.integers(0, 256, 16).astype(np.uint8)
        op = 0xF000 | (x << 8) | nn
        q = _run(op, BASE | MEM_KEEP_I, v, mem=mem)
        b = _run(op, BASE, v, mem=mem)
        assert q["i"] == 0x300
        assert b["i"] == 0x300 + x + 1
        assert np.array_equal(q["v"], b["v"]) and np.array_equal(q["mem"], b["mem"]), (nn, x)


def test_jump_vx_is_the_base_jump_with_v0_set():
    rng = np.random.default_rng(3)
    for x in range(16):
        for _ in range(8):
            v = rng.integers(0, 256, 16).astype(np.uint8)
            nn = int(rng.integers(0, 256))
            op = 0xB000 | (x << 8) | nn
            q = _run(op, BASE | JUMP_VX, v)
            vb = v.copy()
            vb[0] = v[x]
            b = _run(op, BASE, vb)
            assert q["pc"] == b["pc"], (x, nn)
            assert q["pc"] == (((x << 8) | nn) + int(v[x])) & 0xFFF


@pytest.mark.parametrize("n", [1, 2, 3])
def test_no_vf_reset_keeps_vf(n):
    rng = np.random.default_rng(4 + n)
    for _ in range(64):
        v = rng.integers(0, 256, 16).astype(np.uint8)
        for x, y in ((3, 5), (0, 14), (7, 7)):
            op = 0x8000 | (x << 8) | (y << 4) | n
            q = _run(op, BASE | NO_VF_RESET, v)
            b = _run(op, BASE, v)
            assert b["v"][15] == 0                        # the base profile clears VF
            assert q["v"][x] == b["v"][x]
            assert q["v"][15] == v[15]
    # 8FY1: the result lands in VF itself and stays there
    v = np.zeros(16, np.uint8)
    v[15], v[2] = 0x10, 0x03
    assert _run(0x8F21, BASE | NO_VF_RESET, v)["v"][15] == 0x13
    assert _run(0x8F21, BASE, v)["v"][15] == 0


def _rolled(sprite_rows, x0, y0):
    canvas = np.zeros((32, 64), np.uint8)
    for r, byte in enumerate(sprite_rows):
        canvas[r, :8] = [(int(byte) >> (7 - c)) & 1 for c in range(8)]
    return np.roll(canvas, (y0, x0), axis=(0, 1))


def test_pixel_wrap_matches_a_rolled_canvas():
    rng = np.random.default_rng(7)
    cases = [(63, 31, 15), (60, 0, 5), (0, 28, 8), (57, 25, 15), (3, 4, 1), (56, 17, 15)]
    cases += [tuple(int(a) for a in (rng.integers(0, 64), rng.integers(0, 32), rng.integers(1, 16))) for _ in range(200)]
    for x0, y0, n in cases:
        sprite = rng.integers(0, 256, n).astype(np.uint8)
        disp = (rng.random((32, 64)) < 0.3).astype(np.uint8)
        v = np.zeros(16, np.uint8)
        v[1] = x0 + 64 * int(rng.integers(0, 4))              # coordinates are taken mod 64 / 32
        v[2] = y0 + 32 * int(rng.integers(0, 8))
        got = _run(0xD120 | n, BASE | PIXEL_WRAP, v, mem=sprite, disp=disp)
        c = _rolled(sprite, x0, y0)
        assert np.array_equal(got["disp"], disp ^ c), (x0, y0, n)
        assert got["v"][15] == int((disp & c).any()), (x0, y0, n)
        if x0 <= 56 and y0 + n <= 32:                         # fits: the clipped draw agrees
            base = _run(0xD120 | n, BASE, v, mem=sprite, disp=disp)
            assert np.array_equal(base["disp"], got["disp"]) and base["v"][15] == got["v"][15]


def test_clipped_draw_differs_from_wrap_at_the_edges():
    sprite = np.full(4, 0xFF, np.uint8)
    v = np.zeros(16, np.uint8)
    v[1], v[2] = 60, 30
    clip = _run(0xD124, BASE, v, mem=sprite)["disp"]
    wrap = _run(0xD124, BASE | PIXEL_WRAP, v, mem=sprite)["disp"]
    assert clip.sum() == 4 * 2 and wrap.sum() == 8 * 4
    assert wrap[0, 0] == 1 and clip[0, 0] == 0


def _golden(kind):
    rows = []
    for line in open(f"{GOLDEN}/game_descriptors.txt"):
        line = line.split("#")[0].split()
        if line and line[0] == kind:
            rows.append([int(t, 0) for t in line[1:]])
    assert len(rows) >= 4, kind
    return rows


def _u8(*v):
    return np.array(v, np.uint8)


def _idle_batch(n, **profile):
    spec = W.custom_spec([W.assemble([0x1200])], n, keys=W.KEYS_5)   # JP 0x200: registers never change
    return O.OracleBatch(dataclasses.replace(spec, **profile))


def _score_and_done(b, regs):
    """One step of an idle program from V set as given ({register: values}), score baseline 0."""
    s = b.get_state(0, b.E)
    s["v"] = 0
    for r, vals in regs.items():
        s["v"][:, r] = vals
    s["prev_score"] = 0
    b.set_state(0, s)
    _, rew, done = b.step(np.zeros(b.E, np.int32), want_obs=False)
    return rew, done


# (descriptor fields, registers read from each golden row, score column, done column)
GAMES = {
    "pong": (dict(score_reg=_u8(14), score_mode=_u8(1), score_arg=_u8(0)), (14,), 1, None),
    "pong_done": (dict(term_reg=_u8(14), term_value=_u8(9), term_op=_u8(4)), (14,), None, 1),
    "space_flight": (dict(term_reg=_u8(9), term_value=_u8(0), term2_op=_u8(2), term2_reg=_u8(12),
                          term2_value=_u8(0x3E)), (9, 12), None, 2),
    "airplane": (dict(score_reg=_u8(11), score_mode=_u8(2), score_arg=_u8(12), term_reg=_u8(11),
                      term_value=_u8(0), term2_op=_u8(1), term2_reg=_u8(12), term2_value=_u8(6)), (11, 12), 2, 3),
    "shooting_stars": (dict(score_reg=_u8(0), score_mode=_u8(3), score_arg=_u8(128), term_op=_u8(0)), (0,), 1, 2),
    "deep": (dict(term_reg=_u8(11), term_value=_u8(1), term_op=_u8(3)), (11,), None, 1),
    "flight_runner": (dict(term_reg=_u8(5), term_value=_u8(255), term2_op=_u8(1), term2_reg=_u8(7),
                           term2_value=_u8(255)), (5, 7), None, 2),
}


@pytest.mark.parametrize("game", sorted(GAMES))
def test_descriptors_match_the_paper(game):
    prof, regs, score_col, done_col = GAMES[game]
    rows = np.array(_golden(game), dtype=np.int64)
    b = _idle_batch(len(rows), **prof)
    rew, done = _score_and_done(b, {r: rows[:, i] for i, r in enumerate(regs)})
    if score_col is not None:
        assert np.array_equal(rew, rows[:, score_col].astype(np.float32)), (rew, rows[:, score_col])
    if done_col is not None:
        assert np.array_equal(done, rows[:, done_col].astype(np.uint8)), (done, rows[:, done_col])


def test_bcd_score_over_every_register_value():
    b = _idle_batch(256, score_reg=_u8(14), score_mode=_u8(1), score_arg=_u8(0))
    rew, _ = _score_and_done(b, {14: np.arange(256)})
    tens_minus_ones = np.array([int(str(k)[:-1] or "0") - int(str(k)[-1]) for k in range(256)], np.float32)
    assert np.array_equal(rew, tens_minus_ones)


def test_clause_ops_over_every_register_value():
    # op 1..4 against constant 0x3E (ops 2, 3) or 7 (op 4), each register value once
    want = {1: lambda v: v == 0x3E, 2: lambda v: v >= 0x3E, 3: lambda v: v != 0x3E,
            4: lambda v: (str(v)[-1] == "7") or (len(str(v)) > 1 and str(v)[:-1] == "7")}
    for op, f in want.items():
        k = 7 if op == 4 else 0x3E
        b = _idle_batch(256, term_reg=_u8(3), term_value=_u8(k), term_op=_u8(op))
        _, done = _score_and_done(b, {3: np.arange(256)})
        assert np.array_equal(done.astype(bool), np.array([f(v) for v in range(256)])), op
        b = _idle_batch(256, term_op=_u8(0), term2_op=_u8(op), term2_reg=_u8(3), term2_value=_u8(k))
        _, done = _score_and_done(b, {3: np.arange(256)})        # the same op as the second clause
        assert np.array_equal(done.astype(bool), np.array([f(v) for v in range(256)])), op


def _frames_by_hand(m, key, ipf, frame_skip, wait):
    """One env step on a bare machine: each frame runs ipf instructions, or
    stops after a DXYN when `wait`, then ticks the timers."""
    for _ in range(frame_skip):
        for _ in range(ipf):
            s = m.state()
            draws = (int(s["mem"][s["pc"]]) >> 4) == 0xD
            m.execute(1, key)
            if wait and draws:
                break
        m.tick()


def test_display_wait_closed_form():
    # D011 draws, 7101 adds 1 to V1, 1200 loops: with the quirk the first
    # frame stops after the draw and every later frame runs the add once
    rom = W.assemble([0xD011, 0x7101, 0x1200])
    spec = W.custom_spec([rom], 1, keys=W.KEYS_5, instr_per_frame=10, frame_skip=4)
    b = O.OracleBatch(dataclasses.replace(spec, quirks=BASE | DISPLAY_WAIT, term_op=_u8(0)))
    base = O.OracleBatch(dataclasses.replace(spec, term_op=_u8(0)))
    for k in range(1, 4):
        b.step(np.zeros(1, np.int32), want_obs=False)
        base.step(np.zeros(1, np.int32), want_obs=False)
        assert b.get_state(0, 1)["v"][0, 1] == 4 * k - 1
        assert base.get_state(0, 1)["v"][0, 1] == (40 * k + 1) // 3   # the add is instruction 1 mod 3 of 40k


def test_display_wait_matches_frames_run_by_hand():
    spec = W.make_config("c3", num_envs=24)
    spec = dataclasses.replace(spec, quirks=BASE | DISPLAY_WAIT, term_op=np.zeros(spec.num_roms, np.uint8),
                               horizon=np.zeros(24, np.uint32))
    b = O.OracleBatch(spec)
    start = b.get_state(0, b.E)
    acts = spec.actions(0, 5)
    for k in range(5):
        b.step(acts[k], want_obs=False)
    got = O.canonical(b.get_state(0, b.E))
    drew_mid_frame = 0
    for e in range(b.E):
        m = O.Machine(quirks=BASE | DISPLAY_WAIT)
        m.set_state(start[e])
        r = int(spec.env_rom[e])
        for k in range(5):
            a = int(acts[k, e])
            key = int(spec.action_keys[r][a]) if a < spec.num_actions[r] else -1
            _frames_by_hand(m, key, spec.instr_per_frame, spec.frame_skip, True)
        want = O.canonical(np.array([m.state()], dtype=O.STATE_DTYPE))
        for f in ("v", "i", "pc", "sp", "dt", "st", "stack", "mem", "disp", "rng"):
            assert np.array_equal(got[f][e], want[f][0]), (e, f)
        m2 = O.Machine()
        m2.set_state(start[e])
        for k in range(5):
            a = int(acts[k, e])
            key = int(spec.action_keys[r][a]) if a < spec.num_actions[r] else -1
            _frames_by_hand(m2, key, spec.instr_per_frame, spec.frame_skip, False)
        drew_mid_frame += int(m2.state()["pc"] != m.state()["pc"])
    assert drew_mid_frame > 0                 # the quirk changed the run of some envs


def test_set_profile_rejects_out_of_range():
    b = _idle_batch(2)
    L = O.lib()
    none = [None] * 6
    assert L.oracle_set_profile(b._h, 0, *none) != 0                 # no base profile
    assert L.oracle_set_profile(b._h, 1 | (1 << 7), *none) != 0
    mode, arg = _u8(4), _u8(0)
    assert L.oracle_set_profile(b._h, 1, mode.ctypes.data, arg.ctypes.data, None, None, None, None) != 0
    mode[0], arg[0] = 2, 16                                          # negated sum needs a register
    assert L.oracle_set_profile(b._h, 1, mode.ctypes.data, arg.ctypes.data, None, None, None, None) != 0
    assert L.oracle_set_profile(b._h, 1, mode.ctypes.data, None, None, None, None, None) != 0
    op = _u8(5)
    assert L.oracle_set_profile(b._h, 1, None, None, op.ctypes.data, None, None, None) != 0
    op2, reg, val = _u8(1), _u8(16), _u8(0)
    assert L.oracle_set_profile(b._h, 1, None, None, None, op2.ctypes.data, reg.ctypes.data, val.ctypes.data) != 0
    assert L.oracle_set_profile(b._h, 1, None, None, None, op2.ctypes.data, None, val.ctypes.data) != 0
    assert L.oracle_set_profile(b._h, 1 | PIXEL_WRAP | DISPLAY_WAIT, *none) == 0


def test_mixed_workload_exercises_every_flag():
    """The generated mixed-ROM workload of the GPU parity tests reaches each
    quirk: with any one flag on, the oracle's states part from the base
    profile's within a few steps."""
    spec = W.make_config("c3", num_envs=64)
    base = O.OracleBatch(spec)
    acts = spec.actions(0, 6)
    for k in range(6):
        base.step(acts[k], want_obs=False)
    ref = O.canonical(base.get_state(0, base.E))
    for flag in (SHIFT_VX, MEM_KEEP_I, JUMP_VX, NO_VF_RESET, PIXEL_WRAP, DISPLAY_WAIT):
        b = O.OracleBatch(dataclasses.replace(spec, quirks=BASE | flag))
        for k in range(6):
            b.step(acts[k], want_obs=False)
        got = O.canonical(b.get_state(0, b.E))
        assert any(not np.array_equal(got[f], ref[f]) for f in ("v", "i", "pc", "mem", "disp")), hex(flag)
