"""Pins of the oracle's SUPER-CHIP platform (the 128x64 extension the paper
names in Section 5; readings in the oracle's header).

  * A 64x32-mode SUPER-CHIP machine running CHIP-8 code equals the pinned
    CHIP-8 machine with every pixel drawn as a 2x2 block (whole generated
    programs, thousands of instructions).
  * DXYN / DXY0 in the 128x64 mode equal an independent numpy rasteriser
    (clip, and numpy.roll for the wrap quirk), collision flag included.
  * Scrolls equal numpy shifts with zero fill, by pixels of the mode.
  * FX30 glyphs reproduce their pictures (tests/golden/big_font_glyphs.txt);
    FX75 / FX85 round-trip V0..V(min(X, 7)); 00FE / 00FF clear and switch
    mode; 00FD stays on itself.
  * Environment: (4, 128, 64) observations whose last frame is the display
    and whose first three are the previous steps' displays.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import workload as W
from tests.golden_util import big_font_pictures

PIXEL_WRAP = 1 << 5


def _m(ops, quirks=1, hires=False, **regs):
    rom = W.assemble(([0x00FF] if hires else []) + list(ops))
    m = O.Machine(rom, quirks=quirks, schip=True)
    if hires:
        m.execute(1)
    return m


def test_lores_runs_chip8_code_as_2x2_blocks():
    spec = W.make_config("c3", num_envs=1)
    for r in range(6):
        rom = spec.roms[r]
        a, b = O.Machine(rom), O.Machine(rom, schip=True)
        s = a.state()
        s["rng"] = 12345 + r
        a.set_state(s)
        b.set_state(s)
        for k in range(300):
            key = (k // 7) % 17 - 1
            a.execute(10, key)
            b.execute(10, key)
            a.tick()
            b.tick()
            sa, sb = a.state(), b.state()
            for f in ("v", "i", "pc", "sp", "dt", "st", "stack", "mem", "rng"):
                assert np.array_equal(sa[f], sb[f]), (r, k, f)
            assert np.array_equal(np.kron(sa["disp"], np.ones((2, 2), np.uint8)), b.schip()["hd"]), (r, k)


def _raster(sprite_rows, w, x0, y0, wrap):
    canvas = np.zeros((64, 128), np.uint8)
    for r, bits in enumerate(sprite_rows):
        row = [(int(bits) >> (w - 1 - c)) & 1 for c in range(w)]
        canvas[r, :w] = row
    if wrap:
        return np.roll(canvas, (y0, x0), axis=(0, 1))
    out = np.zeros_like(canvas)
    h = min(len(sprite_rows), 64 - y0)
    cw = min(w, 128 - x0)
    out[y0:y0 + h, x0:x0 + cw] = canvas[:h, :cw]
    return out


@pytest.mark.parametrize("wrap", [False, True])
def test_hires_draw_matches_a_rasteriser(wrap):
    rng = np.random.default_rng(3 + wrap)
    cases = [(127, 63, 0), (120, 60, 5), (0, 0, 0), (113, 49, 0), (64, 32, 15)]
    cases += [(int(rng.integers(0, 128)), int(rng.integers(0, 64)), int(rng.integers(0, 16))) for _ in range(150)]
    for x0, y0, n in cases:
        big = n == 0
        data = rng.integers(0, 256, 32 if big else n).astype(np.uint8)
        disp = (rng.random((64, 128)) < 0.3).astype(np.uint8)
        m = _m([0xD120 | n], quirks=1 | (PIXEL_WRAP if wrap else 0), hires=True)
        s = m.state()
        s["v"][1] = x0 + 128 * int(rng.integers(0, 2))
        s["v"][2] = y0 + 64 * int(rng.integers(0, 4))
        s["i"] = 0x300
        s["mem"][0x300:0x300 + len(data)] = data
        m.set_state(s)
        view = m.schip()
        view["hd"] = disp
        m.set_schip(view)
        m.execute(1)
        rows = [(int(data[2 * r]) << 8) | int(data[2 * r + 1]) for r in range(16)] if big else list(data)
        c = _raster(rows, 16 if big else 8, x0, y0, wrap)
        got = m.schip()
        assert np.array_equal(got["hd"], disp ^ c), (x0, y0, n)
        assert m.state()["v"][15] == int((disp & c).any()), (x0, y0, n)


def test_lores_big_sprite_is_blocks_of_a_16x16_draw():
    rng = np.random.default_rng(9)
    for _ in range(40):
        x0, y0 = int(rng.integers(0, 64)), int(rng.integers(0, 32))
        data = rng.integers(0, 256, 32).astype(np.uint8)
        m = _m([0xD120])
        s = m.state()
        s["v"][1], s["v"][2], s["i"] = x0, y0, 0x300
        s["mem"][0x300:0x320] = data
        m.set_state(s)
        m.execute(1)
        rows = [(int(data[2 * r]) << 8) | int(data[2 * r + 1]) for r in range(16)]
        logical = _raster(rows, 16, x0, y0, False)[:32, :64]
        assert np.array_equal(m.schip()["hd"], np.kron(logical, np.ones((2, 2), np.uint8)))


@pytest.mark.parametrize("hires", [True, False])
def test_scrolls_match_numpy_shifts(hires):
    rng = np.random.default_rng(5)
    sc = 1 if hires else 2
    for op, shift in [(0x00C1, (1, 0)), (0x00C7, (7, 0)), (0x00CF, (15, 0)), (0x00FB, (0, 4)), (0x00FC, (0, -4))]:
        m = _m([op], hires=hires)
        disp = (rng.random((64, 128)) < 0.5).astype(np.uint8)
        if not hires:
            disp = np.kron(disp[:32, :64], np.ones((2, 2), np.uint8))
        view = m.schip()
        view["hd"] = disp
        m.set_schip(view)
        m.execute(1)
        dy, dx = shift[0] * sc, shift[1] * sc
        want = np.zeros_like(disp)
        ys, xs = slice(max(dy, 0), 64 + min(dy, 0)), slice(max(dx, 0), 128 + min(dx, 0))
        yd, xd = slice(max(-dy, 0), 64 - max(dy, 0)), slice(max(-dx, 0), 128 - max(dx, 0))
        want[ys, xs] = disp[yd, xd]
        assert np.array_equal(m.schip()["hd"], want), hex(op)


def test_big_digits_match_their_pictures():
    pics = big_font_pictures()
    for d in range(16):
        m = _m([0xF130], hires=True)             # I := big digit V1
        s = m.state()
        s["v"][1], s["v"][2], s["v"][3] = d, 7, 9
        m.set_state(s)
        m.execute(1)
        assert m.state()["i"] == 0x0A0 + 10 * d
        m2 = _m([0xF130, 0xD23A], hires=True)
        s2 = m2.state()
        s2["v"][1], s2["v"][2], s2["v"][3] = d, 7, 9
        m2.set_state(s2)
        m2.execute(2)
        hd = m2.schip()["hd"]
        assert np.array_equal(hd[9:19, 7:15], pics[d]), d
        assert hd.sum() == pics[d].sum()
    assert np.array_equal(O.Machine(b"", schip=True).state()["mem"][0xA0:0x140].reshape(16, 10),
                          np.packbits(pics, axis=2)[:, :, 0])


def test_flag_registers_round_trip():
    for x in range(16):
        top = min(x, 7)
        m = _m([0xF075 | (x << 8), 0x6000, 0x6100, 0x6200, 0x6300, 0x6400, 0x6500, 0x6600, 0x6700, 0x6800,
                0xF085 | (x << 8)])
        s = m.state()
        s["v"] = np.arange(16, dtype=np.uint8) + 100
        m.set_state(s)
        m.execute(11)
        v = m.state()["v"]
        assert np.array_equal(v[:top + 1], np.arange(top + 1) + 100), x
        assert (v[top + 1:9] == 0).all() and np.array_equal(v[9:], np.arange(9, 16) + 100)
        assert np.array_equal(m.schip()["rpl"][:top + 1], np.arange(top + 1) + 100)


def test_mode_switch_clear_and_stop():
    m = _m([0xD125, 0x00FF, 0xD125, 0x00FE, 0x00FD, 0x6001])
    s = m.state()
    s["i"] = 0x50
    m.set_state(s)
    m.execute(1)
    assert m.schip()["hd"].sum() > 0 and m.schip()["hires"] == 0
    m.execute(1)
    assert m.schip()["hd"].sum() == 0 and m.schip()["hires"] == 1
    m.execute(2)
    assert m.schip()["hd"].sum() == 0 and m.schip()["hires"] == 0
    pc = m.state()["pc"]
    m.execute(5)
    assert m.state()["pc"] == pc and m.state()["v"][0] == 0     # stopped on 00FD


def test_env_observations_and_reset():
    spec = W.make_config("s1", num_envs=32)
    b = O.OracleBatch(spec)
    obs0 = b.reset()
    assert obs0.shape == (32, 4, 128, 64) and obs0.sum() == 0
    v = b.get_schip()
    assert (v["hires"] == 0).all() and (v["rpl"] == 0).all() and v["hd"].sum() == 0
    prev = [v["hd"].copy()]
    dones = []
    for k in range(12):
        o, _, d = b.step(spec.actions(k, 1)[0])
        dones.append(d != 0)
        v = b.get_schip()
        live = ~np.any(dones[-3:], axis=0)                 # no reset in the frames compared
        assert np.array_equal(o[:, 3].transpose(0, 2, 1), v["hd"])
        if k >= 2:
            assert np.array_equal(o[live, 0].transpose(0, 2, 1), prev[-3][live])
        assert np.array_equal(o[live, 2].transpose(0, 2, 1), prev[-1][live])
        for f in range(3):                                  # a reset shows the reset display four times
            assert np.array_equal(o[d != 0, f], o[d != 0, 3])
        prev.append(v["hd"].copy())
    assert sum(int(p.sum()) for p in prev) > 0


def test_schip_program_generator():
    """gen_schip_rom is deterministic, keeps the final jump, and emits every
    SUPER-CHIP instruction kind over a workload's programs."""
    a = W.gen_schip_rom(7, 1000)
    assert a == W.gen_schip_rom(7, 1000) and a != W.gen_schip_rom(8, 1000)
    code = W.program_code_slots(1000)
    assert [(a[2 * k] << 8) | a[2 * k + 1] for k in range(code)].count(0x1200) == 1   # the main loop's end
    spec = W.make_config("s1", num_envs=8)
    # the stop instruction is rare: look for it over more programs than the workload's eight
    roms = spec.roms + [W.gen_schip_rom(s, 1792) for s in range(24)]
    ops = [(r[i] << 8) | r[i + 1] for r in roms for i in range(0, len(r), 2)]
    seen = {
        "00FE": any(op == 0x00FE for op in ops), "00FF": any(op == 0x00FF for op in ops),
        "00CN": any(op & 0xFFF0 == 0x00C0 for op in ops), "00FB": 0x00FB in ops, "00FC": 0x00FC in ops,
        "DXY0": any(op & 0xF00F == 0xD000 for op in ops), "FX30": any(op & 0xF0FF == 0xF030 for op in ops),
        "FX75": any(op & 0xF0FF == 0xF075 for op in ops), "FX85": any(op & 0xF0FF == 0xF085 for op in ops),
        "00FD": 0x00FD in ops,
    }
    assert all(seen.values()), seen
    assert spec.platform == 1 and spec.num_envs == 8
