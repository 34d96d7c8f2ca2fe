"""The oracle at the 0xFFF -> 0x000 boundary, pinned by a hand-worked
program (Section 2: a 4 KB address space, programs at 0x200; addresses wrap
mod 4,096 and sprite pixels past the right or bottom edge are clipped).

WRAP_PROGRAM loops: it draws 15 sprite rows from 0xFF8 (rows 8..14 read
0x000..0x006), writes the BCD digits of 240 to 0xFFE..0x000, stores V0..V7
to 0xFFC..0x003 and loads V0..V5 back from 0xFFD..0x002, counts in VC and
jumps to 0xFFF, whose instruction word is RAM[0xFFF] << 8 | RAM[0x000]
= 0x12 << 8 | 0x00 (V3 and V4 as stored), a jump back to 0x200.  After 64
rounds it falls through to a clear and starts over.  The expected values
below were worked out by hand from the standard instruction meanings.
"""
import numpy as np

from oracle import oracle as O

WRAP_PROGRAM = bytes.fromhex(
    "6A12"  # 200 VA = 0x12
    "6312"  # 202 V3 = 0x12
    "6400"  # 204 V4 = 0x00
    "6581"  # 206 V5 = 0x81
    "6642"  # 208 V6 = 0x42
    "6724"  # 20A V7 = 0x24
    "60F0"  # 20C V0 = 240
    "613A"  # 20E V1 = 58
    "6210"  # 210 V2 = 16
    "AFF8"  # 212 I = 0xFF8
    "D12F"  # 214 draw 15 rows at (V1, V2)
    "AFFE"  # 216 I = 0xFFE
    "F033"  # 218 BCD of V0 at I
    "AFFC"  # 21A I = 0xFFC
    "F755"  # 21C store V0..V7 at I, I += 8
    "AFFD"  # 21E I = 0xFFD
    "F565"  # 220 load V0..V5 from I, I += 6
    "7C01"  # 222 VC += 1
    "3C40"  # 224 skip if VC == 0x40
    "1FFF"  # 226 jump 0xFFF
    "00E0"  # 228 clear
    "6C00"  # 22A VC = 0
    "1200"  # 22C jump 0x200
)
LOOP = 20   # instructions from 0x200 through the jump to 0xFFF


def test_first_round_writes_and_reads_across_the_wrap():
    m = O.Machine(WRAP_PROGRAM)
    m.execute(LOOP)
    s = m.state()
    assert s["pc"] == 0xFFF
    # F755 overwrote the BCD digits: V0..V3 at 0xFFC..0xFFF, V4..V7 at 0x000..0x003
    assert list(s["mem"][0xFFC:]) == [240, 58, 16, 0x12]
    assert list(s["mem"][:4]) == [0x00, 0x81, 0x42, 0x24]
    # F565 from 0xFFD: V0..V5 = 58, 16, 0x12, 0x00, 0x81, 0x42; I = 0xFFD + 6 - 0x1000
    assert list(s["v"][:6]) == [58, 16, 0x12, 0x00, 0x81, 0x42]
    assert s["i"] == 0x003
    assert s["v"][0xC] == 1 and s["v"][0xF] == 0
    assert not s["disp"].any()          # the first draw read only zero bytes
    # the instruction at 0xFFF takes its low byte from 0x000: 0x1200
    m.execute(1)
    assert m.state()["pc"] == 0x200


def test_second_draw_reads_sprite_rows_across_the_wrap_and_clips():
    m = O.Machine(WRAP_PROGRAM)
    m.execute(LOOP + 1 + 11)            # through the second round's DXYN
    s = m.state()
    assert s["pc"] == 0x216
    # sprite rows r = 0..14 at (0xFF8 + r) & 0xFFF, drawn at x 58.., y 16 + r;
    # columns 64 and past are clipped
    rows = {4: 0xF0, 5: 58, 6: 16, 7: 0x12, 9: 0x81, 10: 0x42, 11: 0x24}
    want = np.zeros((32, 64), dtype=np.uint8)
    for r, b in rows.items():
        for c in range(8):
            if (b >> (7 - c)) & 1 and 58 + c < 64:
                want[16 + r, 58 + c] = 1
    assert int(want.sum()) == 13
    assert np.array_equal(s["disp"], want)
    assert s["v"][0xF] == 0             # nothing was set before: no collision
    # the same draw again erases every pixel it set: collision
    m.poke(pc=0x214)
    m.execute(1)
    s = m.state()
    assert not s["disp"].any() and s["v"][0xF] == 1


def test_loop_counter_wraps_to_the_clear():
    m = O.Machine(WRAP_PROGRAM)
    m.execute(64 * (LOOP + 1) - 2)      # the 64th round's skip: VC == 0x40
    s = m.state()
    assert s["v"][0xC] == 0x40 and s["pc"] == 0x228
    m.execute(3)                        # clear, VC = 0, jump
    s = m.state()
    assert s["pc"] == 0x200 and s["v"][0xC] == 0 and not s["disp"].any()
