"""Seeded synthetic workloads for the batched CHIP-8 environment step.

This module only draws inputs: ROM images, the env -> ROM map, per-ROM action
sets and reward/termination descriptors, per-env truncation horizons, per-env
RNG seeds and action streams.  It contains none of the emulator's arithmetic,
so both the CPU oracle and the HIP path can consume what it produces.

The paper's game ROMs are third-party files that are not available here, so
seed-generated programs stand in for them.  They keep the paper's shapes: a
program loaded at 0x200 in a 4 KB memory (Section 3.2, "ROM loading and
initialization"; Appendix B.2), a 64x32 display drawn with DXYN, a handful of
keys mapped through an action set (Section 3.3, "Action space optimization"),
a single score register and an equality termination test (Section 3.3,
"Score function design" / "Termination logic").

Every generator uses ``numpy.random.Generator(PCG64(seed))`` so a config is a
pure function of its seed.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

PROGRAM_START = 0x200
MEMORY_SIZE = 4096
# 0x200..0xFFF holds at most 3584 bytes = 1792 two-byte instructions.
MAX_PROGRAM_INSTRUCTIONS = (MEMORY_SIZE - PROGRAM_START) // 2
FONT_START = 0x050
# Scratch bytes below the program, used by the generator as a data area for
# BCD and register saves, like the data areas real games keep.
SCRATCH_START = 0x0A0
SCRATCH_END = 0x200

KEYS_5 = (5, 7, 8, 9, 6)  # the five-key set of the paper's Target Shooter wrapper (Appendix C)
KEYS_8 = (1, 2, 4, 5, 6, 7, 8, 9)


@dataclasses.dataclass(frozen=True)
class OpcodeMix:
    """Relative weights of the opcode classes the generator draws from."""

    draw: float = 0.15      # DXYN
    key: float = 0.10       # EX9E / EXA1
    alu: float = 0.25       # 8XY0..8XY7, 8XYE
    imm: float = 0.20       # 6XNN / 7XNN
    index: float = 0.08     # ANNN / FX1E / FX29
    mem: float = 0.05       # FX33 / FX55 / FX65
    branch: float = 0.12    # 1NNN 2NNN 00EE 3XNN 4XNN 5XY0 9XY0 BNNN
    timer: float = 0.03     # FX07 / FX15 / FX18
    rnd: float = 0.02       # CXNN
    misc: float = 0.005     # 00E0 / FX0A
    draw_n_min: int = 1
    draw_n_max: int = 8
    # Draw-heavy workloads load VX/VY near the screen edges before DXYN.
    edge_bias: bool = False

    def weights(self) -> np.ndarray:
        w = np.array([self.draw, self.key, self.alu, self.imm, self.index,
                      self.mem, self.branch, self.timer, self.rnd, self.misc],
                     dtype=np.float64)
        return w / w.sum()


CLASS_NAMES = ("draw", "key", "alu", "imm", "index", "mem", "branch", "timer", "rnd", "misc")


def _enc(op: int) -> List[int]:
    return [(op >> 8) & 0xFF, op & 0xFF]


# Stores (FX33 / FX55) of structured programs go to this scratch area, below
# the program and above the SUPER-CHIP big font (0x0A0..0x13F).
STORE_START = 0x140
STORE_END = 0x200
MAX_STORE = 16          # FX55 with X = F writes 16 bytes

_CLS = {c: k for k, c in enumerate(CLASS_NAMES)}
# Look-ahead of the quota draw: a class is drawn with probability proportional
# to how far its count trails weight x (instructions so far + _LOOK).
_LOOK = 8


@dataclasses.dataclass
class _Unit:
    """A run of words that control flow only ever enters at its first word."""

    words: List[int]
    skip: bool = False                  # a conditional skip of the next unit
    jump: Optional[int] = None          # forward jump by this many units
    call: Optional[int] = None          # 2NNN to this subroutine
    table: Optional[int] = None         # BNNN jump table, data register index
    table_v0: Optional[int] = None      # the table's V0: a copy of VX (None) or this constant
    terminator: bool = False


@dataclasses.dataclass
class Program:
    """A generated program and where a SUPER-CHIP instruction may replace a word."""

    rom: bytes
    replaceable: np.ndarray    # bool per instruction slot: a single-word unit, not a region's end
    code_slots: int            # instructions before the sprite-data tail


def program_code_slots(n_instr: int) -> int:
    """Instruction slots of a structured program before its sprite-data tail
    (one slot in sixteen, at least eight, is sprite data)."""
    return n_instr - max(8, n_instr // 16)


def gen_program(seed: int, n_instr: int, mix: OpcodeMix = OpcodeMix(),
                action_keys: Sequence[int] = KEYS_5) -> Program:
    """Draw one structured CHIP-8 program of ``n_instr`` two-byte slots.

    Layout, like the code of a real game: a main loop that ends with a jump
    back to 0x200, then subroutines that each end with 00EE, then a tail of
    sprite bytes (one slot in sixteen, at least eight).  Control flow stays in
    the code it came from:
    - 2NNN only targets a subroutine's first word; main calls any subroutine,
      the first half of the subroutines call only the second half, and the
      second half calls nothing, so the stack never holds more than two
      return addresses and 00EE only ever returns to a call;
    - 1NNN jumps forward by 1..16 units inside its own region (a unit is an
      instruction with the set-up instructions in front of it, entered only
      at its first word);
    - every skip (3X, 4X, 5X, 9X, EX9E, EXA1) is followed by a one-word unit
      and is never the last unit before a region's end;
    - BNNN is a four-way jump table: VX <- 6, VX <- VX AND VD, then V0 <- VX
      or V0 <- an even constant below 8, then BNNN with NNN the address of the
      next word, so the target is one of the next four one-word units under
      both the V0 and the VX reading of BNNN (X = NNN's top nibble); with the
      constant the two readings may pick different entries;
    - FX33 and FX55 always follow an ANNN that points at the scratch area
      (one in ten at the sprite tail instead), so stores never rewrite code.
    Opcode classes are drawn by quota (each class with probability
    proportional to how far its count trails its weight), so the program's
    class mix, set-up instructions and region ends included, is close to the
    weights.
    """
    if not (16 <= n_instr <= MAX_PROGRAM_INSTRUCTIONS):
        raise ValueError(f"n_instr must be in [16, {MAX_PROGRAM_INSTRUCTIONS}]")
    rng = np.random.Generator(np.random.PCG64(seed))

    def r(n):  # uniform int in [0, n)
        return int(rng.integers(0, n))

    code_slots = program_code_slots(n_instr)
    data_slots = n_instr - code_slots
    data_start = PROGRAM_START + 2 * code_slots
    data_bytes = 2 * data_slots
    main_len = max(8, code_slots // 2)
    sub_lens: List[int] = []
    left = code_slots - main_len
    while left >= 8:
        s = int(rng.integers(8, 41))
        if left - s < 8:
            s = left
        sub_lens.append(s)
        left -= s
    main_len += left
    n_sub = len(sub_lens)
    leaves = list(range(n_sub // 2, n_sub))
    w = mix.weights()
    counts = np.zeros(len(w))
    emitted = [0.0]
    key_p = min(0.5, 0.8 * w[_CLS["imm"]] / max(w[_CLS["key"]], 1e-9))
    edge_p = min(1.0, 0.8 * w[_CLS["imm"]] / max(w[_CLS["draw"]], 1e-9))
    dense_p = min(0.5, 0.8 * w[_CLS["index"]] / max(w[_CLS["draw"]], 1e-9))

    def pick(allowed: np.ndarray) -> str:
        d = w * (emitted[0] + _LOOK) - counts
        p = (np.maximum(d, 0.0) + 1e-3 * w) * allowed
        if p.sum() <= 0:
            p = allowed.astype(np.float64)
        return CLASS_NAMES[int(rng.choice(len(w), p=p / p.sum()))]

    def store_pointer(size: int) -> int:
        if data_bytes >= 2 * MAX_STORE and r(10) == 0:
            return data_start + r(data_bytes - size + 1)
        return STORE_START + r(STORE_END - STORE_START - size + 1)

    def index_target() -> int:
        c = r(4)
        if c == 0:
            return FONT_START + 5 * r(16)
        if c == 1:
            return data_start + r(data_bytes)
        if c == 2:
            return PROGRAM_START + r(2 * code_slots)
        return STORE_START + r(STORE_END - STORE_START)

    def make_unit(cls: str, single: bool, room: int, callees: Sequence[int]) -> _Unit:
        x, y, nn = r(16), r(16), r(256)
        if cls == "draw":
            n = int(rng.integers(mix.draw_n_min, mix.draw_n_max + 1))
            words = []
            if not single and room >= 3 and mix.edge_bias and rng.random() < dense_p:
                words.append(0xA000 | (data_start + r(data_bytes)))
            if not single and room >= 3 and mix.edge_bias and rng.random() < edge_p:
                if r(2):
                    words.append(0x6000 | (x << 8) | int(rng.integers(56, 71)))
                else:
                    words.append(0x6000 | (y << 8) | int(rng.integers(24, 37)))
            return _Unit(words + [0xD000 | (x << 8) | (y << 4) | n])
        if cls == "key":
            words = []
            if not single and room >= 3 and rng.random() < key_p:
                words.append(0x6000 | (x << 8) | int(action_keys[r(len(action_keys))]))
            return _Unit(words + [0xE000 | (x << 8) | (0x9E if r(2) else 0xA1)], skip=True)
        if cls == "alu":
            return _Unit([0x8000 | (x << 8) | (y << 4) | (0, 1, 2, 3, 4, 5, 6, 7, 0xE)[r(9)]])
        if cls == "imm":
            return _Unit([(0x6000 if r(2) else 0x7000) | (x << 8) | nn])
        if cls == "index":
            c = r(3)
            if c == 0:
                return _Unit([0xA000 | index_target()])
            return _Unit([(0xF01E if c == 1 else 0xF029) | (x << 8)])
        if cls == "mem":
            low = (0x33, 0x55, 0x65)[r(3)]
            if low == 0x65 or single or room < 3:
                return _Unit([0xF065 | (x << 8)])
            size = 3 if low == 0x33 else x + 1
            return _Unit([0xA000 | store_pointer(size), 0xF000 | (x << 8) | low])
        if cls == "branch":
            forms = ["jump", "call", "skip", "skip", "skip", "skip"]
            if not single and room >= 8:
                forms.append("table")
            if room <= 1:
                forms = ["jump", "call"]
            f = forms[r(len(forms))]
            if f == "call" and callees:
                return _Unit([0x2000], call=int(callees[r(len(callees))]))
            if f in ("jump", "call"):
                return _Unit([0x1000], jump=1 + r(16))
            if f == "table":
                return _Unit([0, 0, 0, 0], table=r(16), table_v0=(None if r(2) else 2 * r(4)))
            c = r(4)
            if c == 0:
                return _Unit([0x3000 | (x << 8) | nn], skip=True)
            if c == 1:
                return _Unit([0x4000 | (x << 8) | nn], skip=True)
            return _Unit([(0x5000 if c == 2 else 0x9000) | (x << 8) | (y << 4)], skip=True)
        if cls == "timer":
            return _Unit([0xF000 | (x << 8) | (0x07, 0x15, 0x18)[r(3)]])
        if cls == "rnd":
            return _Unit([0xC000 | (x << 8) | nn])
        return _Unit([0x00E0] if r(2) else [0xF00A | (x << 8)])

    def region(length: int, end_word: int, callees: Sequence[int]) -> List[_Unit]:
        units: List[_Unit] = []
        used = 0
        budget = length - 1
        force_single = 1           # the first unit of every region is one word
        while used < budget:
            room = budget - used
            allowed = np.ones(len(w))
            if room == 1:
                allowed[_CLS["key"]] = 0.0      # no skip right before the region's end
            single = force_single > 0
            u = make_unit(pick(allowed), single, room, callees)
            if len(u.words) > room or (single and len(u.words) > 1):
                raise AssertionError("unit does not fit")    # make_unit respects room and single
            units.append(u)
            used += len(u.words)
            # the region's end (a branch) is charged a share at a time over its units
            emitted[0] += len(u.words) * (1.0 + 1.0 / budget)
            counts[_CLS["branch"]] += len(u.words) / budget
            # classes of table words are fixed (VX <- 6: imm; AND: alu; V0: alu or imm; BNNN: branch)
            ops = u.words if u.table is None else \
                [0x6000, 0x8002, 0x8000 if u.table_v0 is None else 0x6000, 0xB000]
            for op in ops:
                counts[_CLS[opcode_class(op)]] += 1
            force_single = max(force_single - 1, 0)
            if u.skip:
                force_single = max(force_single, 1)
            if u.table is not None:
                force_single = max(force_single, 4)
        units.append(_Unit([end_word], terminator=True))
        return units

    regions = [region(main_len, 0x1000 | PROGRAM_START, list(range(n_sub)))]
    for k, n in enumerate(sub_lens):
        regions.append(region(n, 0x00EE, leaves if k < n_sub // 2 else []))

    # Lay out the regions back to back from 0x200 and resolve targets.
    addr: List[List[int]] = []
    a = PROGRAM_START
    for units in regions:
        row = []
        for u in units:
            row.append(a)
            a += 2 * len(u.words)
        addr.append(row)
    assert a == data_start
    words: List[int] = []
    replaceable: List[bool] = []
    for g, units in enumerate(regions):
        for i, u in enumerate(units):
            if u.jump is not None:
                u.words[0] = 0x1000 | addr[g][min(i + u.jump, len(units) - 1)]
            elif u.call is not None:
                u.words[0] = 0x2000 | addr[1 + u.call][0]
            elif u.table is not None:
                nnn = addr[g][i] + 8
                vx = (nnn >> 8) & 0xF
                v0 = 0x8000 | (vx << 4) if u.table_v0 is None else 0x6000 | u.table_v0
                u.words[:] = [0x6006 | (vx << 8), 0x8002 | (vx << 8) | (u.table << 4), v0, 0xB000 | nnn]
            words.extend(u.words)
            replaceable.extend([len(u.words) == 1 and not u.terminator] * len(u.words))
    out = bytearray()
    for op in words:
        out += bytes(_enc(op))
    out += rng.integers(0, 256, size=data_bytes, dtype=np.uint8).tobytes()
    replaceable.extend([False] * data_slots)
    assert len(out) == 2 * n_instr
    return Program(rom=bytes(out), replaceable=np.array(replaceable, dtype=bool),
                   code_slots=code_slots)


def gen_rom(seed: int, n_instr: int, mix: OpcodeMix = OpcodeMix(),
            action_keys: Sequence[int] = KEYS_5) -> bytes:
    """The bytes of a structured program (gen_program)."""
    return gen_program(seed, n_instr, mix, action_keys).rom


def gen_rom_escape(seed: int, n_instr: int, mix: OpcodeMix = OpcodeMix(),
                   action_keys: Sequence[int] = KEYS_5) -> bytes:
    """An unstructured program that leaves itself: the escape workload.

    Opcodes are drawn one slot at a time with no control-flow structure: a
    bare 00EE may return through an empty stack, a skip may jump over the
    final jump, stores may rewrite the code and BNNN may land anywhere in
    the 255 bytes after its target.  Most such programs leave their own
    code within a few hundred instructions and run on through the font and
    zero memory, which exercises the page-crossing, wrap-around and
    self-modifying paths of an emulator.  Not a stand-in for game code.

    Slot ``n_instr - 1`` is a jump back to 0x200 so the program is a main
    loop.  Jump and call targets are even addresses inside the program.  Some
    classes emit a short prologue in front of the drawn instruction (a key
    value loaded before a key test, a data-area pointer before a store, edge
    coordinates before a draw), as game code does.  Prologues count against
    the instruction budget, so the realised mix is close to, not exactly, the
    weights.
    """
    if not (2 <= n_instr <= MAX_PROGRAM_INSTRUCTIONS):
        raise ValueError(f"n_instr must be in [2, {MAX_PROGRAM_INSTRUCTIONS}]")
    rng = np.random.Generator(np.random.PCG64(seed))
    w = mix.weights()
    end = PROGRAM_START + 2 * (n_instr - 1)       # address of the final jump
    ops: List[int] = []

    def r(n):  # uniform int in [0, n)
        return int(rng.integers(0, n))

    def target():
        return PROGRAM_START + 2 * r(n_instr)

    def data_pointer():
        c = r(3)
        if c == 0:
            return FONT_START + 5 * r(16)
        if c == 1:
            return PROGRAM_START + r(2 * n_instr)
        return SCRATCH_START + r(SCRATCH_END - SCRATCH_START - 16)

    budget = n_instr - 1
    while len(ops) < budget:
        room = budget - len(ops)
        cls = CLASS_NAMES[int(rng.choice(len(w), p=w))]
        x, y, nn = r(16), r(16), r(256)
        seq: List[int]
        if cls == "draw":
            n = int(rng.integers(mix.draw_n_min, mix.draw_n_max + 1))
            seq = []
            if mix.edge_bias and room >= 3:
                seq.append(0x6000 | (x << 8) | int(rng.integers(56, 71)))
                seq.append(0x6000 | (y << 8) | int(rng.integers(24, 37)))
            seq.append(0xD000 | (x << 8) | (y << 4) | n)
        elif cls == "key":
            seq = []
            if room >= 2 and r(2):
                seq.append(0x6000 | (x << 8) | int(action_keys[r(len(action_keys))]))
            seq.append(0xE000 | (x << 8) | (0x9E if r(2) else 0xA1))
        elif cls == "alu":
            n = (0, 1, 2, 3, 4, 5, 6, 7, 0xE)[r(9)]
            seq = [0x8000 | (x << 8) | (y << 4) | n]
        elif cls == "imm":
            seq = [(0x6000 if r(2) else 0x7000) | (x << 8) | nn]
        elif cls == "index":
            c = r(3)
            if c == 0:
                seq = [0xA000 | data_pointer()]
            elif c == 1:
                seq = [0xF01E | (x << 8)]
            else:
                seq = [0xF029 | (x << 8)]
        elif cls == "mem":
            low = (0x33, 0x55, 0x65)[r(3)]
            seq = []
            if low != 0x65 and room >= 2 and r(4) != 0:
                seq.append(0xA000 | (SCRATCH_START + r(SCRATCH_END - SCRATCH_START - 16)))
            seq.append(0xF000 | (x << 8) | low)
        elif cls == "branch":
            c = r(8)
            if c == 0:
                seq = [0x1000 | target()]
            elif c == 1:
                seq = [0x2000 | target()]
            elif c == 2:
                seq = [0x00EE]
            elif c == 3:
                seq = [0x3000 | (x << 8) | nn]
            elif c == 4:
                seq = [0x4000 | (x << 8) | nn]
            elif c == 5:
                seq = [0x5000 | (x << 8) | (y << 4)]
            elif c == 6:
                seq = [0x9000 | (x << 8) | (y << 4)]
            else:
                seq = [0xB000 | (target() & 0xFFF)]
        elif cls == "timer":
            seq = [0xF000 | (x << 8) | (0x07, 0x15, 0x18)[r(3)]]
        elif cls == "rnd":
            seq = [0xC000 | (x << 8) | nn]
        else:
            seq = [0x00E0] if r(2) else [0xF00A | (x << 8)]
        ops.extend(seq[:room])
    ops.append(0x1000 | PROGRAM_START)
    assert len(ops) == n_instr
    out = bytearray()
    for op in ops:
        out += bytes(_enc(op))
    assert PROGRAM_START + len(out) <= MEMORY_SIZE and end == PROGRAM_START + len(out) - 2
    return bytes(out)


def gen_schip_rom(seed: int, n_instr: int, mix: OpcodeMix = OpcodeMix(),
                  action_keys: Sequence[int] = KEYS_8, share: float = 0.12) -> bytes:
    """A SUPER-CHIP program: a structured CHIP-8 program (gen_program) in
    which about ``share`` of the code slots are replaced by SUPER-CHIP
    instructions - mode switches 00FE / 00FF, scrolls 00CN / 00FB / 00FC,
    16x16 sprites DXY0, big digits FX30, flag registers FX75 / FX85 and,
    rarely, the stop instruction 00FD.  Only one-word units that do not end a
    region are replaced, so the control flow of the program stays intact.
    Half of the programs switch to the 128x64 mode in their first
    instruction.
    """
    prog = gen_program(seed, n_instr, mix, action_keys)
    out = bytearray(prog.rom)
    rng = np.random.Generator(np.random.PCG64([seed, 17]))
    kinds = ("lores", "hires", "scd", "scr", "scl", "big", "digit", "save", "load", "stop")
    p = np.array([0.01, 0.01, 0.08, 0.06, 0.06, 0.45, 0.18, 0.08, 0.07, 0.0005])
    slots = np.flatnonzero(prog.replaceable)
    rate = min(1.0, share * prog.code_slots / max(len(slots), 1))
    assert prog.replaceable[0]          # the main loop starts with a one-word unit
    for i in slots:
        if i == 0:
            if rng.random() < 0.5:
                out[0:2] = bytes(_enc(0x00FF))
            continue
        if rng.random() >= rate:
            continue
        k = kinds[int(rng.choice(len(kinds), p=p / p.sum()))]
        x, y = int(rng.integers(0, 16)), int(rng.integers(0, 16))
        op = {"lores": 0x00FE, "hires": 0x00FF, "scd": 0x00C0 | int(rng.integers(1, 16)),
              "scr": 0x00FB, "scl": 0x00FC, "big": 0xD000 | (x << 8) | (y << 4),
              "digit": 0xF030 | (x << 8), "save": 0xF075 | (x << 8), "load": 0xF085 | (x << 8),
              "stop": 0x00FD}[k]
        out[2 * i:2 * i + 2] = bytes(_enc(op))
    return bytes(out)


def opcode_class(op: int) -> str:
    """Classify one opcode into the generator's classes (for mix checks)."""
    hi = op >> 12
    low = op & 0xFF
    if hi == 0xD:
        return "draw"
    if hi == 0xE:
        return "key"
    if hi == 0x8:
        return "alu"
    if hi in (0x6, 0x7):
        return "imm"
    if hi == 0xA or (hi == 0xF and low in (0x1E, 0x29)):
        return "index"
    if hi == 0xF and low in (0x33, 0x55, 0x65):
        return "mem"
    if hi in (0x1, 0x2, 0x3, 0x4, 0x5, 0x9, 0xB) or op == 0x00EE:
        return "branch"
    if hi == 0xF and low in (0x07, 0x15, 0x18):
        return "timer"
    if hi == 0xC:
        return "rnd"
    return "misc"


@dataclasses.dataclass
class EnvSpec:
    """Everything an engine needs to be created, as plain numpy arrays."""

    name: str
    roms: List[bytes]
    env_rom: np.ndarray          # uint16 [E]
    action_keys: np.ndarray      # uint8  [R, 16]
    num_actions: np.ndarray      # uint8  [R]
    score_reg: np.ndarray        # uint8  [R]
    term_reg: np.ndarray         # uint8  [R]
    term_value: np.ndarray       # uint8  [R]
    horizon: np.ndarray          # uint32 [E], 0 = no truncation
    env_seed: np.ndarray         # uint64 [E]
    instr_per_frame: int
    frame_skip: int
    steps: int                   # length of the workload's run
    action_seed: int
    # Environment wrappers (Section 3.2), all off by default: sticky-action
    # probability in units of 2^-24, the no-op-reset maximum, and per ROM a
    # start-up sequence of held keys (one env step each, 16 = no key).
    sticky_q24: int = 0
    noop_max: int = 0
    startup_len: Optional[np.ndarray] = None    # uint8 [R], 0..16
    startup_keys: Optional[np.ndarray] = None   # uint8 [R, 16]

    # Quirk flags (bit 0 = the VIP base profile, bits 1..6 switch single
    # behaviours, see octax.h) and game descriptors per ROM: score mode
    # (0 V[score_reg], 1 BCD difference, 2 negated sum with V[score_arg],
    # 3 capped at score_arg), the op of the termination clause (0 never,
    # 1 ==, 2 >=, 3 !=, 4 either decimal digit ==; None = ==) and a second
    # clause V[term2_reg] term2_op term2_value.
    quirks: int = 1
    score_mode: Optional[np.ndarray] = None     # uint8 [R]
    score_arg: Optional[np.ndarray] = None      # uint8 [R], with score_mode
    term_op: Optional[np.ndarray] = None        # uint8 [R]
    term2_op: Optional[np.ndarray] = None       # uint8 [R]
    term2_reg: Optional[np.ndarray] = None      # uint8 [R]
    term2_value: Optional[np.ndarray] = None    # uint8 [R]

    # Platform: 0 = CHIP-8 (64x32), 1 = SUPER-CHIP (128x64 display, its extra
    # instructions, (4, 128, 64) observations).
    platform: int = 0
    # The opcode mix each generated ROM was drawn with (None for ROMs that
    # were not generated: hand-assembled programs, Target Shooter).
    mixes: Optional[List[OpcodeMix]] = None

    @property
    def has_profile(self) -> bool:
        return bool(self.quirks != 1 or self.score_mode is not None or self.term_op is not None
                    or self.term2_op is not None)

    @property
    def has_wrappers(self) -> bool:
        return bool(self.sticky_q24 or self.noop_max or
                    (self.startup_len is not None and int(np.max(self.startup_len, initial=0)) > 0))

    @property
    def num_envs(self) -> int:
        return int(self.env_rom.shape[0])

    @property
    def num_roms(self) -> int:
        return len(self.roms)

    def actions(self, step0: int, count: int) -> np.ndarray:
        """Actions for steps [step0, step0+count) as int32 [count, E].

        Each env draws uniformly over its ROM's key actions (0..K-1; the
        no-op index K is never drawn).  Step s is generated from its own
        seeded stream so any window can be produced without the ones before.
        """
        k = self.num_actions[self.env_rom].astype(np.int64)
        out = np.empty((count, self.num_envs), dtype=np.int32)
        for i in range(count):
            g = np.random.Generator(np.random.PCG64([self.action_seed, step0 + i]))
            out[i] = (g.integers(0, 1 << 30, size=self.num_envs) % k).astype(np.int32)
        return out

    def subset(self, envs: np.ndarray, name: Optional[str] = None) -> "EnvSpec":
        """The same workload restricted to the listed env indices."""
        envs = np.asarray(envs, dtype=np.int64)
        return dataclasses.replace(
            self, name=name or f"{self.name}[subset {len(envs)}]",
            env_rom=self.env_rom[envs].copy(), horizon=self.horizon[envs].copy(),
            env_seed=self.env_seed[envs].copy())


def with_wrappers(spec: EnvSpec, sticky: float = 0.25, noop_max: int = 30, startup_max: int = 3,
                  seed: int = 0) -> EnvSpec:
    """The spec with the environment wrappers of Section 3.2 switched on.

    Sticky actions with probability ``sticky`` (rounded to a multiple of
    2^-24), no-op reset with up to ``noop_max`` no-op steps, and per ROM a
    start-up sequence of 0..startup_max steps, each holding one of the ROM's
    action keys or none, drawn from ``seed``.
    """
    R = spec.num_roms
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    lens = rng.integers(0, startup_max + 1, size=R).astype(np.uint8)
    akeys = np.asarray(spec.action_keys)
    nact = np.asarray(spec.num_actions).astype(np.int64)
    picks = (rng.random((R, 16)) * (nact[:, None] + 1)).astype(np.int64)   # nact = no key
    keys = np.where(picks < nact[:, None], akeys[np.arange(R)[:, None], np.minimum(picks, 15)], 16)
    return dataclasses.replace(spec, sticky_q24=int(round(sticky * (1 << 24))), noop_max=int(noop_max),
                               startup_len=lens, startup_keys=keys.astype(np.uint8))


def with_profile(spec: EnvSpec, quirks: int = 0x7F, seed: int = 0) -> EnvSpec:
    """The spec with quirk flags and per-ROM game descriptors (Section 3.3).

    ``quirks`` is the flag word (bit 0, the base profile, is always set).
    Per ROM, drawn from ``seed``: a score mode 0..3 with its argument (a
    register for the negated sum, a cap in 64..255 for the capped score); the
    first clause's op (== mostly, else never, either-digit == or !=); and a
    second clause - none, == a random value, >= a value in 0xE0..0xFF, or
    either-digit == - on a random register, so that the clauses end some
    episodes without ending all of them.
    """
    R = spec.num_roms
    rng = np.random.Generator(np.random.PCG64([seed, 13]))
    mode = rng.integers(0, 4, size=R)
    arg = np.where(mode == 2, rng.integers(0, 16, size=R), rng.integers(64, 256, size=R))
    op1 = rng.choice([1, 0, 4, 3], size=R, p=[0.5, 0.15, 0.2, 0.15])
    op2 = rng.choice([0, 1, 2, 4], size=R)
    value = np.where(op2 == 2, rng.integers(0xE0, 0x100, size=R),
                     np.where(op2 == 4, rng.integers(0, 10, size=R), rng.integers(0, 0x100, size=R)))
    u8 = lambda a: np.asarray(a).astype(np.uint8)
    return dataclasses.replace(spec, quirks=int(quirks) | 1, score_mode=u8(mode), score_arg=u8(arg),
                               term_op=u8(op1), term2_op=u8(op2),
                               term2_reg=u8(rng.integers(0, 16, size=R)), term2_value=u8(value))


def _descriptors(n_roms: int, keys: Sequence[Sequence[int]]):
    action_keys = np.zeros((n_roms, 16), dtype=np.uint8)
    num_actions = np.zeros(n_roms, dtype=np.uint8)
    for r_, ks in enumerate(keys):
        action_keys[r_, :len(ks)] = ks
        num_actions[r_] = len(ks)
    score_reg = np.full(n_roms, 5, dtype=np.uint8)     # reward = delta of V5
    term_reg = np.full(n_roms, 6, dtype=np.uint8)      # done when V6 == 0xFF
    term_value = np.full(n_roms, 0xFF, dtype=np.uint8)
    return action_keys, num_actions, score_reg, term_reg, term_value


def geometric_horizons(rng: np.random.Generator, n: int, mean: float) -> np.ndarray:
    return rng.geometric(1.0 / mean, size=n).astype(np.uint32)


def make_config(name: str, num_envs: Optional[int] = None, steps: Optional[int] = None) -> EnvSpec:
    """Named workloads.

    ``c1``  16 envs, one 256-instruction ROM, 5 keys, ipf 10, horizon 1000.
    ``c2``  4,096 envs, one 1,024-instruction ROM, 8 keys, ipf 10, horizon 1000.
    ``c3``  65,536 envs over 16 ROMs of 256..1792 instructions with varying
            draw and branch shares, geometric horizons (mean 500), ipf 10.
    ``c4``  the 32-ROM pool used by the serving loop (groups are drawn by the
            serving module); here E is a placeholder of one env per ROM.
    ``c5``  1,048,576 envs over 64 draw-heavy ROMs (40% DXYN, N up to 15,
            edge-biased coordinates), ipf 20, geometric horizons.
    ``s1``  SUPER-CHIP: 65,536 envs over 8 programs of 256..1792 instructions
            with 12% SUPER-CHIP instructions (gen_schip_rom), 8 keys, ipf 10,
            geometric horizons (mean 500), (4, 128, 64) observations.
    ``ts``  65,536 envs over the three Target Shooter levels (written in Octo
            for this repository, see programs/), a third of the envs each in
            random order, keys 5 7 8 9 6, score V2, done when V3 == 1, ipf 10,
            geometric horizons (mean 500).
    ``escape``  the ``c3`` shape with unstructured programs (gen_rom_escape)
            that leave their own code: wrap-around, page-crossing and
            self-modifying paths.
    ``num_envs`` and ``steps`` override the sizes (for tests at small scale).
    """
    label = name.lower()
    name = "c3" if label == "escape" else label
    generate = gen_rom_escape if label == "escape" else gen_rom
    if name == "c1":
        seed, E, R, L, keys, ipf, steps_ = 0, 16, 1, (256,), KEYS_5, 10, 1000
    elif name == "c2":
        seed, E, R, L, keys, ipf, steps_ = 1, 4096, 1, (1024,), KEYS_8, 10, 10000
    elif name == "c3":
        seed, E, R, L, keys, ipf, steps_ = 2, 65536, 16, None, KEYS_8, 10, 64
    elif name == "c4":
        seed, E, R, L, keys, ipf, steps_ = 3, 32, 32, None, KEYS_8, 10, 200
    elif name == "c5":
        seed, E, R, L, keys, ipf, steps_ = 4, 1 << 20, 64, None, KEYS_8, 20, 1000
    elif name == "ts":
        seed, E, R, L, keys, ipf, steps_ = 5, 65536, 3, None, KEYS_5, 10, 64
    elif name == "s1":
        seed, E, R, L, keys, ipf, steps_ = 6, 65536, 8, None, KEYS_8, 10, 16
    else:
        raise KeyError(name)
    if num_envs is not None:
        E = int(num_envs)
    if steps is not None:
        steps_ = int(steps)
    rng = np.random.Generator(np.random.PCG64(seed))
    roms: List[bytes] = []
    mixes: Optional[List[OpcodeMix]] = []
    for r_ in range(R):
        if name == "ts":
            roms, mixes = target_shooter_roms(), None
            break
        if L is not None:
            n, mix = L[r_], OpcodeMix()
        elif name == "c5":
            n = int(rng.integers(256, MAX_PROGRAM_INSTRUCTIONS + 1))
            mix = OpcodeMix(draw=0.40, key=0.06, alu=0.15, imm=0.12, index=0.10, mem=0.04,
                            branch=0.08, timer=0.03, rnd=0.02, draw_n_max=15, edge_bias=True)
        else:
            n = int(rng.integers(256, MAX_PROGRAM_INSTRUCTIONS + 1))
            draw = float(rng.uniform(0.05, 0.40))
            branch = float(rng.uniform(0.10, 0.30))
            rest = 1.0 - draw - branch
            base = OpcodeMix()
            others = np.array([base.key, base.alu, base.imm, base.index, base.mem,
                               base.timer, base.rnd, base.misc])
            others = others / others.sum() * rest
            mix = OpcodeMix(draw, *others[:5], branch, *others[5:])
        mixes.append(mix)
        if name == "s1":
            roms.append(gen_schip_rom(seed * 1000 + r_, n, mix, keys))
        else:
            roms.append(generate(seed * 1000 + r_, n, mix, keys))
    if R == 1:
        env_rom = np.zeros(E, dtype=np.uint16)
    else:
        # Every ROM gets E/R envs (rounded), in a random order so ROMs mix
        # within every wavefront of consecutive envs.
        env_rom = (np.arange(E) % R).astype(np.uint16)
        env_rom = env_rom[rng.permutation(E)]
    akeys, nact, sreg, treg, tval = _descriptors(R, [keys] * R)
    if name == "ts":   # score V2, game over when V3 == 1 (the Target Shooter wrapper)
        sreg[:], treg[:], tval[:] = 2, 3, 1
    if name in ("c1", "c2"):
        horizon = np.full(E, 1000, dtype=np.uint32)
    else:
        horizon = geometric_horizons(rng, E, 500.0)
    env_seed = rng.integers(0, np.iinfo(np.uint64).max, size=E, dtype=np.uint64, endpoint=True)
    return EnvSpec(name=label, roms=roms, env_rom=env_rom, action_keys=akeys, num_actions=nact,
                   score_reg=sreg, term_reg=treg, term_value=tval, horizon=horizon,
                   env_seed=env_seed, instr_per_frame=ipf, frame_skip=4, steps=steps_,
                   action_seed=seed + 7919, platform=1 if name == "s1" else 0, mixes=mixes)


PROGRAMS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "programs")


def target_shooter_roms() -> List[bytes]:
    """The three Target Shooter levels, assembled from their Octo sources."""
    from . import octo
    out = []
    for level in (1, 2, 3):
        with open(os.path.join(PROGRAMS, f"target_shooter_l{level}.8o")) as f:
            out.append(octo.assemble(f.read()))
    return out


def custom_spec(roms: Sequence[bytes], num_envs: int = 1, *, keys: Sequence[int] = KEYS_5,
                instr_per_frame: int = 10, frame_skip: int = 4, horizon: int = 0,
                seed: int = 0, env_rom: Optional[np.ndarray] = None,
                score_reg: int = 5, term_reg: int = 6, term_value: int = 0xFF,
                name: str = "custom") -> EnvSpec:
    """A spec around explicit ROM bytes (hand-assembled test programs)."""
    R = len(roms)
    if env_rom is None:
        env_rom = (np.arange(num_envs) % R).astype(np.uint16)
    akeys, nact, sreg, treg, tval = _descriptors(R, [keys] * R)
    sreg[:] = score_reg
    treg[:] = term_reg
    tval[:] = term_value
    rng = np.random.Generator(np.random.PCG64(seed))
    return EnvSpec(name=name, roms=list(roms), env_rom=np.asarray(env_rom, dtype=np.uint16),
                   action_keys=akeys, num_actions=nact, score_reg=sreg, term_reg=treg,
                   term_value=tval, horizon=np.full(num_envs, horizon, dtype=np.uint32),
                   env_seed=rng.integers(0, np.iinfo(np.uint64).max, size=num_envs,
                                         dtype=np.uint64, endpoint=True),
                   instr_per_frame=instr_per_frame, frame_skip=frame_skip, steps=0,
                   action_seed=seed + 7919)


def assemble(words: Sequence[int]) -> bytes:
    """Big-endian bytes of a list of 16-bit opcodes (hand-assembled programs)."""
    out = bytearray()
    for wd in words:
        if not 0 <= wd <= 0xFFFF:
            raise ValueError(hex(wd))
        out += bytes(_enc(wd))
    return bytes(out)


@dataclasses.dataclass
class Group:
    """One serving request: a group of envs of one ROM run for ``steps`` steps."""

    gid: int
    arrival: float
    rom: int
    size: int
    steps: int
    seed: int


def serving_groups(n_groups: int, rate: float, seed: int = 3, n_roms: int = 32,
                   max_size: int = 4096, min_steps: int = 200, max_steps: int = 2000) -> List[Group]:
    """Poisson arrivals (``rate`` groups/s) of groups with log-uniform sizes in 1..max_size."""
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    t = 0.0
    out = []
    for g in range(n_groups):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        size = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_size + 1)))))
        size = max(1, min(max_size, size))
        steps = int(rng.integers(min_steps, max_steps + 1))
        out.append(Group(gid=g, arrival=t, rom=int(rng.integers(0, n_roms)), size=size,
                         steps=steps, seed=int(rng.integers(0, 1 << 62))))
    return out


def group_env_seeds(group: Group) -> np.ndarray:
    """Per-env RNG seeds of a serving group: a function of the group only, never of its slots."""
    g = np.random.Generator(np.random.PCG64([group.seed, 2]))
    return g.integers(0, np.iinfo(np.uint64).max, size=group.size, dtype=np.uint64, endpoint=True)


ACTION_CHUNK = 64


def action_stream(group: Group) -> np.random.PCG64:
    """The random stream of a serving group's actions: PCG64 seeded [seed, 3]."""
    return np.random.PCG64([group.seed, 3])


def group_action_words(group: Group, c: int, stream: Optional[np.random.PCG64] = None) -> np.ndarray:
    """The random words of a serving group's action chunk c (steps
    [c * ACTION_CHUNK, (c + 1) * ACTION_CHUNK)) as uint16 [ACTION_CHUNK, size]:
    64-bit outputs c * n .. (c + 1) * n - 1 of its action stream
    (n = ACTION_CHUNK * size / 4), in step-major order.  `stream`, if given,
    must stand at output c * n (a stream drawn chunk after chunk does)."""
    n = ACTION_CHUNK * group.size // 4
    if stream is None:
        stream = action_stream(group)
        stream.advance(c * n)
    return stream.random_raw(n).view(np.uint16).reshape(ACTION_CHUNK, group.size)


def actions_from_words(u: np.ndarray, num_actions: int) -> np.ndarray:
    """(u * num_actions) >> 16 as int32: uniform over the ROM's key actions up
    to a bias below num_actions / 2^16."""
    t = np.multiply(u, num_actions, dtype=np.int32)
    t >>= 16
    return t


def group_actions(group: Group, step0: int, count: int, num_actions: int) -> np.ndarray:
    """Actions of a serving group for steps [step0, step0+count) as int32 [count, size],
    drawn a chunk of ``ACTION_CHUNK`` steps at a time from one stream per chunk
    (group_action_words, actions_from_words), so any window is cheap to produce."""
    out = np.empty((count, group.size), dtype=np.int32)
    s = step0
    while s < step0 + count:
        c = s // ACTION_CHUNK
        lo, hi = s - c * ACTION_CHUNK, min(step0 + count - c * ACTION_CHUNK, ACTION_CHUNK)
        out[s - step0:s - step0 + hi - lo] = actions_from_words(group_action_words(group, c)[lo:hi], num_actions)
        s += hi - lo
    return out


def group_horizons(group: Group, mean: float = 500.0) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64([group.seed, 4]))
    return geometric_horizons(g, group.size, mean)


def mix_summary(rom: bytes, code_slots: Optional[int] = None) -> Dict[str, float]:
    """Fraction of each generator class among the ROM's first ``code_slots``
    instructions (all of them when None)."""
    n = len(rom) // 2 if code_slots is None else code_slots
    ops = [(rom[2 * i] << 8) | rom[2 * i + 1] for i in range(n)]
    counts = {c: 0 for c in CLASS_NAMES}
    for op in ops:
        counts[opcode_class(op)] += 1
    return {c: v / len(ops) for c, v in counts.items()}
