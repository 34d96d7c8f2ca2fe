"""A small assembler for a subset of Octo, the CHIP-8 assembly language the
paper's generated games are written in (Appendix F: the generation pipeline
prompts with the Octo manual and emits Octo programs).

It turns Octo source into ROM bytes loaded at 0x200.  It is input
preparation, like the seeded program generator in workload.py: it holds none
of the emulator's arithmetic.

Supported (the statements of the Octo manual that map to one CHIP-8
instruction, plus its structured control flow):
  comments            # to the end of the line
  labels              : name          (a bare name as a statement calls it)
  directives          :const name value   :alias name vX   :call name   :byte value
  data                a number as a statement emits one byte
  returns             ;   return
  screen              clear           sprite vX vY N
  jumps               jump target     jump0 target
  registers           vX := vY | NN | random NN | delay | key
                      vX += vY | NN   vX -= vY | NN   vX =- vY
                      vX |= vY   vX &= vY   vX ^= vY   vX >>= vY   vX <<= vY
  index               i := NNN | label | hex vX   i += vX
                      bcd vX   save vX   load vX
  timers              delay := vX     buzzer := vX
  conditions          vX == vY|NN  vX != vY|NN  vX < > <= >= vY|NN
                      vX key   vX -key
  control flow        if COND then STATEMENT
                      if COND begin ... [else ...] end
                      loop ... [while COND] ... again
Ordered comparisons are compiled through VF, as in Octo: `vX < vY` becomes
vF := vX; vF -= vY and a test of the borrow flag vF == 0, so they clobber VF.
The statement after `then` must be a single instruction.

Numbers are decimal, 0x hex or 0b binary, or a :const name; label and
constant names may be used before their definition.
"""
from __future__ import annotations

import re
from typing import Dict, List, Optional, Tuple

ORIGIN = 0x200


class OctoError(ValueError):
    pass


_REG = re.compile(r"^v([0-9a-fA-F])$")
_ORDERED = ("<", ">", "<=", ">=")


def _tokens(src: str) -> List[Tuple[str, int]]:
    out = []
    for ln, line in enumerate(src.splitlines(), 1):
        line = line.split("#", 1)[0]
        out += [(t, ln) for t in line.split()]
    return out


class _Asm:
    def __init__(self, src: str):
        self.toks = _tokens(src)
        self.pos = 0
        self.code = bytearray()
        self.labels: Dict[str, int] = {}
        self.consts: Dict[str, int] = {}
        self.aliases: Dict[str, int] = {}
        self.fixups: List[Tuple[int, str, int, int]] = []   # (offset, name, opcode high nibble, line)
        self.blocks: List[dict] = []

    # -- token helpers -------------------------------------------------
    def line(self) -> int:
        p = min(self.pos, len(self.toks) - 1)
        return self.toks[p][1] if self.toks else 0

    def next(self) -> str:
        if self.pos >= len(self.toks):
            raise OctoError("unexpected end of program")
        t = self.toks[self.pos][0]
        self.pos += 1
        return t

    def expect(self, word: str):
        t = self.next()
        if t != word:
            raise OctoError(f"line {self.line()}: expected '{word}', got '{t}'")

    def reg(self, t: Optional[str] = None) -> int:
        t = self.next() if t is None else t
        if t in self.aliases:
            return self.aliases[t]
        m = _REG.match(t)
        if not m:
            raise OctoError(f"line {self.line()}: '{t}' is not a register")
        return int(m.group(1), 16)

    def is_reg(self, t: Optional[str]) -> bool:
        return t is not None and (t in self.aliases or _REG.match(t) is not None)

    def number(self, t: Optional[str] = None, bits: int = 8) -> int:
        t = self.next() if t is None else t
        if t in self.consts:
            v = self.consts[t]
        else:
            try:
                v = int(t, 0)
            except ValueError:
                raise OctoError(f"line {self.line()}: '{t}' is not a number") from None
        lo = -(1 << (bits - 1)) if bits == 8 else 0
        if not lo <= v < (1 << bits):
            raise OctoError(f"line {self.line()}: {v} does not fit in {bits} bits")
        return v & ((1 << bits) - 1)

    def is_number(self, t: Optional[str]) -> bool:
        if t is None:
            return False
        if t in self.consts:
            return True
        try:
            int(t, 0)
            return True
        except ValueError:
            return False

    # -- emission ------------------------------------------------------
    def here(self) -> int:
        return ORIGIN + len(self.code)

    def emit(self, op: int):
        self.code += bytes([(op >> 8) & 0xFF, op & 0xFF])

    def emit_addr(self, high: int, target: str):
        """Emit high-nibble opcode with a 12-bit address (label resolved later)."""
        if self.is_number(target) and target not in self.labels:
            self.emit((high << 12) | self.number(target, bits=12))
        else:
            self.fixups.append((len(self.code), target, high, self.line()))
            self.emit(high << 12)

    # -- conditions ----------------------------------------------------
    def condition(self) -> Tuple[List[int], Tuple[int, int]]:
        """Parse a condition; return (setup instructions, (skip-if-true, skip-if-false) opcodes)."""
        x = self.reg()
        op = self.next()
        if op in ("key", "-key"):
            pressed_skip, released_skip = 0xE09E | (x << 8), 0xE0A1 | (x << 8)
            return ([], (pressed_skip, released_skip) if op == "key" else (released_skip, pressed_skip))
        rhs = self.next()
        if op in ("==", "!="):
            if self.is_reg(rhs):
                y = self.reg(rhs)
                eq, ne = 0x5000 | (x << 8) | (y << 4), 0x9000 | (x << 8) | (y << 4)
            else:
                nn = self.number(rhs)
                eq, ne = 0x3000 | (x << 8) | nn, 0x4000 | (x << 8) | nn
            return ([], (eq, ne) if op == "==" else (ne, eq))
        if op in _ORDERED:
            # borrow flag of a subtraction left in VF: 1 when there is no borrow
            if self.is_reg(rhs):
                y = self.reg(rhs)
                a, b = (x, y) if op in ("<", ">=") else (y, x)     # test a < b (flag 0) or a >= b (flag 1)
                setup = [0x8F00 | (a << 4), 0x8F05 | (b << 4)]      # vF := va ; vF -= vb
            else:
                nn = self.number(rhs)
                if op in ("<", ">="):                              # x < nn : vF := nn ; vF =- vx -> flag = x >= nn
                    setup = [0x6F00 | nn, 0x8F07 | (x << 4)]
                else:                                              # x > nn : vF := nn ; vF -= vx -> flag = nn >= x
                    setup = [0x6F00 | nn, 0x8F05 | (x << 4)]
            flag_zero, flag_one = 0x3F00, 0x3F01                   # skip if vF == 0 / vF == 1
            true_when_zero = op in ("<", ">")
            return (setup, (flag_zero, flag_one) if true_when_zero else (flag_one, flag_zero))
        raise OctoError(f"line {self.line()}: unknown comparison '{op}'")

    # -- statements ----------------------------------------------------
    def statement(self):
        t = self.next()
        if t == ":":
            name = self.next()
            if name in self.labels:
                raise OctoError(f"line {self.line()}: label '{name}' defined twice")
            self.labels[name] = self.here()
        elif t == ":const":
            name = self.next()
            self.consts[name] = self.number(self.next(), bits=12)
        elif t == ":alias":
            name = self.next()
            self.aliases[name] = self.reg()
        elif t == ":call":
            self.emit_addr(0x2, self.next())
        elif t == ":byte":
            self.code.append(self.number())
        elif t in (";", "return"):
            self.emit(0x00EE)
        elif t == "clear":
            self.emit(0x00E0)
        elif t == "jump":
            self.emit_addr(0x1, self.next())
        elif t == "jump0":
            self.emit_addr(0xB, self.next())
        elif t == "sprite":
            x, y = self.reg(), self.reg()
            n = self.number(bits=4)
            self.emit(0xD000 | (x << 8) | (y << 4) | n)
        elif t == "i":
            self.index_statement()
        elif t in ("bcd", "save", "load"):
            x = self.reg()
            self.emit(0xF000 | (x << 8) | {"bcd": 0x33, "save": 0x55, "load": 0x65}[t])
        elif t in ("delay", "buzzer"):
            self.expect(":=")
            x = self.reg()
            self.emit(0xF000 | (x << 8) | (0x15 if t == "delay" else 0x18))
        elif t == "if":
            self.if_statement()
        elif t == "loop":
            self.blocks.append({"kind": "loop", "start": self.here(), "exits": []})
        elif t == "while":
            blk = self.innermost("loop", "while")
            setup, (skip_true, _) = self.condition()
            for op in setup:
                self.emit(op)
            self.emit(skip_true)                   # condition holds: skip the exit jump
            blk["exits"].append(len(self.code))
            self.emit(0x1000)
        elif t == "again":
            blk = self.blocks.pop() if self.blocks and self.blocks[-1]["kind"] == "loop" else None
            if blk is None:
                raise OctoError(f"line {self.line()}: 'again' without 'loop'")
            self.emit(0x1000 | blk["start"])
            for off in blk["exits"]:
                self.patch(off, 0x1000 | self.here())
        elif t == "else":
            blk = self.innermost("if", "else")
            jump_end = len(self.code)
            self.emit(0x1000)
            self.patch(blk["skip_jump"], 0x1000 | self.here())
            blk["skip_jump"] = jump_end
        elif t == "end":
            if not self.blocks or self.blocks[-1]["kind"] != "if":
                raise OctoError(f"line {self.line()}: 'end' without 'begin'")
            blk = self.blocks.pop()
            self.patch(blk["skip_jump"], 0x1000 | self.here())
        elif self.is_reg(t):
            self.register_statement(self.reg(t))
        elif self.is_number(t) and t not in self.labels:
            self.code.append(self.number(t))
        elif re.match(r"^[A-Za-z_][A-Za-z0-9_\-]*$", t):
            self.emit_addr(0x2, t)                 # a bare name calls a subroutine
        else:
            raise OctoError(f"line {self.line()}: cannot assemble '{t}'")

    def innermost(self, kind: str, word: str) -> dict:
        for blk in reversed(self.blocks):
            if blk["kind"] == kind:
                return blk
        raise OctoError(f"line {self.line()}: '{word}' outside a {kind} block")

    def patch(self, off: int, op: int):
        self.code[off] = (op >> 8) & 0xFF
        self.code[off + 1] = op & 0xFF

    def index_statement(self):
        op = self.next()
        if op == "+=":
            self.emit(0xF01E | (self.reg() << 8))
        elif op == ":=":
            t = self.next()
            if t == "hex":
                self.emit(0xF029 | (self.reg() << 8))
            else:
                self.emit_addr(0xA, t)
        else:
            raise OctoError(f"line {self.line()}: unknown index statement 'i {op}'")

    def register_statement(self, x: int):
        op = self.next()
        t = self.next()
        if op == ":=":
            if t == "random":
                self.emit(0xC000 | (x << 8) | self.number())
            elif t == "delay":
                self.emit(0xF007 | (x << 8))
            elif t == "key":
                self.emit(0xF00A | (x << 8))
            elif self.is_reg(t):
                self.emit(0x8000 | (x << 8) | (self.reg(t) << 4))
            else:
                self.emit(0x6000 | (x << 8) | self.number(t))
            return
        alu = {"|=": 1, "&=": 2, "^=": 3, "+=": 4, "-=": 5, ">>=": 6, "=-": 7, "<<=": 0xE}
        if op not in alu:
            raise OctoError(f"line {self.line()}: unknown operator '{op}'")
        if self.is_reg(t):
            self.emit(0x8000 | (x << 8) | (self.reg(t) << 4) | alu[op])
        elif op == "+=":
            self.emit(0x7000 | (x << 8) | self.number(t))
        elif op == "-=":
            self.emit(0x7000 | (x << 8) | ((-self.number(t)) & 0xFF))
        else:
            raise OctoError(f"line {self.line()}: '{op}' needs a register operand")

    def if_statement(self):
        setup, (skip_true, skip_false) = self.condition()
        for op in setup:
            self.emit(op)
        word = self.next()
        if word == "then":
            self.emit(skip_false)                  # condition fails: skip the statement
            start = len(self.code)
            self.statement()
            if len(self.code) - start != 2:
                raise OctoError(f"line {self.line()}: the statement after 'then' must be one instruction")
        elif word == "begin":
            self.emit(skip_true)                   # condition holds: skip the jump past the block
            blk = {"kind": "if", "skip_jump": len(self.code)}
            self.emit(0x1000)
            self.blocks.append(blk)
        else:
            raise OctoError(f"line {self.line()}: expected 'then' or 'begin' after the condition")

    def run(self) -> bytes:
        while self.pos < len(self.toks):
            self.statement()
        if self.blocks:
            raise OctoError(f"unclosed '{self.blocks[-1]['kind']}' block")
        for off, name, high, ln in self.fixups:
            if name in self.labels:
                addr = self.labels[name]
            elif name in self.consts:
                addr = self.consts[name]
            else:
                raise OctoError(f"line {ln}: unknown name '{name}'")
            self.patch(off, (high << 12) | (addr & 0xFFF))
        if len(self.code) > 0x1000 - ORIGIN:
            raise OctoError("program longer than 3,584 bytes")
        return bytes(self.code)


def assemble(src: str) -> bytes:
    """ROM bytes (loaded at 0x200) of an Octo-subset program."""
    return _Asm(src).run()


def labels(src: str) -> Dict[str, int]:
    """Addresses of the program's labels (for tests and debugging)."""
    a = _Asm(src)
    a.run()
    return dict(a.labels)
