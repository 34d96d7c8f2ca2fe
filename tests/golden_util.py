"""Parsers for the hand-written fixtures under tests/golden/."""
import configparser
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ini(name):
    cp = configparser.ConfigParser(inline_comment_prefixes=None, interpolation=None)
    cp.optionxform = str
    cp.read(os.path.join(GOLDEN, name))
    return cp


def program_bytes(sec) -> bytes:
    words = [int(w, 16) for w in sec.get("program", "").split()]
    rom = bytearray()
    for w in words:
        rom += bytes([w >> 8, w & 0xFF])
    data = sec.get("data", "").strip()
    if data:
        addr_s, bytes_s = data.split(":")
        addr = int(addr_s, 16) - 0x200
        vals = [int(b, 16) for b in bytes_s.split()]
        if len(rom) < addr + len(vals):
            rom += bytes(addr + len(vals) - len(rom))
        rom[addr:addr + len(vals)] = bytes(vals)
    return bytes(rom)


def parse_assignments(text):
    out = {}
    for tok in text.split():
        k, v = tok.split("=")
        out[k] = int(v, 16)
    return out


def parse_pixels(text):
    text = text.strip()
    if text == "none":
        return set()
    return {tuple(int(c) for c in p.split(",")) for p in text.split()}


def machine_programs():
    cp = _ini("programs.ini")
    return [(name, cp[name]) for name in cp.sections()]


def env_programs():
    cp = _ini("env_programs.ini")
    return [(name, cp[name]) for name in cp.sections()]


def expand(text, conv=int):
    out = []
    for tok in text.split():
        if "*" in tok:
            v, n = tok.split("*")
            out += [conv(v)] * int(n)
        else:
            out.append(conv(tok))
    return out


def font_glyphs():
    """{digit: [5 row bytes]} from the pictures in font_glyphs.txt."""
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "font_glyphs.txt"))
             if ln.strip() and not ln.startswith("# ") and ln.strip() != "#"]
    glyphs = {}
    i = 0
    while i < len(lines):
        d = int(lines[i], 16)
        rows = []
        for r in range(5):
            pic = lines[i + 1 + r]
            assert len(pic) == 4
            b = 0
            for c, ch in enumerate(pic):
                if ch == "#":
                    b |= 0x80 >> c
            rows.append(b)
        glyphs[d] = rows
        i += 6
    assert sorted(glyphs) == list(range(16))
    return glyphs


def splitmix_vectors():
    out = {}
    for ln in open(os.path.join(GOLDEN, "splitmix64.txt")):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        seed, vals = ln.split(":")
        out[int(seed)] = [int(v) for v in vals.split()]
    return out


def lit_pixels(disp_yx: np.ndarray):
    ys, xs = np.nonzero(disp_yx)
    return {(int(x), int(y)) for x, y in zip(xs, ys)}


def big_font_pictures() -> np.ndarray:
    """[16][10][8] pixel pictures of the SUPER-CHIP digit glyphs."""
    out = np.zeros((16, 10, 8), dtype=np.uint8)
    glyph, row = -1, 0
    for line in open(os.path.join(GOLDEN, "big_font_glyphs.txt")):
        line = line.strip()
        if not line or line.startswith("#") and not set(line) <= {"#", "."}:
            continue
        if len(line) == 1:
            glyph, row = int(line, 16), 0
            continue
        out[glyph, row] = [c == "#" for c in line]
        row += 1
    return out
