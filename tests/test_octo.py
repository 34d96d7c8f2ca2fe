"""Pins of the Octo-subset assembler (workload input preparation).

Encodings are checked against hand-encoded statements (tests/golden); the
structured control flow and the ordered comparisons, which expand into
several instructions, are checked by running the assembled code on the
oracle's machine (itself pinned by the instruction tests) and comparing the
outcome with what the statement means.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import octo
from tests.golden_util import GOLDEN


def _golden():
    rows = []
    for line in open(f"{GOLDEN}/octo_statements.txt"):
        if line.startswith("#") or "|" not in line:
            continue
        stmt, want = line.rsplit("|", 1)
        rows.append((stmt.strip(), bytes.fromhex(want.replace(" ", ""))))
    return rows


@pytest.mark.parametrize("stmt,want", _golden())
def test_statement_encodings(stmt, want):
    assert octo.assemble(stmt) == want, stmt


def _run(src, n, v=None, key=-1):
    m = O.Machine(octo.assemble(src))
    if v is not None:
        s = m.state()
        s["v"] = v
        m.set_state(s)
    m.execute(n, key)
    return m.state()


def test_loop_while_sums():
    src = """
      v0 := 0  v1 := 10
      loop
        v0 += v1
        v1 -= 1
        while v1 != 0
      again
      v2 := 1
      : halt jump halt
    """
    s = _run(src, 200)
    assert s["v"][0] == 55 and s["v"][1] == 0 and s["v"][2] == 1


def test_if_begin_else_end():
    src = """
      if v0 == 2 begin
        v1 := 7
        v2 := 1
      else
        v1 := 9
      end
      v3 := 5
      : halt jump halt
    """
    for v0 in range(4):
        v = np.zeros(16, np.uint8)
        v[0] = v0
        s = _run(src, 20, v)
        assert s["v"][1] == (7 if v0 == 2 else 9) and s["v"][2] == (1 if v0 == 2 else 0) and s["v"][3] == 5


def test_nested_blocks_and_calls():
    src = """
      : main
        v5 := 0
        loop
          v5 += 1
          if v5 == 3 begin
            bump
          end
          while v5 != 6
        again
        : halt jump halt
      : bump
        v6 += 10
        loop v7 += 1 while v7 != 4 again
      ;
    """
    s = _run(src, 400)
    assert s["v"][5] == 6 and s["v"][6] == 10 and s["v"][7] == 4 and s["sp"] == 0


@pytest.mark.parametrize("op", ["<", ">", "<=", ">=", "==", "!="])
@pytest.mark.parametrize("rhs", ["reg", "const"])
def test_comparisons_match_their_meaning(op, rhs):
    vals = np.unique(np.concatenate([[0, 1, 2, 9, 10, 127, 128, 200, 254, 255],
                                     np.random.default_rng(3).integers(0, 256, 22)]))
    py = {"<": np.less, ">": np.greater, "<=": np.less_equal, ">=": np.greater_equal,
          "==": np.equal, "!=": np.not_equal}[op]
    for k in ([9, 128, 255] if rhs == "const" else [None]):
        src = f"if v3 {op} {'v5' if k is None else k} then v4 := 1\n: halt jump halt"
        rom = octo.assemble(src)
        a, b = np.meshgrid(vals, vals, indexing="ij")
        a, b = a.ravel(), b.ravel()
        base = O.blank_state(rom)
        states = np.repeat(base[None], len(a), axis=0)
        states["v"][:, 3] = a
        states["v"][:, 5] = b
        out = O.execute_states(states, n_instr=6)
        want = py(a, b if k is None else k)
        assert np.array_equal(out["v"][:, 4] == 1, want), (op, k)
        assert np.array_equal(out["v"][:, 3], a) and np.array_equal(out["v"][:, 5], b)


def test_key_conditions():
    src = "if v3 key then v4 := 1\nif v3 -key then v6 := 1\n: halt jump halt"
    v = np.zeros(16, np.uint8)
    v[3] = 0xA
    s = _run(src, 6, v, key=0xA)
    assert s["v"][4] == 1 and s["v"][6] == 0
    s = _run(src, 6, v, key=0xB)
    assert s["v"][4] == 0 and s["v"][6] == 1
    s = _run(src, 6, v, key=-1)
    assert s["v"][4] == 0 and s["v"][6] == 1


def test_labels_resolve_forward_and_backward():
    src = """
      jump later
      : back v1 := 2 jump done
      : later v0 := 1 jump back
      : done i := data
      : halt jump halt
      : data 0x11 0x22
    """
    labs = octo.labels(src)
    s = _run(src, 20)
    assert s["v"][0] == 1 and s["v"][1] == 2 and s["i"] == labs["data"]
    rom = octo.assemble(src)
    assert rom[labs["data"] - 0x200:] == bytes([0x11, 0x22])


@pytest.mark.parametrize("bad", [
    "jump nowhere",                          # unknown name
    "if v0 == 1 then if v1 == 2 then v2 := 1",   # more than one instruction after then
    "loop v0 += 1",                          # unclosed loop
    "again",
    "end",
    "else",
    "v0 := 256",
    "sprite v0 v1 16",
    "i := 0x1000",
    ": a : a",
    "v0 ** v1",
    "while v0 == 1",
])
def test_errors(bad):
    with pytest.raises(octo.OctoError):
        octo.assemble(bad)
