"""What the seeded workloads actually execute, measured on the oracle.

The generated programs stand in for game code, so they must run their own
code with the opcode mix their config describes, not fall out of it.  Each
ROM of every generated workload runs on the oracle for 1,000 frames (250
steps, two envs per ROM, the config's own actions) with an execution profile
attached; the tests check the share of instructions fetched inside the ROM's
bytes and the class histogram of the executed words against the weights the
ROM was drawn with.  The escape workload is the opposite case, kept for the
wrap-around paths: its programs leave themselves.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_01764_amd import workload as W

FRAMES = 1000
CLASS_OF = np.array([W.CLASS_NAMES.index(W.opcode_class(op)) for op in range(65536)])


def _profile(name, envs_per_rom=2):
    spec = W.make_config(name, num_envs=1)
    R = spec.num_roms
    spec = W.make_config(name, num_envs=R * envs_per_rom)
    spec.env_rom[:] = np.arange(spec.num_envs) % R     # every ROM runs
    b = O.OracleBatch(spec)
    pc, op = b.profile_execution()
    steps = FRAMES // spec.frame_skip
    acts = spec.actions(0, steps)
    for t in range(steps):
        b.step(acts[t], want_obs=False)
    b.close()
    out = []
    for r in range(R):
        total = float(pc[r].sum())
        inside = float(pc[r, W.PROGRAM_START:W.PROGRAM_START + len(spec.roms[r])].sum()) / total
        hist = np.bincount(CLASS_OF, weights=op[r].astype(np.float64), minlength=len(W.CLASS_NAMES)) / total
        out.append((inside, hist, total))
    return spec, out


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_programs_run_their_code_with_the_configured_mix(name):
    spec, rows = _profile(name)
    for r, ((inside, hist, total), mix) in enumerate(zip(rows, spec.mixes)):
        assert total >= 2 * FRAMES * spec.instr_per_frame
        assert inside >= 0.95, (name, r, inside)
        # per ROM: a 256-instruction program runs only part of its code in 1,000 frames
        w = mix.weights()
        tol = 0.03 + 0.2 * w
        bad = [(c, round(h, 3), round(x, 3)) for c, h, x, t in zip(W.CLASS_NAMES, hist, w, tol)
               if abs(h - x) > t]
        assert not bad, (name, r, bad)
    # over a workload of many ROMs, weighted by what they ran, the mix is tighter
    if len(rows) < 8:
        return
    runs = np.array([t for _, _, t in rows])
    got = sum(h * t for (_, h, t) in rows) / runs.sum()
    want = sum(m.weights() * t for m, t in zip(spec.mixes, runs)) / runs.sum()
    assert (np.abs(got - want) <= 0.01 + 0.1 * want).all(), (name, np.round(got, 3), np.round(want, 3))


def test_mixed_rom_draw_share_spans_the_configured_range():
    """The mixed-ROM workload's ROMs draw 5-40 % DXYN; what they execute spans that range."""
    _, rows = _profile("c3")
    draw = np.array([h[W.CLASS_NAMES.index("draw")] for _, h, _ in rows])
    assert draw.min() < 0.12 and draw.max() > 0.33, draw
    assert (draw > 0.04).all() and (draw < 0.45).all(), draw


def test_draw_heavy_rom_draw_share():
    _, rows = _profile("c5", envs_per_rom=1)
    draw = np.array([h[W.CLASS_NAMES.index("draw")] for _, h, _ in rows])
    assert (np.abs(draw - 0.40) < 0.08).all() and abs(draw.mean() - 0.40) < 0.03, draw


def test_super_chip_programs_stay_in_their_code():
    _, rows = _profile("s1")
    for r, (inside, _, _) in enumerate(rows):
        assert inside >= 0.95, (r, inside)


def test_escape_workload_leaves_its_programs():
    """The unstructured generator is the escape case: most of its ROMs run outside their bytes."""
    _, rows = _profile("escape", envs_per_rom=1)
    inside = np.array([x for x, _, _ in rows])
    assert (inside < 0.5).sum() >= len(inside) // 2, inside


def test_structure_of_generated_programs():
    """Static checks of the control-flow rules: targets, region ends, store pointers."""
    for seed, n in ((5, 256), (6, 1792), (7, 300)):
        prog = W.gen_program(seed, n)
        rom = prog.rom
        code = prog.code_slots
        words = [(rom[2 * k] << 8) | rom[2 * k + 1] for k in range(code)]
        end = W.PROGRAM_START + 2 * code
        returns = [k for k, wd in enumerate(words) if wd == 0x00EE]
        call_targets = {wd & 0xFFF for wd in words if wd >> 12 == 2}
        # every call lands on a subroutine start: the word after a region's end
        starts = {W.PROGRAM_START + 2 * (k + 1) for k, wd in enumerate(words)
                  if wd == 0x00EE or wd == 0x1200}
        assert call_targets <= starts, (seed, sorted(call_targets - starts))
        for k, wd in enumerate(words):
            hi = wd >> 12
            if hi in (1, 2):
                assert W.PROGRAM_START <= (wd & 0xFFF) < end and (wd & 1) == 0
            if hi == 1 and wd != 0x1200:
                assert (wd & 0xFFF) > W.PROGRAM_START + 2 * k       # forward only
            if hi == 0xB:
                assert (wd & 0xFFF) == W.PROGRAM_START + 2 * (k + 1)
                # V0 <- VX, VX <- VX AND VD, VX <- 6 in front of it
                x = (wd >> 8) & 0xF
                v0 = words[k - 1]
                assert v0 == 0x8000 | (x << 4) or (v0 & 0xFFF9) == 0x6000, hex(v0)
                assert words[k - 3] == 0x6006 | (x << 8) and words[k - 2] & 0xFF0F == 0x8002 | (x << 8)
            if hi == 0xF and (wd & 0xFF) in (0x33, 0x55):
                a = words[k - 1]
                assert a >> 12 == 0xA
                size = 3 if (wd & 0xFF) == 0x33 else ((wd >> 8) & 0xF) + 1
                addr = a & 0xFFF
                in_scratch = W.STORE_START <= addr and addr + size <= W.STORE_END
                in_tail = end <= addr and addr + size <= W.PROGRAM_START + len(rom)
                assert in_scratch or in_tail, (seed, k, hex(addr))
        # the slot before each region's end is never a skip
        skips = (0x3, 0x4, 0x5, 0x9)
        for k in returns + [words.index(0x1200)]:
            prev = words[k - 1]
            assert prev >> 12 not in skips and not (prev >> 12 == 0xE and prev & 0xFF in (0x9E, 0xA1))
