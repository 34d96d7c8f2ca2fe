"""Parity of the SUPER-CHIP platform (128x64 display, its instructions,
(4, 128, 64) observations) between the HIP path and the CPU oracle.

Generated SUPER-CHIP programs (12 % of the slots SUPER-CHIP instructions) and
a directed program that runs every SUPER-CHIP instruction, 00FD included;
rewards, done flags and observations every step, and the full state - the
CHIP-8 part and the SUPER-CHIP part (mode, flag registers, display, frame
history) - after every launch.
"""
import dataclasses

import numpy as np
import pytest

from tests.parity_util import compare_schip, compare_states, run_rollouts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_01764_amd import octax
    octax.library()
    return torch


def _s1(n, seed=2, mean_horizon=60.0):
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("s1", num_envs=n)
    rng = np.random.default_rng(seed)
    return dataclasses.replace(spec, horizon=W.geometric_horizons(rng, n, mean_horizon))


def test_schip_generated_programs():
    resets = run_rollouts(_s1(1200), "plain", K=16, launches=3)
    assert resets > 100


def test_schip_graph_replays():
    run_rollouts(_s1(700, seed=3), "plain", K=8, launches=2, graph=True)


def test_schip_with_quirk_flags_and_descriptors():
    from paper_2510_01764_amd import workload as W
    spec = W.with_profile(_s1(900, seed=4), quirks=0x7F, seed=4)
    run_rollouts(spec, "plain", K=12, launches=2)


def test_schip_directed_program():
    from paper_2510_01764_amd import workload as W
    body = [0x00FF, 0xC07F, 0xC13F, 0xC20F, 0xF230, 0xD01A, 0xA300, 0xD010, 0x00C3, 0x00FB, 0xD015,
            0x00FC, 0x6507, 0xF575, 0x6500, 0xF585, 0x00FE, 0xF230, 0xD01A, 0xD010, 0x00C2, 0x00FB,
            0xF185, 0x00FF, 0x3301, 0x1202]
    stop = body[:-2] + [0x00FD]              # a second ROM stops at its end
    spec = W.custom_spec([W.assemble(body), W.assemble(stop)], 300, keys=W.KEYS_8, horizon=50, seed=9)
    spec = dataclasses.replace(spec, platform=1)
    run_rollouts(spec, "plain", K=10, launches=3)


def test_schip_reset_mask_and_observation():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _s1(333, seed=5, mean_horizon=1000.0)
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="plain")
    orc = O.OracleBatch(spec)
    E = spec.num_envs
    act = torch.zeros(E, dtype=torch.int32, device=dev)
    rew = torch.zeros(E, dtype=torch.float32, device=dev)
    done = torch.zeros(E, dtype=torch.uint8, device=dev)
    obs = torch.zeros((E, 4, 128, 64), dtype=torch.uint8, device=dev)
    acts = spec.actions(0, 10)
    for k in range(10):
        act.copy_(torch.from_numpy(acts[k]))
        eng.step(act, None, rew, done)
        orc.step(acts[k], want_obs=False)
    mask = (np.arange(E) % 4 == 1).astype(np.uint8)
    eng.reset(torch.from_numpy(mask).to(dev), obs)
    oo = orc.reset(mask)
    torch.cuda.synchronize()
    assert np.array_equal(obs.cpu().numpy(), oo)
    compare_states(eng.get_state(), orc.get_state(), "schip masked reset")
    compare_schip(eng.get_schip_state(), orc.get_schip(), "schip masked reset")
    eng.close()
    orc.close()


def test_schip_big_font_in_memory():
    from paper_2510_01764_amd import octax as X
    from tests.golden_util import big_font_pictures
    spec = _s1(4)
    eng = X.Engine(spec, kernel="plain")
    mem = eng.get_state()["ram"][:, 0xA0:0x140].reshape(4, 16, 10)
    want = np.packbits(big_font_pictures(), axis=2)[:, :, 0]
    assert all(np.array_equal(m, want) for m in mem)
    eng.close()


def test_schip_sticky_actions():
    from paper_2510_01764_amd import workload as W
    spec = dataclasses.replace(_s1(640, seed=6), sticky_q24=int(0.3 * (1 << 24)))
    assert spec.has_wrappers and spec.noop_max == 0 and spec.startup_len is None
    run_rollouts(spec, "plain", K=12, launches=2)


def test_schip_with_every_wrapper_and_masked_reset():
    """Start-up sequences, no-op resets and sticky actions on SUPER-CHIP envs:
    in automatic resets during K-step launches and in octax_reset."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    spec = W.with_wrappers(_s1(720, seed=7, mean_horizon=30.0), sticky=0.2, noop_max=6, startup_max=3, seed=3)
    resets = run_rollouts(spec, "plain", K=12, launches=3)
    assert resets > 100
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="plain")
    orc = O.OracleBatch(spec)
    compare_states(eng.get_state(), orc.get_state(), "schip wrappers after create")
    compare_schip(eng.get_schip_state(), orc.get_schip(), "schip wrappers after create")
    E = spec.num_envs
    act = torch.zeros(E, dtype=torch.int32, device=dev)
    rew = torch.zeros(E, dtype=torch.float32, device=dev)
    done = torch.zeros(E, dtype=torch.uint8, device=dev)
    acts = spec.actions(0, 6)
    for k in range(6):
        act.copy_(torch.from_numpy(acts[k]))
        eng.step(act, None, rew, done)
        orc.step(acts[k], want_obs=False)
    mask = (np.arange(E) % 3 == 0).astype(np.uint8)
    obs = torch.zeros((E, 4, 128, 64), dtype=torch.uint8, device=dev)
    eng.reset(torch.from_numpy(mask).to(dev), obs)
    oo = orc.reset(mask)
    torch.cuda.synchronize()
    assert np.array_equal(obs.cpu().numpy(), oo)
    compare_states(eng.get_state(), orc.get_state(), "schip wrappers masked reset")
    compare_schip(eng.get_schip_state(), orc.get_schip(), "schip wrappers masked reset")
    eng.close()
    orc.close()


# 128x64 mode; a 16x16 sprite from 0xFF0 (rows 8..15 read 0x000..0x00F) drawn
# at (120, 56) so that both the right and the bottom edge clip it; BCD, bulk
# stores and loads across 0xFFF as in the CHIP-8 wrap program; flag
# registers; scrolls; the instruction at 0xFFF is V3 << 8 | V4 = 0x1202.
SCHIP_WRAP_PROGRAM = bytes.fromhex(
    "00FF"  # 200 128x64 mode
    "6A12" "6312" "6402" "6581" "6642" "6724" "60F0"
    "6178"  # V1 = 120
    "6238"  # V2 = 56
    "AFF0"  # I = 0xFF0
    "D120"  # 16x16 sprite
    "AFFE" "F033" "AFFC" "F755" "AFFD" "F565"
    "F775"  # V0..V7 to the flag registers
    "7C01"
    "00C1"  # scroll down 1
    "00FB"  # scroll right 4
    "3C40" "1FFF"
    "00FE" "6C00" "00FF" "1202"
)


def test_schip_program_space_edges():
    """ROMs of 0 to 3,584 bytes and random bytes as code on the SUPER-CHIP
    platform, and a 128x64 program that reads and writes across 0xFFF."""
    from tests.test_oracle_wrap import WRAP_PROGRAM
    spec = _s1(640, seed=12, mean_horizon=24.0)
    rng = np.random.default_rng(12)
    rnd = lambda n: rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()   # noqa: E731
    full = 0x1000 - 0x200
    roms = [b"", b"\x12", rnd(full), WRAP_PROGRAM + rnd(full - len(WRAP_PROGRAM)),
            SCHIP_WRAP_PROGRAM, SCHIP_WRAP_PROGRAM + rnd(full - len(SCHIP_WRAP_PROGRAM)), rnd(full - 1), rnd(97)]
    assert len(roms) == spec.num_roms
    spec = dataclasses.replace(spec, roms=roms, name="schip-rom-edges")
    run_rollouts(spec, "plain", K=12, launches=3)
