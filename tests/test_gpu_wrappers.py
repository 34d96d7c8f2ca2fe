"""Parity of the environment wrappers (Section 3.2: start-up sequences, no-op
reset, sticky actions) between the HIP path and the CPU oracle.

Mixed-ROM workloads with every wrapper on, short horizons so that automatic
resets (and with them start-up and no-op steps) happen in most launches;
rewards, done flags and observations are compared every step and the full
architectural state (previous key and RNG state included) after each launch.
"""
import dataclasses

import numpy as np
import pytest

from tests.parity_util import compare_states, run_rollouts as _run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_01764_amd import octax
    octax.library()
    return torch


def _wrapped(num_envs, sticky=0.25, noop_max=5, seed=3, mean_horizon=24.0):
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("c3", num_envs=num_envs)
    R = spec.num_roms
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 4, size=R).astype(np.uint8)
    akeys = np.asarray(spec.action_keys)
    nact = np.asarray(spec.num_actions)
    picks = rng.integers(0, nact[0] + 1, size=(R, 16))
    skeys = np.where(picks < nact[:, None], akeys[np.arange(R)[:, None], np.minimum(picks, 15)], 16)
    horizon = W.geometric_horizons(rng, num_envs, mean_horizon)
    return dataclasses.replace(spec, sticky_q24=int(sticky * (1 << 24)), noop_max=noop_max,
                               startup_len=lens, startup_keys=skeys.astype(np.uint8), horizon=horizon)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_wrappers_mixed_roms(kernel):
    spec = _wrapped(1000)
    resets = _run(spec, kernel, K=24, launches=3)
    assert resets > 1000          # start-up and no-op steps ran in many resets


@pytest.mark.parametrize("ipw", [64, 128])
def test_wrappers_fused_block_sizes(ipw):
    spec = _wrapped(700, sticky=0.5, noop_max=3, seed=9)
    _run(spec, "fused", K=16, launches=2, envs_per_block=ipw)


def test_wrappers_graph_rollout():
    spec = _wrapped(1536, sticky=0.1, noop_max=30, seed=4, mean_horizon=40.0)
    _run(spec, "fused", K=32, launches=2, graph=True)


@pytest.mark.parametrize("which", ["sticky", "noop", "startup"])
def test_each_wrapper_alone(which):
    kw = dict(sticky=0.0, noop_max=0)
    if which == "sticky":
        kw["sticky"] = 0.75
    if which == "noop":
        kw["noop_max"] = 9
    spec = _wrapped(600, seed=17, **kw)
    if which != "startup":
        spec = dataclasses.replace(spec, startup_len=None, startup_keys=None)
    _run(spec, "fused", K=20, launches=2)


def test_wrappers_masked_reset():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _wrapped(400, seed=21, mean_horizon=1000.0)
    dev = torch.device("cuda")
    for kernel in ("plain", "fused"):
        eng = X.Engine(spec, kernel=kernel)
        orc = O.OracleBatch(spec)
        E = spec.num_envs
        obs = torch.zeros((E, 4, 64, 32), dtype=torch.uint8, device=dev)
        act = torch.zeros(E, dtype=torch.int32, device=dev)
        rew = torch.zeros(E, dtype=torch.float32, device=dev)
        done = torch.zeros(E, dtype=torch.uint8, device=dev)
        acts = spec.actions(0, 12)
        for k in range(12):
            act.copy_(torch.from_numpy(acts[k]))
            eng.step(act, None, rew, done)
            orc.step(acts[k], want_obs=False)
        mask = (np.arange(E) % 3 == 1).astype(np.uint8)
        eng.reset(torch.from_numpy(mask).to(dev), obs)
        oo = orc.reset(mask)
        torch.cuda.synchronize()
        assert np.array_equal(obs.cpu().numpy(), oo), kernel
        compare_states(eng.get_state(), orc.get_state(), f"masked reset {kernel}")
        eng.close()
        orc.close()


@pytest.mark.parametrize("chains", [1, 2, 5])
def test_wrappers_lone_reset_chains(chains):
    """One block whose envs never truncate except `chains` of them with a
    horizon of one step: each of those resets at every step and runs up to 30
    no-op steps and its start-up sequence, so its lane goes on alone (or with
    one other lane of its wave, for chains = 5) for hundreds of slots after
    the rest of its wave has finished the launch."""
    spec = _wrapped(256, sticky=0.25, noop_max=30, seed=5, mean_horizon=1000.0)
    horizon = np.zeros(256, dtype=np.uint32)          # 0: no truncation
    horizon[[3, 77, 130, 200, 255][:chains]] = 1
    spec = dataclasses.replace(spec, horizon=horizon)
    resets = _run(spec, "fused", K=16, launches=2)
    assert resets >= 2 * 16 * chains


def test_wrappers_by_horizon_placement():
    """Envs dealt over the wavefronts in order of horizon (a ragged last
    wavefront of 40 envs): every env's outputs and state as with the oracle."""
    spec = _wrapped(1000, sticky=0.25, noop_max=12, seed=8, mean_horizon=12.0)
    _run(spec, "fused", K=16, launches=2, placement="by_horizon")
