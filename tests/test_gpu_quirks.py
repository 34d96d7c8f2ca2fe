"""Parity of the quirk flags and game descriptors (score mode, second
termination clause) between the HIP path and the CPU oracle.

Mixed-ROM workloads with the flags on (all together and one at a time) and
per-ROM descriptors (every score mode and termination op), short horizons so that resets happen in most launches;
rewards, done flags and observations are compared every step and the full
architectural state after each launch, for both kernels, every fused block
size, graph replays and the environment wrappers combined.
"""
import dataclasses

import numpy as np
import pytest

from tests.parity_util import run_rollouts

pytestmark = pytest.mark.gpu

FLAGS = {"shift_vx": 1 << 1, "mem_keep_i": 1 << 2, "jump_vx": 1 << 3, "no_vf_reset": 1 << 4, "pixel_wrap": 1 << 5,
         "display_wait": 1 << 6}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_01764_amd import octax
    octax.library()
    return torch


def _profiled(num_envs, quirks=0x7F, seed=5, mean_horizon=24.0, descriptors=True):
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("c3", num_envs=num_envs)
    rng = np.random.default_rng(seed)
    spec = dataclasses.replace(spec, horizon=W.geometric_horizons(rng, num_envs, mean_horizon))
    spec = W.with_profile(spec, quirks=quirks, seed=seed)
    if not descriptors:
        spec = dataclasses.replace(spec, score_mode=None, score_arg=None, term_op=None, term2_op=None,
                                   term2_reg=None, term2_value=None)
    return spec


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_profile_mixed_roms(kernel):
    spec = _profiled(1000)
    resets = run_rollouts(spec, kernel, K=24, launches=3)
    assert resets > 1000


@pytest.mark.parametrize("flag", sorted(FLAGS))
def test_each_quirk_alone(flag):
    spec = _profiled(600, quirks=1 | FLAGS[flag], seed=7, descriptors=False)
    run_rollouts(spec, "fused", K=16, launches=2)


def test_descriptors_only():
    spec = _profiled(800, quirks=1, seed=8)
    assert spec.has_profile and spec.quirks == 1
    run_rollouts(spec, "fused", K=20, launches=2)


@pytest.mark.parametrize("ipw", [64, 128])
def test_profile_fused_block_sizes(ipw):
    spec = _profiled(700, seed=9)
    run_rollouts(spec, "fused", K=16, launches=2, envs_per_block=ipw)


def test_profile_with_wrappers_graph():
    from paper_2510_01764_amd import workload as W
    spec = W.with_wrappers(_profiled(1536, seed=10, mean_horizon=40.0), sticky=0.2, noop_max=12, startup_max=3, seed=2)
    run_rollouts(spec, "fused", K=32, launches=2, graph=True)
    run_rollouts(spec, "plain", K=8, launches=1)
