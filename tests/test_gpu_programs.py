"""Parity of the HIP path with the oracle on the Target Shooter programs
(three levels written in Octo, assembled by paper_2510_01764_amd/octo.py):
real game code with timer-paced loops, random target positions, sprite
collisions and game-over flags, as a second workload beside the generated
programs.
"""
import numpy as np
import pytest

from tests.parity_util import compare_states, run_rollouts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_01764_amd import octax
    octax.library()
    return torch


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_target_shooter_random_actions(kernel):
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("ts", num_envs=3000)
    run_rollouts(spec, kernel, K=32, launches=3)


def test_target_shooter_small_blocks():
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("ts", num_envs=777)
    run_rollouts(spec, "fused", K=24, launches=2, envs_per_block=64)


def test_target_shooter_aiming_policy_replayed():
    """Actions chosen on the oracle by a policy that aims at the target (so
    the games score and end), replayed on the GPU step by step."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    from tests.test_target_shooter import _aim
    spec = W.make_config("ts", num_envs=96)
    orc = O.OracleBatch(spec)
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="fused")
    E = spec.num_envs
    act = torch.zeros(E, dtype=torch.int32, device=dev)
    obs = torch.zeros((E, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros(E, dtype=torch.float32, device=dev)
    done = torch.zeros(E, dtype=torch.uint8, device=dev)
    scored = ended = 0
    for k in range(600):
        a = _aim(orc.get_state(0, E)["v"])
        act.copy_(torch.from_numpy(a))
        eng.step(act, obs if k % 50 == 49 else None, rew, done)
        oo, orw, od = orc.step(a, want_obs=(k % 50 == 49))
        torch.cuda.synchronize()
        assert np.array_equal(rew.cpu().numpy(), orw) and np.array_equal(done.cpu().numpy(), od), k
        if oo is not None:
            assert np.array_equal(obs.cpu().numpy(), oo), k
        scored += int((orw > 0).sum())
        ended += int((od == 1).sum())
    compare_states(eng.get_state(), orc.get_state(), "aiming policy")
    assert scored > 100 and ended > 0
    eng.close()
    orc.close()


def test_target_shooter_full_size_sampled():
    """65,536 envs over the three levels in the benchmark's launch shape
    (K = 64 per graph replay); a sample of envs replayed on the oracle."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("ts")
    K = 64
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="fused")
    act = torch.zeros((K, spec.num_envs), dtype=torch.int32, device=dev)
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)
    g = eng.graph(act, obs, rew, done)
    sample = np.random.default_rng(11).choice(spec.num_envs, size=160, replace=False)
    sample = np.concatenate([sample, [0, 1, 255, 256, spec.num_envs - 1]])
    orc = O.OracleBatch(spec.subset(sample))
    for rep in range(2):
        an = spec.actions(rep * K, K)
        act.copy_(torch.from_numpy(an))
        g.launch()
        torch.cuda.synchronize()
        r_np = rew[:, sample].cpu().numpy()
        d_np = done[:, sample].cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(an[k][sample], want_obs=(k == K - 1))
            assert np.array_equal(r_np[k], orw) and np.array_equal(d_np[k], od), (rep, k)
            if oo is not None:
                assert np.array_equal(obs[k, sample].cpu().numpy(), oo), (rep, k)
    got = np.concatenate([eng.get_state(int(e), 1) for e in sample])
    compare_states(got, orc.get_state(), "full-size Target Shooter sample")
    g.close()
    eng.close()
    orc.close()
