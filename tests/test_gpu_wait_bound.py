"""The fused kernel's bounded waits: a wait that gives up is reported, every
launch still ends, and the engine carries on exactly once its state is
restored.

The give-up is forced from the host with a one-tick wait bound (no long
step is run): the observation-writer waves then stop waiting for their
emulator waves at once and run ahead."""
import numpy as np
import pytest

from tests.parity_util import compare_states

pytestmark = pytest.mark.gpu


def test_a_wait_that_gives_up_is_reported_and_the_engine_carries_on():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    assert torch.cuda.is_available()
    spec = W.make_config("c3", num_envs=700)
    eng = X.Engine(spec, kernel="fused")
    dev = torch.device("cuda")
    K = 6
    acts = spec.actions(0, 2 * K)
    act = torch.from_numpy(acts[:K]).to(dev)
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)

    eng.set_wait_limit(1)                       # one tick: every wait that has to wait gives up
    eng.step_many(act, obs, rew, done)
    with pytest.raises(X.OctaxError) as err:
        eng.status()
    assert err.value.code == X.OCTAX_E_STATE
    eng.status()                                # reported once, then cleared

    # with the derived bound, and its state restored (the frame ring a runaway
    # writer left behind need not match the reported state), the engine
    # continues exactly
    eng.set_wait_limit(0)
    snap = eng.get_state()
    eng.set_state(0, snap)
    orc = O.OracleBatch(spec)
    ost = orc.get_state()
    c = X.canonical(snap)
    for f in ("v", "i", "pc", "sp", "dt", "st", "stack", "t", "prev_score", "rng", "prev_key", "mem", "disp", "hist"):
        ost[f] = c[f]
    orc.set_state(0, ost)
    act.copy_(torch.from_numpy(acts[K:]))
    eng.step_many(act, obs, rew, done)
    torch.cuda.synchronize()
    for k in range(K):
        oo, orw, od = orc.step(acts[K + k])
        assert np.array_equal(obs[k].cpu().numpy(), oo), k
        assert np.array_equal(rew[k].cpu().numpy(), orw) and np.array_equal(done[k].cpu().numpy(), od), k
    eng.status()
    compare_states(eng.get_state(), orc.get_state(), "after the bounded wait")
    eng.close()
    orc.close()
