"""octax_get_state_noalloc (static device scratch, no allocation) against
octax_get_state on the same engine: two calls in a row, the second over a
smaller range, after steps that leave the state non-trivial."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _snap(L, eng, first, count, fn):
    from paper_2510_01764_amd import octax as X
    out = np.zeros(count, dtype=X.ENV_STATE_DTYPE)
    rc = getattr(L, fn)(eng._h, first, count, out.ctypes.data)
    assert rc == X.OCTAX_OK, L.octax_last_error()
    return out


def test_noalloc_snapshot_matches_get_state():
    import torch
    from paper_2510_01764_amd import octax as X
    from paper_2510_01764_amd import workload as W
    assert torch.cuda.is_available()
    L = X.library()
    spec = W.make_config("c3", num_envs=300)
    eng = X.Engine(spec, kernel="fused")
    dev = torch.device("cuda:0")
    K = 12
    act = torch.from_numpy(spec.actions(0, K)).to(dev)
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)
    eng.step_many(act, obs, rew, done)
    for first, count in ((200, 64), (7, 13)):          # the second call is smaller
        want = _snap(L, eng, first, count, "octax_get_state")
        got = _snap(L, eng, first, count, "octax_get_state_noalloc")
        assert want.tobytes() == got.tobytes(), (first, count)
        assert (want["t"] > 0).any() or (want["pc"] != 0x200).any()
    # the range limit is an error, not a fault
    big = np.zeros(X.NOALLOC_MAX_ENVS + 1, dtype=X.ENV_STATE_DTYPE)
    assert L.octax_get_state_noalloc(eng._h, 0, X.NOALLOC_MAX_ENVS + 1, big.ctypes.data) == X.OCTAX_E_INVALID
    assert b"OCTAX_NOALLOC_MAX_ENVS" in L.octax_last_error()
    eng.close()
