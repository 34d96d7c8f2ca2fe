"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer emulation: every comparison is exact (obs bytes, float rewards of
integer deltas, done bits, full architectural state).
"""
import numpy as np
import pytest

from tests.parity_util import Pair, compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_01764_amd import octax
    octax.library()
    return torch


def _spec(name, **kw):
    from paper_2510_01764_amd import workload as W
    return W.make_config(name, **kw)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_c1_every_step_full_state(kernel):
    """16 envs of one 256-instruction ROM, 1000 steps: obs, reward, done every step; state often."""
    spec = _spec("c1")
    p = Pair(spec, kernel=kernel)
    acts = spec.actions(0, spec.steps)
    dones = 0
    for k in range(spec.steps):
        _, d = p.step(acts[k])
        dones += int((d != 0).sum())
        if k < 64 or k % 50 == 0 or d.any():
            p.check_state(f"c1 {kernel} step {k}")
    p.check_state("c1 end")
    assert dones > 0          # the run crosses episode boundaries
    p.close()


@pytest.mark.parametrize("kernel,placement", [("plain", "identity"), ("fused", "by_rom"),
                                              ("fused", "identity"), ("plain", "by_rom"),
                                              ("fused", "by_horizon"), ("plain", "by_horizon")])
def test_mixed_roms_small(kernel, placement):
    """Sixteen ROMs mixed within every wavefront, ragged env count, geometric horizons."""
    spec = _spec("c3", num_envs=1000)
    p = Pair(spec, kernel=kernel, placement=placement)
    acts = spec.actions(0, 120)
    for k in range(120):
        p.step(acts[k], check_obs=(k % 7 == 0 or k > 110))
        if k % 40 == 0:
            p.check_state(f"mixed {kernel}/{placement} step {k}")
    p.check_state("mixed end")
    p.close()


@pytest.mark.parametrize("ipw,lds", [(64, True), (128, False), (256, True), (256, False)])
def test_fused_tunings_agree(ipw, lds):
    spec = _spec("c3", num_envs=777)
    p = Pair(spec, kernel="fused", envs_per_block=ipw, rom_in_lds=lds)
    acts = spec.actions(0, 60)
    for k in range(60):
        p.step(acts[k], check_obs=(k % 10 == 9))
    p.check_state(f"tuning {ipw}/{lds}")
    p.close()


def test_draw_heavy_edges():
    """40% DXYN with N up to 15 near the screen edges, 20 instructions per frame."""
    spec = _spec("c5", num_envs=600)
    p = Pair(spec, kernel="fused")
    acts = spec.actions(0, 50)
    for k in range(50):
        p.step(acts[k], check_obs=True)
    p.check_state("c5 small end")
    q = Pair(spec, kernel="plain")
    for k in range(20):
        q.step(acts[k], check_obs=(k % 5 == 4))
    q.check_state("c5 small plain")
    p.close()
    q.close()


def test_single_env_and_one_lane_tail():
    spec = _spec("c3", num_envs=65)
    for kernel in ("plain", "fused"):
        p = Pair(spec, kernel=kernel)
        acts = spec.actions(0, 30)
        for k in range(30):
            p.step(acts[k])
        p.check_state(f"65 envs {kernel}")
        p.close()
    spec1 = _spec("c1", num_envs=1)
    p = Pair(spec1, kernel="fused")
    acts = spec1.actions(0, 40)
    for k in range(40):
        p.step(acts[k])
    p.check_state("single env")
    p.close()


def test_out_of_range_actions_are_noop():
    spec = _spec("c3", num_envs=300)
    p = Pair(spec, kernel="fused")
    rng = np.random.default_rng(1)
    for k in range(40):
        a = rng.integers(-3, 20, size=spec.num_envs).astype(np.int32)
        a[::5] = np.iinfo(np.int32).min
        a[1::5] = np.iinfo(np.int32).max
        p.step(a, check_obs=(k % 8 == 0))
    p.check_state("out of range actions")
    p.close()


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_step_many_matches_single_steps(kernel):
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c3", num_envs=513)
    K = 24
    acts = spec.actions(0, 3 * K)
    eng = X.Engine(spec, kernel=kernel)
    orc = O.OracleBatch(spec)
    dev = torch.device("cuda")
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)
    for rep in range(3):
        a = torch.from_numpy(acts[rep * K:(rep + 1) * K].copy()).to(dev)
        eng.step_many(a, obs, rew, done)
        torch.cuda.synchronize()
        r_np, d_np, o_np = rew.cpu().numpy(), done.cpu().numpy(), obs.cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(acts[rep * K + k])
            assert np.array_equal(r_np[k], orw) and np.array_equal(d_np[k], od), (rep, k)
            assert np.array_equal(o_np[k], oo), (rep, k)
        compare_states(eng.get_state(), orc.get_state(), f"step_many {kernel} rep {rep}")
    # one observation slot: only the last step's observation is kept
    obs1 = torch.zeros((1, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    a = torch.from_numpy(spec.actions(3 * K, K)).to(dev)
    eng.step_many(a, obs1, rew, done)
    torch.cuda.synchronize()
    an = spec.actions(3 * K, K)
    for k in range(K):
        oo, _, _ = orc.step(an[k])
    assert np.array_equal(obs1[0].cpu().numpy(), oo)
    eng.close()
    orc.close()


def test_graph_replays_with_eager_work_between():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c3", num_envs=700)
    K = 16
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="fused")
    orc = O.OracleBatch(spec)
    act = torch.zeros((K, spec.num_envs), dtype=torch.int32, device=dev)
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)
    g = eng.graph(act, obs, rew, done)
    for rep in range(4):
        an = spec.actions(rep * K, K)
        act.copy_(torch.from_numpy(an))
        g.launch()
        torch.cuda.synchronize()
        junk = torch.arange(1000, device=dev).sum()      # eager work between replays
        assert int(junk) == 499500
        r_np, d_np, o_np = rew.cpu().numpy(), done.cpu().numpy(), obs.cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(an[k])
            assert np.array_equal(r_np[k], orw) and np.array_equal(d_np[k], od), (rep, k)
            assert np.array_equal(o_np[k], oo), (rep, k)
    compare_states(eng.get_state(), orc.get_state(), "graph")
    g.close()
    eng.close()
    orc.close()


def test_reset_mask_and_observation():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c3", num_envs=300)
    dev = torch.device("cuda")
    for kernel in ("plain", "fused"):
        eng = X.Engine(spec, kernel=kernel)
        orc = O.OracleBatch(spec)
        obs = torch.zeros((spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
        eng.reset(None, obs)
        assert not obs.any().item()
        act = torch.zeros(spec.num_envs, dtype=torch.int32, device=dev)
        rew = torch.zeros(spec.num_envs, dtype=torch.float32, device=dev)
        done = torch.zeros(spec.num_envs, dtype=torch.uint8, device=dev)
        acts = spec.actions(0, 25)
        for k in range(25):
            act.copy_(torch.from_numpy(acts[k]))
            eng.step(act, None, rew, done)
            orc.step(acts[k], want_obs=False)
        mask = (np.arange(spec.num_envs) % 3 == 0).astype(np.uint8)
        eng.reset(torch.from_numpy(mask).to(dev), obs)
        oo = orc.reset(mask)
        torch.cuda.synchronize()
        assert np.array_equal(obs.cpu().numpy(), oo), kernel
        compare_states(eng.get_state(), orc.get_state(), f"masked reset {kernel}")
        for k in range(10):
            act.copy_(torch.from_numpy(acts[k]))
            eng.step(act, obs, rew, done)
            oo, _, _ = orc.step(acts[k])
        torch.cuda.synchronize()
        assert np.array_equal(obs.cpu().numpy(), oo), kernel
        eng.close()
        orc.close()


def test_snapshot_restore_continues_exactly():
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c3", num_envs=400)
    dev = torch.device("cuda")
    a = X.Engine(spec, kernel="fused")
    act = torch.zeros(spec.num_envs, dtype=torch.int32, device=dev)
    rew = torch.zeros(spec.num_envs, dtype=torch.float32, device=dev)
    done = torch.zeros(spec.num_envs, dtype=torch.uint8, device=dev)
    acts = spec.actions(0, 80)
    for k in range(40):
        act.copy_(torch.from_numpy(acts[k]))
        a.step(act, None, rew, done)
    snap = a.get_state()
    # the oracle accepts the snapshot through its own state format
    orc = O.OracleBatch(spec)
    ost = orc.get_state()
    from paper_2510_01764_amd.octax import canonical
    c = canonical(snap)
    for f in ("v", "i", "pc", "sp", "dt", "st", "stack", "t", "prev_score", "rng", "prev_key"):
        ost[f] = c[f]
    ost["mem"] = c["mem"]
    ost["disp"] = c["disp"]
    ost["hist"] = c["hist"]
    orc.set_state(0, ost)
    b = X.Engine(spec, kernel="plain")
    b.set_state(0, snap)
    compare_states(b.get_state(), orc.get_state(), "restored")
    obs_a = torch.zeros((spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    obs_b = torch.zeros_like(obs_a)
    rew_b = torch.zeros_like(rew)
    done_b = torch.zeros_like(done)
    for k in range(40, 80):
        act.copy_(torch.from_numpy(acts[k]))
        a.step(act, obs_a, rew, done)
        b.step(act, obs_b, rew_b, done_b)
        oo, orw, od = orc.step(acts[k])
        torch.cuda.synchronize()
        assert torch.equal(obs_a, obs_b) and torch.equal(rew, rew_b) and torch.equal(done, done_b)
        assert np.array_equal(obs_b.cpu().numpy(), oo) and np.array_equal(rew_b.cpu().numpy(), orw)
    compare_states(a.get_state(), orc.get_state(), "after restore")
    a.close()
    b.close()
    orc.close()


def test_full_size_mixed_rom_sampled():
    """65,536 envs over 16 ROMs in the benchmark's launch shape (K = 64 per graph replay);
    a sample of envs is replayed on the oracle (envs are independent)."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c3")
    K = 64
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="fused")
    act = torch.zeros((K, spec.num_envs), dtype=torch.int32, device=dev)
    obs = torch.zeros((K, spec.num_envs, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, spec.num_envs), dtype=torch.float32, device=dev)
    done = torch.zeros((K, spec.num_envs), dtype=torch.uint8, device=dev)
    g = eng.graph(act, obs, rew, done)
    sample = np.random.default_rng(7).choice(spec.num_envs, size=192, replace=False)
    sample = np.concatenate([sample, [0, 1, 63, 64, 255, 256, spec.num_envs - 1]])
    orc = O.OracleBatch(spec.subset(sample))
    for rep in range(2):
        an = spec.actions(rep * K, K)
        act.copy_(torch.from_numpy(an))
        g.launch()
        torch.cuda.synchronize()
        r_np = rew[:, sample].cpu().numpy()
        d_np = done[:, sample].cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(an[k][sample], want_obs=(k == K - 1 or k == 0))
            assert np.array_equal(r_np[k], orw) and np.array_equal(d_np[k], od), (rep, k)
            if oo is not None:
                assert np.array_equal(obs[k, sample].cpu().numpy(), oo), (rep, k)
    got = np.concatenate([eng.get_state(int(e), 1) for e in sample])
    compare_states(got, orc.get_state(), "full-size sample")
    g.close()
    eng.close()
    orc.close()


def test_single_rom_at_scale_full_run():
    """4,096 envs of one 1,024-instruction ROM for 10,000 steps with auto-reset: every
    reward and done flag of every env against the oracle (threaded over the host's
    cores), the last observation and the full final state; the plain kernel agrees."""
    import os
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c2")
    E, S, K = spec.num_envs, spec.steps, 500
    dev = torch.device("cuda")
    orc = O.OracleBatch(spec)
    acts = spec.actions(0, S)
    o_rew, o_done, _ = orc.run_threaded(acts, min(16, len(os.sched_getaffinity(0))))
    out = {}
    for kernel in ("fused", "plain"):
        eng = X.Engine(spec, kernel=kernel)
        obs = torch.zeros((1, E, 4, 64, 32), dtype=torch.uint8, device=dev)
        rew = torch.zeros((K, E), dtype=torch.float32, device=dev)
        done = torch.zeros((K, E), dtype=torch.uint8, device=dev)
        for c in range(S // K):
            a = torch.from_numpy(acts[c * K:(c + 1) * K].copy()).to(dev)
            eng.step_many(a, obs, rew, done)
            torch.cuda.synchronize()
            assert np.array_equal(rew.cpu().numpy(), o_rew[c * K:(c + 1) * K]), (kernel, c)
            assert np.array_equal(done.cpu().numpy(), o_done[c * K:(c + 1) * K]), (kernel, c)
        out[kernel] = (obs[0].cpu().numpy(), eng.get_state())
        eng.close()
    assert int((o_done != 0).sum()) > E, "episodes end and restart during the run"
    compare_states(out["fused"][1], orc.get_state(), "c2 fused final state")
    compare_states(out["plain"][1], orc.get_state(), "c2 plain final state")
    assert np.array_equal(out["fused"][0], out["plain"][0])
    orc.close()


def test_draw_heavy_full_size_sampled():
    """1,048,576 envs over 64 draw-heavy ROMs (40% DXYN, N up to 15 near the edges,
    20 instructions per frame) for the workload's full 1,000 steps, in graph
    replays of K = 50; a sample of 207 envs is replayed on the oracle step by
    step (envs are independent): every step's rewards and done flags, the last
    observation of every replay and the final state."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    spec = _spec("c5")
    E, K, S = spec.num_envs, 50, spec.steps
    assert S % K == 0
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel="fused")
    act = torch.zeros((K, E), dtype=torch.int32, device=dev)
    obs = torch.zeros((1, E, 4, 64, 32), dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, E), dtype=torch.float32, device=dev)
    done = torch.zeros((K, E), dtype=torch.uint8, device=dev)
    g = eng.graph(act, obs, rew, done)
    sample = np.random.default_rng(11).choice(E, size=200, replace=False)
    sample = np.concatenate([sample, [0, 1, 255, 256, E // 2, E - 2, E - 1]])
    orc = O.OracleBatch(spec.subset(sample))
    resets = 0
    for rep in range(S // K):
        an = spec.actions(rep * K, K)
        act.copy_(torch.from_numpy(an))
        g.launch()
        torch.cuda.synchronize()
        r_np = rew[:, sample].cpu().numpy()
        d_np = done[:, sample].cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(an[k][sample], want_obs=(k == K - 1))
            assert np.array_equal(r_np[k], orw) and np.array_equal(d_np[k], od), (rep, k)
        resets += int((d_np != 0).sum())
        assert np.array_equal(obs[0, sample].cpu().numpy(), oo), rep
    assert resets > 100, "episodes end and restart during the run"
    got = np.concatenate([eng.get_state(int(e), 1) for e in sample])
    compare_states(got, orc.get_state(), "c5 full-size sample")
    g.close()
    eng.close()
    orc.close()
