"""Side-by-side runs of the HIP engine and the CPU oracle on the same inputs."""
import numpy as np

FIELDS = ("v", "i", "pc", "sp", "dt", "st", "stack", "t", "prev_score", "rng", "prev_key", "mem", "disp", "hist")


def compare_states(gpu_states, oracle_states, where=""):
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    g = X.canonical(gpu_states)
    o = O.canonical(oracle_states)
    for f in FIELDS:
        a, b = np.asarray(g[f]), np.asarray(o[f])
        if a.shape != b.shape or not np.array_equal(a, b):
            bad = np.argwhere(a != b) if a.shape == b.shape else "shape"
            raise AssertionError(f"{where}: field {f} differs (first mismatches {bad[:5] if not isinstance(bad, str) else bad})")


def compare_gpu_states(a, b, where=""):
    """Two architectural-state snapshots taken from the GPU library."""
    from paper_2510_01764_amd import octax as X
    g, h = X.canonical(a), X.canonical(b)
    for f in FIELDS:
        if not np.array_equal(g[f], h[f]):
            raise AssertionError(f"{where}: field {f} differs")


class Pair:
    """An engine and an oracle batch stepped in lockstep."""

    def __init__(self, spec, kernel="fused", placement=None, envs_per_block=256, rom_in_lds=True):
        import torch
        from oracle import oracle as O
        from paper_2510_01764_amd import octax as X
        self.torch = torch
        self.spec = spec
        self.E = spec.num_envs
        self.eng = X.Engine(spec, kernel=kernel, placement=placement, envs_per_block=envs_per_block,
                            rom_in_lds=rom_in_lds)
        self.orc = O.OracleBatch(spec)
        dev = torch.device("cuda")
        self.obs = torch.zeros((self.E, 4, 64, 32), dtype=torch.uint8, device=dev)
        self.rew = torch.zeros(self.E, dtype=torch.float32, device=dev)
        self.done = torch.zeros(self.E, dtype=torch.uint8, device=dev)
        self.act = torch.zeros(self.E, dtype=torch.int32, device=dev)

    def step(self, actions_np, check_obs=True):
        torch = self.torch
        self.act.copy_(torch.from_numpy(np.ascontiguousarray(actions_np, dtype=np.int32)))
        self.eng.step(self.act, self.obs if check_obs else None, self.rew, self.done)
        oo, orw, od = self.orc.step(actions_np, want_obs=check_obs)
        torch.cuda.synchronize()
        gr, gd = self.rew.cpu().numpy(), self.done.cpu().numpy()
        assert np.array_equal(gr, orw), f"reward differs at envs {np.nonzero(gr != orw)[0][:8]}"
        assert np.array_equal(gd, od), f"done differs at envs {np.nonzero(gd != od)[0][:8]}"
        if check_obs:
            go = self.obs.cpu().numpy()
            if not np.array_equal(go, oo):
                bad = np.unique(np.nonzero(go != oo)[0])
                raise AssertionError(f"obs differs at envs {bad[:8]}")
        return gr, gd

    def check_state(self, where=""):
        compare_states(self.eng.get_state(), self.orc.get_state(), where)

    def close(self):
        self.eng.close()
        self.orc.close()


def schip_pixels(fb):
    """octax_schip_state rows [..., 64, 2] (uint64, bit 63 - (x mod 64)) -> pixels [..., 64, 128]."""
    b = np.ascontiguousarray(fb, dtype=">u8").view(np.uint8)
    return np.unpackbits(b, axis=-1).reshape(fb.shape[:-2] + (64, 128))


def compare_schip(gpu_sx, oracle_sx, where=""):
    """SUPER-CHIP parts of the state: mode, flag registers, display, previous frames."""
    assert np.array_equal(gpu_sx["hires"], oracle_sx["hires"].astype(np.uint32)), f"{where}: hires differs"
    assert np.array_equal(gpu_sx["rpl"], oracle_sx["rpl"]), f"{where}: flag registers differ"
    hd = schip_pixels(gpu_sx["fb"])
    if not np.array_equal(hd, oracle_sx["hd"]):
        raise AssertionError(f"{where}: display differs at envs {np.unique(np.nonzero(hd != oracle_sx['hd'])[0])[:8]}")
    assert np.array_equal(schip_pixels(gpu_sx["hist"]), oracle_sx["hist"]), f"{where}: frame history differs"


def run_rollouts(spec, kernel, K, launches, envs_per_block=256, graph=False, placement=None):
    """K-step launches (or graph replays) of the engine beside the oracle:
    rewards, done flags and observations compared at every step, the full
    architectural state after every launch.  Returns the number of resets."""
    import torch
    from oracle import oracle as O
    from paper_2510_01764_amd import octax as X
    E = spec.num_envs
    dev = torch.device("cuda")
    eng = X.Engine(spec, kernel=kernel, envs_per_block=envs_per_block, placement=placement)
    orc = O.OracleBatch(spec)
    compare_states(eng.get_state(), orc.get_state(), f"{kernel} after create")
    act = torch.zeros((K, E), dtype=torch.int32, device=dev)
    obs = torch.zeros((K, E) + eng.obs_shape, dtype=torch.uint8, device=dev)
    rew = torch.zeros((K, E), dtype=torch.float32, device=dev)
    done = torch.zeros((K, E), dtype=torch.uint8, device=dev)
    g = eng.graph(act, obs, rew, done) if graph else None
    resets = 0
    for rep in range(launches):
        an = spec.actions(rep * K, K)
        act.copy_(torch.from_numpy(an))
        if g is not None:
            g.launch()
        else:
            eng.step_many(act, obs, rew, done)
        torch.cuda.synchronize()
        r_np, d_np, o_np = rew.cpu().numpy(), done.cpu().numpy(), obs.cpu().numpy()
        for k in range(K):
            oo, orw, od = orc.step(an[k])
            assert np.array_equal(r_np[k], orw), (kernel, rep, k, np.nonzero(r_np[k] != orw)[0][:8])
            assert np.array_equal(d_np[k], od), (kernel, rep, k, np.nonzero(d_np[k] != od)[0][:8])
            if not np.array_equal(o_np[k], oo):
                bad = np.unique(np.nonzero(o_np[k] != oo)[0])
                raise AssertionError(f"{kernel} launch {rep} step {k}: obs differs at envs {bad[:8]}")
            resets += int((od != 0).sum())
        compare_states(eng.get_state(), orc.get_state(), f"{kernel} launch {rep}")
        if eng.schip:
            compare_schip(eng.get_schip_state(), orc.get_schip(), f"{kernel} launch {rep}")
    if g is not None:
        g.close()
    eng.close()
    orc.close()
    return resets


def fnv1a64(rows):
    """64-bit FNV-1a of each row of a uint8 matrix [n][m] (vectorised)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    h = np.full(rows.shape[0], 0xCBF29CE484222325, dtype=np.uint64)
    prime = np.uint64(0x100000001B3)
    with np.errstate(over="ignore"):
        for j in range(rows.shape[1]):
            h ^= rows[:, j].astype(np.uint64)
            h *= prime
    return h


def oracle_env_state_bytes(states):
    """Oracle states as octax_env_state records (the bytes octax_get_state
    returns), for digest comparisons."""
    from paper_2510_01764_amd import octax as X
    out = np.zeros(len(states), dtype=X.ENV_STATE_DTYPE)
    for f in ("v", "i", "pc", "sp", "dt", "st", "prev_key", "stack", "t", "prev_score", "rng"):
        out[f] = states[f]
    out["ram"] = states["mem"]
    rows = lambda d: np.packbits(np.ascontiguousarray(d, dtype=np.uint8), axis=-1).view(">u8")[..., 0]
    out["fb"] = rows(states["disp"])
    out["hist"] = rows(states["hist"])
    return out
