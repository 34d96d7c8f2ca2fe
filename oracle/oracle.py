"""ctypes wrapper of the CPU oracle (``chip8_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports it, and it
imports nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chip8_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Mirror of the C struct `oracle_state` (field order and sizes).
STATE_DTYPE = np.dtype([
    ("v", np.uint8, (16,)),
    ("i", np.uint16),
    ("pc", np.uint16),
    ("sp", np.uint8),
    ("dt", np.uint8),
    ("st", np.uint8),
    ("prev_key", np.uint8),
    ("stack", np.uint16, (16,)),
    ("t", np.uint32),
    ("prev_score", np.int32),
    ("rng", np.uint64),
    ("mem", np.uint8, (4096,)),
    ("disp", np.uint8, (32, 64)),
    ("hist", np.uint8, (3, 32, 64)),
], align=True)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, no SIMD intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [i32, i32] + [P] * 11 + [i32, i32]
        L.oracle_destroy.argtypes = [P]
        L.oracle_reset.argtypes = [P, P, P]
        L.oracle_step.argtypes = [P, P, P, P, P]
        L.oracle_run_threaded.argtypes = [P, i32, P, P, P, P, i32]
        L.oracle_run_threaded.restype = i32
        L.oracle_get_state.argtypes = [P, i32, i32, P]
        L.oracle_set_state.argtypes = [P, i32, i32, P]
        L.oracle_state_size.restype = i32
        L.oracle_machine_new.restype = P
        L.oracle_machine_free.argtypes = [P]
        L.oracle_machine_set_quirks.argtypes = [P, ctypes.c_uint32]
        L.oracle_machine_load.argtypes = [P, P, ctypes.c_uint32]
        L.oracle_machine_execute.argtypes = [P, i32]
        L.oracle_machine_tick.argtypes = [P]
        L.oracle_machine_to_state.argtypes = [P, P]
        L.oracle_machine_from_state.argtypes = [P, P]
        L.oracle_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_splitmix64_next.restype = ctypes.c_uint64
        L.oracle_execute_batch.argtypes = [ctypes.c_uint16, i32, i32] + [P] * 7
        L.oracle_execute_states.argtypes = [P, i32, i32, i32]
        L.oracle_set_wrappers.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P]
        L.oracle_set_wrappers.restype = i32
        L.oracle_set_profile.argtypes = [P, ctypes.c_uint32, P, P, P, P, P, P]
        L.oracle_set_profile.restype = i32
        L.oracle_set_platform.argtypes = [P, i32]
        L.oracle_set_platform.restype = i32
        L.oracle_set_exec_profile.argtypes = [P, P, P]
        L.oracle_set_exec_profile.restype = i32
        L.oracle_get_schip.argtypes = [P, i32, i32, P]
        L.oracle_machine_set_platform.argtypes = [P, i32]
        L.oracle_machine_set_platform.restype = i32
        L.oracle_machine_get_schip.argtypes = [P, P]
        L.oracle_machine_get_schip.restype = i32
        L.oracle_machine_set_schip.argtypes = [P, P]
        L.oracle_machine_set_schip.restype = i32
        L.oracle_schip_view_size.restype = i32
        assert L.oracle_schip_view_size() == SCHIP_DTYPE.itemsize, "oracle_schip_view layout mismatch"
        assert L.oracle_state_size() == STATE_DTYPE.itemsize, "oracle_state layout mismatch"
        _lib = L
    return _lib


# SUPER-CHIP view of one env or machine: mode, flag registers, 128x64
# display hd[y][x] and, for an env, its three previous frames.
SCHIP_DTYPE = np.dtype([
    ("hires", np.uint8), ("rpl", np.uint8, (8,)), ("hd", np.uint8, (64, 128)), ("hist", np.uint8, (3, 64, 128)),
])


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def splitmix64(seed: int, count: int) -> list:
    s = ctypes.c_uint64(seed)
    return [int(lib().oracle_splitmix64_next(ctypes.byref(s))) for _ in range(count)]


def execute_batch(op: int, v: np.ndarray, i: Optional[np.ndarray] = None, key: int = -1,
                  rng: Optional[np.ndarray] = None, want_mem: bool = False):
    """Run opcode `op` once from each register file in v [count,16]; returns (v, i, pc, mem)."""
    v = np.ascontiguousarray(v, dtype=np.uint8)
    n = v.shape[0]
    i_in = None if i is None else np.ascontiguousarray(i, dtype=np.uint16)
    r_in = None if rng is None else np.ascontiguousarray(rng, dtype=np.uint64)
    v_out = np.zeros_like(v)
    i_out = np.zeros(n, dtype=np.uint16)
    pc_out = np.zeros(n, dtype=np.uint16)
    mem = np.zeros((n, 4096), dtype=np.uint8) if want_mem else None
    lib().oracle_execute_batch(op, key, n, _p(v), _p(i_in), _p(r_in), _p(v_out), _p(i_out),
                               _p(pc_out), _p(mem))
    return v_out, i_out, pc_out, mem


def execute_states(states: np.ndarray, n_instr: int = 1, key: int = -1) -> np.ndarray:
    """Run n_instr instructions (no timer ticks) from each snapshot; returns new snapshots."""
    s = np.array(states, dtype=STATE_DTYPE, copy=True)
    lib().oracle_execute_states(_p(s), len(s), int(key), int(n_instr))
    return s


def blank_state(rom: bytes = b"") -> np.ndarray:
    """Snapshot of a freshly loaded machine (font at 0x50, program at 0x200)."""
    m = Machine(rom)
    return m.state()


class Machine:
    """One bare CHIP-8 (or SUPER-CHIP) machine: load, execute single
    instructions, tick timers."""

    def __init__(self, rom: bytes = b"", quirks: int = 1, schip: bool = False):
        self._h = lib().oracle_machine_new()
        lib().oracle_machine_set_quirks(self._h, int(quirks))
        if schip and lib().oracle_machine_set_platform(self._h, 1) != 0:
            raise MemoryError("oracle_machine_set_platform")
        self.load(rom)

    def schip(self) -> np.ndarray:
        """SUPER-CHIP view (hires, rpl, hd); raises for a CHIP-8 machine."""
        v = np.zeros(1, dtype=SCHIP_DTYPE)
        if lib().oracle_machine_get_schip(self._h, _p(v)) != 0:
            raise ValueError("not a SUPER-CHIP machine")
        return v[0]

    def set_schip(self, view: np.ndarray):
        a = np.array([view], dtype=SCHIP_DTYPE)
        if lib().oracle_machine_set_schip(self._h, _p(a)) != 0:
            raise ValueError("not a SUPER-CHIP machine")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle_machine_free(self._h)
            self._h = None

    def load(self, rom: bytes):
        buf = np.frombuffer(bytes(rom) or b"\0", dtype=np.uint8).copy()
        lib().oracle_machine_load(self._h, _p(buf), len(rom))

    def execute(self, n: int = 1, key: int = -1):
        for _ in range(n):
            lib().oracle_machine_execute(self._h, int(key))

    def tick(self, n: int = 1):
        for _ in range(n):
            lib().oracle_machine_tick(self._h)

    def state(self) -> np.ndarray:
        s = np.zeros(1, dtype=STATE_DTYPE)
        lib().oracle_machine_to_state(self._h, _p(s))
        return s[0]

    def set_state(self, s: np.ndarray):
        a = np.array([s], dtype=STATE_DTYPE)
        lib().oracle_machine_from_state(self._h, _p(a))

    def poke(self, **fields):
        s = self.state()
        for k, v in fields.items():
            s[k] = v
        self.set_state(s)


class OracleBatch:
    """The oracle environment batch, built from a ``workload.EnvSpec``."""

    def __init__(self, spec):
        self.spec = spec
        roms = spec.roms
        data = np.frombuffer(b"".join(roms) or b"\0", dtype=np.uint8).copy()
        lens = np.array([len(r) for r in roms], dtype=np.uint32)
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint32)
        self._keep = dict(
            data=data, lens=lens, offs=offs,
            env_rom=np.ascontiguousarray(spec.env_rom, dtype=np.uint16),
            akeys=np.ascontiguousarray(spec.action_keys, dtype=np.uint8),
            nact=np.ascontiguousarray(spec.num_actions, dtype=np.uint8),
            sreg=np.ascontiguousarray(spec.score_reg, dtype=np.uint8),
            treg=np.ascontiguousarray(spec.term_reg, dtype=np.uint8),
            tval=np.ascontiguousarray(spec.term_value, dtype=np.uint8),
            hor=np.ascontiguousarray(spec.horizon, dtype=np.uint32),
            seed=np.ascontiguousarray(spec.env_seed, dtype=np.uint64))
        k = self._keep
        self.E = int(spec.num_envs)
        h = lib().oracle_create(self.E, len(roms), _p(data), _p(offs), _p(lens), _p(k["env_rom"]),
                                _p(k["akeys"]), _p(k["nact"]), _p(k["sreg"]), _p(k["treg"]),
                                _p(k["tval"]), _p(k["hor"]), _p(k["seed"]),
                                int(spec.instr_per_frame), int(spec.frame_skip))
        if not h:
            raise ValueError("oracle_create rejected the spec")
        self._h = h
        # quirk flags, game descriptors and wrappers act from the next reset
        # on: configure, then reset all
        u8 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.uint8)
        if getattr(spec, "has_profile", False):
            arrs = [u8(spec.score_mode), u8(spec.score_arg), u8(spec.term_op),
                    u8(spec.term2_op), u8(spec.term2_reg), u8(spec.term2_value)]
            self._keep["profile"] = arrs
            if lib().oracle_set_profile(h, int(spec.quirks), *[_p(a) for a in arrs]) != 0:
                raise ValueError("oracle_set_profile rejected the spec")
        if getattr(spec, "has_wrappers", False):
            sl, sk = u8(spec.startup_len), u8(spec.startup_keys)
            self._keep.update(startup_len=sl, startup_keys=sk)
            rc = lib().oracle_set_wrappers(h, int(spec.sticky_q24), int(spec.noop_max), _p(sl), _p(sk))
            if rc != 0:
                raise ValueError("oracle_set_wrappers rejected the spec")
        self.schip = int(getattr(spec, "platform", 0)) == 1
        if self.schip and lib().oracle_set_platform(h, 1) != 0:
            raise MemoryError("oracle_set_platform")
        self.obs_shape = (4, 128, 64) if self.schip else (4, 64, 32)
        if getattr(spec, "has_profile", False) or getattr(spec, "has_wrappers", False) or self.schip:
            lib().oracle_reset(h, None, None)

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    __del__ = close

    def reset(self, mask: Optional[np.ndarray] = None, want_obs: bool = True):
        obs = np.zeros((self.E,) + self.obs_shape, dtype=np.uint8) if want_obs else None
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        lib().oracle_reset(self._h, _p(m), _p(obs))
        return obs

    def step(self, actions: np.ndarray, want_obs: bool = True):
        a = np.ascontiguousarray(actions, dtype=np.int32)
        assert a.shape == (self.E,)
        obs = np.zeros((self.E,) + self.obs_shape, dtype=np.uint8) if want_obs else None
        rew = np.zeros(self.E, dtype=np.float32)
        done = np.zeros(self.E, dtype=np.uint8)
        lib().oracle_step(self._h, _p(a), _p(obs), _p(rew), _p(done))
        return obs, rew, done

    def run_threaded(self, actions: np.ndarray, threads: int):
        """Steps over actions [K][E] on `threads` POSIX threads; returns (reward, done, threads)."""
        a = np.ascontiguousarray(actions, dtype=np.int32)
        K = a.shape[0]
        obs = np.zeros((self.E,) + self.obs_shape, dtype=np.uint8)
        rew = np.zeros((K, self.E), dtype=np.float32)
        done = np.zeros((K, self.E), dtype=np.uint8)
        used = lib().oracle_run_threaded(self._h, K, _p(a), _p(obs), _p(rew), _p(done), threads)
        return rew, done, used

    def profile_execution(self):
        """Count every instruction run from now on: returns (pc_hist [R][4096],
        op_hist [R][65536]) uint32 arrays that the oracle keeps incrementing."""
        R = len(self.spec.roms)
        pc = np.zeros((R, 4096), dtype=np.uint32)
        op = np.zeros((R, 65536), dtype=np.uint32)
        self._keep["exec_profile"] = (pc, op)
        if lib().oracle_set_exec_profile(self._h, _p(pc), _p(op)) != 0:
            raise ValueError("oracle_set_exec_profile")
        return pc, op

    def get_state(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.E - first if count is None else count
        out = np.zeros(count, dtype=STATE_DTYPE)
        lib().oracle_get_state(self._h, first, count, _p(out))
        return out

    def set_state(self, first: int, states: np.ndarray):
        s = np.ascontiguousarray(states, dtype=STATE_DTYPE)
        lib().oracle_set_state(self._h, first, len(s), _p(s))

    def get_schip(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        """SUPER-CHIP views (hires, rpl, display, previous frames) of envs."""
        assert self.schip, "not a SUPER-CHIP batch"
        count = self.E - first if count is None else count
        out = np.zeros(count, dtype=SCHIP_DTYPE)
        lib().oracle_get_schip(self._h, first, count, _p(out))
        return out


def canonical(states: np.ndarray) -> Dict[str, np.ndarray]:
    """Architectural state as a dict of arrays, for comparison with the GPU library."""
    return {
        "v": states["v"].copy(), "i": states["i"].astype(np.uint16), "pc": states["pc"].astype(np.uint16),
        "sp": states["sp"].astype(np.uint8), "dt": states["dt"].copy(), "st": states["st"].copy(),
        "stack": states["stack"].copy(), "t": states["t"].copy(),
        "prev_score": states["prev_score"].copy(), "rng": states["rng"].copy(),
        "prev_key": states["prev_key"].copy(),
        "mem": states["mem"].copy(), "disp": states["disp"].copy(), "hist": states["hist"].copy(),
    }
