"""Python binding of liboctax (the C ABI in include/octax.h).

Argument marshalling only: every step of the environment runs in the HIP
kernels of liboctax.so.  torch supplies device memory and streams.  The
library must be built (``python -m paper_2510_01764_amd.build``); importing
this module on a machine without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liboctax.so")

OCTAX_ABI_VERSION = 4
OCTAX_QUIRKS_V1 = 1
OCTAX_QUIRK_SHIFT_VX = 1 << 1
OCTAX_QUIRK_MEM_KEEP_I = 1 << 2
OCTAX_QUIRK_JUMP_VX = 1 << 3
OCTAX_QUIRK_NO_VF_RESET = 1 << 4
OCTAX_QUIRK_PIXEL_WRAP = 1 << 5
OCTAX_QUIRK_DISPLAY_WAIT = 1 << 6
OCTAX_OK = 0
OCTAX_E_INVALID = -1
OCTAX_E_NOMEM = -2
OCTAX_E_HIP = -3
OCTAX_E_STATE = -4
OCTAX_KERNEL_PLAIN = 0
OCTAX_KERNEL_FUSED = 1
OCTAX_PLATFORM_CHIP8 = 0
OCTAX_PLATFORM_SCHIP = 1
OCTAX_PLACE_IDENTITY = 0
OCTAX_PLACE_BY_ROM = 1
OCTAX_PLACE_BY_HORIZON = 2
OBS_BYTES = 8192
NOALLOC_MAX_ENVS = 64          # octax_get_state_noalloc's largest range

EXPORTED = (
    "octax_create", "octax_reset", "octax_step", "octax_step_many", "octax_graph_create",
    "octax_graph_launch", "octax_graph_destroy", "octax_get_state", "octax_get_state_noalloc", "octax_set_state",
    "octax_set_kernel", "octax_set_tuning", "octax_set_stream", "octax_info", "octax_destroy",
    "octax_status", "octax_set_wait_limit", "octax_set_step_clock",
    "octax_last_error", "octax_calib_write", "octax_calib_copy", "octax_get_schip_state", "octax_digest",
    "octax_pool_slot_bytes", "octax_pool_create", "octax_pool_admit", "octax_pool_retire",
    "octax_pool_step", "octax_pool_step_budget", "octax_pool_info", "octax_pool_get_state", "octax_pool_destroy",
)


class OctaxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"octax error {code}: {msg}")
        self.code = code


class octax_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("num_envs", ctypes.c_uint32),
        ("num_roms", ctypes.c_uint32), ("instr_per_frame", ctypes.c_uint32),
        ("frame_skip", ctypes.c_uint32), ("quirks", ctypes.c_uint32),
        ("kernel", ctypes.c_uint32), ("placement", ctypes.c_uint32),
        ("envs_per_block", ctypes.c_uint32), ("lanes_per_env", ctypes.c_uint32),
        ("rom_in_lds", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
        ("h_rom_data", ctypes.c_void_p), ("h_rom_offset", ctypes.c_void_p),
        ("h_rom_len", ctypes.c_void_p), ("h_env_rom", ctypes.c_void_p),
        ("h_action_keys", ctypes.c_void_p), ("h_num_actions", ctypes.c_void_p),
        ("h_score_reg", ctypes.c_void_p), ("h_term_reg", ctypes.c_void_p),
        ("h_term_value", ctypes.c_void_p), ("h_horizon", ctypes.c_void_p),
        ("h_env_seed", ctypes.c_void_p), ("stream", ctypes.c_void_p),
        ("sticky_q24", ctypes.c_uint32), ("noop_max", ctypes.c_uint32),
        ("h_startup_len", ctypes.c_void_p), ("h_startup_keys", ctypes.c_void_p),
        ("h_score_mode", ctypes.c_void_p), ("h_score_arg", ctypes.c_void_p),
        ("h_term_op", ctypes.c_void_p), ("h_term2_op", ctypes.c_void_p),
        ("h_term2_reg", ctypes.c_void_p), ("h_term2_value", ctypes.c_void_p),
        ("platform", ctypes.c_uint32), ("reserved2", ctypes.c_uint32),
    ]


class octax_pool_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("num_roms", ctypes.c_uint32),
        ("instr_per_frame", ctypes.c_uint32), ("frame_skip", ctypes.c_uint32),
        ("quirks", ctypes.c_uint32), ("envs_per_block", ctypes.c_uint32),
        ("pool_bytes", ctypes.c_uint64),
        ("h_rom_data", ctypes.c_void_p), ("h_rom_offset", ctypes.c_void_p),
        ("h_rom_len", ctypes.c_void_p), ("h_action_keys", ctypes.c_void_p),
        ("h_num_actions", ctypes.c_void_p), ("h_score_reg", ctypes.c_void_p),
        ("h_term_reg", ctypes.c_void_p), ("h_term_value", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("sticky_q24", ctypes.c_uint32), ("noop_max", ctypes.c_uint32),
        ("h_startup_len", ctypes.c_void_p), ("h_startup_keys", ctypes.c_void_p),
        ("h_score_mode", ctypes.c_void_p), ("h_score_arg", ctypes.c_void_p),
        ("h_term_op", ctypes.c_void_p), ("h_term2_op", ctypes.c_void_p),
        ("h_term2_reg", ctypes.c_void_p), ("h_term2_value", ctypes.c_void_p),
    ]


# octax_env_state as a numpy structured dtype (C layout, natural alignment).
ENV_STATE_DTYPE = np.dtype([
    ("v", np.uint8, (16,)), ("i", np.uint16), ("pc", np.uint16), ("sp", np.uint8),
    ("dt", np.uint8), ("st", np.uint8), ("prev_key", np.uint8), ("stack", np.uint16, (16,)),
    ("t", np.uint32), ("prev_score", np.int32), ("rng", np.uint64), ("ram", np.uint8, (4096,)),
    ("fb", np.uint64, (32,)), ("hist", np.uint64, (3, 32)),
], align=True)

# octax_schip_state: the SUPER-CHIP part of one env's state.
SCHIP_STATE_DTYPE = np.dtype([
    ("hires", np.uint32), ("rpl", np.uint8, (8,)), ("reserved", np.uint32),
    ("fb", np.uint64, (64, 2)), ("hist", np.uint64, (3, 64, 2)),
], align=True)

_lib = None


def _set_wrappers(cfg, spec, keep: dict) -> None:
    """The environment-wrapper, quirk and game-descriptor fields of a config
    from a spec (all off when absent)."""
    cfg.sticky_q24 = int(getattr(spec, "sticky_q24", 0))
    cfg.noop_max = int(getattr(spec, "noop_max", 0))
    if getattr(spec, "startup_len", None) is not None:
        keep["startup_len"] = np.ascontiguousarray(spec.startup_len, dtype=np.uint8)
        keep["startup_keys"] = np.ascontiguousarray(spec.startup_keys, dtype=np.uint8)
        cfg.h_startup_len = keep["startup_len"].ctypes.data
        cfg.h_startup_keys = keep["startup_keys"].ctypes.data
    # quirk flags and game descriptors
    cfg.quirks = int(getattr(spec, "quirks", OCTAX_QUIRKS_V1))
    for f in ("score_mode", "score_arg", "term_op", "term2_op", "term2_reg", "term2_value"):
        if getattr(spec, f, None) is not None:
            keep[f] = np.ascontiguousarray(getattr(spec, f), dtype=np.uint8)
            setattr(cfg, "h_" + f, keep[f].ctypes.data)


def library() -> ctypes.CDLL:
    """Load liboctax.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2510_01764_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "octax_create": ([ctypes.POINTER(octax_config), ctypes.POINTER(P)], i32),
        "octax_reset": ([P, P, P], i32),
        "octax_step": ([P, P, P, P, P], i32),
        "octax_step_many": ([P, u32, P, P, u32, P, P], i32),
        "octax_graph_create": ([P, u32, P, P, u32, P, P, ctypes.POINTER(P)], i32),
        "octax_graph_launch": ([P], i32),
        "octax_graph_destroy": ([P], i32),
        "octax_get_state": ([P, u32, u32, P], i32),
        "octax_get_state_noalloc": ([P, u32, u32, P], i32),
        "octax_get_schip_state": ([P, u32, u32, P], i32),
        "octax_digest": ([P, P], i32),
        "octax_set_state": ([P, u32, u32, P], i32),
        "octax_set_kernel": ([P, u32], i32),
        "octax_set_tuning": ([P, u32, u32], i32),
        "octax_set_stream": ([P, P], i32),
        "octax_info": ([P, ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_uint64)], i32),
        "octax_destroy": ([P], i32),
        "octax_status": ([P], i32),
        "octax_set_wait_limit": ([P, ctypes.c_uint64], i32),
        "octax_set_step_clock": ([P, P, u32, ctypes.POINTER(ctypes.c_uint64)], i32),
        "octax_last_error": ([], ctypes.c_char_p),
        "octax_calib_write": ([P, ctypes.c_uint64, u32, u32, P], i32),
        "octax_calib_copy": ([P, P, ctypes.c_uint64, P], i32),
        "octax_pool_slot_bytes": ([], ctypes.c_uint64),
        "octax_pool_create": ([ctypes.POINTER(octax_pool_config), ctypes.POINTER(P)], i32),
        "octax_pool_admit": ([P, u32, u32, P, P, P, ctypes.POINTER(u32)], i32),
        "octax_pool_retire": ([P, u32], i32),
        "octax_pool_step": ([P, u32, P, P, u32, P, P], i32),
        "octax_pool_step_budget": ([P, u32, P, P, P, u32, P, P], i32),
        "octax_pool_info": ([P] + [ctypes.POINTER(u32)] * 4, i32),
        "octax_pool_get_state": ([P, P, u32, P], i32),
        "octax_pool_destroy": ([P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code: int):
    if code != OCTAX_OK:
        raise OctaxError(code, library().octax_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a contiguous torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream)) or None


# ---------------------------------------------------------------------------
# Thin functions with the C names (arguments are torch tensors or None)
# ---------------------------------------------------------------------------

def octax_reset(eng, d_mask=None, d_obs=None):
    _check(library().octax_reset(eng, _ptr(d_mask), _ptr(d_obs)))


def octax_step(eng, d_action, d_obs, d_reward, d_done):
    _check(library().octax_step(eng, _ptr(d_action), _ptr(d_obs), _ptr(d_reward), _ptr(d_done)))


def octax_step_many(eng, K, d_action, d_obs, obs_slots, d_reward, d_done):
    _check(library().octax_step_many(eng, K, _ptr(d_action), _ptr(d_obs), obs_slots,
                                     _ptr(d_reward), _ptr(d_done)))


def octax_destroy(eng):
    _check(library().octax_destroy(eng))


class Engine:
    """One liboctax engine built from a ``workload.EnvSpec``.

    Output buffers are torch tensors on the engine's device: obs uint8
    [E, 4, 64, 32] ([E, 4, 128, 64] for SUPER-CHIP; [slots, E, ...] for K steps), reward float32 [E] ([K, E]),
    done uint8 [E] ([K, E]); actions int32 [E] ([K, E]).
    """

    def __init__(self, spec, kernel: str = "fused", placement: Optional[str] = None,
                 envs_per_block: int = 256, rom_in_lds: bool = True, stream=None):
        import torch  # noqa: F401  (device memory for the caller's buffers)
        L = library()
        self.spec = spec
        self.E = int(spec.num_envs)
        roms = spec.roms
        data = np.frombuffer(b"".join(roms) or b"\0", dtype=np.uint8).copy()
        lens = np.array([len(r) for r in roms], dtype=np.uint32)
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint32)
        keep = dict(
            data=data, lens=lens, offs=offs,
            env_rom=np.ascontiguousarray(spec.env_rom, dtype=np.uint16),
            akeys=np.ascontiguousarray(spec.action_keys, dtype=np.uint8),
            nact=np.ascontiguousarray(spec.num_actions, dtype=np.uint8),
            sreg=np.ascontiguousarray(spec.score_reg, dtype=np.uint8),
            treg=np.ascontiguousarray(spec.term_reg, dtype=np.uint8),
            tval=np.ascontiguousarray(spec.term_value, dtype=np.uint8),
            hor=np.ascontiguousarray(spec.horizon, dtype=np.uint32),
            seed=np.ascontiguousarray(spec.env_seed, dtype=np.uint64))
        if placement is None:
            placement = "by_rom" if kernel == "fused" else "identity"
        cfg = octax_config()
        cfg.abi_version = OCTAX_ABI_VERSION
        cfg.num_envs = self.E
        cfg.num_roms = len(roms)
        cfg.instr_per_frame = int(spec.instr_per_frame)
        cfg.frame_skip = int(spec.frame_skip)
        cfg.quirks = OCTAX_QUIRKS_V1
        cfg.kernel = {"plain": OCTAX_KERNEL_PLAIN, "fused": OCTAX_KERNEL_FUSED}[kernel]
        cfg.placement = {"identity": OCTAX_PLACE_IDENTITY, "by_rom": OCTAX_PLACE_BY_ROM,
                         "by_horizon": OCTAX_PLACE_BY_HORIZON}[placement]
        cfg.envs_per_block = int(envs_per_block)
        cfg.lanes_per_env = 1
        cfg.rom_in_lds = 1 if rom_in_lds else 0
        cfg.h_rom_data = keep["data"].ctypes.data
        cfg.h_rom_offset = keep["offs"].ctypes.data
        cfg.h_rom_len = keep["lens"].ctypes.data
        cfg.h_env_rom = keep["env_rom"].ctypes.data
        cfg.h_action_keys = keep["akeys"].ctypes.data
        cfg.h_num_actions = keep["nact"].ctypes.data
        cfg.h_score_reg = keep["sreg"].ctypes.data
        cfg.h_term_reg = keep["treg"].ctypes.data
        cfg.h_term_value = keep["tval"].ctypes.data
        cfg.h_horizon = keep["hor"].ctypes.data
        cfg.h_env_seed = keep["seed"].ctypes.data
        cfg.stream = _stream_handle(stream)
        _set_wrappers(cfg, spec, keep)
        cfg.platform = int(getattr(spec, "platform", OCTAX_PLATFORM_CHIP8))
        h = ctypes.c_void_p()
        _check(L.octax_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.kernel = kernel
        self.placement = placement
        self.schip = cfg.platform == OCTAX_PLATFORM_SCHIP
        self.obs_shape = (4, 128, 64) if self.schip else (4, 64, 32)

    @property
    def handle(self):
        return self._h

    def status(self):
        """Raise OctaxError (OCTAX_E_STATE) if a fused launch since the last
        check gave up waiting for a partner wave (synchronizes)."""
        _check(library().octax_status(self._h))

    def set_step_clock(self, stamps, steps: int) -> int:
        """Record per-step clocks of fused launches into a device int64 tensor
        [steps, ceil(E / 64), 2] (None switches it off); returns the clock rate in Hz."""
        hz = ctypes.c_uint64(0)
        if stamps is None:
            _check(library().octax_set_step_clock(self._h, None, 0, ctypes.byref(hz)))
        else:
            import torch
            self._need(stamps, torch.int64, (int(steps), (self.E + 63) // 64, 2), "stamps")
            _check(library().octax_set_step_clock(self._h, _ptr(stamps), int(steps), ctypes.byref(hz)))
        return int(hz.value)

    def set_wait_limit(self, ticks: int):
        """Override the fused kernel's wait bound (device wall-clock ticks, 0 = derived)."""
        _check(library().octax_set_wait_limit(self._h, int(ticks)))

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _check(library().octax_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _need(self, t, dtype, shape, name):
        import torch
        if t is None:
            return
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        del torch

    def reset(self, mask=None, obs=None):
        import torch
        self._need(mask, torch.uint8, (self.E,), "mask")
        self._need(obs, torch.uint8, (self.E,) + self.obs_shape, "obs")
        _check(library().octax_reset(self._h, _ptr(mask), _ptr(obs)))

    def step(self, action, obs, reward, done):
        import torch
        self._need(action, torch.int32, (self.E,), "action")
        self._need(obs, torch.uint8, (self.E,) + self.obs_shape, "obs")
        self._need(reward, torch.float32, (self.E,), "reward")
        self._need(done, torch.uint8, (self.E,), "done")
        _check(library().octax_step(self._h, _ptr(action), _ptr(obs), _ptr(reward), _ptr(done)))

    def step_many(self, action, obs, reward, done):
        import torch
        K = int(action.shape[0])
        self._need(action, torch.int32, (K, self.E), "action")
        slots = 0 if obs is None else int(obs.shape[0])
        self._need(obs, torch.uint8, (slots, self.E) + self.obs_shape, "obs")
        self._need(reward, torch.float32, (K, self.E), "reward")
        self._need(done, torch.uint8, (K, self.E), "done")
        _check(library().octax_step_many(self._h, K, _ptr(action), _ptr(obs), slots,
                                         _ptr(reward), _ptr(done)))

    def graph(self, action, obs, reward, done) -> "Graph":
        import torch
        K = int(action.shape[0])
        self._need(action, torch.int32, (K, self.E), "action")
        slots = 0 if obs is None else int(obs.shape[0])
        self._need(obs, torch.uint8, (slots, self.E) + self.obs_shape, "obs")
        self._need(reward, torch.float32, (K, self.E), "reward")
        self._need(done, torch.uint8, (K, self.E), "done")
        g = ctypes.c_void_p()
        _check(library().octax_graph_create(self._h, K, _ptr(action), _ptr(obs), slots,
                                            _ptr(reward), _ptr(done), ctypes.byref(g)))
        return Graph(g, (action, obs, reward, done))

    def get_state(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.E - first if count is None else int(count)
        out = np.zeros(count, dtype=ENV_STATE_DTYPE)
        _check(library().octax_get_state(self._h, first, count, out.ctypes.data))
        return out

    def get_state_noalloc(self, first: int, count: int) -> np.ndarray:
        """get_state through the library's static device array (at most
        NOALLOC_MAX_ENVS envs; no device allocation)."""
        out = np.zeros(int(count), dtype=ENV_STATE_DTYPE)
        _check(library().octax_get_state_noalloc(self._h, int(first), int(count), out.ctypes.data))
        return out

    def set_state(self, first: int, states: np.ndarray):
        s = np.ascontiguousarray(states, dtype=ENV_STATE_DTYPE)
        _check(library().octax_set_state(self._h, first, len(s), s.ctypes.data))

    def digest(self, out):
        """64-bit FNV-1a of every env's state (octax_env_state bytes) into a
        device int64 tensor [E] (the bits of the uint64 digests)."""
        import torch
        self._need(out, torch.int64, (self.E,), "out")
        _check(library().octax_digest(self._h, _ptr(out)))

    def get_schip_state(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        """SUPER-CHIP mode, flag registers, display and previous frames of envs."""
        count = self.E - first if count is None else int(count)
        out = np.zeros(count, dtype=SCHIP_STATE_DTYPE)
        _check(library().octax_get_schip_state(self._h, first, count, out.ctypes.data))
        return out

    def set_kernel(self, kernel: str):
        _check(library().octax_set_kernel(self._h, {"plain": 0, "fused": 1}[kernel]))
        self.kernel = kernel

    def set_tuning(self, envs_per_block: int, rom_in_lds: bool):
        _check(library().octax_set_tuning(self._h, int(envs_per_block), 1 if rom_in_lds else 0))

    def set_stream(self, stream):
        _check(library().octax_set_stream(self._h, _stream_handle(stream)))

    def info(self):
        n = ctypes.c_uint32()
        b = ctypes.c_uint64()
        _check(library().octax_info(self._h, ctypes.byref(n), ctypes.byref(b)))
        return int(n.value), int(b.value)


class Graph:
    """A captured K-step launch over fixed buffers (octax_graph_*)."""

    def __init__(self, handle, buffers):
        self._h = handle
        self._buffers = buffers   # keep the captured buffers alive

    def launch(self):
        _check(library().octax_graph_launch(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _check(library().octax_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """A liboctax serving pool (octax_pool_*) over a set of ROMs.

    ``roms`` and the per-ROM descriptors come from a ``workload.EnvSpec``
    (its env fields are not used).  Step buffers are indexed by slot:
    action int32 [K, capacity], obs uint8 [slots, capacity, 4, 64, 32] or
    None, reward float32 [K, capacity], done uint8 [K, capacity].
    """

    def __init__(self, spec, pool_bytes: int, envs_per_block: int = 256, stream=None):
        L = library()
        roms = spec.roms
        data = np.frombuffer(b"".join(roms) or b"\0", dtype=np.uint8).copy()
        lens = np.array([len(r) for r in roms], dtype=np.uint32)
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint32)
        keep = dict(data=data, lens=lens, offs=offs,
                    akeys=np.ascontiguousarray(spec.action_keys, dtype=np.uint8),
                    nact=np.ascontiguousarray(spec.num_actions, dtype=np.uint8),
                    sreg=np.ascontiguousarray(spec.score_reg, dtype=np.uint8),
                    treg=np.ascontiguousarray(spec.term_reg, dtype=np.uint8),
                    tval=np.ascontiguousarray(spec.term_value, dtype=np.uint8))
        cfg = octax_pool_config()
        cfg.abi_version = OCTAX_ABI_VERSION
        cfg.num_roms = len(roms)
        cfg.instr_per_frame = int(spec.instr_per_frame)
        cfg.frame_skip = int(spec.frame_skip)
        cfg.quirks = OCTAX_QUIRKS_V1
        cfg.envs_per_block = int(envs_per_block)
        cfg.pool_bytes = int(pool_bytes)
        cfg.h_rom_data = keep["data"].ctypes.data
        cfg.h_rom_offset = keep["offs"].ctypes.data
        cfg.h_rom_len = keep["lens"].ctypes.data
        cfg.h_action_keys = keep["akeys"].ctypes.data
        cfg.h_num_actions = keep["nact"].ctypes.data
        cfg.h_score_reg = keep["sreg"].ctypes.data
        cfg.h_term_reg = keep["treg"].ctypes.data
        cfg.h_term_value = keep["tval"].ctypes.data
        cfg.stream = _stream_handle(stream)
        _set_wrappers(cfg, spec, keep)
        self._keep = keep
        h = ctypes.c_void_p()
        _check(L.octax_pool_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.spec = spec
        self.capacity = self.info()["capacity"]

    @staticmethod
    def slot_bytes() -> int:
        return int(library().octax_pool_slot_bytes())

    def admit(self, rom: int, env_seed: np.ndarray, horizon: np.ndarray):
        """(group id, slots of its envs as uint32 [count]) of the admitted
        group, or None when fewer slots are free."""
        seeds = np.ascontiguousarray(env_seed, dtype=np.uint64)
        hor = np.ascontiguousarray(horizon, dtype=np.uint32)
        if seeds.shape != hor.shape or seeds.ndim != 1:
            raise ValueError("env_seed and horizon must be 1-D of the same length")
        slots = np.zeros(len(seeds), dtype=np.uint32)
        group = ctypes.c_uint32()
        code = library().octax_pool_admit(self._h, int(rom), len(seeds), seeds.ctypes.data,
                                          hor.ctypes.data, slots.ctypes.data, ctypes.byref(group))
        if code == OCTAX_E_NOMEM:
            return None
        _check(code)
        return int(group.value), slots

    def retire(self, group: int):
        _check(library().octax_pool_retire(self._h, int(group)))

    def step(self, action, obs, reward, done, budget=None):
        """K = action.shape[0] steps of every occupied slot; with budget (a
        device uint8 tensor [capacity]) slot s runs min(K, budget[s]) of them."""
        K = int(action.shape[0])
        slots = 0 if obs is None else int(obs.shape[0])
        if budget is None:
            _check(library().octax_pool_step(self._h, K, _ptr(action), _ptr(obs), slots,
                                             _ptr(reward), _ptr(done)))
            return
        import torch
        if budget.dtype != torch.uint8 or tuple(budget.shape) != (self.capacity,) or not budget.is_contiguous():
            raise ValueError(f"budget must be a contiguous uint8 tensor of shape ({self.capacity},)")
        _check(library().octax_pool_step_budget(self._h, K, _ptr(budget), _ptr(action), _ptr(obs), slots,
                                                _ptr(reward), _ptr(done)))

    def info(self) -> dict:
        v = [ctypes.c_uint32() for _ in range(4)]
        _check(library().octax_pool_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("capacity", "free", "largest_free", "groups"), (int(x.value) for x in v)))

    def get_state(self, slots) -> np.ndarray:
        sl = np.ascontiguousarray(slots, dtype=np.uint32)
        out = np.zeros(len(sl), dtype=ENV_STATE_DTYPE)
        _check(library().octax_pool_get_state(self._h, sl.ctypes.data, len(sl), out.ctypes.data))
        return out

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _check(library().octax_pool_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def canonical(states: np.ndarray) -> dict:
    """Architectural state in the oracle's comparison format (pixels unpacked)."""
    def unpack_rows(rows):
        bits = ((rows[..., None] >> np.arange(63, -1, -1, dtype=np.uint64)) & np.uint64(1))
        return bits.astype(np.uint8)  # [..., 32, 64] = [y][x]
    return {
        "v": states["v"].copy(), "i": states["i"].astype(np.uint16), "pc": states["pc"].astype(np.uint16),
        "sp": states["sp"].astype(np.uint8), "dt": states["dt"].copy(), "st": states["st"].copy(),
        "stack": states["stack"].copy(), "t": states["t"].copy(),
        "prev_score": states["prev_score"].copy(), "rng": states["rng"].copy(),
        "prev_key": states["prev_key"].copy(),
        "mem": states["ram"].copy(), "disp": unpack_rows(states["fb"]),
        "hist": unpack_rows(states["hist"]),
    }
