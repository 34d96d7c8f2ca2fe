"""CPU checks of the C ABI library: it loads, exports every declared symbol,
and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2510_01764_amd import octax as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(octax_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = X.library()
    declared = _declared()
    assert {"octax_create", "octax_reset", "octax_step", "octax_destroy"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), name
    for name in X.EXPORTED:
        assert name in declared, f"{name} is bound but not declared in include/"


def test_struct_layouts_match_header():
    # sizes computed by a C compiler from the header itself
    import subprocess
    import tempfile
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "octax.h"\n'
           'int main(){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(octax_config), sizeof(octax_env_state),'
           ' offsetof(octax_env_state, ram), offsetof(octax_config, h_rom_data),'
           ' offsetof(octax_config, sticky_q24), offsetof(octax_env_state, prev_key));'
           ' printf("%zu %zu\\n", offsetof(octax_config, h_score_mode), offsetof(octax_config, h_term2_value));'
           ' printf("%zu %zu %zu\\n", offsetof(octax_config, platform), sizeof(octax_schip_state),'
           ' offsetof(octax_schip_state, fb));}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    assert int(out[0]) == ctypes.sizeof(X.octax_config)
    assert int(out[1]) == X.ENV_STATE_DTYPE.itemsize
    assert int(out[2]) == X.ENV_STATE_DTYPE.fields["ram"][1]
    assert int(out[3]) == X.octax_config.h_rom_data.offset
    assert int(out[4]) == X.octax_config.sticky_q24.offset
    assert int(out[6]) == X.octax_config.h_score_mode.offset
    assert int(out[7]) == X.octax_config.h_term2_value.offset
    assert int(out[8]) == X.octax_config.platform.offset
    assert int(out[9]) == X.SCHIP_STATE_DTYPE.itemsize
    assert int(out[10]) == X.SCHIP_STATE_DTYPE.fields["fb"][1]
    assert int(out[5]) == X.ENV_STATE_DTYPE.fields["prev_key"][1]


def _cfg(**over):
    import numpy as np
    keep = dict(rom=np.frombuffer(bytes([0x12, 0x00]), dtype=np.uint8).copy(),
                off=np.zeros(1, np.uint32), ln=np.array([2], np.uint32),
                env_rom=np.zeros(4, np.uint16), keys=np.zeros(16, np.uint8),
                nact=np.array([5], np.uint8), reg=np.array([5], np.uint8),
                hor=np.zeros(4, np.uint32), seed=np.zeros(4, np.uint64))
    c = X.octax_config()
    c.abi_version = X.OCTAX_ABI_VERSION
    c.num_envs, c.num_roms, c.instr_per_frame, c.frame_skip = 4, 1, 10, 4
    c.quirks = X.OCTAX_QUIRKS_V1
    c.h_rom_data, c.h_rom_offset, c.h_rom_len = keep["rom"].ctypes.data, keep["off"].ctypes.data, keep["ln"].ctypes.data
    c.h_env_rom, c.h_action_keys, c.h_num_actions = keep["env_rom"].ctypes.data, keep["keys"].ctypes.data, keep["nact"].ctypes.data
    c.h_score_reg = c.h_term_reg = c.h_term_value = keep["reg"].ctypes.data
    c.h_horizon, c.h_env_seed = keep["hor"].ctypes.data, keep["seed"].ctypes.data
    for k, v in over.items():
        setattr(c, k, v)
    return c, keep


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("abi_version", 2), ("quirks", 2), ("quirks", 0), ("quirks", 1 | (1 << 7)), ("num_envs", 0), ("num_roms", 0), ("instr_per_frame", 0),
    ("frame_skip", 0), ("frame_skip", 65), ("kernel", 7), ("placement", 9), ("envs_per_block", 96),
    ("lanes_per_env", 4), ("h_env_seed", None),
])
def test_create_rejects_bad_config_without_gpu(field, value):
    L = X.library()
    c, keep = _cfg(**{field: value})
    h = ctypes.c_void_p()
    rc = L.octax_create(ctypes.byref(c), ctypes.byref(h))
    assert rc == X.OCTAX_E_INVALID and not h.value
    assert L.octax_last_error().decode()


def test_create_rejects_bad_wrappers_without_gpu():
    import numpy as np
    L = X.library()
    h = ctypes.c_void_p()
    for over in (dict(sticky_q24=(1 << 24) + 1), dict(noop_max=1001)):
        c, keep = _cfg(**over)
        assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID, over
        assert L.octax_last_error().decode()
    lens, keys = np.array([17], np.uint8), np.zeros(16, np.uint8)
    c, keep = _cfg(h_startup_len=lens.ctypes.data, h_startup_keys=keys.ctypes.data)
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    lens[0], keys[0] = 1, 17
    c, keep = _cfg(h_startup_len=lens.ctypes.data, h_startup_keys=keys.ctypes.data)
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    c, keep = _cfg(h_startup_len=lens.ctypes.data)            # keys missing
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    assert not h.value


def test_create_rejects_bad_descriptors_without_gpu():
    import numpy as np
    L = X.library()
    h = ctypes.c_void_p()
    u = lambda v: np.array([v], np.uint8)
    bad = [
        dict(h_score_mode=u(4), h_score_arg=u(0)),                       # no such score mode
        dict(h_score_mode=u(2), h_score_arg=u(16)),                      # negated sum needs a register
        dict(h_score_mode=u(1)),                                         # argument missing
        dict(h_term_op=u(5)),
        dict(h_term2_op=u(1), h_term2_reg=u(3)),                         # constant missing
        dict(h_term2_op=u(5), h_term2_reg=u(3), h_term2_value=u(9)),
        dict(h_term2_op=u(2), h_term2_reg=u(16), h_term2_value=u(9)),
        dict(quirks=1 | (1 << 7)),
    ]
    for over in bad:
        arrs = {k: v for k, v in over.items() if isinstance(v, np.ndarray)}
        fields = {k: (v.ctypes.data if isinstance(v, np.ndarray) else v) for k, v in over.items()}
        c, keep = _cfg(**fields)
        assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID, over
        assert L.octax_last_error().decode(), over
        assert not h.value
        del arrs


def test_create_rejects_bad_platform_combinations_without_gpu():
    import numpy as np
    L = X.library()
    h = ctypes.c_void_p()
    lens, keys = np.array([1], np.uint8), np.zeros(16, np.uint8)
    for over in (dict(platform=2), dict(platform=1, kernel=X.OCTAX_KERNEL_FUSED),
                 dict(platform=1, kernel=X.OCTAX_KERNEL_FUSED, noop_max=3,
                      h_startup_len=lens.ctypes.data, h_startup_keys=keys.ctypes.data)):
        c, keep = _cfg(**over)
        assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID, over
        assert L.octax_last_error().decode(), over
        assert not h.value
    assert L.octax_get_schip_state(None, 0, 0, None) == X.OCTAX_E_INVALID


def test_create_rejects_long_rom_and_bad_rom_index():
    import numpy as np
    L = X.library()
    c, keep = _cfg()
    keep["ln"][0] = 3585
    h = ctypes.c_void_p()
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    c, keep = _cfg()
    keep["env_rom"][2] = 1
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    c, keep = _cfg()
    keep["keys"][0] = 16
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    del np


def test_null_engine_calls_fail_cleanly():
    L = X.library()
    assert L.octax_step(None, None, None, None, None) == X.OCTAX_E_INVALID
    assert L.octax_step_many(None, 1, None, None, 1, None, None) == X.OCTAX_E_INVALID
    assert L.octax_reset(None, None, None) == X.OCTAX_E_INVALID
    assert L.octax_get_state(None, 0, 1, None) == X.OCTAX_E_INVALID
    assert L.octax_set_kernel(None, 0) == X.OCTAX_E_INVALID
    assert L.octax_set_tuning(None, 256, 1) == X.OCTAX_E_INVALID
    assert L.octax_graph_launch(None) == X.OCTAX_E_INVALID
    assert L.octax_destroy(None) == X.OCTAX_OK
    assert L.octax_create(None, None) == X.OCTAX_E_INVALID


def test_pool_config_layout_matches_header():
    import subprocess
    import tempfile
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "octax.h"\n'
           'int main(){printf("%zu %zu %zu\\n", sizeof(octax_pool_config),'
           ' offsetof(octax_pool_config, pool_bytes), offsetof(octax_pool_config, stream));'
           ' printf("%zu\\n", offsetof(octax_pool_config, h_term2_value));}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "p")
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    assert int(out[0]) == ctypes.sizeof(X.octax_pool_config)
    assert int(out[1]) == X.octax_pool_config.pool_bytes.offset
    assert int(out[2]) == X.octax_pool_config.stream.offset
    assert int(out[3]) == X.octax_pool_config.h_term2_value.offset


def _pool_cfg(**over):
    import numpy as np
    keep = dict(rom=np.frombuffer(bytes([0x12, 0x00]), dtype=np.uint8).copy(),
                off=np.zeros(1, np.uint32), ln=np.array([2], np.uint32),
                keys=np.zeros(16, np.uint8), nact=np.array([5], np.uint8), reg=np.array([5], np.uint8))
    c = X.octax_pool_config()
    c.abi_version = X.OCTAX_ABI_VERSION
    c.num_roms, c.instr_per_frame, c.frame_skip, c.quirks = 1, 10, 4, X.OCTAX_QUIRKS_V1
    c.pool_bytes = 64 * X.library().octax_pool_slot_bytes()
    c.h_rom_data, c.h_rom_offset, c.h_rom_len = keep["rom"].ctypes.data, keep["off"].ctypes.data, keep["ln"].ctypes.data
    c.h_action_keys, c.h_num_actions = keep["keys"].ctypes.data, keep["nact"].ctypes.data
    c.h_score_reg = c.h_term_reg = c.h_term_value = keep["reg"].ctypes.data
    for k, v in over.items():
        setattr(c, k, v)
    return c, keep


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("num_roms", 0), ("pool_bytes", 100), ("instr_per_frame", 0),
    ("quirks", 0), ("quirks", 0x81), ("envs_per_block", 100), ("h_num_actions", None),
])
def test_pool_create_rejects_bad_config_without_gpu(field, value):
    L = X.library()
    c, keep = _pool_cfg(**{field: value})
    h = ctypes.c_void_p()
    assert L.octax_pool_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID
    assert not h.value
    assert L.octax_last_error().decode()


def test_null_pool_calls_fail_cleanly():
    L = X.library()
    group = ctypes.c_uint32()
    slots = (ctypes.c_uint32 * 1)()
    assert L.octax_pool_admit(None, 0, 1, None, None, slots, ctypes.byref(group)) == X.OCTAX_E_INVALID
    assert L.octax_pool_retire(None, 0) == X.OCTAX_E_INVALID
    assert L.octax_pool_step(None, 1, None, None, 1, None, None) == X.OCTAX_E_INVALID
    assert L.octax_pool_info(None, None, None, None, None) == X.OCTAX_E_INVALID
    assert L.octax_pool_get_state(None, None, 1, None) == X.OCTAX_E_INVALID
    assert L.octax_pool_destroy(None) == X.OCTAX_OK
    assert L.octax_pool_create(None, None) == X.OCTAX_E_INVALID
    assert L.octax_pool_slot_bytes() == 5470


def test_create_rejects_fused_steps_beyond_the_wait_bound_without_gpu():
    """The fused kernel's paired waves wait for each other once per step with a
    bound derived from the longest step; configs past 2^20 instruction slots per
    step are refused for it (the plain kernel has no such wait)."""
    L = X.library()
    h = ctypes.c_void_p()
    # 1000 x 64 x (1 + 20) = 1,344,000 slots: over the bound
    c, keep = _cfg(kernel=X.OCTAX_KERNEL_FUSED, instr_per_frame=1000, frame_skip=64, noop_max=20)
    assert L.octax_create(ctypes.byref(c), ctypes.byref(h)) == X.OCTAX_E_INVALID and not h.value
    assert "fused kernel" in L.octax_last_error().decode()


def test_status_and_wait_limit_reject_null_without_gpu():
    L = X.library()
    assert L.octax_status(None) == X.OCTAX_E_INVALID
    assert L.octax_set_wait_limit(None, 5) == X.OCTAX_E_INVALID
