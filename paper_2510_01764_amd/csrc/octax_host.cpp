// Host side of the liboctax C ABI (declared in include/octax.h).
//
// Device memory per env (E envs):
//   regs 16 B, pc_i 4, misc 4, t 4, prev 4, rng 8, dirty 8, stack 32,
//   display 256, frame ring 1024, memory 4096, rom/horizon/env maps 12
//   = 5,468 B per env, plus the power-on images (4 KB per ROM).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "octax_engine.h"

using namespace octax;

namespace {

thread_local std::string g_last_error;

// The 4x5 hexadecimal font of the machine, glyphs 0..F (Appendix B.4 places
// it at 0x050-0x09F).
const uint8_t kFontBytes[80] = {
    0xF0, 0x90, 0x90, 0x90, 0xF0, 0x20, 0x60, 0x20, 0x20, 0x70, 0xF0, 0x10, 0xF0, 0x80, 0xF0,
    0xF0, 0x10, 0xF0, 0x10, 0xF0, 0x90, 0x90, 0xF0, 0x10, 0x10, 0xF0, 0x80, 0xF0, 0x10, 0xF0,
    0xF0, 0x80, 0xF0, 0x90, 0xF0, 0xF0, 0x10, 0x20, 0x40, 0x40, 0xF0, 0x90, 0xF0, 0x90, 0xF0,
    0xF0, 0x90, 0xF0, 0x10, 0xF0, 0xF0, 0x90, 0xF0, 0x90, 0x90, 0xE0, 0x90, 0xE0, 0x90, 0xE0,
    0xF0, 0x80, 0x80, 0x80, 0xF0, 0xE0, 0x90, 0x90, 0x90, 0xE0, 0xF0, 0x80, 0xF0, 0x80, 0xF0,
    0xF0, 0x80, 0xF0, 0x80, 0x80,
};

// The SUPER-CHIP 8x10 digit glyphs 0..F of FX30, at 0x0A0 (ten rows per
// glyph, bit 7 = leftmost pixel; the glyph shapes are this library's own).
const uint8_t kBigFontBytes[160] = {
    0x3C, 0x66, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0x66, 0x3C,   // 0
    0x18, 0x38, 0x78, 0x18, 0x18, 0x18, 0x18, 0x18, 0x18, 0x7E,   // 1
    0x7E, 0xC3, 0x03, 0x03, 0x06, 0x1C, 0x30, 0x60, 0xC0, 0xFF,   // 2
    0x7E, 0xC3, 0x03, 0x03, 0x3E, 0x03, 0x03, 0x03, 0xC3, 0x7E,   // 3
    0x06, 0x0E, 0x1E, 0x36, 0x66, 0xC6, 0xFF, 0x06, 0x06, 0x06,   // 4
    0xFF, 0xC0, 0xC0, 0xC0, 0xFE, 0x03, 0x03, 0x03, 0xC3, 0x7E,   // 5
    0x3E, 0x60, 0xC0, 0xC0, 0xFE, 0xC3, 0xC3, 0xC3, 0xC3, 0x7E,   // 6
    0xFF, 0x03, 0x06, 0x0C, 0x18, 0x30, 0x30, 0x30, 0x30, 0x30,   // 7
    0x7E, 0xC3, 0xC3, 0xC3, 0x7E, 0xC3, 0xC3, 0xC3, 0xC3, 0x7E,   // 8
    0x7E, 0xC3, 0xC3, 0xC3, 0xC3, 0x7F, 0x03, 0x03, 0x06, 0x7C,   // 9
    0x3C, 0x66, 0xC3, 0xC3, 0xC3, 0xFF, 0xC3, 0xC3, 0xC3, 0xC3,   // A
    0xFE, 0xC3, 0xC3, 0xC3, 0xFE, 0xC3, 0xC3, 0xC3, 0xC3, 0xFE,   // B
    0x7E, 0xC3, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0xC3, 0x7E,   // C
    0xFC, 0xC6, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC6, 0xFC,   // D
    0xFF, 0xC0, 0xC0, 0xC0, 0xFC, 0xC0, 0xC0, 0xC0, 0xC0, 0xFF,   // E
    0xFF, 0xC0, 0xC0, 0xC0, 0xFC, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0,   // F
};

}  // namespace

int32_t octax::fail(int32_t code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int32_t octax::hip_fail(hipError_t e, const char *what) {
    return fail(OCTAX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const char *octax::check_wrappers(uint32_t sticky_q24, uint32_t noop_max, const uint8_t *h_startup_len,
                                  const uint8_t *h_startup_keys, uint32_t R, std::vector<uint8_t> &table) {
    if (sticky_q24 > (1u << 24)) return "sticky_q24 > 2^24";
    if (noop_max > 1000) return "noop_max > 1000";
    if (!h_startup_len != !h_startup_keys) return "h_startup_len and h_startup_keys must both be given or both NULL";
    table.assign(17 * (size_t)R, 0);
    if (!h_startup_len) return nullptr;
    for (uint32_t r = 0; r < R; r++) {
        if (h_startup_len[r] > 16) return "start-up sequence longer than 16 steps";
        table[17 * (size_t)r] = h_startup_len[r];
        for (uint32_t i = 0; i < 16; i++) {
            const uint8_t k = h_startup_keys[16 * (size_t)r + i];
            if (i < h_startup_len[r] && k > 16) return "start-up key > 16";
            table[17 * (size_t)r + 1 + i] = k > 16 ? 16 : k;
        }
    }
    return nullptr;
}

const char *octax::check_profile(const octax_config *cfg, std::vector<uint32_t> &desc2) {
    const uint32_t R = cfg->num_roms;
    if (!(cfg->quirks & OCTAX_QUIRKS_V1)) return "quirks must include OCTAX_QUIRKS_V1";
    if (cfg->quirks & ~0x7Fu) return "unknown quirk flag";
    if (!cfg->h_score_mode != !cfg->h_score_arg) return "h_score_mode and h_score_arg must be given together";
    const bool t2 = cfg->h_term2_op || cfg->h_term2_reg || cfg->h_term2_value;
    if (t2 && !(cfg->h_term2_op && cfg->h_term2_reg && cfg->h_term2_value))
        return "h_term2_op, h_term2_reg and h_term2_value must be given together";
    desc2.clear();
    if (!cfg->h_score_mode && !cfg->h_term_op && !t2) return nullptr;
    desc2.assign(R, 0);
    for (uint32_t r = 0; r < R; r++) {
        uint32_t mode = 0, arg = 0, op1 = 1, op2 = 0, reg2 = 0, val2 = 0;
        if (cfg->h_score_mode) {
            mode = cfg->h_score_mode[r];
            arg = cfg->h_score_arg[r];
            if (mode > 3) return "score mode > 3";
            if (mode == 2 && arg > 15) return "score mode 2 needs a register index 0..15 in h_score_arg";
        }
        if (cfg->h_term_op) {
            op1 = cfg->h_term_op[r];
            if (op1 > 4) return "termination op > 4";
        }
        if (t2) {
            op2 = cfg->h_term2_op[r];
            reg2 = cfg->h_term2_reg[r];
            val2 = cfg->h_term2_value[r];
            if (op2 > 4) return "term2 op > 4";
            if (reg2 > 15) return "term2 register index > 15";
        }
        desc2[r] = mode | (arg << 2) | (op1 << 10) | (op2 << 13) | (reg2 << 16) | (val2 << 24);
    }
    return nullptr;
}

octax::Wrap octax::make_wrap(const uint8_t *d_table, const std::vector<uint8_t> &table, uint32_t sticky_q24,
                             uint32_t noop_max, uint32_t ipf, uint32_t frame_skip) {
    Wrap w{};
    bool any_startup = false;
    for (size_t r = 0; r < table.size(); r += 17) any_startup = any_startup || table[r] > 0;
    w.startup = any_startup ? d_table : nullptr;
    w.sticky_q24 = sticky_q24;
    w.noop_max = noop_max;
    w.reset_steps = (any_startup || noop_max) ? 1u : 0u;
    w.ipf = ipf;
    w.frame_skip = frame_skip;
    return w;
}

void octax::block_rom_table(const octax_engine *g, std::vector<uint32_t> &table) {
    const uint32_t ipw = g->envs_per_block;
    const uint32_t blocks = (g->E + ipw - 1) / ipw;
    const uint32_t capacity = fused_pool_pages(ipw) - kPoolFixedPages;
    table.assign(2 * (size_t)kPoolRoms * blocks, kPoolEnd);
    std::vector<uint32_t> count(g->R, 0);
    std::vector<uint32_t> seen;
    for (uint32_t b = 0; b < blocks; b++) {
        const uint32_t lo = b * ipw, hi = std::min(g->E, lo + ipw);
        seen.clear();
        for (uint32_t sl = lo; sl < hi; sl++) {
            if (!g->occupied.empty() && !g->occupied[sl]) continue;
            const uint32_t r = g->rom_of[sl];
            if (count[r]++ == 0) seen.push_back(r);
        }
        std::sort(seen.begin(), seen.end(), [&](uint32_t a, uint32_t c) {
            return count[a] != count[c] ? count[a] > count[c] : a < c;
        });
        uint32_t used = 0;
        uint32_t *row = table.data() + 2 * (size_t)kPoolRoms * b;
        for (uint32_t k = 0; k < seen.size() && k < kPoolRoms; k++) {
            const uint32_t r = seen[k];
            const uint32_t pages = (g->rom_len[r] + 63) / 64;
            const uint32_t staged = std::min(pages, capacity - used);
            row[2 * k] = r;
            row[2 * k + 1] = staged | (pages << 8) | ((kPoolFixedPages + used) << 16);
            used += staged;
        }
        for (uint32_t r : seen) count[r] = 0;
    }
}

namespace {

hipError_t upload_block_roms(octax_engine *g) {
    std::vector<uint32_t> table;
    block_rom_table(g, table);
    if (g->d_block_roms) {
        (void)hipFree(g->d_block_roms);
        g->allocations.erase(std::find(g->allocations.begin(), g->allocations.end(),
                                       static_cast<void *>(g->d_block_roms)));
        g->d_block_roms = nullptr;
    }
    hipError_t e = g->alloc(&g->d_block_roms, table.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(g->d_block_roms, table.data(), table.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice);
}

}  // namespace

hipError_t octax::launch_steps(octax_engine *g, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                               uint32_t obs_slots, float *d_reward, uint8_t *d_done, hipStream_t st,
                               const uint8_t *d_budget) {
    StepIO io{d_action, d_obs, d_reward, d_done, K, obs_slots ? obs_slots : 1, g->ipf, g->frame_skip};
    if (g->schip) return launch_step_schip(g->s, g->roms, io, st);
    if (g->kernel == OCTAX_KERNEL_FUSED) {
        FusedCfg f{g->envs_per_block, g->rom_in_lds, g->d_block_roms,
                   g->wait_override ? g->wait_override : g->wait_ticks, g->d_err, g->d_stamps, g->stamp_steps,
                   d_budget};
        return launch_step_fused(g->s, g->roms, io, f, st);
    }
    return launch_step_plain(g->s, g->roms, io, st);
}

uint64_t octax::fused_wait_ticks(uint64_t slots, uint64_t wall_khz) {
    const uint64_t us = 250000 + 16 * slots;
    return us * wall_khz / 1000;
}

int32_t octax::check_device_error(octax_engine *g, const char *what) {
    hipError_t e = hipStreamSynchronize(g->stream);
    uint32_t word = 0;
    if (e == hipSuccess) e = hipMemcpy(&word, g->d_err, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && word) {
        const uint32_t zero = 0;
        e = hipMemcpy(g->d_err, &zero, 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            return fail(OCTAX_E_STATE, std::string(what) + ": a fused launch gave up waiting for a partner wave; "
                                                           "the observations, rewards and done flags it wrote are not valid");
    }
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, what);
}

namespace {

hipError_t ensure_raw(octax_engine *g, uint32_t count) {
    if (count <= g->raw_capacity) return hipSuccess;
    for (void *p : {static_cast<void *>(g->d_raw), static_cast<void *>(g->d_slot_scratch)}) {
        if (p) {
            (void)hipFree(p);
            g->allocations.erase(std::find(g->allocations.begin(), g->allocations.end(), p));
        }
    }
    g->d_raw = nullptr;
    g->d_slot_scratch = nullptr;
    g->raw_capacity = 0;
    hipError_t e = g->alloc(&g->d_raw, count);
    if (e != hipSuccess) return e;
    e = g->alloc(&g->d_slot_scratch, count);
    if (e != hipSuccess) return e;
    g->raw_capacity = count;
    return hipSuccess;
}

// Packed frame layout of the frame ring (observation store order): pixel
// (x, y) is byte 32x + y of the frame's observation; word l covers bytes
// [16l, 16l + 16) in its low half and [1024 + 16l, ...) in its high half.
int packed_word(int x, int y) { return 2 * (x & 31) + (y >> 4); }
int packed_bit(int x, int y) { return (x >= 32 ? 16 : 0) + (y & 15); }
uint32_t packed_pixel(const uint32_t *frame, int x, int y) {
    return (frame[packed_word(x, y)] >> packed_bit(x, y)) & 1;
}

void raw_to_canonical(const RawState &r, octax_env_state &o) {
    std::memset(&o, 0, sizeof o);
    for (int k = 0; k < 16; k++) o.v[k] = (uint8_t)(r.regs[k >> 2] >> (8 * (k & 3)));
    o.pc = (uint16_t)(r.pc_i & 0xFFF);
    o.i = (uint16_t)((r.pc_i >> 16) & 0xFFF);
    o.sp = (uint8_t)(r.misc & 15);
    o.dt = (uint8_t)(r.misc >> 8);
    o.st = (uint8_t)(r.misc >> 16);
    const uint32_t head = (r.misc >> 24) & 3;
    o.prev_key = (uint8_t)(((r.misc >> 26) & 31) ^ 16);
    for (int k = 0; k < 16; k++) o.stack[k] = (uint16_t)((r.stack[k >> 1] >> (16 * (k & 1))) & 0xFFFF);
    o.t = r.t;
    o.prev_score = r.prev;
    o.rng = r.rng;
    std::memcpy(o.ram, r.ram, 4096);
    std::memcpy(o.fb, r.fb, sizeof o.fb);
    for (int h = 0; h < 3; h++) {
        const uint32_t *frame = r.cols + ((head + 1 + h) & 3) * 64;
        for (int y = 0; y < 32; y++) {
            uint64_t row = 0;
            for (int x = 0; x < 64; x++) row |= (uint64_t)packed_pixel(frame, x, y) << (63 - x);
            o.hist[h][y] = row;
        }
    }
}

void canonical_to_raw(const octax_env_state &o, RawState &r) {
    std::memset(&r, 0, sizeof r);
    for (int k = 0; k < 16; k++) r.regs[k >> 2] |= (uint32_t)o.v[k] << (8 * (k & 3));
    r.pc_i = (o.pc & 0xFFFu) | ((uint32_t)(o.i & 0xFFFu) << 16);
    const uint32_t head = 3;
    r.misc = (o.sp & 15u) | ((uint32_t)o.dt << 8) | ((uint32_t)o.st << 16) | (head << 24) |
             (((o.prev_key < 16 ? o.prev_key : 16u) ^ 16u) << 26);
    for (int k = 0; k < 16; k++) r.stack[k >> 1] |= (uint32_t)(o.stack[k] & 0xFFFu) << (16 * (k & 1));
    r.t = o.t;
    r.prev = o.prev_score;
    r.rng = o.rng;
    r.dirty = ~0ull;   // every page is taken from ram; a later reset restores all of them
    std::memcpy(r.ram, o.ram, 4096);
    std::memcpy(r.fb, o.fb, sizeof r.fb);
    const uint64_t *frames[4] = {o.hist[0], o.hist[1], o.hist[2], o.fb};
    for (int h = 0; h < 4; h++) {
        uint32_t *frame = r.cols + h * 64;   // ring slots 0..3 with head = 3
        for (int y = 0; y < 32; y++)
            for (int x = 0; x < 64; x++)
                if ((frames[h][y] >> (63 - x)) & 1) frame[packed_word(x, y)] |= 1u << packed_bit(x, y);
    }
}

}  // namespace

namespace {

// Device memory of octax_get_state_noalloc: the slot list (first 256 bytes)
// and the gathered records, one copy per GPU for the life of the process.
// Host code never names `scratch` in a device context: it uses the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocSlotBytes = 256;
constexpr size_t kNoAllocBytes = kNoAllocSlotBytes + sizeof(RawState) * OCTAX_NOALLOC_MAX_ENVS;
static_assert(OCTAX_NOALLOC_MAX_ENVS * sizeof(uint32_t) <= kNoAllocSlotBytes, "slot list fits its part");
static_assert(kNoAllocSlotBytes % alignof(RawState) == 0, "records stay aligned");
static_assert(sizeof(RawState) == 5456, "the record size octax.h states");
__device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Address of this GPU's scratch array, looked up once per device with that
// device current.
hipError_t scratch_of(int device, uint8_t **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *octax_last_error(void) { return g_last_error.c_str(); }

int32_t octax_create(const octax_config *cfg, octax_engine **out) {
    if (!out) return fail(OCTAX_E_INVALID, "octax_create: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(OCTAX_E_INVALID, "octax_create: cfg is NULL");
    if (cfg->abi_version != OCTAX_ABI_VERSION) return fail(OCTAX_E_INVALID, "octax_create: abi_version mismatch");
    const uint32_t E = cfg->num_envs, R = cfg->num_roms;
    if (E == 0 || E > (1u << 26)) return fail(OCTAX_E_INVALID, "octax_create: num_envs out of range");
    if (R == 0 || R > 65535) return fail(OCTAX_E_INVALID, "octax_create: num_roms out of range");
    if (cfg->instr_per_frame == 0 || cfg->instr_per_frame > 1000)
        return fail(OCTAX_E_INVALID, "octax_create: instr_per_frame out of range");
    if (cfg->frame_skip == 0 || cfg->frame_skip > 64) return fail(OCTAX_E_INVALID, "octax_create: frame_skip out of range");
    if (cfg->kernel > OCTAX_KERNEL_FUSED) return fail(OCTAX_E_INVALID, "octax_create: unknown kernel");
    if (cfg->placement > OCTAX_PLACE_BY_HORIZON) return fail(OCTAX_E_INVALID, "octax_create: unknown placement");
    if (cfg->lanes_per_env > 1) return fail(OCTAX_E_INVALID, "octax_create: lanes_per_env must be 0 or 1");
    const uint32_t ipw = cfg->envs_per_block ? cfg->envs_per_block : 256;
    if (ipw != 64 && ipw != 128 && ipw != 256) return fail(OCTAX_E_INVALID, "octax_create: envs_per_block must be 64, 128 or 256");
    if (!cfg->h_rom_data || !cfg->h_rom_offset || !cfg->h_rom_len || !cfg->h_env_rom ||
        !cfg->h_action_keys || !cfg->h_num_actions || !cfg->h_score_reg || !cfg->h_term_reg ||
        !cfg->h_term_value || !cfg->h_horizon || !cfg->h_env_seed)
        return fail(OCTAX_E_INVALID, "octax_create: a host array is NULL");
    for (uint32_t r = 0; r < R; r++) {
        if (cfg->h_rom_len[r] > OCTAX_MAX_ROM_BYTES) return fail(OCTAX_E_INVALID, "octax_create: ROM longer than 3584 bytes");
        if (cfg->h_num_actions[r] > 16) return fail(OCTAX_E_INVALID, "octax_create: num_actions > 16");
        if (cfg->h_score_reg[r] > 15 || cfg->h_term_reg[r] > 15) return fail(OCTAX_E_INVALID, "octax_create: register index > 15");
        for (uint32_t a = 0; a < cfg->h_num_actions[r]; a++)
            if (cfg->h_action_keys[16 * r + a] > 15) return fail(OCTAX_E_INVALID, "octax_create: key > 15");
    }
    for (uint32_t e = 0; e < E; e++)
        if (cfg->h_env_rom[e] >= R) return fail(OCTAX_E_INVALID, "octax_create: env_rom >= num_roms");
    std::vector<uint8_t> startup;
    if (const char *err = octax::check_wrappers(cfg->sticky_q24, cfg->noop_max, cfg->h_startup_len,
                                                cfg->h_startup_keys, R, startup))
        return fail(OCTAX_E_INVALID, std::string("octax_create: ") + err);
    std::vector<uint32_t> desc2;
    if (const char *err = octax::check_profile(cfg, desc2))
        return fail(OCTAX_E_INVALID, std::string("octax_create: ") + err);
    if (cfg->platform > OCTAX_PLATFORM_SCHIP) return fail(OCTAX_E_INVALID, "octax_create: unknown platform");
    const bool schip = cfg->platform == OCTAX_PLATFORM_SCHIP;
    if (schip && cfg->kernel != OCTAX_KERNEL_PLAIN)
        return fail(OCTAX_E_INVALID, "octax_create: SUPER-CHIP engines run on the plain kernel");
    uint32_t max_startup = 0;
    for (uint32_t r = 0; r < R; r++) max_startup = std::max<uint32_t>(max_startup, startup[17 * (size_t)r]);
    const uint64_t step_slots = (uint64_t)cfg->instr_per_frame * cfg->frame_skip * (1 + max_startup + cfg->noop_max);
    if (cfg->kernel == OCTAX_KERNEL_FUSED && step_slots > octax::kFusedMaxStepSlots)
        return fail(OCTAX_E_INVALID, "octax_create: the fused kernel takes at most 1,048,576 instruction slots per "
                                     "step (ipf x frame_skip x (1 + start-up steps + noop_max)); use the plain kernel");

    octax_engine *g = new (std::nothrow) octax_engine;
    if (!g) return fail(OCTAX_E_NOMEM, "octax_create: out of host memory");
    g->E = E;
    g->R = R;
    g->ipf = cfg->instr_per_frame;
    g->frame_skip = cfg->frame_skip;
    g->kernel = cfg->kernel;
    g->placement = cfg->placement;
    g->envs_per_block = ipw;
    g->rom_in_lds = cfg->rom_in_lds ? 1 : 0;
    g->schip = schip ? 1 : 0;
    g->stream = static_cast<hipStream_t>(cfg->stream);
    (void)hipGetDevice(&g->device);
    g->step_slots = step_slots;
    g->rom_len.assign(cfg->h_rom_len, cfg->h_rom_len + R);

    // Placement: slot -> env.
    g->env_of.resize(E);
    for (uint32_t e = 0; e < E; e++) g->env_of[e] = e;
    if (g->placement == OCTAX_PLACE_BY_ROM)
        std::stable_sort(g->env_of.begin(), g->env_of.end(),
                         [&](uint32_t a, uint32_t b) { return cfg->h_env_rom[a] < cfg->h_env_rom[b]; });
    if (g->placement == OCTAX_PLACE_BY_HORIZON) {
        // envs by horizon (0: none, after every finite one), then the i-th of
        // them into the i-th slot of the order lane 0 of every wavefront,
        // lane 1 of every wavefront, ... (slots past E skipped)
        std::vector<uint32_t> by_h(E);
        for (uint32_t e = 0; e < E; e++) by_h[e] = e;
        auto key = [&](uint32_t e) { return cfg->h_horizon[e] ? (uint64_t)cfg->h_horizon[e] : (uint64_t)1 << 32; };
        std::stable_sort(by_h.begin(), by_h.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
        const uint32_t waves = (E + 63) / 64;
        uint32_t i = 0;
        for (uint32_t lane = 0; lane < 64; lane++)
            for (uint32_t w = 0; w < waves; w++) {
                const uint32_t sl = w * 64 + lane;
                if (sl < E) g->env_of[sl] = by_h[i++];
            }
    }
    g->slot_of.resize(E);
    g->rom_of.resize(E);
    std::vector<uint32_t> horizon(E);
    std::vector<uint64_t> seed(E);
    for (uint32_t sl = 0; sl < E; sl++) {
        const uint32_t e = g->env_of[sl];
        g->slot_of[e] = sl;
        g->rom_of[sl] = cfg->h_env_rom[e];
        horizon[sl] = cfg->h_horizon[e];
        seed[sl] = cfg->h_env_seed[e];
    }

    // Power-on images and descriptors.
    std::vector<uint8_t> image((size_t)R * kMem, 0);
    std::vector<uint32_t> desc(R);
    for (uint32_t r = 0; r < R; r++) {
        uint8_t *m = image.data() + (size_t)r * kMem;
        std::memcpy(m + kFont, kFontBytes, sizeof kFontBytes);
        std::memcpy(m + kProgram, cfg->h_rom_data + cfg->h_rom_offset[r], cfg->h_rom_len[r]);
        if (schip) std::memcpy(m + kBigFont, kBigFontBytes, sizeof kBigFontBytes);
        desc[r] = cfg->h_score_reg[r] | ((uint32_t)cfg->h_term_reg[r] << 8) |
                  ((uint32_t)cfg->h_term_value[r] << 16) | ((uint32_t)cfg->h_num_actions[r] << 24);
    }

    hipError_t e = hipSuccess;
    uint32_t *rom_of = nullptr, *hor = nullptr, *env_of = nullptr, *d_desc = nullptr, *d_desc2 = nullptr;
    uint8_t *d_img = nullptr, *d_keys = nullptr;
#define TRY(x)                                                    \
    do {                                                          \
        e = (x);                                                  \
        if (e != hipSuccess) {                                    \
            g->free_all();                                        \
            delete g;                                             \
            return e == hipErrorOutOfMemory                       \
                       ? fail(OCTAX_E_NOMEM, "octax_create: device allocation failed") \
                       : hip_fail(e, "octax_create");             \
        }                                                         \
    } while (0)
    TRY(g->alloc(&g->s.regs, 4 * (size_t)E));
    TRY(g->alloc(&g->s.pc_i, E));
    TRY(g->alloc(&g->s.misc, E));
    TRY(g->alloc(&g->s.stack, 8 * (size_t)E));
    TRY(g->alloc(&g->s.t, E));
    TRY(g->alloc(&g->s.prev, E));
    TRY(g->alloc(&g->s.rng, E));
    TRY(g->alloc(&g->s.dirty, E));
    TRY(g->alloc(&g->s.fb, 32 * (size_t)E));
    TRY(g->alloc(&g->s.cols, 256 * (size_t)E));
    TRY(g->alloc(&g->s.ram, (size_t)kMem * E));
    if (schip) {
        TRY(g->alloc(&g->s.hfb, 128 * (size_t)E));
        TRY(g->alloc(&g->s.hring, 640 * (size_t)E));
        TRY(g->alloc(&g->s.sx, 4 * (size_t)E));
    }
    TRY(g->alloc(&rom_of, E));
    TRY(g->alloc(&hor, E));
    TRY(g->alloc(&env_of, E));
    TRY(g->alloc(&d_img, (size_t)R * kMem));
    TRY(g->alloc(&d_keys, 16 * (size_t)R));
    TRY(g->alloc(&d_desc, R));
    TRY(g->alloc(&g->d_startup, startup.size()));
    TRY(hipMemcpy(g->d_startup, startup.data(), startup.size(), hipMemcpyHostToDevice));
    TRY(hipMemcpy(rom_of, g->rom_of.data(), 4 * (size_t)E, hipMemcpyHostToDevice));
    TRY(hipMemcpy(hor, horizon.data(), 4 * (size_t)E, hipMemcpyHostToDevice));
    TRY(hipMemcpy(env_of, g->env_of.data(), 4 * (size_t)E, hipMemcpyHostToDevice));
    TRY(hipMemcpy(g->s.rng, seed.data(), 8 * (size_t)E, hipMemcpyHostToDevice));
    TRY(hipMemcpy(d_img, image.data(), image.size(), hipMemcpyHostToDevice));
    TRY(hipMemcpy(d_keys, cfg->h_action_keys, 16 * (size_t)R, hipMemcpyHostToDevice));
    TRY(hipMemcpy(d_desc, desc.data(), 4 * (size_t)R, hipMemcpyHostToDevice));
    if (!desc2.empty()) {
        TRY(g->alloc(&d_desc2, R));
        TRY(hipMemcpy(d_desc2, desc2.data(), 4 * (size_t)R, hipMemcpyHostToDevice));
    }
    g->s.rom_of = rom_of;
    g->s.horizon = hor;
    g->s.env_of = env_of;
    g->s.num = E;
    g->roms.image = d_img;
    g->roms.keys = d_keys;
    g->roms.desc = d_desc;
    g->roms.desc2 = d_desc2;
    g->roms.quirks = cfg->quirks;
    g->roms.profile = (cfg->quirks != OCTAX_QUIRKS_V1 || d_desc2) ? 1u : 0u;
    g->roms.schip = g->schip;
    g->roms.w = octax::make_wrap(g->d_startup, startup, cfg->sticky_q24, cfg->noop_max, g->ipf, g->frame_skip);
    TRY(upload_block_roms(g));
    {
        int wall_khz = 0;
        TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, g->device));
        g->wait_ticks = octax::fused_wait_ticks(step_slots, wall_khz > 0 ? (uint64_t)wall_khz : 100000u);
    }
    TRY(g->alloc(&g->d_err, 4));
    TRY(hipMemset(g->d_err, 0, 16));
    TRY(launch_reset(g->s, g->roms, nullptr, true, g->stream));
    TRY(hipStreamSynchronize(g->stream));
#undef TRY
    *out = g;
    return OCTAX_OK;
}

int32_t octax_destroy(octax_engine *g) {
    if (!g) return OCTAX_OK;
    const int32_t rc = check_device_error(g, "octax_destroy");
    g->free_all();
    delete g;
    return rc;
}

int32_t octax_status(octax_engine *g) {
    if (!g) return fail(OCTAX_E_INVALID, "octax_status: engine is NULL");
    return check_device_error(g, "octax_status");
}

int32_t octax_set_step_clock(octax_engine *g, uint64_t *d_stamps, uint32_t steps, uint64_t *h_clock_hz) {
    if (!g || (steps && !d_stamps)) return fail(OCTAX_E_INVALID, "octax_set_step_clock: NULL argument");
    if (g->graphs > 0) return fail(OCTAX_E_STATE, "octax_set_step_clock: destroy the engine's graphs first");
    if (h_clock_hz) {
        int khz = 0;
        const hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device);
        if (e != hipSuccess) return hip_fail(e, "octax_set_step_clock");
        *h_clock_hz = 1000ull * (uint64_t)khz;
    }
    g->d_stamps = steps ? d_stamps : nullptr;
    g->stamp_steps = steps;
    return OCTAX_OK;
}

int32_t octax_set_wait_limit(octax_engine *g, uint64_t ticks) {
    if (!g) return fail(OCTAX_E_INVALID, "octax_set_wait_limit: engine is NULL");
    if (g->graphs > 0) return fail(OCTAX_E_STATE, "octax_set_wait_limit: destroy the engine's graphs first");
    g->wait_override = ticks;
    return OCTAX_OK;
}

int32_t octax_reset(octax_engine *g, const uint8_t *d_mask, uint8_t *d_obs) {
    if (!g) return fail(OCTAX_E_INVALID, "octax_reset: engine is NULL");
    hipError_t e = launch_reset(g->s, g->roms, d_mask, false, g->stream);
    if (e == hipSuccess && d_obs)
        e = g->schip ? launch_schip_observe(g->s, d_obs, g->stream) : launch_observe(g->s, d_obs, g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_reset");
}

int32_t octax_digest(octax_engine *g, uint64_t *d_out) {
    if (!g || !d_out) return fail(OCTAX_E_INVALID, "octax_digest: NULL engine or output");
    hipError_t e = launch_digest(g->s, d_out, g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_digest");
}

int32_t octax_get_schip_state(octax_engine *g, uint32_t first, uint32_t count, octax_schip_state *h_out) {
    if (!g || (!h_out && count)) return fail(OCTAX_E_INVALID, "octax_get_schip_state: NULL argument");
    if (!g->schip) return fail(OCTAX_E_INVALID, "octax_get_schip_state: not a SUPER-CHIP engine");
    if ((uint64_t)first + count > g->E) return fail(OCTAX_E_INVALID, "octax_get_schip_state: range outside 0..E");
    hipError_t e = hipStreamSynchronize(g->stream);
    std::vector<uint64_t> ring(640);
    for (uint32_t k = 0; k < count && e == hipSuccess; k++) {
        const uint32_t slot = g->slot_of[first + k];
        uint32_t t = 0, sx[4] = {0, 0, 0, 0};
        octax_schip_state &o = h_out[k];
        e = hipMemcpy(&t, g->s.t + slot, 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(sx, g->s.sx + 4 * (size_t)slot, 16, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(o.fb, g->s.hfb + 128 * (size_t)slot, 1024, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(ring.data(), g->s.hring + 640 * (size_t)slot, 5120, hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        o.hires = sx[0] & 1;
        // the device keeps display row y in row (y + offset) & 63, the offset in bits 8..13 of sx word 0
        const uint32_t roff = (sx[0] >> 8) & 63;
        if (roff) {
            uint64_t rows[64][2];
            std::memcpy(rows, o.fb, sizeof rows);
            for (uint32_t y = 0; y < 64; y++) {
                o.fb[y][0] = rows[(y + roff) & 63][0];
                o.fb[y][1] = rows[(y + roff) & 63][1];
            }
        }
        std::memcpy(o.rpl, &sx[1], 8);
        o.reserved = 0;
        // five ring slots, the display in slot head; frames from before the
        // env's last reset show the reset display
        const uint32_t head = (sx[3] >> 16) & 7;
        for (uint32_t h = 0; h < 3; h++) {
            const uint32_t age = std::min(3 - h, t);
            std::memcpy(o.hist[h], ring.data() + 128 * ((head + 5 - age) % 5), 1024);
        }
    }
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_get_schip_state");
}

int32_t octax_step(octax_engine *g, const int32_t *d_action, uint8_t *d_obs, float *d_reward,
                   uint8_t *d_done) {
    if (!g || !d_action || !d_reward || !d_done)
        return fail(OCTAX_E_INVALID, "octax_step: NULL engine, action, reward or done");
    hipError_t e = launch_steps(g, 1, d_action, d_obs, 1, d_reward, d_done, g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_step");
}

int32_t octax_step_many(octax_engine *g, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                        uint32_t obs_slots, float *d_reward, uint8_t *d_done) {
    if (!g || !d_action || !d_reward || !d_done)
        return fail(OCTAX_E_INVALID, "octax_step_many: NULL engine, action, reward or done");
    if (K == 0) return fail(OCTAX_E_INVALID, "octax_step_many: K == 0");
    if (d_obs && obs_slots == 0) return fail(OCTAX_E_INVALID, "octax_step_many: obs_slots == 0");
    hipError_t e = launch_steps(g, K, d_action, d_obs, obs_slots, d_reward, d_done, g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_step_many");
}

int32_t octax_graph_create(octax_engine *g, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                           uint32_t obs_slots, float *d_reward, uint8_t *d_done, octax_graph **out) {
    if (!out) return fail(OCTAX_E_INVALID, "octax_graph_create: out is NULL");
    *out = nullptr;
    if (!g || !d_action || !d_reward || !d_done)
        return fail(OCTAX_E_INVALID, "octax_graph_create: NULL engine, action, reward or done");
    if (K == 0) return fail(OCTAX_E_INVALID, "octax_graph_create: K == 0");
    if (d_obs && obs_slots == 0) return fail(OCTAX_E_INVALID, "octax_graph_create: obs_slots == 0");
    octax_graph *gr = new (std::nothrow) octax_graph;
    if (!gr) return fail(OCTAX_E_NOMEM, "octax_graph_create: out of host memory");
    gr->eng = g;
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_steps(g, K, d_action, d_obs, obs_slots, d_reward, d_done, cap);
        e = hipStreamEndCapture(cap, &gr->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        delete gr;
        return hip_fail(e, "octax_graph_create");
    }
    g->graphs++;
    *out = gr;
    return OCTAX_OK;
}

int32_t octax_graph_launch(octax_graph *gr) {
    if (!gr) return fail(OCTAX_E_INVALID, "octax_graph_launch: graph is NULL");
    hipError_t e = hipGraphLaunch(gr->exec, gr->eng->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_graph_launch");
}

int32_t octax_graph_destroy(octax_graph *gr) {
    if (!gr) return OCTAX_OK;
    hipError_t e = hipStreamSynchronize(gr->eng->stream);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    gr->eng->graphs--;
    delete gr;
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_graph_destroy");
}

int32_t octax_get_state(octax_engine *g, uint32_t first, uint32_t count, octax_env_state *h_out) {
    if (!g || (!h_out && count)) return fail(OCTAX_E_INVALID, "octax_get_state: NULL argument");
    if ((uint64_t)first + count > g->E) return fail(OCTAX_E_INVALID, "octax_get_state: range outside 0..E");
    if (count == 0) return OCTAX_OK;
    hipError_t e = ensure_raw(g, count);
    std::vector<uint32_t> slots(count);
    for (uint32_t k = 0; k < count; k++) slots[k] = g->slot_of[first + k];
    std::vector<RawState> raw(count);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemcpy(g->d_slot_scratch, slots.data(), 4 * (size_t)count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_pack(g->s, g->d_slot_scratch, count, g->d_raw, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemcpy(raw.data(), g->d_raw, sizeof(RawState) * (size_t)count, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "octax_get_state");
    for (uint32_t k = 0; k < count; k++) raw_to_canonical(raw[k], h_out[k]);
    return check_device_error(g, "octax_get_state");
}

int32_t octax_get_state_noalloc(octax_engine *g, uint32_t first, uint32_t count, octax_env_state *h_out) {
    if (!g || (!h_out && count)) return fail(OCTAX_E_INVALID, "octax_get_state_noalloc: NULL argument");
    if ((uint64_t)first + count > g->E)
        return fail(OCTAX_E_INVALID, "octax_get_state_noalloc: range outside 0..E");
    if (count > OCTAX_NOALLOC_MAX_ENVS)
        return fail(OCTAX_E_INVALID, "octax_get_state_noalloc: count above OCTAX_NOALLOC_MAX_ENVS (64)");
    if (count == 0) return OCTAX_OK;
    uint8_t *base = nullptr;
    hipError_t e = scratch_of(g->device, &base);
    if (e != hipSuccess) return hip_fail(e, "octax_get_state_noalloc: scratch address");
    uint32_t *d_slots = reinterpret_cast<uint32_t *>(base);
    RawState *d_raw = reinterpret_cast<RawState *>(base + kNoAllocSlotBytes);
    uint32_t slots[OCTAX_NOALLOC_MAX_ENVS];
    for (uint32_t k = 0; k < count; k++) slots[k] = g->slot_of[first + k];
    e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemcpy(d_slots, slots, 4 * (size_t)count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_pack(g->s, d_slots, count, d_raw, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    // records come back a few at a time through a buffer on the host stack
    constexpr uint32_t kChunk = 4;
    RawState buf[kChunk];
    for (uint32_t k0 = 0; e == hipSuccess && k0 < count; k0 += kChunk) {
        const uint32_t n = std::min(kChunk, count - k0);
        e = hipMemcpy(buf, d_raw + k0, sizeof(RawState) * n, hipMemcpyDeviceToHost);
        for (uint32_t k = 0; e == hipSuccess && k < n; k++) raw_to_canonical(buf[k], h_out[k0 + k]);
    }
    if (e != hipSuccess) return hip_fail(e, "octax_get_state_noalloc");
    return check_device_error(g, "octax_get_state_noalloc");
}

int32_t octax_set_state(octax_engine *g, uint32_t first, uint32_t count, const octax_env_state *h_in) {
    if (!g || (!h_in && count)) return fail(OCTAX_E_INVALID, "octax_set_state: NULL argument");
    if ((uint64_t)first + count > g->E) return fail(OCTAX_E_INVALID, "octax_set_state: range outside 0..E");
    if (count == 0) return OCTAX_OK;
    hipError_t e = ensure_raw(g, count);
    std::vector<uint32_t> slots(count);
    std::vector<RawState> raw(count);
    for (uint32_t k = 0; k < count; k++) {
        slots[k] = g->slot_of[first + k];
        canonical_to_raw(h_in[k], raw[k]);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemcpy(g->d_slot_scratch, slots.data(), 4 * (size_t)count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->d_raw, raw.data(), sizeof(RawState) * (size_t)count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_unpack(g->s, g->d_slot_scratch, count, g->d_raw, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_set_state");
}

int32_t octax_set_kernel(octax_engine *g, uint32_t kernel) {
    if (!g || kernel > OCTAX_KERNEL_FUSED) return fail(OCTAX_E_INVALID, "octax_set_kernel: bad argument");
    if (g->schip && kernel != OCTAX_KERNEL_PLAIN)
        return fail(OCTAX_E_INVALID, "octax_set_kernel: SUPER-CHIP engines run on the plain kernel");
    if (kernel == OCTAX_KERNEL_FUSED && g->step_slots > kFusedMaxStepSlots)
        return fail(OCTAX_E_INVALID, "octax_set_kernel: the config's steps are too long for the fused kernel");
    g->kernel = kernel;
    return OCTAX_OK;
}

int32_t octax_set_tuning(octax_engine *g, uint32_t envs_per_block, uint32_t rom_in_lds) {
    if (!g || (envs_per_block != 64 && envs_per_block != 128 && envs_per_block != 256))
        return fail(OCTAX_E_INVALID, "octax_set_tuning: envs_per_block must be 64, 128 or 256");
    if (g->graphs > 0) return fail(OCTAX_E_STATE, "octax_set_tuning: destroy the engine's graphs first");
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "octax_set_tuning");
    g->envs_per_block = envs_per_block;
    g->rom_in_lds = rom_in_lds ? 1 : 0;
    e = upload_block_roms(g);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_set_tuning");
}

int32_t octax_set_stream(octax_engine *g, void *stream) {
    if (!g) return fail(OCTAX_E_INVALID, "octax_set_stream: engine is NULL");
    g->stream = static_cast<hipStream_t>(stream);
    return OCTAX_OK;
}

int32_t octax_info(const octax_engine *g, uint32_t *num_envs, uint64_t *device_bytes) {
    if (!g) return fail(OCTAX_E_INVALID, "octax_info: engine is NULL");
    if (num_envs) *num_envs = g->E;
    if (device_bytes) *device_bytes = g->device_bytes;
    return OCTAX_OK;
}

}  // extern "C"
