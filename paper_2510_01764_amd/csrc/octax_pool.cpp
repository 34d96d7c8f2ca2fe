// Serving pool of liboctax (declared in include/octax.h): environment groups
// admitted into free slots of one resident engine and stepped together, one
// fused launch per tick, while groups arrive and leave.
//
// The pool is an engine of `capacity` slots with identity placement and the
// fused kernel.  Membership lives in the device table State::occupied; the
// step kernel skips free slots and whole blocks with no occupied slot.  A
// group takes the lowest-numbered free slots, contiguous or not, so any group
// fits as long as enough slots are free (no fragmentation).  Admission writes
// the group's ROM id, horizons and RNG seeds into its slots (copied, one run
// of consecutive slots at a time, from pinned staging indexed by slot; an
// admission first waits for the copies of the previous one, so staging is
// never rewritten while a copy from it may be pending) and resets the slots
// to the ROM's power-on image.  The page-pool table of the workgroups is
// recomputed on the host when membership changes and uploaded before the
// next step.
#include <hip/hip_runtime.h>

#include <cstring>
#include <iterator>
#include <map>
#include <new>
#include <vector>

#include "octax_engine.h"

using namespace octax;

namespace {

// Device bytes per slot: the engine's state arrays plus the occupancy and
// reset-mask bytes of the pool.
constexpr uint64_t kSlotBytes = 16 + 4 + 4 + 32 + 4 + 4 + 8 + 8 + 256 + 1024 + 4096 + 12 + 2;

}  // namespace

struct octax_pool {
    octax_engine *eng = nullptr;
    uint32_t capacity = 0;
    std::vector<uint64_t> free_bits;            // bit s of word s / 64: slot s is free
    uint32_t free_count = 0;
    std::map<uint32_t, std::vector<uint32_t>> groups;   // group id -> its slots, ascending
    uint32_t next_group = 0;
    uint8_t *d_occupied = nullptr;              // [capacity]
    uint8_t *d_mask = nullptr;                  // [capacity], zero outside an admission
    uint32_t *h_rom_stage = nullptr;            // pinned [capacity]
    uint32_t *h_hor_stage = nullptr;            // pinned [capacity]
    uint64_t *h_seed_stage = nullptr;           // pinned [capacity]
    uint32_t *h_table = nullptr;                // pinned [blocks][kPoolRoms][2]
    size_t table_len = 0;
    hipEvent_t table_done = nullptr;            // the last table upload has been read
    hipEvent_t stage_done = nullptr;            // the last admission's copies have been read
    bool table_dirty = true;

    ~octax_pool() {
        if (eng) (void)octax_destroy(eng);
        for (void *p : {static_cast<void *>(h_rom_stage), static_cast<void *>(h_hor_stage),
                        static_cast<void *>(h_seed_stage), static_cast<void *>(h_table)})
            if (p) (void)hipHostFree(p);
        if (table_done) (void)hipEventDestroy(table_done);
        if (stage_done) (void)hipEventDestroy(stage_done);
    }
};

namespace {

// Runs of consecutive slots of an ascending slot list: (first, length).
std::vector<std::pair<uint32_t, uint32_t>> runs_of(const std::vector<uint32_t> &slots) {
    std::vector<std::pair<uint32_t, uint32_t>> out;
    for (uint32_t s : slots) {
        if (!out.empty() && out.back().first + out.back().second == s) out.back().second++;
        else out.emplace_back(s, 1u);
    }
    return out;
}

hipError_t upload_table(octax_pool *p) {
    octax_engine *g = p->eng;
    std::vector<uint32_t> table;
    block_rom_table(g, table);
    // the previous upload must have left the pinned buffer before it is rewritten
    hipError_t e = hipEventSynchronize(p->table_done);
    if (e != hipSuccess) return e;
    std::memcpy(p->h_table, table.data(), table.size() * sizeof(uint32_t));
    e = hipMemcpyAsync(g->d_block_roms, p->h_table, table.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, g->stream);
    if (e != hipSuccess) return e;
    e = hipEventRecord(p->table_done, g->stream);
    if (e == hipSuccess) p->table_dirty = false;
    return e;
}

}  // namespace

extern "C" {

uint64_t octax_pool_slot_bytes(void) { return kSlotBytes; }

int32_t octax_pool_create(const octax_pool_config *cfg, octax_pool **out) {
    if (!out) return fail(OCTAX_E_INVALID, "octax_pool_create: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(OCTAX_E_INVALID, "octax_pool_create: cfg is NULL");
    if (cfg->abi_version != OCTAX_ABI_VERSION) return fail(OCTAX_E_INVALID, "octax_pool_create: abi_version mismatch");
    const uint64_t cap64 = cfg->pool_bytes / kSlotBytes;
    if (cap64 == 0) return fail(OCTAX_E_INVALID, "octax_pool_create: pool_bytes below one slot");
    if (cap64 > (1u << 26)) return fail(OCTAX_E_INVALID, "octax_pool_create: pool_bytes above 2^26 slots");
    const uint32_t cap = (uint32_t)cap64;
    const uint32_t R = cfg->num_roms;
    if (R == 0 || R > 65535) return fail(OCTAX_E_INVALID, "octax_pool_create: num_roms out of range");

    // the pool's engine: capacity slots, every one initially ROM 0
    std::vector<uint16_t> env_rom(cap, 0);
    std::vector<uint32_t> horizon(cap, 0);
    std::vector<uint64_t> seed(cap, 0);
    octax_config ec{};
    ec.abi_version = cfg->abi_version;
    ec.num_envs = cap;
    ec.num_roms = R;
    ec.instr_per_frame = cfg->instr_per_frame;
    ec.frame_skip = cfg->frame_skip;
    ec.quirks = cfg->quirks;
    ec.kernel = OCTAX_KERNEL_FUSED;
    ec.placement = OCTAX_PLACE_IDENTITY;
    ec.envs_per_block = cfg->envs_per_block;
    ec.lanes_per_env = 1;
    ec.rom_in_lds = 1;
    ec.h_rom_data = cfg->h_rom_data;
    ec.h_rom_offset = cfg->h_rom_offset;
    ec.h_rom_len = cfg->h_rom_len;
    ec.h_env_rom = env_rom.data();
    ec.h_action_keys = cfg->h_action_keys;
    ec.h_num_actions = cfg->h_num_actions;
    ec.h_score_reg = cfg->h_score_reg;
    ec.h_term_reg = cfg->h_term_reg;
    ec.h_term_value = cfg->h_term_value;
    ec.h_horizon = horizon.data();
    ec.h_env_seed = seed.data();
    ec.stream = cfg->stream;
    ec.sticky_q24 = cfg->sticky_q24;
    ec.noop_max = cfg->noop_max;
    ec.h_startup_len = cfg->h_startup_len;
    ec.h_startup_keys = cfg->h_startup_keys;
    ec.h_score_mode = cfg->h_score_mode;
    ec.h_score_arg = cfg->h_score_arg;
    ec.h_term_op = cfg->h_term_op;
    ec.h_term2_op = cfg->h_term2_op;
    ec.h_term2_reg = cfg->h_term2_reg;
    ec.h_term2_value = cfg->h_term2_value;

    octax_pool *p = new (std::nothrow) octax_pool;
    if (!p) return fail(OCTAX_E_NOMEM, "octax_pool_create: out of host memory");
    int32_t rc = octax_create(&ec, &p->eng);
    if (rc != OCTAX_OK) {
        delete p;
        return rc;   // octax_create recorded the message
    }
    octax_engine *g = p->eng;
    p->capacity = cap;
    g->occupied.assign(cap, 0);
    hipError_t e = g->alloc(&p->d_occupied, cap);
    if (e == hipSuccess) e = g->alloc(&p->d_mask, cap);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_occupied, 0, cap, g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_mask, 0, cap, g->stream);
    p->table_len = 2 * (size_t)kPoolRoms * ((cap + g->envs_per_block - 1) / g->envs_per_block);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->h_rom_stage), 4 * (size_t)cap, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->h_hor_stage), 4 * (size_t)cap, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->h_seed_stage), 8 * (size_t)cap, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->h_table), 4 * p->table_len, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->table_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p->table_done, g->stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->stage_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p->stage_done, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        delete p;
        return e == hipErrorOutOfMemory ? fail(OCTAX_E_NOMEM, "octax_pool_create: allocation failed")
                                        : hip_fail(e, "octax_pool_create");
    }
    g->s.occupied = p->d_occupied;
    p->free_bits.assign((cap + 63) / 64, ~0ull);
    if (cap % 64) p->free_bits.back() = (1ull << (cap % 64)) - 1;
    p->free_count = cap;
    *out = p;
    return OCTAX_OK;
}

int32_t octax_pool_admit(octax_pool *p, uint32_t rom, uint32_t count, const uint64_t *h_env_seed,
                         const uint32_t *h_horizon, uint32_t *h_slots, uint32_t *group) {
    if (!p || !h_env_seed || !h_horizon || !h_slots || !group)
        return fail(OCTAX_E_INVALID, "octax_pool_admit: NULL argument");
    octax_engine *g = p->eng;
    if (rom >= g->R) return fail(OCTAX_E_INVALID, "octax_pool_admit: rom >= num_roms");
    if (count == 0 || count > p->capacity) return fail(OCTAX_E_INVALID, "octax_pool_admit: count out of range");
    if (count > p->free_count) return fail(OCTAX_E_NOMEM, "octax_pool_admit: fewer free slots than the group's envs");
    // the lowest-numbered free slots
    std::vector<uint32_t> slots;
    slots.reserve(count);
    for (uint32_t w = 0; w < p->free_bits.size() && slots.size() < count; w++) {
        uint64_t bits = p->free_bits[w];
        while (bits && slots.size() < count) {
            slots.push_back(64 * w + (uint32_t)__builtin_ctzll(bits));
            bits &= bits - 1;
        }
    }
    const auto runs = runs_of(slots);

    hipError_t e = hipEventSynchronize(p->stage_done);
    if (e != hipSuccess) return hip_fail(e, "octax_pool_admit");
    for (uint32_t k = 0; k < count; k++) {
        p->h_rom_stage[slots[k]] = rom;
        p->h_hor_stage[slots[k]] = h_horizon[k];
        p->h_seed_stage[slots[k]] = h_env_seed[k];
    }
    hipStream_t st = g->stream;
    uint32_t *rom_of = const_cast<uint32_t *>(g->s.rom_of);
    uint32_t *hor = const_cast<uint32_t *>(g->s.horizon);
    for (const auto &r : runs) {
        const uint32_t a = r.first, n = r.second;
        if (e == hipSuccess) e = hipMemcpyAsync(rom_of + a, p->h_rom_stage + a, 4 * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hor + a, p->h_hor_stage + a, 4 * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(g->s.rng + a, p->h_seed_stage + a, 8 * (size_t)n, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipEventRecord(p->stage_done, st);
    for (const auto &r : runs)
        if (e == hipSuccess) e = hipMemsetAsync(p->d_mask + r.first, 1, r.second, st);
    // one reset over the span of the group's slots: slots of other groups in it have a zero mask
    const uint32_t lo = slots.front(), span = slots.back() - lo + 1;
    if (e == hipSuccess) e = launch_reset_range(g->s, g->roms, p->d_mask, true, lo, span, st);
    for (const auto &r : runs) {
        if (e == hipSuccess) e = hipMemsetAsync(p->d_mask + r.first, 0, r.second, st);
        if (e == hipSuccess) e = hipMemsetAsync(p->d_occupied + r.first, 1, r.second, st);
    }
    if (e != hipSuccess) return hip_fail(e, "octax_pool_admit");

    for (uint32_t s : slots) {
        p->free_bits[s / 64] &= ~(1ull << (s % 64));
        g->rom_of[s] = rom;
        g->occupied[s] = 1;
    }
    p->free_count -= count;
    const uint32_t id = p->next_group++;
    std::copy(slots.begin(), slots.end(), h_slots);
    p->groups.emplace(id, std::move(slots));
    p->table_dirty = true;
    *group = id;
    return OCTAX_OK;
}

int32_t octax_pool_retire(octax_pool *p, uint32_t group) {
    if (!p) return fail(OCTAX_E_INVALID, "octax_pool_retire: pool is NULL");
    auto it = p->groups.find(group);
    if (it == p->groups.end()) return fail(OCTAX_E_INVALID, "octax_pool_retire: no such group");
    octax_engine *g = p->eng;
    hipError_t e = hipSuccess;
    for (const auto &r : runs_of(it->second))
        if (e == hipSuccess) e = hipMemsetAsync(p->d_occupied + r.first, 0, r.second, g->stream);
    if (e != hipSuccess) return hip_fail(e, "octax_pool_retire");
    for (uint32_t s : it->second) {
        p->free_bits[s / 64] |= 1ull << (s % 64);
        g->occupied[s] = 0;
    }
    p->free_count += (uint32_t)it->second.size();
    p->groups.erase(it);
    p->table_dirty = true;
    return OCTAX_OK;
}

int32_t octax_pool_step_budget(octax_pool *p, uint32_t K, const uint8_t *d_budget, const int32_t *d_action,
                               uint8_t *d_obs, uint32_t obs_slots, float *d_reward, uint8_t *d_done) {
    if (!p || !d_action || !d_reward || !d_done)
        return fail(OCTAX_E_INVALID, "octax_pool_step: NULL pool, action, reward or done");
    if (K == 0) return fail(OCTAX_E_INVALID, "octax_pool_step: K == 0");
    if (d_budget && K > 255) return fail(OCTAX_E_INVALID, "octax_pool_step_budget: K > 255 with step budgets");
    if (d_obs && obs_slots == 0) return fail(OCTAX_E_INVALID, "octax_pool_step: obs_slots == 0");
    octax_engine *g = p->eng;
    hipError_t e = hipSuccess;
    if (p->table_dirty) e = upload_table(p);
    if (e == hipSuccess) e = launch_steps(g, K, d_action, d_obs, obs_slots, d_reward, d_done, g->stream, d_budget);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_pool_step");
}

int32_t octax_pool_step(octax_pool *p, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                        uint32_t obs_slots, float *d_reward, uint8_t *d_done) {
    return octax_pool_step_budget(p, K, nullptr, d_action, d_obs, obs_slots, d_reward, d_done);
}

int32_t octax_pool_info(const octax_pool *p, uint32_t *capacity, uint32_t *free_slots,
                        uint32_t *largest_free, uint32_t *groups) {
    if (!p) return fail(OCTAX_E_INVALID, "octax_pool_info: pool is NULL");
    if (capacity) *capacity = p->capacity;
    if (free_slots) *free_slots = p->free_count;
    if (largest_free) *largest_free = p->free_count;   // any free slots take a group
    if (groups) *groups = (uint32_t)p->groups.size();
    return OCTAX_OK;
}

int32_t octax_pool_get_state(octax_pool *p, const uint32_t *h_slots, uint32_t count, octax_env_state *h_out) {
    if (!p || (count && (!h_slots || !h_out))) return fail(OCTAX_E_INVALID, "octax_pool_get_state: NULL argument");
    // runs of consecutive slots, each one octax_get_state call (env = slot in a pool)
    for (uint32_t k = 0; k < count;) {
        uint32_t n = 1;
        while (k + n < count && h_slots[k + n] == h_slots[k] + n) n++;
        const int32_t rc = octax_get_state(p->eng, h_slots[k], n, h_out + k);
        if (rc != OCTAX_OK) return rc;
        k += n;
    }
    return OCTAX_OK;
}

int32_t octax_pool_destroy(octax_pool *p) {
    if (!p) return OCTAX_OK;
    const int32_t rc = check_device_error(p->eng, "octax_pool_destroy");
    delete p;
    return rc;
}

}  // extern "C"
