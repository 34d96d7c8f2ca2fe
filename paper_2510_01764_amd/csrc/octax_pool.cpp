// Serving pool of liboctax (declared in include/octax.h): environment groups
// admitted into contiguous slot ranges of one resident engine and stepped
// together, one fused launch per tick, while groups arrive and leave.
//
// The pool is an engine of `capacity` slots with identity placement and the
// fused kernel.  Membership lives in the device table State::occupied; the
// step kernel skips free slots and whole blocks with no occupied slot.
// Admission writes the group's ROM id, horizons and RNG seeds into its slots
// (copied from pinned staging indexed by slot; an admission first waits for
// the copies of the previous one, so staging is never rewritten while a copy
// from it may be pending) and resets the slots to the ROM's power-on image.
// The table of ROM images each workgroup stages in LDS is recomputed on the
// host when membership changes and uploaded before the next step.
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
    std::map<uint32_t, uint32_t> free_ranges;   // first slot -> length; disjoint, coalesced
    std::map<uint32_t, uint32_t> groups;        // first slot -> length
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

void release_range(octax_pool *p, uint32_t first, uint32_t len) {
    auto next = p->free_ranges.lower_bound(first);
    if (next != p->free_ranges.end() && first + len == next->first) {
        len += next->second;
        next = p->free_ranges.erase(next);
    }
    if (next != p->free_ranges.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == first) {
            prev->second += len;
            return;
        }
    }
    p->free_ranges.emplace(first, len);
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
    p->free_ranges.emplace(0u, cap);
    *out = p;
    return OCTAX_OK;
}

int32_t octax_pool_admit(octax_pool *p, uint32_t rom, uint32_t count, const uint64_t *h_env_seed,
                         const uint32_t *h_horizon, uint32_t *first_slot) {
    if (!p || !h_env_seed || !h_horizon || !first_slot)
        return fail(OCTAX_E_INVALID, "octax_pool_admit: NULL argument");
    octax_engine *g = p->eng;
    if (rom >= g->R) return fail(OCTAX_E_INVALID, "octax_pool_admit: rom >= num_roms");
    if (count == 0 || count > p->capacity) return fail(OCTAX_E_INVALID, "octax_pool_admit: count out of range");
    auto it = p->free_ranges.begin();
    while (it != p->free_ranges.end() && it->second < count) ++it;
    if (it == p->free_ranges.end()) return fail(OCTAX_E_NOMEM, "octax_pool_admit: no free range of that many slots");
    const uint32_t first = it->first, len = it->second;

    hipError_t e = hipEventSynchronize(p->stage_done);
    if (e != hipSuccess) return hip_fail(e, "octax_pool_admit");
    for (uint32_t k = 0; k < count; k++) {
        p->h_rom_stage[first + k] = rom;
        p->h_hor_stage[first + k] = h_horizon[k];
        p->h_seed_stage[first + k] = h_env_seed[k];
    }
    hipStream_t st = g->stream;
    uint32_t *rom_of = const_cast<uint32_t *>(g->s.rom_of);
    uint32_t *hor = const_cast<uint32_t *>(g->s.horizon);
    e = hipMemcpyAsync(rom_of + first, p->h_rom_stage + first, 4 * (size_t)count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hor + first, p->h_hor_stage + first, 4 * (size_t)count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->s.rng + first, p->h_seed_stage + first, 8 * (size_t)count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(p->stage_done, st);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_mask + first, 1, count, st);
    if (e == hipSuccess) e = launch_reset_range(g->s, g->roms, p->d_mask, true, first, count, st);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_mask + first, 0, count, st);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_occupied + first, 1, count, st);
    if (e != hipSuccess) return hip_fail(e, "octax_pool_admit");

    p->free_ranges.erase(it);
    if (len > count) p->free_ranges.emplace(first + count, len - count);
    p->groups.emplace(first, count);
    for (uint32_t k = 0; k < count; k++) {
        g->rom_of[first + k] = rom;
        g->occupied[first + k] = 1;
    }
    p->table_dirty = true;
    *first_slot = first;
    return OCTAX_OK;
}

int32_t octax_pool_retire(octax_pool *p, uint32_t first_slot) {
    if (!p) return fail(OCTAX_E_INVALID, "octax_pool_retire: pool is NULL");
    auto it = p->groups.find(first_slot);
    if (it == p->groups.end()) return fail(OCTAX_E_INVALID, "octax_pool_retire: no group starts at that slot");
    const uint32_t len = it->second;
    octax_engine *g = p->eng;
    hipError_t e = hipMemsetAsync(p->d_occupied + first_slot, 0, len, g->stream);
    if (e != hipSuccess) return hip_fail(e, "octax_pool_retire");
    p->groups.erase(it);
    for (uint32_t k = 0; k < len; k++) g->occupied[first_slot + k] = 0;
    release_range(p, first_slot, len);
    p->table_dirty = true;
    return OCTAX_OK;
}

int32_t octax_pool_step(octax_pool *p, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                        uint32_t obs_slots, float *d_reward, uint8_t *d_done) {
    if (!p || !d_action || !d_reward || !d_done)
        return fail(OCTAX_E_INVALID, "octax_pool_step: NULL pool, action, reward or done");
    if (K == 0) return fail(OCTAX_E_INVALID, "octax_pool_step: K == 0");
    if (d_obs && obs_slots == 0) return fail(OCTAX_E_INVALID, "octax_pool_step: obs_slots == 0");
    octax_engine *g = p->eng;
    hipError_t e = hipSuccess;
    if (p->table_dirty) e = upload_table(p);
    if (e == hipSuccess) e = launch_steps(g, K, d_action, d_obs, obs_slots, d_reward, d_done, g->stream);
    return e == hipSuccess ? OCTAX_OK : hip_fail(e, "octax_pool_step");
}

int32_t octax_pool_info(const octax_pool *p, uint32_t *capacity, uint32_t *free_slots,
                        uint32_t *largest_free, uint32_t *groups) {
    if (!p) return fail(OCTAX_E_INVALID, "octax_pool_info: pool is NULL");
    uint32_t total = 0, largest = 0;
    for (const auto &r : p->free_ranges) {
        total += r.second;
        largest = std::max(largest, r.second);
    }
    if (capacity) *capacity = p->capacity;
    if (free_slots) *free_slots = total;
    if (largest_free) *largest_free = largest;
    if (groups) *groups = (uint32_t)p->groups.size();
    return OCTAX_OK;
}

int32_t octax_pool_get_state(octax_pool *p, uint32_t first, uint32_t count, octax_env_state *h_out) {
    if (!p) return fail(OCTAX_E_INVALID, "octax_pool_get_state: pool is NULL");
    return octax_get_state(p->eng, first, count, h_out);
}

int32_t octax_pool_destroy(octax_pool *p) {
    if (!p) return OCTAX_OK;
    const int32_t rc = check_device_error(p->eng, "octax_pool_destroy");
    delete p;
    return rc;
}

}  // extern "C"
