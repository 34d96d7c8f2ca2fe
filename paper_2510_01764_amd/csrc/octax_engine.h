// Engine and graph objects of liboctax, shared by the host files of the
// library (octax_host.cpp: the environment API; octax_pool.cpp: the serving
// pool).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/octax.h"
#include "octax_kernels.h"

struct octax_engine {
    uint32_t E = 0, R = 0, ipf = 0, frame_skip = 0;
    uint32_t kernel = OCTAX_KERNEL_PLAIN;
    uint32_t placement = OCTAX_PLACE_IDENTITY;
    uint32_t envs_per_block = 256, rom_in_lds = 1;
    uint32_t schip = 0;                               // platform: 1 = SUPER-CHIP
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t device_bytes = 0;
    std::vector<void *> allocations;
    std::vector<uint32_t> env_of, slot_of, rom_of;   // host copies of the placement
    std::vector<uint32_t> rom_len;                    // ROM bytes per ROM
    std::vector<uint8_t> occupied;                    // serving pool: host copy of State::occupied (empty: all)
    octax::State s{};
    octax::Roms roms{};
    uint32_t *d_block_roms = nullptr;                 // [blocks][kPoolRoms][2] page-pool table, current tuning
    uint8_t *d_startup = nullptr;                     // [R][17] start-up sequences (Wrap::startup)
    uint32_t *d_slot_scratch = nullptr;               // slot lists for get/set_state
    octax::RawState *d_raw = nullptr;
    uint32_t raw_capacity = 0;
    int graphs = 0;
    uint64_t step_slots = 0;                          // longest step: ipf x frame_skip x (1 + reset steps)
    uint64_t wait_ticks = 0;                          // fused pair wait bound (device wall-clock ticks)
    uint64_t wait_override = 0;                       // octax_set_wait_limit (0: derived from the config)
    uint32_t *d_err = nullptr;                        // device error word of the fused kernel
    uint64_t *d_stamps = nullptr;                     // octax_set_step_clock (caller's buffer)
    uint32_t stamp_steps = 0;

    template <class T>
    hipError_t alloc(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16));
        if (e != hipSuccess) return e;
        allocations.push_back(q);
        device_bytes += count * sizeof(T);
        *p = static_cast<T *>(q);
        return hipSuccess;
    }
    void free_all() {
        for (void *p : allocations) (void)hipFree(p);
        allocations.clear();
    }
};

struct octax_graph {
    octax_engine *eng = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace octax {

// Record the message of a failure for octax_last_error and return code.
int32_t fail(int32_t code, const std::string &msg);
int32_t hip_fail(hipError_t e, const char *what);

// Check the environment-wrapper fields of a config and build the [R][17]
// start-up table (count, then 16 keys); returns an error message or null.
const char *check_wrappers(uint32_t sticky_q24, uint32_t noop_max, const uint8_t *h_startup_len,
                           const uint8_t *h_startup_keys, uint32_t R, std::vector<uint8_t> &table);
// Check the quirk flags and game descriptors of a config and build the [R]
// desc2 table (left empty when no descriptor array is given); returns an
// error message or null.
const char *check_profile(const octax_config *cfg, std::vector<uint32_t> &desc2);
// The wrapper parameters of a Roms (d_table: the device copy of the table).
Wrap make_wrap(const uint8_t *d_table, const std::vector<uint8_t> &table, uint32_t sticky_q24,
               uint32_t noop_max, uint32_t ipf, uint32_t frame_skip);

// The fused kernel's page-pool table (octax_kernels.h) for blocks of
// envs_per_block slots: per block, the ROMs of its (occupied) slots from the
// most to the least frequent, each with as many program pages as the pool
// still holds.
void block_rom_table(const octax_engine *g, std::vector<uint32_t> &table);

// Largest step, in instruction slots, that the fused kernel accepts: its
// paired waves wait for each other once per step, with a bound derived from
// this (see fused_wait_ticks).
constexpr uint64_t kFusedMaxStepSlots = 1ull << 20;
// Wait bound of the fused kernel's paired waves for a step of `slots`
// instruction slots: 0.25 s plus 16 us per slot (about ten times the slowest
// slot measured), in ticks of the device wall clock (wall_khz kHz).
uint64_t fused_wait_ticks(uint64_t slots, uint64_t wall_khz);
// Report (and clear) the fused kernel's error word; `what` names the call.
// Synchronizes the engine's stream.
int32_t check_device_error(octax_engine *g, const char *what);

// K fused or plain steps of every env of g on stream st.
hipError_t launch_steps(octax_engine *g, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                        uint32_t obs_slots, float *d_reward, uint8_t *d_done, hipStream_t st,
                        const uint8_t *d_budget = nullptr);

}  // namespace octax
