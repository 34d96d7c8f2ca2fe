// Host-visible launch interface of the liboctax kernels (implemented in the
// .hip files, called from octax_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "octax_device.h"

namespace octax {

struct StepIO {
    const int32_t *action;  // [K][E]
    uint8_t *obs;           // [obs_slots][E][8192] or nullptr
    float *reward;          // [K][E]
    uint8_t *done;          // [K][E]
    uint32_t K;
    uint32_t obs_slots;
    uint32_t ipf;
    uint32_t frame_skip;
};

// LDS layout of the fused kernel, shared with the host so that both agree on
// the size of a block's page pool.  A block of IPW envs (2 * IPW threads)
// owns IPW / 256 of a CU's 160 KB:
//   * the displays: IPW x kFbStride u64 (32 rows + 1 pad row per env);
//   * written-page cache slots: IPW x (64 x slots + 8) bytes;
//   * the writers' staging: (IPW / 64) waves x kStageEnvs x kStageStride u32;
//   * reward, done, a step budget and two step counters per env, and
//     two step counters per wave;
//   * the page pool: everything left, in 64-byte pages.
constexpr uint32_t kFbStride = 33;
constexpr uint32_t kStageEnvs = 4;
constexpr uint32_t kStageStride = 68;
constexpr uint32_t fused_cache_slots(uint32_t ipw) { return ipw == 64 ? 2 : 3; }
constexpr uint32_t fused_lds_bytes(uint32_t ipw) { return 163840u / (256u / ipw); }
constexpr uint32_t fused_fixed_lds(uint32_t ipw) {
    return ipw * kFbStride * 8 + ipw * (64 * fused_cache_slots(ipw) + 8) + (ipw / 64) * kStageEnvs * kStageStride * 4 +
           ipw * (4 + 1 + 1 + 2) + 2 * 4 * (ipw / 64);
}
constexpr uint32_t fused_pool_pages(uint32_t ipw) { return (fused_lds_bytes(ipw) - fused_fixed_lds(ipw)) / 64; }

// The page pool of a fused block holds power-on memory pages read from LDS
// instead of HBM: pool page 0 is a page of zeros (every page past a ROM's
// last byte and below 0x200 outside the font), pool pages 1 and 2 hold
// memory pages 1 and 2 (the font at 0x050..0x09F, the same in every image),
// and from pool page kPoolFixedPages on, the program pages (from 0x200) of
// the block's most frequent ROMs, back to back.  The host describes them in
// a table of kPoolRoms entries per block, two u32 each:
//   [0] ROM id, kPoolEnd after the last entry (first entry kPoolEnd: the
//       block holds no env);
//   [1] staged pages | program pages << 8 | first pool page << 16
//       (program pages = ceil(ROM bytes / 64); the last ROM staged may have
//       fewer staged pages than program pages when the pool is full).
constexpr uint32_t kPoolRoms = 32;
constexpr uint32_t kPoolFixedPages = 3;
constexpr uint32_t kPoolEnd = 0xFFFFFFFFu;

// Fused-kernel tuning.
struct FusedCfg {
    uint32_t envs_per_block;      // 64, 128 or 256
    uint32_t rom_in_lds;          // stage the block's ROM program pages in its LDS page pool
    const uint32_t *block_roms;   // [blocks][kPoolRoms][2] page-pool table (see above)
    uint64_t wait_ticks;          // longest wait of a wave for its partner, in device wall-clock ticks
    uint32_t *err;                // device error word: bit 0 set when a wait gave up
    uint64_t *stamps;             // [stamp_steps][ceil(E / 64)][2] step start / end clocks, or nullptr
    uint32_t stamp_steps;
    const uint8_t *budget;        // [slots] steps of the launch per slot (at most K), or nullptr: K for all
};

hipError_t launch_step_plain(const State &s, const Roms &r, const StepIO &io, hipStream_t st);
hipError_t launch_step_fused(const State &s, const Roms &r, const StepIO &io, const FusedCfg &f,
                             hipStream_t st);
// Power-on state for the slots whose env has mask[env] != 0 (all if mask is
// null).  full_ram: copy every page of the image (first reset after
// allocation), else only pages marked dirty.
hipError_t launch_reset(const State &s, const Roms &r, const uint8_t *mask, bool full_ram,
                        hipStream_t st);
// The same for slots [first, first + count) only.
hipError_t launch_reset_range(const State &s, const Roms &r, const uint8_t *mask, bool full_ram,
                              uint32_t first, uint32_t count, hipStream_t st);
// The emulation steps of a reset (start-up sequence, no-op reset) after
// power-on, for the slots of [first, first + count) selected by mask; a no-op
// when the wrappers run no steps.  launch_reset_range calls it.
hipError_t launch_reset_steps(const State &s, const Roms &r, const uint8_t *mask, uint32_t first,
                              uint32_t count, hipStream_t st);
// Write the observation of every env from its frame ring.
hipError_t launch_observe(const State &s, uint8_t *obs, hipStream_t st);
// 64-bit FNV-1a of every env's state in octax_env_state form, at its env index.
hipError_t launch_digest(const State &s, uint64_t *out, hipStream_t st);
// SUPER-CHIP: K steps; power-on of the display, frame ring, mode and flag
// registers of the selected slots of [first, first + count), then the
// reset's emulation steps (launch_reset_range calls it after the CHIP-8
// part); observations ([E][4][128][64]) from the frame ring.
hipError_t launch_step_schip(const State &s, const Roms &r, const StepIO &io, hipStream_t st);
hipError_t launch_schip_reset(const State &s, const Roms &r, const uint8_t *mask, uint32_t first, uint32_t count,
                              hipStream_t st);
hipError_t launch_schip_observe(const State &s, uint8_t *obs, hipStream_t st);

}  // namespace octax

namespace octax {

// Flat per-env state used to move envs between the SoA arrays and the host.
struct RawState {
    uint32_t regs[4];
    uint32_t pc_i;
    uint32_t misc;
    uint32_t t;
    int32_t prev;
    uint64_t rng;
    uint64_t dirty;
    uint32_t stack[8];
    uint64_t fb[32];
    uint32_t cols[256];
    uint8_t ram[4096];
};

// Gather slots slot_list[0..count) into raw[0..count), or scatter back.
hipError_t launch_pack(const State &s, const uint32_t *slot_list, uint32_t count, RawState *raw,
                       hipStream_t st);
hipError_t launch_unpack(const State &s, const uint32_t *slot_list, uint32_t count,
                         const RawState *raw, hipStream_t st);

}  // namespace octax
