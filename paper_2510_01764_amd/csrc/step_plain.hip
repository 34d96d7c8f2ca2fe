// Plain step kernel: one env per lane, every field of the env's state read
// from and written back to HBM on every step, memory and display accessed in
// HBM/L2, observations stored by each lane for its own env.  This is the
// direct lane-per-instance mapping of a vectorised environment step and the
// baseline the fused kernel is measured against.
#include "octax_core.h"
#include "octax_kernels.h"
#include "octax_plain_mem.h"

namespace octax {
namespace {

// One environment step of emulation with `key` held.
__device__ __forceinline__ void plain_env_step(Core &c, PlainMem &mem, uint32_t key, uint32_t ipf, uint32_t fs,
                                               uint32_t quirks) {
    for (uint32_t f = 0; f < fs; f++) {
        for (uint32_t i = 0; i < ipf; i++)
            if (exec_one(c, mem, key, quirks) && (quirks & kQuirkDisplayWait)) break;   // waits for the next frame
        tick(c);
    }
}

// The display in frame-ring order (see pack_frame).
__device__ __forceinline__ void pack_display(const uint64_t *fb, uint32_t pw[64]) {
    uint32_t hi[32], lo[32];
#pragma unroll
    for (int r = 0; r < 32; r++) {
        const uint64_t row = fb[31 - r];
        hi[r] = (uint32_t)(row >> 32);
        lo[r] = (uint32_t)row;
    }
    rows_to_cols(hi, lo);
    pack_frame(hi, lo, pw);
}

__global__ __launch_bounds__(256) void step_plain_kernel(State s, Roms roms, StepIO io, uint32_t k) {
    const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
    if (!slot_live(s, slot)) return;
    const uint32_t E = s.num;
    const uint32_t env = s.env_of[slot];
    const uint32_t rom = s.rom_of[slot];
    const uint32_t desc = roms.desc[rom];
    const uint32_t desc2 = roms.desc2 ? roms.desc2[rom] : kDesc2Default;

    Core c;
    uint32_t head;
    load_core(s, slot, c, head);
    const uint32_t key = sticky_key(roms, c, action_key(roms, rom, desc, io.action[(size_t)k * E + env]));
    PlainMem mem{s.ram + (size_t)slot * kMem, s.fb + (size_t)slot * 32, s.stack + (size_t)slot * 8,
                 s.dirty[slot]};

    plain_env_step(c, mem, key, io.ipf, io.frame_skip, roms.quirks);

    const int32_t score = score_of(c.r, desc, desc2);
    int32_t prev = s.prev[slot];
    const float reward = (float)(score - prev);
    const uint32_t term = terminated_of(c.r, desc, desc2);
    uint32_t t = s.t[slot] + 1;
    const uint32_t hor = s.horizon[slot];
    const uint32_t trunc = (hor != 0) && (t >= hor);
    const uint32_t done = term | (trunc << 1);
    io.reward[(size_t)k * E + env] = reward;
    io.done[(size_t)k * E + env] = (uint8_t)done;

    uint32_t *ring = s.cols + (size_t)slot * 256;
    uint8_t *obs = io.obs ? io.obs + ((size_t)(k % io.obs_slots) * E + env) * kObsBytes : nullptr;
    if (done) {
        // Automatic reset (Section 3.4): restore the pages written since the
        // last reset, clear everything else; the RNG stream continues.  Then
        // the reset's emulation steps (start-up sequence, no-op reset).
        const uint8_t *img = roms.image + (size_t)rom * kMem;
        uint64_t d = mem.dirty;
        while (d) {
            const uint32_t p = __builtin_ctzll(d);
            d &= d - 1;
            const uint4 *src = reinterpret_cast<const uint4 *>(img + p * 64);
            uint4 *dst = reinterpret_cast<uint4 *>(mem.ram + p * 64);
            for (int q = 0; q < 4; q++) dst[q] = src[q];
        }
        mem.dirty = 0;
        reset_core(c);
        mem.clear();
        for (int q = 0; q < 8; q++) mem.stack[q] = 0;
        if (roms.w.reset_steps)
            run_reset_steps(roms, rom, c, [&](uint32_t rk) { plain_env_step(c, mem, rk, io.ipf, io.frame_skip, roms.quirks); });
        head = 0;
        t = 0;
        prev = score_of(c.r, desc, desc2);   // the score after the reset's steps
    } else {
        prev = score;
        head = (head + 1) & 3;
    }
    uint32_t pw[64];
    pack_display(mem.fb, pw);
    // The frame ring gets the new display; after a reset the stack restarts
    // with it in all four slots.
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
        if (done || q == head) {
            uint4 *dst = reinterpret_cast<uint4 *>(ring + q * 64);
#pragma unroll
            for (int w = 0; w < 16; w++) dst[w] = make_uint4(pw[4 * w], pw[4 * w + 1], pw[4 * w + 2], pw[4 * w + 3]);
        }
    }
    if (obs) {
        // frames 0..2: the three older ring entries, oldest first, then the display
        for (uint32_t fr = 0; fr < 3; fr++) {
            const uint32_t *src = ring + ((head + 1 + fr) & 3) * 64;
            uint8_t *o = obs + fr * 2048;
            for (int w = 0; w < 64; w++) {
                const uint32_t word = src[w];
                store16(o + 16 * w, word & 0xFFFF);
                store16(o + 1024 + 16 * w, word >> 16);
            }
        }
        uint8_t *o = obs + 3 * 2048;
#pragma unroll
        for (int w = 0; w < 64; w++) {
            store16(o + 16 * w, pw[w] & 0xFFFF);
            store16(o + 1024 + 16 * w, pw[w] >> 16);
        }
    }
    store_core(s, slot, c, head);
    s.t[slot] = t;
    s.prev[slot] = prev;
    s.dirty[slot] = mem.dirty;
}

// The emulation steps of a reset (start-up sequence, no-op reset) for the
// slots [first, first + count) whose env has mask[env] != 0, after power-on;
// then the score baseline and the frame ring (the display four times).
__global__ __launch_bounds__(256) void reset_steps_kernel(State s, Roms roms, const uint8_t *mask,
                                                          uint32_t first, uint32_t count) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t slot = first + k;
    if (slot >= s.num) return;
    if (mask && !mask[s.env_of[slot]]) return;
    const uint32_t rom = s.rom_of[slot];
    const uint32_t desc = roms.desc[rom];
    const uint32_t desc2 = roms.desc2 ? roms.desc2[rom] : kDesc2Default;
    Core c;
    uint32_t head;
    load_core(s, slot, c, head);
    PlainMem mem{s.ram + (size_t)slot * kMem, s.fb + (size_t)slot * 32, s.stack + (size_t)slot * 8,
                 s.dirty[slot]};
    run_reset_steps(roms, rom, c, [&](uint32_t rk) { plain_env_step(c, mem, rk, roms.w.ipf, roms.w.frame_skip, roms.quirks); });
    uint32_t pw[64];
    pack_display(mem.fb, pw);
    uint4 *ring = reinterpret_cast<uint4 *>(s.cols + (size_t)slot * 256);
    for (uint32_t q = 0; q < 4; q++)
        for (int w = 0; w < 16; w++) ring[q * 16 + w] = make_uint4(pw[4 * w], pw[4 * w + 1], pw[4 * w + 2], pw[4 * w + 3]);
    store_core(s, slot, c, head);
    s.prev[slot] = score_of(c.r, desc, desc2);
    s.dirty[slot] = mem.dirty;
}

}  // namespace

hipError_t launch_reset_steps(const State &s, const Roms &r, const uint8_t *mask, uint32_t first,
                              uint32_t count, hipStream_t st) {
    if (count == 0 || !r.w.reset_steps) return hipSuccess;
    hipLaunchKernelGGL(reset_steps_kernel, dim3((count + 255) / 256), dim3(256), 0, st, s, r, mask, first, count);
    return hipGetLastError();
}

hipError_t launch_step_plain(const State &s, const Roms &r, const StepIO &io, hipStream_t st) {
    const uint32_t blocks = (s.num + 255) / 256;
    for (uint32_t k = 0; k < io.K; k++) {
        hipLaunchKernelGGL(step_plain_kernel, dim3(blocks), dim3(256), 0, st, s, r, io, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace octax
