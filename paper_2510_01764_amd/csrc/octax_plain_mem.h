// Memory policy of the lane-per-env kernels (plain CHIP-8 step and the
// SUPER-CHIP step): memory, display and stack accessed in HBM/L2 through the
// env's own slices of the state arrays.  See octax_core.h for the operations
// a memory policy supplies.
#pragma once

#include "octax_core.h"

namespace octax {

struct PlainMem {
    uint8_t *ram;
    uint64_t *fb;
    uint32_t *stack;
    uint64_t dirty;

    __device__ __forceinline__ uint32_t fetch(uint32_t pc) const {
        return ((uint32_t)ram[pc] << 8) | ram[(pc + 1) & 0xFFF];
    }
    __device__ __forceinline__ u32x4 load_bytes(uint32_t a, uint32_t count) const {
        u32x4 v = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; k++)
            if ((uint32_t)k < count) or_byte(v, k, ram[(a + k) & 0xFFF]);
        return v;
    }
    __device__ __forceinline__ void store_bytes(uint32_t a, uint32_t count, u32x4 bytes) {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if ((uint32_t)k < count) {
                const uint32_t ak = (a + k) & 0xFFF;
                ram[ak] = (uint8_t)byte_of(bytes, k);
                dirty |= 1ull << (ak >> 6);
            }
        }
    }
    // XOR rows of the sprite onto the display; bits past x = 63 fall off the
    // right of the shifted mask, rows past y = 31 are skipped.  With the
    // pixel-wrap quirk the byte is rotated instead and rows wrap to the top.
    __device__ __forceinline__ uint32_t draw(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n, bool wrap) {
        uint64_t hit = 0;
        for (uint32_t r = 0; r < n; r++) {
            uint32_t yy = y0 + r;
            if (yy >= 32 && !wrap) break;
            yy &= 31;
            const uint64_t s = (uint64_t)ram[(I + r) & 0xFFF] << 56;
            const uint64_t m = wrap ? __builtin_rotateright64(s, x0) : s >> x0;
            const uint64_t row = fb[yy];
            hit |= row & m;
            fb[yy] = row ^ m;
        }
        return hit != 0;
    }
    __device__ __forceinline__ void clear() {
        for (int y = 0; y < 32; y++) fb[y] = 0;
    }
    __device__ __forceinline__ uint32_t stack_get(uint32_t i) const {
        const uint32_t w = stack[i >> 1];
        return (i & 1) ? (w >> 16) : (w & 0xFFFF);
    }
    __device__ __forceinline__ void stack_set(uint32_t i, uint32_t v) {
        const uint32_t w = stack[i >> 1];
        stack[i >> 1] = (i & 1) ? ((w & 0xFFFFu) | (v << 16)) : ((w & 0xFFFF0000u) | v);
    }
};

}  // namespace octax
