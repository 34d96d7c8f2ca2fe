// Reset and observation kernels (Section 3.2, ROM loading and initialization;
// Section 3.2, Environment integration: the (4, 64, 32) frame stack).
#include "octax_core.h"
#include "octax_kernels.h"

namespace octax {
namespace {

// One thread per slot: registers, display, stack, frame ring, counters.
__global__ __launch_bounds__(256) void reset_regs_kernel(State s, const uint8_t *mask, uint32_t first,
                                                         uint32_t count) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t slot = first + k;
    if (slot >= s.num) return;
    const uint32_t env = s.env_of[slot];
    if (mask && !mask[env]) return;
    const uint32_t E = s.num;
    s.regs[0 * E + slot] = 0;
    s.regs[1 * E + slot] = 0;
    s.regs[2 * E + slot] = 0;
    s.regs[3 * E + slot] = 0;
    s.pc_i[slot] = kProgram;
    s.misc[slot] = 0;
    s.t[slot] = 0;
    s.prev[slot] = 0;   // V[score_reg] of the power-on state
    uint4 z = make_uint4(0, 0, 0, 0);
    uint4 *fb = reinterpret_cast<uint4 *>(s.fb + (size_t)slot * 32);
    for (int q = 0; q < 16; q++) fb[q] = z;
    uint4 *stk = reinterpret_cast<uint4 *>(s.stack + (size_t)slot * 8);
    stk[0] = z;
    stk[1] = z;
    uint4 *ring = reinterpret_cast<uint4 *>(s.cols + (size_t)slot * 256);
    for (int q = 0; q < 64; q++) ring[q] = z;
}

// 256 threads per slot, 16 bytes each: memory back to the ROM's power-on
// image (all pages, or only those written since the last reset), then the
// dirty mask is cleared by the last wave to read it.
__global__ __launch_bounds__(256) void reset_ram_kernel(State s, Roms roms, const uint8_t *mask,
                                                        uint32_t full, uint32_t first) {
    const uint32_t slot = first + blockIdx.x;
    if (slot >= s.num) return;
    const uint32_t env = s.env_of[slot];
    if (mask && !mask[env]) return;
    const uint32_t q = threadIdx.x;          // 16-byte chunk, page q / 4
    const uint64_t dirty = s.dirty[slot];
    if (full || ((dirty >> (q >> 2)) & 1)) {
        const uint4 *src = reinterpret_cast<const uint4 *>(roms.image + (size_t)s.rom_of[slot] * kMem);
        uint4 *dst = reinterpret_cast<uint4 *>(s.ram + (size_t)slot * kMem);
        dst[q] = src[q];
    }
    __syncthreads();
    if (q == 0) s.dirty[slot] = 0;
}

// One thread per 16 bytes of observation: frame fr, piece q of the packed
// frame (q < 64: low half of word q; else high half of word q - 64).
__global__ __launch_bounds__(256) void observe_kernel(State s, uint8_t *obs) {
    const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t slot = (uint32_t)(gid >> 9);
    if (!slot_live(s, slot)) return;
    const uint32_t piece = (uint32_t)(gid & 511);
    const uint32_t fr = piece >> 7, q = piece & 127;
    const uint32_t head = s.misc[slot] >> 24 & 3;
    const uint32_t word = s.cols[(size_t)slot * 256 + ((head + 1 + fr) & 3) * 64 + (q & 63)];
    store16(obs + (size_t)s.env_of[slot] * kObsBytes + fr * 2048 + 16 * q, q < 64 ? (word & 0xFFFF) : (word >> 16));
}

}  // namespace

// 64-bit FNV-1a (Fowler, Noll and Vo: offset basis 0xcbf29ce484222325,
// prime 0x100000001b3; each byte is XOR-ed in, then the hash multiplied).
__device__ __forceinline__ void fnv_bytes(uint64_t &h, uint64_t w, int n) {
    for (int i = 0; i < n; i++) {
        h ^= (w >> (8 * i)) & 0xFF;
        h *= 0x100000001b3ull;
    }
}

// One thread per slot: the digest of the env's state in octax_env_state form
// (the bytes octax_get_state returns, in that order), written at its env.
__global__ __launch_bounds__(256) void digest_kernel(State s, uint64_t *out) {
    const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
    if (!slot_live(s, slot)) return;
    const uint32_t E = s.num;
    uint64_t h = 0xcbf29ce484222325ull;
    for (int w = 0; w < 4; w++) fnv_bytes(h, s.regs[w * E + slot], 4);   // V0..VF
    const uint32_t pc_i = s.pc_i[slot], misc = s.misc[slot];
    fnv_bytes(h, (pc_i >> 16) & 0xFFF, 2);                                // I
    fnv_bytes(h, pc_i & 0xFFF, 2);                                        // PC
    fnv_bytes(h, misc & 15, 1);                                           // SP
    fnv_bytes(h, (misc >> 8) & 0xFF, 1);                                  // DT
    fnv_bytes(h, (misc >> 16) & 0xFF, 1);                                 // ST
    fnv_bytes(h, ((misc >> 26) & 31) ^ 16, 1);                            // previous key
    for (int w = 0; w < 8; w++) fnv_bytes(h, s.stack[(size_t)slot * 8 + w], 4);
    fnv_bytes(h, s.t[slot], 4);
    fnv_bytes(h, (uint32_t)s.prev[slot], 4);
    fnv_bytes(h, s.rng[slot], 8);
    const uint64_t *ram = reinterpret_cast<const uint64_t *>(s.ram + (size_t)slot * kMem);
    for (int q = 0; q < 512; q++) fnv_bytes(h, ram[q], 8);
    for (int y = 0; y < 32; y++) fnv_bytes(h, s.fb[(size_t)slot * 32 + y], 8);
    // the three earlier frames, oldest first, from the packed frame ring:
    // pixel (x, y) is bit (x >= 32 ? 16 : 0) + (y & 15) of word 2 (x & 31) + (y >> 4)
    const uint32_t head = (misc >> 24) & 3;
    for (uint32_t f = 0; f < 3; f++) {
        const uint32_t *frame = s.cols + (size_t)slot * 256 + ((head + 1 + f) & 3) * 64;
        for (uint32_t y = 0; y < 32; y++) {
            uint64_t row = 0;
            for (uint32_t x = 0; x < 64; x++) {
                const uint32_t bit = (frame[2 * (x & 31) + (y >> 4)] >> ((x >= 32 ? 16 : 0) + (y & 15))) & 1;
                row |= (uint64_t)bit << (63 - x);
            }
            fnv_bytes(h, row, 8);
        }
    }
    out[s.env_of[slot]] = h;
}

hipError_t launch_digest(const State &s, uint64_t *out, hipStream_t st) {
    if (s.num == 0) return hipSuccess;
    hipLaunchKernelGGL(digest_kernel, dim3((s.num + 255) / 256), dim3(256), 0, st, s, out);
    return hipGetLastError();
}

hipError_t launch_reset(const State &s, const Roms &r, const uint8_t *mask, bool full_ram,
                        hipStream_t st) {
    return launch_reset_range(s, r, mask, full_ram, 0, s.num, st);
}

hipError_t launch_reset_range(const State &s, const Roms &r, const uint8_t *mask, bool full_ram,
                              uint32_t first, uint32_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(reset_ram_kernel, dim3(count), dim3(256), 0, st, s, r, mask, full_ram ? 1u : 0u, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_regs_kernel, dim3((count + 255) / 256), dim3(256), 0, st, s, mask, first, count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (r.schip) return launch_schip_reset(s, r, mask, first, count, st);
    return launch_reset_steps(s, r, mask, first, count, st);
}

hipError_t launch_observe(const State &s, uint8_t *obs, hipStream_t st) {
    const uint64_t threads = (uint64_t)s.num * 512;
    hipLaunchKernelGGL(observe_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st, s, obs);
    return hipGetLastError();
}

}  // namespace octax

namespace octax {
namespace {

// One block per env: copy every field between the SoA arrays and RawState.
__global__ __launch_bounds__(256) void pack_kernel(State s, const uint32_t *slots, uint32_t count,
                                                   RawState *raw, uint32_t to_raw) {
    const uint32_t k = blockIdx.x;
    if (k >= count) return;
    const uint32_t slot = slots[k];
    const uint32_t E = s.num;
    const uint32_t q = threadIdx.x;
    RawState &r = raw[k];
    uint4 *ram = reinterpret_cast<uint4 *>(s.ram + (size_t)slot * kMem);
    uint4 *rram = reinterpret_cast<uint4 *>(r.ram);
    uint32_t *cols = s.cols + (size_t)slot * 256;
    if (to_raw) {
        rram[q] = ram[q];
        r.cols[q] = cols[q];
        if (q < 32) r.fb[q] = s.fb[(size_t)slot * 32 + q];
        if (q < 8) r.stack[q] = s.stack[(size_t)slot * 8 + q];
        if (q < 4) r.regs[q] = s.regs[q * E + slot];
        if (q == 0) {
            r.pc_i = s.pc_i[slot];
            r.misc = s.misc[slot];
            r.t = s.t[slot];
            r.prev = s.prev[slot];
            r.rng = s.rng[slot];
            r.dirty = s.dirty[slot];
        }
    } else {
        ram[q] = rram[q];
        cols[q] = r.cols[q];
        if (q < 32) s.fb[(size_t)slot * 32 + q] = r.fb[q];
        if (q < 8) s.stack[(size_t)slot * 8 + q] = r.stack[q];
        if (q < 4) s.regs[q * E + slot] = r.regs[q];
        if (q == 0) {
            s.pc_i[slot] = r.pc_i;
            s.misc[slot] = r.misc;
            s.t[slot] = r.t;
            s.prev[slot] = r.prev;
            s.rng[slot] = r.rng;
            s.dirty[slot] = r.dirty;
        }
    }
}

}  // namespace

hipError_t launch_pack(const State &s, const uint32_t *slot_list, uint32_t count, RawState *raw,
                       hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(count), dim3(256), 0, st, s, slot_list, count, raw, 1u);
    return hipGetLastError();
}

hipError_t launch_unpack(const State &s, const uint32_t *slot_list, uint32_t count,
                         const RawState *raw, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(count), dim3(256), 0, st, s, slot_list, count,
                       const_cast<RawState *>(raw), 0u);
    return hipGetLastError();
}

}  // namespace octax
