// Device-side definitions shared by the step kernels of liboctax: the
// structure-of-arrays layout of the env state in HBM, packed register access,
// the CXNN random stream and the built-in font.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace octax {

constexpr uint32_t kMem = 4096;
constexpr uint32_t kProgram = 0x200;
constexpr uint32_t kFont = 0x050;
constexpr uint32_t kKeyNone = 16;      // "no key held"
constexpr uint32_t kObsBytes = 8192;   // [4][64][32]
constexpr uint32_t kSchipObsBytes = 32768;   // SUPER-CHIP: [4][128][64]
constexpr uint32_t kBigFont = 0x0A0;          // SUPER-CHIP 8x10 digit glyphs, 10 bytes each

// Env state in device memory, one entry per slot (see octax_host.cpp for the
// byte budget).  Small per-env fields are stored field-major ([field][slot])
// so that a lane-per-env kernel reads them coalesced; big per-env blocks
// (memory, display, frame ring) are slot-major.
struct State {
    uint32_t *regs;      // [4][E]  V0..V15, register 4w+b in byte b of regs[w][slot]
    uint32_t *pc_i;      // [E]     PC | I << 16
    uint32_t *misc;      // [E]     SP | DT << 8 | ST << 16 | ring head << 24 | (previous key ^ 16) << 26
    uint32_t *stack;     // [E][8]  16 return addresses, two per word (entry 2k in the low half)
    uint32_t *t;         // [E]     steps since reset
    int32_t *prev;       // [E]     V[score_reg] after the previous step
    uint64_t *rng;       // [E]     SplitMix64 state
    uint64_t *dirty;     // [E]     bit p: 64-byte page p written since reset
    uint64_t *fb;        // [E][32] display rows, bit 63 - x = pixel (x, y)
    uint32_t *cols;      // [E][4][64] frame ring of packed frames (see pack_frame), slot = misc head
    uint8_t *ram;        // [E][4096]
    // SUPER-CHIP engines only (null otherwise):
    uint64_t *hfb;       // [E][64][2] 128x64 display: row y = hfb[2p] (x 0..63) and hfb[2p+1]
                         //            (x 64..127), p = (y + row offset) & 63, bit 63 - (x mod 64) =
                         //            pixel (x, y)
    uint64_t *hring;     // [E][5][128] frame ring of displays in the same row form, p = y
    uint32_t *sx;        // [E][4] word 0: 1 = 128x64 mode | row offset of hfb << 8; words 1, 2: flag
                         //        registers 0..7, one byte each;
                         //        word 3: ring slot of the display and per-step observation info
    const uint32_t *rom_of;   // [E] ROM id
    const uint32_t *horizon;  // [E]
    const uint32_t *env_of;   // [E] env index (output position) of each slot
    const uint8_t *occupied;  // [E] slot holds an env (serving pool); null: every slot does
    uint32_t num;             // E
};

// Slot holds an env that steps.
__device__ __forceinline__ bool slot_live(const State &s, uint32_t slot) {
    return slot < s.num && (s.occupied == nullptr || s.occupied[slot] != 0);
}

// Per-ROM tables.
// Environment wrappers (Section 3.2: start-up sequences that skip menus,
// no-op reset, sticky actions), all off when zero / null, and the emulation
// rate the steps of a reset run at.
struct Wrap {
    const uint8_t *startup;   // [R][17]: start-up steps (0..16), then the key held in each (16 = none)
    uint32_t sticky_q24;      // P(the previous step's key is held again) * 2^24, 0..2^24
    uint32_t noop_max;        // no-op steps after a reset: uniform in 0..noop_max
    uint32_t reset_steps;     // nonzero when a reset runs emulation steps (start-up or no-op)
    uint32_t ipf;             // instructions per frame
    uint32_t frame_skip;      // frames per step
};

struct Roms {
    const uint8_t *image;    // [R][4096] power-on memory: font at 0x50, program at 0x200
    const uint8_t *keys;     // [R][16]
    const uint32_t *desc;    // [R] score_reg | term_reg << 8 | term_value << 16 | num_actions << 24
    // Game descriptors beyond desc, or null (all zero): [R] score mode |
    // term2 op << 2 | term2 reg << 4 | term2 value << 8 (score mode 1 = BCD
    // difference; term2 op 0 none, 1 ==, 2 >=).
    const uint32_t *desc2;
    uint32_t quirks;         // quirk flags of the whole batch (bit 0 = the VIP base profile)
    uint32_t profile;        // nonzero when quirks != base or desc2 is set
    uint32_t schip;          // 1: SUPER-CHIP platform (128x64 display, its instructions)
    Wrap w;
};

// ---------------------------------------------------------------------------
// V registers packed four to a 32-bit word (byte b of word w is V[4w+b]),
// held as one 4-word vector value.  Indexing it with a per-lane register
// number lowers to compare/select on the four VGPRs (never to memory).
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Regs {
    u32x4 w;
};

// V[x]: v_perm picks byte x & 7 out of a register pair (selector 0x0C gives a
// zero byte), the pair chosen by bit 3 of x.
__device__ __forceinline__ uint32_t vget(const Regs &r, uint32_t x) {
    const uint32_t sel = 0x0C0C0C00u | (x & 7);
    const uint32_t lo = __builtin_amdgcn_perm(r.w.y, r.w.x, sel);
    const uint32_t hi = __builtin_amdgcn_perm(r.w.w, r.w.z, sel);
    return (x & 8) ? hi : lo;
}

__device__ __forceinline__ void vset(Regs &r, uint32_t x, uint32_t val) {
    const uint32_t sh = (x & 3) * 8;
    const uint32_t m = 0xFFu << sh;
    const uint32_t s = (val & 0xFFu) << sh;
    const uint32_t q = x >> 2;
    r.w.x = (q == 0) ? ((r.w.x & ~m) | s) : r.w.x;
    r.w.y = (q == 1) ? ((r.w.y & ~m) | s) : r.w.y;
    r.w.z = (q == 2) ? ((r.w.z & ~m) | s) : r.w.z;
    r.w.w = (q == 3) ? ((r.w.w & ~m) | s) : r.w.w;
}

__device__ __forceinline__ void set_vf(Regs &r, uint32_t f) { r.w.w = (r.w.w & 0x00FFFFFFu) | (f << 24); }

// ---------------------------------------------------------------------------
// CXNN randomness: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  The
// state advances by the golden-ratio increment and the output is the
// 64-bit finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
// xor-shift 31) of the new state.  CXNN keeps the top byte.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix_next(uint64_t &s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint32_t rnd_byte(uint64_t &s) { return (uint32_t)(splitmix_next(s) >> 56); }

// 16-byte observation store of one thread (the plain kernel and reset, each
// thread writing its own env's observation): plain stores, which on MI355X
// stream to HBM faster than hinted ones here (28 against 94 M env steps/s for
// the plain kernel, measured).
__device__ __forceinline__ void store_stream(void *dst, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    u32x4 v = {a, b, c, d};
    *reinterpret_cast<u32x4 *>(dst) = v;
}

// ---------------------------------------------------------------------------
// Observation expansion: four column bits -> four 0/1 bytes.
// n * 0x00204081 places bit j of n at bit 8j (j = 0..3) with no carries
// between the copies; the mask keeps those bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread4(uint32_t col, uint32_t shift) {
    return (__builtin_amdgcn_ubfe(col, shift, 4) * 0x00204081u) & 0x01010101u;
}

// 32 pixels of one column (bit y = pixel y) -> 32 bytes at dst (16-byte aligned).
__device__ __forceinline__ void store_column(uint8_t *dst, uint32_t col) {
    store_stream(dst, spread4(col, 0), spread4(col, 4), spread4(col, 8), spread4(col, 12));
    store_stream(dst + 16, spread4(col, 16), spread4(col, 20), spread4(col, 24), spread4(col, 28));
}

// ---------------------------------------------------------------------------
// 32 x 64 bit-matrix transpose of one frame held in registers.
// rows[y] (bit 63 - x = pixel (x, y)) -> cols[x] (bit y = pixel (x, y)).
// Recursive block swap on 32-bit words (Warren, Hacker's Delight, 2nd ed.,
// section 7-3): five rounds swap the off-diagonal j x j blocks for
// j = 16, 8, 4, 2, 1.  It is applied to the high and low halves of the rows
// with the row order reversed, which yields bit y = row y.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void transpose32(uint32_t a[32]) {
    uint32_t m = 0x0000FFFFu;
#pragma unroll
    for (int j = 16; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
        for (int k = 0; k < 32; k = (k + j + 1) & ~j) {
            uint32_t t = (a[k] ^ (a[k + j] >> j)) & m;
            a[k] ^= t;
            a[k + j] ^= (t << j);
        }
    }
}

// Frame rows -> columns 0..63.  hi[r] must hold the high words of rows in
// reverse order (hi[r] = row[31 - r] >> 32) and lo[r] the low words.
__device__ __forceinline__ void rows_to_cols(uint32_t hi[32], uint32_t lo[32]) {
    transpose32(hi);   // hi[x] = column x (x = 0..31)
    transpose32(lo);   // lo[x] = column 32 + x
}

// Packed frame: 64 words in observation store order.  The observation of a
// frame is 2048 bytes, [x][y]; word l holds in its low half the 16 pixels of
// bytes [16l, 16l + 16) (column l / 2, rows 16 (l % 2) ..) and in its high
// half those of bytes [1024 + 16l, ...) (column 32 + l / 2, same rows).
// Lane l of a wave therefore stores the two 16-byte pieces of word l and a
// wave's store instruction covers 1 KB of contiguous observation.
__device__ __forceinline__ void pack_frame(const uint32_t hi[32], const uint32_t lo[32], uint32_t w[64]) {
#pragma unroll
    for (int m = 0; m < 32; m++) {
        w[2 * m] = __builtin_amdgcn_perm(lo[m], hi[m], 0x05040100u);      // hi.lo16 | lo.lo16 << 16
        w[2 * m + 1] = __builtin_amdgcn_perm(lo[m], hi[m], 0x07060302u);  // hi.hi16 | lo.hi16 << 16
    }
}

// 16 pixel bits -> 16 bytes at dst.
__device__ __forceinline__ void store16(uint8_t *dst, uint32_t bits) {
    store_stream(dst, spread4(bits, 0), spread4(bits, 4), spread4(bits, 8), spread4(bits, 12));
}

// The low 16 pixel bits of `bits` as 16 bytes (byte i = bit i).
__device__ __forceinline__ u32x4 spread16(uint32_t bits) {
    return u32x4{spread4(bits, 0), spread4(bits, 4), spread4(bits, 8), spread4(bits, 12)};
}

// 16 observation bytes at dst (16-byte aligned), for stores in which a
// wavefront covers 1 KB of contiguous observation: plain stores for the fused
// kernel (the hint measured no faster there, and slower where the stores
// alone set the time), ...
__device__ __forceinline__ void store_obs(uint8_t *dst, u32x4 v) {
    *reinterpret_cast<u32x4 *>(dst) = v;
}
// ... and stores with the nontemporal hint for the SUPER-CHIP step, whose
// emulation reads displays, memory pages and state from HBM while its
// observations stream out: the hinted stores leave that data in the caches
// (8 % more env steps/s at 65,536 envs, measured against plain stores on the
// same device).
__device__ __forceinline__ void store_obs_nt(uint8_t *dst, u32x4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(dst));
}

}  // namespace octax
