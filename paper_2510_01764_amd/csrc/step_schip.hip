// SUPER-CHIP step (the platform extension the paper names in Section 5: a
// 128x64 display and extra instructions) with two kinds of block:
//   * emulation, lane per env like the plain kernel (state, memory and the
//     1 KB display in HBM), 64 envs per block; it ends by writing the
//     display into the env's five-slot frame ring;
//   * observations, one 64-thread block per env: the env's frame ring is
//     staged in LDS and each thread writes 32-byte half columns, so a
//     block's stores cover the env's 32 KB of (4, 128, 64) observation
//     contiguously.
// One launch per step holds the emulation of step k and the observation
// blocks of step k - 1, so the two can share the machine; the ring has five
// slots so that the emulation of step k never writes a frame the
// observations of step k - 1 read.
//
// The SUPER-CHIP instructions and the readings taken for them:
//   00CN  scroll the display down N rows        (pixels of the current mode;
//   00FB  scroll right 4 columns                 a 64x32-mode pixel is a 2x2
//   00FC  scroll left 4 columns                  block of the 128x64 display)
//   00FD  stop: the program stays on this instruction
//   00FE  64x32 mode, display cleared;  00FF  128x64 mode, display cleared
//   DXYN  8xN sprite at (VX mod W, VY mod H) of the current mode; DXY0 a
//         16x16 sprite of 32 bytes; clipping, wrapping and VF as for CHIP-8
//   FX30  I = the 8x10 glyph of digit VX & 15 (10 bytes each at kBigFont)
//   FX75  flag registers 0..min(X, 7) = V0..; FX85 the reverse
// Every other instruction is the CHIP-8 one (exec_grouped), quirk flags
// included.
#include "octax_core.h"
#include "octax_grouped.h"
#include "octax_kernels.h"
#include "octax_plain_mem.h"

namespace octax {
namespace {

typedef unsigned __int128 u128;

// Each bit of a 16-bit pattern twice (bit i -> bits 2i and 2i + 1): a row of
// a 64x32-mode sprite on the 128x64 display.
__device__ __forceinline__ uint32_t double_bits(uint32_t b) {
    uint32_t x = b & 0xFFFF;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x | (x << 1);
}

struct SchipMem : PlainMem {
    uint64_t *hd;      // [64][2] display rows, row y of the display in physical row (y + roff) & 63
    const uint8_t *img;    // the ROM's power-on image
    uint32_t hires;
    uint32_t roff;     // row offset of the display (a scroll down moves it instead of the rows)
    uint32_t rpl0, rpl1;   // flag registers 0..3 and 4..7, byte k = register k

    // Memory reads: a page not written since the reset equals the ROM's
    // power-on image, which all envs of the ROM share (it stays in cache);
    // written pages come from the env's own memory.  Reads are aligned dwords
    // (which never straddle a page) through global-memory pointers: a byte at
    // a time, the scattered reads of 64 lanes are bound by the memory
    // system's request rate.
    __device__ __forceinline__ uint32_t rd4(uint32_t a) const {
        typedef __attribute__((address_space(1))) const uint32_t glb_u32;
        a &= 0xFFC;
        const glb_u32 *base = (const glb_u32 *)(((dirty >> (a >> 6)) & 1) ? ram : img);
        return base[a >> 2];
    }
    // Bytes a .. a + 4*NW - 1 (12-bit wrap) as NW words, byte k at bits
    // 8 (k % 4) of word k / 4: NW + 1 aligned dwords shifted into place.
    template <int NW>
    __device__ __forceinline__ void run(uint32_t a, uint32_t (&w)[NW]) const {
        uint32_t d[NW + 1];
#pragma unroll
        for (int i = 0; i <= NW; i++) d[i] = rd4((a & ~3u) + 4 * i);
#pragma unroll
        for (int i = 0; i < NW; i++) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], a & 3);
    }
    // The instruction word at pc: one dword, and the next one only when pc is
    // its last byte.
    __device__ __forceinline__ uint32_t fetch(uint32_t pc) const {
        const uint32_t d0 = rd4(pc);
        const uint32_t d1 = (pc & 3) == 3 ? rd4(pc + 1) : 0u;
        const uint32_t w = __builtin_amdgcn_alignbyte(d1, d0, pc & 3);
        return ((w & 0xFF) << 8) | ((w >> 8) & 0xFF);
    }
    // The grouped cycle's fetch: the word at pc and the top of the stack.
    __device__ __forceinline__ uint32_t fetch(uint32_t pc, uint32_t sp, uint32_t &ret) const {
        ret = stack_get((sp - 1) & 15);
        return fetch(pc);
    }
    // The top of the stack is read from memory at every fetch: nothing to update.
    __device__ __forceinline__ void stack_popped(uint32_t) const {}
    static constexpr bool kOneAccess = false;   // separate draw, load and store calls
    // count (1..16) bytes from a; bytes past count are unspecified (the
    // caller masks them).
    __device__ __forceinline__ u32x4 load_bytes(uint32_t a, uint32_t count) const {
        uint32_t w[4];
        run<4>(a, w);
        return u32x4{w[0], w[1], w[2], w[3]};
    }

    // Physical row p as a 128-bit word, pixel x at bit 127 - x.
    __device__ __forceinline__ u128 row(uint32_t y) const {
        return ((u128)hd[2 * y] << 64) | hd[2 * y + 1];
    }
    __device__ __forceinline__ void set_row(uint32_t y, u128 v) {
        hd[2 * y] = (uint64_t)(v >> 64);
        hd[2 * y + 1] = (uint64_t)v;
    }
    __device__ __forceinline__ uint32_t scale() const { return hires ? 1u : 2u; }

    // DXYN / DXY0 with the raw register values (see the header).  A sprite
    // row is at most 32 display pixels wide (16 pixels, doubled in the 64x32
    // mode), so it lands in two neighbouring 32-pixel words of the 128-pixel
    // row: word q = X / 32 shifted right by X % 32 and word q + 1 (mod 4 with
    // wrap, dropped past the right edge without) the rest.  The words and
    // shifts are the same for every row of the draw, so each display row
    // costs two 32-bit shifts and two 32-bit read-XOR-writes.  In memory a
    // row is two u64, pixels 0..63 then 64..127 with pixel x at bit
    // 63 - (x mod 64), so pixel word q is dword q ^ 1 of the row.  The loads
    // are batched by hand (memory bytes may alias the display for the
    // compiler): all sprite bytes first, in one round of dword loads, then
    // the two words of every sprite row's display rows before any of their
    // stores (the rows of one draw are distinct, so this order changes no
    // result).
    template <bool wrap>
    __device__ __forceinline__ uint32_t draw_s(uint32_t vx, uint32_t vy, uint32_t I, uint32_t n) {
        const uint32_t sc = scale();
        const uint32_t W = 128 / sc, H = 64 / sc;
        const uint32_t x0 = vx & (W - 1), y0 = vy & (H - 1);
        const bool big = n == 0;
        const uint32_t h = big ? 16 : n;
        const uint32_t X = x0 * sc;
        // sprite rows drawn: all h when wrapping, else those above the bottom edge
        const uint32_t rows = wrap ? h : min(h, H - y0);
        uint32_t sw[8];   // 32 bytes from I: a 16x16 sprite, two per row, high byte first; else one per row
        run<8>(I, sw);
        const uint32_t q = X >> 5, sh = X & 31;
        const bool spill = sh != 0 && (wrap || q < 3);
        const uint32_t d0 = q ^ 1, d1 = ((q + 1) & 3) ^ 1;
        uint32_t *disp = reinterpret_cast<uint32_t *>(hd);
        uint32_t hit = 0;
#pragma unroll
        for (int r0 = 0; r0 < 16; r0 += 16) {
            uint32_t lo[16], hi[16], y[16], o0[16][2], o1[16][2];
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int r = r0 + i;
                const uint32_t b0 = big ? __builtin_amdgcn_ubfe(sw[r >> 1], 16 * (r & 1), 8)
                                        : __builtin_amdgcn_ubfe(sw[r >> 2], 8 * (r & 3), 8);
                const uint32_t b1 = big ? __builtin_amdgcn_ubfe(sw[r >> 1], 16 * (r & 1) + 8, 8) : 0u;
                const uint32_t bits = (uint32_t)r < rows ? (b0 << 8) | b1 : 0u;   // pixel 0 at bit 15
                const uint32_t B = sc == 2 ? double_bits(bits) : bits << 16;       // pixel 0 at bit 31
                lo[i] = B >> sh;
                hi[i] = spill ? B << (32 - sh) : 0u;
                uint32_t py = y0 + r;
                py = py >= H ? py - H : py;
                y[i] = py * sc + roff;   // physical row of the sprite row (its first, in the 64x32 mode)
#pragma unroll
                for (int d = 0; d < 2; d++) {
                    const bool on = (uint32_t)r < rows && (uint32_t)d < sc;
                    const uint32_t p = (y[i] + d) & 63;
                    o0[i][d] = on ? disp[4 * p + d0] : 0u;
                    o1[i][d] = on ? disp[4 * p + d1] : 0u;
                }
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                if ((uint32_t)(r0 + i) >= rows) continue;
#pragma unroll
                for (int d = 0; d < 2; d++) {
                    if ((uint32_t)d < sc) {
                        const uint32_t p = (y[i] + d) & 63;
                        hit |= (o0[i][d] & lo[i]) | (o1[i][d] & hi[i]);
                        disp[4 * p + d0] = o0[i][d] ^ lo[i];
                        disp[4 * p + d1] = o1[i][d] ^ hi[i];
                    }
                }
            }
        }
        return hit != 0;
    }
    // Scrolls by physical pixels.  Down by s rows: display row y - s becomes
    // row y by moving the row offset back by s, and the s rows that come in
    // at the top (the physical rows of those that left at the bottom) are
    // cleared.  Sideways: every row shifted, sixteen rows at a time, a
    // chunk's loads before its stores.
    __device__ __forceinline__ void scroll_down(uint32_t s) {
        roff = (roff - s) & 63;
        for (uint32_t j = 0; j < s; j++) set_row((roff + j) & 63, (u128)0);
    }
    __device__ __forceinline__ void scroll_side(uint32_t s, bool right) {
        for (uint32_t y0 = 0; y0 < 64; y0 += 16) {
            u128 v[16];
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = row(y0 + j);
#pragma unroll
            for (int j = 0; j < 16; j++) set_row(y0 + j, right ? v[j] >> s : v[j] << s);
        }
    }
    // The CHIP-8 entry points of the instruction cycle; DXYN and 00E0 never
    // reach it (exec_schip takes them), these keep its interface whole.
    __device__ __forceinline__ uint32_t draw(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n, bool wrap) {
        return wrap ? draw_s<true>(x0, y0, I, n) : draw_s<false>(x0, y0, I, n);
    }
    __device__ __forceinline__ void clear() {
        for (uint32_t q = 0; q < 128; q++) hd[q] = 0;
        roff = 0;
    }
};

// One SUPER-CHIP instruction; returns whether it was a DXYN.
__device__ __forceinline__ bool exec_schip(Core &c, SchipMem &mem, uint32_t key, uint32_t quirks) {
    const uint32_t op = mem.fetch(c.pc);
    const uint32_t pc2 = (c.pc + 2) & 0xFFF;
    const uint32_t x = (op >> 8) & 0xF;
    const uint32_t sc = mem.scale();
    if ((op & 0xFFF0) == 0x00C0) {
        mem.scroll_down((op & 0xF) * sc);
        c.pc = pc2;
        return false;
    }
    switch (op) {
    case 0x00E0: mem.clear(); c.pc = pc2; return false;
    case 0x00FB: mem.scroll_side(4 * sc, true); c.pc = pc2; return false;
    case 0x00FC: mem.scroll_side(4 * sc, false); c.pc = pc2; return false;
    case 0x00FD: return false;   // stopped: PC stays
    case 0x00FE: mem.hires = 0; mem.clear(); c.pc = pc2; return false;
    case 0x00FF: mem.hires = 1; mem.clear(); c.pc = pc2; return false;
    default: break;
    }
    if ((op >> 12) == 0xD) {
        // the wrap flag is the batch's, so this branch is uniform
        const uint32_t vx = vget(c.r, x), vy = vget(c.r, (op >> 4) & 0xF);
        set_vf(c.r, (quirks & kQuirkPixelWrap) ? mem.draw_s<true>(vx, vy, c.I, op & 0xF)
                                               : mem.draw_s<false>(vx, vy, c.I, op & 0xF));
        c.pc = pc2;
        return true;
    }
    const uint32_t low = op & 0xF0FF;
    if (low == 0xF030) {
        c.I = kBigFont + 10 * (vget(c.r, x) & 15);
        c.pc = pc2;
        return false;
    }
    if (low == 0xF075 || low == 0xF085) {
        const u32x4 m = byte_mask(min(x, 7u) + 1);   // bytes 0..min(X, 7) of V0..V7
        if (low == 0xF075) {
            mem.rpl0 = (mem.rpl0 & ~m.x) | (c.r.w.x & m.x);
            mem.rpl1 = (mem.rpl1 & ~m.y) | (c.r.w.y & m.y);
        } else {
            c.r.w.x = (c.r.w.x & ~m.x) | (mem.rpl0 & m.x);
            c.r.w.y = (c.r.w.y & ~m.y) | (mem.rpl1 & m.y);
        }
        c.pc = pc2;
        return false;
    }
    // every other instruction: the branch-free grouped CHIP-8 cycle, so a
    // wave pays for one pass rather than for each handler its lanes need
    return exec_grouped(c, mem, key, quirks);
}

__device__ __forceinline__ void schip_env_step(Core &c, SchipMem &mem, uint32_t key, uint32_t ipf, uint32_t fs,
                                               uint32_t quirks) {
    for (uint32_t f = 0; f < fs; f++) {
        for (uint32_t i = 0; i < ipf; i++)
            if (exec_schip(c, mem, key, quirks) && (quirks & kQuirkDisplayWait)) break;
        tick(c);
    }
}

// Word 3 of an env's State::sx: bits 16..18 = frame-ring slot of the
// current display; bits 0..7 / 8..15 = what the observation of the last
// even / odd step needs (ring slot of its display | min(steps since reset,
// 3) << 3).  The observation of step k reads its byte while the emulation of
// step k + 1 writes the other one.
constexpr uint32_t kRingSlots = 5;
__device__ __forceinline__ uint32_t ring_head(uint32_t w3) { return (w3 >> 16) & 7; }

// Ring slot of observation frame f (0 = oldest) for a display in slot head,
// t steps after the env's last reset: frames from before the reset show the
// reset display.
__device__ __forceinline__ uint32_t frame_slot(uint32_t head, uint32_t t, uint32_t f) {
    const uint32_t age = min(3 - f, t);
    return (head + kRingSlots - age) % kRingSlots;
}

// The memory policy of slot's env, its display mode and flag registers.
__device__ __forceinline__ SchipMem schip_mem(const State &s, uint32_t slot, const uint8_t *img) {
    const uint32_t *sx = s.sx + (size_t)slot * 4;
    SchipMem mem;
    mem.ram = s.ram + (size_t)slot * kMem;
    mem.fb = nullptr;
    mem.stack = s.stack + (size_t)slot * 8;
    mem.dirty = s.dirty[slot];
    mem.hd = s.hfb + (size_t)slot * 128;
    mem.img = img;
    mem.hires = sx[0] & 1;             // sx word 0: mode | row offset << 8
    mem.roff = (sx[0] >> 8) & 63;
    mem.rpl0 = sx[1];
    mem.rpl1 = sx[2];
    return mem;
}

// Copy the display into ring slot `head`, rows in display order (physical
// row (y + roff) & 63 into ring row y): eight loads, then their stores.
__device__ __forceinline__ void ring_put(const State &s, uint32_t slot, uint32_t head, const uint64_t *hd,
                                         uint32_t roff) {
    uint4 *ring = reinterpret_cast<uint4 *>(s.hring + ((size_t)slot * kRingSlots + head) * 128);
    const uint4 *disp = reinterpret_cast<const uint4 *>(hd);
    for (uint32_t w = 0; w < 64; w += 8) {
        const uint4 a0 = disp[(w + roff) & 63], a1 = disp[(w + 1 + roff) & 63];
        const uint4 a2 = disp[(w + 2 + roff) & 63], a3 = disp[(w + 3 + roff) & 63];
        const uint4 a4 = disp[(w + 4 + roff) & 63], a5 = disp[(w + 5 + roff) & 63];
        const uint4 a6 = disp[(w + 6 + roff) & 63], a7 = disp[(w + 7 + roff) & 63];
        uint4 *dst = ring + w;
        dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
        dst[4] = a4; dst[5] = a5; dst[6] = a6; dst[7] = a7;
    }
}

// Emulation of env step k for one slot.
__device__ __forceinline__ void schip_emulate(const State &s, const Roms &roms, const StepIO &io, uint32_t k,
                                              uint32_t slot) {
    if (!slot_live(s, slot)) return;
    const uint32_t E = s.num;
    const uint32_t env = s.env_of[slot];
    const uint32_t rom = s.rom_of[slot];
    const uint32_t desc = roms.desc[rom];
    const uint32_t desc2 = roms.desc2 ? roms.desc2[rom] : kDesc2Default;

    Core c;
    uint32_t unused_head;   // the CHIP-8 ring head of misc; SUPER-CHIP keeps its own in sx word 3
    load_core(s, slot, c, unused_head);
    const uint32_t key = sticky_key(roms, c, action_key(roms, rom, desc, io.action[(size_t)k * E + env]));
    uint32_t *sx = s.sx + (size_t)slot * 4;
    const uint32_t w3 = sx[3];
    SchipMem mem = schip_mem(s, slot, roms.image + (size_t)rom * kMem);

    schip_env_step(c, mem, key, io.ipf, io.frame_skip, roms.quirks);

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

    if (done) {
        // Automatic reset (Section 3.4): power-on state, RNG stream continued.
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
        mem.hires = 0;
        mem.rpl0 = mem.rpl1 = 0;
        for (int q = 0; q < 8; q++) mem.stack[q] = 0;
        if (roms.w.reset_steps)   // start-up sequence and no-op reset
            run_reset_steps(roms, rom, c, [&](uint32_t rk) {
                schip_env_step(c, mem, rk, io.ipf, io.frame_skip, roms.quirks);
            });
        t = 0;
        prev = score_of(c.r, desc, desc2);
    } else {
        prev = score;
    }
    // The new display goes into the next ring slot; the observations of the
    // reset step and the three after it read the reset display for the
    // frames from before the reset (frame_slot), so a reset writes one slot.
    const uint32_t head = (ring_head(w3) + 1) % kRingSlots;
    ring_put(s, slot, head, mem.hd, mem.roff);
    const uint32_t sh = 8 * (k & 1);
    const uint32_t info = head | (min(t, 3u) << 3);
    sx[3] = (w3 & ~(0xFFu << sh) & ~(7u << 16)) | (info << sh) | (head << 16);
    store_core(s, slot, c, 0);
    s.t[slot] = t;
    s.prev[slot] = prev;
    s.dirty[slot] = mem.dirty;
    sx[0] = mem.hires | (mem.roff << 8);
    sx[1] = mem.rpl0;
    sx[2] = mem.rpl1;
}

// Observations of one env (a 64-thread block): its ring (5 KB) staged in
// LDS; then 32 threads transpose one 32x32 bit block each (frame f, rows
// 32h .. 32h + 31, pixels 32w .. 32w + 31; Hacker's Delight, 2nd ed., section
// 7-3) into packed columns in LDS; then every thread expands 16 pixels of a
// column into bytes per store, so each store instruction writes 1 KB of the
// env's observation contiguously.
__device__ __forceinline__ void schip_observe_env(const State &s, uint8_t *obs, uint32_t slot, uint32_t head,
                                                  uint32_t t) {
    __shared__ uint64_t ring[kRingSlots * 128];
    __shared__ uint32_t cols[4][128][2];   // [frame][column x][h]: bit y = pixel (x, 32h + y)
    const uint32_t tid = threadIdx.x;
    const uint64_t *src = s.hring + (size_t)slot * kRingSlots * 128;
#pragma unroll
    for (uint32_t q = 0; q < kRingSlots * 2; q++) ring[tid + 64 * q] = src[tid + 64 * q];
    __syncthreads();
    if (tid < 32) {
        const uint32_t f = tid >> 3, h = (tid >> 2) & 1, w = tid & 3;
        const uint64_t *rows = ring + frame_slot(head, t, f) * 128;
        // a[r]: pixels 32w .. 32w + 31 of row 32h + 31 - r, pixel 32w + c at
        // bit 31 - c (the high or low half of the row's u64)
        uint32_t a[32];
#pragma unroll
        for (int r = 0; r < 32; r++) {
            const uint64_t v = rows[2 * (32 * h + 31 - r) + (w >> 1)];
            a[r] = (w & 1) ? (uint32_t)v : (uint32_t)(v >> 32);
        }
        transpose32(a);   // a[c] = column 32w + c, bit y = row 32h + y
#pragma unroll
        for (int c = 0; c < 32; c++) cols[f][32 * w + c][h] = a[c];
    }
    __syncthreads();
    uint8_t *o = obs + (size_t)s.env_of[slot] * kSchipObsBytes;
#pragma unroll 8
    for (uint32_t q = 0; q < kSchipObsBytes / 1024; q++) {
        const uint32_t off = q * 1024 + 16 * tid;   // byte of the observation: [frame][x][y]
        const uint32_t f = off >> 13, x = (off >> 6) & 127, y0 = off & 63;
        store_obs_nt(o + off, spread16(cols[f][x][y0 >> 5] >> (y0 & 31)));
    }
}

// Launch j of a K-step run: blocks [0, emu_blocks) emulate step j (j < K),
// the next E blocks (when obs_step is set) write the observations of step
// j - 1.
__global__ __launch_bounds__(64) void schip_launch_kernel(State s, Roms roms, StepIO io, uint32_t j,
                                                          uint32_t emu_blocks, uint8_t *obs_step) {
    if (blockIdx.x < emu_blocks) {
        schip_emulate(s, roms, io, j, blockIdx.x * 64 + threadIdx.x);
        return;
    }
    const uint32_t slot = blockIdx.x - emu_blocks;
    if (!slot_live(s, slot)) return;   // uniform over the block
    const uint32_t info = (s.sx[(size_t)slot * 4 + 3] >> (8 * ((j - 1) & 1))) & 0xFF;
    schip_observe_env(s, obs_step, slot, info & 7, info >> 3);
}

// Power-on of the SUPER-CHIP part of the selected slots: display, frame
// ring, mode, flag registers and ring bookkeeping.
__global__ __launch_bounds__(256) void schip_reset_kernel(State s, const uint8_t *mask, uint32_t first,
                                                          uint32_t count) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t slot = first + k;
    if (slot >= s.num) return;
    if (mask && !mask[s.env_of[slot]]) return;
    const uint4 z = make_uint4(0, 0, 0, 0);
    uint4 *hd = reinterpret_cast<uint4 *>(s.hfb + (size_t)slot * 128);
    for (int q = 0; q < 64; q++) hd[q] = z;
    uint4 *ring = reinterpret_cast<uint4 *>(s.hring + (size_t)slot * kRingSlots * 128);
    for (uint32_t q = 0; q < kRingSlots * 64; q++) ring[q] = z;
    reinterpret_cast<uint4 *>(s.sx)[slot] = z;
}

// The emulation steps of a reset (start-up sequence, no-op reset) for the
// selected slots, after their power-on (CHIP-8 part and SUPER-CHIP part);
// the resulting display goes into ring slot 0, which the power-on made the
// display's slot with no step since the reset.
__global__ __launch_bounds__(64) void schip_reset_steps_kernel(State s, Roms roms, const uint8_t *mask,
                                                               uint32_t first, uint32_t count) {
    const uint32_t k = blockIdx.x * 64 + threadIdx.x;
    if (k >= count) return;
    const uint32_t slot = first + k;
    if (slot >= s.num) return;
    if (mask && !mask[s.env_of[slot]]) return;
    const uint32_t rom = s.rom_of[slot];
    const uint32_t desc = roms.desc[rom];
    const uint32_t desc2 = roms.desc2 ? roms.desc2[rom] : kDesc2Default;
    Core c;
    uint32_t unused_head;
    load_core(s, slot, c, unused_head);
    SchipMem mem = schip_mem(s, slot, roms.image + (size_t)rom * kMem);
    run_reset_steps(roms, rom, c, [&](uint32_t rk) {
        schip_env_step(c, mem, rk, roms.w.ipf, roms.w.frame_skip, roms.quirks);
    });
    ring_put(s, slot, 0, mem.hd, mem.roff);
    store_core(s, slot, c, 0);
    s.prev[slot] = score_of(c.r, desc, desc2);
    s.dirty[slot] = mem.dirty;
    uint32_t *sx = s.sx + (size_t)slot * 4;
    sx[0] = mem.hires | (mem.roff << 8);
    sx[1] = mem.rpl0;
    sx[2] = mem.rpl1;
}

// Observations of every env from its current ring state (octax_reset).
__global__ __launch_bounds__(64) void schip_observe_kernel(State s, uint8_t *obs) {
    const uint32_t slot = blockIdx.x;
    if (!slot_live(s, slot)) return;
    schip_observe_env(s, obs, slot, ring_head(s.sx[(size_t)slot * 4 + 3]), s.t[slot]);
}

}  // namespace

hipError_t launch_step_schip(const State &s, const Roms &r, const StepIO &io, hipStream_t st) {
    const uint32_t emu = (s.num + 63) / 64;
    for (uint32_t j = 0; j <= io.K; j++) {
        const uint32_t eb = j < io.K ? emu : 0;
        uint8_t *obs = (io.obs && j >= 1) ? io.obs + (size_t)((j - 1) % io.obs_slots) * s.num * kSchipObsBytes : nullptr;
        const uint32_t blocks = eb + (obs ? s.num : 0);
        if (blocks == 0) continue;
        hipLaunchKernelGGL(schip_launch_kernel, dim3(blocks), dim3(64), 0, st, s, r, io, j, eb, obs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_schip_reset(const State &s, const Roms &r, const uint8_t *mask, uint32_t first, uint32_t count,
                              hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(schip_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, st, s, mask, first, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !r.w.reset_steps) return e;
    hipLaunchKernelGGL(schip_reset_steps_kernel, dim3((count + 63) / 64), dim3(64), 0, st, s, r, mask, first, count);
    return hipGetLastError();
}

hipError_t launch_schip_observe(const State &s, uint8_t *obs, hipStream_t st) {
    if (s.num == 0) return hipSuccess;
    hipLaunchKernelGGL(schip_observe_kernel, dim3(s.num), dim3(64), 0, st, s, obs);
    return hipGetLastError();
}

}  // namespace octax
