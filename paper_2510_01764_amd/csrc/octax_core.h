// The CHIP-8 instruction cycle (Section 3.2: fetch a 16-bit word at PC and
// advance PC, decode its nibbles, execute one of the 35 instructions) for one
// machine held in registers.  Memory, display and stack live wherever the
// kernel keeps them; a kernel supplies that through the `Mem` policy:
//   uint32_t fetch(pc)              big-endian word at pc, pc+1 (12-bit wrap)
//   u32x4    load_bytes(a, count)   bytes a .. a+count-1 (count 1..16), byte k
//                                   of the result = memory[a + k], rest zero
//   void     store_bytes(a, count, bytes)  the inverse (marks pages dirty)
//   uint32_t draw(x0, y0, I, n)     XOR an n-row sprite from memory at I onto
//                                   the display at (x0, y0), clipped;
//                                   returns 1 on collision
//   void     clear()                blank display
//   uint32_t stack_get(i), void stack_set(i, v)
// Semantics are those of the OCTAX_QUIRKS_V1 profile documented in octax.h.
#pragma once

#include "octax_device.h"

namespace octax {

struct Core {
    Regs r;
    uint32_t pc;   // 12-bit
    uint32_t I;    // 12-bit
    uint32_t sp;   // 0..15
    uint32_t dt;
    uint32_t st;
    uint64_t rng;
    uint32_t pkey;   // key held in the previous step (sticky actions), kKeyNone after a reset
};

__device__ __forceinline__ void skip(Core &c) { c.pc = (c.pc + 2) & 0xFFF; }

// Mask of the first `count` bytes (0..16) of a 16-byte vector.
__device__ __forceinline__ u32x4 byte_mask(uint32_t count) {
    u32x4 m;
    m.x = count >= 4 ? 0xFFFFFFFFu : (1u << (8 * count)) - 1;
    m.y = count >= 8 ? 0xFFFFFFFFu : count <= 4 ? 0u : (1u << (8 * (count - 4))) - 1;
    m.z = count >= 12 ? 0xFFFFFFFFu : count <= 8 ? 0u : (1u << (8 * (count - 8))) - 1;
    m.w = count >= 16 ? 0xFFFFFFFFu : count <= 12 ? 0u : (1u << (8 * (count - 12))) - 1;
    return m;
}

// Byte k (0..15) of a 16-byte vector; used with k a constant of an unrolled
// loop, so the selection folds away.
__device__ __forceinline__ uint32_t byte_of(const u32x4 &v, int k) {
    const uint32_t w = k < 4 ? v.x : k < 8 ? v.y : k < 12 ? v.z : v.w;
    return (w >> (8 * (k & 3))) & 0xFF;
}

// v with byte k (0..15, a constant of an unrolled loop) or-ed with b.
__device__ __forceinline__ void or_byte(u32x4 &v, int k, uint32_t b) {
    const uint32_t s = b << (8 * (k & 3));
    if (k < 4) v.x |= s;
    else if (k < 8) v.y |= s;
    else if (k < 12) v.z |= s;
    else v.w |= s;
}

// Quirk flags (octax.h): bit 0 is the VIP base profile, bits 1..6 switch one
// behaviour each to the SUPER-CHIP / later-interpreter one.
constexpr uint32_t kQuirkShiftVx = 1u << 1;    // 8XY6 / 8XYE shift VX in place
constexpr uint32_t kQuirkMemKeepI = 1u << 2;   // FX55 / FX65 leave I unchanged
constexpr uint32_t kQuirkJumpVx = 1u << 3;     // BNNN jumps to XNN + VX
constexpr uint32_t kQuirkNoVfReset = 1u << 4;  // 8XY1/2/3 leave VF unchanged
constexpr uint32_t kQuirkPixelWrap = 1u << 5;  // sprites wrap at the right and bottom edges
constexpr uint32_t kQuirkDisplayWait = 1u << 6; // a DXYN ends the frame's instructions

// One instruction; returns whether it was a DXYN (the display-wait quirk ends
// the frame after one).
template <class Mem>
__device__ __forceinline__ bool exec_one(Core &c, Mem &mem, uint32_t key, uint32_t quirks = 0) {
    const uint32_t op = mem.fetch(c.pc);
    c.pc = (c.pc + 2) & 0xFFF;
    const uint32_t x = (op >> 8) & 0xF;
    const uint32_t y = (op >> 4) & 0xF;
    const uint32_t n = op & 0xF;
    const uint32_t nn = op & 0xFF;
    const uint32_t nnn = op & 0xFFF;
    const uint32_t vx = vget(c.r, x);
    const uint32_t vy = vget(c.r, y);
    switch (op >> 12) {
    case 0x0:
        if (op == 0x00E0) {
            mem.clear();
        } else if (op == 0x00EE) {
            c.sp = (c.sp - 1) & 15;
            c.pc = mem.stack_get(c.sp);
        }
        break;
    case 0x1:
        c.pc = nnn;
        break;
    case 0x2:
        mem.stack_set(c.sp, c.pc);
        c.sp = (c.sp + 1) & 15;
        c.pc = nnn;
        break;
    case 0x3:
        if (vx == nn) skip(c);
        break;
    case 0x4:
        if (vx != nn) skip(c);
        break;
    case 0x5:
        if (n == 0 && vx == vy) skip(c);
        break;
    case 0x6:
        vset(c.r, x, nn);
        break;
    case 0x7:
        vset(c.r, x, vx + nn);
        break;
    case 0x8: {
        uint32_t res = 0, flag = 0;
        bool write = true, has_flag = true;
        const bool keep_vf = quirks & kQuirkNoVfReset;
        const uint32_t ssrc = (quirks & kQuirkShiftVx) ? vx : vy;   // shift source
        switch (n) {
        case 0x0: res = vy; has_flag = false; break;
        case 0x1: res = vx | vy; flag = 0; has_flag = !keep_vf; break;
        case 0x2: res = vx & vy; flag = 0; has_flag = !keep_vf; break;
        case 0x3: res = vx ^ vy; flag = 0; has_flag = !keep_vf; break;
        case 0x4: res = vx + vy; flag = res >> 8; break;
        case 0x5: res = vx - vy; flag = vx >= vy; break;
        case 0x6: res = ssrc >> 1; flag = ssrc & 1; break;
        case 0x7: res = vy - vx; flag = vy >= vx; break;
        case 0xE: res = ssrc << 1; flag = ssrc >> 7; break;
        default: write = false; break;
        }
        if (write) {
            vset(c.r, x, res);
            if (has_flag) set_vf(c.r, flag);
        }
        break;
    }
    case 0x9:
        if (n == 0 && vx != vy) skip(c);
        break;
    case 0xA:
        c.I = nnn;
        break;
    case 0xB:
        c.pc = (nnn + ((quirks & kQuirkJumpVx) ? vx : (c.r.w.x & 0xFF))) & 0xFFF;
        break;
    case 0xC:
        vset(c.r, x, rnd_byte(c.rng) & nn);
        break;
    case 0xD:
        set_vf(c.r, mem.draw(vx & 63, vy & 31, c.I, n, (quirks & kQuirkPixelWrap) != 0));
        break;
    case 0xE:
        if (nn == 0x9E) {
            if (key == (vx & 15)) skip(c);
        } else if (nn == 0xA1) {
            if (key != (vx & 15)) skip(c);
        }
        break;
    default:  // 0xF
        switch (nn) {
        case 0x07: vset(c.r, x, c.dt); break;
        case 0x0A:
            if (key < 16) vset(c.r, x, key);
            else c.pc = (c.pc - 2) & 0xFFF;
            break;
        case 0x15: c.dt = vx; break;
        case 0x18: c.st = vx; break;
        case 0x1E: c.I = (c.I + vx) & 0xFFF; break;
        case 0x29: c.I = kFont + 5 * (vx & 15); break;
        case 0x33: {
            const uint32_t bcd = (vx / 100) | (((vx / 10) % 10) << 8) | ((vx % 10) << 16);
            mem.store_bytes(c.I, 3, u32x4{bcd, 0, 0, 0});
            break;
        }
        case 0x55:
            // V0..VX are packed in memory order in the register vector
            mem.store_bytes(c.I, x + 1, c.r.w);
            if (!(quirks & kQuirkMemKeepI)) c.I = (c.I + x + 1) & 0xFFF;
            break;
        case 0x65: {
            const u32x4 b = mem.load_bytes(c.I, x + 1);
            const u32x4 m = byte_mask(x + 1);
            c.r.w = (c.r.w & ~m) | (b & m);
            if (!(quirks & kQuirkMemKeepI)) c.I = (c.I + x + 1) & 0xFFF;
            break;
        }
        default: break;
        }
        break;
    }
    return (op >> 12) == 0xD;
}

// One 60 Hz tick of the delay and sound timers.
__device__ __forceinline__ void tick(Core &c) {
    c.dt -= (c.dt > 0);
    c.st -= (c.st > 0);
}

// Load / store the register part of an env's state from the SoA arrays.
__device__ __forceinline__ void load_core(const State &s, uint32_t slot, Core &c, uint32_t &head) {
    const uint32_t E = s.num;
    c.r.w.x = s.regs[0 * E + slot];
    c.r.w.y = s.regs[1 * E + slot];
    c.r.w.z = s.regs[2 * E + slot];
    c.r.w.w = s.regs[3 * E + slot];
    const uint32_t pi = s.pc_i[slot];
    c.pc = pi & 0xFFF;
    c.I = (pi >> 16) & 0xFFF;
    const uint32_t m = s.misc[slot];
    c.sp = m & 15;
    c.dt = (m >> 8) & 0xFF;
    c.st = (m >> 16) & 0xFF;
    head = (m >> 24) & 3;
    c.pkey = ((m >> 26) & 31) ^ kKeyNone;
    c.rng = s.rng[slot];
}

__device__ __forceinline__ void store_core(const State &s, uint32_t slot, const Core &c, uint32_t head) {
    const uint32_t E = s.num;
    s.regs[0 * E + slot] = c.r.w.x;
    s.regs[1 * E + slot] = c.r.w.y;
    s.regs[2 * E + slot] = c.r.w.z;
    s.regs[3 * E + slot] = c.r.w.w;
    s.pc_i[slot] = c.pc | (c.I << 16);
    s.misc[slot] = c.sp | (c.dt << 8) | (c.st << 16) | (head << 24) | ((c.pkey ^ kKeyNone) << 26);
    s.rng[slot] = c.rng;
}

// Power-on registers (Section 3.2, ROM loading and initialization).
__device__ __forceinline__ void reset_core(Core &c) {
    c.r.w = u32x4{0, 0, 0, 0};
    c.pc = kProgram;
    c.I = 0;
    c.sp = 0;
    c.dt = 0;
    c.st = 0;
    c.pkey = kKeyNone;
}

// Game descriptors beyond desc (Section 3.3 and the game list of Appendix
// C.3), packed per ROM: score mode (bits 0..1) | score argument << 2 |
// op of the first termination clause << 10 | op of the second << 13 |
// second clause's register << 16 | its constant << 24.  kDesc2Default is the
// plain form (score V[score_reg], termination V[term_reg] == term_value).
constexpr uint32_t kDesc2Default = 1u << 10;

// Score: mode 0 V, 1 (V / 10) - (V % 10), 2 -(V + V[arg]), 3 V if V <= arg else 0,
// with V = V[score_reg].
__device__ __forceinline__ int32_t score_of(const Regs &r, uint32_t desc, uint32_t desc2) {
    const uint32_t v = vget(r, desc & 15);
    const uint32_t mode = desc2 & 3, arg = (desc2 >> 2) & 0xFF;
    if (mode == 0) return (int32_t)v;
    if (mode == 1) return (int32_t)(v / 10) - (int32_t)(v % 10);
    if (mode == 2) return -(int32_t)(v + vget(r, arg & 15));
    return v <= arg ? (int32_t)v : 0;
}

// One termination clause on register value v and constant k: op 0 never,
// 1 ==, 2 >=, 3 !=, 4 either decimal digit of v equals k.
__device__ __forceinline__ bool clause_holds(uint32_t op, uint32_t v, uint32_t k) {
    return (op == 1 && v == k) || (op == 2 && v >= k) || (op == 3 && v != k) ||
           (op == 4 && (v / 10 == k || v % 10 == k));
}

// Termination: the first clause (V[term_reg] against term_value) or the second.
__device__ __forceinline__ uint32_t terminated_of(const Regs &r, uint32_t desc, uint32_t desc2) {
    const bool t1 = clause_holds((desc2 >> 10) & 7, vget(r, (desc >> 8) & 15), (desc >> 16) & 0xFF);
    const bool t2 = clause_holds((desc2 >> 13) & 7, vget(r, (desc2 >> 16) & 15), desc2 >> 24);
    return (t1 || t2) ? 1u : 0u;
}

// Sticky actions (Section 3.2): with probability sticky_q24 / 2^24 the key
// held in the previous step is held again instead of `key`.  One draw from
// the env's SplitMix64 stream per step, only when the wrapper is on.
__device__ __forceinline__ uint32_t sticky_key(const Roms &roms, Core &c, uint32_t key) {
    if (roms.w.sticky_q24 && (uint32_t)(splitmix_next(c.rng) >> 40) < roms.w.sticky_q24) key = c.pkey;
    c.pkey = key;
    return key;
}

// The emulation steps of a reset, after power-on (Section 3.2): the ROM's
// start-up sequence, one environment step per entry with its key held, then
// the no-op reset's steps with no key held, their number drawn uniformly
// from 0..noop_max by Lemire's multiply-shift on the top 32 bits of one
// SplitMix64 draw.  step(key) runs one environment step.
template <class StepFn>
__device__ __forceinline__ void run_reset_steps(const Roms &roms, uint32_t rom, Core &c, StepFn step) {
    if (roms.w.startup) {
        const uint8_t *su = roms.w.startup + (size_t)rom * 17;
        const uint32_t n = su[0];
        for (uint32_t i = 0; i < n; i++) step((uint32_t)su[1 + i]);
    }
    if (roms.w.noop_max) {
        const uint64_t u = splitmix_next(c.rng);
        const uint32_t n = (uint32_t)(((u >> 32) * ((uint64_t)roms.w.noop_max + 1)) >> 32);
        for (uint32_t i = 0; i < n; i++) step(kKeyNone);
    }
    c.pkey = kKeyNone;
}

// The held key of a step: the action's key, or none for the no-op and for
// out-of-range actions.
__device__ __forceinline__ uint32_t action_key(const Roms &roms, uint32_t rom, uint32_t desc, int32_t a) {
    const int32_t nact = (int32_t)(desc >> 24);
    return (a >= 0 && a < nact) ? roms.keys[rom * 16 + a] & 15 : kKeyNone;
}

}  // namespace octax
