// The CHIP-8 instruction cycle regrouped by opcode class for wavefront
// execution (same semantics as exec_one in octax_core.h, the OCTAX_QUIRKS_V1
// profile of octax.h).
//
// In a wavefront of independent machines nearly every one of the 35
// instructions is present in every instruction slot, so a switch executes
// the union of all handlers behind a tree of divergent branches.  Here the
// instructions are grouped instead:
//   * memory and stack classes (DXYN, FX33, FX55, FX65, 00E0, 2NNN, 00EE)
//     and the random byte of CXNN are blocks that run only for the lanes
//     that need them (skipped when no lane of the wave does);
//   * every register effect - the value written to VX and the flag written
//     to VF, the next PC (jumps, calls, returns, skips, FX0A wait), I, DT and
//     ST - is computed for all lanes with selects, in one pass, without
//     branches.
#pragma once

#include "octax_core.h"

namespace octax {

// V[x] = val when en (a select per register word, no branch).
__device__ __forceinline__ void vset_if(Regs &r, uint32_t x, uint32_t val, bool en) {
    const uint32_t sh = (x & 3) * 8;
    const uint32_t m = en ? (0xFFu << sh) : 0u;
    const uint32_t s = (val & 0xFFu) << sh;
    const uint32_t q = x >> 2;
    const uint32_t m0 = q == 0 ? m : 0u, m1 = q == 1 ? m : 0u, m2 = q == 2 ? m : 0u, m3 = q == 3 ? m : 0u;
    r.w.x = (r.w.x & ~m0) | (s & m0);
    r.w.y = (r.w.y & ~m1) | (s & m1);
    r.w.z = (r.w.z & ~m2) | (s & m2);
    r.w.w = (r.w.w & ~m3) | (s & m3);
}

template <class Mem>
__device__ __forceinline__ void exec_grouped(Core &c, Mem &mem, uint32_t key) {
    const uint32_t op = mem.fetch(c.pc);
    const uint32_t pc2 = (c.pc + 2) & 0xFFF;
    const uint32_t h = op >> 12;
    const uint32_t x = (op >> 8) & 0xF;
    const uint32_t y = (op >> 4) & 0xF;
    const uint32_t n = op & 0xF;
    const uint32_t nn = op & 0xFF;
    const uint32_t nnn = op & 0xFFF;
    const uint32_t vx = vget(c.r, x);
    const uint32_t vy = vget(c.r, y);
    const bool isF = h == 0xF;

    // ---- memory, stack and random classes (read the old I and V) ----
    if (h == 0xD) set_vf(c.r, mem.draw(vx & 63, vy & 31, c.I, n));
    if (isF && nn == 0x33) {
        const uint32_t bcd = (vx / 100) | (((vx / 10) % 10) << 8) | ((vx % 10) << 16);
        mem.store_bytes(c.I, 3, u32x4{bcd, 0, 0, 0});
    }
    if (isF && nn == 0x55) mem.store_bytes(c.I, x + 1, c.r.w);   // V0..VX are in memory order
    if (isF && nn == 0x65) {
        const u32x4 b = mem.load_bytes(c.I, x + 1);
        const u32x4 m = byte_mask(x + 1);
        c.r.w = (c.r.w & ~m) | (b & m);
    }
    if (op == 0x00E0) mem.clear();
    if (h == 0x2) mem.stack_set(c.sp, pc2);
    uint32_t ret = 0;
    if (op == 0x00EE) ret = mem.stack_get((c.sp - 1) & 15);
    uint32_t rnd = 0;
    if (h == 0xC) rnd = rnd_byte(c.rng);

    // ---- VX and VF ----
    const uint32_t a_add = vx + vy;
    const uint32_t r8 = n == 0x0 ? vy : n == 0x1 ? (vx | vy) : n == 0x2 ? (vx & vy) : n == 0x3 ? (vx ^ vy)
                      : n == 0x4 ? a_add : n == 0x5 ? (vx - vy) : n == 0x6 ? (vy >> 1)
                      : n == 0x7 ? (vy - vx) : (vy << 1);
    const uint32_t f8 = n == 0x4 ? (a_add >> 8) : n == 0x5 ? (uint32_t)(vx >= vy) : n == 0x6 ? (vy & 1)
                      : n == 0x7 ? (uint32_t)(vy >= vx) : n == 0xE ? (vy >> 7) : 0u;
    const bool alu_ok = (n <= 0x7) || (n == 0xE);
    const bool key_held = key < 16;
    const uint32_t res = h == 0x6 ? nn : h == 0x7 ? (vx + nn) : h == 0x8 ? r8 : h == 0xC ? (rnd & nn)
                       : nn == 0x07 ? c.dt : key;
    const bool wr = (h == 0x6) || (h == 0x7) || (h == 0x8 && alu_ok) || (h == 0xC) ||
                    (isF && (nn == 0x07 || (nn == 0x0A && key_held)));
    vset_if(c.r, x, res, wr);
    const bool wf = h == 0x8 && alu_ok && n != 0;   // the flag is written after the result
    c.r.w.w = wf ? ((c.r.w.w & 0x00FFFFFFu) | (f8 << 24)) : c.r.w.w;

    // ---- PC, SP, I, timers ----
    const uint32_t kx = vx & 15;
    const bool skip = (h == 0x3 && vx == nn) || (h == 0x4 && vx != nn) ||
                      (h == 0x5 && n == 0 && vx == vy) || (h == 0x9 && n == 0 && vx != vy) ||
                      (h == 0xE && ((nn == 0x9E && key == kx) || (nn == 0xA1 && key != kx)));
    const uint32_t v0 = c.r.w.x & 0xFF;   // after this instruction's writes: BNNN reads V0 only
    c.pc = (h == 0x1 || h == 0x2) ? nnn
         : h == 0xB ? ((nnn + v0) & 0xFFF)
         : op == 0x00EE ? ret
         : (isF && nn == 0x0A && !key_held) ? c.pc
         : skip ? ((pc2 + 2) & 0xFFF) : pc2;
    c.sp = h == 0x2 ? ((c.sp + 1) & 15) : op == 0x00EE ? ((c.sp - 1) & 15) : c.sp;
    const uint32_t I = c.I;
    c.I = h == 0xA ? nnn
        : !isF ? I
        : nn == 0x1E ? ((I + vx) & 0xFFF)
        : nn == 0x29 ? (kFont + 5 * kx)
        : (nn == 0x55 || nn == 0x65) ? ((I + x + 1) & 0xFFF) : I;
    c.dt = (isF && nn == 0x15) ? vx : c.dt;
    c.st = (isF && nn == 0x18) ? vx : c.st;
}

}  // namespace octax
