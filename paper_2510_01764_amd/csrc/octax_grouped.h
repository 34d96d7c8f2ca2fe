// The CHIP-8 instruction cycle regrouped by opcode class for wavefront
// execution (same semantics as exec_one in octax_core.h, the OCTAX_QUIRKS_V1
// profile of octax.h).
//
// In a wavefront of independent machines nearly every one of the 35
// instructions is present in every instruction slot, so a switch executes
// the union of all handlers behind a tree of divergent branches, each with
// its exec-mask bookkeeping on the scalar unit.  Here the instructions are
// grouped instead:
//   * the fetch reads the instruction word and the return address on top of
//     the stack, for every lane;
//   * the memory and display classes (DXYN, FX33/FX55, FX65, 00E0), the
//     stack write of 2NNN and the random byte of CXNN are blocks that run
//     only for the lanes that need them and are skipped when no lane of the
//     wave does;
//   * every register effect - the value written to VX and the flag written
//     to VF, the next PC (jumps, calls, returns, skips, FX0A wait), SP, I, DT
//     and ST - is computed for all lanes with selects, in one pass, without
//     branches.
// The memory policy supplies fetch(pc, sp, ret) (instruction word at pc and
// ret = stack[(sp - 1) & 15]) and stack_popped(sp) (called after a return
// with the new SP) besides the operations listed in octax_core.h.  A policy
// with kOneAccess also supplies access(), one call that performs the memory
// access of DXYN, FX33, FX55 or FX65 for every lane that has one (all four
// read at most sixteen bytes around I), used unless the pixel-wrap quirk is
// on.
#pragma once

#include "octax_core.h"

namespace octax {

// Branch-free select.  The operands are evaluated before the call, so the
// compiler sees a select of two values; written as nested conditional
// expressions over the same opcode field, the chains below would be merged
// into a switch and lowered to divergent branches.
__device__ __forceinline__ uint32_t pick(bool c, uint32_t a, uint32_t b) { return c ? a : b; }

// V[x] = val when en: a bitfield insert of the byte into the register word
// that holds V[x], the other words kept (no branch).
__device__ __forceinline__ void vset_if(Regs &r, uint32_t x, uint32_t val, bool en) {
    const uint32_t sh = (x & 3) * 8;
    const uint32_t m = 0xFFu << sh;
    const uint32_t s = (val & 0xFFu) << sh;
    const uint32_t q = pick(en, x >> 2, 4u);
    r.w.x = pick(q == 0, (r.w.x & ~m) | s, r.w.x);
    r.w.y = pick(q == 1, (r.w.y & ~m) | s, r.w.y);
    r.w.z = pick(q == 2, (r.w.z & ~m) | s, r.w.z);
    r.w.w = pick(q == 3, (r.w.w & ~m) | s, r.w.w);
}

// One instruction; returns whether it was a DXYN (for the display-wait quirk).
template <class Mem>
__device__ __forceinline__ bool exec_grouped(Core &c, Mem &mem, uint32_t key, uint32_t quirks = 0) {
    uint32_t ret;   // stack[(SP - 1) & 15]
    const uint32_t op = mem.fetch(c.pc, c.sp, ret);
    const uint32_t pc2 = (c.pc + 2) & 0xFFF;
    const uint32_t h = op >> 12;
    const uint32_t x = __builtin_amdgcn_ubfe(op, 8, 4);
    const uint32_t y = __builtin_amdgcn_ubfe(op, 4, 4);
    const uint32_t n = op & 0xF;
    const uint32_t nn = op & 0xFF;
    const uint32_t nnn = op & 0xFFF;
    const uint32_t vx = vget(c.r, x);
    const uint32_t vy = vget(c.r, y);
    const bool isF = h == 0xF;

    // ---- memory, display, stack and random classes (read the old I and V) ----
    // FX33 stores three BCD digits of VX, FX55 V0..VX (in memory order in the
    // register vector), FX65 loads V0..VX.
    const bool st = isF & ((nn == 0x33) | (nn == 0x55));
    const bool ld = isF & (nn == 0x65);
    const bool bcd = nn == 0x33;
    bool separate = true;
    if constexpr (Mem::kOneAccess) {
        if (!(quirks & kQuirkPixelWrap)) {
            // one memory access per lane for DXYN, FX33, FX55 and FX65
            separate = false;
            const bool longw = __builtin_amdgcn_ballot_w64((h == 0xD) & (n > 8)) != 0;   // among the drawing lanes
            if ((h == 0xD) | st | ld) {
                const uint32_t digits = (vx / 100) | (((vx / 10) % 10) << 8) | ((vx % 10) << 16);
                u32x4 data = bcd ? u32x4{digits, 0, 0, 0} : c.r.w;
                const uint32_t count = (h == 0xD) ? n : (bcd ? 3u : x + 1);
                const uint32_t hit = mem.access(h == 0xD, st, c.I, count, vx & 63, vy & 31, longw, data);
                if (h == 0xD) set_vf(c.r, hit);
                if (ld) {
                    const u32x4 m = byte_mask(x + 1);
                    c.r.w = (c.r.w & ~m) | (data & m);
                }
            }
        }
    }
    if (separate) {
        if (h == 0xD) set_vf(c.r, mem.draw(vx & 63, vy & 31, c.I, n, (quirks & kQuirkPixelWrap) != 0));
        if (st) {
            const uint32_t digits = (vx / 100) | (((vx / 10) % 10) << 8) | ((vx % 10) << 16);
            const u32x4 bytes = bcd ? u32x4{digits, 0, 0, 0} : c.r.w;
            mem.store_bytes(c.I, bcd ? 3u : x + 1, bytes);
        }
        if (ld) {
            const u32x4 b = mem.load_bytes(c.I, x + 1);
            const u32x4 m = byte_mask(x + 1);
            c.r.w = (c.r.w & ~m) | (b & m);
        }
    }
    if (op == 0x00E0) mem.clear();
    if (h == 0x2) mem.stack_set(c.sp, pc2);
    uint32_t rnd = 0;
    if (h == 0xC) rnd = rnd_byte(c.rng);

    // ---- VX and VF ----
    // 8XYn: a select tree on the bits of n (0 LD, 1 OR, 2 AND, 3 XOR, 4 ADD,
    // 5 SUB, 6 SHR, 7 SUBN), then E SHL.
    const bool n1 = n & 1, n2 = n & 2, n4 = n & 4, nE = n == 0xE;
    const uint32_t sum = vx + vy;
    const uint32_t ss = pick(quirks & kQuirkShiftVx, vx, vy);   // shift source
    const uint32_t r01 = pick(n1, vx | vy, vy);
    const uint32_t r23 = pick(n1, vx ^ vy, vx & vy);
    const uint32_t r45 = pick(n1, vx - vy, sum);
    const uint32_t r67 = pick(n1, vy - vx, ss >> 1);
    const uint32_t r8 = pick(nE, ss << 1, pick(n4, pick(n2, r67, r45), pick(n2, r23, r01)));
    const uint32_t f45 = pick(n1, (uint32_t)(vx >= vy), sum >> 8);
    const uint32_t f67 = pick(n1, (uint32_t)(vy >= vx), ss & 1);
    const uint32_t f8 = pick(nE, ss >> 7, pick(n4, pick(n2, f67, f45), 0u));
    const bool alu_ok = (n <= 0x7) | nE;
    const bool key_held = key < 16;
    const uint32_t resF = pick(nn == 0x07, c.dt, key);
    const uint32_t res = pick(h == 0x6, nn, pick(h == 0x7, vx + nn, pick(h == 0x8, r8, pick(h == 0xC, rnd & nn, resF))));
    const bool wr = (h == 0x6) | (h == 0x7) | ((h == 0x8) & alu_ok) | (h == 0xC) |
                    (isF & ((nn == 0x07) | ((nn == 0x0A) & key_held)));
    vset_if(c.r, x, res, wr);
    // the flag is written after the result; 8XY1/2/3 keep VF with the quirk
    const bool wf = (h == 0x8) & alu_ok & (n != 0) & !((quirks & kQuirkNoVfReset) && (n <= 3));
    c.r.w.w = pick(wf, (c.r.w.w & 0x00FFFFFFu) | (f8 << 24), c.r.w.w);

    // ---- PC, SP, I, timers ----
    // skips: 3XNN / 4XNN compare VX with NN, 5XY0 / 9XY0 VX with VY, EX9E /
    // EXA1 the held key with VX & 15; 4, 9 and A1 skip on inequality
    const uint32_t kx = vx & 15;
    const bool cmp_nn = (h == 0x3) | (h == 0x4);
    const bool cmp_vy = ((h == 0x5) | (h == 0x9)) & (n == 0);
    const bool cmp_key = (h == 0xE) & ((nn == 0x9E) | (nn == 0xA1));
    const uint32_t lhs = pick(cmp_key, key, vx);
    const uint32_t rhs = pick(cmp_nn, nn, pick(cmp_vy, vy, kx));
    const bool neg = (h == 0x4) | (h == 0x9) | ((h == 0xE) & (nn == 0xA1));
    const bool skip = (cmp_nn | cmp_vy | cmp_key) & ((lhs == rhs) != neg);
    // BNNN writes no register: this is V0 (or VX with the quirk) before it
    const uint32_t v0 = pick(quirks & kQuirkJumpVx, vx, c.r.w.x & 0xFF);
    const bool ret_op = op == 0x00EE;
    const bool wait_key = isF & (nn == 0x0A) & !key_held;
    const uint32_t seq = pick(wait_key, c.pc, pick(skip, (pc2 + 2) & 0xFFF, pc2));
    c.pc = pick((h == 0x1) | (h == 0x2), nnn, pick(h == 0xB, (nnn + v0) & 0xFFF, pick(ret_op, ret, seq)));
    c.sp = pick(h == 0x2, (c.sp + 1) & 15, pick(ret_op, (c.sp - 1) & 15, c.sp));
    if (ret_op) mem.stack_popped(c.sp);
    const uint32_t I = c.I;
    const uint32_t iF = pick(nn == 0x1E, (I + vx) & 0xFFF,
                             pick(nn == 0x29, kFont + 5 * kx,
                                  pick(((nn == 0x55) | (nn == 0x65)) & !(quirks & kQuirkMemKeepI), (I + x + 1) & 0xFFF, I)));
    c.I = pick(h == 0xA, nnn, pick(isF, iF, I));
    c.dt = pick(isF & (nn == 0x15), vx, c.dt);
    c.st = pick(isF & (nn == 0x18), vx, c.st);
    return h == 0xD;
}

}  // namespace octax
