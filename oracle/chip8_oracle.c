/*
 * CPU oracle for the batched CHIP-8 environment step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, scalar CHIP-8
 * interpreter and RL wrapper used to check the HIP path.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU library: every
 * constant below is written out here from the paper and the CHIP-8
 * definition.  The product never calls it.
 *
 * Sources followed:
 *   - Section 3.2 ("How does Octax work?"): memory loaded at 0x200, font at
 *     0x50, sixteen registers, I, PC, 64x32 display; fetch reads a 16-bit
 *     instruction and advances PC; decode splits nibbles; execute dispatches
 *     to one handler per instruction; ALU ops set a carry/borrow flag; the
 *     wrapper runs several instructions per frame, ticks the 60 Hz timers,
 *     skips 4 frames per step, stacks 4 frames into a (4, 64, 32) boolean
 *     observation and maps actions to a key subset plus a no-op.
 *   - Section 3.3: reward from a score register, termination from a
 *     register test.
 *   - Appendix B.2-B.4: 4 KB memory, V0-VF with VF the flag register, XOR
 *     drawing with collision when a pixel turns off, 16-key keypad, 60 Hz
 *     delay and sound timers, 4x5 hex font at 0x050-0x09F, BCD (FX33) and
 *     bulk register store/load (FX55/FX65).
 * The paper does not print per-opcode semantics.  Where it is silent the
 * classic COSMAC VIP meaning is used (shift from VY, FX55/FX65 advance I,
 * BNNN adds V0, 8XY1/2/3 clear VF, flag written after the result), sprites
 * start at wrapped coordinates and clip at the right and bottom edges, the
 * stack holds 16 entries with a wrapping pointer, and CXNN draws from a
 * per-env SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014).
 *
 * Parity notes: the font glyph bytes are the standard CHIP-8 hex font (the
 * paper fixes only their addresses); the RNG stream is pinned to the
 * published SplitMix64 definition, not to the paper's JAX keys.
 *
 * Environment wrappers (Section 3.2, "Environment integration": start-up
 * sequences that skip menus, no-op reset and sticky actions).  The paper
 * names them without defining them; the readings taken here:
 *   - sticky actions: at every step, with probability sticky_q24 / 2^24, the
 *     key held in the previous step is held again instead of the action's
 *     key; after a reset the previous key is "none";
 *   - start-up sequence: every reset runs, after power-on, one environment
 *     step (frame_skip frames) per entry of the ROM's start-up list, with
 *     that entry's key held;
 *   - no-op reset: then a number of no-op steps (no key held) drawn
 *     uniformly from 0..noop_max;
 *   - after these steps the frame stack holds the resulting display four
 *     times, the score baseline is the score register's value, and
 *     terminations during them are ignored;
 *   - (see below for the quirk flags)
 *   - the random draws come from the env's own SplitMix64 stream, in a fixed
 *     order: one draw at the start of a step when sticky actions are on, one
 *     draw after the start-up sequence when no-op reset is on.  A 64-bit draw
 *     u decides stickiness as (u >> 40) < sticky_q24, and the no-op count is
 *     ((u >> 32) * (noop_max + 1)) >> 32 (Lemire's multiply-shift range
 *     reduction, without rejection).
 *
 * Quirk flags and game descriptors (the variants real games need; Section
 * 3.3 and Appendix B).  The base profile is the VIP one above; each flag
 * switches one behaviour to the SUPER-CHIP / later-interpreter one:
 *   QUIRK_SHIFT_VX      8XY6 / 8XYE shift VX in place (VY is not read);
 *   QUIRK_MEM_KEEP_I    FX55 / FX65 leave I unchanged;
 *   QUIRK_JUMP_VX       BNNN jumps to XNN + VX (X = the second nibble);
 *   QUIRK_NO_VF_RESET   8XY1 / 8XY2 / 8XY3 leave VF unchanged;
 *   QUIRK_PIXEL_WRAP    sprite pixels past the right or bottom edge wrap to
 *                       the other side instead of being clipped;
 *   QUIRK_DISPLAY_WAIT  a DXYN ends the frame: the instructions left in the
 *                       frame's budget are not run (the interpreter waits
 *                       for the display interrupt that starts the next one).
 * Score modes (the forms the game list of Appendix C.3 prints), V = V[score_reg]:
 *   0  V;
 *   1  (V // 10) - (V % 10), Pong's player-minus-opponent score;
 *   2  -(V + V[score_arg]), Airplane's -V[11] - V[12];
 *   3  V when V <= score_arg, else 0, Shooting Stars' cap at 128.
 * Termination: up to two clauses, OR-ed, each a test of one register against
 * a constant with op 0 = never, 1 ==, 2 >=, 3 !=, 4 = either decimal digit
 * (V // 10 or V % 10) equals it (Pong: either score reaches 9).  The first
 * clause is V[term_reg] op term_value, op == unless term_op says otherwise;
 * the second V[term2_reg] op2 term2_value (Space Flight, Airplane, Flight
 * Runner).
 */
#define QUIRK_BASE 1u
#define QUIRK_SHIFT_VX (1u << 1)
#define QUIRK_MEM_KEEP_I (1u << 2)
#define QUIRK_JUMP_VX (1u << 3)
#define QUIRK_NO_VF_RESET (1u << 4)
#define QUIRK_PIXEL_WRAP (1u << 5)
#define QUIRK_DISPLAY_WAIT (1u << 6)
#define QUIRK_ALL 0x7Fu
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MEM_BYTES 4096
#define PROGRAM_ADDR 0x200
#define FONT_ADDR 0x050
#define SCREEN_W 64
#define SCREEN_H 32
#define STACK_DEPTH 16
#define MAX_ROM_BYTES (MEM_BYTES - PROGRAM_ADDR)

/* The 4x5 hexadecimal font, glyphs 0..F, five rows each, high nibble = pixels. */
static const uint8_t oracle_font[80] = {
    0xF0, 0x90, 0x90, 0x90, 0xF0, /* 0 */
    0x20, 0x60, 0x20, 0x20, 0x70, /* 1 */
    0xF0, 0x10, 0xF0, 0x80, 0xF0, /* 2 */
    0xF0, 0x10, 0xF0, 0x10, 0xF0, /* 3 */
    0x90, 0x90, 0xF0, 0x10, 0x10, /* 4 */
    0xF0, 0x80, 0xF0, 0x10, 0xF0, /* 5 */
    0xF0, 0x80, 0xF0, 0x90, 0xF0, /* 6 */
    0xF0, 0x10, 0x20, 0x40, 0x40, /* 7 */
    0xF0, 0x90, 0xF0, 0x90, 0xF0, /* 8 */
    0xF0, 0x90, 0xF0, 0x10, 0xF0, /* 9 */
    0xF0, 0x90, 0xF0, 0x90, 0x90, /* A */
    0xE0, 0x90, 0xE0, 0x90, 0xE0, /* B */
    0xF0, 0x80, 0x80, 0x80, 0xF0, /* C */
    0xE0, 0x90, 0x90, 0x90, 0xE0, /* D */
    0xF0, 0x80, 0xF0, 0x80, 0xF0, /* E */
    0xF0, 0x80, 0xF0, 0x80, 0x80, /* F */
};

/* SUPER-CHIP (the platform extension Section 5 names: a 128x64 display and
 * extra instructions).  The readings taken, in the terms of the Octo
 * manual's SUPER-CHIP mode:
 *   - the display is 128x64; in the 64x32 (low-resolution) mode each pixel
 *     is a 2x2 block of it, and 00FE / 00FF switch to 64x32 / 128x64 and
 *     clear the display; power-on is 64x32;
 *   - DXYN draws 8xN at (VX mod W, VY mod H) of the current mode (W x H),
 *     DXY0 a 16x16 sprite of 32 bytes (two per row); clipping, wrapping and
 *     VF (1 iff a lit pixel was turned off) as for CHIP-8;
 *   - 00CN scrolls down N rows, 00FB right and 00FC left 4 columns, in
 *     pixels of the current mode; 00FD stops the program (it stays on that
 *     instruction);
 *   - FX30 points I at the 8x10 glyph of digit VX & 15 (16 glyphs, 10 bytes
 *     each, at BIGFONT_ADDR); FX75 / FX85 store / load V0..V(min(X, 7)) to
 *     and from eight flag registers, cleared at power-on;
 *   - observations are (4, 128, 64).
 * All other instructions are those of the CHIP-8 profile, quirk flags
 * included. */
#define HSCREEN_W 128
#define HSCREEN_H 64
#define BIGFONT_ADDR 0x0A0

/* The 8x10 digit glyphs 0..F of FX30 (drawn for this oracle; the paper fixes
 * none), ten rows each, bit 7 = leftmost pixel. */
static const uint8_t oracle_bigfont[160] = {
    0x3C, 0x66, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0x66, 0x3C, /* 0 */
    0x18, 0x38, 0x78, 0x18, 0x18, 0x18, 0x18, 0x18, 0x18, 0x7E, /* 1 */
    0x7E, 0xC3, 0x03, 0x03, 0x06, 0x1C, 0x30, 0x60, 0xC0, 0xFF, /* 2 */
    0x7E, 0xC3, 0x03, 0x03, 0x3E, 0x03, 0x03, 0x03, 0xC3, 0x7E, /* 3 */
    0x06, 0x0E, 0x1E, 0x36, 0x66, 0xC6, 0xFF, 0x06, 0x06, 0x06, /* 4 */
    0xFF, 0xC0, 0xC0, 0xC0, 0xFE, 0x03, 0x03, 0x03, 0xC3, 0x7E, /* 5 */
    0x3E, 0x60, 0xC0, 0xC0, 0xFE, 0xC3, 0xC3, 0xC3, 0xC3, 0x7E, /* 6 */
    0xFF, 0x03, 0x06, 0x0C, 0x18, 0x30, 0x30, 0x30, 0x30, 0x30, /* 7 */
    0x7E, 0xC3, 0xC3, 0xC3, 0x7E, 0xC3, 0xC3, 0xC3, 0xC3, 0x7E, /* 8 */
    0x7E, 0xC3, 0xC3, 0xC3, 0xC3, 0x7F, 0x03, 0x03, 0x06, 0x7C, /* 9 */
    0x3C, 0x66, 0xC3, 0xC3, 0xC3, 0xFF, 0xC3, 0xC3, 0xC3, 0xC3, /* A */
    0xFE, 0xC3, 0xC3, 0xC3, 0xFE, 0xC3, 0xC3, 0xC3, 0xC3, 0xFE, /* B */
    0x7E, 0xC3, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0xC3, 0x7E, /* C */
    0xFC, 0xC6, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC3, 0xC6, 0xFC, /* D */
    0xFF, 0xC0, 0xC0, 0xC0, 0xFC, 0xC0, 0xC0, 0xC0, 0xC0, 0xFF, /* E */
    0xFF, 0xC0, 0xC0, 0xC0, 0xFC, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, /* F */
};

/* SUPER-CHIP part of a machine, allocated only for SUPER-CHIP machines. */
typedef struct {
    uint8_t hires;                       /* 1: 128x64 mode */
    uint8_t rpl[8];                      /* FX75 / FX85 flag registers */
    uint8_t hd[HSCREEN_H][HSCREEN_W];    /* hd[y][x] is 0 or 1 */
    uint8_t hist[3][HSCREEN_H][HSCREEN_W]; /* the env's three previous frames, oldest first */
} oracle_schip;

/* One emulated machine (Appendix B.2). */
typedef struct {
    uint8_t v[16];
    uint16_t i;
    uint16_t pc;
    uint8_t sp;
    uint8_t dt;
    uint8_t st;
    uint16_t stack[STACK_DEPTH];
    uint8_t mem[MEM_BYTES];
    uint8_t disp[SCREEN_H][SCREEN_W]; /* disp[y][x] is 0 or 1 */
    uint64_t rng;                     /* SplitMix64 state */
    uint32_t quirks;                  /* QUIRK_* flags; 0 or QUIRK_BASE = the VIP profile */
    oracle_schip *sx;                 /* SUPER-CHIP state, NULL for a CHIP-8 machine */
} oracle_machine;

/* Exported snapshot of one environment.  Field order is part of the
 * oracle's ctypes interface (oracle.py mirrors it). */
typedef struct {
    uint8_t v[16];
    uint16_t i;
    uint16_t pc;
    uint8_t sp;
    uint8_t dt;
    uint8_t st;
    uint8_t prev_key;   /* key held in the previous step (sticky actions), 16 = none */
    uint16_t stack[STACK_DEPTH];
    uint32_t t;
    int32_t prev_score;
    uint64_t rng;
    uint8_t mem[MEM_BYTES];
    uint8_t disp[SCREEN_H][SCREEN_W];
    uint8_t hist[3][SCREEN_H][SCREEN_W];
} oracle_state;

/* One RL environment around a machine (Section 3.2, "Environment integration"). */
typedef struct {
    oracle_machine m;
    uint8_t hist[3][SCREEN_H][SCREEN_W]; /* the three frames before the current one, oldest first */
    uint32_t t;                          /* steps since the last reset */
    int32_t prev_score;
    uint16_t rom;
    uint32_t horizon;
    int prev_key;                        /* key held in the previous step, -1 = none */
} oracle_env;

typedef struct {
    int num_envs;
    int num_roms;
    uint8_t (*rom)[MAX_ROM_BYTES];
    uint32_t *rom_len;
    uint8_t (*action_keys)[16];
    uint8_t *num_actions;
    uint8_t *score_reg;
    uint8_t *term_reg;
    uint8_t *term_value;
    int instr_per_frame;
    int frame_skip;
    uint32_t sticky_q24;                 /* environment wrappers, off when zero */
    uint32_t noop_max;
    uint8_t *startup_len;                /* [R] */
    uint8_t (*startup_keys)[16];         /* [R][16], 16 = no key */
    uint32_t quirks;
    uint8_t *score_mode;                 /* [R] or NULL (all 0) */
    uint8_t *score_arg;                  /* [R]: register (mode 2) or cap (mode 3) */
    uint8_t *term_op;                    /* [R] or NULL (all 1, ==) */
    uint8_t *term2_op;                   /* [R]: 0 none, 1 ==, 2 >=, 3 !=, 4 digit == ; or NULL */
    uint8_t *term2_reg;
    uint8_t *term2_value;
    int schip;                           /* 1: SUPER-CHIP machines */
    uint32_t *pc_hist;                   /* [R][4096] executed instructions by PC, or NULL */
    uint32_t *op_hist;                   /* [R][65536] executed instructions by word, or NULL */
    oracle_env *env;
} oracle_batch;

/* Observation bytes of one env: (4, 64, 32), or (4, 128, 64) for SUPER-CHIP. */
static size_t obs_bytes(const oracle_batch *b)
{
    return b->schip ? 4 * HSCREEN_W * HSCREEN_H : 4 * SCREEN_W * SCREEN_H;
}

/* ------------------------------------------------------------------ */
/* Random bytes for CXNN: SplitMix64.  The state advances by the golden */
/* gamma, the output is the published 64-bit finaliser of the new      */
/* state, and CXNN keeps its top byte.                                   */
/* ------------------------------------------------------------------ */
uint64_t oracle_splitmix64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ */
/* Machine                                                              */
/* ------------------------------------------------------------------ */

/* Power-on state (Section 3.2, "ROM loading and initialization"): memory
 * cleared, font at 0x50, program at 0x200, registers, I, stack and timers
 * zero, PC = 0x200, display cleared.  The RNG stream is left as it is. */
void oracle_machine_load(oracle_machine *m, const uint8_t *rom, uint32_t len)
{
    memset(m->v, 0, sizeof m->v);
    m->i = 0;
    m->pc = PROGRAM_ADDR;
    m->sp = 0;
    m->dt = 0;
    m->st = 0;
    memset(m->stack, 0, sizeof m->stack);
    memset(m->mem, 0, sizeof m->mem);
    memcpy(m->mem + FONT_ADDR, oracle_font, sizeof oracle_font);
    memcpy(m->mem + PROGRAM_ADDR, rom, len);
    memset(m->disp, 0, sizeof m->disp);
    if (m->sx) {
        memcpy(m->mem + BIGFONT_ADDR, oracle_bigfont, sizeof oracle_bigfont);
        m->sx->hires = 0;
        memset(m->sx->rpl, 0, sizeof m->sx->rpl);
        memset(m->sx->hd, 0, sizeof m->sx->hd);
    }
}

/* SUPER-CHIP DXYN / DXY0 (see the SUPER-CHIP notes above). */
static void schip_draw(oracle_machine *m, int x, int y, int n)
{
    oracle_schip *sx = m->sx;
    int scale = sx->hires ? 1 : 2;
    int W = HSCREEN_W / scale, H = HSCREEN_H / scale;
    int w = n == 0 ? 16 : 8, h = n == 0 ? 16 : n;
    int x0 = m->v[x] % W, y0 = m->v[y] % H;
    int wrap = (m->quirks & QUIRK_PIXEL_WRAP) != 0;
    int collided = 0;
    for (int row = 0; row < h; row++) {
        int py = y0 + row;
        if (py >= H) {
            if (!wrap)
                break;
            py -= H;
        }
        for (int col = 0; col < w; col++) {
            int px = x0 + col;
            if (px >= W) {
                if (!wrap)
                    break;
                px -= W;
            }
            uint8_t bits = m->mem[(m->i + row * (w / 8) + col / 8) & 0xFFF];
            if (!((bits >> (7 - col % 8)) & 1))
                continue;
            for (int dy = 0; dy < scale; dy++)
                for (int dx = 0; dx < scale; dx++) {
                    uint8_t *p = &sx->hd[py * scale + dy][px * scale + dx];
                    if (*p)
                        collided = 1;
                    *p ^= 1;
                }
        }
    }
    m->v[0xF] = (uint8_t)collided;
}

/* SUPER-CHIP 00CN / 00FB / 00FC: move the display down, right or left by
 * (dy, dx) physical pixels, clearing what comes in. */
static void schip_scroll(oracle_schip *sx, int dy, int dx)
{
    uint8_t out[HSCREEN_H][HSCREEN_W];
    for (int y = 0; y < HSCREEN_H; y++)
        for (int x = 0; x < HSCREEN_W; x++) {
            int sy = y - dy, sx_ = x - dx;
            out[y][x] = (sy >= 0 && sy < HSCREEN_H && sx_ >= 0 && sx_ < HSCREEN_W) ? sx->hd[sy][sx_] : 0;
        }
    memcpy(sx->hd, out, sizeof out);
}

/* The SUPER-CHIP instructions; returns 1 when op was one of them. */
static int schip_execute(oracle_machine *m, uint16_t op)
{
    oracle_schip *sx = m->sx;
    int x = (op >> 8) & 0xF, scale = sx->hires ? 1 : 2;
    if ((op & 0xFFF0) == 0x00C0) {                /* SCD N */
        schip_scroll(sx, (op & 0xF) * scale, 0);
        return 1;
    }
    switch (op) {
    case 0x00E0: memset(sx->hd, 0, sizeof sx->hd); return 1;
    case 0x00FB: schip_scroll(sx, 0, 4 * scale); return 1;
    case 0x00FC: schip_scroll(sx, 0, -4 * scale); return 1;
    case 0x00FD: m->pc = (uint16_t)((m->pc + MEM_BYTES - 2) & 0xFFF); return 1;
    case 0x00FE: sx->hires = 0; memset(sx->hd, 0, sizeof sx->hd); return 1;
    case 0x00FF: sx->hires = 1; memset(sx->hd, 0, sizeof sx->hd); return 1;
    default: break;
    }
    if ((op >> 12) == 0xD) {
        schip_draw(m, x, (op >> 4) & 0xF, op & 0xF);
        return 1;
    }
    if ((op & 0xF0FF) == 0xF030) {
        m->i = (uint16_t)(BIGFONT_ADDR + 10 * (m->v[x] % 16));
        return 1;
    }
    if ((op & 0xF0FF) == 0xF075 || (op & 0xF0FF) == 0xF085) {
        int top = x < 7 ? x : 7;
        for (int k = 0; k <= top; k++) {
            if ((op & 0xFF) == 0x75)
                sx->rpl[k] = m->v[k];
            else
                m->v[k] = sx->rpl[k];
        }
        return 1;
    }
    return 0;
}

static void skip_next(oracle_machine *m) { m->pc = (uint16_t)((m->pc + 2) & 0xFFF); }

/* Draw an n-row sprite from memory at I with its top-left corner at
 * (VX mod 64, VY mod 32).  Every set sprite bit flips its pixel; pixels past
 * the right or bottom edge are not drawn.  VF = 1 iff some pixel went from
 * 1 to 0 (Appendix B.3). */
static void draw_sprite(oracle_machine *m, int x, int y, int n)
{
    int x0 = m->v[x] % SCREEN_W;
    int y0 = m->v[y] % SCREEN_H;
    int wrap = (m->quirks & QUIRK_PIXEL_WRAP) != 0;
    int collided = 0;
    for (int row = 0; row < n; row++) {
        int py = y0 + row;
        if (py >= SCREEN_H) {
            if (!wrap)
                break;
            py -= SCREEN_H;
        }
        uint8_t bits = m->mem[(m->i + row) & 0xFFF];
        for (int col = 0; col < 8; col++) {
            int px = x0 + col;
            if (px >= SCREEN_W) {
                if (!wrap)
                    break;
                px -= SCREEN_W;
            }
            int sprite_pixel = (bits >> (7 - col)) & 1;
            if (sprite_pixel) {
                if (m->disp[py][px] == 1)
                    collided = 1;
                m->disp[py][px] ^= 1;
            }
        }
    }
    m->v[0xF] = (uint8_t)collided;
}

/* Fetch, decode and execute one instruction.  key is the held key
 * (0..15) or -1 when none is held. */
void oracle_machine_execute(oracle_machine *m, int key)
{
    /* fetch: big-endian 16-bit word at PC, then PC += 2 */
    uint16_t op = (uint16_t)((m->mem[m->pc] << 8) | m->mem[(m->pc + 1) & 0xFFF]);
    m->pc = (uint16_t)((m->pc + 2) & 0xFFF);
    if (m->sx && schip_execute(m, op))
        return;

    /* decode */
    int x = (op >> 8) & 0xF;
    int y = (op >> 4) & 0xF;
    int n = op & 0xF;
    int nn = op & 0xFF;
    int nnn = op & 0xFFF;
    uint8_t *V = m->v;

    /* execute */
    switch (op >> 12) {
    case 0x0:
        if (op == 0x00E0) {                       /* CLS */
            memset(m->disp, 0, sizeof m->disp);
        } else if (op == 0x00EE) {                /* RET */
            m->sp = (uint8_t)((m->sp + STACK_DEPTH - 1) % STACK_DEPTH);
            m->pc = m->stack[m->sp];
        }                                         /* 0NNN: ignored */
        break;
    case 0x1:                                     /* JP NNN */
        m->pc = (uint16_t)nnn;
        break;
    case 0x2:                                     /* CALL NNN */
        m->stack[m->sp] = m->pc;
        m->sp = (uint8_t)((m->sp + 1) % STACK_DEPTH);
        m->pc = (uint16_t)nnn;
        break;
    case 0x3:                                     /* SE VX, NN */
        if (V[x] == nn)
            skip_next(m);
        break;
    case 0x4:                                     /* SNE VX, NN */
        if (V[x] != nn)
            skip_next(m);
        break;
    case 0x5:                                     /* SE VX, VY */
        if (n == 0 && V[x] == V[y])
            skip_next(m);
        break;
    case 0x6:                                     /* LD VX, NN */
        V[x] = (uint8_t)nn;
        break;
    case 0x7:                                     /* ADD VX, NN (no flag) */
        V[x] = (uint8_t)((V[x] + nn) % 256);
        break;
    case 0x8: {
        int vx = V[x], vy = V[y];
        switch (n) {
        case 0x0: V[x] = (uint8_t)vy; break;
        case 0x1: V[x] = (uint8_t)(vx | vy); if (!(m->quirks & QUIRK_NO_VF_RESET)) V[0xF] = 0; break;
        case 0x2: V[x] = (uint8_t)(vx & vy); if (!(m->quirks & QUIRK_NO_VF_RESET)) V[0xF] = 0; break;
        case 0x3: V[x] = (uint8_t)(vx ^ vy); if (!(m->quirks & QUIRK_NO_VF_RESET)) V[0xF] = 0; break;
        case 0x4: {
            int sum = vx + vy;
            V[x] = (uint8_t)(sum % 256);
            V[0xF] = (uint8_t)(sum > 255);
            break;
        }
        case 0x5: {
            int no_borrow = vx >= vy;
            V[x] = (uint8_t)((vx - vy + 256) % 256);
            V[0xF] = (uint8_t)no_borrow;
            break;
        }
        case 0x6: {
            int src = (m->quirks & QUIRK_SHIFT_VX) ? vx : vy;
            int out = src % 2;
            V[x] = (uint8_t)(src / 2);
            V[0xF] = (uint8_t)out;
            break;
        }
        case 0x7: {
            int no_borrow = vy >= vx;
            V[x] = (uint8_t)((vy - vx + 256) % 256);
            V[0xF] = (uint8_t)no_borrow;
            break;
        }
        case 0xE: {
            int src = (m->quirks & QUIRK_SHIFT_VX) ? vx : vy;
            int out = src / 128;
            V[x] = (uint8_t)((src * 2) % 256);
            V[0xF] = (uint8_t)out;
            break;
        }
        default: break;                           /* not an instruction */
        }
        break;
    }
    case 0x9:                                     /* SNE VX, VY */
        if (n == 0 && V[x] != V[y])
            skip_next(m);
        break;
    case 0xA:                                     /* LD I, NNN */
        m->i = (uint16_t)nnn;
        break;
    case 0xB:                                     /* JP V0, NNN (JP VX, XNN with QUIRK_JUMP_VX) */
        m->pc = (uint16_t)((nnn + ((m->quirks & QUIRK_JUMP_VX) ? V[x] : V[0])) & 0xFFF);
        break;
    case 0xC:                                     /* RND VX, NN */
        V[x] = (uint8_t)((oracle_splitmix64_next(&m->rng) >> 56) & (uint64_t)nn);
        break;
    case 0xD:                                     /* DRW VX, VY, N */
        draw_sprite(m, x, y, n);
        break;
    case 0xE:
        if (nn == 0x9E) {                         /* SKP VX */
            if (key >= 0 && key == V[x] % 16)
                skip_next(m);
        } else if (nn == 0xA1) {                  /* SKNP VX */
            if (!(key >= 0 && key == V[x] % 16))
                skip_next(m);
        }
        break;
    case 0xF:
        switch (nn) {
        case 0x07: V[x] = m->dt; break;           /* LD VX, DT */
        case 0x0A:                                /* LD VX, K */
            if (key >= 0)
                V[x] = (uint8_t)key;
            else
                m->pc = (uint16_t)((m->pc + MEM_BYTES - 2) & 0xFFF);
            break;
        case 0x15: m->dt = V[x]; break;           /* LD DT, VX */
        case 0x18: m->st = V[x]; break;           /* LD ST, VX */
        case 0x1E: m->i = (uint16_t)((m->i + V[x]) & 0xFFF); break;
        case 0x29: m->i = (uint16_t)(FONT_ADDR + 5 * (V[x] % 16)); break;
        case 0x33: {                              /* BCD */
            int value = V[x];
            m->mem[m->i] = (uint8_t)(value / 100);
            m->mem[(m->i + 1) & 0xFFF] = (uint8_t)((value / 10) % 10);
            m->mem[(m->i + 2) & 0xFFF] = (uint8_t)(value % 10);
            break;
        }
        case 0x55:                                /* LD [I], V0..VX */
            for (int k = 0; k <= x; k++)
                m->mem[(m->i + k) & 0xFFF] = V[k];
            if (!(m->quirks & QUIRK_MEM_KEEP_I))
                m->i = (uint16_t)((m->i + x + 1) & 0xFFF);
            break;
        case 0x65:                                /* LD V0..VX, [I] */
            for (int k = 0; k <= x; k++)
                V[k] = m->mem[(m->i + k) & 0xFFF];
            if (!(m->quirks & QUIRK_MEM_KEEP_I))
                m->i = (uint16_t)((m->i + x + 1) & 0xFFF);
            break;
        default: break;
        }
        break;
    }
}

/* One 60 Hz timer tick: both timers count down to zero. */
void oracle_machine_tick(oracle_machine *m)
{
    if (m->dt > 0)
        m->dt--;
    if (m->st > 0)
        m->st--;
}

/* ------------------------------------------------------------------ */
/* Environment                                                          */
/* ------------------------------------------------------------------ */

/* One environment step's worth of emulation with `key` held (-1: none).
 * With an execution profile attached, every instruction is counted by the
 * env's ROM and its PC, and by its 16-bit word, before it runs. */
static void run_step_frames(const oracle_batch *b, oracle_env *e, int key)
{
    oracle_machine *m = &e->m;
    for (int f = 0; f < b->frame_skip; f++) {
        for (int k = 0; k < b->instr_per_frame; k++) {
            int draws = (m->mem[m->pc] >> 4) == 0xD;
            if (b->pc_hist) {
                uint16_t op = (uint16_t)((m->mem[m->pc] << 8) | m->mem[(m->pc + 1) & 0xFFF]);
                b->pc_hist[(size_t)e->rom * MEM_BYTES + m->pc]++;
                b->op_hist[(size_t)e->rom * 65536 + op]++;
            }
            oracle_machine_execute(m, key);
            if (draws && (m->quirks & QUIRK_DISPLAY_WAIT))
                break;
        }
        oracle_machine_tick(m);
    }
}

/* Score of an env (Section 3.3), in the ROM's score mode (see the header). */
static int32_t env_score(const oracle_batch *b, const oracle_env *e)
{
    int r = e->rom;
    int v = e->m.v[b->score_reg[r]];
    int mode = b->score_mode ? b->score_mode[r] : 0;
    switch (mode) {
    case 1:
        return v / 10 - v % 10;
    case 2:
        return -(v + e->m.v[b->score_arg[r] & 15]);
    case 3:
        return v <= b->score_arg[r] ? v : 0;
    default:
        return v;
    }
}

/* One termination clause: register value v against constant c. */
static int clause_holds(int op, int v, int c)
{
    switch (op) {
    case 1:
        return v == c;
    case 2:
        return v >= c;
    case 3:
        return v != c;
    case 4:
        return v / 10 == c || v % 10 == c;
    default:
        return 0;
    }
}

/* Termination (Section 3.3): either clause holds. */
static int env_terminated(const oracle_batch *b, const oracle_env *e)
{
    int r = e->rom;
    int t = clause_holds(b->term_op ? b->term_op[r] : 1, e->m.v[b->term_reg[r]], b->term_value[r]);
    if (b->term2_op)
        t = t || clause_holds(b->term2_op[r], e->m.v[b->term2_reg[r]], b->term2_value[r]);
    return t;
}

/* Reset: power-on, then the ROM's start-up sequence and the no-op steps of
 * the no-op-reset wrapper (see the header). */
static void env_reset(const oracle_batch *b, oracle_env *e)
{
    oracle_machine_load(&e->m, b->rom[e->rom], b->rom_len[e->rom]);
    if (b->startup_len) {
        for (int i = 0; i < b->startup_len[e->rom]; i++) {
            int k = b->startup_keys[e->rom][i];
            run_step_frames(b, e, k < 16 ? k : -1);
        }
    }
    if (b->noop_max) {
        uint64_t u = oracle_splitmix64_next(&e->m.rng);
        uint64_t n = ((u >> 32) * ((uint64_t)b->noop_max + 1)) >> 32;
        for (uint64_t i = 0; i < n; i++)
            run_step_frames(b, e, -1);
    }
    for (int k = 0; k < 3; k++)
        memcpy(e->hist[k], e->m.disp, sizeof e->m.disp);
    if (e->m.sx)
        for (int k = 0; k < 3; k++)
            memcpy(e->m.sx->hist[k], e->m.sx->hd, sizeof e->m.sx->hd);
    e->t = 0;
    e->prev_score = env_score(b, e);
    e->prev_key = -1;
}

/* obs[k][x][y] for k = 0..3: the three stored frames then the display. */
static void env_observe(const oracle_env *e, uint8_t *obs)
{
    if (e->m.sx) {                    /* SUPER-CHIP: obs[k][x][y], 128 x 64 */
        const oracle_schip *sx = e->m.sx;
        for (int k = 0; k < 4; k++) {
            const uint8_t(*frame)[HSCREEN_W] = (k < 3) ? sx->hist[k] : sx->hd;
            for (int x = 0; x < HSCREEN_W; x++)
                for (int y = 0; y < HSCREEN_H; y++)
                    obs[(k * HSCREEN_W + x) * HSCREEN_H + y] = frame[y][x];
        }
        return;
    }
    for (int k = 0; k < 4; k++) {
        const uint8_t(*frame)[SCREEN_W] = (k < 3) ? e->hist[k] : e->m.disp;
        for (int x = 0; x < SCREEN_W; x++)
            for (int y = 0; y < SCREEN_H; y++)
                obs[(k * SCREEN_W + x) * SCREEN_H + y] = frame[y][x];
    }
}

static void env_step(const oracle_batch *b, oracle_env *e, int32_t action, uint8_t *obs,
                     float *reward, uint8_t *done)
{
    int r = e->rom;
    int key = -1;
    if (action >= 0 && action < b->num_actions[r])
        key = b->action_keys[r][action];
    /* sticky actions: the previous step's key again with probability sticky_q24 / 2^24 */
    if (b->sticky_q24 && (oracle_splitmix64_next(&e->m.rng) >> 40) < b->sticky_q24)
        key = e->prev_key;
    e->prev_key = key;

    uint8_t before[SCREEN_H][SCREEN_W];
    memcpy(before, e->m.disp, sizeof before);
    oracle_schip *sx = e->m.sx;
    if (sx) {                         /* the SUPER-CHIP frame history moves the same way */
        memcpy(sx->hist[0], sx->hist[1], sizeof sx->hd);
        memcpy(sx->hist[1], sx->hist[2], sizeof sx->hd);
        memcpy(sx->hist[2], sx->hd, sizeof sx->hd);
    }

    run_step_frames(b, e, key);

    memcpy(e->hist[0], e->hist[1], sizeof before);
    memcpy(e->hist[1], e->hist[2], sizeof before);
    memcpy(e->hist[2], before, sizeof before);

    int32_t score = env_score(b, e);
    *reward = (float)(score - e->prev_score);
    e->prev_score = score;

    int terminated = env_terminated(b, e);
    e->t += 1;
    int truncated = e->horizon > 0 && e->t >= e->horizon;
    *done = (uint8_t)(terminated | (truncated << 1));
    if (terminated || truncated)
        env_reset(b, e);
    if (obs)
        env_observe(e, obs);
}

/* ------------------------------------------------------------------ */
/* Exported interface (ctypes)                                          */
/* ------------------------------------------------------------------ */

oracle_batch *oracle_create(int num_envs, int num_roms, const uint8_t *rom_data,
                            const uint32_t *rom_offset, const uint32_t *rom_len,
                            const uint16_t *env_rom, const uint8_t *action_keys,
                            const uint8_t *num_actions, const uint8_t *score_reg,
                            const uint8_t *term_reg, const uint8_t *term_value,
                            const uint32_t *horizon, const uint64_t *env_seed,
                            int instr_per_frame, int frame_skip)
{
    if (num_envs < 0 || num_roms < 1 || instr_per_frame < 0 || frame_skip < 0)
        return NULL;
    for (int r = 0; r < num_roms; r++)
        if (rom_len[r] > MAX_ROM_BYTES || score_reg[r] > 15 || term_reg[r] > 15 ||
            num_actions[r] > 16)
            return NULL;
    for (int e = 0; e < num_envs; e++)
        if (env_rom[e] >= num_roms)
            return NULL;
    oracle_batch *b = calloc(1, sizeof *b);
    if (!b)
        return NULL;
    b->num_envs = num_envs;
    b->num_roms = num_roms;
    b->rom = calloc((size_t)num_roms, sizeof *b->rom);
    b->rom_len = calloc((size_t)num_roms, sizeof *b->rom_len);
    b->action_keys = calloc((size_t)num_roms, sizeof *b->action_keys);
    b->num_actions = calloc((size_t)num_roms, 1);
    b->score_reg = calloc((size_t)num_roms, 1);
    b->term_reg = calloc((size_t)num_roms, 1);
    b->term_value = calloc((size_t)num_roms, 1);
    b->env = calloc((size_t)(num_envs > 0 ? num_envs : 1), sizeof *b->env);
    if (!b->rom || !b->rom_len || !b->action_keys || !b->num_actions || !b->score_reg ||
        !b->term_reg || !b->term_value || !b->env) {
        free(b->rom); free(b->rom_len); free(b->action_keys); free(b->num_actions);
        free(b->score_reg); free(b->term_reg); free(b->term_value); free(b->env); free(b);
        return NULL;
    }
    for (int r = 0; r < num_roms; r++) {
        memcpy(b->rom[r], rom_data + rom_offset[r], rom_len[r]);
        b->rom_len[r] = rom_len[r];
        memcpy(b->action_keys[r], action_keys + 16 * r, 16);
        b->num_actions[r] = num_actions[r];
        b->score_reg[r] = score_reg[r];
        b->term_reg[r] = term_reg[r];
        b->term_value[r] = term_value[r];
    }
    b->instr_per_frame = instr_per_frame;
    b->frame_skip = frame_skip;
    for (int e = 0; e < num_envs; e++) {
        b->env[e].rom = env_rom[e];
        b->env[e].horizon = horizon[e];
        b->env[e].m.rng = env_seed[e];
        env_reset(b, &b->env[e]);
    }
    return b;
}

void oracle_destroy(oracle_batch *b)
{
    if (!b)
        return;
    for (int e = 0; e < b->num_envs; e++)
        free(b->env[e].m.sx);
    free(b->rom); free(b->rom_len); free(b->action_keys); free(b->num_actions);
    free(b->score_reg); free(b->term_reg); free(b->term_value); free(b->env);
    free(b->startup_len); free(b->startup_keys);
    free(b->score_mode); free(b->score_arg); free(b->term_op);
    free(b->term2_op); free(b->term2_reg); free(b->term2_value);
    free(b);
}

/* Configure the quirk flags and the game descriptors (score mode and its
 * argument, the ops of both termination clauses, the second clause's register
 * and constant; see the header).  score_mode and score_arg come together, as
 * do term2_op, term2_reg and term2_value; any group may be NULL.  Out-of-range
 * values change nothing and return -1.  They apply from the next reset and
 * step on; callers reset after this. */
static uint8_t *copy_bytes(const uint8_t *src, int n, int *fail)
{
    uint8_t *dst = NULL;
    if (src) {
        dst = malloc((size_t)n);
        if (dst)
            memcpy(dst, src, (size_t)n);
        else
            *fail = 1;
    }
    return dst;
}

int oracle_set_profile(oracle_batch *b, uint32_t quirks, const uint8_t *score_mode, const uint8_t *score_arg,
                       const uint8_t *term_op, const uint8_t *term2_op, const uint8_t *term2_reg,
                       const uint8_t *term2_value)
{
    int R = b->num_roms, fail = 0;
    if ((quirks & ~QUIRK_ALL) || !(quirks & QUIRK_BASE))
        return -1;
    if (!score_mode != !score_arg || !term2_op != !term2_reg || !term2_op != !term2_value)
        return -1;
    for (int r = 0; r < R; r++) {
        if (score_mode && (score_mode[r] > 3 || (score_mode[r] == 2 && score_arg[r] > 15)))
            return -1;
        if (term_op && term_op[r] > 4)
            return -1;
        if (term2_op && (term2_op[r] > 4 || term2_reg[r] > 15))
            return -1;
    }
    free(b->score_mode); free(b->score_arg); free(b->term_op);
    free(b->term2_op); free(b->term2_reg); free(b->term2_value);
    b->score_mode = copy_bytes(score_mode, R, &fail);
    b->score_arg = copy_bytes(score_arg, R, &fail);
    b->term_op = copy_bytes(term_op, R, &fail);
    b->term2_op = copy_bytes(term2_op, R, &fail);
    b->term2_reg = copy_bytes(term2_reg, R, &fail);
    b->term2_value = copy_bytes(term2_value, R, &fail);
    if (fail)
        return -2;
    b->quirks = quirks;
    for (int e = 0; e < b->num_envs; e++)
        b->env[e].m.quirks = quirks;
    return 0;
}

/* Configure the environment wrappers (all off after oracle_create).  They
 * apply from the next reset and step on; callers reset after this.
 * startup_len / startup_keys may be NULL (no start-up sequences). */
int oracle_set_wrappers(oracle_batch *b, uint32_t sticky_q24, uint32_t noop_max,
                        const uint8_t *startup_len, const uint8_t *startup_keys)
{
    if (sticky_q24 > (1u << 24) || noop_max > 1000)
        return -1;
    free(b->startup_len); free(b->startup_keys);
    b->startup_len = NULL;
    b->startup_keys = NULL;
    if (startup_len) {
        b->startup_len = calloc((size_t)b->num_roms, 1);
        b->startup_keys = calloc((size_t)b->num_roms, sizeof *b->startup_keys);
        if (!b->startup_len || !b->startup_keys)
            return -2;
        for (int r = 0; r < b->num_roms; r++) {
            if (startup_len[r] > 16)
                return -1;
            b->startup_len[r] = startup_len[r];
            memcpy(b->startup_keys[r], startup_keys + 16 * r, 16);
        }
    }
    b->sticky_q24 = sticky_q24;
    b->noop_max = noop_max;
    return 0;
}

/* Reset the envs whose mask byte is non-zero (all when mask is NULL) and
 * write the observation of every env into obs [E][4][64][32] if given. */
void oracle_reset(oracle_batch *b, const uint8_t *mask, uint8_t *obs)
{
    for (int e = 0; e < b->num_envs; e++) {
        if (!mask || mask[e])
            env_reset(b, &b->env[e]);
        if (obs)
            env_observe(&b->env[e], obs + (size_t)e * obs_bytes(b));
    }
}

/* One environment step of every env.  obs may be NULL (not materialised). */
void oracle_step(oracle_batch *b, const int32_t *action, uint8_t *obs, float *reward,
                 uint8_t *done)
{
    for (int e = 0; e < b->num_envs; e++)
        env_step(b, &b->env[e], action[e], obs ? obs + (size_t)e * obs_bytes(b) : NULL, &reward[e], &done[e]);
}

typedef struct {
    oracle_batch *b;
    int first, last, steps;
    const int32_t *action; /* [steps][E] */
    uint8_t *obs;          /* [E][4][64][32], rewritten every step */
    float *reward;         /* [steps][E] */
    uint8_t *done;         /* [steps][E] */
} oracle_shard;

static void *run_shard(void *arg)
{
    oracle_shard *s = arg;
    int E = s->b->num_envs;
    for (int k = 0; k < s->steps; k++)
        for (int e = s->first; e < s->last; e++)
            env_step(s->b, &s->b->env[e], s->action[(size_t)k * E + e],
                     s->obs + (size_t)e * obs_bytes(s->b),
                     &s->reward[(size_t)k * E + e], &s->done[(size_t)k * E + e]);
    return NULL;
}

/* Run `steps` steps with the envs split into `threads` contiguous shards,
 * one POSIX thread each; observations are materialised every step into one
 * reused [E][4][64][32] buffer.  Returns the number of threads used. */
int oracle_run_threaded(oracle_batch *b, int steps, const int32_t *action, uint8_t *obs,
                        float *reward, uint8_t *done, int threads)
{
    if (threads < 1 || b->pc_hist)
        threads = 1;                  /* the execution profile's counters are not shared safely */
    if (threads > b->num_envs)
        threads = b->num_envs > 0 ? b->num_envs : 1;
    pthread_t *tid = calloc((size_t)threads, sizeof *tid);
    unsigned char *started = calloc((size_t)threads, 1);
    oracle_shard *sh = calloc((size_t)threads, sizeof *sh);
    int used = 0;
    if (!tid || !started || !sh) {    /* no memory for the bookkeeping: run every env here */
        free(tid);
        free(started);
        free(sh);
        oracle_shard all = {b, 0, b->num_envs, steps, action, obs, reward, done};
        run_shard(&all);
        return 1;
    }
    for (int t = 0; t < threads; t++) {
        sh[t].b = b;
        sh[t].first = (int)((long)b->num_envs * t / threads);
        sh[t].last = (int)((long)b->num_envs * (t + 1) / threads);
        sh[t].steps = steps;
        sh[t].action = action;
        sh[t].obs = obs;
        sh[t].reward = reward;
        sh[t].done = done;
    }
    for (int t = 0; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, run_shard, &sh[t]) == 0) {
            started[t] = 1;
            used++;
        } else {
            run_shard(&sh[t]);        /* no thread: this shard runs here */
        }
    }
    for (int t = 0; t < threads; t++)
        if (started[t])               /* join only the threads that were created */
            pthread_join(tid[t], NULL);
    free(tid);
    free(started);
    free(sh);
    return used > 0 ? threads : 1;
}

void oracle_get_state(const oracle_batch *b, int first, int count, oracle_state *out)
{
    for (int k = 0; k < count; k++) {
        const oracle_env *e = &b->env[first + k];
        oracle_state *s = &out[k];
        memset(s, 0, sizeof *s);
        memcpy(s->v, e->m.v, 16);
        s->i = e->m.i;
        s->pc = e->m.pc;
        s->sp = e->m.sp;
        s->dt = e->m.dt;
        s->st = e->m.st;
        memcpy(s->stack, e->m.stack, sizeof s->stack);
        s->t = e->t;
        s->prev_score = e->prev_score;
        s->rng = e->m.rng;
        s->prev_key = (uint8_t)(e->prev_key < 0 ? 16 : e->prev_key);
        memcpy(s->mem, e->m.mem, MEM_BYTES);
        memcpy(s->disp, e->m.disp, sizeof s->disp);
        memcpy(s->hist, e->hist, sizeof s->hist);
    }
}

void oracle_set_state(oracle_batch *b, int first, int count, const oracle_state *in)
{
    for (int k = 0; k < count; k++) {
        oracle_env *e = &b->env[first + k];
        const oracle_state *s = &in[k];
        memcpy(e->m.v, s->v, 16);
        e->m.i = s->i & 0xFFF;
        e->m.pc = s->pc & 0xFFF;
        e->m.sp = s->sp % STACK_DEPTH;
        e->m.dt = s->dt;
        e->m.st = s->st;
        for (int j = 0; j < STACK_DEPTH; j++)
            e->m.stack[j] = s->stack[j] & 0xFFF;
        e->t = s->t;
        e->prev_score = s->prev_score;
        e->m.rng = s->rng;
        e->prev_key = s->prev_key < 16 ? s->prev_key : -1;
        memcpy(e->m.mem, s->mem, MEM_BYTES);
        for (int y = 0; y < SCREEN_H; y++)
            for (int x = 0; x < SCREEN_W; x++) {
                e->m.disp[y][x] = s->disp[y][x] & 1;
                for (int h = 0; h < 3; h++)
                    e->hist[h][y][x] = s->hist[h][y][x] & 1;
            }
    }
}

int oracle_state_size(void) { return (int)sizeof(oracle_state); }
int oracle_machine_size(void) { return (int)sizeof(oracle_machine); }

/* Single-machine access for unit tests of individual instructions. */
oracle_machine *oracle_machine_new(void) { return calloc(1, sizeof(oracle_machine)); }
void oracle_machine_free(oracle_machine *m)
{
    if (m)
        free(m->sx);
    free(m);
}

/* SUPER-CHIP view of one machine or env (tests): mode, flag registers,
 * display and, for an env, its three previous frames. */
typedef struct {
    uint8_t hires;
    uint8_t rpl[8];
    uint8_t hd[HSCREEN_H][HSCREEN_W];
    uint8_t hist[3][HSCREEN_H][HSCREEN_W];
} oracle_schip_view;

int oracle_schip_view_size(void) { return (int)sizeof(oracle_schip_view); }

/* Make a single machine a SUPER-CHIP one (or back); reload it after this. */
int oracle_machine_set_platform(oracle_machine *m, int schip)
{
    free(m->sx);
    m->sx = schip ? calloc(1, sizeof(oracle_schip)) : NULL;
    return (schip && !m->sx) ? -2 : 0;
}

static void schip_to_view(const oracle_schip *sx, oracle_schip_view *v)
{
    v->hires = sx->hires;
    memcpy(v->rpl, sx->rpl, sizeof v->rpl);
    memcpy(v->hd, sx->hd, sizeof v->hd);
    memcpy(v->hist, sx->hist, sizeof v->hist);
}

int oracle_machine_get_schip(const oracle_machine *m, oracle_schip_view *v)
{
    if (!m->sx)
        return -1;
    schip_to_view(m->sx, v);
    return 0;
}

int oracle_machine_set_schip(oracle_machine *m, const oracle_schip_view *v)
{
    if (!m->sx)
        return -1;
    m->sx->hires = v->hires ? 1 : 0;
    memcpy(m->sx->rpl, v->rpl, sizeof v->rpl);
    for (int y = 0; y < HSCREEN_H; y++)
        for (int x = 0; x < HSCREEN_W; x++)
            m->sx->hd[y][x] = v->hd[y][x] & 1;
    return 0;
}

/* Make every env of a batch a SUPER-CHIP machine (schip = 1) or a CHIP-8
 * one; applies from the next reset on, so callers reset after this. */
/* Attach (or, with NULL, detach) an execution profile: pc_hist [R][4096]
 * and op_hist [R][65536] counters owned by the caller, which every
 * instruction run from then on increments (step, reset steps and start-up
 * sequences alike).  The counters are plain, so a profiled batch runs its
 * threaded rollouts on one thread. */
int oracle_set_exec_profile(oracle_batch *b, uint32_t *pc_hist, uint32_t *op_hist)
{
    if ((pc_hist == NULL) != (op_hist == NULL))
        return -1;
    b->pc_hist = pc_hist;
    b->op_hist = op_hist;
    return 0;
}

int oracle_set_platform(oracle_batch *b, int schip)
{
    for (int e = 0; e < b->num_envs; e++)
        if (oracle_machine_set_platform(&b->env[e].m, schip) != 0)
            return -2;
    b->schip = schip ? 1 : 0;
    return 0;
}

void oracle_get_schip(const oracle_batch *b, int first, int count, oracle_schip_view *out)
{
    for (int k = 0; k < count; k++)
        if (b->env[first + k].m.sx)
            schip_to_view(b->env[first + k].m.sx, &out[k]);
}
/* Quirk flags of a single machine (QUIRK_*; a new machine has none, which
 * behaves as the base profile). */
void oracle_machine_set_quirks(oracle_machine *m, uint32_t quirks) { m->quirks = quirks; }
void oracle_machine_to_state(const oracle_machine *m, oracle_state *s)
{
    memset(s, 0, sizeof *s);
    memcpy(s->v, m->v, 16);
    s->i = m->i;
    s->pc = m->pc;
    s->sp = m->sp;
    s->dt = m->dt;
    s->st = m->st;
    memcpy(s->stack, m->stack, sizeof s->stack);
    s->rng = m->rng;
    memcpy(s->mem, m->mem, MEM_BYTES);
    memcpy(s->disp, m->disp, sizeof s->disp);
}
void oracle_machine_from_state(oracle_machine *m, const oracle_state *s)
{
    memcpy(m->v, s->v, 16);
    m->i = s->i & 0xFFF;
    m->pc = s->pc & 0xFFF;
    m->sp = s->sp % STACK_DEPTH;
    m->dt = s->dt;
    m->st = s->st;
    for (int j = 0; j < STACK_DEPTH; j++)
        m->stack[j] = s->stack[j] & 0xFFF;
    m->rng = s->rng;
    memcpy(m->mem, s->mem, MEM_BYTES);
    for (int y = 0; y < SCREEN_H; y++)
        for (int x = 0; x < SCREEN_W; x++)
            m->disp[y][x] = s->disp[y][x] & 1;
}

/* Execute one opcode on `count` machines that differ only in V, I and RNG
 * state (exhaustive operand sweeps in the tests).  The opcode sits at 0x200
 * of an otherwise freshly loaded machine. */
void oracle_execute_batch(uint16_t op, int key, int count, const uint8_t *v_in,
                          const uint16_t *i_in, const uint64_t *rng_in, uint8_t *v_out,
                          uint16_t *i_out, uint16_t *pc_out, uint8_t *mem_out /* [count][4096] or NULL */)
{
    static __thread oracle_machine m;
    uint8_t rom[2] = {(uint8_t)(op >> 8), (uint8_t)(op & 0xFF)};
    for (int k = 0; k < count; k++) {
        oracle_machine_load(&m, rom, 2);
        memcpy(m.v, v_in + 16 * k, 16);
        m.i = i_in ? (uint16_t)(i_in[k] & 0xFFF) : 0;
        m.rng = rng_in ? rng_in[k] : 0;
        oracle_machine_execute(&m, key);
        memcpy(v_out + 16 * k, m.v, 16);
        if (i_out)
            i_out[k] = m.i;
        if (pc_out)
            pc_out[k] = m.pc;
        if (mem_out)
            memcpy(mem_out + (size_t)MEM_BYTES * k, m.mem, MEM_BYTES);
    }
}

/* Run n_instr instructions (no timer ticks) on each of `count` full
 * snapshots in place; display, memory and registers all come from the
 * snapshot.  Used by the tests to start from arbitrary machine states. */
void oracle_execute_states(oracle_state *states, int count, int key, int n_instr)
{
    static __thread oracle_machine m;
    for (int k = 0; k < count; k++) {
        oracle_machine_from_state(&m, &states[k]);
        for (int j = 0; j < n_instr; j++)
            oracle_machine_execute(&m, key);
        uint32_t t = states[k].t;
        int32_t prev = states[k].prev_score;
        uint8_t hist[3][SCREEN_H][SCREEN_W];
        memcpy(hist, states[k].hist, sizeof hist);
        oracle_machine_to_state(&m, &states[k]);
        states[k].t = t;
        states[k].prev_score = prev;
        memcpy(states[k].hist, hist, sizeof hist);
    }
}
