/*
 * octax.h - C ABI of the MI355X batched CHIP-8 environment library (liboctax.so).
 *
 * The library runs many independent CHIP-8 machines, each wrapped as a
 * reinforcement-learning environment, on one AMD Instinct MI355X (gfx950).
 * What one environment step computes follows the paper "Octax: Accelerated
 * CHIP-8 Arcade Environments for Reinforcement Learning in JAX":
 *   - Section 3.2 ("How does Octax work?"): programs loaded at 0x200 in a 4 KB
 *     memory with the font at 0x50; a fetch-decode-execute cycle over the
 *     35-instruction set; several instructions per 60 Hz frame; delay and
 *     sound timers ticked once per frame; frame skip 4; a (4, 64, 32)
 *     observation of the last four frames; actions mapped to a key subset
 *     plus a no-op; functional state updates (state in, new state out).
 *   - Section 3.3: reward from a score register, termination from a
 *     register test.
 *   - Section 3.4: Gymnax-compatible environments, i.e. automatic reset when
 *     an episode ends, returning the observation of the reset state.
 *   - Appendix B: memory map, registers, 64x32 XOR display with collision
 *     flag, 16-key keypad, timers, 4x5 hex font at 0x050-0x09F.
 * The paper does not print per-instruction semantics; the library fixes one
 * documented profile, OCTAX_QUIRKS_V1:
 *   8XY6/8XYE shift VY into VX (VF = bit shifted out); FX55/FX65 leave
 *   I = I + X + 1; BNNN jumps to NNN + V0; 8XY1/8XY2/8XY3 clear VF; every
 *   flag is written after the result; 8XY5/8XY7 set VF = 1 when there is
 *   no borrow (equal operands included); DXYN starts at (VX mod 64,
 *   VY mod 32), clips at the right and bottom edges and sets VF = 1 iff a
 *   lit pixel was turned off (N = 0 draws nothing); the stack has 16
 *   entries and its pointer wraps; I and PC are 12-bit; instruction words
 *   not in the set do nothing; EX9E/EXA1 test key VX & 15; FX0A with no key
 *   held repeats itself; CXNN = (top byte of the env's next SplitMix64
 *   output) & NN.
 *
 * Environment step (per env): the action selects the held key for the whole
 * step (0 <= a < num_actions: action_keys[rom][a]; any other value: no key);
 * frame_skip frames of instr_per_frame instructions, each frame followed by a
 * timer tick; the new frame joins the observation stack (oldest first, the
 * current display last); reward = score - previous score as a float, the
 * score being V[score_reg] (or a function of it, see h_score_mode);
 * terminated = (V[term_reg] == term_value) (or other clauses, see
 * h_term_op); truncated = (steps since
 * reset >= horizon, when horizon > 0); done = terminated | truncated << 1;
 * on done the env is reset (its RNG stream is not reseeded) and the
 * observation returned is that of the reset state.
 *
 * Conventions for every entry point:
 *   - Return value: OCTAX_OK (0) or a negative OCTAX_E_* code; the message
 *     of the last failure on the calling thread is octax_last_error().  An
 *     argument error enqueues no GPU work.
 *   - Pointers named d_* are device pointers on the engine's GPU, owned by
 *     the caller, contiguous, with the layout given; h_* pointers are host
 *     memory owned by the caller.  The engine owns its own device state.
 *   - reset, step, step_many and graph launches are asynchronous on the
 *     engine's stream; create, destroy, get_state and set_state synchronize.
 *   - Every output is a pure function of the config and the call sequence;
 *     it does not depend on the kernel, the tuning or the env placement.
 *   - Observation layout: uint8 [E][4][64][32] = [env][frame][x][y] (SUPER-CHIP
 *     engines: [E][4][128][64], see octax_config.platform), values
 *     0/1, frame 3 the newest.
 */
#ifndef OCTAX_H
#define OCTAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCTAX_ABI_VERSION 4u
#define OCTAX_QUIRKS_V1 1u

/* Quirk flags, OR-ed with OCTAX_QUIRKS_V1 in the config's quirks field.
 * Games written for later interpreters (SUPER-CHIP and others; the paper's
 * Appendix B lists the variants and Section 3.3 its game set) rely on some
 * of them; each switches one behaviour of the profile above, for every env
 * of the engine:
 *   SHIFT_VX      8XY6 / 8XYE shift VX in place (VY is not read);
 *   MEM_KEEP_I    FX55 / FX65 leave I unchanged;
 *   JUMP_VX       BNNN jumps to XNN + VX, X being the second nibble;
 *   NO_VF_RESET   8XY1 / 8XY2 / 8XY3 leave VF unchanged;
 *   PIXEL_WRAP    DXYN draws all N rows and wraps pixels past the right or
 *                 bottom edge to the other side instead of clipping them;
 *   DISPLAY_WAIT  a DXYN ends its frame: the instructions left in that
 *                 frame's instr_per_frame budget are not run (the VIP waits
 *                 for the display interrupt, which starts the next frame). */
#define OCTAX_QUIRK_SHIFT_VX (1u << 1)
#define OCTAX_QUIRK_MEM_KEEP_I (1u << 2)
#define OCTAX_QUIRK_JUMP_VX (1u << 3)
#define OCTAX_QUIRK_NO_VF_RESET (1u << 4)
#define OCTAX_QUIRK_PIXEL_WRAP (1u << 5)
#define OCTAX_QUIRK_DISPLAY_WAIT (1u << 6)

#define OCTAX_MAX_ROM_BYTES 3584u   /* 0x200..0xFFF */
#define OCTAX_OBS_BYTES 8192u       /* 4 * 64 * 32 */
#define OCTAX_SCHIP_OBS_BYTES 32768u /* 4 * 128 * 64, SUPER-CHIP engines */

enum octax_status {
    OCTAX_OK = 0,
    OCTAX_E_INVALID = -1, /* bad argument or config */
    OCTAX_E_NOMEM = -2,   /* device or host allocation failed; pool full */
    OCTAX_E_HIP = -3,     /* a HIP runtime call failed */
    OCTAX_E_STATE = -4    /* call not valid in the engine's current state */
};

/* Step kernels. */
enum octax_kernel {
    OCTAX_KERNEL_PLAIN = 0, /* one env per lane, state through HBM every step */
    OCTAX_KERNEL_FUSED = 1  /* K steps per launch, LDS-staged ROM and display, coalesced obs */
};

/* Platforms. */
enum octax_platform {
    OCTAX_PLATFORM_CHIP8 = 0,    /* 64x32 display, the profile above */
    OCTAX_PLATFORM_SCHIP = 1     /* SUPER-CHIP: 128x64 display and its instructions (see octax_config) */
};

/* Placement of envs in the engine's state slots. */
enum octax_placement {
    OCTAX_PLACE_IDENTITY = 0,  /* slot = env index */
    OCTAX_PLACE_BY_ROM = 1,    /* slots sorted by ROM id (stable), so workgroups share ROMs */
    OCTAX_PLACE_BY_HORIZON = 2 /* envs in order of truncation horizon (shortest first, 0 = none last,
                                  stable), dealt round-robin over the wavefronts of 64 slots: the envs
                                  that reset most often, whose resets run the start-up and no-op steps
                                  of Section 3.2, land in different wavefronts */
};

typedef struct octax_config {
    uint32_t abi_version;      /* must be OCTAX_ABI_VERSION */
    uint32_t num_envs;         /* E >= 1 */
    uint32_t num_roms;         /* R >= 1 */
    uint32_t instr_per_frame;  /* instructions per 60 Hz frame, 1..1000 */
    uint32_t frame_skip;       /* frames per step, 1..64 (paper default 4) */
    uint32_t quirks;           /* OCTAX_QUIRKS_V1 | any OCTAX_QUIRK_* flags */
    uint32_t kernel;           /* enum octax_kernel */
    uint32_t placement;        /* enum octax_placement */
    uint32_t envs_per_block;   /* fused kernel: envs per workgroup (0 = default) */
    uint32_t lanes_per_env;    /* fused kernel: lanes per env; only 1 is implemented (0 = 1) */
    uint32_t rom_in_lds;       /* fused kernel: 1 = stage ROM images in LDS, 0 = read through L2 */
    uint32_t reserved;
    /* host arrays, copied at create */
    const uint8_t *h_rom_data;     /* concatenated ROM bytes */
    const uint32_t *h_rom_offset;  /* [R] offset of ROM r in h_rom_data */
    const uint32_t *h_rom_len;     /* [R] 0..OCTAX_MAX_ROM_BYTES */
    const uint16_t *h_env_rom;     /* [E] ROM of each env, < R */
    const uint8_t *h_action_keys;  /* [R][16] key of each action */
    const uint8_t *h_num_actions;  /* [R] 0..16; action == num_actions is the no-op */
    const uint8_t *h_score_reg;    /* [R] 0..15 */
    const uint8_t *h_term_reg;     /* [R] 0..15 */
    const uint8_t *h_term_value;   /* [R] */
    const uint32_t *h_horizon;     /* [E] truncation horizon, 0 = none */
    const uint64_t *h_env_seed;    /* [E] initial SplitMix64 state of each env */
    void *stream;                  /* hipStream_t for all work; NULL = null stream */
    /* Environment wrappers (Section 3.2: start-up sequences that skip menus,
     * no-op reset, sticky actions); zero / NULL turns each off.
     *   sticky_q24: at every step the key held in the previous step is held
     *     again with probability sticky_q24 / 2^24 (0..2^24); after a reset
     *     the previous key is none.
     *   every reset (automatic or octax_reset) runs, after power-on, one
     *     environment step per entry of the env's ROM's start-up list with
     *     that key held (h_startup_len [R] entries, 0..16, keys in
     *     h_startup_keys [R][16], 0..15 or 16 = none), then a number of no-op
     *     steps drawn uniformly from 0..noop_max (0..1000).  The frame stack
     *     then holds the resulting display four times, the score baseline is
     *     the score register, and terminations during these steps are ignored.
     *   The draws come from the env's SplitMix64 stream: one at the start of
     *     a step when sticky_q24 != 0, deciding (u >> 40) < sticky_q24; one
     *     after the start-up steps when noop_max != 0, giving
     *     ((u >> 32) * (noop_max + 1)) >> 32 no-op steps. */
    uint32_t sticky_q24;
    uint32_t noop_max;
    const uint8_t *h_startup_len;   /* [R] or NULL */
    const uint8_t *h_startup_keys;  /* [R][16] or NULL (with h_startup_len) */
    /* Game descriptors beyond a score register and one == test, in the
     * forms the paper's game list prints (Section 3.3; Appendix C.3); NULL
     * keeps the plain forms.  With V = V[score_reg]:
     *   h_score_mode [R] with h_score_arg [R] (given together):
     *     0  score = V;
     *     1  score = V / 10 - V % 10 (Pong: two players' points in one
     *        register, player minus opponent);
     *     2  score = -(V + V[h_score_arg]) (Airplane: -V[11] - V[12]);
     *     3  score = V if V <= h_score_arg, else 0 (Shooting Stars' cap).
     *   Termination is two clauses, OR-ed, each comparing a register with a
     *   constant by op 0 = never, 1 ==, 2 >=, 3 !=, 4 = either decimal digit
     *   (V / 10 or V % 10) equals it:
     *     h_term_op [R]: the op of V[term_reg] against term_value (NULL: ==);
     *     h_term2_op, h_term2_reg, h_term2_value [R] (given together): a
     *     second clause V[h_term2_reg] op h_term2_value (Space Flight:
     *     V[9] == 0 or V[12] >= 0x3E). */
    const uint8_t *h_score_mode;    /* [R] 0..3 or NULL */
    const uint8_t *h_score_arg;     /* [R] register 0..15 (mode 2) or cap (mode 3) */
    const uint8_t *h_term_op;       /* [R] 0..4 or NULL */
    const uint8_t *h_term2_op;      /* [R] 0..4 or NULL */
    const uint8_t *h_term2_reg;     /* [R] 0..15 */
    const uint8_t *h_term2_value;   /* [R] */
    /* Platform (enum octax_platform).  SUPER-CHIP is the extension Section 5
     * names: a 128x64 display (the 64x32 mode draws 2x2 blocks on it) and the
     * instructions 00CN (scroll down N rows), 00FB / 00FC (scroll right /
     * left 4 columns; scroll amounts are in pixels of the current mode),
     * 00FD (stop: the program stays on that instruction), 00FE / 00FF (64x32
     * / 128x64 mode, display cleared), DXY0 (16x16 sprite, 32 bytes),
     * FX30 (I = 8x10 glyph of digit VX & 15, 10 bytes each at 0x0A0) and
     * FX75 / FX85 (store / load V0..V(min(X, 7)) in eight flag registers).
     * Power-on is the 64x32 mode with the flag registers cleared.
     * Observations are uint8 [E][4][128][64] = [env][frame][x][y].
     * SUPER-CHIP engines are created with OCTAX_KERNEL_PLAIN (they run
     * their own lane-per-env kernels; OCTAX_E_INVALID otherwise). */
    uint32_t platform;
    uint32_t reserved2;
} octax_config;

/* SUPER-CHIP part of one env's state (octax_get_schip_state). */
typedef struct octax_schip_state {
    uint32_t hires;           /* 1: 128x64 mode */
    uint8_t rpl[8];           /* flag registers of FX75 / FX85 */
    uint32_t reserved;
    uint64_t fb[64][2];       /* display row y: fb[y][0] holds x 0..63, fb[y][1] x 64..127, bit 63 - (x mod 64) */
    uint64_t hist[3][64][2];  /* the three frames before fb, oldest first, same packing */
} octax_schip_state;

/* Architectural state of one env (get_state / set_state). */
typedef struct octax_env_state {
    uint8_t v[16];          /* V0..VF */
    uint16_t i;             /* index register, 12-bit */
    uint16_t pc;            /* program counter, 12-bit */
    uint8_t sp;             /* stack pointer 0..15 */
    uint8_t dt;             /* delay timer */
    uint8_t st;             /* sound timer */
    uint8_t prev_key;       /* key held in the previous step (sticky actions), 16 = none */
    uint16_t stack[16];     /* return addresses */
    uint32_t t;             /* steps since the last reset */
    int32_t prev_score;     /* score (see h_score_mode) after the previous step */
    uint64_t rng;           /* SplitMix64 state */
    uint8_t ram[4096];      /* memory */
    uint64_t fb[32];        /* display row y: bit (63 - x) is pixel (x, y) */
    uint64_t hist[3][32];   /* the three frames before fb, oldest first, same packing */
} octax_env_state;

typedef struct octax_engine octax_engine;
typedef struct octax_graph octax_graph;

/*
 * Create an engine: validates cfg, allocates the state of E envs in device
 * memory (about 5.6 KB per env), copies the ROM images and descriptors and
 * resets every env (Section 3.2, ROM loading and initialization).  On
 * success *out owns the engine; on failure *out is NULL and nothing leaks.
 * Errors: OCTAX_E_INVALID (any field out of range, ROM too long, env_rom
 * >= R, wrong abi_version, quirks without OCTAX_QUIRKS_V1 or with unknown
 * flags), OCTAX_E_NOMEM, OCTAX_E_HIP.
 */
int32_t octax_create(const octax_config *cfg, octax_engine **out);

/*
 * Digest of every env's state: d_out[env] = 64-bit FNV-1a (Fowler-Noll-Vo;
 * offset basis 0xcbf29ce484222325, prime 0x100000001b3, XOR then multiply
 * per byte) over the env's octax_env_state, i.e. over exactly the bytes
 * octax_get_state would return for it, in their order (for SUPER-CHIP
 * engines: the CHIP-8 part of the state).  A cheap whole-batch parity and
 * determinism check: equal digests for equal states, computed on the device
 * without copying the state out.  Asynchronous on the engine's stream.
 * d_out: device uint64 [E].  Errors: OCTAX_E_INVALID (NULL engine or
 * output), OCTAX_E_HIP.
 */
int32_t octax_digest(octax_engine *g, uint64_t *d_out);

/*
 * SUPER-CHIP state of envs [first, first + count) into h_out[0..count): mode,
 * flag registers, 128x64 display and the three previous frames (the
 * registers, memory and timers come from octax_get_state).  Synchronizes.
 * There is no setter for this part: octax_set_state writes the CHIP-8
 * registers, memory and timers of a SUPER-CHIP env and leaves its display,
 * mode and flag registers as they are.
 * Errors: OCTAX_E_INVALID (NULL engine or output, range outside 0..E, or a
 * CHIP-8 engine), OCTAX_E_HIP.
 */
int32_t octax_get_schip_state(octax_engine *g, uint32_t first, uint32_t count, octax_schip_state *h_out);

/*
 * Reset the envs whose d_mask byte is non-zero (all envs when d_mask is
 * NULL) to the power-on state of their ROM (Section 3.2, ROM loading and
 * initialization): memory = font + program, registers, I, stack and timers
 * zero, PC = 0x200, display and frame stack blank, step count zero; then
 * the reset steps of the wrappers, if any (see octax_config).  Each env's
 * RNG stream continues.  If d_obs is not NULL the observation of every
 * env (reset or not) is written to d_obs [E][4][64][32] ([E][4][128][64]
 * for SUPER-CHIP).
 * d_mask: device uint8 [E] or NULL.  Errors: OCTAX_E_INVALID (NULL engine),
 * OCTAX_E_HIP.
 */
int32_t octax_reset(octax_engine *eng, const uint8_t *d_mask, uint8_t *d_obs);

/*
 * One environment step of every env (Section 3.2, Environment integration;
 * Section 3.3 reward and termination; Section 3.4 automatic reset).
 * d_action: device int32 [E]; out-of-range values are the no-op.
 * d_obs: device uint8 [E][4][64][32], [E][4][128][64] for SUPER-CHIP (may be
 * NULL: not written).
 * d_reward: device float [E]; d_done: device uint8 [E], bit 0 terminated,
 * bit 1 truncated.  Errors: OCTAX_E_INVALID (NULL engine/action/reward/done),
 * OCTAX_E_HIP.
 */
int32_t octax_step(octax_engine *eng, const int32_t *d_action, uint8_t *d_obs,
                   float *d_reward, uint8_t *d_done);

/*
 * K consecutive environment steps (the same semantics as K octax_step
 * calls): one launch for the fused kernel, one per step for the plain
 * kernel, K + 1 for SUPER-CHIP with observations (K without).
 * d_action: device int32 [K][E]; d_reward: float [K][E]; d_done: uint8
 * [K][E]; d_obs: uint8 [obs_slots][E][4][64][32] (per-env shape
 * [4][128][64] for SUPER-CHIP) where step k writes slot k % obs_slots
 * (obs_slots = K keeps the whole rollout, obs_slots = 1 keeps the last),
 * or NULL.
 * Errors: OCTAX_E_INVALID (K == 0, obs_slots == 0 with d_obs, NULL
 * arguments), OCTAX_E_HIP.
 */
int32_t octax_step_many(octax_engine *eng, uint32_t K, const int32_t *d_action,
                        uint8_t *d_obs, uint32_t obs_slots, float *d_reward, uint8_t *d_done);

/*
 * Capture octax_step_many(eng, K, d_action, d_obs, obs_slots, d_reward,
 * d_done) into a HIP graph with these fixed buffers.  Each
 * octax_graph_launch replays it on the engine's stream: the caller rewrites
 * d_action between replays and reads the outputs after them.  The graph
 * holds the engine; destroy graphs before their engine.
 * Errors: as octax_step_many, plus OCTAX_E_HIP if capture fails.
 */
int32_t octax_graph_create(octax_engine *eng, uint32_t K, const int32_t *d_action,
                           uint8_t *d_obs, uint32_t obs_slots, float *d_reward,
                           uint8_t *d_done, octax_graph **out);
int32_t octax_graph_launch(octax_graph *g);
int32_t octax_graph_destroy(octax_graph *g);

/*
 * Copy the architectural state of envs [first, first+count) to h_out
 * (count entries).  Synchronizes the engine's stream first.
 * Errors: OCTAX_E_INVALID (range outside 0..E, NULL), OCTAX_E_HIP.
 */
int32_t octax_get_state(octax_engine *eng, uint32_t first, uint32_t count,
                        octax_env_state *h_out);

/*
 * octax_get_state for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it).
 * Same result as octax_get_state for the same range, but the slot list and
 * the gathered records go through a static device array of the library
 * (256 B + OCTAX_NOALLOC_MAX_ENVS records of 5,456 B, about 350 KB), held on
 * every GPU the library runs on until the process ends; the call allocates
 * no device memory.  At most OCTAX_NOALLOC_MAX_ENVS envs per call: take a
 * larger range in pieces.  Every call on one GPU shares that GPU's array, so
 * calls that overlap in time on one GPU (from several host threads) race
 * and must be serialized by the caller.  Synchronizes the engine's stream.
 * Errors: OCTAX_E_INVALID (range outside 0..E, count above the maximum,
 * NULL), OCTAX_E_HIP.
 */
#define OCTAX_NOALLOC_MAX_ENVS 64u
int32_t octax_get_state_noalloc(octax_engine *eng, uint32_t first, uint32_t count,
                                octax_env_state *h_out);

/*
 * Overwrite the state of envs [first, first+count) from h_in (I, PC, stack
 * entries masked to 12 bits, SP to 4 bits, display bits as given).  The
 * next step continues from it exactly as from the state it was saved from.
 * Errors: OCTAX_E_INVALID, OCTAX_E_HIP.
 */
int32_t octax_set_state(octax_engine *eng, uint32_t first, uint32_t count,
                        const octax_env_state *h_in);

/*
 * Select the step kernel (enum octax_kernel) for subsequent calls; the
 * state layout is the same for both, so results do not change.
 * Errors: OCTAX_E_INVALID.
 */
int32_t octax_set_kernel(octax_engine *eng, uint32_t kernel);

/*
 * Fused-kernel tuning for subsequent calls: envs_per_block in {64, 128, 256},
 * rom_in_lds 0/1 (stage the block's two most frequent ROM images in LDS).
 * Results do not change.  Errors: OCTAX_E_INVALID.
 */
int32_t octax_set_tuning(octax_engine *eng, uint32_t envs_per_block, uint32_t rom_in_lds);

/*
 * Bind the engine to another stream (hipStream_t, NULL = null stream).
 */
int32_t octax_set_stream(octax_engine *eng, void *stream);

/* Number of envs, and device bytes held by the engine. */
int32_t octax_info(const octax_engine *eng, uint32_t *num_envs, uint64_t *device_bytes);

/*
 * Destroy an engine (synchronizes its stream, frees its device memory).
 * NULL is accepted.  Errors: OCTAX_E_HIP; OCTAX_E_STATE as octax_status
 * (the engine is destroyed all the same).
 */
int32_t octax_destroy(octax_engine *eng);

/*
 * Completion check of the asynchronous calls.  In a fused launch each
 * emulator wave and its observation-writer wave wait for each other once per
 * step; every such wait is bounded (0.25 s plus 16 us per instruction slot of
 * the longest step the config allows, on the device wall clock), so every
 * launch ends.  A wait that gives up sets the engine's device error word:
 * that launch's observations, rewards and done flags are not valid, and nor
 * need the envs' state be (a writer wave that ran ahead may have staged the
 * wrong keys and frame history): restore it with octax_set_state or
 * octax_reset before going on.  octax_status
 * synchronizes the engine's stream and returns OCTAX_E_STATE once if the
 * word is set since the last check, clearing it; octax_get_state,
 * octax_get_state_noalloc, octax_destroy and the pool's get_state and
 * destroy report it the same way (get_state after filling h_out).  The
 * fused kernel therefore takes configs with at most 1,048,576 instruction
 * slots per step (instr_per_frame x frame_skip x (1 + longest start-up
 * sequence + noop_max)); octax_create and octax_set_kernel reject longer
 * ones for it (the plain kernel has no such wait and takes them).
 * Errors: OCTAX_E_INVALID (NULL), OCTAX_E_STATE, OCTAX_E_HIP.
 */
int32_t octax_status(octax_engine *eng);

/*
 * Replace the derived wait bound of the fused kernel by `ticks` of the
 * device wall clock (0 restores the derived bound).  A diagnostic hook: a
 * tiny bound makes the waits give up, so the error path can be exercised
 * without a long step.  Errors: OCTAX_E_INVALID (NULL), OCTAX_E_STATE
 * (graphs of the engine exist: they hold the old bound).
 */
int32_t octax_set_wait_limit(octax_engine *eng, uint64_t ticks);

/*
 * Step clock of the fused kernel (measurement of the per-step latency inside
 * a multi-step launch).  With d_stamps set, every fused launch records for
 * each step k < steps and each wave pair w (w = 0 .. ceil(E / 64) - 1, the
 * 64 consecutive slots of emulator wave w) two readings of the device wall
 * clock: d_stamps[(k * ceil(E / 64) + w) * 2] when the emulator wave starts
 * step k, and [... + 1] when the paired observation-writer wave has issued
 * the last observation store of step k.  The latency of step k is then the
 * largest end minus the smallest start over all pairs.  Pairs with no live
 * env write nothing.  d_stamps is caller-owned device memory of
 * steps * ceil(E / 64) * 2 uint64 that stays valid while launches run; NULL
 * (or steps = 0) switches the clock off.  *h_clock_hz (if not NULL) receives
 * the clock's rate.  Graphs keep the setting they were captured with.
 * Errors: OCTAX_E_INVALID (NULL engine, or d_stamps NULL with steps > 0),
 * OCTAX_E_STATE (graphs of the engine exist), OCTAX_E_HIP.
 */
int32_t octax_set_step_clock(octax_engine *eng, uint64_t *d_stamps, uint32_t steps, uint64_t *h_clock_hz);

/*
 * Serving pool: continuous batching of environment groups (requests) that
 * arrive and finish at different times, all stepped by one fused launch per
 * tick while their state stays resident in device memory.
 *
 * A pool holds `capacity` env slots, fixed at creation from a device-memory
 * budget (pool_bytes / octax_pool_slot_bytes()).  octax_pool_admit places a
 * group of `count` envs of one ROM in the `count` lowest-numbered free slots,
 * contiguous or not, and resets them to the power-on state of that ROM
 * (Section 3.2, ROM loading and initialization); with fewer free slots it
 * returns OCTAX_E_NOMEM and changes nothing, so the caller keeps the request
 * queued (admission is by memory only: free slots never fragment).
 * octax_pool_step runs K environment steps (the semantics of
 * octax_step_many) of every occupied slot; free slots are neither read nor
 * written.  octax_pool_retire frees a group's slots.  A group's results do
 * not depend on its slots or on the other groups in the pool: each env's
 * RNG stream starts from the seed given at admission.
 *
 * Buffers of octax_pool_step are indexed by slot: d_action int32 [K][capacity],
 * d_obs uint8 [obs_slots][capacity][4][64][32] (or NULL), d_reward float
 * [K][capacity], d_done uint8 [K][capacity]; only occupied slots are used.
 * Admission, retirement and steps are ordered on the pool's stream; admit
 * and retire return without waiting for the device.  Host arrays passed to
 * admit are copied before it returns.
 */
typedef struct octax_pool_config {
    uint32_t abi_version;      /* must be OCTAX_ABI_VERSION */
    uint32_t num_roms;         /* R >= 1 */
    uint32_t instr_per_frame;  /* 1..1000 */
    uint32_t frame_skip;       /* 1..64 */
    uint32_t quirks;           /* OCTAX_QUIRKS_V1 | any OCTAX_QUIRK_* flags */
    uint32_t envs_per_block;   /* fused kernel tuning: 64, 128 or 256 (0 = 256) */
    uint64_t pool_bytes;       /* device-memory budget of the env slots */
    const uint8_t *h_rom_data;     /* as in octax_config */
    const uint32_t *h_rom_offset;  /* [R] */
    const uint32_t *h_rom_len;     /* [R] */
    const uint8_t *h_action_keys;  /* [R][16] */
    const uint8_t *h_num_actions;  /* [R] */
    const uint8_t *h_score_reg;    /* [R] */
    const uint8_t *h_term_reg;     /* [R] */
    const uint8_t *h_term_value;   /* [R] */
    void *stream;                  /* hipStream_t; NULL = null stream */
    uint32_t sticky_q24;           /* environment wrappers, as in octax_config */
    uint32_t noop_max;
    const uint8_t *h_startup_len;  /* [R] or NULL */
    const uint8_t *h_startup_keys; /* [R][16] or NULL */
    const uint8_t *h_score_mode;   /* game descriptors, as in octax_config */
    const uint8_t *h_score_arg;
    const uint8_t *h_term_op;
    const uint8_t *h_term2_op;
    const uint8_t *h_term2_reg;
    const uint8_t *h_term2_value;
} octax_pool_config;

typedef struct octax_pool octax_pool;

/* Device bytes of one env slot of a pool. */
uint64_t octax_pool_slot_bytes(void);

/*
 * Create a pool (allocates capacity slots and the ROM images, synchronizes).
 * Errors: OCTAX_E_INVALID (bad field, budget below one slot), OCTAX_E_NOMEM,
 * OCTAX_E_HIP.
 */
int32_t octax_pool_create(const octax_pool_config *cfg, octax_pool **out);

/*
 * Admit a group: count envs of ROM `rom`, env k with RNG seed h_env_seed[k]
 * and truncation horizon h_horizon[k] (0 = none).  On success h_slots[k]
 * (caller-owned, count entries) is env k's slot, in ascending order, and
 * *group the group's id for octax_pool_retire.  Errors: OCTAX_E_INVALID
 * (rom >= R, count == 0 or > capacity, NULL), OCTAX_E_NOMEM (fewer than
 * count free slots: nothing changed), OCTAX_E_HIP.
 */
int32_t octax_pool_admit(octax_pool *p, uint32_t rom, uint32_t count, const uint64_t *h_env_seed,
                         const uint32_t *h_horizon, uint32_t *h_slots, uint32_t *group);

/*
 * Free the slots of a group.  Steps already enqueued still see it.
 * Errors: OCTAX_E_INVALID (no such group).
 */
int32_t octax_pool_retire(octax_pool *p, uint32_t group);

/* K environment steps of every occupied slot (buffers as described above).
 * Errors: OCTAX_E_INVALID (K == 0, NULL action/reward/done, obs_slots == 0
 * with d_obs), OCTAX_E_HIP. */
int32_t octax_pool_step(octax_pool *p, uint32_t K, const int32_t *d_action, uint8_t *d_obs,
                        uint32_t obs_slots, float *d_reward, uint8_t *d_done);

/* As octax_pool_step, with a step budget per slot: d_budget uint8 [capacity]
 * (device), slot s runs min(K, d_budget[s]) steps of this call and stops
 * there, its state, frame history and RNG stream exactly those after that
 * many steps, so that a group whose last step falls inside a call of K steps
 * ends on it.  Outputs of a slot for steps at or past its budget are
 * unspecified.  NULL d_budget: every slot runs K steps.  The
 * budget array is read when the launch runs (stream order).
 * Errors: those of octax_pool_step, and OCTAX_E_INVALID for K > 255 with a
 * budget array. */
int32_t octax_pool_step_budget(octax_pool *p, uint32_t K, const uint8_t *d_budget, const int32_t *d_action,
                               uint8_t *d_obs, uint32_t obs_slots, float *d_reward, uint8_t *d_done);

/* Capacity, free slots, the largest group admissible now (equal to the free
 * slots: any free slots take a group) and number of groups. */
int32_t octax_pool_info(const octax_pool *p, uint32_t *capacity, uint32_t *free_slots,
                        uint32_t *largest_free, uint32_t *groups);

/* Architectural state of the envs in slots h_slots[0..count) into
 * h_out[0..count) (synchronizes).  The observation history is that of the
 * env in the slot.  Errors as octax_get_state. */
int32_t octax_pool_get_state(octax_pool *p, const uint32_t *h_slots, uint32_t count, octax_env_state *h_out);

/* Destroy a pool (synchronizes its stream).  NULL is accepted. */
int32_t octax_pool_destroy(octax_pool *p);

/*
 * Roofline calibration (no part of the environment step): stream `bytes`
 * (a multiple of 16) of the 32-bit value v into d_dst (nontemporal != 0: with
 * the nontemporal store hint), or copy `bytes` from d_src to d_dst,
 * asynchronously on `stream` (hipStream_t, NULL = null stream).  The measured rate of these kernels on the same device is the
 * attainable HBM bandwidth the step kernels are compared with, and the copy
 * kernel's hardware counters calibrate byte counters.  Returns 0, -1 for a
 * bad argument, -3 if the launch failed.
 */
int32_t octax_calib_write(void *d_dst, uint64_t bytes, uint32_t v, uint32_t nontemporal, void *stream);
int32_t octax_calib_copy(const void *d_src, void *d_dst, uint64_t bytes, void *stream);

/* Message describing the last failure on this thread ("" if none). */
const char *octax_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OCTAX_H */
