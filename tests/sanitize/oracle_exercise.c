/*
 * Drives the CPU oracle (oracle/chip8_oracle.c) through every entry point on
 * inputs that reach its edge cases, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize_cpu.py compiles and runs
 * it; any report aborts the process).  It checks no result: the pins and the
 * parity tests do that.  Inputs: random bytes as programs (every opcode,
 * invalid words included), ROM sizes from 0 to the full 3,584 bytes, actions
 * in and out of range, every quirk flag, game descriptors of every mode and
 * clause op, the environment wrappers, the SUPER-CHIP platform, masked
 * resets, state round trips, the execution profile and the threaded runner.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_batch oracle_batch;
oracle_batch *oracle_create(int num_envs, int num_roms, const uint8_t *rom_data, const uint32_t *rom_offset,
                            const uint32_t *rom_len, const uint16_t *env_rom, const uint8_t *action_keys,
                            const uint8_t *num_actions, const uint8_t *score_reg, const uint8_t *term_reg,
                            const uint8_t *term_value, const uint32_t *horizon, const uint64_t *env_seed,
                            int instr_per_frame, int frame_skip);
void oracle_destroy(oracle_batch *b);
int oracle_set_profile(oracle_batch *b, uint32_t quirks, const uint8_t *score_mode, const uint8_t *score_arg,
                       const uint8_t *term_op, const uint8_t *term2_op, const uint8_t *term2_reg,
                       const uint8_t *term2_value);
int oracle_set_wrappers(oracle_batch *b, uint32_t sticky_q24, uint32_t noop_max, const uint8_t *startup_len,
                        const uint8_t *startup_keys);
int oracle_set_platform(oracle_batch *b, int schip);
int oracle_set_exec_profile(oracle_batch *b, uint32_t *pc_hist, uint32_t *op_hist);
void oracle_reset(oracle_batch *b, const uint8_t *mask, uint8_t *obs);
void oracle_step(oracle_batch *b, const int32_t *action, uint8_t *obs, float *reward, uint8_t *done);
int oracle_run_threaded(oracle_batch *b, int steps, const int32_t *action, uint8_t *obs, float *reward,
                        uint8_t *done, int threads);
int oracle_state_size(void);
void oracle_get_state(const oracle_batch *b, int first, int count, void *out);
void oracle_set_state(oracle_batch *b, int first, int count, const void *in);

/* xorshift64* for the inputs (not the method's random numbers) */
static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return (uint32_t)((rs * 0x2545F4914F6CDD1Dull) >> 32);
}

#define NUM_ENVS 48
#define NUM_ROMS 8
#define FULL_ROM 3584

static void run_case(int quirk_case, int wrappers, int schip, int steps)
{
    static uint8_t data[NUM_ROMS * FULL_ROM];
    uint32_t off[NUM_ROMS], len[NUM_ROMS];
    uint8_t keys[NUM_ROMS * 16], nact[NUM_ROMS], sreg[NUM_ROMS], treg[NUM_ROMS], tval[NUM_ROMS];
    uint16_t env_rom[NUM_ENVS];
    uint32_t horizon[NUM_ENVS];
    uint64_t seed[NUM_ENVS];
    const uint32_t sizes[NUM_ROMS] = {0, 1, 2, 3, FULL_ROM - 1, FULL_ROM, 700, 1500};
    uint32_t pos = 0;
    for (int r = 0; r < NUM_ROMS; r++) {
        off[r] = pos;
        len[r] = sizes[r];
        for (uint32_t i = 0; i < len[r]; i++)
            data[pos + i] = (uint8_t)rnd();
        /* some programs start with a few valid words so that draws, calls and stores happen early */
        if (len[r] >= 16) {
            const uint16_t head[8] = {0xA050, 0xD015, 0x2208, 0x6F33, 0xF033, 0xF255, 0xF165, 0x00EE};
            for (int w = 0; w < 8; w++) {
                data[pos + 2 * w] = (uint8_t)(head[w] >> 8);
                data[pos + 2 * w + 1] = (uint8_t)head[w];
            }
        }
        pos += len[r];
        for (int k = 0; k < 16; k++)
            keys[16 * r + k] = (uint8_t)(rnd() & 15);
        nact[r] = (uint8_t)(1 + rnd() % 16);
        sreg[r] = (uint8_t)(rnd() & 15);
        treg[r] = (uint8_t)(rnd() & 15);
        tval[r] = (uint8_t)rnd();
    }
    for (int e = 0; e < NUM_ENVS; e++) {
        env_rom[e] = (uint16_t)(e % NUM_ROMS);
        horizon[e] = (e % 3 == 0) ? 0u : 1u + rnd() % 40u;
        seed[e] = ((uint64_t)rnd() << 32) | rnd();
    }
    oracle_batch *b = oracle_create(NUM_ENVS, NUM_ROMS, data, off, len, env_rom, keys, nact, sreg, treg, tval,
                                    horizon, seed, 7 + quirk_case, 4);
    if (!b) {
        fprintf(stderr, "oracle_create failed\n");
        exit(2);
    }
    if (quirk_case) {
        uint8_t smode[NUM_ROMS], sarg[NUM_ROMS], top[NUM_ROMS], t2op[NUM_ROMS], t2reg[NUM_ROMS], t2val[NUM_ROMS];
        for (int r = 0; r < NUM_ROMS; r++) {
            smode[r] = (uint8_t)(r % 4);
            sarg[r] = (uint8_t)(smode[r] == 2 ? rnd() % 16 : rnd() & 0xFF);
            top[r] = (uint8_t)(r % 5);
            t2op[r] = (uint8_t)((r + 2) % 5);
            t2reg[r] = (uint8_t)(rnd() & 15);
            t2val[r] = (uint8_t)rnd();
        }
        const uint32_t quirks = quirk_case == 1 ? 0x3Fu : 0x7Fu;
        if (oracle_set_profile(b, quirks, smode, sarg, top, t2op, t2reg, t2val) != 0) {
            fprintf(stderr, "oracle_set_profile failed\n");
            exit(2);
        }
    }
    if (wrappers) {
        uint8_t slen[NUM_ROMS], skeys[NUM_ROMS * 16];
        for (int r = 0; r < NUM_ROMS; r++) {
            slen[r] = (uint8_t)(rnd() % 17);
            for (int k = 0; k < 16; k++)
                skeys[16 * r + k] = (uint8_t)(rnd() % 17);   /* 16: no key */
        }
        if (oracle_set_wrappers(b, 1u << 22, 5, slen, skeys) != 0) {
            fprintf(stderr, "oracle_set_wrappers failed\n");
            exit(2);
        }
    }
    if (schip && oracle_set_platform(b, 1) != 0) {
        fprintf(stderr, "oracle_set_platform failed\n");
        exit(2);
    }
    const size_t ob = schip ? 4 * 128 * 64 : 4 * 64 * 32;
    uint8_t *obs = malloc(NUM_ENVS * ob);
    float *rew = malloc(sizeof(float) * NUM_ENVS * (size_t)steps);
    uint8_t *done = malloc((size_t)NUM_ENVS * (size_t)steps);
    int32_t *act = malloc(sizeof(int32_t) * NUM_ENVS * (size_t)steps);
    uint32_t *pc_hist = calloc((size_t)NUM_ROMS * 4096, sizeof(uint32_t));
    uint32_t *op_hist = calloc((size_t)NUM_ROMS * 65536, sizeof(uint32_t));
    if (!obs || !rew || !done || !act || !pc_hist || !op_hist)
        exit(3);
    for (int i = 0; i < NUM_ENVS * steps; i++)
        act[i] = (int32_t)(rnd() % 20) - 2;   /* -2..17: out of range on both sides */
    oracle_reset(b, NULL, obs);
    if (oracle_set_exec_profile(b, pc_hist, op_hist) != 0)
        exit(2);
    for (int k = 0; k < steps / 2; k++)
        oracle_step(b, act + (size_t)k * NUM_ENVS, (k % 3 == 0) ? obs : NULL, rew, done);
    oracle_set_exec_profile(b, NULL, NULL);
    uint8_t mask[NUM_ENVS];
    for (int e = 0; e < NUM_ENVS; e++)
        mask[e] = (uint8_t)(rnd() & 1);
    oracle_reset(b, mask, obs);
    const int ss = oracle_state_size();
    uint8_t *st = malloc((size_t)ss * NUM_ENVS);
    if (!st)
        exit(3);
    oracle_get_state(b, 0, NUM_ENVS, st);
    oracle_set_state(b, 0, NUM_ENVS, st);
    oracle_get_state(b, NUM_ENVS / 2, NUM_ENVS / 2, st);
    oracle_set_state(b, 0, NUM_ENVS / 2, st);
    oracle_run_threaded(b, steps / 2, act, obs, rew, done, 3);
    free(st);
    free(obs);
    free(rew);
    free(done);
    free(act);
    free(pc_hist);
    free(op_hist);
    oracle_destroy(b);
}

int main(void)
{
    for (int schip = 0; schip < 2; schip++)
        for (int quirk_case = 0; quirk_case < 3; quirk_case++)
            for (int wrappers = 0; wrappers < 2; wrappers++)
                run_case(quirk_case, wrappers, schip, 60);
    printf("oracle exercised: %d cases\n", 12);
    return 0;
}
