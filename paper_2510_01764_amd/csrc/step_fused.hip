// Fused step kernel: K environment steps per launch for a block of envs that
// stays resident for the whole launch.
//
//   * registers, PC, I, timers and the RNG state of each env live in VGPRs for
//     all K steps (one env per lane);
//   * the display (32 rows of 64 bits), the call stack and the power-on
//     images of up to two ROMs are staged in LDS; code fetches and sprite
//     reads of memory pages not written since the reset are served from the
//     staged image, written pages from the env's memory in HBM;
//   * each step ends with a per-lane 32x64 bit transpose of the display into
//     64 column words (the observation is x-major), staged in LDS, and a
//     wave-cooperative pass that expands the four frames of each env into
//     bytes with fully coalesced 1 KB stores per instruction;
//   * the state goes back to HBM once per launch.
#include "octax_core.h"
#include "octax_kernels.h"

namespace octax {
namespace {

constexpr uint32_t kNoRom = 0xFFFFFFFFu;
constexpr int kFbStride = 33;      // u64 per env row block: odd stride spreads lanes over banks
constexpr int kStageStride = 68;   // u32 per env column block (64 + 4 pad, 16-byte aligned)

template <int IPW>
struct Shared {
    uint64_t fb[IPW][kFbStride];
    uint32_t stage[IPW][kStageStride];
    uint32_t stack[IPW][9];
    uint8_t img[2][kMem];
};

template <int IPW>
struct FusedMem {
    Shared<IPW> &sh;
    uint32_t lane;
    int32_t lidx;          // staged image index or -1
    const uint8_t *gimg;   // power-on image in HBM
    uint8_t *ram;          // env memory in HBM
    uint64_t dirty;

    __device__ __forceinline__ uint32_t read(uint32_t a) const {
        if ((dirty >> (a >> 6)) & 1) return ram[a];
        if (lidx >= 0) return sh.img[lidx][a];
        return gimg[a];
    }
    __device__ __forceinline__ void write(uint32_t a, uint32_t v) {
        ram[a] = (uint8_t)v;
        dirty |= 1ull << (a >> 6);
    }
    __device__ __forceinline__ uint32_t draw(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n) {
        uint64_t hit = 0;
        for (uint32_t r = 0; r < n; r++) {
            const uint32_t yy = y0 + r;
            if (yy >= 32) break;
            const uint64_t m = ((uint64_t)read((I + r) & 0xFFF) << 56) >> x0;
            const uint64_t row = sh.fb[lane][yy];
            hit |= row & m;
            sh.fb[lane][yy] = row ^ m;
        }
        return hit != 0;
    }
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int y = 0; y < 32; y++) sh.fb[lane][y] = 0;
    }
    __device__ __forceinline__ uint32_t stack_get(uint32_t i) const {
        const uint32_t w = sh.stack[lane][i >> 1];
        return (i & 1) ? (w >> 16) : (w & 0xFFFF);
    }
    __device__ __forceinline__ void stack_set(uint32_t i, uint32_t v) {
        const uint32_t w = sh.stack[lane][i >> 1];
        sh.stack[lane][i >> 1] = (i & 1) ? ((w & 0xFFFFu) | (v << 16)) : ((w & 0xFFFF0000u) | v);
    }
};

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16 column bits -> 16 bytes at dst.
__device__ __forceinline__ void store16(uint8_t *dst, uint32_t bits) {
    store_stream(dst, spread4(bits, 0), spread4(bits, 4), spread4(bits, 8), spread4(bits, 12));
}

template <int IPW>
__global__ __launch_bounds__(IPW) void step_fused_kernel(State s, Roms roms, StepIO io, FusedCfg cfg) {
    __shared__ Shared<IPW> sh;
    const uint32_t l = threadIdx.x;
    const uint32_t lane64 = l & 63;
    const uint32_t wave_base = l & ~63u;
    const uint32_t slot = blockIdx.x * IPW + l;
    const uint32_t E = s.num;
    const bool active = slot < E;

    // Stage the block's ROM images.
    uint32_t brom0 = kNoRom, brom1 = kNoRom;
    if (cfg.rom_in_lds) {
        brom0 = cfg.block_roms[blockIdx.x * 2 + 0];
        brom1 = cfg.block_roms[blockIdx.x * 2 + 1];
        for (uint32_t q = l; q < 2 * kMem / 16; q += IPW) {
            const uint32_t which = q / (kMem / 16);
            const uint32_t rid = which ? brom1 : brom0;
            if (rid != kNoRom) {
                reinterpret_cast<uint4 *>(sh.img[which])[q % (kMem / 16)] =
                    reinterpret_cast<const uint4 *>(roms.image + (size_t)rid * kMem)[q % (kMem / 16)];
            }
        }
    }

    Core c;
    uint32_t head = 0, env = 0, rom = 0, desc = 0, t = 0, hor = 0;
    int32_t prev = 0;
    uint64_t dirty = 0;
    if (active) {
        load_core(s, slot, c, head);
        env = s.env_of[slot];
        rom = s.rom_of[slot];
        desc = roms.desc[rom];
        t = s.t[slot];
        hor = s.horizon[slot];
        prev = s.prev[slot];
        dirty = s.dirty[slot];
        const uint4 *fb4 = reinterpret_cast<const uint4 *>(s.fb + (size_t)slot * 32);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const uint4 v = fb4[q];
            sh.fb[l][2 * q] = (uint64_t)v.x | ((uint64_t)v.y << 32);
            sh.fb[l][2 * q + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
        }
        const uint4 *st4 = reinterpret_cast<const uint4 *>(s.stack + (size_t)slot * 8);
        const uint4 a0 = st4[0], a1 = st4[1];
        sh.stack[l][0] = a0.x; sh.stack[l][1] = a0.y; sh.stack[l][2] = a0.z; sh.stack[l][3] = a0.w;
        sh.stack[l][4] = a1.x; sh.stack[l][5] = a1.y; sh.stack[l][6] = a1.z; sh.stack[l][7] = a1.w;
    } else {
        reset_core(c);
        c.rng = 0;
    }
    const int32_t lidx = (rom == brom0) ? 0 : (rom == brom1) ? 1 : -1;
    const uint8_t *gimg = roms.image + (size_t)rom * kMem;
    uint8_t *ram = s.ram + (size_t)slot * kMem;
    __syncthreads();

    for (uint32_t k = 0; k < io.K; k++) {
        uint32_t done = 0;
        if (active) {
            const uint32_t key = action_key(roms, rom, desc, io.action[(size_t)k * E + env]);
            FusedMem<IPW> mem{sh, l, lidx, gimg, ram, dirty};
            for (uint32_t f = 0; f < io.frame_skip; f++) {
                for (uint32_t i = 0; i < io.ipf; i++) exec_one(c, mem, key);
                tick(c);
            }
            const int32_t score = (int32_t)vget(c.r, desc & 15);
            const float reward = (float)(score - prev);
            const uint32_t term = vget(c.r, (desc >> 8) & 15) == ((desc >> 16) & 0xFF);
            t += 1;
            const uint32_t trunc = (hor != 0) && (t >= hor);
            done = term | (trunc << 1);
            io.reward[(size_t)k * E + env] = reward;
            io.done[(size_t)k * E + env] = (uint8_t)done;
            if (done) {
                // Automatic reset (Section 3.4); the RNG stream continues.
                uint64_t d = mem.dirty;
                while (d) {
                    const uint32_t p = __builtin_ctzll(d);
                    d &= d - 1;
                    const uint4 *src = reinterpret_cast<const uint4 *>(gimg + p * 64);
                    uint4 *dst = reinterpret_cast<uint4 *>(ram + p * 64);
                    for (int q = 0; q < 4; q++) dst[q] = src[q];
                }
                mem.dirty = 0;
                reset_core(c);
                mem.clear();
                for (int q = 0; q < 8; q++) sh.stack[l][q] = 0;
                head = 0;
                t = 0;
                prev = 0;
            } else {
                prev = score;
                head = (head + 1) & 3;
            }
            dirty = mem.dirty;
            // display rows -> 64 column words, staged for the cooperative pass
            uint32_t hi[32], lo[32];
#pragma unroll
            for (int r = 0; r < 32; r++) {
                const uint64_t row = sh.fb[l][31 - r];
                hi[r] = (uint32_t)(row >> 32);
                lo[r] = (uint32_t)row;
            }
            rows_to_cols(hi, lo);
            uint4 *stg = reinterpret_cast<uint4 *>(sh.stage[l]);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                stg[q] = make_uint4(hi[4 * q], hi[4 * q + 1], hi[4 * q + 2], hi[4 * q + 3]);
                stg[8 + q] = make_uint4(lo[4 * q], lo[4 * q + 1], lo[4 * q + 2], lo[4 * q + 3]);
            }
        }
        wave_sync();

        // Cooperative pass over the wave's envs: frame ring update and the
        // observation, one env at a time.  Lane x owns column x of every
        // frame: it is the only lane that writes or reads ring word x, so
        // ring traffic is ordered by program order alone, and it stores the
        // 32 bytes of column x of each frame (a wave covers 2 KB per frame).
        const uint32_t nj = (E > blockIdx.x * IPW + wave_base)
                                ? min(64u, E - (blockIdx.x * IPW + wave_base)) : 0u;
        uint8_t *obs_k = io.obs ? io.obs + (size_t)(k % io.obs_slots) * E * kObsBytes : nullptr;
        for (uint32_t j = 0; j < nj; j++) {
            const uint32_t jl = wave_base + j;
            const uint32_t jslot = blockIdx.x * IPW + jl;
            const uint32_t jhead = __builtin_amdgcn_readlane(head, j);
            const uint32_t jdone = __builtin_amdgcn_readlane(done, j);
            uint32_t *ring = s.cols + (size_t)jslot * 256 + lane64;
            const uint32_t c3 = sh.stage[jl][lane64];
            uint32_t c0 = 0, c1 = 0, c2 = 0;
            if (jdone) {
                ring[64] = 0;
                ring[128] = 0;
                ring[192] = 0;
            } else if (obs_k) {
                c0 = ring[((jhead + 1) & 3) * 64];
                c1 = ring[((jhead + 2) & 3) * 64];
                c2 = ring[((jhead + 3) & 3) * 64];
            }
            ring[jhead * 64] = c3;
            if (obs_k) {
                const uint32_t jenv = __builtin_amdgcn_readlane(env, j);
                uint8_t *o = obs_k + (size_t)jenv * kObsBytes + 32 * lane64;
                store16(o, c0);
                store16(o + 16, c0 >> 16);
                store16(o + 2048, c1);
                store16(o + 2048 + 16, c1 >> 16);
                store16(o + 4096, c2);
                store16(o + 4096 + 16, c2 >> 16);
                store16(o + 6144, c3);
                store16(o + 6144 + 16, c3 >> 16);
            }
        }
        wave_sync();
    }

    if (active) {
        store_core(s, slot, c, head);
        s.t[slot] = t;
        s.prev[slot] = prev;
        s.dirty[slot] = dirty;
        uint4 *fb4 = reinterpret_cast<uint4 *>(s.fb + (size_t)slot * 32);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const uint64_t a = sh.fb[l][2 * q], b = sh.fb[l][2 * q + 1];
            fb4[q] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
        }
        uint4 *st4 = reinterpret_cast<uint4 *>(s.stack + (size_t)slot * 8);
        st4[0] = make_uint4(sh.stack[l][0], sh.stack[l][1], sh.stack[l][2], sh.stack[l][3]);
        st4[1] = make_uint4(sh.stack[l][4], sh.stack[l][5], sh.stack[l][6], sh.stack[l][7]);
    }
}

template <int IPW>
hipError_t launch_ipw(const State &s, const Roms &r, const StepIO &io, const FusedCfg &f, hipStream_t st) {
    const uint32_t blocks = (s.num + IPW - 1) / IPW;
    hipLaunchKernelGGL(step_fused_kernel<IPW>, dim3(blocks), dim3(IPW), 0, st, s, r, io, f);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_fused(const State &s, const Roms &r, const StepIO &io, const FusedCfg &f,
                             hipStream_t st) {
    switch (f.envs_per_block) {
    case 64: return launch_ipw<64>(s, r, io, f, st);
    case 128: return launch_ipw<128>(s, r, io, f, st);
    case 256: return launch_ipw<256>(s, r, io, f, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace octax
