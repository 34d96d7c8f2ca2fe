// Fused step kernel: K environment steps per launch for a block of envs that
// stays resident for the whole launch.
//
//   * registers, PC, I, timers and the RNG state of each env live in VGPRs for
//     all K steps (one env per lane of an emulator wave);
//   * the display (32 rows of 64 bits), the call stack and the power-on
//     images of up to two ROMs are staged in LDS; code fetches and sprite
//     reads of memory pages not written since the reset are served from the
//     staged image, written pages from two LDS cache slots per env or from
//     the env's memory in HBM;
//   * observations are written by a second set of waves of the same block:
//     after each step they copy the displays out of LDS, transpose each one
//     (32x64 bits) into a packed frame (64 words in observation store order)
//     and expand it into bytes with 1 KB contiguous stores per instruction,
//     while the emulator waves already run the next step;
//   * a frame is written, when it is computed, into the four observations it
//     belongs to (step k as frame 3, step k+1 as frame 2, ...), so the writer
//     waves issue no global loads between their observation stores: on CDNA
//     a load waits for every earlier store of the wave to complete;
//   * free slots of a serving pool are skipped, and blocks without an env
//     exit at once;
//   * the state goes back to HBM once per launch.
#include "octax_grouped.h"
#include "octax_kernels.h"

namespace octax {
namespace {

typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(1))) uint8_t glb_u8;
typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));

constexpr int kPrologueEnvs = 16;  // envs whose ring frames one prologue round loads

// LDS of one block (sizes in octax_kernels.h).  The display of lane l is
// fb[l][0..31], one padded 33-row stride per lane, so a lane's rows are
// contiguous (sprite rows are addressed with immediate offsets) and lanes
// reading the same row index spread over the banks.  The page pool and the
// cache slots are read up to 14 bytes before and one byte past a page (see
// FusedMem), so neither is first or last.  At every block size the block
// uses at most IPW / 256 of the CU's 160 KB, so 256 envs per CU stay
// resident.
template <int IPW>
struct Shared {
    static constexpr uint32_t kSlots = fused_cache_slots(IPW);
    static constexpr uint32_t kCacheStride = 64 * kSlots + 8;   // + 8 pad bytes: lanes spread over banks
    static constexpr uint32_t kPoolPages = fused_pool_pages(IPW);
    uint64_t fb[IPW][kFbStride];
    uint8_t pool[kPoolPages][64];
    uint8_t cache[IPW][kCacheStride];
    uint32_t stage[IPW / 64][kStageEnvs][kStageStride];
    float rew[IPW];           // reward and done bits of the step just emulated, for the writer waves
    uint8_t done[IPW];
    uint8_t budget[IPW];      // steps of the launch per env when the launch has step budgets
    uint8_t lready[IPW];      // per-lane progress (variants with reset steps): steps published, mod 256
    uint8_t ltaken[IPW];      // displays taken, mod 256
    uint32_t ready[IPW / 64]; // steps emulated by emulator wave w
    uint32_t taken[IPW / 64]; // displays taken by writer wave w
};
template <int IPW>
constexpr bool layout_ok() {
    return sizeof(Shared<IPW>) <= fused_lds_bytes(IPW) &&
           offsetof(Shared<IPW>, pool) >= 16 && offsetof(Shared<IPW>, cache) >= offsetof(Shared<IPW>, pool) + 16 &&
           offsetof(Shared<IPW>, stage) >= offsetof(Shared<IPW>, cache) + 16 &&
           sizeof(Shared<IPW>) >= offsetof(Shared<IPW>, stage) + 16 &&
           Shared<IPW>::kPoolPages > kPoolFixedPages;
}
static_assert(layout_ok<64>() && layout_ok<128>() && layout_ok<256>(),
              "LDS layout: within the block's share, page pool and cache slots neither first nor last");

// Memory of one env in the fused kernel.
//   * pages not written since the reset read from the power-on image: from
//     the block's page pool when it holds the page (always for the pages below
//     0x200 and past the ROM's last byte; for program pages, when the block
//     staged them), else through a cache slot filled from the image in HBM;
//   * written pages are kept in two to four LDS cache slots per env,
//     write-back: a write fills a slot (from the image for a clean page, from
//     the env's memory in HBM for a written one) and marks it modified; HBM
//     receives a modified page only when its slot is reused and when the
//     launch ends.  A read of an uncached written page fills a slot from HBM.
//     Slots are replaced in fill order, except that an access to the slot
//     due next moves the replacement pointer past it (a page in use is not
//     evicted next);
//   * multi-byte accesses (fetch, FX33/FX55/FX65, DXYN rows) touch at most
//     two pages; when both are readable from LDS all their LDS accesses are
//     issued back to back (one round trip per instruction, not one per byte).
// So the emulator waves touch HBM only on cache misses and resets: under the
// observation stores of the writer waves every global access of a wave waits
// behind them.
//   * the call stack is held in registers: 16 return addresses two to a
//     word, and the top entry stack[(SP - 1) & 15] apart, kept current on
//     every call and return, which is what the instruction cycle reads.
template <int IPW>
struct FusedMem {
    Shared<IPW> &sh;
    uint32_t lane;
    uint32_t pool_rom;       // pool byte offset of the env's program page 8 (0x200)
    uint32_t staged;         // program pages of the env's ROM held in the pool
    uint32_t rom_pages;      // program pages of the env's ROM (beyond: zero pages)
    const glb_u8 *gimg;      // power-on image in HBM
    glb_u8 *ram;             // env memory in HBM
    uint64_t dirty;
    uint32_t tags;           // slot i at bits 8i..8i+7: page | valid << 6 | modified << 7
    uint32_t stk[8];         // stack entry i in the 16-bit half i & 1 of stk[i >> 1]
    uint32_t top;            // stack[(SP - 1) & 15]
    uint32_t vic = 0;        // slot replaced next
    static constexpr uint32_t kSlots = Shared<IPW>::kSlots;
    static constexpr bool kOneAccess = true;   // access() serves DXYN, FX33, FX55 and FX65

    __device__ __forceinline__ lds_u8 *slot_ptr(uint32_t s) const {
        return (lds_u8 *)&sh.cache[lane][0] + 64 * s;
    }
    __device__ __forceinline__ bool is_dirty(uint32_t p) const { return (dirty >> p) & 1; }
    __device__ __forceinline__ uint32_t tag(uint32_t s) const { return (tags >> (8 * s)) & 0xFF; }
    // Slot holding page p, or -1.  All tag bytes are compared at once: byte s
    // of v is zero exactly when slot s holds p (valid bit included), and the
    // lowest zero byte is found with the borrow test of a SWAR zero-byte scan.
    __device__ __forceinline__ int32_t find(uint32_t p) const {
        const uint32_t v = (tags ^ __builtin_amdgcn_perm(0u, p | 0x40u, 0u)) & 0x7F7F7F7Fu;   // tag byte in all four bytes
        const uint32_t z = (v - 0x01010101u) & ~v & 0x80808080u;
        return z ? (int32_t)(__builtin_ctz(z | 0x80000000u) >> 3) : -1;
    }
    // Pick the slot for page p, never slot `keep` (-1: none); the slot's old
    // tag is returned in `old`.
    __device__ __forceinline__ static uint32_t next_slot(uint32_t s) { return s + 1 == kSlots ? 0u : s + 1; }
    // The slot to replace: in fill order from the replacement pointer, the
    // first slot without modified data (a clean page costs no write-back and
    // comes back cheaply), else the slot at the pointer; never `keep`.
    __device__ __forceinline__ uint32_t victim(int32_t keep, uint32_t &old) const {
        uint32_t s = vic;
        if ((int32_t)s == keep) s = next_slot(s);
        uint32_t pick = s;
        bool found = false;
#pragma unroll
        for (uint32_t i = 0; i < kSlots; i++) {
            const uint32_t c = (vic + i) % kSlots;
            const bool ok = !found && (int32_t)c != keep && !(tag(c) & 0x80);
            pick = ok ? c : pick;
            found = found || ok;
        }
        old = tag(pick);
        return pick;
    }
    // Slots are replaced in fill order: the next victim follows the slot filled.
    __device__ __forceinline__ void set_tag(uint32_t s, uint32_t t) {
        tags = (tags & ~(0xFFu << (8 * s))) | (t << (8 * s));
        vic = next_slot(s);
    }
    // An access to written page p: when p sits in the slot due for
    // replacement, the replacement pointer moves on to the next slot.
    __device__ __forceinline__ void touch(uint32_t p) {
        const bool at_vic = (int)is_dirty(p) & (int)((tag(vic) & 0x7F) == (p | 0x40));
        vic = at_vic ? next_slot(vic) : vic;
    }
    // Write a modified slot's page back to HBM (16 bytes a piece, from
    // registers read before the slot is overwritten).
    __device__ __forceinline__ void write_back(uint32_t old, uint4 v0, uint4 v1, uint4 v2, uint4 v3) {
        uint4 *dst = reinterpret_cast<uint4 *>((uint8_t *)ram + (old & 63) * 64);
        dst[0] = v0;
        dst[1] = v1;
        dst[2] = v2;
        dst[3] = v3;
    }
    __device__ __forceinline__ uint32_t fill_from_ram(uint32_t p, int32_t keep) {
        uint32_t old;
        const uint32_t s = victim(keep, old);
        uint4 *slot = reinterpret_cast<uint4 *>(&sh.cache[lane][64 * s]);
        const bool wb = old & 0x80;
        uint4 o0 = {}, o1 = {}, o2 = {}, o3 = {};
        if (wb) {
            o0 = slot[0];
            o1 = slot[1];
            o2 = slot[2];
            o3 = slot[3];
        }
        const uint4 *src = reinterpret_cast<const uint4 *>((const uint8_t *)ram + p * 64);
        const uint4 f0 = src[0], f1 = src[1], f2 = src[2], f3 = src[3];
        slot[0] = f0;
        slot[1] = f1;
        slot[2] = f2;
        slot[3] = f3;
        // the write-back stores go out after the fill has arrived, so the
        // wait for the fill does not include them
        if (wb) write_back(old, o0, o1, o2, o3);
        set_tag(s, p | 0x40);
        return s;
    }
    // Pool byte offset of clean page p, with in_pool false when the pool does
    // not hold it (a program page of a ROM the block did not stage).
    __device__ __forceinline__ uint32_t pool_off(uint32_t p, bool &in_pool) const {
        const uint32_t q = p - 8;                  // program page index (wraps below 0x200)
        const bool low = p < 8, font = (p == 1) | (p == 2);
        const bool prog = !low & (q < staged);
        const bool beyond = !low & (q >= rom_pages);
        in_pool = low | prog | beyond;
        return prog ? pool_rom + 64 * q : (font ? 64 * p : 0u);
    }
    __device__ __forceinline__ uint32_t fill_from_image(uint32_t p, int32_t keep) {
        uint32_t old;
        const uint32_t s = victim(keep, old);
        uint4 *slot = reinterpret_cast<uint4 *>(&sh.cache[lane][64 * s]);
        if (old & 0x80) write_back(old, slot[0], slot[1], slot[2], slot[3]);
        bool in_pool;
        const uint32_t off = pool_off(p, in_pool);
        if (in_pool) {
            const uint4 *src = reinterpret_cast<const uint4 *>(&sh.pool[0][0] + off);
            slot[0] = src[0];
            slot[1] = src[1];
            slot[2] = src[2];
            slot[3] = src[3];
        } else {
            const uint4 *g = reinterpret_cast<const uint4 *>((const uint8_t *)gimg + p * 64);
            slot[0] = g[0];
            slot[1] = g[1];
            slot[2] = g[2];
            slot[3] = g[3];
        }
        set_tag(s, p | 0x40);
        return s;
    }
    // Write every modified slot back (end of the launch).
    __device__ __forceinline__ void flush() {
#pragma unroll
        for (uint32_t s = 0; s < kSlots; s++) {
            const uint32_t t = tag(s);
            if ((t & 0xC0) == 0xC0) {
                const uint4 *slot = reinterpret_cast<const uint4 *>(&sh.cache[lane][64 * s]);
                write_back(t, slot[0], slot[1], slot[2], slot[3]);
            }
        }
        tags &= ~0x80808080u;
    }
    // Slow path of the selects below: make page p readable from LDS.  A
    // written page that is not cached is filled from the env's memory in HBM,
    // a clean page that the pool does not hold from the power-on image in
    // HBM; slot `keep` is not reused.  Returns the page's slot, or -1 for a
    // page of the pool.
    __device__ __forceinline__ int32_t make_resident(uint32_t p, int32_t keep) {
        int32_t s = find(p);
        bool in_pool;
        (void)pool_off(p, in_pool);
        if (s < 0 && is_dirty(p)) s = (int32_t)fill_from_ram(p, keep);
        else if (s < 0 && !in_pool) s = (int32_t)fill_from_image(p, keep);
        return s;
    }
    // LDS address of byte a, computed with selects only: the cache slot of
    // its page, else the pool for a clean page.  `slow` is raised when
    // neither holds (the address is then some other byte of the block's
    // LDS).
    __device__ __forceinline__ const lds_u8 *lds_byte(uint32_t a, bool &slow) const {
        return lds_page_sel(a >> 6, slow) + (a & 63);
    }
    // Instruction word at pc, and the return address stack[(sp - 1) & 15]
    // (the register copy of the top).  Both code bytes are read from pc's page;
    // lanes whose pc is the last byte of a page, or whose page is not in LDS,
    // take the slow path afterwards.
    __device__ __forceinline__ uint32_t fetch(uint32_t pc, uint32_t sp, uint32_t &ret) {
        const uint32_t a1 = (pc + 1) & 0xFFF;
        bool slow = (pc & 63) == 63;
        const lds_u8 *b0 = lds_byte(pc, slow);
        uint32_t op = ((uint32_t)b0[0] << 8) | b0[1];
        ret = top;
        if (slow) {
            make_resident(a1 >> 6, make_resident(pc >> 6, -1));
            bool no = false;
            op = ((uint32_t)*lds_byte(pc, no) << 8) | *lds_byte(a1, no);
        }
        touch(pc >> 6);
        return op;
    }
    // The instruction word alone (the switch cycle of exec_one).
    __device__ __forceinline__ uint32_t fetch(uint32_t pc) {
        uint32_t ret;
        return fetch(pc, 0u, ret);
    }
    // Sixteen bytes of a run of memory that lies on page q0 from byte `off`
    // on and goes on at page q1 (both LDS page bases; off may be below 0 or
    // the run may end before q1 is reached: those bytes are unspecified).
    // The five aligned dwords covering the run are read, dword w of the run's
    // page space from q0 while w < 16 and from q1 after (page ends are dword
    // boundaries, and every page base in LDS is dword aligned), and shifted
    // into place with v_alignbyte.  Byte k of the run lands at bits 8k.  The
    // dwords read outside the two pages lie inside the block's LDS (neither
    // the pool nor the slots is first or last in it).
    __device__ __forceinline__ u32x4 window16(const lds_u8 *q0, const lds_u8 *q1, int32_t off) const {
        const int32_t w0 = off >> 2;
        uint32_t d[5];
#pragma unroll
        for (int i = 0; i < 5; i++) {
            const int32_t w = w0 + i;
            d[i] = *(const lds_u32 *)((w < 16 ? q0 : q1 - 64) + 4 * w);
        }
        const uint32_t sb = (uint32_t)off & 3;
        u32x4 v;
#pragma unroll
        for (int i = 0; i < 4; i++) v[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sb);
        return v;
    }
    // count (1..16) bytes from address a on (12-bit wrap), on at most two
    // pages; byte k lands at bits 8k of the vector.  Bytes past count are
    // left unspecified: the caller masks them.
    __device__ __forceinline__ u32x4 load_bytes(uint32_t a, uint32_t count) {
        const uint32_t off = a & 63;
        const uint32_t p0 = a >> 6, p1 = ((a + count - 1) & 0xFFF) >> 6;
        bool slow = false;
        const lds_u8 *q0 = lds_page_sel(p0, slow), *q1 = lds_page_sel(p1, slow);
        if (slow) {
            make_resident(p1, make_resident(p0, -1));
            bool no = false;
            q0 = lds_page_sel(p0, no);
            q1 = lds_page_sel(p1, no);
        }
        touch(p0);
        touch(p1);
        return window16(q0, q1, (int32_t)off);
    }
    // count (1..16) bytes from address a on (12-bit wrap), byte k of `bytes`
    // to a + k: both pages are made resident in cache slots, then the five
    // aligned dwords covering the run are read and written back with the
    // run's bytes merged in under a byte mask (dwords the run does not reach
    // are written back unchanged).
    __device__ __forceinline__ void store_bytes(uint32_t a, uint32_t count, u32x4 bytes) {
        const uint32_t p0 = a >> 6, p1 = ((a + count - 1) & 0xFFF) >> 6;
        touch(p0);
        touch(p1);
        int32_t s0 = find(p0);
        if (s0 < 0) s0 = (int32_t)(is_dirty(p0) ? fill_from_ram(p0, -1) : fill_from_image(p0, -1));
        int32_t s1 = s0;
        if (p1 != p0) {
            s1 = find(p1);
            if (s1 < 0) s1 = (int32_t)(is_dirty(p1) ? fill_from_ram(p1, s0) : fill_from_image(p1, s0));
        }
        const uint32_t off = a & 63;
        lds_u8 *c0 = slot_ptr((uint32_t)s0), *c1 = slot_ptr((uint32_t)s1);
        const uint32_t w0 = off >> 2, sb = off & 3;
        // the data and its byte mask, one dword before and after: window dword
        // i is dwords i and i + 1 of these shifted right by 4 - sb bytes
        const u32x4 m = byte_mask(count);
        const uint32_t x[6] = {0u, bytes[0], bytes[1], bytes[2], bytes[3], 0u};
        const uint32_t mk[6] = {0u, m[0], m[1], m[2], m[3], 0u};
        lds_u32 *ptr[5];
        uint32_t old[5];
#pragma unroll
        for (int i = 0; i < 5; i++) {
            const uint32_t w = w0 + i;
            ptr[i] = (lds_u32 *)((w < 16 ? c0 : c1 - 64) + 4 * w);
            old[i] = *ptr[i];
        }
#pragma unroll
        for (int i = 0; i < 5; i++) {
            const uint32_t val = sb ? __builtin_amdgcn_alignbyte(x[i + 1], x[i], 4 - sb) : x[i + 1];
            const uint32_t msk = sb ? __builtin_amdgcn_alignbyte(mk[i + 1], mk[i], 4 - sb) : mk[i + 1];
            *ptr[i] = (old[i] & ~msk) | (val & msk);
        }
        tags |= (0x80u << (8 * s0)) | (0x80u << (8 * s1));
        dirty |= (1ull << p0) | (1ull << p1);
    }
    // Page p readable from LDS for a read, or held in a cache slot for a
    // store (slow path): filled from the env's memory in HBM when written, else
    // from the power-on image (the pool or HBM); slot `keep` is not reused.
    // Returns the page's slot, or -1 for a page read from the pool.
    __device__ __forceinline__ int32_t ensure(uint32_t p, int32_t keep, bool st) {
        int32_t s = find(p);
        bool in_pool;
        (void)pool_off(p, in_pool);
        if (s < 0 && is_dirty(p)) s = (int32_t)fill_from_ram(p, keep);
        else if (s < 0 && (st || !in_pool)) s = (int32_t)fill_from_image(p, keep);
        return s;
    }
    // The memory access of one instruction, for the lanes that have one:
    // DXYN (dr: the sprite's rows drawn, the collision flag returned), FX65
    // (count bytes at I returned in `data`) or FX33 / FX55 (st: count bytes
    // of `data` stored at I).  Each reads at most sixteen bytes around I on
    // at most two pages, so one page lookup, one slow path and one read of
    // five aligned dwords serve all three; a store merges its bytes into the
    // dwords read and writes them back.  A DXYN's dwords cover a window of
    // display rows as in draw() (window row w: byte w of the run from I - sh0).
    __device__ __forceinline__ uint32_t access(bool dr, bool st, uint32_t I, uint32_t count, uint32_t x0,
                                               uint32_t y0, bool longw, u32x4 &data) {
        const uint32_t cnt = dr ? min(count, 32 - y0) : count;
        const uint32_t b = min(y0, longw ? 17u : 24u);
        const uint32_t sh0 = dr ? y0 - b : 0u;          // window rows above the sprite
        const uint32_t p0 = I >> 6, p1 = ((I + max(cnt, 1u) - 1) & 0xFFF) >> 6;
        touch(p0);
        touch(p1);
        int32_t s0 = find(p0), s1 = find(p1);
        bool in0, in1;
        const uint32_t o0 = pool_off(p0, in0), o1 = pool_off(p1, in1);
        // readable: cached, or clean and in the pool; a store needs the slot
        const bool ok = ((int)(s0 >= 0) | ((int)!st & (int)!is_dirty(p0) & (int)in0)) &
                        ((int)(s1 >= 0) | ((int)!st & (int)!is_dirty(p1) & (int)in1));
        lds_u8 *pool = (lds_u8 *)&sh.pool[0][0];
        lds_u8 *q0 = s0 >= 0 ? slot_ptr((uint32_t)s0) : pool + o0;
        lds_u8 *q1 = s1 >= 0 ? slot_ptr((uint32_t)s1) : pool + o1;
        if (!ok) {
            s0 = ensure(p0, -1, st);
            s1 = ensure(p1, s0, st);
            q0 = s0 >= 0 ? slot_ptr((uint32_t)s0) : pool + o0;
            q1 = s1 >= 0 ? slot_ptr((uint32_t)s1) : pool + o1;
        }
        const int32_t off = (int32_t)(I & 63) - (int32_t)sh0;
        const int32_t w0 = off >> 2;
        const uint32_t sb = (uint32_t)off & 3;
        lds_u32 *ptr[5];
        uint32_t d[5];
#pragma unroll
        for (int i = 0; i < 5; i++) {
            const int32_t w = w0 + i;
            ptr[i] = (lds_u32 *)((w < 16 ? q0 : q1 - 64) + 4 * w);
            d[i] = *ptr[i];
        }
        u32x4 v;
#pragma unroll
        for (int i = 0; i < 4; i++) v[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sb);
        uint64_t hit = 0;
        if (st) {
            // the data and its byte mask, one dword before and after: dword i
            // of the window is dwords i and i + 1 of these shifted right by
            // 4 - sb bytes
            const u32x4 m = byte_mask(count);
            const uint32_t x[6] = {0u, data[0], data[1], data[2], data[3], 0u};
            const uint32_t mk[6] = {0u, m[0], m[1], m[2], m[3], 0u};
#pragma unroll
            for (int i = 0; i < 5; i++) {
                const uint32_t val = sb ? __builtin_amdgcn_alignbyte(x[i + 1], x[i], 4 - sb) : x[i + 1];
                const uint32_t msk = sb ? __builtin_amdgcn_alignbyte(mk[i + 1], mk[i], 4 - sb) : mk[i + 1];
                *ptr[i] = (d[i] & ~msk) | (val & msk);
            }
            tags |= (0x80u << (8 * (uint32_t)s0)) | (0x80u << (8 * (uint32_t)s1));
            dirty |= (1ull << p0) | (1ull << p1);
        } else if (dr) {
            const uint32_t vm = ((1u << cnt) - 1) << sh0;   // window rows of the sprite
            lds_u64 *fbw = (lds_u64 *)&sh.fb[lane][0] + b;
            if (vm & 0x000Fu) hit |= draw_rows<0, 4>(fbw, x0, vm, v);
            if (vm & 0x00F0u) hit |= draw_rows<4, 4>(fbw, x0, vm, v);
            if (longw && (vm & 0x7F00u)) hit |= draw_rows<8, 7>(fbw, x0, vm, v);
        } else {
            data = v;
        }
        return hit != 0;
    }
    // LDS base of page p, computed with selects only (see lds_byte).
    __device__ __forceinline__ lds_u8 *lds_page_sel(uint32_t p, bool &slow) const {
        const int32_t s = find(p);
        bool in_pool;
        const uint32_t off = pool_off(p, in_pool);
        slow = slow | ((s < 0) & (is_dirty(p) | !in_pool));
        return s >= 0 ? slot_ptr((uint32_t)s) : (lds_u8 *)&sh.pool[0][0] + off;
    }
    // Window rows [W0, W0 + NR): one batch of LDS reads, then the XOR and the
    // row writes.  Window row w is display row b + w (at fbw[w]); its sprite
    // byte is byte w of `spr` (the sixteen memory bytes from I - sh0).  Bit w
    // of vm marks the sprite's rows; the other rows get an empty mask and are
    // written back unchanged.
    template <int W0, int NR>
    __device__ __forceinline__ uint64_t draw_rows(lds_u64 *fbw, uint32_t x0, uint32_t vm, const u32x4 &spr) {
        uint64_t row[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) row[r] = fbw[W0 + r];
        uint64_t hit = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const int w = W0 + r;
            const uint32_t sb = __builtin_amdgcn_ubfe(spr[w >> 2], 8 * (w & 3), 8) * __builtin_amdgcn_ubfe(vm, w, 1);
            const uint64_t m = ((uint64_t)sb << 56) >> x0;
            hit |= row[r] & m;
            fbw[w] = row[r] ^ m;
        }
        return hit;
    }
    // DXYN at (x0, y0) = (VX & 63, VY & 31): rows below the screen are
    // clipped, pixels past x = 63 fall off the shifted mask.  Sprite bytes
    // are at I + r (12-bit wrap), on at most two pages.  Rows are taken in a
    // window of display rows that lies inside the env's 32 rows, so every
    // window row can be written back without a per-row condition: 15 rows
    // from b = min(y0, 17) when some drawing lane of the wave has N > 8, else
    // 8 rows from b = min(y0, 24).  The window's sprite bytes are the sixteen
    // memory bytes from I - sh0 (sh0 = y0 - b rows above the sprite), read as
    // five dwords; the bytes outside the sprite are masked.
    __device__ __forceinline__ uint32_t draw(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n) {
        const uint32_t cnt = min(n, 32 - y0);
        const bool longw = __builtin_amdgcn_ballot_w64(n > 8) != 0;   // among the drawing lanes
        const uint32_t b = min(y0, longw ? 17u : 24u);
        const uint32_t sh0 = y0 - b;                    // window rows above the sprite
        const uint32_t vm = ((1u << cnt) - 1) << sh0;   // window rows of the sprite
        lds_u64 *fbw = (lds_u64 *)&sh.fb[lane][0] + b;
        const uint32_t off = I & 63;
        const uint32_t p0 = I >> 6, p1 = ((I + max(cnt, 1u) - 1) & 0xFFF) >> 6;
        bool slow = false;
        const lds_u8 *q0 = lds_page_sel(p0, slow), *q1 = lds_page_sel(p1, slow);
        if (slow) {
            make_resident(p1, make_resident(p0, -1));
            bool no = false;
            q0 = lds_page_sel(p0, no);
            q1 = lds_page_sel(p1, no);
        }
        touch(p0);
        touch(p1);
        const u32x4 spr = window16(q0, q1, (int32_t)off - (int32_t)sh0);
        uint64_t hit = 0;
        if (vm & 0x000Fu) hit |= draw_rows<0, 4>(fbw, x0, vm, spr);
        if (vm & 0x00F0u) hit |= draw_rows<4, 4>(fbw, x0, vm, spr);
        if (longw && (vm & 0x7F00u)) hit |= draw_rows<8, 7>(fbw, x0, vm, spr);
        return hit != 0;
    }
    // DXYN with the pixel-wrap quirk: all n rows are drawn, row y0 + r at
    // (y0 + r) & 31, and the sprite byte is rotated so that pixels past
    // x = 63 land at the left edge.  A loop over the env's own rows.
    __device__ __forceinline__ uint32_t draw_wrap(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n) {
        const uint32_t off = I & 63;
        const uint32_t p0 = I >> 6, p1 = ((I + max(n, 1u) - 1) & 0xFFF) >> 6;
        bool slow = false;
        const lds_u8 *q0 = lds_page_sel(p0, slow), *q1 = lds_page_sel(p1, slow);
        if (slow) {
            make_resident(p1, make_resident(p0, -1));
            bool no = false;
            q0 = lds_page_sel(p0, no);
            q1 = lds_page_sel(p1, no);
        }
        touch(p0);
        touch(p1);
        lds_u64 *fb = (lds_u64 *)&sh.fb[lane][0];
        uint64_t hit = 0;
        for (uint32_t r = 0; r < n; r++) {
            const uint32_t sb = off + r < 64 ? q0[off + r] : q1[off + r - 64];
            const uint64_t m = __builtin_rotateright64((uint64_t)sb << 56, x0);
            const uint32_t yy = (y0 + r) & 31;
            const uint64_t row = fb[yy];
            hit |= row & m;
            fb[yy] = row ^ m;
        }
        return hit != 0;
    }
    __device__ __forceinline__ uint32_t draw(uint32_t x0, uint32_t y0, uint32_t I, uint32_t n, bool wrap) {
        return wrap ? draw_wrap(x0, y0, I, n) : draw(x0, y0, I, n);
    }
    __device__ __forceinline__ void clear() {
        lds_u64 *fb = (lds_u64 *)&sh.fb[lane][0];
#pragma unroll
        for (int y = 0; y < 32; y++) fb[y] = 0;
    }
    // Stack entry i (0..15), picked out of the registers with masks (a
    // select between array elements would be folded into an indexed load,
    // which puts the whole structure in scratch memory).
    __device__ __forceinline__ uint32_t stack_get(uint32_t i) const {
        uint32_t w = 0;
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) w |= stk[j] & (0u - (uint32_t)((i >> 1) == j));
        return __builtin_amdgcn_ubfe(w, (i & 1) * 16, 16);
    }
    // A call stores its return address at entry i = SP, which becomes the top.
    __device__ __forceinline__ void stack_set(uint32_t i, uint32_t v) {
        const uint32_t sh16 = (i & 1) * 16;
        const uint32_t m = 0xFFFFu << sh16, nv = (v & 0xFFFF) << sh16;
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t mj = m & (0u - (uint32_t)((i >> 1) == j));
            stk[j] = (stk[j] & ~mj) | (nv & mj);
        }
        top = v & 0xFFFF;
    }
    // After a return SP is sp: the new top is stack[(sp - 1) & 15].
    __device__ __forceinline__ void stack_popped(uint32_t sp) { top = stack_get((sp - 1) & 15); }
    __device__ __forceinline__ void stack_clear() {
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) stk[j] = 0;
        top = 0;
    }
    // Restore the written pages from the image (automatic reset).
    __device__ __forceinline__ void restore_pages() {
        uint64_t d = dirty;
        while (d) {
            const uint32_t p = __builtin_ctzll(d);
            d &= d - 1;
            uint4 *dst = reinterpret_cast<uint4 *>((uint8_t *)ram + p * 64);
            bool in_pool;
            const uint32_t off = pool_off(p, in_pool);
            if (in_pool) {
                const uint4 *src = reinterpret_cast<const uint4 *>(&sh.pool[0][0] + off);
#pragma unroll
                for (int q = 0; q < 4; q++) dst[q] = src[q];
            } else {
                const uint4 *src = reinterpret_cast<const uint4 *>((const uint8_t *)gimg + p * 64);
#pragma unroll
                for (int q = 0; q < 4; q++) dst[q] = src[q];
            }
        }
        dirty = 0;
        tags = 0;
    }
};

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Step counters shared by the two waves of a pair.  The fences order LDS
// only, so the writer waves' observation stores in flight are not waited for.
__device__ __forceinline__ void set_flag(uint32_t *f, uint32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t get_flag(const uint32_t *f) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}
// Wait until the flag reaches v.  The partner wave raises it within a step.
// The wait is bounded by `limit` ticks of the device wall clock, derived by
// the host from the longest step the config allows, so that every wave ends
// whatever happens; a wait that gives up sets bit 0 of the engine's error
// word (one lane, a global atomic), which the host reports: the outputs of
// that launch are not valid.
__device__ __forceinline__ void wait_flag(const uint32_t *f, uint32_t v, uint64_t limit, uint32_t *err) {
    if (get_flag(f) < v) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (get_flag(f) < v) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                if (__lane_id() == 0) __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Per-lane step counters (variants with reset steps): a byte per env, counting
// modulo 256; a partner is never more than one step ahead, so a difference
// of zero or one is all they ever hold.
__device__ __forceinline__ void set_lane_flag(uint8_t *f, uint32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __hip_atomic_store(f, (uint8_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t get_lane_flag(const uint8_t *f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Bounded wait of a per-lane loop in which no lane can go on: true while it
// may go on waiting (after a short sleep); false once `limit` ticks have
// passed since the wait began, after setting bit 0 of the error word.
__device__ __forceinline__ bool keep_waiting(bool &waiting, uint64_t &since, uint64_t limit, uint32_t *err) {
    const uint64_t now = __builtin_amdgcn_s_memrealtime();
    if (!waiting) {
        waiting = true;
        since = now;
    }
    if (now - since > limit) {
        if (__lane_id() == 0) __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        waiting = false;
        return false;
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
}

// One environment step of emulation with `key` held: frame_skip frames of
// ipf instructions, each followed by a timer tick.  With the display-wait
// quirk (kProfile variants only) a lane's DXYN ends its frame: the lane sits
// out the frame's remaining instruction slots.  With kSparse (the per-lane
// variants), an instruction slot run by at most kSparseLanes lanes takes the
// switch of exec_one instead of the grouped cycle: with few lanes left (the
// envs still in their reset steps at the end of a launch) the wave then runs
// only the handlers those lanes need, instead of the grouped cycle's selects
// for every class.  Both are the same instruction set (octax_core.h).
constexpr uint32_t kSparseLanes = 4;
template <bool kProfile, bool kSparse, class Mem>
__device__ __forceinline__ void run_frames(Core &c, Mem &mem, uint32_t key, uint32_t ipf, uint32_t fs,
                                           uint32_t quirks) {
    for (uint32_t f = 0; f < fs; f++) {
        bool run = true;
        for (uint32_t i = 0; i < ipf; i++) {
            if (!kProfile || run) {
                bool drew;
                if (kSparse && __builtin_popcountll(__builtin_amdgcn_ballot_w64(true)) <= kSparseLanes) {
                    const uint32_t sp0 = c.sp;
                    drew = exec_one(c, mem, key, quirks);
                    // a call sets the register copy of the top entry itself, a return pops it
                    if (c.sp == ((sp0 - 1) & 15)) mem.stack_popped(c.sp);
                } else {
                    drew = exec_grouped(c, mem, key, quirks);
                }
                run = !(drew && (quirks & kQuirkDisplayWait));
            }
        }
        tick(c);
    }
}

// Lane l's share of two consecutive expanded frames, one 4 KB piece of an
// observation: bytes [16l, 16l+16) and [1024+16l, ...) of each frame.
__device__ __forceinline__ void store_pair(uint8_t *o, uint32_t lane64, u32x4 a0, u32x4 a1, u32x4 b0, u32x4 b1) {
    store_obs(o + 16 * lane64, a0);
    store_obs(o + 1024 + 16 * lane64, a1);
    store_obs(o + 2048 + 16 * lane64, b0);
    store_obs(o + 3072 + 16 * lane64, b1);
}

// Envs per round of the writers' cooperative pass: the staging area of a
// wave holds kStageEnvs packed frames, the frames of steps k - 1 and k of
// each env of the round.
constexpr uint32_t kPairEnvs = kStageEnvs / 2;

// The range of slots a block serves.  The hardware deals the blocks of a
// launch to the eight XCDs in turn (block b to XCD b % 8); the mapping gives
// each XCD one contiguous run of slot ranges, so the CUs of an XCD write
// neighbouring observations (on MI355X the observation stores run about a
// fifth faster than with consecutive ranges spread over the XCDs).  Any
// grid size maps one to one.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    constexpr uint32_t kXcds = 8;
    const uint32_t x = b % kXcds, i = b / kXcds;
    const uint32_t per = nb / kXcds, rem = nb % kXcds;
    return x * per + min(x, rem) + i;
}

// Wave roles.  A block runs IPW envs with 2 * IPW threads: waves
// 0 .. IPW/64 - 1 emulate (one env per lane, thread l is env l) and waves
// IPW/64 .. 2 * IPW/64 - 1 write observations (thread IPW + l serves env l).
// Emulator wave w and writer wave w form a pair that synchronises through
// two LDS step counters instead of block barriers:
//   * the emulator raises ready[w] to k + 1 when the display of step k is
//     final (auto-reset included), and starts step k + 1 once taken[w] says
//     that display has been copied;
//   * the writer copies the display of step k into registers when ready[w]
//     allows, raises taken[w], then transposes, expands and stores it while
//     the emulator runs step k + 1.
// The observation stores and the emulation thus share each SIMD as two waves,
// and each pair runs at its own pace: a slow step of one pair does not hold
// up the other pairs of the block.
//
// kRollout separates the K-step launches (graph-captured rollouts) from the
// K = 1 launches of octax_step into two instantiations of the same code, so
// profiles report them apart.  kResetSteps instantiates the emulation steps
// of a reset (start-up sequence, no-op reset); without those wrappers the
// kernel carries no second copy of the instruction cycle.  kProfile
// instantiates the quirk flags and the extra game descriptors (score mode,
// second termination clause); without them those selects fold away.
template <int IPW, bool kRollout, bool kResetSteps, bool kProfile>
__global__ __launch_bounds__(2 * IPW) void step_fused_kernel(State s, Roms roms, StepIO io, FusedCfg cfg) {
    __shared__ Shared<IPW> sh;
    const uint32_t tid = threadIdx.x;
    const bool emu = __builtin_amdgcn_readfirstlane(tid) < (uint32_t)IPW;   // wave-uniform role
    const uint32_t l = emu ? tid : tid - IPW;                                 // env of this thread
    const uint32_t lane64 = l & 63;
    const uint32_t wave = l >> 6;
    const uint32_t wave_base = l & ~63u;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);   // slot range of this block
    const uint32_t slot = blk * IPW + l;
    const uint32_t E = s.num;
    const uint32_t K = io.K;
    const bool active = slot_live(s, slot);
    // steps this launch runs for the slot: K, or the slot's budget (at most
    // K; a serving pool's group stops at its last step inside a launch)
    const uint32_t steps = (cfg.budget && active) ? min(K, (uint32_t)cfg.budget[slot]) : K;
    // A block with no env (free range of a serving pool) has nothing to do:
    // the host marks it in the block's pool table (no ROM listed).
    const uint32_t *ptab = cfg.block_roms + (size_t)blk * kPoolRoms * 2;
    if (ptab[0] == kPoolEnd) return;
    const uint32_t live = active ? 1u : 0u;
    const uint32_t wave_slot0 = blk * IPW + wave_base;
    const uint32_t nj = (E > wave_slot0) ? min(64u, E - wave_slot0) : 0u;   // slots of this wave

    // Fill the block's page pool (all threads): the zero page, memory pages 1
    // and 2 (the font; the same in every image, taken from the first listed
    // ROM's) and, with ROM staging on, the program pages the table lists.
    {
        uint4 *pool4 = reinterpret_cast<uint4 *>(&sh.pool[0][0]);
        const uint4 *img0 = reinterpret_cast<const uint4 *>(roms.image + (size_t)ptab[0] * kMem);
        for (uint32_t q = tid; q < 12; q += 2 * IPW) pool4[q] = q < 4 ? make_uint4(0, 0, 0, 0) : img0[q];
        for (uint32_t j = 0; cfg.rom_in_lds && j < kPoolRoms && ptab[2 * j] != kPoolEnd; j++) {
            const uint32_t info = ptab[2 * j + 1];
            const uint32_t n16 = (info & 0xFF) * 4, first16 = (info >> 16) * 4;
            const uint4 *src = reinterpret_cast<const uint4 *>(roms.image + (size_t)ptab[2 * j] * kMem + kProgram);
            for (uint32_t q = tid; q < n16; q += 2 * IPW) pool4[first16 + q] = src[q];
        }
    }

    Core c;
    uint32_t head = 0, env = 0, rom = 0, desc = 0, desc2 = kDesc2Default, t = 0, hor = 0, tags = 0;
    uint4 stack_in[2] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
    const uint32_t quirks = kProfile ? roms.quirks : 0u;   // 0: the base profile
    int32_t prev = 0;
    uint64_t dirty = 0;
    u32x4 keys = {0, 0, 0, 0};   // the ROM's 16 action keys, one byte each
    reset_core(c);
    c.rng = 0;
    if (active) {
        head = (s.misc[slot] >> 24) & 3;
        env = s.env_of[slot];
        rom = s.rom_of[slot];
        desc = roms.desc[rom];
        if (kProfile && roms.desc2) desc2 = roms.desc2[rom];
        keys = *reinterpret_cast<const u32x4 *>(roms.keys + (size_t)rom * 16);
    }
    const uint32_t nact = desc >> 24;
    // Key held for an action: the ROM's key for 0 <= a < num_actions, else none.
    auto held_key = [&](int32_t a) -> uint32_t {
        const uint32_t ua = (uint32_t)a;
        const uint32_t word = (ua & 8) ? ((ua & 4) ? keys.w : keys.z) : ((ua & 4) ? keys.y : keys.x);
        return (ua < nact) ? (__builtin_amdgcn_ubfe(word, (ua & 3) * 8, 8) & 15) : kKeyNone;
    };
    // Emulator lanes keep the held keys of 64 consecutive steps in
    // registers, one byte each, loaded 64 steps at a time (the loads of a
    // batch go out together: one round trip per 64 steps).
    u32x16 kp = {};
    auto load_keys = [&](uint32_t k0) {
#pragma unroll
        for (int w = 0; w < 16; w++) {
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const uint32_t kk = k0 + 4 * w + b;
                const int32_t *row = io.action + (size_t)kk * E;   // wave-uniform row base
                const int32_t a = kk < K ? row[env] : -1;
                word |= held_key(a) << (8 * b);
            }
            kp[w] = word;
        }
    };
    auto key_of_step = [&](uint32_t kk) -> uint32_t {
        return __builtin_amdgcn_ubfe(kp[(kk >> 2) & 15], (kk & 3) * 8, 8);
    };
    if (emu && active) {
        load_keys(0);
        load_core(s, slot, c, head);
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
        stack_in[0] = st4[0];
        stack_in[1] = st4[1];
    }
    // This env's ROM in the pool table: its staged and program pages, and
    // where they start.  A ROM the table does not list has no staged page,
    // and all its program pages read through the cache slots.
    uint32_t staged = 0, rom_pages = 56, pool_rom = 0;
    for (uint32_t j = 0; j < kPoolRoms && ptab[2 * j] != kPoolEnd; j++) {
        const uint32_t info = ptab[2 * j + 1];
        if (ptab[2 * j] == rom) {
            staged = cfg.rom_in_lds ? (info & 0xFF) : 0u;
            rom_pages = (info >> 8) & 0xFF;
            pool_rom = 64 * (info >> 16);
        }
    }
    const glb_u8 *gimg = (const glb_u8 *)(roms.image + (size_t)rom * kMem);
    glb_u8 *ram = (glb_u8 *)(s.ram + (size_t)slot * kMem);
    const size_t obs_step = (size_t)E * kObsBytes;
    auto obs_of = [&](uint32_t kk, uint32_t e) -> uint8_t * {
        return io.obs + (size_t)(kk % io.obs_slots) * obs_step + (size_t)e * kObsBytes;
    };

    // Writers, prologue: the three frames before this launch fill the lower
    // halves of observations 0 and 1 (frame f of step k is the frame of step
    // k - 3 + f).  All loads of a chunk of envs are issued before its stores.
    if (!emu && io.obs) {
        for (uint32_t j0 = 0; j0 < nj; j0 += kPrologueEnvs) {
            uint32_t w[kPrologueEnvs][3];
#pragma unroll
            for (int jj = 0; jj < kPrologueEnvs; jj++) {
                const uint32_t j = min(j0 + jj, nj - 1);
                const uint32_t jh = __builtin_amdgcn_readlane(head, j);
                const uint32_t *ring = s.cols + (size_t)(wave_slot0 + j) * 256 + lane64;
                w[jj][0] = ring[jh * 64];                 // step -1
                w[jj][1] = ring[((jh + 3) & 3) * 64];     // step -2
                w[jj][2] = ring[((jh + 2) & 3) * 64];     // step -3
            }
#pragma unroll
            for (int jj = 0; jj < kPrologueEnvs; jj++) {
                const uint32_t j = j0 + jj;
                if (j >= nj) break;
                if (!__builtin_amdgcn_readlane(live, j)) continue;
                const uint32_t je = __builtin_amdgcn_readlane(env, j);
                const u32x4 m1a = spread16(w[jj][0]), m1b = spread16(w[jj][0] >> 16);
                const u32x4 m2a = spread16(w[jj][1]), m2b = spread16(w[jj][1] >> 16);
                const u32x4 m3a = spread16(w[jj][2]), m3b = spread16(w[jj][2] >> 16);
                store_pair(obs_of(0, je), lane64, m3a, m3b, m2a, m2b);                 // steps -3, -2
                if (__builtin_amdgcn_readlane(steps, j) > 1)
                    store_pair(obs_of(1, je), lane64, m2a, m2b, m1a, m1b);               // steps -2, -1
            }
        }
    }
    if (tid < IPW / 64) {
        sh.ready[tid] = 0;
        sh.taken[tid] = 0;
    }
    if (tid < IPW) {
        sh.lready[tid] = 0;
        sh.ltaken[tid] = 0;
        sh.budget[tid] = (uint8_t)min(steps, 255u);
    }
    __syncthreads();

    // Step clock (optional): wave pair gw records, on the device wall clock,
    // when its emulator wave starts step k and when its writer wave has issued
    // the last store of step k.
    const uint32_t gw = wave_slot0 / 64, nwaves = (E + 63) / 64;
    auto stamp = [&](uint32_t k, uint32_t which) {
        if (cfg.stamps && k < cfg.stamp_steps && nj > 0 && lane64 == 0)
            cfg.stamps[((size_t)k * nwaves + gw) * 2 + which] = __builtin_amdgcn_s_memrealtime();
    };

    FusedMem<IPW> mem{sh, l, pool_rom, staged, rom_pages, gimg, ram, dirty, tags,
                      {stack_in[0].x, stack_in[0].y, stack_in[0].z, stack_in[0].w,
                       stack_in[1].x, stack_in[1].y, stack_in[1].z, stack_in[1].w}, 0u};
    mem.top = mem.stack_get((c.sp - 1) & 15);
    // End of an emulator wave: the state goes back to HBM once per launch.
    // (Called at the end of each emulator loop, so that none of the
    // emulator's registers stay live in the writer waves' loops.)
    auto emu_epilogue = [&]() {
        if (!active) return;
        mem.flush();
        store_core(s, slot, c, head);
        s.t[slot] = t;
        s.prev[slot] = prev;
        s.dirty[slot] = mem.dirty;
        uint4 *fb4 = reinterpret_cast<uint4 *>(s.fb + (size_t)slot * 32);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const uint64_t a = sh.fb[l][2 * q], b = sh.fb[l][2 * q + 1];
            fb4[q] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
        }
        uint4 *st4 = reinterpret_cast<uint4 *>(s.stack + (size_t)slot * 8);
        st4[0] = make_uint4(mem.stk[0], mem.stk[1], mem.stk[2], mem.stk[3]);
        st4[1] = make_uint4(mem.stk[4], mem.stk[5], mem.stk[6], mem.stk[7]);
    };
    // Writer lanes: their env's packed frame of step -1 (the first of the pair
    // that step 0 stores), from the env's frame ring.
    auto load_prev = [&](uint32_t (&pb)[64]) {
#pragma unroll
        for (int q = 0; q < 64; q++) pb[q] = 0;
        if (active && io.obs) {
            const uint4 *r4 = reinterpret_cast<const uint4 *>(s.cols + (size_t)slot * 256 + head * 64);
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const uint4 v = r4[q];
                pb[4 * q] = v.x;
                pb[4 * q + 1] = v.y;
                pb[4 * q + 2] = v.z;
                pb[4 * q + 3] = v.w;
            }
        }
    };
    if constexpr (kResetSteps) {
        // Per-lane progress (variants whose resets run emulation steps).  A
        // reset here runs a ROM's start-up sequence and up to noop_max no-op
        // steps before the step can return its observation; in lockstep the
        // whole wave would wait for that lane.  Instead every lane keeps its
        // own step counter and reset phase, and the wave runs step-sized slots
        // (frame_skip frames of ipf instructions) for all lanes that can go on:
        //   * emulator lane l publishes step k (display final, reward and done
        //     in LDS) by raising lready[l] to k + 1, and runs the slot of step
        //     k + 1 once ltaken[l] says that display has been copied; slots of
        //     a reset's steps need no such wait (step k's display is not
        //     published before the reset ends), and a slot starts when no
        //     lane is left waiting;
        //   * writer lane l copies its env's display whenever a new step is
        //     published, and the wave stores the frames of all lanes that had
        //     one, four envs per round, each into the observations of its own
        //     steps.
        if (emu) {
            uint32_t k = 0;          // the step this lane emulates next
            uint32_t phase = 0;      // 0: a step; 1: start-up steps of a reset; 2: its no-op steps
            uint32_t si = 0, left = 0;
            uint32_t kblock = 0;     // first step of the loaded key batch
            float pend_rew = 0.f;
            uint32_t pend_done = 0;
            const uint8_t *su = roms.w.startup ? roms.w.startup + (size_t)rom * 17 : nullptr;
            const uint32_t n_startup = su ? su[0] : 0u;
            bool waiting = false;
            uint64_t since = 0;
            while (true) {
                const bool want = active && k < steps;
                if (!__builtin_amdgcn_ballot_w64(want)) break;
                // A slot starts once no lane waits for its display to be
                // copied: the lanes of a reset then run their reset steps in
                // the same slots as the other lanes' steps, instead of in
                // slots of their own while those lanes wait.
                bool run = want && (phase != 0 || k == 0 || ((get_lane_flag(&sh.ltaken[l]) - k) & 0xFF) == 0);
                if (__builtin_amdgcn_ballot_w64(want && !run)) {
                    if (keep_waiting(waiting, since, cfg.wait_ticks, cfg.err)) continue;
                    run = want;      // gave up (reported): go on regardless
                } else {
                    waiting = false;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                // a step whose display is final this slot is published at the
                // slot's end by all its lanes at once, so the writer takes the
                // slot's frames in one pass
                bool pub = false;
                float pub_rew = 0.f;
                uint32_t pub_done = 0;
                if (run) {
                    uint32_t key = kKeyNone;
                    if (phase == 0) {
                        if ((k & 63) == 0 && k != kblock) {
                            load_keys(k);
                            kblock = k;
                        }
                        key = sticky_key(roms, c, key_of_step(k));
                    }
                    else if (phase == 1) key = su[1 + si];
                    run_frames<kProfile, true>(c, mem, key, io.ipf, io.frame_skip, quirks);
                    if (phase == 0) {
                        const int32_t score = score_of(c.r, desc, desc2);
                        const float reward = (float)(score - prev);
                        const uint32_t term = terminated_of(c.r, desc, desc2);
                        t += 1;
                        const uint32_t trunc = (hor != 0) && (t >= hor);
                        const uint32_t done = term | (trunc << 1);
                        if (done) {
                            // Automatic reset (Section 3.4); the RNG stream continues.
                            mem.restore_pages();
                            reset_core(c);
                            mem.clear();
                            mem.stack_clear();
                            phase = 1;
                            si = 0;
                            pend_rew = reward;
                            pend_done = done;
                        } else {
                            prev = score;
                            head = (head + 1) & 3;
                            pub = true;
                            pub_rew = reward;
                            pub_done = done;
                        }
                    } else if (phase == 1) {
                        si += 1;
                    } else {
                        left -= 1;
                    }
                    // the start-up sequence done, draw the no-op steps; those done, the reset ends
                    if (phase == 1 && si >= n_startup) {
                        phase = 2;
                        left = 0;
                        if (roms.w.noop_max) {
                            const uint64_t u = splitmix_next(c.rng);
                            left = (uint32_t)(((u >> 32) * ((uint64_t)roms.w.noop_max + 1)) >> 32);
                        }
                    }
                    if (phase == 2 && left == 0) {
                        c.pkey = kKeyNone;
                        head = 0;
                        t = 0;
                        prev = score_of(c.r, desc, desc2);   // the score after the reset's steps
                        phase = 0;
                        pub = true;
                        pub_rew = pend_rew;
                        pub_done = pend_done;
                    }
                }
                if (pub) {
                    sh.rew[l] = pub_rew;
                    sh.done[l] = (uint8_t)pub_done;
                }
                if (pub) {
                    set_lane_flag(&sh.lready[l], k + 1);
                    k += 1;
                }
            }
            emu_epilogue();
        } else {
            uint32_t pa[64], pb[64];   // packed frames of the current and the previous step
            load_prev(pb);
            uint32_t kw = 0;         // steps whose display this lane has taken
            bool waiting = false;
            uint64_t since = 0;
            while (true) {
                const bool want = active && kw < steps;
                if (!__builtin_amdgcn_ballot_w64(want)) break;
                bool have = want && ((get_lane_flag(&sh.lready[l]) - kw) & 0xFF) != 0;
                if (!__builtin_amdgcn_ballot_w64(have)) {
                    if (keep_waiting(waiting, since, cfg.wait_ticks, cfg.err)) continue;
                    have = want;     // gave up (reported): take the displays as they are
                } else {
                    waiting = false;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                uint32_t hi[32], lo[32];
#pragma unroll
                for (int r = 0; r < 32; r++) {
                    const uint64_t row = sh.fb[l][31 - r];
                    hi[r] = (uint32_t)(row >> 32);
                    lo[r] = (uint32_t)row;
                }
                uint32_t done = 0;
                if (have) {
                    done = sh.done[l];
                    const float wrew = sh.rew[l];
                    set_lane_flag(&sh.ltaken[l], kw + 1);
                    io.reward[(size_t)kw * E + env] = wrew;
                    io.done[(size_t)kw * E + env] = (uint8_t)done;
                    head = done ? 0u : (head + 1) & 3;
                }
                rows_to_cols(hi, lo);
                pack_frame(hi, lo, pa);
                // the lanes with a new frame, two per round (rank: place among
                // them); each stages its frames of steps kw - 1 and kw and
                // goes out as in the lockstep pass, into its own steps'
                // observations
                const uint64_t hmask = __builtin_amdgcn_ballot_w64(have);
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(hmask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)hmask, 0u));
                uint64_t rem = hmask;
                for (uint32_t r0 = 0; rem; r0 += kPairEnvs) {
                    if (have && rank - r0 < kPairEnvs) {
                        uint4 *stp = reinterpret_cast<uint4 *>(sh.stage[wave][2 * (rank - r0)]);
                        uint4 *stc = reinterpret_cast<uint4 *>(sh.stage[wave][2 * (rank - r0) + 1]);
#pragma unroll
                        for (int q = 0; q < 16; q++) {
                            stp[q] = make_uint4(pb[4 * q], pb[4 * q + 1], pb[4 * q + 2], pb[4 * q + 3]);
                            stc[q] = make_uint4(pa[4 * q], pa[4 * q + 1], pa[4 * q + 2], pa[4 * q + 3]);
                        }
                    }
                    wave_sync();
#pragma unroll
                    for (uint32_t jj = 0; jj < kPairEnvs; jj++) {
                        if (!rem) break;
                        const uint32_t j = (uint32_t)__builtin_ctzll(rem);
                        rem &= rem - 1;
                        const uint32_t kj = __builtin_amdgcn_readlane(kw, j);
                        const uint32_t je = __builtin_amdgcn_readlane(env, j);
                        const uint32_t jdone = __builtin_amdgcn_readlane(done, j);
                        const uint32_t cw = sh.stage[wave][2 * jj + 1][lane64];
                        // the frames before a reset belong to the old episode
                        const uint32_t pv = jdone ? cw : sh.stage[wave][2 * jj][lane64];
                        if (io.obs) {
                            const u32x4 p0 = spread16(pv), p1 = spread16(pv >> 16);
                            const u32x4 c0 = spread16(cw), c1 = spread16(cw >> 16);
                            store_pair(obs_of(kj, je) + 4096, lane64, p0, p1, c0, c1);
                            // (observations past the env's last step of the launch are not
                            // written: with fewer observation slots than steps they would
                            // overwrite the slot of one that is)
                            const uint32_t sj = __builtin_amdgcn_readlane(steps, j);
                            if (kj + 2 < sj) store_pair(obs_of(kj + 2, je), lane64, p0, p1, c0, c1);
                            if (jdone) {
                                store_pair(obs_of(kj, je), lane64, c0, c1, c0, c1);
                                if (kj + 1 < sj) store_pair(obs_of(kj + 1, je), lane64, c0, c1, c0, c1);
                            }
                        }
                        if (kj + 4 >= __builtin_amdgcn_readlane(steps, j)) {
                            const uint32_t jh = __builtin_amdgcn_readlane(head, j);
                            uint32_t *ring = s.cols + (size_t)(wave_slot0 + j) * 256 + lane64;
                            ring[jh * 64] = cw;
                            if (jdone) {
                                ring[((jh + 1) & 3) * 64] = cw;
                                ring[((jh + 2) & 3) * 64] = cw;
                                ring[((jh + 3) & 3) * 64] = cw;
                            }
                        }
                    }
                    wave_sync();
                }
                // this lane's frame of its step kw is the first of its next pair
#pragma unroll
                for (int q = 0; q < 64; q++) pb[q] = have ? pa[q] : pb[q];
                kw += have ? 1u : 0u;
            }
        }
    } else if (emu) {
        for (uint32_t k = 0; k < K; k++) {
            // the display of step k - 1 must have been copied before it changes
            if (k > 0) wait_flag(&sh.taken[wave], k, cfg.wait_ticks, cfg.err);
            stamp(k, 0);
            if (k > 0 && (k & 63) == 0 && active) load_keys(k);
            // (the step count of a budgeted launch is read from LDS, so that it
            // does not hold a register through the emulator loop)
            if (active && (!cfg.budget || k < sh.budget[l])) {
                const uint32_t key = sticky_key(roms, c, key_of_step(k));
                run_frames<kProfile, false>(c, mem, key, io.ipf, io.frame_skip, quirks);
                const int32_t score = score_of(c.r, desc, desc2);
                const float reward = (float)(score - prev);
                const uint32_t term = terminated_of(c.r, desc, desc2);
                t += 1;
                const uint32_t trunc = (hor != 0) && (t >= hor);
                const uint32_t done = term | (trunc << 1);
                sh.rew[l] = reward;
                sh.done[l] = (uint8_t)done;
                if (done) {
                    // Automatic reset (Section 3.4); the RNG stream continues.
                    mem.restore_pages();
                    reset_core(c);
                    mem.clear();
                    mem.stack_clear();
                    if (kResetSteps) {
                        run_reset_steps(roms, rom, c, [&](uint32_t rkey) {
                            run_frames<kProfile, false>(c, mem, rkey, io.ipf, io.frame_skip, quirks);
                        });
                    }
                    head = 0;
                    t = 0;
                    prev = score_of(c.r, desc, desc2);   // the score after the reset's steps
                } else {
                    prev = score;
                    head = (head + 1) & 3;
                }
            }
            set_flag(&sh.ready[wave], k + 1);
        }
        emu_epilogue();
    } else {
        // Each step k stores two 4 KB pieces per env: frames k - 1 and k are
        // the upper half of observation k and the lower half of observation
        // k + 2.  The packed frame of step k - 1 stays in registers; the two
        // arrays trade roles from one step to the next.
        uint32_t pa[64], pb[64];   // packed frames of the current and the previous step
        load_prev(pb);
        auto wstep = [&](uint32_t k, uint32_t (&pw)[64], const uint32_t (&pp)[64]) __attribute__((always_inline)) {
            // Copy the display, reward and done bits of step k once final
            // and let the emulator go on.
            wait_flag(&sh.ready[wave], k + 1, cfg.wait_ticks, cfg.err);
            uint32_t hi[32], lo[32];
#pragma unroll
            for (int r = 0; r < 32; r++) {
                const uint64_t row = sh.fb[l][31 - r];
                hi[r] = (uint32_t)(row >> 32);
                lo[r] = (uint32_t)row;
            }
            const bool ran = active && k < steps;   // this lane's env ran step k
            const uint32_t done = ran ? sh.done[l] : 0u;
            const float wrew = sh.rew[l];
            set_flag(&sh.taken[wave], k + 1);
            // the last four frames of each env's steps go into its ring; the
            // observations past an env's last step of the launch are not
            // written (with fewer observation slots than steps they would
            // overwrite the slot of one that is)
            const uint64_t ring_bits = __builtin_amdgcn_ballot_w64(ran && k + 4 >= steps);
            const uint64_t k1_bits = __builtin_amdgcn_ballot_w64(ran && k + 1 < steps);
            const uint64_t k2_bits = __builtin_amdgcn_ballot_w64(ran && k + 2 < steps);
            const bool ring_step = ring_bits != 0;
            if (ran) {
                io.reward[(size_t)k * E + env] = wrew;
                io.done[(size_t)k * E + env] = (uint8_t)done;
                head = done ? 0u : (head + 1) & 3;
            }
            const uint64_t ran_bits = __builtin_amdgcn_ballot_w64(ran);
            if (!(io.obs || ring_step)) {
                stamp(k, 1);
                return;
            }
            rows_to_cols(hi, lo);
            pack_frame(hi, lo, pw);
            // observations k (upper half), k + 2 (lower half) and, after a
            // reset, k and k + 1 (lower half), at env 0
            uint8_t *const o_k = io.obs ? obs_of(k, 0) : nullptr;
            uint8_t *const o_k1 = io.obs ? obs_of(k + 1, 0) : nullptr;
            uint8_t *const o_k2 = io.obs ? obs_of(k + 2, 0) : nullptr;
            // Cooperative pass, two envs per round: stage their packed
            // frames of steps k - 1 and k, then each lane expands its 16 + 16
            // pixels of the four frames into bytes and the round's pieces go
            // out, observation k before observation k + 2.  The env's
            // observation base is wave-uniform, so a store is one scalar add
            // and the store itself.
            for (uint32_t r0 = 0; r0 < nj; r0 += kPairEnvs) {
                if (active && lane64 - r0 < kPairEnvs) {
                    uint4 *stp = reinterpret_cast<uint4 *>(sh.stage[wave][2 * (lane64 - r0)]);
                    uint4 *stc = reinterpret_cast<uint4 *>(sh.stage[wave][2 * (lane64 - r0) + 1]);
#pragma unroll
                    for (int q = 0; q < 16; q++) {
                        stp[q] = make_uint4(pp[4 * q], pp[4 * q + 1], pp[4 * q + 2], pp[4 * q + 3]);
                        stc[q] = make_uint4(pw[4 * q], pw[4 * q + 1], pw[4 * q + 2], pw[4 * q + 3]);
                    }
                }
                wave_sync();
                const uint32_t n = __builtin_amdgcn_readfirstlane(min(r0 + kPairEnvs, nj) - r0);
                // slots of the round that hold a live env (wave-uniform)
                const uint32_t rmask = (uint32_t)(ran_bits >> r0) & ((1u << n) - 1);
                uint32_t cw[kPairEnvs], pv[kPairEnvs], jdone[kPairEnvs];
#pragma unroll
                for (uint32_t jj = 0; jj < kPairEnvs; jj++) {
                    cw[jj] = sh.stage[wave][2 * jj + 1][lane64];
                    jdone[jj] = __builtin_amdgcn_readlane(done, r0 + jj);
                    // the frames before a reset belong to the old episode:
                    // the stack restarts with the display after the reset
                    pv[jj] = jdone[jj] ? cw[jj] : sh.stage[wave][2 * jj][lane64];
                }
                if (io.obs) {
                    // env by env: its four expanded frame halves, then its pieces
#pragma unroll
                    for (uint32_t jj = 0; jj < kPairEnvs; jj++) {
                        if (!((rmask >> jj) & 1)) continue;
                        const uint64_t eo = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(env, r0 + jj) * kObsBytes;
                        const u32x4 p0 = spread16(pv[jj]), p1 = spread16(pv[jj] >> 16);
                        const u32x4 c0 = spread16(cw[jj]), c1 = spread16(cw[jj] >> 16);
                        store_pair(o_k + eo + 4096, lane64, p0, p1, c0, c1);
                        if ((k2_bits >> (r0 + jj)) & 1) store_pair(o_k2 + eo, lane64, p0, p1, c0, c1);
                        if (jdone[jj]) {
                            store_pair(o_k + eo, lane64, c0, c1, c0, c1);
                            if ((k1_bits >> (r0 + jj)) & 1) store_pair(o_k1 + eo, lane64, c0, c1, c0, c1);
                        }
                    }
                }
                // the last four frames of the launch stay in the ring; a
                // reset fills the three slots before the new head with the
                // display after the reset
                if (ring_step) {
#pragma unroll
                    for (uint32_t jj = 0; jj < kPairEnvs; jj++) {
                        if (!((ring_bits >> (r0 + jj)) & 1)) continue;
                        const uint32_t jh = __builtin_amdgcn_readlane(head, r0 + jj);
                        uint32_t *ring = s.cols + (size_t)(wave_slot0 + r0 + jj) * 256 + lane64;
                        ring[jh * 64] = cw[jj];
                        if (jdone[jj]) {
                            ring[((jh + 1) & 3) * 64] = cw[jj];
                            ring[((jh + 2) & 3) * 64] = cw[jj];
                            ring[((jh + 3) & 3) * 64] = cw[jj];
                        }
                    }
                }
                wave_sync();
            }
            stamp(k, 1);
        };
        for (uint32_t k = 0; k < K; k++) {
            wstep(k, pa, pb);
#pragma unroll
            for (int q = 0; q < 64; q++) pb[q] = pa[q];
        }
    }
}

template <int IPW, bool kResetSteps, bool kProfile>
hipError_t launch_variant(const State &s, const Roms &r, const StepIO &io, const FusedCfg &f, hipStream_t st) {
    const uint32_t blocks = (s.num + IPW - 1) / IPW;
    if (io.K == 1)
        hipLaunchKernelGGL((step_fused_kernel<IPW, false, kResetSteps, kProfile>), dim3(blocks), dim3(2 * IPW), 0, st,
                           s, r, io, f);
    else
        hipLaunchKernelGGL((step_fused_kernel<IPW, true, kResetSteps, kProfile>), dim3(blocks), dim3(2 * IPW), 0, st,
                           s, r, io, f);
    return hipGetLastError();
}

template <int IPW>
hipError_t launch_ipw(const State &s, const Roms &r, const StepIO &io, const FusedCfg &f, hipStream_t st) {
    if (r.profile)
        return r.w.reset_steps ? launch_variant<IPW, true, true>(s, r, io, f, st)
                               : launch_variant<IPW, false, true>(s, r, io, f, st);
    return r.w.reset_steps ? launch_variant<IPW, true, false>(s, r, io, f, st)
                           : launch_variant<IPW, false, false>(s, r, io, f, st);
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
