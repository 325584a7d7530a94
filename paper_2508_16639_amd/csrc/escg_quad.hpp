// escg_quad.hpp -- branch-free update of four horizontally adjacent 2x2 blocks
// ("a quad": one Philox call) held in LDS.
//
// A quad covers two lattice rows (a = top, c = bottom) and eight columns.
// The two 8-byte row segments are transposed with v_perm into one dword per
// block, B = [A, B, C, D] (top-left, top-right, bottom-left, bottom-right).
// For block word w:
//   * w & 0x38 (von Neumann: bits 3-4 edge, bit 5 orientation) or w & 0x78
//     (Moore: bits 3-5 pair, bit 6 orientation) is the byte offset of an
//     8-byte LDS entry {weights, scatter}: `weights` holds 2*Sp in the byte
//     of the selected cell x and 2 in the byte of its neighbour y (0 in the
//     other two), so v_dot4_u32_u8(B, weights, base) is the address of the
//     pair's rule entry straight from the block dword; the scatter v_perm
//     selector writes (x', y') back into their places and keeps the other
//     two sites.  The 8 (16) entries span 16 (32) dwords, so the 64 lanes'
//     lookups never meet in a bank except on the same dword (a broadcast).
//   * the action is picked by comparing w with thresholds pre-shifted into
//     word space (u = w >> 8 < T  <=>  w <= (T << 8) - 1), which selects
//     one of three rule tables (base);
//   * the pair rule is one LDS lookup: rule[action][x][y] = x' | y' << 8.
// Same species, exchange, selection and reproduction are all table entries,
// so there are no branches and no equality test.
#pragma once

#include "escg_device.hpp"

namespace escg {

// Per-job constants of the quad update (all uniform).  kProb: the job has
// dominance probabilities; a selection then looks up the pair's thresholds
// A, B (LDS tables of Sp*Sp u32 each) and compares v = u - T1 with them:
// v < A the selected cell wins, else v < B the neighbour wins, else nothing.
// Those three outcomes are rule tables 3, 4, 5.
template <bool kProb>
struct QuadCtxT {
    static constexpr bool kProbabilistic = kProb;
    const uint2 *sel;     // LDS: 16 {dot weights, scatter selector}
    uint32_t selmask;     // byte offset of w's entry: w & selmask
    const uint8_t *rule;  // LDS: rule tables, byte addressed
    uint32_t W1, W2;      // word-space thresholds (w <= W1: first table ...)
    uint32_t B1, B2, B3;  // byte offsets of the three rule tables to use
    // kProb only
    const uint8_t *ab;    // LDS: A table, then B table (Sp*Sp u32 each)
    uint32_t boff;        // byte offset of the B table from A
    uint32_t T1;          // selection draws are u = T1 .. T2 - 1
    uint32_t Bsel;        // byte offset of the deterministic selection table
    uint32_t Bo, so;      // outcome tables: Bo + {0, so, 2 so}
};
using QuadCtx = QuadCtxT<false>;

// Host-computed word-space thresholds and table choice for (T1, T2) in
// [0, 2^24]: first = w <= W1 ? B1 : (w <= W2 ? B2 : B3), equivalent to
// exchange if u < T1, selection if u < T2, else reproduction, u = w >> 8.
struct ActionSplit {
    uint32_t W1, W2, a1, a2, a3; // a* = action index 0 ex, 1 sel, 2 rep
};

__host__ __device__ inline ActionSplit split_actions(uint32_t T1, uint32_t T2)
{
    ActionSplit s;
    // w <= (T << 8) - 1 is u < T for T >= 1; T = 0 never holds, so the
    // first comparison then maps to whatever the second one would give.
    if (T1 >= 1) {
        s.W1 = (uint32_t)(((uint64_t)T1 << 8) - 1);
        s.a1 = 0;
    } else {
        s.W1 = 0;
        s.a1 = T2 >= 1 ? 1u : 2u; // w == 0 -> u == 0: selection iff T2 >= 1
    }
    if (T2 >= 1) {
        s.W2 = (uint32_t)(((uint64_t)T2 << 8) - 1);
        s.a2 = 1;
    } else {
        s.W2 = 0;
        s.a2 = 2;
    }
    s.a3 = 2;
    return s;
}

// Builds the selector table (16 entries {weights, scatter}, 128 B) and the
// rule tables
// (3*Sp*Sp u16, plus the three selection outcomes when `prob`: 6*Sp*Sp) in
// LDS with the workgroup's threads.  dom: 32 dominance masks (LDS or
// global).  Entry i = (w >> 3) & 15 of block word w.  Von Neumann: bits 0-1
// of i pick the edge, bit 2 the orientation (entries 8-15 unused).  Moore:
// bits 0-2 pick one of eight pair slots (the four edges, then the diagonals
// (A,D), (B,C) twice each), bit 3 the orientation.
__device__ inline void build_quad_luts(uint2 *sel, uint16_t *rule, uint32_t Sp,
                                       const uint32_t *dom, bool moore,
                                       bool prob = false)
{
    for (uint32_t i = threadIdx.x; i < 16; i += blockDim.x) {
        const uint32_t e = moore ? (i & 7u) : (i & 3u);
        const uint32_t o = moore ? (i >> 3) & 1u : (i >> 2) & 1u;
        // pair sites as byte positions of B = [A, B, C, D]
        const uint32_t f = (e == 0)   ? 0u
                           : (e == 1) ? 2u
                           : (e == 2) ? 0u
                           : (e == 3) ? 1u
                           : (e & 1u) ? 1u   // (B, C)
                                      : 0u;  // (A, D)
        const uint32_t s = (e == 0)   ? 1u
                           : (e == 1) ? 3u
                           : (e == 2) ? 2u
                           : (e == 3) ? 3u
                           : (e & 1u) ? 2u
                                      : 3u;
        const uint32_t cell = o ? s : f, nbr = o ? f : s;
        // rule entry offset (2 * (x * Sp + y)) as a byte dot product
        const uint32_t weights = ((2u * Sp) << (8 * cell)) | (2u << (8 * nbr));
        uint32_t scatter = 0;
        for (uint32_t b = 0; b < 4; ++b) {
            const uint32_t src = (b == cell) ? 4u : (b == nbr) ? 5u : b;
            scatter |= src << (8 * b);
        }
        sel[i] = make_uint2(weights, scatter);
    }
    const uint32_t n = 3 * Sp * Sp;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t a = i / (Sp * Sp), xy = i - a * Sp * Sp;
        uint32_t x = xy / Sp, y = xy - (xy / Sp) * Sp;
        const uint32_t u = a == 0 ? 0u : (a == 1 ? 1u : 2u);
        // evaluate the pair rule with thresholds that force action a
        DomTable dt{dom};
        pair_rule(u, 1u, 2u, dt, x, y);
        rule[i] = (uint16_t)(x | (y << 8));
    }
    if (!prob)
        return;
    // selection outcomes: 3 the selected cell wins, 4 the neighbour wins,
    // 5 nothing; a win needs two different occupied sites
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t a = i / (Sp * Sp), xy = i - a * Sp * Sp;
        uint32_t x = xy / Sp, y = xy - (xy / Sp) * Sp;
        const bool fight = x != y && x != 0 && y != 0;
        if (fight && a == 0)
            y = 0;
        else if (fight && a == 1)
            x = 0;
        rule[n + i] = (uint16_t)(x | (y << 8));
    }
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo,
                                         uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// The selector pair of block word w.
template <class Ctx>
__device__ __forceinline__ uint2 sel_of(uint32_t w, const Ctx &c)
{
    return *reinterpret_cast<const uint2 *>(
        reinterpret_cast<const uint8_t *>(c.sel) + (w & c.selmask));
}

// One block: B = [A, B, C, D] -> updated dword, given the block's selector
// pair s = sel_of(w) (loaded by the caller, so that the lookups of a quad
// can be issued early).
template <class Ctx>
__device__ __forceinline__ uint32_t block_update_sel(uint32_t B, uint32_t w,
                                                     uint2 s, const Ctx &c)
{
    // select values, not lvalues (an lvalue ?: selects addresses and keeps
    // the context in scratch memory)
    const uint32_t b1 = c.B1, b2 = c.B2, b3 = c.B3;
    uint32_t base = (w <= c.W2) ? b2 : b3;
    base = (w <= c.W1) ? b1 : base;
    if constexpr (Ctx::kProbabilistic) {
        // 4 * (x * Sp + y): the pair's A and B entries (u32)
        const uint32_t ai = 2u * __builtin_amdgcn_udot4(B, s.x, 0u, false);
        const uint32_t A = *reinterpret_cast<const uint32_t *>(c.ab + ai);
        const uint32_t Bt =
            *reinterpret_cast<const uint32_t *>(c.ab + c.boff + ai);
        const uint32_t v = (w >> 8) - c.T1;
        const uint32_t so = c.so, zero = 0u;
        const uint32_t o = c.Bo + ((v >= A) ? so : zero) + ((v >= Bt) ? so : zero);
        base = (base == c.Bsel) ? o : base;
    }
    const uint32_t off = __builtin_amdgcn_udot4(B, s.x, base, false);
    const uint32_t out = *reinterpret_cast<const uint16_t *>(c.rule + off);
    return perm(out, B, s.y);
}

template <class Ctx>
__device__ __forceinline__ uint32_t block_update(uint32_t B, uint32_t w,
                                                 const Ctx &c)
{
    return block_update_sel(B, w, sel_of(w, c), c);
}

// The four selector pairs of a quad's words.
struct QuadSel {
    uint2 s[4];
};

template <class Ctx>
__device__ __forceinline__ QuadSel quad_sel(const Words &w, const Ctx &c)
{
    QuadSel q;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        q.s[k] = sel_of(w.w[k], c);
    return q;
}

// The four blocks of a quad (block j = [a(2j), a(2j+1), c(2j), c(2j+1)] of
// its window) updated in place, with the selector pairs already loaded.
template <class Ctx>
__device__ __forceinline__ void quad_blocks_update(uint32_t &b0, uint32_t &b1,
                                                   uint32_t &b2, uint32_t &b3,
                                                   const Words &w,
                                                   const QuadSel &qs,
                                                   const Ctx &c)
{
    b0 = block_update_sel(b0, w.w[0], qs.s[0], c);
    b1 = block_update_sel(b1, w.w[1], qs.s[1], c);
    b2 = block_update_sel(b2, w.w[2], qs.s[2], c);
    b3 = block_update_sel(b3, w.w[3], qs.s[3], c);
}

// Row segments (8 bytes each, little-endian: byte k = column k of the
// segment) -> four updated segments in place, with the selector pairs
// already loaded.
template <class Ctx>
__device__ __forceinline__ void quad_update_sel(uint32_t &a0, uint32_t &a1,
                                                uint32_t &c0, uint32_t &c1,
                                                const Words &w,
                                                const QuadSel &qs,
                                                const Ctx &c)
{
    // transpose: block j = [a(2j), a(2j+1), c(2j), c(2j+1)]
    uint32_t b0 = perm(a0, c0, 0x01000504u);
    uint32_t b1 = perm(a0, c0, 0x03020706u);
    uint32_t b2 = perm(a1, c1, 0x01000504u);
    uint32_t b3 = perm(a1, c1, 0x03020706u);
    quad_blocks_update(b0, b1, b2, b3, w, qs, c);
    // back to rows
    a0 = perm(b1, b0, 0x05040100u);
    c0 = perm(b1, b0, 0x07060302u);
    a1 = perm(b3, b2, 0x05040100u);
    c1 = perm(b3, b2, 0x07060302u);
}

// The same, looking the selector pairs up itself.
template <class Ctx>
__device__ __forceinline__ void quad_update(uint32_t &a0, uint32_t &a1,
                                            uint32_t &c0, uint32_t &c1,
                                            const Words &w, const Ctx &c)
{
    quad_update_sel(a0, a1, c0, c1, w, quad_sel(w, c), c);
}

// Quad whose columns start 8-byte aligned in LDS (offset ox = 0).
template <class Ctx>
__device__ __forceinline__ void quad_even(uint8_t *lat, uint32_t pa,
                                          uint32_t pc, const Words &w,
                                          const Ctx &c)
{
    uint2 ra = *reinterpret_cast<const uint2 *>(lat + pa);
    uint2 rc = *reinterpret_cast<const uint2 *>(lat + pc);
    quad_update(ra.x, ra.y, rc.x, rc.y, w, c);
    *reinterpret_cast<uint2 *>(lat + pa) = ra;
    *reinterpret_cast<uint2 *>(lat + pc) = rc;
}

// Odd-offset quads (ox = 1): the window is columns 1..8 of the aligned
// 8-byte segment at pa (and the same LS further for the bottom row), the
// ninth column being the first of the next segment.  The blocks are built
// straight from the aligned loads, ra / rc = columns 0..7 of the two rows
// and x = (bottom ninth byte) | (top ninth byte) << 16:
//   B0 = [a1 a2 c1 c2], B2 = [a5 a6 c5 c6]  one v_perm each,
//   n = [a4 c4 a7 c7], B1 = [a3 a4 c3 c4], B3 = [a7 a8 c7 c8],
// six v_perm in all (aligning the rows first and transposing them takes
// eight).
__device__ __forceinline__ void odd_blocks(uint2 ra, uint2 rc, uint32_t x,
                                           uint32_t &b0, uint32_t &b1,
                                           uint32_t &b2, uint32_t &b3)
{
    b0 = perm(ra.x, rc.x, 0x02010605u);
    b2 = perm(ra.y, rc.y, 0x02010605u);
    const uint32_t m = perm(ra.x, rc.x, 0x0C0C0307u); // [a3 c3 0 0]
    const uint32_t n = perm(ra.y, rc.y, 0x03070004u); // [a4 c4 a7 c7]
    b1 = perm(n, m, 0x05010400u);
    b3 = perm(x, n, 0x04030602u);
}

// The ninth bytes of an odd quad's two rows as one dword (bottom in byte
// 0, top in byte 2): each byte load fills one half of it.
__device__ __forceinline__ uint32_t odd_ninth(const uint8_t *lat, uint32_t ea,
                                              uint32_t ec)
{
    return (uint32_t)lat[ec] | ((uint32_t)lat[ea] << 16);
}

// Writes an odd quad's updated blocks back as columns 1..8 of the two rows
// (b8 at +1, b16 at +2, b32 at +4, b8 at the ninth byte ea / ec): per row
// one v_perm gives [c1 - c2 c3] (b8 from bits 0-7, b16 from bits 16-31),
// one gives [c5 c6 c8 c7] (the ninth byte from bits 16-23) and one more
// [c4 c5 c6 c7]; six v_perm in all.
__device__ __forceinline__ void odd_store(uint8_t *lat, uint32_t pa,
                                          uint32_t pc, uint32_t ea,
                                          uint32_t ec, uint32_t b0,
                                          uint32_t b1, uint32_t b2,
                                          uint32_t b3)
{
    const uint32_t a1 = perm(b1, b0, 0x04010C00u);  // [a1 - a2 a3]
    const uint32_t a5 = perm(b3, b2, 0x04050100u);  // [a5 a6 a8 a7]
    const uint32_t a4 = perm(a5, b1, 0x07050401u);  // [a4 a5 a6 a7]
    const uint32_t c1 = perm(b1, b0, 0x06030C02u);  // [c1 - c2 c3]
    const uint32_t c5 = perm(b3, b2, 0x06070302u);  // [c5 c6 c8 c7]
    const uint32_t c4 = perm(c5, b1, 0x07050403u);  // [c4 c5 c6 c7]
    lat[pa + 1] = (uint8_t)a1;
    *reinterpret_cast<uint16_t *>(lat + pa + 2) = (uint16_t)(a1 >> 16);
    *reinterpret_cast<uint32_t *>(lat + pa + 4) = a4;
    lat[ea] = (uint8_t)(a5 >> 16);
    lat[pc + 1] = (uint8_t)c1;
    *reinterpret_cast<uint16_t *>(lat + pc + 2) = (uint16_t)(c1 >> 16);
    *reinterpret_cast<uint32_t *>(lat + pc + 4) = c4;
    lat[ec] = (uint8_t)(c5 >> 16);
}

// Quad whose columns start one byte after an 8-byte boundary (ox = 1):
// pa / pc are the aligned addresses, ea / ec the addresses of the ninth byte
// (the column after the 8-byte boundary, possibly wrapped by the caller).
template <class Ctx>
__device__ __forceinline__ void quad_odd(uint8_t *lat, uint32_t pa,
                                         uint32_t pc, uint32_t ea,
                                         uint32_t ec, const Words &w,
                                         const Ctx &c)
{
    const uint2 ra = *reinterpret_cast<const uint2 *>(lat + pa);
    const uint2 rc = *reinterpret_cast<const uint2 *>(lat + pc);
    uint32_t b0, b1, b2, b3;
    odd_blocks(ra, rc, odd_ninth(lat, ea, ec), b0, b1, b2, b3);
    quad_blocks_update(b0, b1, b2, b3, w, quad_sel(w, c), c);
    odd_store(lat, pa, pc, ea, ec, b0, b1, b2, b3);
}

// Load and store halves of quad_even / quad_odd (ox = 0 / 1, uniform), for
// callers that keep the next quad's rows in flight while updating one:
// pa is the aligned LDS offset of the top row, the bottom row is LS further.
struct QuadRows {
    uint32_t a0, a1, c0, c1;
};

__device__ __forceinline__ QuadRows quad_load(const uint8_t *lat, uint32_t pa,
                                              uint32_t LS, uint32_t ox)
{
    const uint2 ra = *reinterpret_cast<const uint2 *>(lat + pa);
    const uint2 rc = *reinterpret_cast<const uint2 *>(lat + pa + LS);
    if (ox == 0)
        return QuadRows{ra.x, ra.y, rc.x, rc.y};
    const uint32_t xa = lat[pa + 8], xc = lat[pa + LS + 8];
    return QuadRows{__builtin_amdgcn_alignbyte(ra.y, ra.x, 1),
                    __builtin_amdgcn_alignbyte(xa, ra.y, 1),
                    __builtin_amdgcn_alignbyte(rc.y, rc.x, 1),
                    __builtin_amdgcn_alignbyte(xc, rc.y, 1)};
}

// A quad of an even-offset pass (ox = 0) read from a copy of the region
// stored one column to the right of 8-byte alignment: its window starts at
// byte -1 of the aligned segment at pa.  The column before the segment is
// byte 3 of the dword at pa - 4.
__device__ __forceinline__ QuadRows quad_load_left(const uint8_t *lat,
                                                   uint32_t pa, uint32_t LS)
{
    const uint2 ra = *reinterpret_cast<const uint2 *>(lat + pa);
    const uint2 rc = *reinterpret_cast<const uint2 *>(lat + pa + LS);
    const uint32_t ya = *reinterpret_cast<const uint32_t *>(lat + pa - 4);
    const uint32_t yc = *reinterpret_cast<const uint32_t *>(lat + pa + LS - 4);
    return QuadRows{__builtin_amdgcn_alignbyte(ra.x, ya, 3),
                    __builtin_amdgcn_alignbyte(ra.y, ra.x, 3),
                    __builtin_amdgcn_alignbyte(rc.x, yc, 3),
                    __builtin_amdgcn_alignbyte(rc.y, rc.x, 3)};
}

__device__ __forceinline__ void quad_store(uint8_t *lat, uint32_t pa,
                                           uint32_t LS, uint32_t ox,
                                           const QuadRows &q)
{
    const uint32_t pc = pa + LS;
    if (ox == 0) {
        *reinterpret_cast<uint2 *>(lat + pa) = make_uint2(q.a0, q.a1);
        *reinterpret_cast<uint2 *>(lat + pc) = make_uint2(q.c0, q.c1);
        return;
    }
    // bytes 1..8 of the window: b8 at +1, b16 at +2, b32 at +4, b8 at +8
    lat[pa + 1] = (uint8_t)q.a0;
    *reinterpret_cast<uint16_t *>(lat + pa + 2) = (uint16_t)(q.a0 >> 8);
    *reinterpret_cast<uint32_t *>(lat + pa + 4) =
        __builtin_amdgcn_alignbyte(q.a1, q.a0, 3);
    lat[pa + 8] = (uint8_t)(q.a1 >> 24);
    lat[pc + 1] = (uint8_t)q.c0;
    *reinterpret_cast<uint16_t *>(lat + pc + 2) = (uint16_t)(q.c0 >> 8);
    *reinterpret_cast<uint32_t *>(lat + pc + 4) =
        __builtin_amdgcn_alignbyte(q.c1, q.c0, 3);
    lat[pc + 8] = (uint8_t)(q.c1 >> 24);
}

// One block addressed site by site (irregular quads: lattice edges with
// wrap inside the quad, or blocks past the row end).
template <class Ctx>
__device__ __forceinline__ void block_bytes(uint8_t *lat, uint32_t pA,
                                            uint32_t pB, uint32_t pC,
                                            uint32_t pD, uint32_t w,
                                            const Ctx &c)
{
    uint32_t B = (uint32_t)lat[pA] | ((uint32_t)lat[pB] << 8) |
                 ((uint32_t)lat[pC] << 16) | ((uint32_t)lat[pD] << 24);
    B = block_update(B, w, c);
    lat[pA] = (uint8_t)B;
    lat[pB] = (uint8_t)(B >> 8);
    lat[pC] = (uint8_t)(B >> 16);
    lat[pD] = (uint8_t)(B >> 24);
}

} // namespace escg
