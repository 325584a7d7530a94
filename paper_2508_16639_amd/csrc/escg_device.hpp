// escg_device.hpp -- device building blocks of the ESCG hot path on gfx950.
//
// Schedule and random-number contract (shared by every kernel here; the
// result of a job is a pure function of it):
//
//   key      = (lo32(seed), hi32(seed)); every draw is one Philox4x32-7
//              block (Salmon et al., SC'11: seven rounds, the fewest with
//              which Philox4x32 passes TestU01's BigCrush) with counter
//              (c0, c1, c2, c3)
//   init     site n = row*L + col: word (n & 3) of counter
//              (n >> 2, 0, kTagInit << 8, replica); value = (w * (S+1)) >> 32
//   offsets  MCS t, pass p: word p of (0, t, kTagOffset << 8, replica);
//              ox = bit 0, oy = bit 1
//   blocks   pass p tiles the lattice into 2x2 blocks with top-left corner
//              (2*by + oy, 2*bx + ox) mod L; block (by, bx) uses word
//              (bx & 3) of counter (by*Q + (bx >> 2), t, (kTagPass << 8) | p,
//              replica), Q = ceil((L/2) / 4) quads per block row
//   word w   edge = (w >> 3) & 3: (A,B), (C,D), (A,C), (B,D) with A
//              top-left, B top-right, C bottom-left, D bottom-right; bit 5
//              set: the second site of the edge is the selected cell (Moore:
//              pair slot (w >> 3) & 7, orientation bit 6); u = w >> 8 is the
//              24-bit action draw: exchange if u < T1, selection if u < T2,
//              else reproduction; the remaining low bits are unused
//
// The pair rule follows the paper's Algorithm "Elementary Step" (same
// species: no change; migration swaps; interaction empties the dominated
// site when both are occupied, the selected cell's win tested first;
// reproduction fills an empty site with the other site's species), with the
// Dominance Check algorithm as a bitmask test.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace escg {

// Rounds of every Philox4x32 draw of the schedule.
constexpr int kPhiloxRounds = 7;

constexpr uint32_t kTagInit = 1u;
constexpr uint32_t kTagOffset = 2u;
constexpr uint32_t kTagPass = 3u;

// Philox4x32 constants (Salmon et al., SC'11, Sec. 4): multipliers and the
// Weyl key increments (golden ratio, sqrt(3) - 1).
constexpr uint32_t kMulA = 0xD2511F53u;
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

struct Words {
    uint32_t w[4];
};

// a ^ b ^ k in one gfx950 instruction (v_bitop3_b32 with truth table 0x96);
// k must be wave-uniform (it is read from a scalar register).
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b,
                                             uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96"
        : "=v"(r)
        : "v"(a), "v"(b), "s"(k));
    return r;
}

// A per-lane (vector register) copy of a wave-uniform value.  The gfx950
// VALU reads at most one scalar operand per instruction, so a select between
// two uniform constants otherwise needs a v_mov of one of them every time;
// copies made once before a loop avoid that.
__device__ __forceinline__ uint32_t vgpr_copy(uint32_t k)
{
    uint32_t r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(k));
    return r;
}

// One Philox round: (c0, c1, c2, c3) with round key (k0, k1).
#define ESCG_PHILOX_ROUND(X0, X1)                                             \
    do {                                                                      \
        const uint64_t pa = (uint64_t)kMulA * c0;                             \
        const uint64_t pb = (uint64_t)kMulB * c2;                             \
        const uint32_t n0 = X0((uint32_t)(pb >> 32), c1, k0);                 \
        const uint32_t n2 = X1((uint32_t)(pa >> 32), c3, k1);                 \
        c1 = (uint32_t)pb;                                                    \
        c3 = (uint32_t)pa;                                                    \
        c0 = n0;                                                              \
        c2 = n2;                                                              \
        k0 += kWeylA;                                                         \
        k1 += kWeylB;                                                         \
    } while (0)

__device__ __forceinline__ uint32_t xor3_c(uint32_t a, uint32_t b, uint32_t k)
{
    return a ^ b ^ k;
}

// The kPhiloxRounds rounds for a counter whose word c0 varies across the
// wave and whose words c1..c3 and key are wave-uniform (all callers here).
// The first rounds are written in C so the compiler keeps their uniform
// parts in scalar registers; from the point where both XOR inputs of a word
// vary across lanes, the three-way XOR is one v_bitop3 instead of two v_xor.
__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, uint32_t k0, uint32_t k1)
{
    static_assert(kPhiloxRounds >= 3, "the first three rounds are unrolled");
    ESCG_PHILOX_ROUND(xor3_c, xor3_c);   // c0 varies; c1..c3 uniform
    ESCG_PHILOX_ROUND(xor3_c, xor3_c);   // c2, c3 vary; c0, c1 uniform
    ESCG_PHILOX_ROUND(xor3_vvs, xor3_c); // c0, c1, c2 vary; c3 uniform
#pragma unroll
    for (int r = 3; r < kPhiloxRounds; ++r)
        ESCG_PHILOX_ROUND(xor3_vvs, xor3_vvs);
    Words o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// What philox() computes from the varying word c0 before the other counter
// words enter: with c1 (the MCS) and c2 (tag and pass) uniform and c3 (the
// replica) and the key fixed for a job, the first round's product of c0
// and the second round's product of the first round's c2 depend on c0, c3
// and k1 only.  A quad visited every pass of every MCS keeps them.
struct PhiloxHead {
    uint32_t h, l; // the second round's product kMulB * c2 (high, low)
    uint32_t y;    // low half of the first round's product kMulA * c0
};

__device__ __forceinline__ PhiloxHead philox_head(uint32_t c0, uint32_t c3,
                                                  uint32_t k1)
{
    const uint64_t pa = (uint64_t)kMulA * c0;
    const uint32_t x = (uint32_t)(pa >> 32) ^ c3 ^ k1; // the first round's c2
    const uint64_t pb = (uint64_t)kMulB * x;
    return PhiloxHead{(uint32_t)(pb >> 32), (uint32_t)pb, (uint32_t)pa};
}

// philox(c0, c1, c2, c3, k0, k1) for hd = philox_head(c0, c3, k1).
__device__ __forceinline__ Words philox_from_head(const PhiloxHead &hd,
                                                  uint32_t c1, uint32_t c2,
                                                  uint32_t k0, uint32_t k1)
{
    static_assert(kPhiloxRounds >= 3, "the first three rounds are unrolled");
    // first round, uniform half: the new c0 and c1
    const uint64_t pb1 = (uint64_t)kMulB * c2;
    const uint32_t u0 = (uint32_t)(pb1 >> 32) ^ c1 ^ k0;
    const uint32_t u1 = (uint32_t)pb1;
    k0 += kWeylA;
    k1 += kWeylB;
    // second round: its product of c0 is uniform, that of c2 is the head's
    const uint64_t pa2 = (uint64_t)kMulA * u0;
    uint32_t c0 = hd.h ^ u1 ^ k0;
    uint32_t c2n = (uint32_t)(pa2 >> 32) ^ hd.y ^ k1;
    c1 = hd.l;
    uint32_t c3 = (uint32_t)pa2;
    c2 = c2n;
    k0 += kWeylA;
    k1 += kWeylB;
    ESCG_PHILOX_ROUND(xor3_vvs, xor3_c); // c0, c1, c2 vary; c3 uniform
#pragma unroll
    for (int r = 3; r < kPhiloxRounds; ++r)
        ESCG_PHILOX_ROUND(xor3_vvs, xor3_vvs);
    Words o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}
#undef ESCG_PHILOX_ROUND

// The same rounds for a counter and key that are uniform across the wave
// (the per-MCS offset draw): plain C, so the compiler keeps every round on
// the scalar unit (s_mul_i32 / s_mul_hi_u32) and the vector unit is free.
__device__ __forceinline__ Words philox_uniform(uint32_t c0, uint32_t c1,
                                                uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < kPhiloxRounds; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Words o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

__device__ __forceinline__ uint32_t pick(const Words &q, uint32_t i)
{
    // i in 0..3; selects between values (not lvalues, whose ?: would select
    // addresses and force the words into scratch memory)
    const uint32_t w0 = q.w[0], w1 = q.w[1], w2 = q.w[2], w3 = q.w[3];
    const uint32_t lo = (i & 1u) ? w1 : w0;
    const uint32_t hi = (i & 1u) ? w3 : w2;
    return (i & 2u) ? hi : lo;
}

// Dominance for S <= 7: bit (a*8 + b) of a 64-bit word set iff a beats b.
struct DomPacked {
    uint64_t bits;
    __device__ __forceinline__ bool beats(uint32_t a, uint32_t b) const
    {
        return (bits >> (((a << 3) | b) & 63u)) & 1u;
    }
};

// Dominance for any S <= 31: per-species bitmasks staged in LDS.
struct DomTable {
    const uint32_t *dom; // 32 entries (LDS)
    __device__ __forceinline__ bool beats(uint32_t a, uint32_t b) const
    {
        return (dom[a & 31u] >> (b & 31u)) & 1u;
    }
};

// The pair rule on (x = selected cell, y = neighbour) for 24-bit draw u.
template <class Dom>
__device__ __forceinline__ void pair_rule(uint32_t u, uint32_t T1, uint32_t T2,
                                          const Dom &d, uint32_t &x,
                                          uint32_t &y)
{
    const uint32_t ox = x, oy = y;
    uint32_t nx = ox, ny = oy;
    if (u < T1) { // exchange
        nx = oy;
        ny = ox;
    } else if (u < T2) { // selection
        const bool diff = ox != oy;
        if (diff && d.beats(ox, oy))
            ny = 0;
        else if (diff && d.beats(oy, ox))
            nx = 0;
    } else { // reproduction
        if (oy == 0)
            ny = ox;
        else if (ox == 0)
            nx = oy;
    }
    x = nx;
    y = ny;
}

// Updates one 2x2 block in LDS.  pA..pD are the LDS byte offsets of the
// block's top-left, top-right, bottom-left and bottom-right sites.  Von
// Neumann: bits 3-4 of w pick the edge, bit 5 the orientation; Moore: bits
// 3-5 pick one of the eight pair slots (edges, then the diagonals (A,D),
// (B,C) twice each), bit 6 the orientation.  ab (global, or null): the
// selection thresholds of a job with dominance probabilities, A at
// [x * Sp + y] and B at [Sp * Sp + x * Sp + y]; a selection draw u then
// compares v = u - T1 with them (v < A: the selected cell wins, else
// v < B: the neighbour wins, else nothing).
template <class Dom>
__device__ __forceinline__ void update_block(uint8_t *lat, uint32_t pA,
                                             uint32_t pB, uint32_t pC,
                                             uint32_t pD, uint32_t w,
                                             uint32_t T1, uint32_t T2,
                                             const Dom &d, bool moore,
                                             const uint32_t *ab = nullptr,
                                             uint32_t Sp = 8)
{
    const uint32_t e = moore ? (w >> 3) & 7u : (w >> 3) & 3u;
    const uint32_t o = moore ? (w >> 6) & 1u : (w >> 5) & 1u;
    // value selects (not lvalue ?:, which would select addresses)
    uint32_t f = (e & 1u) ? pC : pA, s = (e & 1u) ? pD : pB;     // 0, 1
    f = (e == 2) ? pA : (e == 3) ? pB : f;                       // 2, 3
    s = (e == 2) ? pC : (e == 3) ? pD : s;
    f = (e >= 4) ? ((e & 1u) ? pB : pA) : f;                     // 4..7
    s = (e >= 4) ? ((e & 1u) ? pC : pD) : s;
    if (o) {
        const uint32_t t = f;
        f = s;
        s = t;
    }
    uint32_t x = lat[f], y = lat[s];
    const uint32_t u = w >> 8;
    if (ab && u >= T1 && u < T2) {
        if (x != y && x != 0 && y != 0) {
            const uint32_t i = (x & (Sp - 1)) * Sp + (y & (Sp - 1));
            const uint32_t v = u - T1;
            if (v < ab[i])
                y = 0;
            else if (v < ab[Sp * Sp + i])
                x = 0;
        }
    } else {
        pair_rule(u, T1, T2, d, x, y);
    }
    lat[f] = (uint8_t)x;
    lat[s] = (uint8_t)y;
}

// Number of bytes of v that differ from s (valid for byte values < 0x80):
// per byte, (b ^ s) + 0x7F sets bit 7 exactly when b != s, with no carry
// into the next byte.
__device__ __forceinline__ uint32_t bytes_ne(uint32_t v, uint32_t s)
{
    return __popc(((v ^ (s * 0x01010101u)) + 0x7F7F7F7Fu) & 0x80808080u);
}

// Sum over the 64 lanes of a wave, returned to every lane.  DPP adds within
// rows of 16 lanes (row_shr 1, 2, 4, 8 leave each row's sum in its lane 15),
// then row_bcast:15 and row_bcast:31 carry the row sums to lane 63: all VALU,
// no LDS round trips.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Species counting for values 0..7 (densities_kernel): v_perm with the byte
// table {1, 2, 4, ..., 128} maps every byte of a dword to its one-hot code
// (bytes 12, used as padding, map to 0), so the count of species s in the
// dword is popcount(code & (0x01010101 << s)).
constexpr uint32_t kOneHotLo = 0x08040201u; // table bytes 0..3
constexpr uint32_t kOneHotHi = 0x80402010u; // table bytes 4..7

__device__ __forceinline__ uint32_t one_hot_bytes(uint32_t v)
{
    return __builtin_amdgcn_perm(kOneHotHi, kOneHotLo, v);
}

} // namespace escg
