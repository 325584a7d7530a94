// escg_lds.hpp -- one Monte Carlo step on a lattice held whole in LDS.
//
// Layout: the tables live in static LDS (LdsTables); the kernel's dynamic
// LDS holds the lattice with row stride LS = L rounded up to 8 (padding
// bytes hold pad_byte(S)).
#pragma once

#include "escg_quad.hpp"

namespace escg {

// Per-workgroup tables in static LDS (their addresses are known at compile
// time, so table lookups need no base-address arithmetic).  SP = 8 serves
// S <= 7 (values 0..7), SP = 32 any S <= 31.
template <int SP>
struct LdsTables {
    uint2 sel[16];                // {weights, scatter} entries, entry
                                  // (w & selmask) / 8 of block word w
    uint32_t selmask;             // 0x38 (von Neumann) or 0x78 (Moore)
    uint16_t rule[6 * SP * SP];   // (x', y') per action (3 used without
                                  // dominance probabilities), x, y
    uint32_t ab[2 * SP * SP];     // selection thresholds A, B per (x, y)
                                  // (jobs with dominance probabilities)
    uint32_t dom[32];             // dominance masks
    uint32_t cnt[64];             // count slots (S <= 7: 8 per linear
                                  // sum) or two count rows (S > 7)
    uint32_t misc[4];
};

// Row padding must match no species: for S <= 7 it is 12, which the v_perm
// code tables of the counts map to a zero byte (the value sum takes off 12
// per padding byte); above that 0x40, past every species.
__host__ __device__ inline uint8_t pad_byte(uint32_t S)
{
    return S <= 7 ? (uint8_t)12 : (uint8_t)0x40;
}

__host__ __device__ inline uint32_t row_stride(uint32_t L)
{
    return (L + 7) & ~7u;
}

// A thread's share of the quads of a lattice held whole in LDS, fixed for
// the job: one quad column qx (Q = ceil(L/8) quads per block row) and the
// block rows by0, by0 + rstep, ... < L/2.  The quad's Philox counter word
// is by * Q + qx, so it and the LDS offset advance by constants.
struct LdsWalk {
    uint32_t by0, rstep;
    uint32_t c0, cstep;   // counter word of the first quad, rstep * Q
    uint32_t pa0, pstep;  // LDS offset of the first quad's top row (oy = 0)
    uint32_t col;         // first byte of the quad in its row: 8 * qx
    uint32_t dnext;       // (column after the quad, wrapped) - col, mod 2^32
    bool active, full;    // full: four blocks (else the row's last quad)
};

__device__ inline LdsWalk lds_walk(uint32_t L, uint32_t LS)
{
    const uint32_t Lb = L >> 1, Q = (Lb + 3) >> 2;
    LdsWalk W;
    W.rstep = min(blockDim.x / Q, Lb);
    W.by0 = threadIdx.x / Q;
    const uint32_t qx = threadIdx.x - W.by0 * Q;
    W.active = W.by0 < W.rstep;
    W.full = 4u * qx + 4u <= Lb;
    W.col = 8u * qx;
    W.dnext = ((W.col + 8u == L) ? 0u : W.col + 8u) - W.col;
    W.c0 = W.by0 * Q + qx;
    W.cstep = W.rstep * Q;
    W.pa0 = 2u * W.by0 * LS + W.col;
    W.pstep = 2u * W.rstep * LS;
    return W;
}

// The Philox heads (philox_head) of a thread's quads, the k-th at block row
// by0 + k * rstep, when a thread has at most kLdsHeads quads (every L when
// blockDim / ceil(L/8) * kLdsHeads >= L/2, e.g. L <= 256 at 512 threads):
// a quad's counter word, the replica and the key are the same every pass of
// every MCS of the job, so the heads are computed once per job.
constexpr uint32_t kLdsHeads = 8;

struct LdsHeads {
    PhiloxHead q[kLdsHeads];
};

__device__ inline bool lds_heads_fit(const LdsWalk &W, uint32_t L)
{
    return W.rstep * kLdsHeads >= (L >> 1);
}

__device__ inline LdsHeads lds_heads(const LdsWalk &W, uint32_t replica,
                                     uint32_t k1)
{
    LdsHeads H;
#pragma unroll
    for (uint32_t k = 0; k < kLdsHeads; ++k)
        H.q[k] = philox_head(W.c0 + k * W.cstep, replica, k1);
    return H;
}

// One quad of pass (ox, oy) at block row by, top row at LDS offset pa.
template <class Ctx>
__device__ __forceinline__ void lds_quad(uint8_t *lat, uint32_t L,
                                         uint32_t LS, const LdsWalk &W,
                                         uint32_t ox, uint32_t oy,
                                         uint32_t by, uint32_t pa,
                                         const Words &r, const Ctx &qc)
{
    const uint32_t Lb = L >> 1;
    // the bottom row of the last block row wraps to row 0
    const uint32_t pc = (oy && by == Lb - 1u) ? W.col : pa + LS;
    if (W.full) {
        if (ox == 0)
            quad_even(lat, pa, pc, r, qc);
        else
            quad_odd(lat, pa, pc, pa + W.dnext, pc + W.dnext, r, qc);
    } else {
        // last quad of a row with fewer than four blocks
        const uint32_t rowA = pa - W.col, rowC = pc - W.col;
        for (uint32_t j = 0; j < 4; ++j) {
            if (W.col / 2u + j < Lb) {
                const uint32_t x0 = W.col + 2u * j + ox;
                const uint32_t x1 = (x0 + 1u == L) ? 0u : x0 + 1u;
                block_bytes(lat, rowA + x0, rowA + x1, rowC + x0, rowC + x1,
                            pick(r, j), qc);
            }
        }
    }
}

// Pass p of MCS t for this thread's quads; w = word p of the MCS's offset
// draw (ox = bit 0, oy = bit 1, uniform).  With heads (kHeads: H holds the
// thread's quads' Philox heads, lds_heads_fit) the draws start from them.
template <bool kHeads = false, class Ctx>
__device__ __forceinline__ void lds_pass(uint8_t *lat, uint32_t L,
                                         uint32_t LS, const LdsWalk &W,
                                         uint32_t w, uint32_t p, uint32_t t,
                                         uint32_t replica, uint32_t k0,
                                         uint32_t k1, const Ctx &qc,
                                         const LdsHeads *H = nullptr)
{
    const uint32_t Lb = L >> 1;
    const uint32_t ox = w & 1u, oy = (w >> 1) & 1u;
    const uint32_t ctr2 = (kTagPass << 8) | p;
    if (!W.active)
        return;
    uint32_t c0 = W.c0, pa = W.pa0 + oy * LS;
    if constexpr (kHeads) {
#pragma unroll
        for (uint32_t k = 0; k < kLdsHeads; ++k) {
            const uint32_t by = W.by0 + k * W.rstep;
            if (by >= Lb)
                break;
            const Words r = philox_from_head(H->q[k], t, ctr2, k0, k1);
            lds_quad(lat, L, LS, W, ox, oy, by, pa, r, qc);
            pa += W.pstep;
        }
    } else {
        for (uint32_t by = W.by0; by < Lb; by += W.rstep) {
            const Words r = philox(c0, t, ctr2, replica, k0, k1);
            lds_quad(lat, L, LS, W, ox, oy, by, pa, r, qc);
            pa += W.pstep;
            c0 += W.cstep;
        }
    }
}

// One MCS (four passes) on an L x L lattice held whole in LDS with row
// stride LS.
template <bool kHeads = false, class Ctx>
__device__ __forceinline__ void lds_mcs(uint8_t *lat, uint32_t L, uint32_t LS,
                                        uint32_t t, uint32_t replica,
                                        uint32_t k0, uint32_t k1,
                                        const Ctx &qc, const LdsWalk &W,
                                        const LdsHeads *H = nullptr)
{
    const Words off =
        philox_uniform(0u, t, kTagOffset << 8, replica, k0, k1);
    // a loop, not unrolled: with the heads the pass body holds kLdsHeads
    // quads, and four copies of it would not be inlined (p picks its word by
    // selects, not by indexing, which would keep the words in scratch)
#pragma unroll 1
    for (uint32_t p = 0; p < 4; ++p) {
        const uint32_t wp = p == 0   ? off.w[0]
                            : p == 1 ? off.w[1]
                            : p == 2 ? off.w[2]
                                     : off.w[3];
        lds_pass<kHeads>(lat, L, LS, W, __builtin_amdgcn_readfirstlane(wp), p,
                         t, replica, k0, k1, qc, H);
        __syncthreads();
    }
}

template <bool kProb = false, int SP>
__device__ inline QuadCtxT<kProb> make_quad_ctx(const LdsTables<SP> &T,
                                                uint32_t T1, uint32_t T2)
{
    QuadCtxT<kProb> qc;
    qc.sel = T.sel;
    qc.selmask = T.selmask;
    qc.rule = reinterpret_cast<const uint8_t *>(T.rule);
    const ActionSplit a = split_actions(T1, T2);
    const uint32_t tb = SP * SP * 2u; // bytes per rule table
    qc.W1 = a.W1;
    qc.W2 = a.W2;
    qc.B1 = a.a1 * tb;
    qc.B2 = a.a2 * tb;
    qc.B3 = a.a3 * tb;
    qc.B2 = vgpr_copy(qc.B2); // the selects in block_update read B2, B3
    qc.B3 = vgpr_copy(qc.B3); // as vector operands
    qc.ab = reinterpret_cast<const uint8_t *>(T.ab);
    qc.boff = SP * SP * 4u;
    qc.T1 = T1;
    qc.Bsel = 1u * tb;
    qc.Bo = 3u * tb;
    qc.so = tb;
    return qc;
}

// Fills the tables of a job (dominance masks from `dom`, global or LDS;
// `moore`: the 8-way neighbourhood's pair slots; `ab`: the selection
// thresholds A, B (2 * SP * SP u32, global) of a job with dominance
// probabilities, else null).
template <int SP>
__device__ inline void setup_tables(LdsTables<SP> &T, const uint32_t *dom,
                                    bool moore, const uint32_t *ab = nullptr)
{
    for (uint32_t i = threadIdx.x; i < 32; i += blockDim.x)
        T.dom[i] = dom[i];
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x)
        T.cnt[i] = 0;
    if (threadIdx.x == 0)
        T.selmask = moore ? 0x78u : 0x38u;
    if (ab)
        for (uint32_t i = threadIdx.x; i < 2 * SP * SP; i += blockDim.x)
            T.ab[i] = ab[i];
    __syncthreads();
    build_quad_luts(T.sel, T.rule, SP, T.dom, moore, ab != nullptr);
    __syncthreads();
}

} // namespace escg
