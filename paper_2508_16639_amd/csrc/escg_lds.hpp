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
    uint2 sel[256];               // {gather, scatter} selectors
    uint16_t rule[3 * SP * SP];   // (x', y') per action, x, y
    uint32_t dom[32];             // dominance masks
    uint32_t cnt[64];             // two count rows
    uint32_t misc[4];
};

// Row padding must match no species: for S <= 7 (one-hot counting) it is
// 12, which v_perm maps to a zero byte; above that 0x40, past every species.
__host__ __device__ inline uint8_t pad_byte(uint32_t S)
{
    return S <= 7 ? (uint8_t)12 : (uint8_t)0x40;
}

__host__ __device__ inline uint32_t row_stride(uint32_t L)
{
    return (L + 7) & ~7u;
}

// One MCS (four passes) on an L x L lattice held whole in LDS with row
// stride LS.  Work item = one quad (by, qx); the quad's Philox counter is
// by*Q + qx, the index of the work item.
__device__ __forceinline__ void lds_mcs(uint8_t *lat, uint32_t L, uint32_t LS,
                                        uint32_t t, uint32_t replica,
                                        uint32_t k0, uint32_t k1,
                                        const QuadCtx &qc, uint32_t by0,
                                        uint32_t qx0, uint32_t dby,
                                        uint32_t dqx)
{
    const uint32_t Lb = L >> 1, Q = (Lb + 3) >> 2, nq = Lb * Q;
    const Words off = philox10(0u, t, kTagOffset << 8, replica, k0, k1);
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        const uint32_t ox = off.w[p] & 1u, oy = (off.w[p] >> 1) & 1u;
        const uint32_t ctr2 = (kTagPass << 8) | p;
        uint32_t by = by0, qx = qx0;
        for (uint32_t qi = threadIdx.x; qi < nq; qi += blockDim.x) {
            const Words r = philox10(qi, t, ctr2, replica, k0, k1);
            const uint32_t r0 = 2u * by + oy;
            const uint32_t r1 = (r0 + 1u == L) ? 0u : r0 + 1u;
            const uint32_t rowA = r0 * LS, rowC = r1 * LS;
            const uint32_t col = 8u * qx;
            if (4u * qx + 4u <= Lb) {
                if (ox == 0) {
                    quad_even(lat, rowA + col, rowC + col, r, qc);
                } else {
                    const uint32_t e = (col + 8u == L) ? 0u : col + 8u;
                    quad_odd(lat, rowA + col, rowC + col, rowA + e, rowC + e,
                             r, qc);
                }
            } else {
                // last quad of a row with fewer than four blocks
                for (uint32_t j = 0; j < 4; ++j) {
                    if (4u * qx + j < Lb) {
                        const uint32_t c0 = col + 2u * j + ox;
                        const uint32_t c1 = (c0 + 1u == L) ? 0u : c0 + 1u;
                        block_bytes(lat, rowA + c0, rowA + c1, rowC + c0,
                                    rowC + c1, pick(r, j), qc);
                    }
                }
            }
            qx += dqx;
            by += dby;
            if (qx >= Q) {
                qx -= Q;
                ++by;
            }
        }
        __syncthreads();
    }
}

template <int SP>
__device__ inline QuadCtx make_quad_ctx(const LdsTables<SP> &T, uint32_t T1,
                                        uint32_t T2)
{
    QuadCtx qc;
    qc.sel = T.sel;
    qc.rule = reinterpret_cast<const uint8_t *>(T.rule);
    const ActionSplit a = split_actions(T1, T2);
    qc.W1 = a.W1;
    qc.W2 = a.W2;
    qc.B1 = a.a1 * SP * SP * 2u;
    qc.B2 = a.a2 * SP * SP * 2u;
    qc.B3 = a.a3 * SP * SP * 2u;
    qc.dotw = (2u * SP) | (2u << 8);
    return qc;
}

// Fills the tables of a job (dominance masks from `dom`, global or LDS).
template <int SP>
__device__ inline void setup_tables(LdsTables<SP> &T, const uint32_t *dom)
{
    for (uint32_t i = threadIdx.x; i < 32; i += blockDim.x)
        T.dom[i] = dom[i];
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x)
        T.cnt[i] = 0;
    __syncthreads();
    build_quad_luts(T.sel, T.rule, SP, T.dom);
    __syncthreads();
}

} // namespace escg
