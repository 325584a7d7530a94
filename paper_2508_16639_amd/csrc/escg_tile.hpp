// escg_tile.hpp -- phases of the persistent tiled kernel for large lattices.
//
// The L x L lattice (L % 8 == 0) is cut into TY x TX equal tiles of TH x TW
// sites (TW % 8 == 0, TH even, TH >= 4).  Each workgroup keeps one tile in
// LDS for the whole run, inside a region with a 4-row halo above and below
// and an 8-column halo left and right (8 keeps quads aligned with the
// Philox quads of the global block grid; 4 would do for validity).  During
// one MCS the four passes run over every block of the region; a site's
// value after a pass depends only on its own 2x2 block, so the stale halo
// corrupts at most one more ring of sites per pass and the interior is exact
// after four passes.  Between MCS every tile publishes the 4-row / 8-column
// border strips of its interior into a double-buffered exchange area and
// rebuilds its halo from the eight neighbours' strips.
//
// Region coordinates: LDS row r <-> global row R0 - 4 + r, LDS column c <->
// global column g0 - 8 + c (mod L); row stride LS = TW + 24 (the spare bytes
// cover the ninth byte of odd-offset quads).  Interior = rows [4, TH + 4),
// columns [8, TW + 8).
#pragma once

#include "escg_quad.hpp"

namespace escg {

struct TileGeom {
    uint32_t L, TH, TW, TY, TX;
    __host__ __device__ uint32_t LS() const { return TW + 24; }
    __host__ __device__ uint32_t RH() const { return TH + 8; }
    __host__ __device__ uint32_t region_bytes() const { return RH() * LS(); }
    // exchange slot: top strip (TW dwords), bottom (TW), left (2 TH),
    // right (2 TH)
    __host__ __device__ uint32_t slot_dwords() const
    {
        return 2 * TW + 4 * TH;
    }
};

// Loads the tile's region (interior plus halo) from the global lattice.
__device__ inline void tile_load(uint8_t *lat, const uint8_t *g,
                                 const TileGeom &G, uint32_t ty, uint32_t tx)
{
    const uint32_t L = G.L, LS = G.LS(), R0 = ty * G.TH, g0 = tx * G.TW;
    const uint32_t dwr = (G.TW + 16) >> 2, rows = G.RH();
    for (uint32_t i = threadIdx.x; i < rows * dwr; i += blockDim.x) {
        const uint32_t r = i / dwr, j = i - r * dwr;
        const uint32_t gr = (R0 + L - 4 + r) % L;
        const uint32_t gc = (g0 + L - 8 + 4 * j) % L;
        *reinterpret_cast<uint32_t *>(lat + r * LS + 4 * j) =
            *reinterpret_cast<const uint32_t *>(g + (size_t)gr * L + gc);
    }
    // spare columns (read only by the last odd-offset quad of a row)
    for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x)
        *reinterpret_cast<uint2 *>(lat + r * LS + G.TW + 16) = make_uint2(0, 0);
}

// Stores the interior back to the global lattice.
__device__ inline void tile_store(const uint8_t *lat, uint8_t *g,
                                  const TileGeom &G, uint32_t ty, uint32_t tx)
{
    const uint32_t L = G.L, LS = G.LS(), R0 = ty * G.TH, g0 = tx * G.TW;
    const uint32_t dwr = G.TW >> 2;
    for (uint32_t i = threadIdx.x; i < G.TH * dwr; i += blockDim.x) {
        const uint32_t r = i / dwr, j = i - r * dwr;
        *reinterpret_cast<uint32_t *>(g + (size_t)(R0 + r) * L + g0 + 4 * j) =
            *reinterpret_cast<const uint32_t *>(lat + (r + 4) * LS + 8 +
                                                4 * j);
    }
}

// One MCS over the region: all quads of all block rows, four passes.
__device__ __forceinline__ void tile_mcs(uint8_t *lat, const TileGeom &G,
                                         uint32_t ty, uint32_t tx, uint32_t t,
                                         uint32_t replica, uint32_t k0,
                                         uint32_t k1, const QuadCtx &qc)
{
    const uint32_t L = G.L, LS = G.LS(), Q = L >> 3, Lb = L >> 1;
    const uint32_t NJ = (G.TW + 16) >> 3;        // quads per block row
    const uint32_t qbase = (tx * G.TW) / 8 + Q - 1; // global quad of js = 0
    // global block row of LDS block row k is R0/2 - 2 + k (mod L/2)
    const uint32_t bybase = (ty * G.TH) / 2 + Lb - 2;
    const Words off = philox10(0u, t, kTagOffset << 8, replica, k0, k1);
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        const uint32_t ox = off.w[p] & 1u, oy = (off.w[p] >> 1) & 1u;
        const uint32_t nbr = (G.RH() - oy) >> 1;
        const uint32_t ctr2 = (kTagPass << 8) | p;
        const uint32_t items = nbr * NJ;
        uint32_t k = threadIdx.x / NJ, js = threadIdx.x - k * NJ;
        const uint32_t dk = blockDim.x / NJ, djs = blockDim.x - dk * NJ;
        for (uint32_t i = threadIdx.x; i < items; i += blockDim.x) {
            const uint32_t lr = oy + 2 * k;
            uint32_t by = bybase + k;
            by -= (by >= Lb) ? Lb : 0u;
            by -= (by >= Lb) ? Lb : 0u;
            uint32_t qx = qbase + js;
            qx -= (qx >= Q) ? Q : 0u;
            qx -= (qx >= Q) ? Q : 0u;
            const Words r = philox10(by * Q + qx, t, ctr2, replica, k0, k1);
            const uint32_t pa = lr * LS + 8 * js, pc = pa + LS;
            if (ox == 0)
                quad_even(lat, pa, pc, r, qc);
            else
                quad_odd(lat, pa, pc, pa + 8, pc + 8, r, qc);
            js += djs;
            k += dk;
            if (js >= NJ) {
                js -= NJ;
                ++k;
            }
        }
        __syncthreads();
    }
}

// Device-coherent word store / load for the exchange area: relaxed
// agent-scope atomics compile to sc1 stores and loads, which are coherent
// across XCDs without L2 writeback or invalidation.
__device__ __forceinline__ void xstore(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t xload(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Writes the interior's border strips into exchange slot `slot`.
__device__ inline void tile_publish(const uint8_t *lat, uint32_t *slot,
                                    const TileGeom &G)
{
    const uint32_t LS = G.LS(), TH = G.TH, TW = G.TW, dwr = TW >> 2;
    uint32_t *top = slot, *bot = slot + TW, *left = slot + 2 * TW,
             *right = left + 2 * TH;
    for (uint32_t i = threadIdx.x; i < 4 * dwr; i += blockDim.x) {
        const uint32_t r = i / dwr, j = i - r * dwr;
        xstore(top + i, *reinterpret_cast<const uint32_t *>(
                            lat + (4 + r) * LS + 8 + 4 * j));
        xstore(bot + i, *reinterpret_cast<const uint32_t *>(
                            lat + (TH + r) * LS + 8 + 4 * j));
    }
    for (uint32_t i = threadIdx.x; i < 2 * TH; i += blockDim.x) {
        const uint32_t r = i >> 1, j = i & 1u;
        xstore(left + i, *reinterpret_cast<const uint32_t *>(
                             lat + (4 + r) * LS + 8 + 4 * j));
        xstore(right + i, *reinterpret_cast<const uint32_t *>(
                              lat + (4 + r) * LS + TW + 4 * j));
    }
}

// Rebuilds the halo from the neighbours' strips in their slot `s` (nb:
// base of the exchange area; slot of tile T is nb + (2 T + s) * slot_dwords).
__device__ inline void tile_gather(uint8_t *lat, const uint32_t *nb,
                                   const TileGeom &G, uint32_t ty,
                                   uint32_t tx, uint32_t s)
{
    const uint32_t LS = G.LS(), TH = G.TH, TW = G.TW, dwr = TW >> 2;
    const uint32_t sd = G.slot_dwords();
    const uint32_t up = (ty + G.TY - 1) % G.TY, dn = (ty + 1) % G.TY;
    const uint32_t lf = (tx + G.TX - 1) % G.TX, rt = (tx + 1) % G.TX;
    auto slot = [&](uint32_t y, uint32_t x) {
        return nb + (size_t)(2 * (y * G.TX + x) + s) * sd;
    };
    const uint32_t *sU = slot(up, tx), *sD = slot(dn, tx);
    const uint32_t *sUL = slot(up, lf), *sUR = slot(up, rt);
    const uint32_t *sDL = slot(dn, lf), *sDR = slot(dn, rt);
    const uint32_t *sL = slot(ty, lf), *sR = slot(ty, rt);
    // rows 0..3 from the bottom strips above, rows TH+4.. from top strips below
    const uint32_t wdw = dwr + 4; // dwords per halo row: 2 + dwr + 2
    for (uint32_t i = threadIdx.x; i < 8 * wdw; i += blockDim.x) {
        const uint32_t h = i / wdw, j = i - h * wdw; // h: 0..3 top, 4..7 bottom
        const uint32_t r = h & 3u;
        const bool topside = h < 4;
        const uint32_t lr = topside ? r : TH + 4 + r;
        const uint32_t *mid = topside ? sU + TW : sD;      // bottom / top strip
        const uint32_t *lft = topside ? sUL + TW : sDL;
        const uint32_t *rgt = topside ? sUR + TW : sDR;
        const uint32_t *src;
        if (j < 2)
            src = lft + r * dwr + dwr - 2 + j;
        else if (j < dwr + 2)
            src = mid + r * dwr + j - 2;
        else
            src = rgt + r * dwr + j - 2 - dwr;
        const uint32_t v = xload(src);
        *reinterpret_cast<uint32_t *>(lat + lr * LS + 4 * j) = v;
    }
    // columns 0..7 and TW+8..TW+15 of rows 4..TH+3 from the side strips
    for (uint32_t i = threadIdx.x; i < 4 * TH; i += blockDim.x) {
        const uint32_t side = i / (2 * TH), q = i - side * 2 * TH;
        const uint32_t r = q >> 1, j = q & 1u;
        const uint32_t v = xload(side == 0 ? sL + 2 * TW + 2 * TH + q // right
                                           : sR + 2 * TW + q);         // left
        const uint32_t c = side == 0 ? 4 * j : TW + 8 + 4 * j;
        *reinterpret_cast<uint32_t *>(lat + (4 + r) * LS + c) = v;
    }
}

// Adds the interior's species counts into cnt[0..S] (LDS, zeroed).  SM == 8:
// one-hot byte codes (values 0..7); else byte compares per species.
template <int SM>
__device__ __forceinline__ void tile_count(const uint8_t *lat,
                                           const TileGeom &G, uint32_t S,
                                           uint32_t *cnt)
{
    const uint32_t LS = G.LS(), dwr = G.TW >> 2, n = G.TH * dwr;
    uint32_t c[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s)
        c[s] = 0;
    uint32_t mine = 0;
    uint32_t r = threadIdx.x / dwr, j = threadIdx.x - r * dwr;
    const uint32_t dr = blockDim.x / dwr, dj = blockDim.x - dr * dwr;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(
            lat + (4 + r) * LS + 8 + 4 * j);
        if (SM == 8) {
            const uint32_t h = one_hot_bytes(v);
#pragma unroll
            for (int s = 0; s < SM; ++s)
                if ((uint32_t)s <= S)
                    c[s] += __popc(h & (0x01010101u << s));
        } else {
            ++mine;
#pragma unroll
            for (int s = 0; s < SM; ++s)
                if ((uint32_t)s <= S)
                    c[s] += bytes_ne(v, (uint32_t)s);
        }
        j += dj;
        r += dr;
        if (j >= dwr) {
            j -= dwr;
            ++r;
        }
    }
#pragma unroll
    for (int s = 0; s < SM; ++s) {
        if ((uint32_t)s <= S) {
            const uint32_t tot = wave_sum(SM == 8 ? c[s] : 4u * mine - c[s]);
            if ((threadIdx.x & 63u) == 0 && tot)
                atomicAdd(&cnt[s], tot);
        }
    }
}

} // namespace escg
