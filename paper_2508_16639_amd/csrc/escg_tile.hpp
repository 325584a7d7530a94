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
// rebuilds its halo from the eight neighbours' strips, which carry a tag bit
// that tells fresh words from stale ones.
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
    // (r, j) advance by (dr, dj) with a carry: no division in the loop; the
    // global row R0 - 4 + r and column g0 - 8 + 4 j lie in (-8, L + 8), so
    // adding L and subtracting it at most twice wraps them
    uint32_t r = threadIdx.x / dwr, j = threadIdx.x - r * dwr;
    const uint32_t dr = blockDim.x / dwr, dj = blockDim.x - dr * dwr;
    for (uint32_t i = threadIdx.x; i < rows * dwr; i += blockDim.x) {
        uint32_t gr = R0 + L - 4 + r;
        gr = min(gr, gr - L);
        gr = min(gr, gr - L);
        uint32_t gc = g0 + L - 8 + 4 * j;
        gc = min(gc, gc - L);
        gc = min(gc, gc - L);
        *reinterpret_cast<uint32_t *>(lat + r * LS + 4 * j) =
            *reinterpret_cast<const uint32_t *>(g + (size_t)gr * L + gc);
        j += dj;
        r += dr;
        if (j >= dwr) {
            j -= dwr;
            ++r;
        }
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
    uint32_t r = threadIdx.x / dwr, j = threadIdx.x - r * dwr;
    const uint32_t dr = blockDim.x / dwr, dj = blockDim.x - dr * dwr;
    for (uint32_t i = threadIdx.x; i < G.TH * dwr; i += blockDim.x) {
        *reinterpret_cast<uint32_t *>(g + (size_t)(R0 + r) * L + g0 + 4 * j) =
            *reinterpret_cast<const uint32_t *>(lat + (r + 4) * LS + 8 +
                                                4 * j);
        j += dj;
        r += dr;
        if (j >= dwr) {
            j -= dwr;
            ++r;
        }
    }
}

// A thread's share of the region's quads, fixed for the whole run: one quad
// column js and the block rows r0, r0 + rstep, ... .  The global block row
// of LDS block row k is R0/2 - 2 + k (mod L/2) and the global quad column
// of js is g0/8 - 1 + js (mod L/8), for either offset, so the Philox counter
// word c0 = by * Q + qx of the first quad and its LDS offset advance by
// constants (one wrap test for c0 because rstep <= L/2).
struct TileWalk {
    uint32_t c0;     // counter word of the first quad
    uint32_t pa0;    // LDS offset of its top row for oy = 0
    uint32_t r0;     // first block row
    uint32_t rstep;  // block rows per step
    uint32_t cstep;  // rstep * Q
    uint32_t pstep;  // 2 * rstep * LS
    uint32_t wrap;   // (L/2) * Q counter words per pass
    bool active;
};

__device__ inline TileWalk tile_walk(const TileGeom &G, uint32_t ty,
                                     uint32_t tx)
{
    const uint32_t L = G.L, LS = G.LS(), Q = L >> 3, Lb = L >> 1;
    const uint32_t NJ = (G.TW + 16) >> 3; // quads per block row
    TileWalk W;
    W.rstep = min(blockDim.x / NJ, Lb);
    W.r0 = threadIdx.x / NJ;
    const uint32_t js = threadIdx.x - W.r0 * NJ;
    W.active = W.r0 < W.rstep;
    const uint32_t qx = ((tx * G.TW) / 8 + Q - 1 + js) % Q;
    const uint32_t by = ((ty * G.TH) / 2 + Lb - 2 + W.r0) % Lb;
    W.c0 = by * Q + qx;
    W.pa0 = 2 * W.r0 * LS + 8 * js;
    W.cstep = W.rstep * Q;
    W.pstep = 2 * W.rstep * LS;
    W.wrap = Lb * Q;
    return W;
}

// Threads for a tile: enough quad columns times rows per step that the
// block rows split into equal numbers of steps (at most 1024).
__host__ __device__ inline uint32_t tile_threads(const TileGeom &G,
                                                 uint32_t cap)
{
    const uint32_t NJ = (G.TW + 16) >> 3, nbr = G.RH() >> 1;
    uint32_t maxr = cap / NJ;
    if (maxr == 0)
        return 0;
    const uint32_t steps = (nbr + maxr - 1) / maxr;
    const uint32_t rows = (nbr + steps - 1) / steps;
    const uint32_t nt = (rows * NJ + 63) / 64 * 64;
    return nt < cap ? nt : cap;
}

// Pass p of MCS t for this thread's quads; w = word p of the MCS's offset
// draw (ox = bit 0, oy = bit 1, uniform).
template <class Ctx>
__device__ __forceinline__ void tile_pass(uint8_t *lat, const TileGeom &G,
                                          const TileWalk &W, uint32_t w,
                                          uint32_t p, uint32_t t,
                                          uint32_t replica, uint32_t k0,
                                          uint32_t k1, const Ctx &qc)
{
    const uint32_t LS = G.LS();
    const uint32_t ox = w & 1u, oy = (w >> 1) & 1u;
    const uint32_t nbr = (G.RH() - oy) >> 1;
    const uint32_t ctr2 = (kTagPass << 8) | p;
    if (!W.active)
        return;
    uint32_t c0 = W.c0, pa = W.pa0 + oy * LS;
    if (ox == 0) {
        for (uint32_t k = W.r0; k < nbr; k += W.rstep) {
            const Words r = philox(c0, t, ctr2, replica, k0, k1);
            quad_even(lat, pa, pa + LS, r, qc);
            pa += W.pstep;
            c0 += W.cstep;
            c0 = min(c0, c0 - W.wrap);
        }
    } else {
        for (uint32_t k = W.r0; k < nbr; k += W.rstep) {
            const Words r = philox(c0, t, ctr2, replica, k0, k1);
            quad_odd(lat, pa, pa + LS, pa + 8, pa + LS + 8, r, qc);
            pa += W.pstep;
            c0 += W.cstep;
            c0 = min(c0, c0 - W.wrap);
        }
    }
}

// One MCS over the region: all quads of all block rows, four passes.
template <class Ctx>
__device__ __forceinline__ void tile_mcs(uint8_t *lat, const TileGeom &G,
                                         const TileWalk &W, uint32_t t,
                                         uint32_t replica, uint32_t k0,
                                         uint32_t k1, const Ctx &qc)
{
    const Words off =
        philox_uniform(0u, t, kTagOffset << 8, replica, k0, k1);
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        tile_pass(lat, G, W, __builtin_amdgcn_readfirstlane(off.w[p]), p, t,
                  replica, k0, k1, qc);
        __syncthreads();
    }
}

// Balanced alternative to TileWalk when a pass has at most kListSlots *
// blockDim quads: quad q = tid + i * blockDim (i < kListSlots) in row-major
// order over (LDS block row, quad column), so every wave of the workgroup
// gets the same number of quads up to one, and with 1024 threads the four
// SIMDs of the CU get equal shares (a column walk leaves the SIMD that
// holds one wave fewer idle for a quarter of each pass).  A thread keeps
// the LDS offset (oy = 0) and the Philox counter word of each of its quads;
// a pass with oy = 1 has one block row fewer and skips the quads of the
// last row.
constexpr uint32_t kListSlots = 3;

struct TileList {
    uint32_t pa[kListSlots];
    uint32_t c0[kListSlots];
};

__host__ __device__ inline bool tile_list_fits(const TileGeom &G,
                                               uint32_t threads)
{
    return (G.RH() >> 1) * ((G.TW + 16) >> 3) <= kListSlots * threads;
}

__device__ inline TileList tile_list(const TileGeom &G, uint32_t ty,
                                     uint32_t tx)
{
    const uint32_t L = G.L, LS = G.LS(), Q = L >> 3, Lb = L >> 1;
    const uint32_t NJ = (G.TW + 16) >> 3;
    const uint32_t bx = (tx * G.TW) / 8 + Q - 1, by = (ty * G.TH) / 2 + Lb - 2;
    TileList T;
#pragma unroll
    for (uint32_t i = 0; i < kListSlots; ++i) {
        const uint32_t q = threadIdx.x + i * blockDim.x;
        const uint32_t row = q / NJ, col = q - row * NJ;
        T.pa[i] = 2 * row * LS + 8 * col;
        T.c0[i] = ((by + row) % Lb) * Q + (bx + col) % Q;
    }
    return T;
}

// The list walk keeps two copies of the region in LDS: buffer 0 (column c
// of row r at r * LS + c, as every other phase uses it) and buffer 1, the
// same one column to the right of 8-byte alignment (column c at byte
// r * LS + c - 1 of `lat1`), so that the windows of odd-offset quads
// (columns 8j+1 .. 8j+8) are aligned there.  A pass reads the buffer the
// previous pass wrote and writes the buffer in which its own windows are
// aligned (buffer ox), except that the last pass of an MCS writes buffer 0
// for the halo exchange.  Every write of a pass but that one is then an
// aligned 8-byte store; only reads after a change of parity (and the last
// pass when odd) are misaligned.  A pass that changes buffers leaves the
// cells its quads do not cover (column 0 when ox = 1, the first and last
// rows when oy = 1) stale in the buffer it writes.  That cannot reach the
// tile's interior: a block update moves information by one cell per pass,
// so a value left at the region's edge after pass p (0..3) of an MCS moves
// at most 3 - p cells inward before the MCS ends, and the halo (4 rows, 8
// columns) is gathered anew after every MCS.  The interior, the counts and
// the published border strips are those of an in-place pass, byte for
// byte.
//
// The Philox words and selector pairs of slot i + 1 are computed and loaded
// before slot i is updated, so the selector lookups are in flight during
// the update (prefetching the rows too measured no faster and needs more
// registers than the 1024-thread launch allows without spills).  Those of
// slot 0 arrive in (rf, sf), and the pass leaves the next pass's there
// before its barrier (the selector table is constant, the words depend on
// the counter only).
template <bool kOdd, bool kSrc1, bool kDst1, class Ctx>
__device__ __forceinline__ void tile_pass_list_db(uint8_t *lat, uint8_t *lat1,
                                                  const TileGeom &G,
                                                  const TileList &T,
                                                  uint32_t w, uint32_t p,
                                                  uint32_t t,
                                                  uint32_t replica,
                                                  uint32_t k0, uint32_t k1,
                                                  const Ctx &qc, Words &rf,
                                                  QuadSel &sf)
{
    const uint32_t LS = G.LS();
    const uint32_t oy = (w >> 1) & 1u;
    const uint32_t nq = ((G.RH() - oy) >> 1) * ((G.TW + 16) >> 3);
    const uint32_t ctr2 = (kTagPass << 8) | p, dy = oy * LS;
    const uint8_t *src = kSrc1 ? lat1 : lat;
    uint8_t *dst = kDst1 ? lat1 : lat;
    bool v[kListSlots];
    QuadRows q[kListSlots];
    Words r[kListSlots];
    QuadSel qs[kListSlots];
#pragma unroll
    for (uint32_t i = 0; i < kListSlots; ++i)
        v[i] = threadIdx.x + i * blockDim.x < nq;
    // the waves with a quad in every slot issue first (wave priority), so
    // that the waves of a SIMD reach the pass barrier closer together
    if (v[kListSlots - 1])
        __builtin_amdgcn_s_setprio(1);
    r[0] = rf;
    qs[0] = sf;
#pragma unroll
    for (uint32_t i = 0; i < kListSlots; ++i) {
        const uint32_t pa = T.pa[i] + dy;
        if (v[i]) {
            if (kOdd == kSrc1) // aligned in the source buffer
                q[i] = quad_load(src, pa, LS, 0u);
            else if (kOdd) // buffer 0, window at +1
                q[i] = quad_load(src, pa, LS, 1u);
            else // buffer 1, window at -1
                q[i] = quad_load_left(src, pa, LS);
        }
        if (i + 1 < kListSlots && v[i + 1]) {
            r[i + 1] = philox(T.c0[i + 1], t, ctr2, replica, k0, k1);
            qs[i + 1] = quad_sel(r[i + 1], qc);
        }
        if (v[i]) {
            quad_update_sel(q[i].a0, q[i].a1, q[i].c0, q[i].c1, r[i], qs[i],
                            qc);
            // aligned unless an odd pass writes buffer 0
            quad_store(dst, pa, LS, (kOdd && !kDst1) ? 1u : 0u, q[i]);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (p < 3) { // the next pass's first slot, before the barrier
        rf = philox(T.c0[0], t, (kTagPass << 8) | (p + 1), replica, k0, k1);
        sf = quad_sel(rf, qc);
    }
}

// One pass of the list walk with word w (offsets), the lattice in buffer 1
// when cur1; returns where the pass left it.  lat1: buffer 1 as above (an
// 8-aligned address, RH * LS bytes from byte -1 on).
template <class Ctx>
__device__ __forceinline__ bool tile_pass_list(uint8_t *lat, uint8_t *lat1,
                                               const TileGeom &G,
                                               const TileList &T, uint32_t w,
                                               uint32_t p, bool cur1,
                                               uint32_t t, uint32_t replica,
                                               uint32_t k0, uint32_t k1,
                                               const Ctx &qc, Words &rf,
                                               QuadSel &sf)
{
    const bool odd = w & 1u, dst1 = odd && p < 3;
#define ESCG_PASS(O, S1, D1)                                                  \
    tile_pass_list_db<O, S1, D1>(lat, lat1, G, T, w, p, t, replica, k0, k1,  \
                                 qc, rf, sf)
    if (!odd)
        cur1 ? ESCG_PASS(false, true, false) : ESCG_PASS(false, false, false);
    else if (dst1)
        cur1 ? ESCG_PASS(true, true, true) : ESCG_PASS(true, false, true);
    else
        cur1 ? ESCG_PASS(true, true, false) : ESCG_PASS(true, false, false);
#undef ESCG_PASS
    return dst1;
}

// One MCS of the list walk; the lattice is in buffer 0 before and after.
template <class Ctx>
__device__ __forceinline__ void tile_mcs_list(uint8_t *lat, uint8_t *lat1,
                                              const TileGeom &G,
                                              const TileList &T, uint32_t t,
                                              uint32_t replica, uint32_t k0,
                                              uint32_t k1, const Ctx &qc)
{
    const Words off =
        philox_uniform(0u, t, kTagOffset << 8, replica, k0, k1);
    Words rf = philox(T.c0[0], t, kTagPass << 8, replica, k0, k1);
    QuadSel sf = quad_sel(rf, qc); // slot 0 of pass 0
    bool cur1 = false;
    // unrolled (the passes then know p, and pass 0 reads buffer 0): 3.5 %
    // faster than one copy of each kind of pass in a loop, at 14 copies
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        const uint32_t wp = __builtin_amdgcn_readfirstlane(off.w[p]);
        cur1 = tile_pass_list(lat, lat1, G, T, wp, p, cur1, t, replica, k0,
                              k1, qc, rf, sf);
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

// Exchange area: two slots per tile, slot s of tile T at dword
// (s * tiles + T) * slot_dwords.  The strips published after the tile's
// e-th MCS of a launch go to slot e & 1, every byte carrying the tag bit
// ((e >> 1) & 1) in bit 7 (species values stay below 0x80).  A reader
// therefore recognises fresh data word by word, with no separate flag, and
// a slot's previous content (from MCS e - 2) always carries the other tag.
// Before the first MCS, slot 0 holds tag 0 and slot 1 tag 1, which the
// first use of each slot (e = 2, tag 1; e = 1, tag 0) does not match.
__host__ __device__ inline uint32_t exch_slot(uint32_t e) { return e & 1u; }
__host__ __device__ inline uint32_t exch_tag(uint32_t e)
{
    return ((e >> 1) & 1u) ? 0x80808080u : 0u;
}

// Writes the interior's border strips, tagged with `tag` (0 or 0x80808080),
// into one exchange slot.
__device__ inline void tile_publish(const uint8_t *lat, uint32_t *slot,
                                    const TileGeom &G, uint32_t tag)
{
    const uint32_t LS = G.LS(), TH = G.TH, TW = G.TW, dwr = TW >> 2;
    uint32_t *top = slot, *bot = slot + TW, *left = slot + 2 * TW,
             *right = left + 2 * TH;
    for (uint32_t i = threadIdx.x; i < 4 * dwr; i += blockDim.x) {
        const uint32_t r = i / dwr, j = i - r * dwr;
        xstore(top + i, tag | *reinterpret_cast<const uint32_t *>(
                                  lat + (4 + r) * LS + 8 + 4 * j));
        xstore(bot + i, tag | *reinterpret_cast<const uint32_t *>(
                                  lat + (TH + r) * LS + 8 + 4 * j));
    }
    for (uint32_t i = threadIdx.x; i < 2 * TH; i += blockDim.x) {
        const uint32_t r = i >> 1, j = i & 1u;
        xstore(left + i, tag | *reinterpret_cast<const uint32_t *>(
                                   lat + (4 + r) * LS + 8 + 4 * j));
        xstore(right + i, tag | *reinterpret_cast<const uint32_t *>(
                                    lat + (4 + r) * LS + TW + 4 * j));
    }
}

// Halo word i of the region (i < 8 * (TW/4 + 4) + 4 * TH): its source in the
// neighbours' slot `s` and its LDS destination.
struct HaloWord {
    const uint32_t *src;
    uint32_t dst;
};

struct HaloMap {
    const uint32_t *sU, *sD, *sUL, *sUR, *sDL, *sDR, *sL, *sR;
    uint32_t LS, TH, TW, dwr, wdw;

    __device__ HaloMap(const uint32_t *nb, const TileGeom &G, uint32_t ty,
                       uint32_t tx, uint32_t s)
    {
        LS = G.LS();
        TH = G.TH;
        TW = G.TW;
        dwr = TW >> 2;
        wdw = dwr + 4; // dwords per halo row: 2 + dwr + 2
        const uint32_t sd = G.slot_dwords(), T = G.TY * G.TX;
        const uint32_t up = (ty + G.TY - 1) % G.TY, dn = (ty + 1) % G.TY;
        const uint32_t lf = (tx + G.TX - 1) % G.TX, rt = (tx + 1) % G.TX;
        const uint32_t *base = nb + (size_t)s * T * sd;
        auto slot = [&](uint32_t y, uint32_t x) {
            return base + (size_t)(y * G.TX + x) * sd;
        };
        sU = slot(up, tx);
        sD = slot(dn, tx);
        sUL = slot(up, lf);
        sUR = slot(up, rt);
        sDL = slot(dn, lf);
        sDR = slot(dn, rt);
        sL = slot(ty, lf);
        sR = slot(ty, rt);
    }
    __device__ uint32_t count() const { return 8 * wdw + 4 * TH; }
    __device__ HaloWord at(uint32_t i) const
    {
        HaloWord w;
        if (i < 8 * wdw) {
            // rows 0..3 from the bottom strips of the tiles above, rows
            // TH+4.. from the top strips of the tiles below
            const uint32_t h = i / wdw, j = i - h * wdw;
            const uint32_t r = h & 3u;
            const bool topside = h < 4;
            const uint32_t lr = topside ? r : TH + 4 + r;
            const uint32_t *mid = topside ? sU + TW : sD;
            const uint32_t *lft = topside ? sUL + TW : sDL;
            const uint32_t *rgt = topside ? sUR + TW : sDR;
            if (j < 2)
                w.src = lft + r * dwr + dwr - 2 + j;
            else if (j < dwr + 2)
                w.src = mid + r * dwr + j - 2;
            else
                w.src = rgt + r * dwr + j - 2 - dwr;
            w.dst = lr * LS + 4 * j;
        } else {
            // columns 0..7 and TW+8..TW+15 of rows 4..TH+3 from the right
            // strip of the left neighbour and the left strip of the right one
            const uint32_t k = i - 8 * wdw;
            const uint32_t side = k / (2 * TH), q = k - side * 2 * TH;
            const uint32_t r = q >> 1, j = q & 1u;
            w.src = side == 0 ? sL + 2 * TW + 2 * TH + q : sR + 2 * TW + q;
            w.dst = (4 + r) * LS + (side == 0 ? 4 * j : TW + 8 + 4 * j);
        }
        return w;
    }
};

// Polls one exchange word until it carries `tag` (bit 7 of its low byte).
// Returns 0 with the word in v, 1 if another workgroup raised the abort
// word, 2 after spin_limit polls.
__device__ __forceinline__ uint32_t await_word(const uint32_t *src,
                                               uint32_t tag, uint32_t &v,
                                               const uint32_t *abort,
                                               uint32_t spin_limit)
{
    uint32_t spins = 0;
    while ((v ^ tag) & 0x80u) {
        if ((++spins & 63u) == 0) {
            if (xload(abort))
                return 1;
            if (spins > spin_limit)
                return 2;
        }
        __builtin_amdgcn_s_sleep(1);
        v = xload(src);
    }
    return 0;
}

// A thread's first two halo words (i = tid and tid + blockDim), fixed for
// the run: dword offsets of their sources from the start of exchange slot 0
// and their LDS destinations.  Later words (only when the halo has more than
// 2 * blockDim words) are mapped on the fly.
struct HaloPlan {
    uint32_t n;            // halo words
    uint32_t src_a, src_b; // dword offsets into slot 0
    uint32_t dst_a, dst_b; // LDS byte offsets
};

__device__ inline HaloPlan halo_plan(const uint32_t *nb, const TileGeom &G,
                                     uint32_t ty, uint32_t tx)
{
    const HaloMap M(nb, G, ty, tx, 0);
    HaloPlan P;
    P.n = M.count();
    const uint32_t i = threadIdx.x, bd = blockDim.x;
    const HaloWord a = M.at(i < P.n ? i : 0), b = M.at(i + bd < P.n ? i + bd : 0);
    P.src_a = (uint32_t)(a.src - nb);
    P.src_b = (uint32_t)(b.src - nb);
    P.dst_a = a.dst;
    P.dst_b = b.dst;
    return P;
}

// Rebuilds the halo from the neighbours' strips in exchange slot `s`
// (dword offset s_off = s * tiles * slot_dwords) once they carry `tag`.
// Each thread keeps two words in flight; `between()` runs after the first
// loads are issued and before they are awaited (every thread calls it
// exactly once, so it may contain wave-wide operations), which hides the
// load latency behind other work.  Returns the worst await_word status of
// this thread (0 = all words arrived).
template <class Fn>
__device__ inline uint32_t tile_gather(uint8_t *lat, const uint32_t *nb,
                                       const HaloPlan &P, const TileGeom &G,
                                       uint32_t ty, uint32_t tx,
                                       uint32_t s_off, uint32_t tag,
                                       const uint32_t *abort,
                                       uint32_t spin_limit, Fn &&between)
{
    const uint32_t n = P.n, bd = blockDim.x;
    uint32_t i = threadIdx.x;
    bool one = i < n, two = i + bd < n;
    const uint32_t *sa = nb + s_off + P.src_a, *sb = nb + s_off + P.src_b;
    uint32_t da = P.dst_a, db = P.dst_b;
    uint32_t va = one ? xload(sa) : 0u;
    uint32_t vb = two ? xload(sb) : 0u;
    between();
    uint32_t status = 0;
    while (one) {
        status = await_word(sa, tag, va, abort, spin_limit);
        if (!status && two)
            status = await_word(sb, tag, vb, abort, spin_limit);
        if (status)
            break;
        *reinterpret_cast<uint32_t *>(lat + da) = va & 0x7F7F7F7Fu;
        if (two)
            *reinterpret_cast<uint32_t *>(lat + db) = vb & 0x7F7F7F7Fu;
        i += 2 * bd;
        one = i < n;
        two = i + bd < n;
        if (one) {
            const HaloMap M(nb + s_off, G, ty, tx, 0);
            const HaloWord a = M.at(i);
            sa = a.src;
            da = a.dst;
            va = xload(sa);
            if (two) {
                const HaloWord b = M.at(i + bd);
                sb = b.src;
                db = b.dst;
                vb = xload(sb);
            }
        }
    }
    return status;
}

__device__ inline uint32_t tile_gather(uint8_t *lat, const uint32_t *nb,
                                       const TileGeom &G, uint32_t ty,
                                       uint32_t tx, uint32_t s, uint32_t tag,
                                       const uint32_t *abort,
                                       uint32_t spin_limit)
{
    const HaloPlan P = halo_plan(nb, G, ty, tx);
    return tile_gather(lat, nb, P, G, ty, tx,
                       s * G.TY * G.TX * G.slot_dwords(), tag, abort,
                       spin_limit, [] {});
}

// Species counts of the interior, S > 7: byte compares per species, added
// into cnt[0..S] (LDS, zeroed).  A thread walks one column of dwords down the
// rows (rstep rows apart), so its LDS address advances by a constant.
__device__ __forceinline__ void tile_count_wide(const uint8_t *lat,
                                                const TileGeom &G, uint32_t S,
                                                uint32_t *cnt)
{
    constexpr int SM = 32;
    const uint32_t LS = G.LS(), dwr = G.TW / 4;
    const uint32_t rstep = blockDim.x / dwr; // >= 1: TW / 4 <= blockDim
    const uint32_t r0 = threadIdx.x / dwr, j = threadIdx.x - r0 * dwr;
    uint32_t c[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s)
        c[s] = 0;
    uint32_t mine = 0;
    if (r0 < rstep) {
        const uint8_t *p = lat + (4 + r0) * LS + 8 + 4 * j;
        for (uint32_t r = r0; r < G.TH; r += rstep, p += rstep * LS) {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
            ++mine;
#pragma unroll
            for (int s = 0; s < SM; ++s)
                if ((uint32_t)s <= S)
                    c[s] += bytes_ne(v, (uint32_t)s);
        }
    }
#pragma unroll
    for (int s = 0; s < SM; ++s) {
        if ((uint32_t)s <= S) {
            const uint32_t tot = wave_sum(4u * mine - c[s]);
            if ((threadIdx.x & 63u) == 0 && tot)
                atomicAdd(&cnt[s], tot);
        }
    }
}

// Species counts of the interior, S <= 7 (site values 0..7), without one
// popcount or reduction per species.  With NS = 4, 6 or 8 states covering
// 0..S, the interior's counts n_s follow from NS - 1 linear sums:
//   q = 0 .. NS-3: n_{q+1} (species 1 .. NS-2),
//   q = NS-2:      V = sum of the site values,
// then n_{NS-1} = (V - sum_{s=1}^{NS-2} s n_s) / (NS - 1) (exact) and
// n_0 = sites - sum_{s>=1} n_s.
// Species 2p+1 and 2p+2 share one v_perm code table (value 2p+1 -> 0x01,
// 2p+2 -> 0x10, other values -> 0): summed bytewise, the low nibbles of the
// codes count species 2p+1 and the high nibbles 2p+2, and v_dot8_u32_u4
// adds up either set of nibbles.  V is summed bytewise too (v_add3), then
// by v_dot4.  A nibble gains at most 2 per row (two dwords per row), so rows
// are taken in groups of at most 7; a V byte stays below 7 * 14.
// Each thread walks one column of dword pairs (as tile_count_wide, eight
// sites per row) and adds its NS - 1 sums into LDS slots
// part[q * 32 + (lane & 31)] (atomics, so any number of threads may share a
// slot); tile_count_flush reduces the slots after a barrier.
constexpr uint32_t kCountSlots = 32;

__host__ __device__ inline uint32_t count_states(uint32_t S)
{
    return S < 4 ? 4u : (S < 6 ? 6u : 8u);
}

__host__ __device__ constexpr uint64_t pair_code_table(int p)
{
    return (0x01ull << (8 * (2 * p + 1))) | (0x10ull << (8 * (2 * p + 2)));
}

template <int NS>
__device__ __forceinline__ void tile_count_sums(const uint8_t *lat,
                                                const TileGeom &G,
                                                uint32_t *part)
{
    constexpr int NP = (NS - 2) / 2; // code tables
    const uint32_t LS = G.LS(), dwr = G.TW >> 3;
    const uint32_t rstep = blockDim.x / dwr; // >= 1: TW / 8 <= blockDim
    const uint32_t r0 = threadIdx.x / dwr, j = threadIdx.x - r0 * dwr;
    uint32_t n[NS - 1];
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        n[q] = 0;
    if (r0 < rstep) {
        const uint8_t *p = lat + (4 + r0) * LS + 8 + 8 * j;
        const uint32_t pstep = rstep * LS;
        uint32_t r = r0;
        while (r < G.TH) {
            uint32_t sv = 0, cp[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k)
                cp[k] = 0;
            for (uint32_t g = 0; g < 7 && r < G.TH; ++g) {
                const uint2 v = *reinterpret_cast<const uint2 *>(p);
                sv += v.x + v.y;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint64_t t = pair_code_table(k);
                    const uint32_t hi = (uint32_t)(t >> 32), lo = (uint32_t)t;
                    cp[k] += __builtin_amdgcn_perm(hi, lo, v.x) +
                             __builtin_amdgcn_perm(hi, lo, v.y);
                }
                r += rstep;
                p += pstep;
            }
            n[NS - 2] = __builtin_amdgcn_udot4(sv, 0x01010101u, n[NS - 2],
                                               false);
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                n[2 * k] = __builtin_amdgcn_udot8(cp[k], 0x01010101u,
                                                  n[2 * k], false);
                n[2 * k + 1] = __builtin_amdgcn_udot8(cp[k], 0x10101010u,
                                                      n[2 * k + 1], false);
            }
        }
    }
    uint32_t *slot = part + (threadIdx.x & (kCountSlots - 1));
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        atomicAdd(slot + q * kCountSlots, n[q]);
}

__device__ inline void tile_count_sums(const uint8_t *lat, const TileGeom &G,
                                       uint32_t S, uint32_t *part)
{
    const uint32_t ns = count_states(S);
    if (ns == 4)
        tile_count_sums<4>(lat, G, part);
    else if (ns == 6)
        tile_count_sums<6>(lat, G, part);
    else
        tile_count_sums<8>(lat, G, part);
}

// Flush, step 1 (lane of the flushing wave): the sum of slots 4j .. 4j+3 of
// sum q = lane / 8, j = lane % 8, which it also clears; 0 for q >= nq.
__device__ __forceinline__ uint32_t count_slot_sum(uint32_t *part,
                                                   uint32_t lane, uint32_t nq)
{
    const uint32_t q = lane >> 3, j = lane & 7u;
    if (q >= nq)
        return 0;
    uint4 *p = reinterpret_cast<uint4 *>(part + q * kCountSlots + 4 * j);
    const uint4 x = *p;
    *p = make_uint4(0u, 0u, 0u, 0u);
    return x.x + x.y + x.z + x.w;
}

// Flush, step 3: the count of species s from the NS - 1 sums T (uniform).
template <int NS>
__device__ __forceinline__ uint32_t count_species(uint32_t s,
                                                  const uint32_t (&T)[NS - 1],
                                                  uint32_t sites)
{
    uint32_t direct = 0, weighted = 0, v = 0;
#pragma unroll
    for (int q = 0; q < NS - 2; ++q) {
        direct += T[q];
        weighted += (uint32_t)(q + 1) * T[q];
        v = (s == (uint32_t)q + 1) ? T[q] : v;
    }
    const uint32_t last = (T[NS - 2] - weighted) / (uint32_t)(NS - 1);
    v = (s == (uint32_t)NS - 1) ? last : v;
    return (s == 0) ? sites - direct - last : v;
}

// Adds the interior's counts (from the slots, which it clears) to
// row[0..S] (global atomics).  Called by all 64 lanes of one wave after a
// barrier that follows tile_count_sums; step 2 adds the eight partial sums
// of each q with DPP (quad swaps, then row_shr:4 so that lane 8q+4 holds the
// total).
template <int NS>
__device__ __forceinline__ void tile_count_flush(uint32_t *part, uint32_t S,
                                                 uint32_t sites,
                                                 uint32_t *row)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t v = count_slot_sum(part, lane, NS - 1);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    uint32_t T[NS - 1];
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        T[q] = (uint32_t)__builtin_amdgcn_readlane((int)v, 8 * q + 4);
    const uint32_t c = count_species<NS>(lane, T, sites);
    if (lane <= S && c)
        atomicAdd(row + lane, c);
}

__device__ inline void tile_count_flush(uint32_t *part, uint32_t S,
                                        uint32_t sites, uint32_t *row)
{
    const uint32_t ns = count_states(S);
    if (ns == 4)
        tile_count_flush<4>(part, S, sites, row);
    else if (ns == 6)
        tile_count_flush<6>(part, S, sites, row);
    else
        tile_count_flush<8>(part, S, sites, row);
}

} // namespace escg
