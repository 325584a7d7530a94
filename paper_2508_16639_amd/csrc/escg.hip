// escg.hip -- HIP kernels (gfx950) and the C ABI of the ESCG hot path.
//
// Kernels
//   init_kernel        counter-RNG initial lattice, one Philox call per
//                      4 sites, dword stores
//   densities_kernel   species counts: per-lane SWAR byte compares, wave
//                      reduction, one atomic per workgroup and species
//   lds_*_kernel       whole lattice resident in LDS for the entire run
//                      (L <= 404): four block passes per MCS separated by
//                      workgroup barriers, counts and the stop test after
//                      every MCS, one workgroup per job; the batch variant is
//                      persistent and pulls jobs from a queue
//   tile_mcs_kernel    large lattices: one launch per MCS, each workgroup
//                      stages a tile plus a 4-row / 8-column halo in LDS,
//                      runs the four passes there (a 4-site halo covers the
//                      four passes' dependency cone), counts its interior and
//                      writes it to the other buffer of a ping-pong pair
//
// See escg_device.hpp for the schedule / random-number contract.
#include "escg_device.hpp"
#include "escg_quad.hpp"
#include "escg_lds.hpp"
#include "escg_tile.hpp"
#include "escg.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

using namespace escg;

namespace {

constexpr uint32_t kResultWords = ESCG_BATCH_RESULT_WORDS;

// ---------------------------------------------------------------------------
// Job descriptor of the LDS-resident kernels
// ---------------------------------------------------------------------------
struct JobDev {
    uint64_t seed;
    uint64_t lat_off;     // byte offset of the lattice in the base pointer
    uint64_t dom_packed;  // DomPacked bits (S <= 7)
    uint32_t *counts;     // optional per-MCS count rows (max_mcs+1)*(S+1)
    uint32_t *result;     // optional {flag, t_ext, counts[0..S]}
    uint32_t L, S, T1, T2;
    uint32_t replica, mcs0, max_mcs, mode;
    uint32_t init, result_words, moore, pad1;
    const uint32_t *ab;   // selection thresholds (dominance probabilities)
    uint32_t dom[32];
};

__host__ __device__ inline bool stop_met(const uint32_t *c, uint32_t S,
                                         uint32_t mode)
{
    if (mode == ESCG_STOP_NONE)
        return false;
    uint32_t alive = 0;
    for (uint32_t s = 1; s <= S; ++s)
        alive += c[s] > 0u;
    return mode == ESCG_STOP_FIRST_EXTINCTION ? alive < S : alive <= 1u;
}

// Counts sites of value 0..S (S > 7) among ndw dwords of LDS by byte
// compares; adds into cnt[0..S] (LDS, zeroed beforehand).  Bytes that are
// not sites hold pad_byte(S), which matches no species.
__device__ __forceinline__ void count_dwords_wide(const uint32_t *lat32,
                                                  uint32_t ndw, uint32_t S,
                                                  uint32_t *cnt)
{
    constexpr int SM = 32;
    uint32_t c[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s)
        c[s] = 0;
    uint32_t mine = 0;
    for (uint32_t i = threadIdx.x; i < ndw; i += blockDim.x) {
        const uint32_t v = lat32[i];
        ++mine;
#pragma unroll
        for (int s = 0; s < SM; ++s)
            if ((uint32_t)s <= S)
                c[s] += bytes_ne(v, (uint32_t)s);
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

// Whole-lattice counts for S <= 7 from the linear sums of tile_count_sums:
// every thread walks the dword pairs i = tid, tid + blockDim, ... of the LDS
// lattice (padding bytes, value 12, get code 0 and add 12 each to the value
// sum, which the caller takes off) in groups of at most 7 pairs, and adds
// its NS - 1 sums to part[q * 8 + (lane & 7)] with LDS atomics.  The slots
// are cleared once per job and then accumulate: each MCS's sums are the
// differences of two cumulative totals (exact modulo 2^32).
template <int NS>
__device__ __forceinline__ void lds_count_sums(const uint32_t *lat32,
                                               uint32_t ndw, uint32_t *part)
{
    constexpr int NP = (NS - 2) / 2;
    const uint2 *lat64 = reinterpret_cast<const uint2 *>(lat32);
    const uint32_t np = ndw >> 1, nt = blockDim.x; // ndw is even
    uint32_t n[NS - 1];
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        n[q] = 0;
    uint32_t i = threadIdx.x;
    while (i < np) {
        uint32_t sv = 0, cp[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            cp[k] = 0;
        for (uint32_t g = 0; g < 7 && i < np; ++g, i += nt) {
            const uint2 v = lat64[i];
            sv += v.x + v.y;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const uint64_t t = pair_code_table(k);
                const uint32_t hi = (uint32_t)(t >> 32), lo = (uint32_t)t;
                cp[k] += __builtin_amdgcn_perm(hi, lo, v.x) +
                         __builtin_amdgcn_perm(hi, lo, v.y);
            }
        }
        n[NS - 2] = __builtin_amdgcn_udot4(sv, 0x01010101u, n[NS - 2], false);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            n[2 * k] = __builtin_amdgcn_udot8(cp[k], 0x01010101u, n[2 * k],
                                              false);
            n[2 * k + 1] = __builtin_amdgcn_udot8(cp[k], 0x10101010u,
                                                  n[2 * k + 1], false);
        }
    }
    uint32_t *slot = part + (threadIdx.x & 7u);
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        atomicAdd(slot + 8 * q, n[q]);
}

// One MCS's counts c[0..7] (uniform; c[s] = 0 for s >= NS) after a barrier
// that follows lds_count_sums: every wave adds the eight slots of each sum
// (DPP quad swaps and row_shr:4, total in lane 8q+4), takes the previous
// cumulative totals `prev` off and derives the species counts.
template <int NS>
__device__ __forceinline__ void lds_count_close(const uint32_t *part,
                                                uint32_t (&prev)[7],
                                                uint32_t sites, uint32_t pads,
                                                uint32_t (&c)[8])
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t v = lane < 8u * (NS - 1) ? part[lane] : 0u;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    uint32_t D[NS - 1];
#pragma unroll
    for (int q = 0; q < NS - 1; ++q) {
        const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)v, 8 * q + 4);
        D[q] = T - prev[q];
        prev[q] = T;
    }
    D[NS - 2] -= 12u * pads; // padding bytes in the value sum
#pragma unroll
    for (int s = 0; s < 8; ++s)
        c[s] = s < NS ? count_species<NS>((uint32_t)s, D, sites) : 0u;
}

// c[k] for a per-lane index k <= 7 (c uniform).
__device__ __forceinline__ uint32_t pick8(const uint32_t (&c)[8], uint32_t k)
{
    uint32_t v = c[0];
#pragma unroll
    for (uint32_t s = 1; s < 8; ++s)
        v = (k == s) ? c[s] : v;
    return v;
}

// stop_met on uniform counts c[0..7] (S <= 7), without indexing by S.
__device__ __forceinline__ bool stop_met8(const uint32_t (&c)[8], uint32_t S,
                                          uint32_t mode)
{
    if (mode == ESCG_STOP_NONE)
        return false;
    uint32_t alive = 0;
#pragma unroll
    for (uint32_t s = 1; s < 8; ++s)
        alive += (s <= S && c[s] > 0u) ? 1u : 0u;
    return mode == ESCG_STOP_FIRST_EXTINCTION ? alive < S : alive <= 1u;
}

template <bool kPacked, bool kProb>
__device__ void run_job_lds(const JobDev &J, uint8_t *base, uint8_t *smem,
                            LdsTables<kPacked ? 8 : 32> &TB)
{
    uint32_t *s_cnt = TB.cnt;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t L = J.L, S = J.S, LS = row_stride(L);
    uint8_t *lat = smem;
    uint32_t *lat32 = reinterpret_cast<uint32_t *>(lat);
    const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
    uint8_t *g = base + J.lat_off;

    setup_tables(TB, J.dom, J.moore != 0, kProb ? J.ab : nullptr);
    // row padding bytes match no species
    if (LS != L)
        for (uint32_t r = tid; r < L; r += nt)
            for (uint32_t c = L; c < LS; ++c)
                lat[r * LS + c] = pad_byte(S);
    if (J.init) {
        const uint32_t nw = (L * L) >> 2;
        for (uint32_t i = tid; i < nw; i += nt) {
            const Words w = philox(i, 0u, kTagInit << 8, J.replica, k0, k1);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t n = 4u * i + j, r = n / L, c = n - r * L;
                lat[r * LS + c] =
                    (uint8_t)(((uint64_t)pick(w, j) * (S + 1u)) >> 32);
            }
        }
    } else if ((L & 3u) == 0) {
        const uint32_t dwr = L >> 2, nw = L * dwr;
        const uint32_t *g32 = reinterpret_cast<const uint32_t *>(g);
        for (uint32_t i = tid; i < nw; i += nt) {
            const uint32_t r = i / dwr, c = i - r * dwr;
            lat32[(r * LS >> 2) + c] = g32[i];
        }
    } else {
        const uint32_t hr = L >> 1, nh = L * hr;
        const uint16_t *g16 = reinterpret_cast<const uint16_t *>(g);
        for (uint32_t i = tid; i < nh; i += nt) {
            const uint32_t r = i / hr, c = i - r * hr;
            reinterpret_cast<uint16_t *>(lat)[(r * LS >> 1) + c] = g16[i];
        }
    }
    if (kPacked)
        for (uint32_t i = tid; i < 64; i += nt)
            s_cnt[i] = 0; // count slots (lds_count_sums), cleared per job
    __syncthreads();
    const auto qc = make_quad_ctx<kProb>(TB, J.T1, J.T2);
    const LdsWalk W = lds_walk(L, LS);
    const uint32_t ndw = (LS * L) >> 2;
    // the Philox heads of this thread's quads, once per job, when they fit
    const bool heads = lds_heads_fit(W, L);
    LdsHeads H;
    if (heads)
        H = lds_heads(W, J.replica, k1);

    // counts of the current state: S <= 7 into c[] (uniform, every wave),
    // else into the LDS row `row` of s_cnt; returns the stop test
    uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t prev[7] = {0, 0, 0, 0, 0, 0, 0};
    const uint32_t sites = L * L, pads = (LS - L) * L;
    const uint32_t ns = count_states(S);
    uint32_t cur = 0;
    bool stop;
    if constexpr (kPacked) {
        if (ns == 4) {
            lds_count_sums<4>(lat32, ndw, s_cnt);
            __syncthreads();
            lds_count_close<4>(s_cnt, prev, sites, pads, c);
        } else if (ns == 6) {
            lds_count_sums<6>(lat32, ndw, s_cnt);
            __syncthreads();
            lds_count_close<6>(s_cnt, prev, sites, pads, c);
        } else {
            lds_count_sums<8>(lat32, ndw, s_cnt);
            __syncthreads();
            lds_count_close<8>(s_cnt, prev, sites, pads, c);
        }
        stop = stop_met8(c, S, J.mode);
        if (J.counts && tid <= S)
            J.counts[tid] = pick8(c, tid);
    } else {
        count_dwords_wide(lat32, ndw, S, s_cnt);
        __syncthreads();
        stop = stop_met(s_cnt, S, J.mode);
        if (J.counts && tid <= S)
            J.counts[tid] = s_cnt[tid];
    }
    uint32_t t = 0;
    while (!stop && t < J.max_mcs) {
        const uint32_t nxt = cur ^ 1u;
        if (!kPacked && tid < 32)
            s_cnt[nxt * 32 + tid] = 0;
        if (heads)
            lds_mcs<true>(lat, L, LS, J.mcs0 + t, J.replica, k0, k1, qc, W,
                          &H);
        else
            lds_mcs(lat, L, LS, J.mcs0 + t, J.replica, k0, k1, qc, W);
        ++t;
        if constexpr (kPacked) {
            if (ns == 4) {
                lds_count_sums<4>(lat32, ndw, s_cnt);
                __syncthreads();
                lds_count_close<4>(s_cnt, prev, sites, pads, c);
            } else if (ns == 6) {
                lds_count_sums<6>(lat32, ndw, s_cnt);
                __syncthreads();
                lds_count_close<6>(s_cnt, prev, sites, pads, c);
            } else {
                lds_count_sums<8>(lat32, ndw, s_cnt);
                __syncthreads();
                lds_count_close<8>(s_cnt, prev, sites, pads, c);
            }
            stop = stop_met8(c, S, J.mode);
            if (J.counts && tid <= S)
                J.counts[(size_t)t * (S + 1) + tid] = pick8(c, tid);
        } else {
            count_dwords_wide(lat32, ndw, S, s_cnt + nxt * 32);
            __syncthreads();
            cur = nxt;
            stop = stop_met(s_cnt + cur * 32, S, J.mode);
            if (J.counts && tid <= S)
                J.counts[(size_t)t * (S + 1) + tid] = s_cnt[cur * 32 + tid];
        }
    }
    if ((L & 3u) == 0) {
        const uint32_t dwr = L >> 2, nw = L * dwr;
        uint32_t *g32 = reinterpret_cast<uint32_t *>(g);
        for (uint32_t i = tid; i < nw; i += nt) {
            const uint32_t r = i / dwr, c = i - r * dwr;
            g32[i] = lat32[(r * LS >> 2) + c];
        }
    } else {
        const uint32_t hr = L >> 1, nh = L * hr;
        uint16_t *g16 = reinterpret_cast<uint16_t *>(g);
        for (uint32_t i = tid; i < nh; i += nt) {
            const uint32_t r = i / hr, c = i - r * hr;
            g16[i] = reinterpret_cast<const uint16_t *>(lat)[(r * LS >> 1) + c];
        }
    }
    if (J.result) {
        for (uint32_t i = tid; i < J.result_words; i += nt) {
            uint32_t v = 0;
            if (i == 0)
                v = stop ? 1u : 0u;
            else if (i == 1)
                v = t;
            else if (i - 2 <= S)
                v = kPacked ? pick8(c, i - 2) : s_cnt[cur * 32 + (i - 2)];
            J.result[i] = v;
        }
    }
    __syncthreads();
}

template <bool kPacked, bool kProb>
__global__ __launch_bounds__(512) void lds_single_kernel(JobDev J,
                                                         uint8_t *base)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LdsTables<kPacked ? 8 : 32> TB;
    run_job_lds<kPacked, kProb>(J, base, smem, TB);
}

template <bool kPacked, bool kProb>
__global__ __launch_bounds__(512) void lds_batch_kernel(
    const JobDev *__restrict__ jobs, const uint32_t *__restrict__ order,
    uint32_t n, uint32_t *queue, uint8_t *base)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LdsTables<kPacked ? 8 : 32> TB;
    for (;;) {
        if (threadIdx.x == 0)
            TB.misc[0] = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t qi = TB.misc[0];
        __syncthreads();
        if (qi >= n)
            return;
        run_job_lds<kPacked, kProb>(jobs[order[qi]], base, smem, TB);
    }
}

// ---------------------------------------------------------------------------
// Large lattices: one launch per MCS over tiles with halos
// ---------------------------------------------------------------------------
constexpr int kTileH = 64;
constexpr int kTileW = 128;
constexpr int kHaloR = 4;
constexpr int kHaloC = 8;
constexpr int kTileThreads = 256;

struct TileArgs {
    const uint8_t *src;
    uint8_t *dst;
    uint32_t *counts;     // S+1 words of this MCS's row (zeroed) or null
    const uint32_t *done; // non-null and nonzero: only copy src to dst
    uint64_t seed;
    uint64_t dom_packed;
    const uint32_t *ab;   // selection thresholds (global) or null
    uint32_t L, S, T1, T2, replica, t, moore;
    uint32_t dom[32];
};

template <bool kPacked>
__global__ __launch_bounds__(kTileThreads) void tile_mcs_kernel(TileArgs a)
{
    constexpr uint32_t LS = kTileW + 2 * kHaloC; // LDS row stride
    constexpr uint32_t RH = kTileH + 2 * kHaloR;
    __shared__ __align__(16) uint8_t lat[RH * LS];
    __shared__ uint32_t s_dom[32];
    __shared__ uint32_t s_cnt[32];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t L = a.L, S = a.S, Lb = L >> 1, Q = (Lb + 3) >> 2;
    const uint32_t R0 = blockIdx.y * kTileH, g0 = blockIdx.x * kTileW;
    const uint32_t th = min((uint32_t)kTileH, L - R0);
    const uint32_t tw = min((uint32_t)kTileW, L - g0);
    const bool aligned = (L & 3u) == 0;

    if (a.done && *a.done) { // stopped: carry the state over unchanged
        for (uint32_t i = tid; i < th * tw; i += nt) {
            const uint32_t r = i / tw, c = i - r * tw;
            const size_t gi = (size_t)(R0 + r) * L + g0 + c;
            a.dst[gi] = a.src[gi];
        }
        return;
    }
    if (tid < 32) {
        s_dom[tid] = a.dom[tid];
        s_cnt[tid] = 0;
    }
    // Stage rows R0-4 .. R0+th+4 and columns g0-8 .. g0+tw+8 (mod L).
    {
        const uint32_t rows = th + 2 * kHaloR, dwr = (tw + 2 * kHaloC) >> 2;
        for (uint32_t i = tid; i < rows * dwr; i += nt) {
            const uint32_t lr = i / dwr, j = i - lr * dwr;
            const uint32_t gr = (R0 + L - kHaloR + lr) % L;
            const uint32_t gc = (g0 + L - kHaloC + 4 * j) % L;
            uint32_t v;
            if (aligned) {
                v = *reinterpret_cast<const uint32_t *>(a.src + (size_t)gr * L +
                                                        gc);
            } else {
                v = 0;
                for (uint32_t b = 0; b < 4; ++b) {
                    const uint32_t c = (gc + b) % L;
                    v |= (uint32_t)a.src[(size_t)gr * L + c] << (8 * b);
                }
            }
            *reinterpret_cast<uint32_t *>(&lat[lr * LS + 4 * j]) = v;
        }
    }
    __syncthreads();

    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    DomPacked dp{a.dom_packed};
    DomTable dt{s_dom};
    const Words off =
        philox_uniform(0u, a.t, kTagOffset << 8, a.replica, k0, k1);
    const int bx_base = (int)(g0 >> 1) - kHaloC / 2; // global bx of m = 0
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        const uint32_t ox = off.w[p] & 1u, oy = (off.w[p] >> 1) & 1u;
        const uint32_t nbr = (th + 2 * kHaloR - oy) >> 1;
        const uint32_t nbc = (tw + 2 * kHaloC - ox) >> 1;
        const uint32_t nqs = (nbc + 3) >> 2;
        const uint32_t ctr2 = (kTagPass << 8) | p;
        for (uint32_t i = tid; i < nbr * nqs; i += nt) {
            const uint32_t k = i / nqs, js = i - k * nqs;
            const uint32_t lr = oy + 2 * k;
            const uint32_t gr = (R0 + L - kHaloR + lr) % L;
            const uint32_t by = (gr - oy) >> 1;
            const uint32_t m0 = 4 * js;
            const uint32_t mlast = min(m0 + 3, nbc - 1);
            int bxf = bx_base + (int)m0, bxl = bx_base + (int)mlast;
            bxf += bxf < 0 ? (int)Lb : 0;
            bxf -= bxf >= (int)Lb ? (int)Lb : 0;
            bxl += bxl < 0 ? (int)Lb : 0;
            bxl -= bxl >= (int)Lb ? (int)Lb : 0;
            const uint32_t qf = (uint32_t)bxf >> 2, ql = (uint32_t)bxl >> 2;
            const Words rf = philox(by * Q + qf, a.t, ctr2, a.replica, k0, k1);
            Words rl = rf;
            if (ql != qf)
                rl = philox(by * Q + ql, a.t, ctr2, a.replica, k0, k1);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t m = m0 + j;
                const uint32_t lc = ox + 2 * m;
                if (m < nbc && lc >= (uint32_t)(kHaloC - kHaloR) &&
                    lc + 1 < tw + kHaloC + kHaloR) {
                    int bx = bx_base + (int)m;
                    bx += bx < 0 ? (int)Lb : 0;
                    bx -= bx >= (int)Lb ? (int)Lb : 0;
                    const uint32_t q = (uint32_t)bx >> 2;
                    const uint32_t w = pick(q == qf ? rf : rl, (uint32_t)bx & 3u);
                    const uint32_t pA = lr * LS + lc;
                    if (kPacked)
                        update_block(lat, pA, pA + 1, pA + LS, pA + LS + 1, w,
                                     a.T1, a.T2, dp, a.moore != 0, a.ab, 8u);
                    else
                        update_block(lat, pA, pA + 1, pA + LS, pA + LS + 1, w,
                                     a.T1, a.T2, dt, a.moore != 0, a.ab, 32u);
                }
            }
        }
        __syncthreads();
    }

    // Interior: LDS rows 4 .. th+4, columns 8 .. tw+8.
    uint32_t ne[kPacked ? 8 : 32];
    constexpr int SM = kPacked ? 8 : 32;
#pragma unroll
    for (int s = 0; s < SM; ++s)
        ne[s] = 0;
    uint32_t mine = 0;
    if (aligned && (tw & 3u) == 0) {
        const uint32_t dwr = tw >> 2;
        for (uint32_t i = tid; i < th * dwr; i += nt) {
            const uint32_t r = i / dwr, j = i - r * dwr;
            const uint32_t v = *reinterpret_cast<const uint32_t *>(
                &lat[(r + kHaloR) * LS + kHaloC + 4 * j]);
            *reinterpret_cast<uint32_t *>(a.dst + (size_t)(R0 + r) * L + g0 +
                                          4 * j) = v;
            ++mine;
#pragma unroll
            for (int s = 0; s < SM; ++s)
                if ((uint32_t)s <= S)
                    ne[s] += bytes_ne(v, (uint32_t)s);
        }
        mine *= 4;
    } else {
        for (uint32_t i = tid; i < th * tw; i += nt) {
            const uint32_t r = i / tw, c = i - r * tw;
            const uint32_t v = lat[(r + kHaloR) * LS + kHaloC + c];
            a.dst[(size_t)(R0 + r) * L + g0 + c] = (uint8_t)v;
            ++mine;
#pragma unroll
            for (int s = 0; s < SM; ++s)
                if ((uint32_t)s <= S)
                    ne[s] += (v != (uint32_t)s) ? 1u : 0u;
        }
    }
    if (a.counts) {
#pragma unroll
        for (int s = 0; s < SM; ++s) {
            if ((uint32_t)s <= S) {
                const uint32_t c = wave_sum(mine - ne[s]);
                if ((tid & 63u) == 0 && c)
                    atomicAdd(&s_cnt[s], c);
            }
        }
        __syncthreads();
        if (tid <= S && s_cnt[tid])
            atomicAdd(&a.counts[tid], s_cnt[tid]);
    }
}

// ---------------------------------------------------------------------------
// Large lattices: persistent tiled kernel (one launch for all MCS)
// ---------------------------------------------------------------------------

// Sticky per-device error word: set when a persistent kernel's bounded wait
// for a neighbour gives up (only possible if its workgroups were not all
// resident).  Read and cleared by escg_async_status().
__device__ uint32_t g_async_error;

struct TiledArgs {
    uint8_t *lattice;   // in/out
    uint32_t *exch;     // exchange slot 0 of this job (T * slot_dwords), slot
                        // 1 at exch + xstride; tags pre-set (exch_tag)
    uint32_t *abort;    // 1 word, zeroed
    uint32_t *counts;   // rows (n+1)*(S+1) with rows 1..n zeroed, or null
    uint64_t seed;
    TileGeom G;
    uint32_t S, T1, T2, replica, mcs0, n_mcs, spin_limit, moore;
    uint32_t xstride;   // dwords from slot 0 to slot 1 of the exchange area
    uint32_t wg0;       // multi-job launches: first workgroup of this job
    const uint32_t *ab;   // selection thresholds (global) or null
    uint32_t dom[32];
};

// One tile of one job for all of its MCS: load the tile and halo into LDS,
// then per MCS the four passes, the tagged publish of the border strips, the
// interior counts (overlapped with the first halo loads) and the halo
// gather; finally store the interior.  `a` is the job (kernel argument or a
// global table entry: its fields are read once into registers).
// kList: the quads of a pass by TileList (else TileWalk); one walk per
// instantiation keeps the other's code and registers out of the MCS loop.
template <bool kPacked, bool kProb, bool kList>
__device__ __forceinline__ void persistent_tile(const TiledArgs &a,
                                                uint32_t tile)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LdsTables<kPacked ? 8 : 32> TB;
    __shared__ __align__(16) uint32_t s_part[8 * kCountSlots];
    uint32_t *s_cnt = TB.cnt;
    uint32_t *s_misc = TB.misc;
    uint8_t *lat = smem;
    const TileGeom G = a.G;
    const uint32_t tid = threadIdx.x, S = a.S;
    const uint32_t ty = tile / G.TX, tx = tile - (tile / G.TX) * G.TX;
    const uint64_t seed = a.seed;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t sd = G.slot_dwords(), xs = a.xstride;
    uint8_t *const glat = a.lattice;
    uint32_t *const exch = a.exch;
    uint32_t *const abort_w = a.abort;
    uint32_t *const counts = a.counts;
    const uint32_t mcs0 = a.mcs0, n_mcs = a.n_mcs, replica = a.replica;
    const uint32_t spin_limit = a.spin_limit;

    if (tid == 0)
        s_misc[0] = 0;
    for (uint32_t i = tid; i < 8 * kCountSlots; i += blockDim.x)
        s_part[i] = 0;
    tile_load(lat, glat, G, ty, tx);
    setup_tables(TB, a.dom, a.moore != 0, kProb ? a.ab : nullptr);
    const auto qc = make_quad_ctx<kProb>(TB, a.T1, a.T2); // after a barrier
    const HaloPlan HP = halo_plan(exch, G, ty, tx);

    bool aborted = false;
    const TileWalk W = tile_walk(G, ty, tx);
    TileList TL;
    if constexpr (kList)
        TL = tile_list(G, ty, tx);
    // (a plain loop: the same loop written as a lambda taking the walk
    // measured 10 % slower per MCS on mid-size lattices)
    for (uint32_t t = 0; t < n_mcs; ++t) {
        if constexpr (kList)
            tile_mcs_list(lat, lat + G.region_bytes() + 8, G, TL, mcs0 + t,
                          replica, k0, k1, qc);
        else
            tile_mcs(lat, G, W, mcs0 + t, replica, k0, k1, qc);
        // publish, count and gather touch disjoint parts of the region:
        // border strips and interior are read, only the halo is written
        const uint32_t e = t + 1, slot = exch_slot(e), tag = exch_tag(e);
        tile_publish(lat, exch + (size_t)slot * xs + (size_t)tile * sd, G,
                     tag);
        // the tags replace flags: each halo word is awaited on its own; the
        // counts run while the first halo loads are in flight
        const uint32_t st = tile_gather(
            lat, exch, HP, G, ty, tx, slot * xs, tag, abort_w, spin_limit,
            [&] {
                if (counts) {
                    if (kPacked)
                        tile_count_sums(lat, G, S, s_part);
                    else
                        tile_count_wide(lat, G, S, s_cnt);
                }
            });
        if (st) {
            if (st == 2) {
                xstore(abort_w, 1u);
                atomicOr(&g_async_error, 1u);
            }
            s_misc[0] = 1;
        }
        __syncthreads();
        if (counts) {
            uint32_t *row = counts + (size_t)(t + 1) * (S + 1);
            if constexpr (kPacked) {
                if (tid < 64) // one wave; the slots are next used 4 barriers on
                    tile_count_flush(s_part, S, G.TH * G.TW, row);
            } else if (tid <= S) {
                atomicAdd(&row[tid], s_cnt[tid]);
                s_cnt[tid] = 0;
            }
        }
        if (s_misc[0]) {
            aborted = true;
            break;
        }
    }
    if (!aborted)
        tile_store(lat, glat, G, ty, tx);
}

// XCD-aware tile of workgroup b of a job with T tiles: workgroups are dealt
// round-robin to the 8 XCDs, so when T % 8 == 0 each XCD gets a contiguous
// band of tiles (neighbours share an L2).  b counts from a multiple of 8.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t T)
{
    return (T % 8u == 0) ? (b & 7u) * (T >> 3) + (b >> 3) : b;
}

// All MCS of one large lattice in one cooperative launch (one workgroup per
// tile).
template <bool kPacked, bool kProb, bool kList>
__global__ __launch_bounds__(1024) void tiled_persistent_kernel(TiledArgs a)
{
    persistent_tile<kPacked, kProb, kList>(a, xcd_tile(blockIdx.x,
                                                       a.G.TY * a.G.TX));
}

// Several large lattices in one launch: job j owns workgroups
// [wg0_j, wg0_j + T_j) (wg0_j a multiple of 8 when T_j is; workgroups in
// the gaps exit at once) and runs its own MCS count.  The tiles of a job
// wait only for each other, and the launch holds no more workgroups than
// the device keeps resident at once, so every tile becomes resident even
// while other kernels hold CUs for a while (they never wait for this one).
template <bool kPacked, bool kProb, bool kList>
__global__ __launch_bounds__(1024) void tiled_persistent_multi_kernel(
    const TiledArgs *__restrict__ jobs, uint32_t njobs)
{
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].wg0 <= b)
            lo = mid;
        else
            hi = mid;
    }
    const TiledArgs &a = jobs[lo];
    const uint32_t T = a.G.TY * a.G.TX, local = b - a.wg0;
    if (local >= T)
        return;
    persistent_tile<kPacked, kProb, kList>(a, xcd_tile(local, T));
}

// One MCS of a large lattice per launch with the tile phases above: each
// workgroup loads its tile and halo from `src`, runs the four passes and
// stores the interior to `dst`.  No waits between workgroups, so launches can
// share the GPU with other work.
struct StepArgs {
    const uint8_t *src;
    uint8_t *dst;
    uint32_t *counts; // this MCS's row (S+1, zeroed) or null
    const uint32_t *done; // non-null and nonzero: only carry src to dst
    uint64_t seed;
    TileGeom G;
    uint32_t S, T1, T2, replica, t, moore;
    const uint32_t *ab;   // selection thresholds (global) or null
    uint32_t dom[32];
};

template <bool kPacked, bool kProb>
__global__ __launch_bounds__(512) void tiled_step_kernel(StepArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LdsTables<kPacked ? 8 : 32> TB;
    __shared__ __align__(16) uint32_t s_part[8 * kCountSlots];
    uint32_t *s_cnt = TB.cnt;
    uint8_t *lat = smem;
    const TileGeom G = a.G;
    const uint32_t tid = threadIdx.x, S = a.S;
    const uint32_t ty = blockIdx.x / G.TX, tx = blockIdx.x - ty * G.TX;
    if (a.done && *a.done) { // stopped: carry the tile over unchanged
        const uint32_t dwr = G.TW >> 2, R0 = ty * G.TH, g0 = tx * G.TW;
        for (uint32_t i = tid; i < G.TH * dwr; i += blockDim.x) {
            const uint32_t r = i / dwr, j = i - r * dwr;
            const size_t gi = (size_t)(R0 + r) * G.L + g0 + 4 * j;
            *reinterpret_cast<uint32_t *>(a.dst + gi) =
                *reinterpret_cast<const uint32_t *>(a.src + gi);
        }
        return;
    }
    for (uint32_t i = tid; i < 8 * kCountSlots; i += blockDim.x)
        s_part[i] = 0;
    tile_load(lat, a.src, G, ty, tx);
    setup_tables(TB, a.dom, a.moore != 0, kProb ? a.ab : nullptr);
    const auto qc = make_quad_ctx<kProb>(TB, a.T1, a.T2);
    tile_mcs(lat, G, tile_walk(G, ty, tx), a.t, a.replica, (uint32_t)a.seed,
             (uint32_t)(a.seed >> 32), qc);
    tile_store(lat, a.dst, G, ty, tx);
    if (a.counts) {
        if (kPacked)
            tile_count_sums(lat, G, S, s_part);
        else
            tile_count_wide(lat, G, S, s_cnt);
        __syncthreads();
        if constexpr (kPacked) {
            if (tid < 64)
                tile_count_flush(s_part, S, G.TH * G.TW, a.counts);
        } else if (tid <= S && s_cnt[tid]) {
            atomicAdd(&a.counts[tid], s_cnt[tid]);
        }
    }
}

// One MCS of many large lattices per launch: the tiles of every job form one
// grid (job i owns workgroups [wg0_i, wg0_{i+1})), so jobs too small to fill
// the GPU alone advance together.  Each job ping-pongs between its lattice
// and a scratch buffer: step k reads the lattice when k is even.
struct BatchStepJob {
    uint8_t *lattice;
    uint8_t *scratch;
    uint64_t seed;
    TileGeom G;
    uint32_t S, T1, T2, replica, t0;
    uint32_t wg0, moore;
    const uint32_t *ab;   // selection thresholds (global) or null
    uint32_t dom[32];
};

constexpr uint32_t kBatchStepThreads = 512;

template <bool kPacked, bool kProb>
__global__ __launch_bounds__(kBatchStepThreads) void tiled_step_batch_kernel(
    const BatchStepJob *jobs, uint32_t njobs, uint32_t k)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LdsTables<kPacked ? 8 : 32> TB;
    // the job owning this workgroup: last i with wg0_i <= blockIdx.x
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].wg0 <= b)
            lo = mid;
        else
            hi = mid;
    }
    const BatchStepJob &J = jobs[lo];
    const TileGeom G = J.G;
    const uint32_t tile = b - J.wg0, ty = tile / G.TX, tx = tile - ty * G.TX;
    const uint8_t *src = (k & 1u) ? J.scratch : J.lattice;
    uint8_t *dst = (k & 1u) ? J.lattice : J.scratch;
    uint8_t *lat = smem;
    tile_load(lat, src, G, ty, tx);
    setup_tables(TB, J.dom, J.moore != 0, kProb ? J.ab : nullptr);
    const auto qc = make_quad_ctx<kProb>(TB, J.T1, J.T2);
    tile_mcs(lat, G, tile_walk(G, ty, tx), J.t0 + k, J.replica,
             (uint32_t)J.seed, (uint32_t)(J.seed >> 32), qc);
    tile_store(lat, dst, G, ty, tx);
}


// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void init_kernel(uint32_t *lat32, uint32_t ndw, uint32_t S,
                            uint64_t seed, uint32_t replica)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ndw;
         i += gridDim.x * blockDim.x) {
        const Words w = philox(i, 0u, kTagInit << 8, replica, k0, k1);
        uint32_t v = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            v |= (uint32_t)(((uint64_t)w.w[j] * (S + 1u)) >> 32) << (8 * j);
        lat32[i] = v;
    }
}

template <int SM>
__global__ __launch_bounds__(256) void densities_kernel(const uint32_t *lat32,
                                                        uint32_t ndw,
                                                        uint32_t S,
                                                        uint32_t *counts)
{
    __shared__ uint32_t s_cnt[32];
    if (threadIdx.x < 32)
        s_cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t c[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s)
        c[s] = 0;
    uint32_t mine = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ndw;
         i += gridDim.x * blockDim.x) {
        const uint32_t v = lat32[i];
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
    }
#pragma unroll
    for (int s = 0; s < SM; ++s) {
        if ((uint32_t)s <= S) {
            const uint32_t tot = wave_sum(SM == 8 ? c[s] : 4u * mine - c[s]);
            if ((threadIdx.x & 63u) == 0 && tot)
                atomicAdd(&s_cnt[s], tot);
        }
    }
    __syncthreads();
    if (threadIdx.x <= S && s_cnt[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void copy_u32_kernel(uint32_t *dst, const uint32_t *src, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Stop test between tile MCS launches.  st = {done, flag, t_ext}; cnt2 holds
// two rows of 32 counts, row `row` is the state after t_after MCS; the other
// row is cleared for the next MCS.
__global__ void check_stop_kernel(uint32_t *st, uint32_t *cnt2, uint32_t row,
                                  uint32_t S, uint32_t mode, uint32_t t_after,
                                  uint32_t *result)
{
    if (threadIdx.x != 0)
        return;
    const uint32_t *c = cnt2 + row * 32;
    if (!st[0]) {
        const bool met = stop_met(c, S, mode);
        for (uint32_t s = 0; s <= S; ++s)
            result[2 + s] = c[s];
        result[0] = met ? 1u : 0u;
        result[1] = t_after;
        if (met)
            st[0] = 1u;
    }
    for (uint32_t s = 0; s < 32; ++s)
        cnt2[(row ^ 1u) * 32 + s] = 0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Derived {
    uint32_t T1, T2;
    uint64_t packed;
    bool small; // S <= 7: packed dominance
    bool prob;  // dominance probabilities: selection thresholds in `ab`
    std::vector<uint32_t> ab;      // A then B tables, Sp * Sp u32 each
    const uint32_t *d_ab = nullptr; // `ab` on the device (set by the caller)
};

// Selection thresholds of a job with dominance probabilities (P = the 0/1
// matrix when `p` has none, which reproduces the deterministic rule): for
// x != y in 1..S, with R = T2 - T1 and in double, A = floor(P_xy R) and
// B = A + floor(P_yx (R - A)), P_xy counting only where x dominates y.
// Table stride Sp = 8 (S <= 7) or 32.
std::vector<uint32_t> selection_thresholds(const escg_params *p, uint32_t T1,
                                           uint32_t T2, uint32_t Sp = 0)
{
    const uint32_t S = p->S, R = T2 - T1;
    if (Sp == 0)
        Sp = S <= 7 ? 8u : 32u;
    std::vector<uint32_t> ab(2u * Sp * Sp, 0u);
    auto prob = [&](uint32_t a, uint32_t b) {
        if (!((p->dom[a] >> b) & 1u))
            return 0.0;
        return p->dom_prob ? p->dom_prob[(a - 1) * S + (b - 1)] : 1.0;
    };
    for (uint32_t x = 1; x <= S; ++x)
        for (uint32_t y = 1; y <= S; ++y) {
            if (x == y)
                continue;
            const uint32_t A = (uint32_t)std::floor(prob(x, y) * (double)R);
            const uint32_t B =
                A + (uint32_t)std::floor(prob(y, x) * (double)(R - A));
            ab[x * Sp + y] = A;
            ab[Sp * Sp + x * Sp + y] = B;
        }
    return ab;
}

// The calling thread's last error text and kernel path (escg_last_error,
// escg_last_route).
thread_local char g_last_error[160] = "";
thread_local uint32_t g_last_route = 0;

escg_status last_hip(hipError_t e)
{
    if (e == hipSuccess)
        return ESCG_OK;
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s",
                  hipGetErrorName(e), hipGetErrorString(e));
    return ESCG_EDEVICE;
}

// The no-allocation entry point's scratch: one array per GPU, held until
// the process ends.  Its name is only a host-side stand-in for the device
// copy; host code uses the address hipGetSymbolAddress returns for the
// current device (each GPU has its own copy at its own address).
static __device__ __align__(256) uint8_t scratch[ESCG_STATIC_SCRATCH_BYTES];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
escg_status static_scratch(uint8_t **out)
{
    static std::mutex mu;
    static std::vector<uint8_t *> addr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return last_hip(hipGetLastError());
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev)
        addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return last_hip(e != hipSuccess ? e : hipErrorInvalidSymbol);
        addr[dev] = static_cast<uint8_t *>(ptr);
    }
    *out = addr[dev];
    return ESCG_OK;
}

// Scratch of one call: stream-ordered allocations released after the call's
// last launch (base == null), or carved in order from a fixed device span
// (base != null: the no-allocation entry point's static array).
struct Arena {
    hipStream_t st;
    uint8_t *base = nullptr;
    size_t cap = 0, used = 0;
    std::vector<void *> owned;
    explicit Arena(hipStream_t s, uint8_t *b = nullptr, size_t c = 0)
        : st(s), base(b), cap(c) {}
    ~Arena()
    {
        for (void *q : owned)
            (void)hipFreeAsync(q, st);
    }
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    escg_status take(size_t bytes, void **out)
    {
        *out = nullptr;
        if (!base) {
            if (hipMallocAsync(out, bytes, st) != hipSuccess) {
                *out = nullptr;
                return ESCG_ENOMEM;
            }
            owned.push_back(*out);
            return ESCG_OK;
        }
        if (used + round(bytes) > cap) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "needs %zu bytes of static scratch, %zu available",
                          used + round(bytes), cap);
            return ESCG_ENOMEM;
        }
        *out = base + used;
        used += round(bytes);
        return ESCG_OK;
    }
};

// Copies host words into new scratch of `ar`.
escg_status upload_words(const std::vector<uint32_t> &h, Arena &ar,
                         const uint32_t **out)
{
    void *q = nullptr;
    escg_status s = ar.take(h.size() * 4, &q);
    if (s != ESCG_OK)
        return s;
    if (hipMemcpyAsync(q, h.data(), h.size() * 4, hipMemcpyHostToDevice,
                       ar.st) != hipSuccess)
        return ESCG_EDEVICE;
    *out = static_cast<const uint32_t *>(q);
    return ESCG_OK;
}

// A tile shape the tiled paths accept for side L.
bool valid_shape(uint32_t L, uint32_t TH, uint32_t TW)
{
    return L % 8 == 0 && TW >= 8 && TW % 8 == 0 && L % TW == 0 && TH >= 4 &&
           TH % 2 == 0 && L % TH == 0;
}

escg_status validate(const escg_params *p)
{
    if (!p)
        return ESCG_EINVAL;
    if (p->L < 2 || (p->L & 1u) || p->L > ESCG_MAX_L)
        return ESCG_EINVAL;
    if (p->S < 1 || p->S > ESCG_MAX_SPECIES)
        return ESCG_EINVAL;
    if (p->flags & ~ESCG_FLAG_MOORE)
        return ESCG_EINVAL;
    if (p->dom_prob)
        for (uint32_t i = 0; i < p->S * p->S; ++i)
            if (!(p->dom_prob[i] >= 0.0 && p->dom_prob[i] <= 1.0))
                return ESCG_EINVAL;
    const double r[3] = {p->rate_ex, p->rate_sel, p->rate_rep};
    for (double v : r)
        if (!(v >= 0.0) || !std::isfinite(v))
            return ESCG_EINVAL;
    if (!((p->rate_ex + p->rate_sel) + p->rate_rep > 0.0))
        return ESCG_EINVAL;
    if (p->dom[0] != 0)
        return ESCG_EINVAL;
    const escg_launch &ln = p->launch;
    if (ln.route > ESCG_ROUTE_PERSISTENT || ln.wg_per_cu > 8)
        return ESCG_EINVAL;
    if (ln.threads != 0 &&
        (ln.threads % 64 != 0 || ln.threads < 64 || ln.threads > 1024))
        return ESCG_EINVAL;
    if ((ln.tile_h != 0 || ln.tile_w != 0) &&
        !valid_shape(p->L, ln.tile_h, ln.tile_w))
        return ESCG_EINVAL;
    const uint32_t valid = (p->S >= 31 ? 0xFFFFFFFFu : ((2u << p->S) - 1u)) &
                           ~1u;
    for (uint32_t a = 1; a < 32; ++a) {
        if (a > p->S && p->dom[a] != 0)
            return ESCG_EINVAL;
        if (p->dom[a] & ~valid)
            return ESCG_EINVAL;
    }
    return ESCG_OK;
}

Derived derive(const escg_params *p)
{
    Derived d;
    escg_thresholds(p, &d.T1, &d.T2);
    d.small = p->S <= 7;
    d.prob = p->dom_prob != nullptr;
    if (d.prob)
        d.ab = selection_thresholds(p, d.T1, d.T2);
    d.packed = 0;
    if (d.small)
        for (uint32_t a = 1; a <= p->S; ++a)
            for (uint32_t b = 1; b <= p->S; ++b)
                if ((p->dom[a] >> b) & 1u)
                    d.packed |= 1ull << (a * 8 + b);
    return d;
}

inline hipStream_t S_(void *s) { return reinterpret_cast<hipStream_t>(s); }

struct DeviceInfo {
    int cus = 0;
    size_t lds_max = 0;
};

DeviceInfo device_info()
{
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return DeviceInfo{};
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev)
        cache.resize(dev + 1);
    if (cache[dev].cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            cache[dev].cus = prop.multiProcessorCount;
            cache[dev].lds_max = prop.sharedMemPerBlock;
        }
    }
    return cache[dev];
}

// Static LDS of the kernels (tables) and dynamic LDS of a whole lattice.
size_t static_lds_bytes(uint32_t S)
{
    return S <= 7 ? sizeof(LdsTables<8>) : sizeof(LdsTables<32>);
}

// The tiled kernels add the count slots (tile_count_sums) to the tables.
// Dynamic LDS of a tiled kernel: the region, twice for the list walk (its
// passes alternate between two copies).
size_t tiled_lds_bytes(const TileGeom &G, bool list)
{
    return (list ? 2u : 1u) * (size_t)G.region_bytes();
}

size_t tiled_static_lds_bytes(uint32_t S)
{
    return static_lds_bytes(S) + sizeof(uint32_t) * 8 * kCountSlots;
}

size_t lds_job_bytes(uint32_t L, uint32_t /*S*/)
{
    return (size_t)row_stride(L) * L;
}

// Largest even L whose whole lattice (plus tables) fits one workgroup's LDS.
uint32_t lds_max_L(uint32_t S)
{
    const DeviceInfo di = device_info();
    const size_t lds = di.lds_max ? di.lds_max : 65536;
    const size_t reserve = static_lds_bytes(S) + 64;
    uint32_t L = 2;
    while (lds_job_bytes(L + 2, S) + reserve <= lds)
        L += 2;
    return lds_job_bytes(L, S) + reserve <= lds ? L : 0;
}



// Raises the dynamic-LDS limit of a kernel when the runtime supports it; a
// refusal is not an error by itself (the launch reports real failures), so
// the sticky error it leaves is cleared.
void allow_dynamic_lds(const void *fn, size_t bytes)
{
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) != hipSuccess)
        (void)hipGetLastError();
}

JobDev make_job(const escg_params *p, const Derived &d, uint64_t off,
                uint32_t mcs0, uint32_t max_mcs, uint32_t mode, uint32_t init,
                uint32_t *counts, uint32_t *result, uint32_t result_words)
{
    JobDev J;
    std::memset(&J, 0, sizeof(J));
    J.seed = p->seed;
    J.lat_off = off;
    J.dom_packed = d.packed;
    J.counts = counts;
    J.result = result;
    J.L = p->L;
    J.S = p->S;
    J.T1 = d.T1;
    J.T2 = d.T2;
    J.replica = p->replica;
    J.mcs0 = mcs0;
    J.max_mcs = max_mcs;
    J.mode = mode;
    J.init = init;
    J.result_words = result_words;
    J.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
    J.ab = d.d_ab;
    for (int i = 0; i < 32; ++i)
        J.dom[i] = p->dom[i];
    return J;
}

uint32_t lds_threads(uint32_t Lmax) { return Lmax <= 128 ? 256u : 512u; }

// The instantiation of a kernel template <bool kPacked, bool kProb>.
#define ESCG_KERNEL2(K, packed, prob)                                         \
    ((packed) ? ((prob) ? (const void *)K<true, true>                         \
                        : (const void *)K<true, false>)                       \
              : ((prob) ? (const void *)K<false, true>                        \
                        : (const void *)K<false, false>))

// The persistent kernel for (S <= 7, dominance probabilities, list walk).
const void *persistent_kernel(bool packed, bool prob, bool list)
{
    static const void *const fns[8] = {
        (const void *)tiled_persistent_kernel<false, false, false>,
        (const void *)tiled_persistent_kernel<false, false, true>,
        (const void *)tiled_persistent_kernel<false, true, false>,
        (const void *)tiled_persistent_kernel<false, true, true>,
        (const void *)tiled_persistent_kernel<true, false, false>,
        (const void *)tiled_persistent_kernel<true, false, true>,
        (const void *)tiled_persistent_kernel<true, true, false>,
        (const void *)tiled_persistent_kernel<true, true, true>};
    return fns[(packed ? 4 : 0) | (prob ? 2 : 0) | (list ? 1 : 0)];
}

escg_status launch_lds_single(const JobDev &J, bool small, uint8_t *base,
                              hipStream_t st)
{
    const size_t lds = lds_job_bytes(J.L, J.S);
    const uint32_t nt = lds_threads(J.L);
    const void *fn = ESCG_KERNEL2(lds_single_kernel, small, J.ab != nullptr);
    allow_dynamic_lds(fn, lds);
    JobDev j = J;
    void *args[] = {&j, &base};
    return last_hip(hipLaunchKernel(fn, dim3(1), dim3(nt), args, lds, st));
}

escg_status launch_densities(const uint8_t *lat, uint32_t N, uint32_t S,
                             uint32_t *counts, hipStream_t st)
{
    const uint32_t ndw = N >> 2;
    const uint32_t blocks = std::max(1u, std::min(2048u, (ndw + 255) / 256));
    const uint32_t *l32 = reinterpret_cast<const uint32_t *>(lat);
    if (S <= 7)
        hipLaunchKernelGGL(densities_kernel<8>, dim3(blocks), dim3(256), 0, st,
                           l32, ndw, S, counts);
    else
        hipLaunchKernelGGL(densities_kernel<32>, dim3(blocks), dim3(256), 0,
                           st, l32, ndw, S, counts);
    return last_hip(hipGetLastError());
}

void launch_fill(uint32_t *p, size_t n, uint32_t v, hipStream_t st)
{
    const uint32_t blocks =
        (uint32_t)std::max<size_t>(1, std::min<size_t>(1024, (n + 255) / 256));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, st, p, n,
                       v);
}

void launch_copy(uint8_t *dst, const uint8_t *src, size_t bytes,
                 hipStream_t st)
{
    const size_t n = bytes >> 2;
    const uint32_t blocks =
        (uint32_t)std::max<size_t>(1, std::min<size_t>(4096, (n + 255) / 256));
    hipLaunchKernelGGL(copy_u32_kernel, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<uint32_t *>(dst),
                       reinterpret_cast<const uint32_t *>(src), n);
}

TileArgs tile_args(const escg_params *p, const Derived &d)
{
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seed = p->seed;
    a.dom_packed = d.packed;
    a.L = p->L;
    a.S = p->S;
    a.T1 = d.T1;
    a.T2 = d.T2;
    a.replica = p->replica;
    a.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
    a.ab = d.d_ab;
    for (int i = 0; i < 32; ++i)
        a.dom[i] = p->dom[i];
    return a;
}

void launch_tile_mcs(const TileArgs &a, bool small, hipStream_t st)
{
    const dim3 grid((a.L + kTileW - 1) / kTileW, (a.L + kTileH - 1) / kTileH);
    if (small)
        hipLaunchKernelGGL(tile_mcs_kernel<true>, grid, dim3(kTileThreads), 0,
                           st, a);
    else
        hipLaunchKernelGGL(tile_mcs_kernel<false>, grid, dim3(kTileThreads), 0,
                           st, a);
}

// Tile geometry for the persistent kernel: equal tiles, TW % 8 == 0, TH
// even and >= 4, all tiles co-resident.  Cost model: the busiest CU's region
// area (halo included) plus a fixed per-MCS synchronisation charge.
struct TiledPlan {
    bool ok = false;
    TileGeom G{};
    uint32_t threads = 0;
    size_t lds = 0;
    bool list = false; // quads by TileList (persistent kernel only)
};

// Quad iterations of a pass (oy = 0) on the busiest SIMD, with waves dealt
// to the four SIMDs of a CU in turn: a wave takes as many iterations as its
// busiest lane.  Column walk (TileWalk) or row-major list (TileList).
uint32_t walk_simd_load(const TileGeom &G, uint32_t nt, bool list)
{
    const uint32_t NJ = (G.TW + 16) >> 3, nbr = G.RH() >> 1;
    const uint32_t nq = nbr * NJ, Lb = G.L >> 1;
    const uint32_t rstep = std::min(nt / NJ, Lb);
    uint32_t simd[4] = {0, 0, 0, 0};
    for (uint32_t w = 0; w * 64 < nt; ++w) {
        uint32_t it = 0;
        for (uint32_t t = w * 64; t < std::min(nt, w * 64 + 64); ++t) {
            uint32_t n = 0;
            if (list)
                n = t < nq ? (nq - t + nt - 1) / nt : 0;
            else if (rstep && t / NJ < rstep)
                n = (nbr - t / NJ + rstep - 1) / rstep;
            it = std::max(it, n);
        }
        simd[w & 3] += it;
    }
    return std::max(std::max(simd[0], simd[1]), std::max(simd[2], simd[3]));
}

// Workgroup size for a tile (0: the tile is too wide): see tile_threads;
// the counts walk one column of dword pairs per thread (tile_count_sums), so
// TW / 8 threads are needed (TW / 4 for S > 7, tile_count_wide).
uint32_t tiled_threads(const TileGeom &G, uint32_t cap)
{
    const uint32_t nt = std::max(64u, tile_threads(G, cap));
    if (tile_threads(G, cap) == 0 || G.TW / 4 > nt)
        return 0;
    return nt;
}

// Automatic routing sends a single job with L % 8 == 0 to the persistent
// kernel from this side on.
constexpr uint32_t kPersistentMinL = 72;


// Launch choices that shape a plan: a forced tile shape (0, 0: free) and a
// workgroup size cap (0: 1024 for the persistent kernel, 512 per MCS).
struct PlanHints {
    uint32_t TH = 0, TW = 0, threads = 0;
};

PlanHints plan_hints(const escg_params *p)
{
    PlanHints h;
    h.TH = p->launch.tile_h;
    h.TW = p->launch.tile_w;
    h.threads = p->launch.threads;
    return h;
}

TiledPlan plan_tiled_uncached(uint32_t L, uint32_t S, const PlanHints &h)
{
    TiledPlan best;
    if (L % 8 != 0 || L < 16)
        return best;
    const DeviceInfo di = device_info();
    const int cus = std::max(1, di.cus);
    const size_t lds_max = di.lds_max ? di.lds_max : 65536;
    double best_cost = 1e300;
    const uint32_t oTH = h.TH, oTW = h.TW;
    const bool forced = oTH != 0 && valid_shape(L, oTH, oTW);
    if (oTH != 0 && !forced)
        return best;
    const uint32_t cap = h.threads ? h.threads : 1024u;
    for (uint32_t TW = 8; TW <= L; TW += 8) {
        if (L % TW || (forced && TW != oTW))
            continue;
        for (uint32_t TH = 4; TH <= L; TH += 2) {
            if (L % TH || (forced && TH != oTH))
                continue;
            TileGeom G{L, TH, TW, L / TH, L / TW};
            const uint32_t T = G.TY * G.TX;
            const size_t lds = G.region_bytes();
            if (lds + tiled_static_lds_bytes(S) + 64 > lds_max)
                continue;
            uint32_t nt = tiled_threads(G, cap);
            if (nt == 0)
                continue;
            // the balanced list walk where it lowers the busiest SIMD's load
            // (and its two region buffers fit)
            bool list = false;
            uint32_t load = walk_simd_load(G, nt, false);
            const bool list_lds =
                tiled_lds_bytes(G, true) + tiled_static_lds_bytes(S) + 64 <=
                lds_max;
            for (uint32_t n = cap & ~255u; n >= 256 && list_lds; n -= 256) {
                // ties: more waves
                if (!tile_list_fits(G, n) || G.TW / 4 > n)
                    continue;
                const uint32_t l = walk_simd_load(G, n, true);
                if (l < load) {
                    load = l;
                    nt = n;
                    list = true;
                }
            }
            const void *fn = persistent_kernel(S <= 7, false, list);
            const size_t lds_used = tiled_lds_bytes(G, list);
            allow_dynamic_lds(fn, lds_used);
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, fn, nt, lds_used) != hipSuccess)
                (void)hipGetLastError();
            if (per_cu < 1 || T > (uint32_t)cus * (uint32_t)per_cu)
                continue;
            const double waves = std::ceil((double)T / cus);
            const double cost = waves * (double)(TH + 8) * (TW + 16) + 8000.0;
            if (cost < best_cost) {
                best_cost = cost;
                best.ok = true;
                best.G = G;
                best.threads = nt;
                best.lds = lds_used;
                best.list = list;
            }
        }
    }
    return best;
}

using PlanKey = std::tuple<int, uint32_t, bool, uint32_t, uint32_t, uint32_t>;

TiledPlan plan_tiled(uint32_t L, uint32_t S, const PlanHints &h)
{
    static std::mutex mu;
    static std::map<PlanKey, TiledPlan> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const PlanKey key = std::make_tuple(dev, L, S <= 7, h.TH, h.TW, h.threads);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end())
            return it->second;
    }
    const TiledPlan plan = plan_tiled_uncached(L, S <= 7 ? 7u : 31u, h);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = plan;
    return plan;
}

// Tile geometry for the per-MCS kernel: equal tiles dividing L, TW % 8 == 0,
// TH even >= 4; no residency requirement.  Cost: halo-inflated area over
// the whole grid plus a per-tile launch charge, assuming the tiles spread
// evenly over the CUs.
TiledPlan plan_step_uncached(uint32_t L, uint32_t S, const PlanHints &h)
{
    TiledPlan best;
    if (L % 8 != 0 || L < 16)
        return best;
    const DeviceInfo di = device_info();
    const double cus = std::max(1, di.cus);
    const size_t lds_max = di.lds_max ? di.lds_max : 65536;
    double best_cost = 1e300;
    const uint32_t oTH = h.TH, oTW = h.TW;
    const bool forced = oTH != 0 && valid_shape(L, oTH, oTW);
    if (oTH != 0 && !forced)
        return best;
    const uint32_t cap = std::min(h.threads ? h.threads : 512u, 512u);
    for (uint32_t TW = 8; TW <= L && TW <= 512; TW += 8) {
        if (L % TW || (forced && TW != oTW))
            continue;
        for (uint32_t TH = 4; TH <= L && TH <= 512; TH += 2) {
            if (L % TH || (forced && TH != oTH))
                continue;
            TileGeom G{L, TH, TW, L / TH, L / TW};
            const size_t lds = G.region_bytes();
            if (lds + tiled_static_lds_bytes(S) + 64 > lds_max)
                continue;
            if (tiled_threads(G, cap) == 0)
                continue;
            const double T = (double)G.TY * G.TX;
            const double area = (double)(TH + 8) * (TW + 16);
            // work per CU, rounded up to whole tiles, plus a fixed cost per
            // tile for the load / table setup / store
            const double waves = std::ceil(T / (2.0 * cus));
            const double cost = waves * 2.0 * (area + 3000.0);
            if (cost < best_cost) {
                best_cost = cost;
                best.ok = true;
                best.G = G;
                best.threads = tiled_threads(G, cap);
                best.lds = lds;
            }
        }
    }
    return best;
}

TiledPlan plan_step(uint32_t L, uint32_t S, const PlanHints &h)
{
    static std::mutex mu;
    static std::map<PlanKey, TiledPlan> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const PlanKey key = std::make_tuple(dev, L, S <= 7, h.TH, h.TW, h.threads);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end())
            return it->second;
    }
    const TiledPlan plan = plan_step_uncached(L, S <= 7 ? 7u : 31u, h);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = plan;
    return plan;
}

StepArgs step_args(const escg_params *p, const Derived &d,
                   const TiledPlan &sp)
{
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seed = p->seed;
    a.G = sp.G;
    a.S = p->S;
    a.T1 = d.T1;
    a.T2 = d.T2;
    a.replica = p->replica;
    a.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
    a.ab = d.d_ab;
    for (int i = 0; i < 32; ++i)
        a.dom[i] = p->dom[i];
    return a;
}

void launch_step(const StepArgs &a, const TiledPlan &sp, bool small,
                 hipStream_t st)
{
    const uint32_t T = sp.G.TY * sp.G.TX;
    const void *fn = ESCG_KERNEL2(tiled_step_kernel, small, a.ab != nullptr);
    allow_dynamic_lds(fn, sp.lds);
    StepArgs aa = a;
    void *args[] = {&aa};
    (void)hipLaunchKernel(fn, dim3(T), dim3(sp.threads), args, sp.lds, st);
}

// Runs n_mcs MCS of a large lattice with the persistent kernel.  Returns
// ESCG_EUNSUPPORTED (nothing enqueued) if no plan fits or the cooperative
// launch is refused; the caller then uses the per-MCS tiled kernel.
// Bytes of the persistent kernel's exchange area for a plan: two slots per
// tile plus the abort word (padded).
size_t exchange_bytes(const TiledPlan &plan)
{
    const size_t T = (size_t)plan.G.TY * plan.G.TX;
    return (2 * T * plan.G.slot_dwords() + 64) * 4;
}

// area: exchange_bytes(plan) bytes of scratch for this launch (its tags and
// abort word are initialised here).  abort_out (device word, or null):
// receives the launch's abort word (nonzero if a tile gave up waiting for a
// neighbour, leaving the lattice invalid).
escg_status run_tiled_persistent(const escg_params *p, const Derived &d,
                                 const TiledPlan &plan, uint8_t *lattice,
                                 uint32_t mcs0, uint32_t n_mcs,
                                 uint32_t *counts, hipStream_t st,
                                 uint8_t *area, uint32_t *abort_out = nullptr)
{
    if (!plan.ok)
        return ESCG_EUNSUPPORTED;
    const TileGeom G = plan.G;
    const uint32_t T = G.TY * G.TX;
    const size_t slot_area = (size_t)T * G.slot_dwords(); // dwords
    uint8_t *scr = area;
    TiledArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lattice = lattice;
    a.exch = reinterpret_cast<uint32_t *>(scr);
    a.abort = a.exch + 2 * slot_area;
    a.xstride = (uint32_t)slot_area;
    a.counts = counts;
    a.seed = p->seed;
    a.G = G;
    a.S = p->S;
    a.T1 = d.T1;
    a.T2 = d.T2;
    a.replica = p->replica;
    a.mcs0 = mcs0;
    a.n_mcs = n_mcs;
    a.spin_limit = 1u << 22; // polls (seconds), then abort with an error
    a.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
    a.ab = d.d_ab;
    for (int i = 0; i < 32; ++i)
        a.dom[i] = p->dom[i];
    // slot 0 tagged 0, slot 1 tagged 1: neither matches its first use
    launch_fill(a.exch, slot_area, exch_tag(2) ^ 0x80808080u, st);
    launch_fill(a.exch + slot_area, slot_area, exch_tag(1) ^ 0x80808080u, st);
    launch_fill(a.abort, 64, 0, st);
    if (counts)
        launch_fill(counts + (p->S + 1), (size_t)n_mcs * (p->S + 1), 0, st);
    void *args[] = {&a};
    const void *fn = persistent_kernel(d.small, d.prob, plan.list);
    allow_dynamic_lds(fn, plan.lds);
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(T), dim3(plan.threads),
                                              args, (unsigned)plan.lds, st);
    escg_status s = ESCG_OK;
    if (e != hipSuccess) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "cooperative launch of %u x %u refused: %s", T,
                      plan.threads, hipGetErrorName(e));
        (void)hipGetLastError();
        s = ESCG_EUNSUPPORTED;
    }
    if (s == ESCG_OK && abort_out)
        launch_copy(reinterpret_cast<uint8_t *>(abort_out),
                    reinterpret_cast<const uint8_t *>(a.abort), 4, st);
    return s;
}

// Run-until on the persistent kernel: chunks of MCS with per-MCS counts;
// after each chunk the host reads the counts and finds the first MCS that
// meets the stop condition; if it lies inside the chunk, the chunk is re-run
// from its saved start up to that MCS, so the lattice is left exactly at the
// stopping state.  ESCG_EUNSUPPORTED (nothing but a lattice copy enqueued)
// if the persistent launch is refused on the first chunk.
escg_status run_until_persistent(const escg_params *p, const Derived &d,
                                 uint8_t *lattice, uint32_t mcs0,
                                 uint32_t max_mcs, uint32_t mode,
                                 uint32_t *d_result, hipStream_t st)
{
    const uint32_t L = p->L, S = p->S, N = L * L, W = S + 1;
    const uint32_t chunk_max = 1024;
    const TiledPlan plan = plan_tiled(L, S, plan_hints(p));
    if (!plan.ok)
        return ESCG_EUNSUPPORTED;
    // counts of a chunk, then the launches' abort words, then the saved
    // lattice, then the exchange area
    const size_t cnt_bytes = (size_t)(chunk_max + 1) * W * 4;
    const size_t lat_off = (cnt_bytes + 8 + 255) & ~(size_t)255;
    const size_t ex_off = (lat_off + N + 255) & ~(size_t)255;
    uint8_t *scr = nullptr;
    if (hipMallocAsync((void **)&scr, ex_off + exchange_bytes(plan), st) !=
        hipSuccess)
        return ESCG_ENOMEM;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(scr);
    uint32_t *abort_w = reinterpret_cast<uint32_t *>(scr + cnt_bytes);
    uint8_t *saved = scr + lat_off;
    uint8_t *area = scr + ex_off;
    std::vector<uint32_t> h((size_t)(chunk_max + 1) * W);
    std::vector<uint32_t> res(S + 3, 0);
    escg_status s = ESCG_OK;
    auto finish = [&](uint32_t flag, uint32_t t, const uint32_t *row) {
        res[0] = flag;
        res[1] = t;
        for (uint32_t v = 0; v < W; ++v)
            res[2 + v] = row[v];
        if (hipMemcpyAsync(d_result, res.data(), res.size() * 4,
                           hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            s = ESCG_EDEVICE;
    };
    // each launch's own abort word (abort_w[0]: the chunk, abort_w[1]: a
    // re-run) is read back with the counts; any nonzero word means that
    // launch gave up a neighbour wait and its lattice is invalid
    uint32_t aw[2] = {0, 0};
    auto fetch = [&](uint32_t rows) {
        return hipMemcpyAsync(h.data(), cnt, (size_t)rows * W * 4,
                              hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipMemcpyAsync(aw, abort_w, sizeof(aw), hipMemcpyDeviceToHost,
                              st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    auto timed_out = [&](uint32_t from, uint32_t n) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "persistent kernel aborted (neighbour wait timed out) "
                      "in MCS %u..%u", from, from + n - 1);
        return ESCG_ETIMEOUT;
    };
    // the input state
    launch_fill(cnt, W, 0, st);
    launch_fill(abort_w, 2, 0, st);
    s = launch_densities(lattice, N, S, cnt, st);
    if (s == ESCG_OK && !fetch(1))
        s = ESCG_EDEVICE;
    if (s == ESCG_OK && (mode != ESCG_STOP_NONE && stop_met(h.data(), S, mode))) {
        finish(1, 0, h.data());
        (void)hipFreeAsync(scr, st);
        return s;
    }
    uint32_t t = 0, chunk = 64;
    std::vector<uint32_t> last(h.begin(), h.begin() + W);
    while (s == ESCG_OK && t < max_mcs) {
        const uint32_t n = std::min(chunk, max_mcs - t);
        launch_copy(saved, lattice, N, st);
        s = run_tiled_persistent(p, d, plan, lattice, mcs0 + t, n, cnt, st,
                                 area, abort_w);
        if (s != ESCG_OK)
            break; // EUNSUPPORTED on the first chunk: the caller falls back
        if (!fetch(n + 1)) {
            s = ESCG_EDEVICE;
            break;
        }
        if (aw[0]) {
            s = timed_out(mcs0 + t, n);
            break;
        }
        uint32_t hit = 0;
        for (uint32_t k = 1; k <= n && mode != ESCG_STOP_NONE; ++k)
            if (stop_met(h.data() + (size_t)k * W, S, mode)) {
                hit = k;
                break;
            }
        if (hit) {
            if (hit < n) {
                launch_copy(lattice, saved, N, st);
                s = run_tiled_persistent(p, d, plan, lattice, mcs0 + t, hit,
                                         nullptr, st, area, abort_w + 1);
                if (s != ESCG_OK)
                    break;
                if (!fetch(0)) {
                    s = ESCG_EDEVICE;
                    break;
                }
                if (aw[1]) {
                    s = timed_out(mcs0 + t, hit);
                    break;
                }
            }
            finish(1, t + hit, h.data() + (size_t)hit * W);
            break;
        }
        std::copy(h.begin() + (size_t)n * W, h.begin() + (size_t)(n + 1) * W,
                  last.begin());
        t += n;
        chunk = std::min(chunk_max, chunk * 2);
        if (t == max_mcs)
            finish(0, max_mcs, last.data());
    }
    if (s == ESCG_OK && max_mcs == 0)
        finish(0, 0, last.data());
    (void)hipFreeAsync(scr, st);
    return s;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

// ---------------------------------------------------------------------------
// Several large lattices in one persistent launch (escg_step_batch)
// ---------------------------------------------------------------------------

// Workgroup size of the multi-job persistent kernel: one workgroup per CU
// (the kernel's registers allow no second one), the same for every job of a
// launch.
constexpr uint32_t kMultiThreads = 1024;

// Tile plan of a job inside a multi-job launch: the shape with the least
// workgroup time T * (4 * busiest-SIMD quad load per pass + a fixed
// exchange and barrier share per MCS), so large jobs take few, large tiles
// and leave CUs for other jobs.
TiledPlan plan_multi_uncached(uint32_t L, uint32_t S, const PlanHints &h)
{
    TiledPlan best;
    if (L % 8 != 0 || L < 16)
        return best;
    const DeviceInfo di = device_info();
    const size_t lds_max = di.lds_max ? di.lds_max : 65536;
    const uint32_t nt = kMultiThreads;
    const bool forced = h.TH != 0 && valid_shape(L, h.TH, h.TW);
    if (h.TH != 0 && !forced)
        return best;
    double best_cost = 1e300;
    for (uint32_t TW = 8; TW <= L; TW += 8) {
        if (L % TW || (forced && TW != h.TW))
            continue;
        for (uint32_t TH = 4; TH <= L; TH += 2) {
            if (L % TH || (forced && TH != h.TH))
                continue;
            const TileGeom G{L, TH, TW, L / TH, L / TW};
            const size_t lds = G.region_bytes();
            if (lds + tiled_static_lds_bytes(S) + 64 > lds_max ||
                G.TW / 4 > nt)
                continue;
            const bool list =
                tile_list_fits(G, nt) &&
                tiled_lds_bytes(G, true) + tiled_static_lds_bytes(S) + 64 <=
                    lds_max;
            if (!list && tiled_threads(G, nt) == 0)
                continue;
            const double T = (double)G.TY * G.TX;
            const double cost =
                T * (4.0 * walk_simd_load(G, nt, list) + 24.0);
            if (cost < best_cost) {
                best_cost = cost;
                best.ok = true;
                best.G = G;
                best.threads = nt;
                best.lds = tiled_lds_bytes(G, list);
                best.list = list;
            }
        }
    }
    return best;
}

TiledPlan plan_multi(uint32_t L, uint32_t S, const PlanHints &h)
{
    static std::mutex mu;
    static std::map<PlanKey, TiledPlan> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const PlanKey key = std::make_tuple(dev, L, S <= 7, h.TH, h.TW, 0u);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end())
            return it->second;
    }
    const TiledPlan plan = plan_multi_uncached(L, S <= 7 ? 7u : 31u, h);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = plan;
    return plan;
}

const void *persistent_multi_kernel(bool packed, bool prob, bool list)
{
    static const void *const fns[8] = {
        (const void *)tiled_persistent_multi_kernel<false, false, false>,
        (const void *)tiled_persistent_multi_kernel<false, false, true>,
        (const void *)tiled_persistent_multi_kernel<false, true, false>,
        (const void *)tiled_persistent_multi_kernel<false, true, true>,
        (const void *)tiled_persistent_multi_kernel<true, false, false>,
        (const void *)tiled_persistent_multi_kernel<true, false, true>,
        (const void *)tiled_persistent_multi_kernel<true, true, false>,
        (const void *)tiled_persistent_multi_kernel<true, true, true>};
    return fns[(packed ? 4 : 0) + (prob ? 2 : 0) + (list ? 1 : 0)];
}

// Workgroups that one multi-job launch may hold: what the device keeps
// resident at once for the kernel (with `lds` bytes of dynamic LDS), capped
// by the caller's max_wgs (0: no cap).
uint32_t multi_capacity(const void *fn, size_t lds, uint32_t max_wgs)
{
    allow_dynamic_lds(fn, lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn,
                                                     kMultiThreads, lds) !=
        hipSuccess)
        (void)hipGetLastError();
    const DeviceInfo di = device_info();
    uint32_t cap = (uint32_t)std::max(0, per_cu) * (uint32_t)std::max(0, di.cus);
    if (max_wgs)
        cap = std::min(cap, max_wgs);
    return cap;
}

// One multi-job launch of the jobs `idx` (same kernel instantiation; their
// padded workgroup ranges already fit `cap`): job table, exchange areas and
// abort words in one stream-ordered allocation.
escg_status launch_multi(const std::vector<uint32_t> &idx,
                         const std::vector<TiledPlan> &plans,
                         const escg_params *P, uint8_t *const *lats,
                         const uint32_t *mcs0, const uint32_t *nm, bool packed,
                         bool prob, bool list, hipStream_t st)
{
    const uint32_t m = (uint32_t)idx.size();
    const uint32_t Sp = packed ? 8u : 32u, abw = 2u * Sp * Sp;
    std::vector<TiledArgs> tbl(m);
    std::vector<uint32_t> ab_all;
    if (prob)
        ab_all.resize((size_t)m * abw);
    size_t slot_dw = 0, lds = 0;
    uint32_t wg = 0;
    for (uint32_t i = 0; i < m; ++i) {
        const uint32_t j = idx[i];
        const escg_params *p = &P[j];
        const TiledPlan &pl = plans[j];
        const Derived d = derive(p);
        if (prob) {
            const std::vector<uint32_t> ab =
                selection_thresholds(p, d.T1, d.T2, Sp);
            std::copy(ab.begin(), ab.end(), ab_all.begin() + (size_t)i * abw);
        }
        const uint32_t T = pl.G.TY * pl.G.TX;
        if (T % 8u == 0)
            wg = (wg + 7u) & ~7u; // XCD bands (xcd_tile) need wg0 % 8 == 0
        TiledArgs &a = tbl[i];
        std::memset(&a, 0, sizeof(a));
        a.lattice = lats[j];
        a.seed = p->seed;
        a.G = pl.G;
        a.S = p->S;
        a.T1 = d.T1;
        a.T2 = d.T2;
        a.replica = p->replica;
        a.mcs0 = mcs0[j];
        a.n_mcs = nm[j];
        a.spin_limit = 1u << 22; // polls (seconds), then abort with an error
        a.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
        a.wg0 = wg;
        for (int q = 0; q < 32; ++q)
            a.dom[q] = p->dom[q];
        a.xstride = (uint32_t)slot_dw; // offset of slot 0, set below
        slot_dw += (size_t)T * pl.G.slot_dwords();
        wg += T;
        lds = std::max(lds, pl.lds);
    }
    // layout: table | thresholds | slot 0 of every job | slot 1 of every
    // job | abort words (64 B apart)
    const size_t tbl_bytes = (sizeof(TiledArgs) * m + 255) & ~(size_t)255;
    const size_t ab_bytes = (ab_all.size() * 4 + 255) & ~(size_t)255;
    const size_t slot_bytes = (slot_dw * 4 + 255) & ~(size_t)255;
    const size_t total = tbl_bytes + ab_bytes + 2 * slot_bytes + 64 * (size_t)m;
    uint8_t *dev = nullptr;
    if (hipMallocAsync((void **)&dev, total, st) != hipSuccess)
        return ESCG_ENOMEM;
    uint32_t *slot0 = reinterpret_cast<uint32_t *>(dev + tbl_bytes + ab_bytes);
    uint32_t *abort0 =
        reinterpret_cast<uint32_t *>(dev + tbl_bytes + ab_bytes + 2 * slot_bytes);
    for (uint32_t i = 0; i < m; ++i) {
        TiledArgs &a = tbl[i];
        a.exch = slot0 + a.xstride;
        a.xstride = (uint32_t)(slot_bytes / 4);
        a.abort = abort0 + 16 * i;
        a.ab = prob ? reinterpret_cast<const uint32_t *>(dev + tbl_bytes) +
                          (size_t)i * abw
                    : nullptr;
    }
    // slot 0 tagged 0, slot 1 tagged 1: neither matches its first use
    launch_fill(slot0, slot_bytes / 4, exch_tag(2) ^ 0x80808080u, st);
    launch_fill(slot0 + slot_bytes / 4, slot_bytes / 4,
                exch_tag(1) ^ 0x80808080u, st);
    launch_fill(abort0, 16 * (size_t)m, 0, st);
    escg_status s = ESCG_OK;
    if (hipMemcpyAsync(dev, tbl.data(), sizeof(TiledArgs) * m,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        (prob && hipMemcpyAsync(dev + tbl_bytes, ab_all.data(),
                                ab_all.size() * 4, hipMemcpyHostToDevice,
                                st) != hipSuccess))
        s = last_hip(hipGetLastError());
    if (s == ESCG_OK) {
        const void *fn = persistent_multi_kernel(packed, prob, list);
        allow_dynamic_lds(fn, lds);
        const TiledArgs *tp = reinterpret_cast<const TiledArgs *>(dev);
        uint32_t nj = m;
        void *args[] = {&tp, &nj};
        s = last_hip(hipLaunchKernel(fn, dim3(wg), dim3(kMultiThreads), args,
                                     lds, st));
    }
    (void)hipFreeAsync(dev, st);
    return s;
}

// The persistent part of escg_step_batch: jobs with a multi-job plan run in
// launches of whole jobs, grouped by kernel instantiation, each launch
// holding at most `cap` workgroups; jobs left over (no plan, or more tiles
// than one launch holds) are returned in `rest`.  dry_run: plan only (the
// same `rest`, nothing enqueued).
escg_status step_batch_persistent(uint32_t n, const escg_params *P,
                                  uint8_t *const *lats, const uint32_t *mcs0,
                                  const uint32_t *nm, uint32_t max_wgs,
                                  hipStream_t st, std::vector<uint32_t> &rest,
                                  bool &launched, bool dry_run)
{
    launched = false;
    std::vector<TiledPlan> plans(n);
    std::vector<uint32_t> keys(n, 8u);
    for (uint32_t j = 0; j < n; ++j) {
        if (nm[j] == 0)
            continue;
        plans[j] = plan_multi(P[j].L, P[j].S, plan_hints(&P[j]));
        if (!plans[j].ok) {
            rest.push_back(j);
            continue;
        }
        keys[j] = (P[j].S <= 7 ? 4u : 0u) + (P[j].dom_prob ? 2u : 0u) +
                  (plans[j].list ? 1u : 0u);
    }
    for (uint32_t key = 0; key < 8; ++key) {
        const bool packed = key & 4u, prob = key & 2u, list = key & 1u;
        // longest chunks first, so a launch's jobs end at similar times
        std::vector<uint32_t> idx;
        size_t lds = 0;
        for (uint32_t j = 0; j < n; ++j)
            if (keys[j] == key) {
                idx.push_back(j);
                lds = std::max(lds, plans[j].lds);
            }
        if (idx.empty())
            continue;
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
            return nm[a] > nm[b];
        });
        const uint32_t cap = multi_capacity(
            persistent_multi_kernel(packed, prob, list), lds, max_wgs);
        std::vector<uint32_t> cur;
        uint32_t wg = 0;
        for (size_t k = 0; k <= idx.size(); ++k) {
            uint32_t T = 0, need = 0;
            if (k < idx.size()) {
                const TileGeom &G = plans[idx[k]].G;
                T = G.TY * G.TX;
                if (T > cap) {
                    rest.push_back(idx[k]);
                    continue;
                }
                need = ((T % 8u == 0) ? ((wg + 7u) & ~7u) : wg) + T;
            }
            if (k == idx.size() || need > cap) {
                if (!cur.empty() && !dry_run) {
                    const escg_status s = launch_multi(
                        cur, plans, P, lats, mcs0, nm, packed, prob, list, st);
                    if (s != ESCG_OK)
                        return s;
                    launched = true;
                }
                cur.clear();
                wg = 0;
                if (k == idx.size())
                    break;
                need = T;
            }
            cur.push_back(idx[k]);
            wg = need;
        }
    }
    return ESCG_OK;
}

// The path of a single job (escg_step_mcs, escg_run_until_extinction) from
// its launch choice: forced, or automatic (persistent for L % 8 == 0 and
// L >= kPersistentMinL when a resident plan exists, else the whole lattice
// in one workgroup's LDS when it fits, else per-MCS tiled launches).
enum class Route { kLds, kTiled, kPersistent, kUnsupported };

Route choose_route(const escg_params *p)
{
    const uint32_t L = p->L, S = p->S;
    const bool fits_lds = L <= lds_max_L(S);
    const auto plan_ok = [&] {
        return (L & 7u) == 0 && plan_tiled(L, S, plan_hints(p)).ok;
    };
    switch (p->launch.route) {
    case ESCG_ROUTE_LDS:
        return fits_lds ? Route::kLds : Route::kUnsupported;
    case ESCG_ROUTE_TILED:
        return Route::kTiled;
    case ESCG_ROUTE_PERSISTENT:
        return plan_ok() ? Route::kPersistent : Route::kUnsupported;
    default:
        if ((L & 7u) == 0 && L >= kPersistentMinL && plan_ok())
            return Route::kPersistent;
        return fits_lds ? Route::kLds : Route::kTiled;
    }
}



} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *escg_last_error(void) { return g_last_error; }

const char *escg_status_str(escg_status s)
{
    switch (s) {
    case ESCG_OK: return "ok";
    case ESCG_EINVAL: return "invalid argument";
    case ESCG_ENOMEM: return "device allocation failed";
    case ESCG_EDEVICE: return "HIP runtime error";
    case ESCG_EUNSUPPORTED: return "unsupported request";
    case ESCG_ETIMEOUT: return "device wait timed out";
    default: return "unknown status";
    }
}

escg_status escg_circulant_dom(uint32_t S, uint32_t kmask, uint32_t *h_dom)
{
    if (!h_dom || S < 1 || S > ESCG_MAX_SPECIES)
        return ESCG_EINVAL;
    for (int i = 0; i < 32; ++i)
        h_dom[i] = 0;
    for (uint32_t i = 1; i <= S; ++i)
        for (uint32_t j = 1; j <= S; ++j) {
            const uint32_t k = (j + S - i) % S;
            if (k != 0 && ((kmask >> k) & 1u))
                h_dom[i] |= 1u << j;
        }
    return ESCG_OK;
}

escg_status escg_dom_from_matrix(uint32_t S, const uint8_t *h_D,
                                 uint32_t *h_dom)
{
    if (!h_dom || !h_D || S < 1 || S > ESCG_MAX_SPECIES)
        return ESCG_EINVAL;
    for (int i = 0; i < 32; ++i)
        h_dom[i] = 0;
    for (uint32_t i = 1; i <= S; ++i)
        for (uint32_t j = 1; j <= S; ++j)
            if (h_D[(i - 1) * S + (j - 1)])
                h_dom[i] |= 1u << j;
    return ESCG_OK;
}

escg_status escg_eps_from_mobility(double M, uint32_t L, double *eps)
{
    if (!eps || L == 0 || !(M >= 0) || !std::isfinite(M))
        return ESCG_EINVAL;
    *eps = M * (double)L * (double)L / 2.0;
    return ESCG_OK;
}

escg_status escg_thresholds(const escg_params *p, uint32_t *T1, uint32_t *T2)
{
    if (!p || !T1 || !T2)
        return ESCG_EINVAL;
    const double ex = p->rate_ex, sel = p->rate_sel, rep = p->rate_rep;
    if (!(ex >= 0 && sel >= 0 && rep >= 0) || !std::isfinite(ex) ||
        !std::isfinite(sel) || !std::isfinite(rep))
        return ESCG_EINVAL;
    const double tot = (ex + sel) + rep;
    if (!(tot > 0))
        return ESCG_EINVAL;
    *T1 = (uint32_t)std::floor(std::ldexp(ex / tot, 24));
    *T2 = (uint32_t)std::floor(std::ldexp((ex + sel) / tot, 24));
    return ESCG_OK;
}

escg_status escg_init(const escg_params *p, uint8_t *d_lattice, void *stream)
{
    escg_status s = validate(p);
    if (s != ESCG_OK)
        return s;
    if (!d_lattice || !aligned4(d_lattice))
        return ESCG_EINVAL;
    const uint32_t ndw = (uint32_t)(((uint64_t)p->L * p->L) >> 2);
    const uint32_t blocks = std::max(1u, std::min(8192u, (ndw + 255) / 256));
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, S_(stream),
                       reinterpret_cast<uint32_t *>(d_lattice), ndw, p->S,
                       p->seed, p->replica);
    return last_hip(hipGetLastError());
}

escg_status escg_densities(const escg_params *p, const uint8_t *d_lattice,
                           uint32_t *d_counts, void *stream)
{
    escg_status s = validate(p);
    if (s != ESCG_OK)
        return s;
    if (!d_lattice || !d_counts || !aligned4(d_lattice))
        return ESCG_EINVAL;
    hipStream_t st = S_(stream);
    launch_fill(d_counts, p->S + 1, 0, st);
    return launch_densities(d_lattice, p->L * p->L, p->S, d_counts, st);
}

// escg_step_mcs with its scratch from `ar` (stream-ordered or the static
// array).  With a fixed arena every byte the call will take is checked
// against it before anything is enqueued.
escg_status step_mcs(const escg_params *p, uint8_t *d_lattice, uint32_t mcs0,
                     uint32_t n_mcs, uint32_t *d_counts, Arena &ar)
{
    escg_status s = validate(p);
    if (s != ESCG_OK)
        return s;
    if (!d_lattice || !aligned4(d_lattice))
        return ESCG_EINVAL;
    hipStream_t st = ar.st;
    Derived d = derive(p);
    const uint32_t L = p->L, S = p->S, N = L * L;
    const Route r = choose_route(p);
    if (r == Route::kUnsupported)
        return ESCG_EUNSUPPORTED;
    const bool persistent = r == Route::kPersistent;
    const TiledPlan plan =
        persistent ? plan_tiled(L, S, plan_hints(p)) : TiledPlan{};
    if (ar.base) {
        const size_t ab = d.prob ? Arena::round(d.ab.size() * 4) : 0;
        const size_t rest =
            r == Route::kLds ? 0
                             : Arena::round(persistent
                                                ? std::max<size_t>(
                                                      exchange_bytes(plan), N)
                                                : N);
        if (n_mcs > 0 && ab + rest > ar.cap) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "needs %zu bytes of static scratch, %zu available",
                          ab + rest, ar.cap);
            return ESCG_ENOMEM;
        }
    }
    if (d.prob) {
        s = upload_words(d.ab, ar, &d.d_ab);
        if (s != ESCG_OK)
            return s;
    }
    if (r == Route::kLds) {
        JobDev J = make_job(p, d, 0, mcs0, n_mcs, ESCG_STOP_NONE, 0, d_counts,
                            nullptr, 0);
        g_last_route = ESCG_ROUTE_LDS;
        return launch_lds_single(J, d.small, d_lattice, st);
    }
    if (d_counts) {
        launch_fill(d_counts, (size_t)(n_mcs + 1) * (S + 1), 0, st);
        s = launch_densities(d_lattice, N, S, d_counts, st);
        if (s != ESCG_OK)
            return s;
    }
    if (n_mcs == 0)
        return ESCG_OK;
    // one span serves the exchange area or, if the cooperative launch is
    // refused, the ping-pong lattice of the per-MCS launches
    void *span = nullptr;
    s = ar.take(persistent ? std::max<size_t>(exchange_bytes(plan), N) : N,
                &span);
    if (s != ESCG_OK)
        return s;
    if (persistent) {
        s = run_tiled_persistent(p, d, plan, d_lattice, mcs0, n_mcs, d_counts,
                                 st, static_cast<uint8_t *>(span));
        if (s != ESCG_EUNSUPPORTED) {
            g_last_route = ESCG_ROUTE_PERSISTENT;
            return s;
        }
        s = ESCG_OK; // refused at launch: one tiled launch per MCS instead
    }
    g_last_route = ESCG_ROUTE_TILED;
    uint8_t *other = static_cast<uint8_t *>(span);
    uint8_t *cur = d_lattice, *nxt = other;
    const TiledPlan sp = plan_step(L, S, plan_hints(p));
    if (sp.ok) {
        StepArgs a = step_args(p, d, sp);
        for (uint32_t k = 0; k < n_mcs; ++k) {
            a.src = cur;
            a.dst = nxt;
            a.t = mcs0 + k;
            a.counts =
                d_counts ? d_counts + (size_t)(k + 1) * (S + 1) : nullptr;
            launch_step(a, sp, d.small, st);
            std::swap(cur, nxt);
        }
    } else {
        TileArgs a = tile_args(p, d);
        for (uint32_t k = 0; k < n_mcs; ++k) {
            a.src = cur;
            a.dst = nxt;
            a.t = mcs0 + k;
            a.counts =
                d_counts ? d_counts + (size_t)(k + 1) * (S + 1) : nullptr;
            launch_tile_mcs(a, d.small, st);
            std::swap(cur, nxt);
        }
    }
    if (cur != d_lattice)
        launch_copy(d_lattice, cur, N, st);
    return last_hip(hipGetLastError());
}

escg_status escg_step_mcs(const escg_params *p, uint8_t *d_lattice,
                          uint32_t mcs0, uint32_t n_mcs, uint32_t *d_counts,
                          void *stream)
{
    Arena ar(S_(stream));
    return step_mcs(p, d_lattice, mcs0, n_mcs, d_counts, ar);
}

escg_status escg_step_mcs_static(const escg_params *p, uint8_t *d_lattice,
                                 uint32_t mcs0, uint32_t n_mcs,
                                 uint32_t *d_counts, void *stream)
{
    uint8_t *base = nullptr;
    escg_status s = static_scratch(&base);
    if (s != ESCG_OK)
        return s;
    Arena ar(S_(stream), base, ESCG_STATIC_SCRATCH_BYTES);
    return step_mcs(p, d_lattice, mcs0, n_mcs, d_counts, ar);
}

escg_status escg_run_until_extinction(const escg_params *p, uint8_t *d_lattice,
                                      uint32_t mcs0, uint32_t max_mcs,
                                      uint32_t mode, uint32_t *d_result,
                                      void *stream)
{
    escg_status s = validate(p);
    if (s != ESCG_OK)
        return s;
    if (!d_lattice || !d_result || !aligned4(d_lattice) ||
        mode > ESCG_STOP_NONE)
        return ESCG_EINVAL;
    hipStream_t st = S_(stream);
    Derived d = derive(p);
    Arena ar(st);
    if (d.prob) {
        s = upload_words(d.ab, ar, &d.d_ab);
        if (s != ESCG_OK)
            return s;
    }
    const uint32_t L = p->L, S = p->S, N = L * L;
    const Route r = choose_route(p);
    if (r == Route::kUnsupported)
        return ESCG_EUNSUPPORTED;
    if (r == Route::kPersistent) {
        s = run_until_persistent(p, d, d_lattice, mcs0, max_mcs, mode,
                                 d_result, st);
        if (s != ESCG_EUNSUPPORTED) {
            g_last_route = ESCG_ROUTE_PERSISTENT;
            return s;
        }
        s = ESCG_OK; // refused at launch: one tiled launch per MCS instead
    }
    if (r == Route::kLds) {
        JobDev J = make_job(p, d, 0, mcs0, max_mcs, mode, 0, nullptr,
                            d_result, S + 3);
        g_last_route = ESCG_ROUTE_LDS;
        return launch_lds_single(J, d.small, d_lattice, st);
    }
    g_last_route = ESCG_ROUTE_TILED;
    // Large lattice: tile MCS launches with a device stop flag, polled by
    // the host every chunk.
    uint8_t *scr = nullptr;
    const size_t flags_off = ((size_t)N + 255) & ~(size_t)255;
    if (hipMallocAsync((void **)&scr, flags_off + 512, st) != hipSuccess)
        return ESCG_ENOMEM;
    uint8_t *other = scr;
    uint32_t *stw = reinterpret_cast<uint32_t *>(scr + flags_off);
    uint32_t *cnt2 = stw + 4; // two rows of 32 counts
    launch_fill(stw, 4 + 64, 0, st);
    s = launch_densities(d_lattice, N, S, cnt2, st);
    if (s != ESCG_OK)
        return s;
    hipLaunchKernelGGL(check_stop_kernel, dim3(1), dim3(64), 0, st, stw, cnt2,
                       0u, S, mode, 0u, d_result);
    TileArgs a = tile_args(p, d);
    a.done = stw;
    const TiledPlan sp = plan_step(L, S, plan_hints(p));
    StepArgs sa = sp.ok ? step_args(p, d, sp) : StepArgs{};
    sa.done = stw;
    uint8_t *cur = d_lattice, *nxt = other;
    uint32_t launched = 0;
    const uint32_t chunk = 32;
    while (launched < max_mcs) {
        uint32_t done = 0;
        if (hipMemcpyAsync(&done, stw, sizeof(done), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            (void)hipFreeAsync(scr, st);
            return ESCG_EDEVICE;
        }
        if (done)
            break;
        const uint32_t n = std::min(chunk, max_mcs - launched);
        for (uint32_t k = 0; k < n; ++k) {
            const uint32_t t = launched + k;
            if (sp.ok) {
                sa.src = cur;
                sa.dst = nxt;
                sa.t = mcs0 + t;
                sa.counts = cnt2 + ((t + 1) & 1u) * 32;
                launch_step(sa, sp, d.small, st);
            } else {
                a.src = cur;
                a.dst = nxt;
                a.t = mcs0 + t;
                a.counts = cnt2 + ((t + 1) & 1u) * 32;
                launch_tile_mcs(a, d.small, st);
            }
            hipLaunchKernelGGL(check_stop_kernel, dim3(1), dim3(64), 0, st,
                               stw, cnt2, (t + 1) & 1u, S, mode, t + 1,
                               d_result);
            std::swap(cur, nxt);
        }
        launched += n;
    }
    if (cur != d_lattice)
        launch_copy(d_lattice, cur, N, st);
    s = last_hip(hipGetLastError());
    (void)hipFreeAsync(scr, st);
    return s;
}

uint32_t escg_batch_max_L(uint32_t S)
{
    return (S < 1 || S > ESCG_MAX_SPECIES) ? 0u : lds_max_L(S);
}

uint32_t escg_last_route(void) { return g_last_route; }

escg_status escg_tile_plan(const escg_params *p, uint32_t persistent,
                           uint32_t *TH, uint32_t *TW, uint32_t *threads)
{
    escg_status s = validate(p);
    if (s != ESCG_OK)
        return s;
    if (!TH || !TW || !threads)
        return ESCG_EINVAL;
    if (persistent > 2)
        return ESCG_EINVAL;
    const PlanHints h = plan_hints(p);
    const TiledPlan tp = persistent == 2   ? plan_multi(p->L, p->S, h)
                         : persistent == 1 ? plan_tiled(p->L, p->S, h)
                                           : plan_step(p->L, p->S, h);
    if (!tp.ok)
        return ESCG_EUNSUPPORTED;
    *TH = tp.G.TH;
    *TW = tp.G.TW;
    *threads = tp.threads;
    return ESCG_OK;
}

escg_status escg_async_status(int reset)
{
    if (hipDeviceSynchronize() != hipSuccess)
        return last_hip(hipGetLastError());
    uint32_t v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_async_error), sizeof(v), 0,
                            hipMemcpyDeviceToHost) != hipSuccess)
        return last_hip(hipGetLastError());
    if (reset && v) {
        const uint32_t z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_async_error), &z, sizeof(z), 0,
                              hipMemcpyHostToDevice) != hipSuccess)
            return last_hip(hipGetLastError());
    }
    return v ? ESCG_ETIMEOUT : ESCG_OK;
}

escg_status escg_step_batch(uint32_t n, const escg_params *h_params,
                            uint8_t *const *h_lattices, const uint32_t *h_mcs0,
                            const uint32_t *h_n_mcs, void *stream)
{
    if (n == 0)
        return ESCG_OK;
    if (!h_params || !h_lattices || !h_mcs0 || !h_n_mcs)
        return ESCG_EINVAL;
    std::vector<std::pair<uintptr_t, uintptr_t>> spans(n);
    for (uint32_t j = 0; j < n; ++j) {
        const escg_params *p = &h_params[j];
        escg_status s = validate(p);
        if (s != ESCG_OK)
            return s;
        if (!h_lattices[j] || !aligned4(h_lattices[j]))
            return ESCG_EINVAL;
        const uintptr_t a = reinterpret_cast<uintptr_t>(h_lattices[j]);
        spans[j] = {a, a + (uintptr_t)p->L * p->L};
    }
    std::sort(spans.begin(), spans.end());
    for (uint32_t j = 1; j < n; ++j)
        if (spans[j].first < spans[j - 1].second)
            return ESCG_EINVAL; // lattices overlap
    hipStream_t st = S_(stream);
    // persistent multi-job launches unless the per-MCS path is asked for;
    // the jobs they cannot take keep their MCS count for per-MCS launches.
    // Everything is planned before anything is enqueued.
    const bool multi = h_params[0].launch.route != ESCG_ROUTE_TILED;
    const uint32_t max_wgs = h_params[0].launch.max_wgs;
    std::vector<uint32_t> nm(h_n_mcs, h_n_mcs + n);
    if (multi) {
        std::vector<uint32_t> rest;
        bool none = false;
        const escg_status s = step_batch_persistent(
            n, h_params, h_lattices, h_mcs0, h_n_mcs, max_wgs, st, rest, none,
            true);
        if (s != ESCG_OK)
            return s;
        std::vector<uint32_t> left(n, 0u);
        for (uint32_t j : rest)
            left[j] = h_n_mcs[j];
        nm = left;
    }
    // per-MCS plans of the jobs left to that path (a tile shape asked for
    // that only the persistent path can take yields to the planner's)
    std::vector<TiledPlan> plans(n);
    for (uint32_t j = 0; j < n; ++j) {
        if (nm[j] == 0)
            continue;
        const escg_params *p = &h_params[j];
        plans[j] = plan_step(p->L, p->S, plan_hints(p));
        if (!plans[j].ok && p->launch.tile_h) {
            PlanHints h = plan_hints(p);
            h.TH = h.TW = 0;
            plans[j] = plan_step(p->L, p->S, h);
        }
        if (!plans[j].ok) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "job %u: L = %u has no tile plan (needs L %% 8 == 0, "
                          "L >= 16)", j, p->L);
            return ESCG_EUNSUPPORTED;
        }
    }
    bool persistent = false;
    if (multi) {
        std::vector<uint32_t> rest;
        const escg_status s = step_batch_persistent(
            n, h_params, h_lattices, h_mcs0, h_n_mcs, max_wgs, st, rest,
            persistent, false);
        if (s != ESCG_OK)
            return s;
    }
    h_n_mcs = nm.data();
    for (int packed = 1; packed >= 0; --packed) {
        // jobs of this kernel instantiation, longest chunk first, so the jobs
        // still running at step k are a prefix of the table
        std::vector<uint32_t> idx;
        for (uint32_t j = 0; j < n; ++j)
            if ((h_params[j].S <= 7) == (packed == 1) && h_n_mcs[j] > 0)
                idx.push_back(j);
        if (idx.empty())
            continue;
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
            return h_n_mcs[a] > h_n_mcs[b];
        });
        const uint32_t m = (uint32_t)idx.size();
        std::vector<BatchStepJob> tbl(m);
        std::vector<uint32_t> wg_end(m);
        size_t scratch_bytes = 0, lds = 0;
        uint32_t wg = 0;
        // with any job carrying dominance probabilities the group runs the
        // probabilistic kernel; the others then get thresholds from their
        // 0/1 matrix (the same rule)
        bool prob = false;
        for (uint32_t j : idx)
            prob = prob || h_params[j].dom_prob != nullptr;
        const uint32_t Sp = packed ? 8u : 32u, abw = 2u * Sp * Sp;
        std::vector<uint32_t> ab_all;
        if (prob)
            ab_all.resize((size_t)m * abw);
        for (uint32_t i = 0; i < m; ++i) {
            const uint32_t j = idx[i];
            const escg_params *p = &h_params[j];
            const Derived d = derive(p);
            if (prob) {
                const std::vector<uint32_t> ab =
                    selection_thresholds(p, d.T1, d.T2);
                std::copy(ab.begin(), ab.end(),
                          ab_all.begin() + (size_t)i * abw);
            }
            BatchStepJob &J = tbl[i];
            std::memset(&J, 0, sizeof(J));
            J.lattice = h_lattices[j];
            J.seed = p->seed;
            J.G = plans[j].G;
            J.S = p->S;
            J.T1 = d.T1;
            J.T2 = d.T2;
            J.replica = p->replica;
            J.t0 = h_mcs0[j];
            J.wg0 = wg;
            J.moore = (p->flags & ESCG_FLAG_MOORE) ? 1u : 0u;
            for (int q = 0; q < 32; ++q)
                J.dom[q] = p->dom[q];
            wg += J.G.TY * J.G.TX;
            wg_end[i] = wg;
            scratch_bytes += ((size_t)p->L * p->L + 255) & ~(size_t)255;
            lds = std::max(lds, plans[j].lds);
        }
        const size_t tbl_bytes = (sizeof(BatchStepJob) * m + 255) & ~(size_t)255;
        const size_t ab_bytes = ab_all.size() * 4;
        uint8_t *dev = nullptr;
        if (hipMallocAsync((void **)&dev,
                           tbl_bytes + ((ab_bytes + 255) & ~(size_t)255) +
                               scratch_bytes,
                           st) !=
            hipSuccess)
            return ESCG_ENOMEM;
        const uint32_t *d_ab = reinterpret_cast<const uint32_t *>(dev + tbl_bytes);
        size_t off = tbl_bytes + ((ab_bytes + 255) & ~(size_t)255);
        for (uint32_t i = 0; i < m; ++i) {
            tbl[i].scratch = dev + off;
            tbl[i].ab = prob ? d_ab + (size_t)i * abw : nullptr;
            off += ((size_t)tbl[i].G.L * tbl[i].G.L + 255) & ~(size_t)255;
        }
        if (prob &&
            hipMemcpyAsync(dev + tbl_bytes, ab_all.data(), ab_bytes,
                           hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipFreeAsync(dev, st);
            return ESCG_EDEVICE;
        }
        BatchStepJob *d_tbl = reinterpret_cast<BatchStepJob *>(dev);
        if (hipMemcpyAsync(d_tbl, tbl.data(), sizeof(BatchStepJob) * m,
                           hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipFreeAsync(dev, st);
            return ESCG_EDEVICE;
        }
        const void *fn =
            ESCG_KERNEL2(tiled_step_batch_kernel, packed == 1, prob);
        allow_dynamic_lds(fn, lds);
        uint32_t active = m;
        const uint32_t steps = h_n_mcs[idx[0]];
        for (uint32_t k = 0; k < steps; ++k) {
            while (active > 0 && h_n_mcs[idx[active - 1]] <= k)
                --active;
            const uint32_t grid = wg_end[active - 1];
            const BatchStepJob *tp = d_tbl;
            uint32_t na = active, kk = k;
            void *args[] = {&tp, &na, &kk};
            (void)hipLaunchKernel(fn, dim3(grid), dim3(kBatchStepThreads), args,
                                  lds, st);
        }
        // an odd number of steps leaves the state in the scratch buffer
        for (uint32_t i = 0; i < m; ++i)
            if (h_n_mcs[idx[i]] & 1u)
                launch_copy(tbl[i].lattice, tbl[i].scratch,
                            (size_t)tbl[i].G.L * tbl[i].G.L, st);
        escg_status s = last_hip(hipGetLastError());
        (void)hipFreeAsync(dev, st);
        if (s != ESCG_OK)
            return s;
    }
    g_last_route = persistent ? ESCG_ROUTE_PERSISTENT : ESCG_ROUTE_TILED;
    return ESCG_OK;
}

escg_status escg_batch_run(uint32_t n, const escg_params *h_params,
                           const uint64_t *h_offsets, uint8_t *d_lattices,
                           const uint32_t *h_mcs0, const uint32_t *h_max_mcs,
                           uint32_t mode, uint32_t init, uint32_t *d_results,
                           void *stream)
{
    if (n == 0)
        return ESCG_OK;
    if (!h_params || !h_offsets || !d_lattices || !h_max_mcs || !d_results ||
        mode > ESCG_STOP_NONE || !aligned4(d_lattices))
        return ESCG_EINVAL;
    std::vector<JobDev> jobs(n);
    std::vector<uint32_t> order(n);
    uint32_t Lmax = 0;
    size_t lds_need = 0;
    bool all_small = true;
    std::vector<std::pair<uint64_t, uint64_t>> spans(n);
    for (uint32_t j = 0; j < n; ++j) {
        const escg_params *p = &h_params[j];
        escg_status s = validate(p);
        if (s != ESCG_OK)
            return s;
        if (p->L > lds_max_L(p->S))
            return ESCG_EINVAL;
        if (h_offsets[j] & 3u)
            return ESCG_EINVAL;
        const Derived d = derive(p);
        all_small = all_small && d.small;
        Lmax = std::max(Lmax, p->L);
        lds_need = std::max(lds_need, lds_job_bytes(p->L, p->S));
        jobs[j] = make_job(p, d, h_offsets[j], h_mcs0 ? h_mcs0[j] : 0,
                           h_max_mcs[j], mode, init ? 1u : 0u, nullptr,
                           d_results + (size_t)j * kResultWords, kResultWords);
        spans[j] = {h_offsets[j], h_offsets[j] + (uint64_t)p->L * p->L};
    }
    {
        std::vector<std::pair<uint64_t, uint64_t>> sp = spans;
        std::sort(sp.begin(), sp.end());
        for (uint32_t j = 1; j < n; ++j)
            if (sp[j].first < sp[j - 1].second)
                return ESCG_EINVAL;
    }
    // one kernel instantiation serves the whole batch: with any S > 7 job
    // every job runs with the larger S > 7 tables and must fit beside them
    if (!all_small)
        for (uint32_t j = 0; j < n; ++j)
            if (h_params[j].L > lds_max_L(ESCG_MAX_SPECIES))
                return ESCG_EINVAL;
    // Longest jobs first (cost ~ L^2 * MCS budget).
    for (uint32_t j = 0; j < n; ++j)
        order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        const double ca = (double)jobs[a].L * jobs[a].L * jobs[a].max_mcs;
        const double cb = (double)jobs[b].L * jobs[b].L * jobs[b].max_mcs;
        return ca > cb;
    });
    // with any job carrying dominance probabilities the batch runs the
    // probabilistic kernel; every job then gets selection thresholds (from
    // its 0/1 matrix when it has no probabilities: the same rule), with the
    // kernel's table stride
    bool prob = false;
    for (uint32_t j = 0; j < n; ++j)
        prob = prob || h_params[j].dom_prob != nullptr;
    const uint32_t Sp = all_small ? 8u : 32u, abw = 2u * Sp * Sp;
    std::vector<uint32_t> ab_all;
    if (prob) {
        ab_all.resize((size_t)n * abw);
        for (uint32_t j = 0; j < n; ++j) {
            const std::vector<uint32_t> ab = selection_thresholds(
                &h_params[j], jobs[j].T1, jobs[j].T2, Sp);
            std::copy(ab.begin(), ab.end(), ab_all.begin() + (size_t)j * abw);
        }
    }
    hipStream_t st = S_(stream);
    const size_t tbl = sizeof(JobDev) * n, ord = sizeof(uint32_t) * n;
    const size_t ab_off = (tbl + ord + 256 + 255) & ~(size_t)255;
    uint8_t *dev = nullptr;
    if (hipMallocAsync((void **)&dev, ab_off + ab_all.size() * 4, st) !=
        hipSuccess)
        return ESCG_ENOMEM;
    JobDev *d_jobs = reinterpret_cast<JobDev *>(dev);
    uint32_t *d_order = reinterpret_cast<uint32_t *>(dev + tbl);
    uint32_t *d_queue = reinterpret_cast<uint32_t *>(dev + tbl + ord + 128);
    if (prob)
        for (uint32_t j = 0; j < n; ++j)
            jobs[j].ab =
                reinterpret_cast<const uint32_t *>(dev + ab_off) + (size_t)j * abw;
    escg_status s = ESCG_OK;
    if (hipMemcpyAsync(d_jobs, jobs.data(), tbl, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(d_order, order.data(), ord, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        (prob && hipMemcpyAsync(dev + ab_off, ab_all.data(), ab_all.size() * 4,
                                hipMemcpyHostToDevice, st) != hipSuccess)) {
        (void)hipFreeAsync(dev, st);
        return ESCG_EDEVICE;
    }
    launch_fill(d_queue, 1, 0, st);
    // launch choices of the batch: those of h_params[0] (workgroup size
    // capped at the kernel's 512, resident workgroups per CU capped at what
    // fits)
    const escg_launch &ln = h_params[0].launch;
    const size_t lds = lds_need;
    const uint32_t nt = ln.threads ? std::min(ln.threads, 512u)
                                   : lds_threads(Lmax);
    const void *fn = ESCG_KERNEL2(lds_batch_kernel, all_small, prob);
    allow_dynamic_lds(fn, lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (ln.wg_per_cu)
        per_cu = std::min(per_cu, (int)ln.wg_per_cu);
    const DeviceInfo di = device_info();
    uint32_t grid =
        std::min<uint32_t>(n, (uint32_t)std::max(1, di.cus) * per_cu);
    if (ln.max_wgs)
        grid = std::min(grid, ln.max_wgs);
    const JobDev *aj = d_jobs;
    const uint32_t *ao = d_order;
    uint32_t an = n;
    uint32_t *aq = d_queue;
    uint8_t *al = d_lattices;
    void *args[] = {&aj, &ao, &an, &aq, &al};
    s = last_hip(hipLaunchKernel(fn, dim3(grid), dim3(nt), args, lds, st));
    (void)hipFreeAsync(dev, st);
    return s;
}

} // extern "C"
