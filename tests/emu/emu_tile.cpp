// CPU check of the persistent tiled kernel's phases (tile_load, tile_mcs,
// tile_publish, tile_gather, tile_count, tile_store) against the oracle.
#include "escg_lds.hpp"
#include "escg_tile.hpp"
#include <vector>
#include <cstdlib>
emu_dim3 threadIdx, blockDim, blockIdx, gridDim;
static bool bad_buffer = false;  // a list MCS left the lattice in buffer 1
using namespace escg;
extern "C" void orc_o2_run(uint32_t L, uint32_t S, const uint8_t *D, double ex, double sel, double rep,
  uint64_t seed, uint32_t replica, int rounds, int nbhd, const double *P, uint32_t mcs0, uint32_t n_mcs, uint8_t *grid, uint32_t *counts);
extern "C" void orc_thresholds(double ex, double sel, double rep, uint32_t *T1, uint32_t *T2);
extern "C" void orc_circulant_matrix(uint32_t S, uint32_t kmask, uint8_t *D);
// Runs tile_pass for every thread of a bd-thread workgroup, pass by pass
// (threads of one pass touch disjoint blocks, so sequential order is exact).
static void emu_tile_mcs(uint8_t *lat, const TileGeom &G, uint32_t ty, uint32_t tx, uint32_t t,
                         uint32_t rep, uint32_t k0, uint32_t k1, const QuadCtx &qc, uint32_t bd) {
  const Words off = philox(0u, t, kTagOffset << 8, rep, k0, k1);
  blockDim.x = bd;
  for (uint32_t p = 0; p < 4; ++p)
    for (threadIdx.x = 0; threadIdx.x < bd; ++threadIdx.x) {
      const TileWalk W = tile_walk(G, ty, tx);
      tile_pass(lat, G, W, off.w[p], p, t, rep, k0, k1, qc);
    }
  blockDim.x = 1; threadIdx.x = 0;
}
// The same with the balanced list walk (tile_pass_list), bd threads.
static void emu_tile_mcs_list(uint8_t *lat, const TileGeom &G, uint32_t ty, uint32_t tx, uint32_t t,
                              uint32_t rep, uint32_t k0, uint32_t k1, const QuadCtx &qc, uint32_t bd) {
  const Words off = philox(0u, t, kTagOffset << 8, rep, k0, k1);
  uint8_t *lat1 = lat + G.region_bytes() + 8;  // the second region buffer
  blockDim.x = bd;
  bool cur1 = false;
  for (uint32_t p = 0; p < 4; ++p) {
    bool next = false;
    for (threadIdx.x = 0; threadIdx.x < bd; ++threadIdx.x) {
      const TileList TL = tile_list(G, ty, tx);
      Words rf = philox(TL.c0[0], t, (kTagPass << 8) | p, rep, k0, k1);
      QuadSel sf = quad_sel(rf, qc);
      next = tile_pass_list(lat, lat1, G, TL, off.w[p], p, cur1, t, rep, k0, k1, qc, rf, sf);
    }
    cur1 = next;
  }
  if (cur1) { bad_buffer = true; }
  blockDim.x = 1; threadIdx.x = 0;
}
static uint32_t list_threads(const TileGeom &G) {
  const uint32_t nq = (G.RH() >> 1) * ((G.TW + 16) >> 3);
  uint32_t bd = (nq + 3 * 64 - 1) / (3 * 64) * 64;
  return tile_list_fits(G, bd) ? bd : 0;
}
static uint32_t g_cap = 1024;
int main() {
  blockDim.x = 1; threadIdx.x = 0;
  int bad = 0, cases = 0;
  struct C { uint32_t L, TH, TW, S; } cs[] = {{16,4,8,3},{16,8,16,3},{32,8,8,5},{48,6,24,3},{64,16,32,5},{80,10,40,8},{64,64,64,3},{128,32,64,5},{40,20,8,2},{24,12,24,3}};
  double rates[][3] = {{0.5,1,1},{13.1,1,1},{0,1,1},{1,1,0},{1,0,1}};
  uint32_t caps[] = {1024, 64, 32};
  int ci = 0;
  for (bool moore : {false, true}) for (auto c : cs) for (auto& r : rates) {
    g_cap = caps[ci++ % 3];
    if (tile_threads(TileGeom{c.L, c.TH, c.TW, c.L / c.TH, c.L / c.TW}, g_cap) == 0) g_cap = 1024;
    uint32_t S = c.S, L = c.L;
    uint32_t kmask = S == 5 ? 0b1010 : (S == 8 ? 0b100110 : 0b10);
    std::vector<uint8_t> D(S * S); orc_circulant_matrix(S, kmask, D.data());
    if (S == 2) { D[1] = 1; D[2] = 1; }
    uint32_t dom[32] = {0};
    for (uint32_t a = 1; a <= S; ++a) for (uint32_t b = 1; b <= S; ++b) if (D[(a-1)*S+(b-1)]) dom[a] |= 1u << b;
    uint32_t T1, T2; orc_thresholds(r[0], r[1], r[2], &T1, &T2);
    TileGeom G{L, c.TH, c.TW, L / c.TH, L / c.TW};
    uint32_t T = G.TY * G.TX;
    std::vector<uint8_t> g(L * L); srand(L + S * 7 + T1);
    for (auto& v : g) v = rand() % (S + 1);
    std::vector<std::vector<uint8_t>> sm(T, std::vector<uint8_t>(2 * G.region_bytes() + 64, 0));
    static LdsTables<8> T8; static LdsTables<32> T32;
    const size_t area = (size_t)T * G.slot_dwords();
    std::vector<uint32_t> exch(2 * area, 0);
    for (size_t i = area; i < 2 * area; ++i) exch[i] = 0x80808080u;
    uint32_t abort_word = 0;
    std::vector<QuadCtx> qcs(T);
    for (uint32_t t = 0; t < T; ++t) {
      uint8_t* s = sm[t].data();
      if (S <= 7) { setup_tables(T8, dom, moore); qcs[t] = make_quad_ctx(T8, T1, T2); }
      else { setup_tables(T32, dom, moore); qcs[t] = make_quad_ctx(T32, T1, T2); }
      tile_load(s, g.data(), G, t / G.TX, t % G.TX);
    }
    uint64_t seed = 99 + L; uint32_t rep = 2, mcs0 = 5, n = 5;
    std::vector<uint32_t> cnt((n + 1) * (S + 1), 0);
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t e = k + 1, sl = exch_slot(e), tag = exch_tag(e);
      {  // nothing published for this MCS yet: every halo word must read stale
        std::vector<uint8_t> tmp(sm[0]);
        for (uint32_t t = 0; t < T; ++t)
          if (tile_gather(tmp.data(), exch.data(), G, t / G.TX, t % G.TX, sl, tag, &abort_word, 64) != 2) {
            bad++; printf("STALE NOT DETECTED L=%u k=%u tile=%u\n", L, k, t); }
      }
      for (uint32_t t = 0; t < T; ++t) {
        uint8_t* lat = sm[t].data();
        if ((k & 1) && list_threads(G))
          emu_tile_mcs_list(lat, G, t / G.TX, t % G.TX, mcs0 + k, rep, (uint32_t)seed, (uint32_t)(seed >> 32), qcs[t], list_threads(G));
        else
          emu_tile_mcs(lat, G, t / G.TX, t % G.TX, mcs0 + k, rep, (uint32_t)seed, (uint32_t)(seed >> 32), qcs[t], tile_threads(G, g_cap));
        tile_publish(lat, exch.data() + (size_t)(sl * T + t) * G.slot_dwords(), G, tag);
        uint32_t sc[64] = {0};
        static uint32_t part[8 * 32];
        const uint32_t bdc = (k & 1) ? 64 : (S <= 7 ? G.TW / 8 : G.TW / 4);  // even k: one row per step, many row groups
        blockDim.x = bdc;  // several rows per step, idle threads when bdc % (TW/8) != 0
        for (threadIdx.x = 0; threadIdx.x < blockDim.x; ++threadIdx.x)
          if (S <= 7) tile_count_sums(lat, G, S, part); else tile_count_wide(lat, G, S, sc);
        if (S <= 7) {
          // flush: step 1 per lane, step 2 (eight-lane sums) here, step 3 per lane
          const uint32_t ns = count_states(S);
          uint32_t lv[64], T8[8] = {0};
          for (uint32_t l = 0; l < 64; ++l) lv[l] = count_slot_sum(part, l, ns - 1);
          for (uint32_t l = 0; l < 64; ++l) T8[l >> 3] += lv[l];
          for (uint32_t i = 0; i < 8 * 32; ++i) if (part[i]) { bad++; printf("SLOT NOT CLEARED\n"); break; }
          for (uint32_t l = 0; l <= S; ++l) {
            uint32_t c = 0;
            if (ns == 4) { uint32_t T[3] = {T8[0], T8[1], T8[2]}; c = count_species<4>(l, T, G.TH * G.TW); }
            else if (ns == 6) { uint32_t T[5] = {T8[0], T8[1], T8[2], T8[3], T8[4]}; c = count_species<6>(l, T, G.TH * G.TW); }
            else { uint32_t T[7] = {T8[0], T8[1], T8[2], T8[3], T8[4], T8[5], T8[6]}; c = count_species<8>(l, T, G.TH * G.TW); }
            sc[l] = c;
          }
        }
        blockDim.x = 1; threadIdx.x = 0;
        for (uint32_t s2 = 0; s2 <= S; ++s2) cnt[(k + 1) * (S + 1) + s2] += sc[s2];
      }
      for (uint32_t t = 0; t < T; ++t)
        if (tile_gather(sm[t].data(), exch.data(), G, t / G.TX, t % G.TX, sl, tag, &abort_word, 64)) {
          bad++; printf("GATHER TIMEOUT L=%u k=%u tile=%u\n", L, k, t); }
    }
    std::vector<uint8_t> out(L * L, 0xEE);
    for (uint32_t t = 0; t < T; ++t) tile_store(sm[t].data(), out.data(), G, t / G.TX, t % G.TX);
    // per-MCS variant: every MCS reloads each tile (+halo) from src and
    // stores the interior into dst
    std::vector<uint8_t> cur = g, nxt(L * L, 0xEE);
    for (uint32_t k = 0; k < n; ++k) {
      for (uint32_t t = 0; t < T; ++t) {
        uint8_t* lat = sm[t].data();
        tile_load(lat, cur.data(), G, t / G.TX, t % G.TX);
        emu_tile_mcs(lat, G, t / G.TX, t % G.TX, mcs0 + k, rep, (uint32_t)seed, (uint32_t)(seed >> 32), qcs[t], tile_threads(G, g_cap));
        tile_store(lat, nxt.data(), G, t / G.TX, t % G.TX);
      }
      std::swap(cur, nxt);
    }
    std::vector<uint8_t> ref = g;
    std::vector<uint32_t> rcnt((n + 1) * (S + 1), 0);
    orc_o2_run(L, S, D.data(), r[0], r[1], r[2], seed, rep, kPhiloxRounds, moore ? 8 : 4, nullptr, mcs0, n, ref.data(), rcnt.data());
    for (size_t q = S + 1; q < rcnt.size(); ++q)
      if (rcnt[q] != cnt[q]) { bad++; printf("COUNT MISMATCH L=%u S=%u idx=%zu %u vs %u\n", L, S, q, cnt[q], rcnt[q]); break; }
    if (cur != ref) { bad++; printf("PER-MCS MISMATCH L=%u TH=%u TW=%u S=%u\n", L, c.TH, c.TW, S); }
    cases++;
    if (out != ref) { bad++; size_t d = 0; for (size_t i = 0; i < out.size(); ++i) d += out[i] != ref[i];
      printf("MISMATCH L=%u TH=%u TW=%u S=%u rates=%g,%g,%g: %zu sites differ\n", L, c.TH, c.TW, S, r[0], r[1], r[2], d); }
  }
  if (bad_buffer) printf("LIST MCS ENDED IN BUFFER 1\n");
  printf("%d/%d tiled cases ok\n", cases - bad, cases);
  return bad != 0 || bad_buffer;
}
