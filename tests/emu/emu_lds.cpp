// CPU check of the quad update + whole-lattice pass logic against the oracle
// (single emulated thread: work items run one after another, which is the
// parallel result because blocks are disjoint).
#include "escg_lds.hpp"
#include <cmath>
#include <vector>
#include <cstdlib>
emu_dim3 threadIdx, blockDim, blockIdx, gridDim;
using namespace escg;
extern "C" void orc_o2_run(uint32_t L, uint32_t S, const uint8_t *D, double ex, double sel, double rep,
  uint64_t seed, uint32_t replica, int rounds, int nbhd, const double *P, uint32_t mcs0, uint32_t n_mcs, uint8_t *grid, uint32_t *counts);
extern "C" void orc_thresholds(double ex, double sel, double rep, uint32_t *T1, uint32_t *T2);
extern "C" void orc_circulant_matrix(uint32_t S, uint32_t kmask, uint8_t *D);
int main(int argc, char** argv) {
  blockDim.x = 1; threadIdx.x = 0;
  int bad = 0, cases = 0;
  uint32_t Ls[] = {2, 4, 6, 8, 10, 16, 30, 62, 64, 100, 130};
  double rates[][3] = {{0.5,1,1},{1,1,1},{0,1,1},{1,0,1},{1,1,0},{0,0,1},{0,1,0},{1,0,0},{51.2,1,1}};
  for (bool prob : {false, true}) for (bool moore : {false, true}) for (uint32_t S : {1u, 2u, 3u, 5u, 8u}) for (uint32_t L : Ls) for (auto& r : rates) {
    uint32_t kmask = S == 5 ? 0b1010 : (S == 8 ? 0b100110 : 0b10);
    std::vector<uint8_t> D(S * S); orc_circulant_matrix(S, kmask, D.data());
    if (S == 2) { D[1] = 1; D[2] = 1; } // mutual dominance: orientation matters
    uint32_t dom[32] = {0};
    for (uint32_t a = 1; a <= S; ++a) for (uint32_t b = 1; b <= S; ++b) if (D[(a-1)*S+(b-1)]) dom[a] |= 1u << b;
    uint32_t T1, T2; orc_thresholds(r[0], r[1], r[2], &T1, &T2);
    uint32_t LS = row_stride(L);
    std::vector<uint8_t> smem(LS * L + 64, 0);
    static LdsTables<8> T8; static LdsTables<32> T32;
    // dominance probabilities on every edge of D, thresholds as the host
    // code computes them
    std::vector<double> P(S * S, 0.0);
    for (uint32_t a = 0; a < S; ++a) for (uint32_t b = 0; b < S; ++b) if (D[a*S+b]) P[a*S+b] = 0.15 + 0.2 * ((a + 2 * b) % 4);
    const uint32_t Sp = S <= 7 ? 8 : 32, R = T2 - T1;
    std::vector<uint32_t> ab(2 * Sp * Sp, 0);
    for (uint32_t x = 1; x <= S; ++x) for (uint32_t y = 1; y <= S; ++y) if (x != y) {
      double pxy = D[(x-1)*S+(y-1)] ? P[(x-1)*S+(y-1)] : 0.0, pyx = D[(y-1)*S+(x-1)] ? P[(y-1)*S+(x-1)] : 0.0;
      uint32_t A = (uint32_t)floor(pxy * (double)R), B = A + (uint32_t)floor(pyx * (double)(R - A));
      ab[x*Sp+y] = A; ab[Sp*Sp + x*Sp+y] = B; }
    const uint32_t *abp = prob ? ab.data() : nullptr;
    QuadCtxT<false> qc; QuadCtxT<true> qcp;
    if (S <= 7) { setup_tables(T8, dom, moore, abp); qc = make_quad_ctx<false>(T8, T1, T2); qcp = make_quad_ctx<true>(T8, T1, T2); }
    else { setup_tables(T32, dom, moore, abp); qc = make_quad_ctx<false>(T32, T1, T2); qcp = make_quad_ctx<true>(T32, T1, T2); }
    uint8_t* lat = smem.data();
    std::vector<uint8_t> g(L * L);
    srand(L * 131 + S);
    for (auto& v : g) v = rand() % (S + 1);
    for (uint32_t rr = 0; rr < L; ++rr) { for (uint32_t c = 0; c < L; ++c) lat[rr*LS+c] = g[rr*L+c]; for (uint32_t c = L; c < LS; ++c) lat[rr*LS+c] = pad_byte(S); }
    uint64_t seed = 0x1234567890ull + L; uint32_t rep = 3, mcs0 = 17, n = 6;
    uint32_t Lb = L/2, Q = (Lb+3)/4;
    (void)Lb; (void)Q;
    // every thread of an nt-thread workgroup, pass by pass (threads of one
    // pass touch disjoint blocks); nt cycles through 256, 512 and 64
    const uint32_t nts[] = {256, 512, 64};
    blockDim.x = nts[cases % 3];
    for (uint32_t t = 0; t < n; ++t) {
      const Words off = philox(0u, mcs0 + t, kTagOffset << 8, rep, (uint32_t)seed, (uint32_t)(seed >> 32));
      // every other case starts the draws from the per-quad Philox heads
      // where a thread's quads fit them
      for (uint32_t p = 0; p < 4; ++p)
        for (threadIdx.x = 0; threadIdx.x < blockDim.x; ++threadIdx.x) {
          const LdsWalk W = lds_walk(L, LS);
          const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
          if ((cases & 1) && lds_heads_fit(W, L)) {
            const LdsHeads H = lds_heads(W, rep, k1);
            if (prob) lds_pass<true>(lat, L, LS, W, off.w[p], p, mcs0 + t, rep, k0, k1, qcp, &H);
            else lds_pass<true>(lat, L, LS, W, off.w[p], p, mcs0 + t, rep, k0, k1, qc, &H);
          } else {
            if (prob) lds_pass(lat, L, LS, W, off.w[p], p, mcs0 + t, rep, k0, k1, qcp);
            else lds_pass(lat, L, LS, W, off.w[p], p, mcs0 + t, rep, k0, k1, qc);
          }
        }
    }
    blockDim.x = 1; threadIdx.x = 0;
    std::vector<uint8_t> ref = g;
    orc_o2_run(L, S, D.data(), r[0], r[1], r[2], seed, rep, kPhiloxRounds, moore ? 8 : 4, prob ? P.data() : nullptr, mcs0, n, ref.data(), nullptr);
    bool ok = true;
    for (uint32_t rr = 0; rr < L; ++rr) { for (uint32_t c = 0; c < L; ++c) if (lat[rr*LS+c] != ref[rr*L+c]) ok = false; for (uint32_t c = L; c < LS; ++c) if (lat[rr*LS+c] != pad_byte(S)) ok = false; }
    cases++; if (!ok) { bad++; if (bad < 400) printf("MISMATCH prob=%d moore=%d S=%u L=%u rates=%g,%g,%g\n", (int)prob, (int)moore, S, L, r[0], r[1], r[2]); }
  }
  printf("%d/%d cases ok\n", cases - bad, cases);
  return bad != 0;
}
