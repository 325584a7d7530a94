/*
 * escg_oracle.c -- plain, slow, single-threaded CPU oracle for the ESCG
 * Monte Carlo hot path (arxiv 2508.16639).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may use it.  It shares no code, header, table
 * or constant with the HIP path; the two are written separately from the
 * same definitions and compared byte for byte.
 *
 * Two oracles live here:
 *
 *   O1  the classic random-sequential update (RSU) of the paper: the
 *       Elementary Step algorithm (Ch. "Project Execution", Sec. "Single
 *       Threaded ESCG in C++", Algorithm "Elementary Step") repeated N = L*L
 *       times per Monte Carlo step inside the Overall ESCG Loop algorithm,
 *       with the Dominance Check algorithm and the circulant dominance
 *       matrix equation of the same section.  Results are defined only in
 *       distribution; pinned by exact Markov chains on tiny lattices and by
 *       invariants.
 *
 *   O2  the parallel-schedule reference: the same pair rule applied on a
 *       conflict-free 2x2-block (Margolus) schedule driven by the
 *       counter-based Philox4x32 generator with 7 rounds (the fewest with
 *       which Salmon et al. report it passing TestU01's BigCrush; the paper
 *       itself uses Mersenne Twister and cuRAND, so the generator is this
 *       schedule's own choice).  It defines the GPU path's result exactly.  The paper has no such schedule (it uses racy atomics, Sec.
 *       "ESCG Performance Bottlenecks"); the schedule's definition is stated
 *       in full at o2_pass() below.  Pinned by the L=2 reduction to one RSU
 *       step, an exact one-pass distribution at L=4, invariants, and
 *       statistical agreement with O1.
 *
 * All arithmetic of the method is integer except the action thresholds,
 * which are computed once per job in IEEE-754 double (thresholds()).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-R, Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As   */
/* Easy as 1, 2, 3", SC'11, Sec. 4 (the Philox S-box and key schedule).      */
/* One round maps (X0,X1,X2,X3) with round key (K0,K1) to                    */
/*   (hi(M1*X2) ^ X1 ^ K0,  lo(M1*X2),  hi(M0*X0) ^ X3 ^ K1,  lo(M0*X0))     */
/* and the key is bumped by the Weyl constants between rounds.               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u /* golden ratio */
#define PHILOX_W1 0xBB67AE85u /* sqrt(3) - 1 */

void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds,
                    uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < rounds; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One 32-bit word of Philox4x32-R (R = rounds; the schedule uses 7) under */
/* the job key (seed). */
static uint32_t draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t c3, int word, int rounds)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32(ctr, key, rounds, out);
    return out[word];
}

/* Stream tags, placed in bits 8..15 of counter word 2. */
#define TAG_INIT   1u
#define TAG_OFFSET 2u
#define TAG_PASS   3u
#define TAG_RSU    4u

/* Action codes, in the paper's roulette order: migration (exchange) first,
 * then interaction (selection), then reproduction (Algorithm "Elementary
 * Step"). */
#define ACT_EXCHANGE  0
#define ACT_SELECTION 1
#define ACT_REPRODUCE 2

/* ------------------------------------------------------------------------ */
/* Dominance (Sec. "Single Threaded ESCG in C++")                             */
/* ------------------------------------------------------------------------ */

/* Circulant dominance matrix C(S, K): D[i][j] = 1 iff (j - i + S) mod S is
 * in K (circulant-matrix equation).  D is stored flat and row-major, S*S
 * bytes, row i = species i+1, as the paper stores it.  kmask bit k set <=>
 * offset k is in K. */
void orc_circulant_matrix(uint32_t S, uint32_t kmask, uint8_t *D)
{
    for (uint32_t i = 0; i < S; ++i)
        for (uint32_t j = 0; j < S; ++j)
            D[i * S + j] = (uint8_t)((kmask >> ((j - i + S) % S)) & 1u);
}

/* Algorithm "Dominance Check": false if either site is empty, else the
 * matrix entry at ((species-1)*S + (neighbour-1)). */
static int dominates(uint8_t species, uint8_t neighbour, uint32_t S,
                     const uint8_t *D)
{
    if (species == 0 || neighbour == 0)
        return 0;
    return D[(uint32_t)(species - 1) * S + (uint32_t)(neighbour - 1)] == 1;
}

/* The pair rule of Algorithm "Elementary Step": `cell` is the selected
 * site, `nbr` the chosen neighbour.  Same species: nothing happens.
 * Migration swaps.  Interaction: if the neighbour is occupied, the dominated
 * one of the two (cell first) becomes empty.  Reproduction: the occupied one
 * of the two copies itself into the empty one. */
static void pair_rule(int action, uint8_t *cell, uint8_t *nbr, uint32_t S,
                      const uint8_t *D)
{
    uint8_t species = *cell, neighbour = *nbr;
    if (species == neighbour)
        return;
    if (action == ACT_EXCHANGE) {
        *cell = neighbour;
        *nbr = species;
    } else if (action == ACT_SELECTION) {
        if (neighbour != 0) {
            if (dominates(species, neighbour, S, D))
                *nbr = 0;
            else if (dominates(neighbour, species, S, D))
                *cell = 0;
        }
    } else {
        if (neighbour == 0)
            *nbr = species;
        else if (species == 0)
            *cell = neighbour;
    }
}

/* Exposed for the truth-table tests. */
void orc_pair_rule(int action, uint8_t x, uint8_t y, uint32_t S,
                   const uint8_t *D, uint8_t out[2])
{
    pair_rule(action, &x, &y, S, D);
    out[0] = x;
    out[1] = y;
}

/* ------------------------------------------------------------------------ */
/* Probabilistic dominance (the interaction variant the paper adopts to      */
/* replicate Park, Chen and Szolnoki, Sec. "Extending Current Literature"): */
/* a directed edge a -> b of the dominance matrix carries a probability      */
/* P[(a-1)*S + (b-1)] in [0, 1] that a selection between the two succeeds.   */
/* As in the Dominance Check order, the selected cell's win is tried first   */
/* (probability P_xy, zero unless x dominates y); only if it fails is the    */
/* neighbour's win tried (P_yx).  P equal to the 0/1 matrix D gives the      */
/* deterministic rule.  P == NULL means deterministic.                       */
/* ------------------------------------------------------------------------ */
static double win_prob(uint8_t a, uint8_t b, uint32_t S, const uint8_t *D,
                       const double *P)
{
    if (!dominates(a, b, S, D))
        return 0.0;
    return P[(uint32_t)(a - 1) * S + (uint32_t)(b - 1)];
}

/* O1's selection with probabilities: f uniform on [0, 1). */
static void selection_prob_f(double f, uint8_t *cell, uint8_t *nbr, uint32_t S,
                             const uint8_t *D, const double *P)
{
    uint8_t x = *cell, y = *nbr;
    if (x == y || x == 0 || y == 0)
        return;
    double pxy = win_prob(x, y, S, D, P), pyx = win_prob(y, x, S, D, P);
    if (f < pxy)
        *nbr = 0;
    else if (f < pxy + pyx * (1.0 - pxy))
        *cell = 0;
}

/* O2's selection with probabilities: v uniform on {0, ..., R-1}, R = T2 - T1
 * (the selection draw u minus T1).  x wins if v < A, else y wins if v < B,
 * with A = floor(P_xy R) and B = A + floor(P_yx (R - A)), in double. */
static void selection_prob_v(uint32_t v, uint32_t R, uint8_t *cell,
                             uint8_t *nbr, uint32_t S, const uint8_t *D,
                             const double *P)
{
    uint8_t x = *cell, y = *nbr;
    if (x == y || x == 0 || y == 0)
        return;
    uint32_t A = (uint32_t)floor(win_prob(x, y, S, D, P) * (double)R);
    uint32_t B = A + (uint32_t)floor(win_prob(y, x, S, D, P) * (double)(R - A));
    if (v < A)
        *nbr = 0;
    else if (v < B)
        *cell = 0;
}

/* ------------------------------------------------------------------------ */
/* Action thresholds.  The paper draws r uniform on [0, mu+sigma+eps] and    */
/* picks migration if r < eps, interaction if r < eps + mu, else            */
/* reproduction (Algorithm "Elementary Step"; rates normalised to a roulette */
/* in Sec. "Single Threaded ESCG in C++").  O2 replaces the float draw by a  */
/* 24-bit integer u and two integer thresholds, computed here in double, in */
/* this order:  tot = (ex + sel) + rep;  T1 = floor(2^24 * ex / tot);        */
/* T2 = floor(2^24 * (ex + sel) / tot).                                      */
/* ------------------------------------------------------------------------ */
void orc_thresholds(double ex, double sel, double rep, uint32_t *T1,
                    uint32_t *T2)
{
    double tot = (ex + sel) + rep;
    *T1 = (uint32_t)floor(ldexp(ex / tot, 24));
    *T2 = (uint32_t)floor(ldexp((ex + sel) / tot, 24));
}

static int action_of(uint32_t u24, uint32_t T1, uint32_t T2)
{
    if (u24 < T1)
        return ACT_EXCHANGE;
    if (u24 < T2)
        return ACT_SELECTION;
    return ACT_REPRODUCE;
}

/* ------------------------------------------------------------------------ */
/* Initial lattice (Sec. "Single Threaded ESCG in C++", grid initialised     */
/* i.i.d.): each site is uniform over {0, 1, ..., S}, i.e. empty with        */
/* probability 1/(S+1).  Site n = row*L + col draws word n&3 of             */
/* Philox(ctr = (n>>2, 0, TAG_INIT<<8, replica), key = seed) and maps it by  */
/* floor(w * (S+1) / 2^32).                                                  */
/* ------------------------------------------------------------------------ */
void orc_init(uint32_t L, uint32_t S, uint64_t seed, uint32_t replica,
              int rounds, uint8_t *grid)
{
    uint64_t N = (uint64_t)L * L;
    for (uint64_t n = 0; n < N; ++n) {
        uint32_t w = draw(seed, (uint32_t)(n >> 2), 0u, TAG_INIT << 8, replica,
                          (int)(n & 3u), rounds);
        grid[n] = (uint8_t)(((uint64_t)w * (uint64_t)(S + 1u)) >> 32);
    }
}

/* Species counts including empty sites (the densities() of the Overall ESCG
 * Loop algorithm, before division by N).  counts has S+1 entries. */
void orc_counts(uint32_t L, uint32_t S, const uint8_t *grid, uint32_t *counts)
{
    uint64_t N = (uint64_t)L * L;
    for (uint32_t v = 0; v <= S; ++v)
        counts[v] = 0;
    for (uint64_t n = 0; n < N; ++n)
        if (grid[n] <= S)
            counts[grid[n]]++;
}

/* ------------------------------------------------------------------------ */
/* O2: the parallel schedule.                                                */
/*                                                                           */
/* One Monte Carlo step (MCS) t = four passes p = 0..3 in order.  Pass p     */
/* takes a uniform offset (ox, oy) in {0,1}^2 from bits 0 and 1 of word p   */
/* of Philox(ctr = (0, t, TAG_OFFSET<<8, replica)).  It tiles the lattice    */
/* into (L/2)^2 disjoint 2x2 blocks whose top-left site is                   */
/* (2*by + oy, 2*bx + ox); block sites A = top-left, B = top-right,          */
/* C = bottom-left, D = bottom-right, all modulo L (periodic boundary).      */
/* Every block takes one 32-bit word w: word (bx & 3) of                     */
/* Philox(ctr = (by*Q + (bx>>2), t, (TAG_PASS<<8) | p, replica)) with        */
/* Q = ceil((L/2)/4), so one Philox call serves four horizontally adjacent   */
/* blocks of one block row.  From w:                                         */
/*   von Neumann neighbourhood (nbhd = 4):                                   */
/*   bits 3-4  edge:        0 -> (A,B)  1 -> (C,D)  2 -> (A,C)  3 -> (B,D)   */
/*   bit  5    orientation: 0 -> the first site of the edge is the selected  */
/*                          cell, 1 -> the second one is                     */
/*   Moore neighbourhood (nbhd = 8):                                         */
/*   bits 3-5  pair: 0 -> (A,B)  1 -> (C,D)  2 -> (A,C)  3 -> (B,D)          */
/*                   4 -> (A,D)  5 -> (B,C)  6 -> (A,D)  7 -> (B,C)          */
/*             (a diagonal lies inside a block for one offset in four, an    */
/*             axis edge for one in two, so the diagonals take two slots:    */
/*             every one of the 4N Moore pairs is then updated with the same */
/*             probability 1/16 per pass, as under random-sequential steps)  */
/*   bit  6    orientation, as bit 5 above                                   */
/*   bits 8-31 u24, the action by the thresholds above                       */
/*   (bits 0-2 and 6-7, resp. 7, are unused; the pair bits sit at bit 3 so   */
/*   that a block's pair is the byte offset w & 0x38 (0x78) of an 8-byte     */
/*   table entry, a choice of this schedule, not of the paper)               */
/* and the pair rule is applied to (selected cell, neighbour).  Blocks are   */
/* disjoint, so the order in which blocks are visited is irrelevant.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t L, S;
    const uint8_t *D;
    uint32_t T1, T2;
    uint64_t seed;
    uint32_t replica;
    int rounds;
    int nbhd;        /* 4 (von Neumann) or 8 (Moore) */
    const double *P; /* dominance probabilities or NULL (deterministic) */
} o2_job;

static void o2_pass(const o2_job *j, uint32_t t, uint32_t p, uint8_t *grid)
{
    uint32_t L = j->L, Lb = L / 2, Q = (Lb + 3) / 4;
    uint32_t woff = draw(j->seed, 0u, t, TAG_OFFSET << 8, j->replica, (int)p,
                         j->rounds);
    uint32_t ox = woff & 1u, oy = (woff >> 1) & 1u;
    for (uint32_t by = 0; by < Lb; ++by) {
        for (uint32_t bx = 0; bx < Lb; ++bx) {
            uint32_t w = draw(j->seed, by * Q + (bx >> 2), t,
                              (TAG_PASS << 8) | p, j->replica, (int)(bx & 3u),
                              j->rounds);
            uint32_t r0 = 2 * by + oy, r1 = (r0 + 1) % L;
            uint32_t c0 = 2 * bx + ox, c1 = (c0 + 1) % L;
            uint64_t A = (uint64_t)r0 * L + c0, B = (uint64_t)r0 * L + c1;
            uint64_t C = (uint64_t)r1 * L + c0, Dd = (uint64_t)r1 * L + c1;
            uint64_t first, second;
            uint32_t pair = j->nbhd == 8 ? (w >> 3) & 7u : (w >> 3) & 3u;
            uint32_t orient = j->nbhd == 8 ? (w >> 6) & 1u : (w >> 5) & 1u;
            switch (pair) {
            case 0: first = A; second = B; break;
            case 1: first = C; second = Dd; break;
            case 2: first = A; second = C; break;
            case 3: first = B; second = Dd; break;
            case 4: case 6: first = A; second = Dd; break;
            default: first = B; second = C; break;
            }
            uint64_t cell = first, nbr = second;
            if (orient) {
                cell = second;
                nbr = first;
            }
            int action = action_of(w >> 8, j->T1, j->T2);
            if (j->P && action == ACT_SELECTION)
                selection_prob_v((w >> 8) - j->T1, j->T2 - j->T1, &grid[cell],
                                 &grid[nbr], j->S, j->D, j->P);
            else
                pair_rule(action, &grid[cell], &grid[nbr], j->S, j->D);
        }
    }
}

static void o2_mcs(const o2_job *j, uint32_t t, uint8_t *grid)
{
    for (uint32_t p = 0; p < 4; ++p)
        o2_pass(j, t, p, grid);
}

static o2_job make_job(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                       double sel, double rep, uint64_t seed, uint32_t replica,
                       int rounds, int nbhd, const double *P)
{
    o2_job j;
    j.L = L; j.S = S; j.D = D; j.seed = seed; j.replica = replica;
    j.rounds = rounds; j.nbhd = nbhd; j.P = P;
    orc_thresholds(ex, sel, rep, &j.T1, &j.T2);
    return j;
}

/* One pass only, for the one-pass distribution tests. */
void orc_o2_pass(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                 double sel, double rep, uint64_t seed, uint32_t replica,
                 int rounds, int nbhd, const double *P, uint32_t t,
                 uint32_t p, uint8_t *grid)
{
    o2_job j = make_job(L, S, D, ex, sel, rep, seed, replica, rounds, nbhd, P);
    o2_pass(&j, t, p, grid);
}

/* n_mcs MCS starting at absolute MCS index mcs0.  counts (if non-NULL) gets
 * (n_mcs+1) rows of S+1: row k = state after k of these MCS (row 0 = input
 * state), following the Overall ESCG Loop, which records densities before
 * each MCS and once more at the end. */
void orc_o2_run(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                double sel, double rep, uint64_t seed, uint32_t replica,
                int rounds, int nbhd, const double *P, uint32_t mcs0,
                uint32_t n_mcs, uint8_t *grid, uint32_t *counts)
{
    o2_job j = make_job(L, S, D, ex, sel, rep, seed, replica, rounds, nbhd, P);
    if (counts)
        orc_counts(L, S, grid, counts);
    for (uint32_t k = 0; k < n_mcs; ++k) {
        o2_mcs(&j, mcs0 + k, grid);
        if (counts)
            orc_counts(L, S, grid, counts + (size_t)(k + 1) * (S + 1));
    }
}

/* Stop conditions, checked on the counts after every MCS (and at the start):
 *   mode 0, first extinction: some species 1..S has count 0;
 *   mode 1, monoculture (the paper's stasis(), Sec. "Metal ESCG
 *           Implementation"): at most one species 1..S remains. */
static int stop_met(uint32_t S, const uint32_t *c, int mode)
{
    uint32_t alive = 0, extinct = 0;
    for (uint32_t s = 1; s <= S; ++s) {
        if (c[s] > 0)
            alive++;
        else
            extinct++;
    }
    return mode == 0 ? extinct > 0 : alive <= 1;
}

/* Runs until the stop condition holds or max_mcs MCS have been done.
 * result = {flag, t_ext, counts[0..S]}: flag 1 if the condition was met at
 * MCS t_ext (relative to mcs0; 0 means the input state already met it),
 * else flag 0 and t_ext = max_mcs.  The lattice is left in the state at
 * t_ext. */
void orc_o2_run_until(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                      double sel, double rep, uint64_t seed, uint32_t replica,
                      int rounds, int nbhd, const double *P, uint32_t mcs0,
                      uint32_t max_mcs, int mode, uint8_t *grid,
                      uint32_t *result)
{
    o2_job j = make_job(L, S, D, ex, sel, rep, seed, replica, rounds, nbhd, P);
    uint32_t *c = result + 2;
    uint32_t t = 0;
    orc_counts(L, S, grid, c);
    int met = stop_met(S, c, mode);
    while (!met && t < max_mcs) {
        o2_mcs(&j, mcs0 + t, grid);
        t++;
        orc_counts(L, S, grid, c);
        met = stop_met(S, c, mode);
    }
    result[0] = (uint32_t)met;
    result[1] = t;
}

/* ------------------------------------------------------------------------ */
/* O1: random-sequential update, Algorithm "Elementary Step" N times per     */
/* MCS.  Its own random stream: elementary step number k (64-bit, counted    */
/* from 0 at mcs0 * N) uses Philox(ctr = (lo(k), hi(k), TAG_RSU<<8,          */
/* replica)): word 0 picks the cell, floor(w0 * N / 2^32); word 1 picks the */
/* neighbour: bits 0-1 (up, down, left, right) for the von Neumann          */
/* neighbourhood, bits 0-2 (those four, then up-left, up-right, down-left,   */
/* down-right) for the Moore neighbourhood; words 2 and 3 give a double     */
/* r in [0, tot) with 53 random bits, and the roulette is the paper's:       */
/* r < eps migration, r < eps + sel interaction, else reproduction.          */
/* ------------------------------------------------------------------------ */
static void o1_step(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                    double sel, double tot, uint64_t seed, uint32_t replica,
                    int rounds, int nbhd, const double *P, uint64_t k,
                    uint8_t *grid)
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), TAG_RSU << 8, replica};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32(ctr, key, rounds, w);
    uint64_t N = (uint64_t)L * L;
    uint64_t i = ((uint64_t)w[0] * N) >> 32;
    uint32_t row = (uint32_t)(i / L), col = (uint32_t)(i % L);
    uint32_t nr = row, nc = col;
    uint32_t up = (row + L - 1) % L, down = (row + 1) % L;
    uint32_t left = (col + L - 1) % L, right = (col + 1) % L;
    switch (nbhd == 8 ? (w[1] & 7u) : (w[1] & 3u)) {
    case 0: nr = up; break;
    case 1: nr = down; break;
    case 2: nc = left; break;
    case 3: nc = right; break;
    case 4: nr = up; nc = left; break;
    case 5: nr = up; nc = right; break;
    case 6: nr = down; nc = left; break;
    default: nr = down; nc = right; break;
    }
    uint64_t ni = (uint64_t)nr * L + nc;
    uint64_t bits53 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
    double r = ldexp((double)bits53, -53) * tot;
    int action;
    if (r < ex)
        action = ACT_EXCHANGE;
    else if (r < ex + sel)
        action = ACT_SELECTION;
    else
        action = ACT_REPRODUCE;
    if (P && action == ACT_SELECTION)
        selection_prob_f((r - ex) / sel, &grid[i], &grid[ni], S, D, P);
    else
        pair_rule(action, &grid[i], &grid[ni], S, D);
}

void orc_o1_run(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                double sel, double rep, uint64_t seed, uint32_t replica,
                int rounds, int nbhd, const double *P, uint32_t mcs0,
                uint32_t n_mcs, uint8_t *grid, uint32_t *counts)
{
    uint64_t N = (uint64_t)L * L;
    double tot = (ex + sel) + rep;
    if (counts)
        orc_counts(L, S, grid, counts);
    for (uint32_t m = 0; m < n_mcs; ++m) {
        uint64_t k0 = (uint64_t)(mcs0 + m) * N;
        for (uint64_t n = 0; n < N; ++n)
            o1_step(L, S, D, ex, sel, tot, seed, replica, rounds, nbhd, P,
                    k0 + n, grid);
        if (counts)
            orc_counts(L, S, grid, counts + (size_t)(m + 1) * (S + 1));
    }
}

/* Elementary steps one at a time (for the exact-chain tests): steps
 * k0 .. k0 + n - 1 of the O1 stream. */
void orc_o1_steps(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                  double sel, double rep, uint64_t seed, uint32_t replica,
                  int rounds, int nbhd, const double *P, uint64_t k0,
                  uint64_t n, uint8_t *grid)
{
    double tot = (ex + sel) + rep;
    for (uint64_t k = 0; k < n; ++k)
        o1_step(L, S, D, ex, sel, tot, seed, replica, rounds, nbhd, P, k0 + k,
                grid);
}

void orc_o1_run_until(uint32_t L, uint32_t S, const uint8_t *D, double ex,
                      double sel, double rep, uint64_t seed, uint32_t replica,
                      int rounds, int nbhd, const double *P, uint32_t mcs0,
                      uint32_t max_mcs, int mode, uint8_t *grid,
                      uint32_t *result)
{
    uint64_t N = (uint64_t)L * L;
    double tot = (ex + sel) + rep;
    uint32_t *c = result + 2;
    uint32_t t = 0;
    orc_counts(L, S, grid, c);
    int met = stop_met(S, c, mode);
    while (!met && t < max_mcs) {
        uint64_t k0 = (uint64_t)(mcs0 + t) * N;
        for (uint64_t n = 0; n < N; ++n)
            o1_step(L, S, D, ex, sel, tot, seed, replica, rounds, nbhd, P,
                    k0 + n, grid);
        t++;
        orc_counts(L, S, grid, c);
        met = stop_met(S, c, mode);
    }
    result[0] = (uint32_t)met;
    result[1] = t;
}
