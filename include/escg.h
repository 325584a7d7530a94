/*
 * escg.h -- C ABI of the MI355X (gfx950) ESCG Monte Carlo library.
 *
 * The library advances L x L periodic von Neumann lattices of uint8 species
 * states (0 = empty, 1..S) by the elementary step of an Evolutionary Spatial
 * Cyclic Game: a site and one of its four neighbours interact by exchange
 * (the paper's migration), selection (interaction through the dominance
 * matrix) or reproduction into an empty site (arxiv 2508.16639, Sec.
 * "Single Threaded ESCG in C++": Algorithm "Elementary Step", Algorithm
 * "Dominance Check", the circulant dominance matrix equation and the action
 * probability normalisation).
 *
 * Updates run on a conflict-free schedule: one Monte Carlo step (MCS) is
 * four passes; each pass tiles the lattice into disjoint 2x2 blocks at a
 * random offset and updates one random internal edge per block, so one MCS
 * is L*L elementary steps, as in the paper's Overall ESCG Loop.  All random
 * numbers come from Philox4x32-7 (Salmon et al., SC'11) keyed by the job
 * seed, with counters built from (site or block, MCS index, pass, replica):
 * a result depends only on (parameters, input lattice, absolute MCS index),
 * never on launch shape, batching, co-running jobs or how a run is split.
 * The block words, thresholds and stream tags are defined in the library
 * source (escg_device.hpp).
 *
 * Conventions for every entry point:
 *   - Return value: ESCG_OK (0) or a negative escg_status.  Parameters are
 *     validated on the host before anything is enqueued; on any error
 *     nothing is enqueued and no output is touched.
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     current device, caller-owned, e.g. torch tensors' data_ptr()).
 *     Pointers named h_* are host pointers read before the call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Work is enqueued asynchronously on it; outputs are valid once the
 *     stream has completed.  Exception: escg_run_until_extinction on a
 *     lattice too large for one workgroup's LDS synchronises the stream
 *     while it runs (it polls the stop flag between chunks of MCS).
 *   - Lattices are row-major uint8[L*L], site (row, col) at row*L + col.
 *     Every site value must be in 0..S; other values give unspecified
 *     (but memory-safe) results.
 *   - Calls on different streams may run concurrently, on different
 *     lattices.  Scratch memory is stream-ordered (hipMallocAsync) and
 *     private to each call.
 */
#ifndef ESCG_H
#define ESCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t escg_status;
#define ESCG_OK             0
#define ESCG_EINVAL        (-1) /* invalid argument; nothing enqueued        */
#define ESCG_ENOMEM        (-2) /* device scratch allocation failed           */
#define ESCG_EDEVICE       (-3) /* a HIP call failed                          */
#define ESCG_EUNSUPPORTED  (-4) /* valid request this library cannot run      */
#define ESCG_ETIMEOUT      (-5) /* a device wait exceeded its spin bound      */

#define ESCG_MAX_SPECIES   31u
#define ESCG_MAX_L         46340u /* L*L fits in 31 bits                      */

/* Stop conditions (checked on the species counts after every MCS and on the
 * input state).  The paper stops at monoculture (its stasis check, Sec.
 * "Metal ESCG Implementation"); the extinction workloads stop at the first
 * extinction of any species. */
#define ESCG_STOP_FIRST_EXTINCTION 0u /* some species 1..S has count 0       */
#define ESCG_STOP_MONOCULTURE      1u /* at most one species 1..S remains    */
#define ESCG_STOP_NONE             2u /* run the full MCS budget              */

/* Kernel paths of a single job (escg_launch.route, escg_last_route): the
 * whole lattice in one workgroup's LDS; one tiled launch per MCS; the
 * persistent tiled kernel (all MCS in one cooperative launch, every tile
 * resident in LDS). */
#define ESCG_ROUTE_LDS        1u
#define ESCG_ROUTE_TILED      2u
#define ESCG_ROUTE_PERSISTENT 3u

/* Launch choices of one call (all zero: the library decides).  They select
 * among kernels that produce the same bytes, so they change speed and
 * occupancy, never results; they are read per call, so threads driving the
 * library with different choices do not interfere.
 *   route     0, or ESCG_ROUTE_LDS / ESCG_ROUTE_TILED / ESCG_ROUTE_PERSISTENT
 *             to force that path of escg_step_mcs / escg_run_until_extinction
 *             (ESCG_EUNSUPPORTED, nothing enqueued, if it cannot run this
 *             job: LDS needs L <= escg_batch_max_L(S), persistent needs
 *             L % 8 == 0 and a tile plan whose tiles are all resident).
 *             Automatic: persistent if L % 8 == 0 and L >= 72, else the
 *             whole lattice in one workgroup's LDS if it fits, else one
 *             tiled launch per MCS.
 *   tile_h, tile_w   tile shape of the tiled paths (both 0: the planner's
 *             cost model); must divide L with tile_w % 8 == 0, tile_h even
 *             >= 4 (EINVAL otherwise); a shape whose tile does not fit the
 *             LDS is ESCG_EUNSUPPORTED.
 *   threads   workgroup size cap of the tiled paths and the batch kernel
 *             (0: automatic; else a multiple of 64, 64..1024, EINVAL
 *             otherwise).
 *   wg_per_cu escg_batch_run only: resident workgroups per compute unit
 *             (0: as many as fit; else 1..8, capped by what fits).
 *   max_wgs   escg_batch_run and escg_step_batch (read from their first
 *             job): at most this many workgroups in one launch (0: as many
 *             as the device keeps resident), so that work on another stream
 *             keeps the remaining CUs. */
typedef struct escg_launch {
    uint32_t route;
    uint32_t tile_h, tile_w;
    uint32_t threads;
    uint32_t wg_per_cu;
    uint32_t max_wgs;
} escg_launch;

/* Job parameters.  Rates are named by role; only their ratios matter (the
 * paper normalises them into a roulette).  dom[a] bit b (1 <= a, b <= S) is
 * set iff species a dominates species b (the paper's flat matrix entry
 * D[(a-1)*S + (b-1)]); dom[0], bit 0 and bits above S must be zero. */
typedef struct escg_params {
    uint32_t L;        /* lattice side, even, 2 <= L <= ESCG_MAX_L          */
    uint32_t S;        /* species, 1 <= S <= ESCG_MAX_SPECIES               */
    uint32_t dom[32];  /* dominance bitmasks, see above                     */
    double   rate_ex;  /* exchange (migration) rate  >= 0, finite           */
    double   rate_sel; /* selection (interaction) rate >= 0, finite         */
    double   rate_rep; /* reproduction rate >= 0, finite; sum > 0           */
    uint64_t seed;     /* Philox key                                        */
    uint32_t replica;  /* independent stream id under the same seed         */
    uint32_t flags;    /* ESCG_FLAG_*; other bits must be 0                 */
    const double *dom_prob; /* NULL, or S*S dominance probabilities (host)  */
    escg_launch launch; /* kernel choice for this call; all zero = automatic */
} escg_params;

/* dom_prob: probabilistic dominance, the interaction variant the paper uses
 * to replicate Park, Chen and Szolnoki (Sec. "Extending Current
 * Literature"): entry (a-1)*S + (b-1), in [0, 1], is the probability that a
 * selection of species a against species b succeeds where dom[a] has bit b
 * (entries elsewhere are ignored).  The selected cell's win is tried first,
 * then the neighbour's, as in the Dominance Check.  A selection draw u
 * (T1 <= u < T2) decides both: with R = T2 - T1 and, in double,
 * A = floor(P_xy R), B = A + floor(P_yx (R - A)), the selected cell x wins
 * if u - T1 < A, else the neighbour y wins if u - T1 < B, else nothing
 * happens.  dom_prob equal to the 0/1 matrix gives the deterministic rule
 * bit for bit.  Read during the call only.  EINVAL if an entry is not in
 * [0, 1]. */

/* flags: the 8-way Moore neighbourhood instead of the 4-way von Neumann one
 * (the paper's --neighbourhood option, Sec. "Single Threaded ESCG in C++").
 * A random-sequential step then picks one of a site's eight neighbours; in
 * the block schedule a block word's bits 3-5 pick one of eight pair slots,
 * the four axis edges (A,B), (C,D), (A,C), (B,D) once each and the two
 * diagonals (A,D), (B,C) twice each, and bit 6 the orientation, which
 * updates every one of the 4N Moore pairs at the same rate, 1/16 per
 * pass. */
#define ESCG_FLAG_MOORE 1u

/* Human-readable name of a status code (static storage). */
const char *escg_status_str(escg_status s);

/* Name and description of the last HIP error this thread's calls turned into
 * ESCG_EDEVICE ("" if none); valid until the thread's next failing call. */
const char *escg_last_error(void);

/* Circulant dominance C(S, K) of the paper's circulant matrix equation:
 * species i dominates j iff (j - i) mod S is in K.  kmask bit k set <=> k in
 * K (bit 0 ignored).  Writes dom[0..31].  EINVAL if S is out of range or dom
 * is NULL. */
escg_status escg_circulant_dom(uint32_t S, uint32_t kmask, uint32_t *h_dom);

/* Dominance bitmasks from the paper's flat S*S matrix (Algorithm "Dominance
 * Check" layout; nonzero entry = dominates).  EINVAL on NULL or bad S. */
escg_status escg_dom_from_matrix(uint32_t S, const uint8_t *h_D,
                                 uint32_t *h_dom);

/* Exchange rate for mobility M on an L x L lattice: *eps = M * L * L / 2,
 * i.e. M = 2 eps / N with N = L * L sites, the convention of the cited
 * three-species mobility study whose results the paper replicates (Sec.
 * "Extending Current Literature").  The paper's own rate listing (Sec.
 * "Single Threaded ESCG in C++") writes eps = 2 M N, a factor of four away;
 * the library keeps its reading in this one function.  EINVAL if M is
 * negative or not finite, L is 0, or eps is NULL.  Host only. */
escg_status escg_eps_from_mobility(double M, uint32_t L, double *eps);

/* The two 24-bit action thresholds of the job: an elementary step with
 * uniform 24-bit draw u is an exchange if u < T1, a selection if
 * T1 <= u < T2, else a reproduction, where (in IEEE double, this order)
 * tot = (ex + sel) + rep, T1 = floor(2^24 ex / tot),
 * T2 = floor(2^24 (ex + sel) / tot).  This is the paper's roulette
 * (Algorithm "Elementary Step": migration first, then interaction, then
 * reproduction) with the float draw replaced by integers.  EINVAL on bad
 * rates or NULL. */
escg_status escg_thresholds(const escg_params *p, uint32_t *T1, uint32_t *T2);

/* Fills d_lattice (uint8[L*L]) with the initial state: every site i.i.d.
 * uniform over {0, ..., S} (0 = empty), drawn from (seed, replica, site).
 * The paper initialises occupied sites uniformly over species with a chosen
 * empty probability (Sec. "Single Threaded ESCG in C++"); here that
 * probability is 1/(S+1). */
escg_status escg_init(const escg_params *p, uint8_t *d_lattice, void *stream);

/* Species counts of d_lattice: d_counts (uint32[S+1]) receives, for
 * v = 0..S, the number of sites equal to v (the paper's densities() before
 * division by L*L, Algorithm "Overall ESCG Loop"). */
escg_status escg_densities(const escg_params *p, const uint8_t *d_lattice,
                           uint32_t *d_counts, void *stream);

/* Advances d_lattice in place by n_mcs Monte Carlo steps whose absolute
 * indices are mcs0 .. mcs0 + n_mcs - 1 (the index keys the random streams,
 * so splitting a run into several calls gives the same bytes).  If d_counts
 * is non-NULL it receives uint32[(n_mcs + 1) * (S + 1)]: row k holds the
 * species counts after k of these MCS, row 0 those of the input (the
 * paper's per-MCS density record).  n_mcs = 0 only writes row 0. */
escg_status escg_step_mcs(const escg_params *p, uint8_t *d_lattice,
                          uint32_t mcs0, uint32_t n_mcs, uint32_t *d_counts,
                          void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as escg_step_mcs, with the same arguments, results (byte for
 * byte), routing and launch choices, but the call allocates nothing.  Every
 * scratch buffer it needs (the persistent kernel's exchange area and abort
 * word, the per-MCS path's ping-pong lattice, the selection thresholds of
 * dominance probabilities) is carved from one file-scope device array of
 * ESCG_STATIC_SCRATCH_BYTES bytes per GPU, which the library holds until the
 * process ends.  A call that would need more returns ESCG_ENOMEM with
 * nothing enqueued and escg_last_error() giving the bytes needed (the
 * per-MCS tiled path takes L*L bytes, the persistent path max(exchange
 * area, L*L), dominance probabilities 8 KiB more: every L <= 8184 fits).  Calls on one GPU share its
 * array and each call initialises what it uses, so calls whose work
 * overlaps on the device (different streams, or different host threads)
 * race on it and give undefined results: serialise them. */
#define ESCG_STATIC_SCRATCH_BYTES (64u << 20)
escg_status escg_step_mcs_static(const escg_params *p, uint8_t *d_lattice,
                                 uint32_t mcs0, uint32_t n_mcs,
                                 uint32_t *d_counts, void *stream);

/* Runs from absolute MCS mcs0 until the stop condition `mode` holds or
 * max_mcs MCS have been done.  d_result (uint32[S + 3]) receives
 * {flag, t_ext, counts[0..S]}: flag = 1 if the condition held after t_ext
 * MCS of this call (t_ext = 0: the input already met it), else flag = 0 and
 * t_ext = max_mcs; counts are those of the returned lattice, which is the
 * state at t_ext.  The paper's loop stops at monoculture (stasis());
 * ESCG_STOP_NONE runs all max_mcs MCS. */
escg_status escg_run_until_extinction(const escg_params *p, uint8_t *d_lattice,
                                      uint32_t mcs0, uint32_t max_mcs,
                                      uint32_t mode, uint32_t *d_result,
                                      void *stream);

/* Largest L that escg_batch_run accepts for S species (the whole lattice and
 * the S-dependent rule tables must fit one workgroup's LDS); 0 for invalid S. */
uint32_t escg_batch_max_L(uint32_t S);

/* Many independent jobs in one launch of a persistent kernel: each
 * workgroup takes jobs from a queue (longest first), keeps the job's
 * lattice in LDS for its whole run, and writes it back at the end.
 *   h_params[n]      job parameters (L <= escg_batch_max_L())
 *   h_offsets[n]     byte offset of job j's lattice inside d_lattices;
 *                    lattices must not overlap
 *   h_mcs0[n]        absolute MCS index each job starts at (NULL = all 0)
 *   h_max_mcs[n]     MCS budget per job
 *   mode             stop condition (ESCG_STOP_*), as in
 *                    escg_run_until_extinction
 *   init             nonzero: the lattice is first initialised as by
 *                    escg_init (then mcs0 is still honoured); zero: the
 *                    lattice in d_lattices is the input state
 *   d_results        uint32[n * 34]: job j's {flag, t_ext, counts[0..S]}
 *                    at d_results + 34 j (unused tail words are zeroed)
 * Every job's output equals escg_run_until_extinction on the same job
 * alone, byte for byte.  n == 0 returns ESCG_OK and touches nothing (the
 * pointers may be NULL); with n > 0 a NULL array, an unknown mode,
 * misaligned or overlapping lattices or an invalid job give ESCG_EINVAL
 * with nothing enqueued. */
#define ESCG_BATCH_RESULT_WORDS 34u
escg_status escg_batch_run(uint32_t n, const escg_params *h_params,
                           const uint64_t *h_offsets, uint8_t *d_lattices,
                           const uint32_t *h_mcs0, const uint32_t *h_max_mcs,
                           uint32_t mode, uint32_t init, uint32_t *d_results,
                           void *stream);

/* Advances n independent jobs, job j by h_n_mcs[j] MCS from absolute MCS
 * h_mcs0[j], all jobs together.  This is the step of the paper's overall
 * loop (Algorithm "Overall ESCG Loop", N elementary steps per MCS) for a set
 * of simulations at once; each job's result equals escg_step_mcs on that
 * job alone, byte for byte.  Two paths, chosen by h_params[0].launch.route:
 *   ESCG_ROUTE_TILED as below; any other value (0, ESCG_ROUTE_PERSISTENT,
 *             ESCG_ROUTE_LDS): persistent launches holding several jobs:
 *             every tile of every job stays in LDS for all of the job's MCS
 *             and exchanges halos with its own job's tiles only; jobs are
 *             packed whole into launches of at most max_wgs workgroups (or
 *             what the device keeps resident), longest chunk first, one
 *             launch after the other on the stream; a job with more tiles
 *             than one launch holds runs per MCS as below.  A launch's tiles
 *             wait only for each other and never for other work, so they
 *             all become resident even while other streams' kernels hold
 *             CUs for a while; a wait that exceeds its bound (seconds) is
 *             reported by escg_async_status as ESCG_ETIMEOUT.
 *   ESCG_ROUTE_TILED: one launch per MCS for all jobs: the tiles of every
 *             job still running form one grid, so lattices too small to
 *             fill the GPU on their own share it.
 *   h_params[n]      job parameters; every L must be a multiple of 8 and
 *                    >= 16 (ESCG_EUNSUPPORTED otherwise, nothing enqueued,
 *                    escg_last_error() names the job)
 *   h_lattices[n]    device pointers to each job's uint8[L*L] lattice,
 *                    4-byte aligned, pairwise disjoint, updated in place
 *   h_mcs0[n], h_n_mcs[n]  start MCS and number of MCS per job (0: untouched)
 * No counts are recorded (escg_densities reads a lattice afterwards).
 * n == 0 returns ESCG_OK and touches nothing; with n > 0 a NULL array gives
 * ESCG_EINVAL.  escg_last_route() afterwards: ESCG_ROUTE_PERSISTENT if any
 * persistent launch was made, else ESCG_ROUTE_TILED.
 * Scratch (stream-ordered): per persistent launch a job table, two exchange
 * slots per tile and an abort word per job; per-MCS path: one ping-pong
 * lattice per job. */
escg_status escg_step_batch(uint32_t n, const escg_params *h_params,
                            uint8_t *const *h_lattices, const uint32_t *h_mcs0,
                            const uint32_t *h_n_mcs, void *stream);

/* Which kernel path the calling thread's last escg_step_mcs with n_mcs > 0,
 * escg_run_until_extinction or escg_step_batch enqueued (ESCG_ROUTE_*; 0
 * before any such call).  When the persistent path is planned but its cooperative launch is
 * refused, the call falls back to per-MCS launches and escg_last_error()
 * says why. */
uint32_t escg_last_route(void);

/* The tile shape and workgroup size that a path would use for job p (its
 * L, S and launch choices) on the current device: persistent = 1 the
 * single-job persistent kernel, 2 a multi-job persistent launch of
 * escg_step_batch, 0 the per-MCS tiled kernel.  EUNSUPPORTED if that path
 * cannot run the job, EINVAL for invalid parameters, persistent > 2 or
 * NULL outputs. */
escg_status escg_tile_plan(const escg_params *p, uint32_t persistent,
                           uint32_t *TH, uint32_t *TW, uint32_t *threads);

/* Synchronises the current device and reports errors that asynchronous
 * kernels can only record on the device: ESCG_ETIMEOUT if a persistent
 * kernel abandoned a bounded wait for a neighbouring workgroup since the
 * last reset (its outputs are then invalid), else ESCG_OK (or ESCG_EDEVICE
 * if the synchronisation fails).  reset != 0 clears the record. */
escg_status escg_async_status(int reset);

#ifdef __cplusplus
}
#endif

#endif /* ESCG_H */
