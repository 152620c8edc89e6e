/*
 * pdit.h -- C ABI of the MI355X (gfx950) p-dit sweep library for the
 * symmetric quadratic assignment problem.
 *
 * The method (Duffee, Burling-Smith et al., "P-dit Probabilistic Ising
 * Machine for Solving the Quadratic Assignment Problem"):
 *   - the objective is Eq. 1, E(p) = sum_i sum_j D_ij F_{p(i) p(j)}, for
 *     symmetric integer D (distances between locations) and F (flows
 *     between facilities); p(i) is the facility at location i;
 *   - there is one p-dit per location; a sweep ("iteration", Results,
 *     "Implementation") updates locations 0..N-1 in order;
 *   - the update of location r considers swapping its facility with that of
 *     every location s (s = r meaning "stay") and draws s with the Gibbs
 *     probability of Eq. 5, exp(-beta dE_rs) / sum_k exp(-beta dE_rk), where
 *     dE is the exact integer swap change of Eq. 3;
 *   - dE is read from the influence matrix H = D F[p,p] (H_ik =
 *     sum_j D_ij F_{p(j) p(k)}); for symmetric data the influence of Eq. 2
 *     is I_i^{p(k)} = -2 H_ik, and after an accepted swap H is brought up to
 *     date by an O(N^2) rank-1 update (Methods, "CPU-PIM Algorithm": the
 *     influence is kept incrementally);
 *   - replicas (the paper's duplicated replica sets, "GPU Implementations")
 *     are independent chains and run in parallel.
 *
 * Random numbers: the update of location r in global sweep g of replica k
 * of instance n uses word 0 of Philox4x32-10 (Salmon et al., SC'11) with
 * key (lo32(seed), hi32(seed)) and counter (r, g, k, n); u24 = word0 >> 8.
 * The draw takes the first candidate s with C_s * 2^24 > u24 * Z, where
 * C_s is the running sum over s' <= s of q_s' = rint(expf(-fl32(beta *
 * fl32(dE_s' - min dE))) * 2^25) and Z = C_{N-1}.  All integer work (H, dE,
 * E) is exact; energies are reported as int64.
 *
 * Conventions for every entry point:
 *   - every pointer argument named as "device" is device memory of the
 *     context's GPU (for example a torch tensor's data_ptr()); the caller
 *     owns it and must keep it alive until the context's stream has passed
 *     the call;
 *   - matrices are row-major, int32, N x N; permutations are int32 rows of
 *     length N (entry i = facility at location i, 0-based);
 *   - calls are ordered on the context's stream and may return before the
 *     GPU has finished; pdit_sync() waits and reports deferred errors;
 *   - a context is not thread-safe: use one per host thread;
 *   - the return value is PDIT_OK (0) or a negative status; the library
 *     never aborts or prints; pdit_last_error() gives a message.
 */
#ifndef PDIT_H
#define PDIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PDIT_OK 0
#define PDIT_EINVAL (-1)    /* null pointer, N < 2, N > PDIT_NMAX, R < 1, n_sweeps < 0, bad option */
#define PDIT_ENOTSYM (-2)   /* D or F is not symmetric */
#define PDIT_EBADPERM (-3)  /* a permutation row is not a permutation of 0..N-1 */
#define PDIT_EOVERFLOW (-4) /* an exact integer bound does not fit the requested arithmetic, or
                               an entry of D or F equals INT32_MIN */
#define PDIT_ENOMEM (-5)    /* device allocation failed */
#define PDIT_EDEVICE (-6)   /* HIP runtime error (text in pdit_last_error) */
#define PDIT_EBETA (-7)     /* an inverse temperature is NaN, infinite or negative */
#define PDIT_ESTATE (-8)    /* query before any run, or buffers of the wrong run */
#define PDIT_ECHECK (-9)    /* a paranoid recheck (pdit_opts.paranoid) found a replica whose state
                               differs from its recomputation from p (Eq. 1) */

#define PDIT_NMAX 512       /* largest supported instance size */

/* How H = D F[p,p] is recomputed at the start of a run (step "H recompute"). */
#define PDIT_RECOMPUTE_AUTO 0   /* cheapest exact mode for the data */
#define PDIT_RECOMPUTE_PLAIN 1  /* vector ALU, int64 accumulation */
#define PDIT_RECOMPUTE_I8 2     /* int8 MFMA, int32 accumulation: needs |D|,|F| <= 127 */
#define PDIT_RECOMPUTE_BF16 3   /* bf16 MFMA, fp32 accumulation: needs |D|,|F| <= 256 and |H| < 2^24 */
#define PDIT_RECOMPUTE_SPLIT 4  /* int8 MFMA on 7-bit byte planes, int64 combine: needs |D|,|F| < 2^14 */

/* Which sweep kernel runs. */
#define PDIT_SWEEP_AUTO 0   /* fast kernel when the instance fits it, else large */
#define PDIT_SWEEP_PLAIN 1  /* one workgroup per replica, H in device memory */
#define PDIT_SWEEP_FAST 2   /* replica state on chip, speculative row evaluation; needs
                               |dE| < 2^30 - 1 and N <= 256.  N <= 128: the table of swap energy
                               changes in LDS, |D|, |F| <= 32767; N <= 160: 2H int32 in LDS;
                               N <= 256: 2H int16 in LDS, |2H| <= 32767 */
#define PDIT_SWEEP_CLIQUE 3 /* clique flows (Methods, "CPU-PIM Algorithm", tai256c): F[a][b] =
                               c(a) c(b) for a != b with c in {0, 1} (a clique on a facility
                               subset, unit flows), F[a][a] = 0, D with a zero diagonal, N <= 512,
                               (4N + 2) max|D| < 2^30.  The energy depends only on the set S of
                               locations holding clique facilities; with g(x) = sum_{j in S}
                               D[x][j] an exchange inside a class changes nothing and one across
                               the classes changes E by 2 (g(s) - g(r) - D[r][s]) (r in S), so a
                               candidate costs O(1) and an accepted move O(N).  Same dynamics and
                               results as the other kernels.  AUTO picks it for N > 128 when the
                               data qualify (FAST keeps the general on-chip kernels); CLIQUE
                               forces it (PDIT_EINVAL when they do not).  pdit_last_plan reports
                               PDIT_SWEEP_CLIQUE. */
#define PDIT_SWEEP_LARGE 4  /* no stored H, any N <= PDIT_NMAX: for the update of location r
                               (Eq. 3 with I = -2H, H = D F[p,p]) column r of H is recomputed as
                               D f with f = F[p(r)][p(.)], row r as F^T applied to row r of D
                               ordered by facility (2 N^2 multiply-adds on rows of D and F that
                               all replicas share through the cache), diag H is kept on chip and
                               moved in O(N) per accepted exchange.  One pass over D and F
                               serves several consecutive locations: eight with values <= 16383
                               (int8 planes, MFMA products), three with values <= 32767 (two in
                               batched runs); an accepted exchange corrects the later ones'
                               sums in O(N).  512 threads per replica.
                               Same dynamics and results as the other kernels.  AUTO picks it
                               wherever the fast kernel does not fit: single runs, beta-range
                               selection, periodic tempering (diag H is the state saved
                               between periods) and batched runs (a persistent group per copy
                               layout, product width and H width). */
#define PDIT_SWEEP_REG 5    /* G = D F[p,:] in registers, 128 < N <= 256: lane j of wave w
                               of the replica's four keeps the 4 x 64 tile of G at rows
                               4j .. 4j+3 and facilities 64w .. 64w+63 (H[i][k] = G[i][p(k)])
                               as packed int16 pairs, exact while |H| <= 32767; an accepted
                               exchange of the facilities a = p(r), b = p(s) adds the rank-1
                               term (D[i][r] - D[i][s]) (F[b][c] - F[a][c]) and moves no
                               column; D and F are 8-bit copies in LDS ([0, 255] or
                               [-128, 127]) shared by the two replicas of a workgroup.  Same
                               dynamics and results as the other kernels.  AUTO picks it for
                               single-instance runs wherever the data fit; REG forces it
                               (PDIT_EOVERFLOW when they do not). */

typedef struct pdit_ctx pdit_t;

typedef struct {
    int device;           /* HIP device ordinal */
    void *stream;         /* hipStream_t to run on; NULL = the device's null stream */
    int recompute;        /* PDIT_RECOMPUTE_* */
    int sweep;            /* PDIT_SWEEP_* */
    int blocks_per_cu;    /* batched runs: resident workgroups per CU of the persistent
                             kernels (one replica each); 0 = as many as fit */
    int seq_threshold;    /* fast kernel: accepted moves in a sweep above which the next sweep
                             runs one update at a time; < 0 = default: max(4, N/4) for
                             N <= 128, 3 above */
    int paranoid;         /* nonzero: pdit_run_sweeps runs one sweep per launch and after each
                             one recomputes every replica from its permutation and checks it
                             (see pdit_run_sweeps); 0 = off (the default) */
} pdit_opts;

typedef struct {
    int64_t updates;      /* p-dit updates done (stays included) */
    int64_t accepted;     /* updates that swapped two facilities */
    int64_t ties;         /* draws within 2^-20 of a boundary between two candidates */
} pdit_counters_t;

/* One instance of a batched run (pdit_run_sweeps_batch). */
typedef struct {
    int32_t N;            /* instance size, 2..PDIT_NMAX */
    int32_t R;            /* replicas of this instance, >= 1 */
    const int32_t *D;     /* device, N x N, symmetric */
    const int32_t *F;     /* device, N x N, symmetric */
    int32_t *perm;        /* device, R x N, in/out */
    const float *beta;    /* device, n_sweeps values */
    int32_t *choices;     /* optional (NULL: not recorded): device int32 R x n_sweeps x N, the
                             drawn candidate of every update of this instance */
    int64_t *E_trace;     /* optional (NULL: not recorded): device int64 R x n_sweeps, the
                             energy after every sweep */
} pdit_instance;

/* Fills *opts with the defaults (device 0, null stream, AUTO modes). */
void pdit_default_opts(pdit_opts *opts);

/* Creates a context on opts->device (opts may be NULL for defaults).
 * *out receives the context; on error *out is NULL. */
int pdit_create(pdit_t **out, const pdit_opts *opts);

/* Waits for the context's stream, frees everything it owns.  NULL is a no-op. */
int pdit_destroy(pdit_t *ctx);

/*
 * Runs n_sweeps sweeps (Results, "Implementation": every p-dit initiates one
 * update per iteration; Eq. 3 and Eq. 5) on R independent replicas of one
 * instance.
 *   N       instance size, 2..PDIT_NMAX
 *   D, F    device int32 N x N, symmetric (PDIT_ENOTSYM otherwise)
 *   R       replicas, >= 1
 *   perm    device int32 R x N, in/out: initial permutations, replaced by the
 *           final ones (PDIT_EBADPERM if a row is not a permutation)
 *   beta    device float n_sweeps: inverse temperature of each sweep,
 *           finite and >= 0 (PDIT_EBETA otherwise)
 *   seed    Philox key
 * Sweep t uses global sweep index g = offset + t, where offset is the
 * context's sweep offset, which then advances by n_sweeps; so two calls of
 * T1 and T2 sweeps give the same result as one call of T1 + T2.  H is
 * recomputed exactly from perm at the start of every call.  The best state
 * (pdit_best) carries over between calls with the same N and R and is reset
 * otherwise.  Validation reads small summaries back to the host, so the call
 * synchronises once before the sweeps are queued; the sweeps themselves run
 * asynchronously.
 *
 * With opts.paranoid set, each sweep is its own launch (same draws and
 * results), and after each one the call synchronises and checks every
 * replica: its permutation and best permutation are permutations of 0..N-1;
 * its energy and best energy equal Eq. 1 recomputed exactly from them
 * (H = D F[p,p], E = tr H, the run's own recompute mode); and where H is
 * kept in device memory between updates (the plain kernel) every entry of H
 * equals the recomputation.  The first failing sweep returns PDIT_ECHECK,
 * with the sweep index and the counts in pdit_last_error, and leaves the
 * state of that sweep in place.  Recording (pdit_set_recording) is not
 * available in this mode (PDIT_EINVAL).
 */
int pdit_run_sweeps(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                    int32_t *perm, const float *beta, int64_t n_sweeps, uint64_t seed);

/*
 * Runs n_sweeps sweeps on every replica of n_inst instances of uneven size
 * (the paper's independent duplicated replica sets, Results "GPU
 * Implementations" and Methods "GPU-PIM Algorithm": persistent kernels over
 * duplicates x replicas).  Each instance is validated and given exact widths
 * as in pdit_run_sweeps; the (instance, replica) work items are handed out
 * largest N first by persistent kernels (the on-chip kernel for N <= 128
 * when the data fit it, the plain kernel otherwise), whose launches are
 * captured once in a HIP graph and replayed while the batch keeps the same
 * shape and buffers.  Instance n's replicas use Philox counter word 3 = n.
 * Replica state is laid out instance after instance: R_total = sum R_n
 * energies, and permutation rows of each instance's own length N_n.
 *   inst   host array of n_inst descriptors (device pointers inside)
 * The sweep offset and best state behave as in pdit_run_sweeps.  Recording
 * goes through each instance's choices and E_trace pointers (pdit_set_recording
 * applies to single-instance runs only); the buffers are part of what the
 * captured graph was built for, so changing them captures a new graph.
 */
int pdit_run_sweeps_batch(pdit_t *ctx, int32_t n_inst, const pdit_instance *inst,
                          int64_t n_sweeps, uint64_t seed);

/* Parallel tempering (pdit_run_pt). */
#define PDIT_PT_MAXL 64     /* largest number of replicas per set */
typedef struct {
    int32_t L;              /* replicas per set, 1..PDIT_PT_MAXL: rows k L .. k L + L - 1 of
                               perm form set k */
    const float *beta;      /* device float L: inverse temperature of each rung, ascending
                               (rung 0 is the hottest), finite and >= 0 */
    int32_t *slot;          /* device int32 R, in/out: rung of each replica in its set; each
                               set's values a permutation of 0..L-1 (PDIT_EINVAL otherwise) */
    int32_t *since_top;     /* device int32 R / L, in/out: exchange passes since the set's top
                               rung last changed hands (start at 0) */
    int64_t period_sweeps;  /* sweeps between exchange passes (4 in the paper) */
    int32_t timeout;        /* passes without the top rung changing hands after which it trades
                               with the bottom rung (100 in the paper); <= 0: never */
    int32_t schedule;       /* PDIT_PT_AUTO, PDIT_PT_PERIODIC or PDIT_PT_FUSED (below) */
    int32_t dynamics;       /* PDIT_PT_SEQUENTIAL: sweeps as in pdit_run_sweeps;
                               PDIT_PT_CUPIM: iterations as in pdit_run_cupim (Methods,
                               "GPU-CUPIM Algorithm": the same exchange rules) on its on-chip
                               kernel, N <= 128 and |D|, |F| <= 127 (PDIT_EOVERFLOW
                               otherwise), and the periodic schedule */
} pdit_pt;

#define PDIT_PT_SEQUENTIAL 0
#define PDIT_PT_CUPIM 1

/* How pdit_run_pt launches its work; every schedule gives the same results.
 *   PERIODIC  one sweep launch per period (each replica's state saved and
 *             reloaded between them) and one exchange launch per period.
 *   FUSED     N <= 128 and data that fit the fast kernel (PDIT_SWEEP_FAST):
 *             every period in one cooperative launch per group of whole sets
 *             that are resident at once; the members of a set meet on the
 *             device after each period and run the pass themselves.  A
 *             meeting that does not complete within max(20 s, 1000 times the
 *             waiting member's period) ends the call with PDIT_EDEVICE (the
 *             outputs are then undefined); with resident members it cannot
 *             happen.  Ends with a host synchronisation.
 *   AUTO      FUSED where it applies, else PERIODIC. */
#define PDIT_PT_AUTO 0
#define PDIT_PT_PERIODIC 1
#define PDIT_PT_FUSED 2

/*
 * Parallel tempering (Results, "Implementation"; Methods, "CPU-PIM
 * Algorithm"): n_periods periods, each of period_sweeps sweeps on every
 * replica at beta[slot[k]], followed by one exchange pass per set.  The pass
 * visits the rungs from the lowest beta up; when the replica on rung i+1 has
 * an energy greater than or equal to the replica on rung i, their
 * configurations change rungs (slot values are exchanged; states and random
 * streams stay with the replicas).  When the top rung has not changed hands
 * for `timeout` passes it trades with the bottom rung.  Replica k draws from
 * its own Philox stream (counter word 2 = k); sweep offset, best state and
 * counters (totals of the call) behave as in pdit_run_sweeps, with
 * n_periods x period_sweeps sweeps.  Each replica's on-chip state carries
 * from one period to the next.  Recording is not available.
 */
int pdit_run_pt(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                int32_t *perm, const pdit_pt *pt, int64_t n_periods, uint64_t seed);

/*
 * GPU-CUPIM, concurrent updates (Results, "GPU Implementations"; Methods,
 * "GPU-CUPIM Algorithm"): a different dynamics from pdit_run_sweeps.  In
 * each iteration every location draws (Eq. 5, the same weights and Philox
 * stream as a sweep) from a snapshot of the swap energy changes (Eq. 3)
 * taken at the iteration's start.  Location r proposes exchanging its
 * facility with its draw s != r; the proposal's key is (snapshot dE, r),
 * smaller first -- the larger energy decrease wins, a tie goes to the lower
 * proposing index -- and a proposal is applied when it holds the smallest
 * key at both of its locations (one round; losers stay).  All applied
 * exchanges are disjoint and happen together; then the snapshot is
 * refreshed.  Arguments, sweep offset, best state (checked once per
 * iteration) and outputs as in pdit_run_sweeps; counters: updates = N per
 * iteration, accepted = applied exchanges, ties = draws within the tie
 * band.  Any N <= PDIT_NMAX: with N <= 128 and |D|, |F| <= 127 the
 * replica's snapshot stays on chip (one launch; the refresh on int8 MFMA);
 * otherwise the snapshot H + H^T lives in device memory and each iteration
 * is a draw, a resolve and an exact H recompute in the cheapest mode the
 * data allow (pdit_last_plan: PDIT_SWEEP_LARGE), which needs
 * 8 |H| + 16 max|D| max|F| < 2^53 (PDIT_EOVERFLOW otherwise).  Recording is
 * not available.  (pdit_run_pt with PDIT_PT_CUPIM keeps the on-chip limits.)
 */
int pdit_run_cupim(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                   int32_t *perm, const float *beta, int64_t n_sweeps, uint64_t seed);

/*
 * Beta-range selection (Results, "Implementation", Figure 2b; Methods,
 * "CPU-PIM Algorithm"): short trials at fixed beta, without exchanges, on an
 * ascending grid; the averaged ending energies fall with beta and turn up
 * again where the replicas freeze.  For every grid value g, R trial
 * replicas start from the rows of perm (unchanged by the call) and run
 * trial_sweeps sweeps (400 in the paper) at beta grid[g]; trial replica k of
 * grid value g draws as replica g R + k of a run from sweep 0 (the
 * context's sweep offset is neither used nor advanced).  Then, with Smax and
 * Smin the largest and smallest sums of ending energies:
 *   range[0] = lo, the first g whose sum is at most the level lying
 *              level_pct percent of Smax - Smin above Smin
 *              (100 E_sum[g] <= level_pct Smax + (100 - level_pct) Smin,
 *              exact).  The paper takes the energy that has dropped to about
 *              40% between the minimum and the maximum: level_pct = 40; 60
 *              gives the other reading of its wording (a drop of 40% from
 *              the maximum);
 *   range[1] = hi, two grid values past the first g holding Smin (at most
 *              G - 1);
 *   ladder[i] = grid[lo] (grid[hi] / grid[lo])^(i / (L - 1)), evaluated in
 *              double on the host and rounded to float, ladder[0] = grid[lo]
 *              and ladder[L - 1] = grid[hi] exactly: a parallel-tempering
 *              ladder (pdit_pt.beta) of L rungs.
 *   perm     device int32 R x N, the trials' starting permutations
 *   grid     device float G, finite, > 0, strictly ascending (PDIT_EBETA)
 *   level_pct  0..100 (PDIT_EINVAL otherwise)
 *   E_sum    device int64 G, out: summed ending energies (exact; the mean
 *            times R)
 *   ladder   device float L (L >= 2), out;   range: device int32 2, out
 * R * N * (bound on |H|) must stay below 2^59 (PDIT_EOVERFLOW).  The
 * context's replica state becomes that of the G * R trial replicas
 * (pdit_energy, pdit_best, pdit_replica_counters report them).  The rule
 * reads the sums back, so the call ends with a host synchronisation.
 * Recording is not available.
 */
int pdit_beta_select(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, const float *grid, int32_t G, int64_t trial_sweeps,
                     uint64_t seed, int32_t L, int32_t level_pct, int64_t *E_sum, float *ladder,
                     int32_t *range);

/* Result of pdit_autotune. */
typedef struct {
    int blocks_per_cu;    /* chosen resident workgroups per CU */
    int seq_threshold;    /* chosen sequential-sweep threshold */
    double best_ms;       /* trial time of the chosen setting */
    int cached;           /* 1: taken from the autotune cache file, no trials run */
} pdit_tuning;

/*
 * Times short trial batches (n_trial_sweeps sweeps of the given instances,
 * on private copies of their permutations, so nothing the caller owns
 * changes) for every resident-workgroups-per-CU count and a few sequential
 * thresholds, and stores the fastest setting in the context's options for
 * later runs.  *out may be NULL.
 *
 * Cache: if the environment variable PDIT_AUTOTUNE_CACHE names a file, the
 * setting is looked up there first, keyed by the device architecture, its
 * compute-unit count and the batch's shape (every instance's N, R and data
 * width: max(|D|, |F|) within 8, 16 or 32 bits, from the same validation as
 * a run); a hit applies the stored setting without trials (out->cached = 1),
 * a miss runs the trials and appends one line "key blocks_per_cu
 * seq_threshold best_ms" (the last line of a key wins).  The file is plain
 * text; concurrent writers are not coordinated.
 */
int pdit_autotune(pdit_t *ctx, int32_t n_inst, const pdit_instance *inst, int64_t n_trial_sweeps,
                  uint64_t seed, pdit_tuning *out);

/* E_out: device int64 R_total; current energies (Eq. 1) of the last run's
 * final permutations. */
int pdit_energy(pdit_t *ctx, int64_t *E_out);

/* E_best: device int64 R_total; perm_best: device int32, R_total rows of the
 * instance's N (packed instance after instance).  The lowest energy seen
 * since the best state was last reset, and the first permutation that
 * reached it (the best result an algorithm logs: Methods, "Hardware and Data
 * Reporting Details"). */
int pdit_best(pdit_t *ctx, int64_t *E_best, int32_t *perm_best);

/* Host struct: totals over all replicas of the last run (updates: one per
 * p-dit per sweep or iteration, Results "Implementation"; accepted moves;
 * draws in the tie band). */
int pdit_counters(pdit_t *ctx, pdit_counters_t *out);

/* Device int64 R_total x 3: per-replica (updates, accepted, ties) of the last run. */
int pdit_replica_counters(pdit_t *ctx, int64_t *out);

/* Sets / reads the global index of the next sweep (Philox counter word 1). */
int pdit_set_sweep_offset(pdit_t *ctx, uint64_t offset);
int pdit_get_sweep_offset(pdit_t *ctx, uint64_t *offset);

/* Forgets the best state: the next run starts it from its initial state. */
int pdit_reset(pdit_t *ctx);

/* Waits for the context's stream; returns any deferred device-side error. */
int pdit_sync(pdit_t *ctx);

/* Message of the last error on this context ("" if none).  Valid until the
 * next call on the context. */
const char *pdit_last_error(const pdit_t *ctx);

/*
 * Recording for tests and tracing; buffers apply to the next run only and
 * are then cleared.  choices: device int32 R_total x n_sweeps x N, the drawn
 * candidate of every update; E_trace: device int64 R_total x n_sweeps, the
 * energy after every sweep.  Either may be NULL.  Single-instance runs only.
 */
int pdit_set_recording(pdit_t *ctx, int32_t *choices, int64_t *E_trace);

/*
 * Step "H recompute" on its own: H = D F[p,p] and E = trace(H) (= Eq. 1)
 * for R permutations, in the given PDIT_RECOMPUTE_* mode (PDIT_EOVERFLOW if
 * that mode is not exact for the data).
 *   H_out  device int64 R x N x N (may be NULL), E_out device int64 R.
 * Afterwards pdit_last_timing reports the recompute (H in the library's own
 * buffer and its trace) as recompute_ms and the copy to H_out as sweep_ms,
 * and pdit_last_plan the mode that ran.
 */
int pdit_h_recompute(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, int mode, int64_t *H_out, int64_t *E_out);

/*
 * The energy changes the sweep kernels compute for the update of location r
 * (Eq. 3 specialised to symmetric data), for each of R permutations:
 *   delta_out  device int64 R x N; entry s is the change of swapping the
 *              facilities at r and s (0 at s = r).
 */
int pdit_debug_delta(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, int32_t r, int64_t *delta_out);

/*
 * The same steps on the context's own replica state: replica `replica` of
 * instance `inst` of the last pdit_run_sweeps, pdit_run_sweeps_batch,
 * pdit_run_cupim or pdit_run_pt (inst 0 for single-instance runs), read
 * through the D, F and perm pointers that run was given (the caller keeps
 * them alive; the replica's permutation as the stream reaches this call).
 *   pdit_debug_H      H = D F[p,p] of that replica (Eq. 2 with I = -2H for
 *                     symmetric data), location-indexed, as int64 whatever the
 *                     run stored: H_out device int64 N x N.
 *   pdit_debug_delta_replica  Eq. 3 for the update of location r of that
 *                     replica: delta_out device int64 N (0 at s = r).
 * PDIT_ESTATE before any such run; PDIT_EINVAL for an inst, replica or r out
 * of range.
 */
int pdit_debug_H(pdit_t *ctx, int32_t inst, int32_t replica, int64_t *H_out);
int pdit_debug_delta_replica(pdit_t *ctx, int32_t inst, int32_t replica, int32_t r,
                             int64_t *delta_out);

/*
 * The sweep kernels' Gibbs choice on its own: for each of M rows of N energy
 * changes (device int64 M x N) and device float beta[M], device uint32
 * u24[M], writes the chosen candidate (device int32 M) and a tie flag
 * (device int32 M, may be NULL).
 */
int pdit_debug_choice(pdit_t *ctx, int32_t N, int32_t M, const int64_t *delta, const float *beta,
                      const uint32_t *u24, int32_t *choice, int32_t *tie);

/* Device durations of the last run's steps, from HIP events recorded on the
 * context's stream around them (waits for the events): recompute_ms covers
 * the H recompute, sweep_ms the sweep kernel.  Either pointer may be NULL. */
int pdit_last_timing(pdit_t *ctx, double *recompute_ms, double *sweep_ms);

/* What the last single-instance run used: *sweep is PDIT_SWEEP_PLAIN,
 * PDIT_SWEEP_FAST, PDIT_SWEEP_CLIQUE, PDIT_SWEEP_LARGE or PDIT_SWEEP_REG,
 * *size_class the on-chip kernel's size class (16, 32, 64, 96, 128, 160 or
 * 256; 256 for the register kernel; 0 for the other kernels), *recompute
 * the PDIT_RECOMPUTE_*
 * mode of the H recompute.  Any pointer may be NULL. */
int pdit_last_plan(pdit_t *ctx, int *sweep, int *size_class, int *recompute);

/* Philox4x32-10 word 0 >> 8 for M counters (device uint32 M x 4) under seed,
 * written to device uint32 M. */
int pdit_debug_uniform24(pdit_t *ctx, int32_t M, const uint32_t *ctr, uint64_t seed,
                         uint32_t *out);

/* Size of the device work space of pdit_run_sweeps_noalloc, per GPU. */
#define PDIT_NOALLOC_SCRATCH_BYTES (64 << 20)

/*
 * pdit_run_sweeps for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid hipMalloc, code that must not grow the
 * device heap): no context, no hipMalloc, hipFree or allocating library
 * call.  The same sweeps, kernels and results as pdit_run_sweeps with the
 * given options (recording is not available).
 *
 * Work space: a device array of PDIT_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs this call on, until the process ends.  It
 * holds the instance summary, the clique membership, the copies of D and F
 * of the kernel without a stored H (up to 4 MiB), D and F in the MFMA
 * operand format of the H recompute (up to 1 MiB) and the initial H of every
 * replica (R N^2 int32, or int64 when the bound on |H| needs it); a run
 * that needs more returns PDIT_ENOMEM with a message.  Every call on a GPU
 * uses that GPU's one array (and one host copy of the instance summary), so
 * calls that overlap on one GPU, from two host threads or on two streams,
 * race: serialise them.  Nothing in the array needs clearing between calls.
 *
 *   opts       device, stream, sweep, recompute and seq_threshold as for
 *              pdit_create (NULL: the defaults); blocks_per_cu is unused;
 *              paranoid must be 0 (its rechecks need buffers: PDIT_EINVAL)
 *   N, D, F, R, perm, beta, n_sweeps, seed   as for pdit_run_sweeps
 *   sweep_offset  global index of the first sweep (Philox counter word 1)
 *   init_best  nonzero: E_best and perm_best start from the initial state;
 *              zero: they hold a previous best state and are updated
 *   E          device int64 R, out: energies of the final permutations
 *   E_best     device int64 R, in/out;  perm_best: device int32 R x N, in/out
 *   counters   device int64 R x 3, out: (updates, accepted, ties) per replica
 *   err        optional host buffer of err_len bytes: the error message
 * Validation synchronises the stream once, as in pdit_run_sweeps; the
 * sweeps then run asynchronously on the stream.
 */
int pdit_run_sweeps_noalloc(const pdit_opts *opts, int32_t N, const int32_t *D, const int32_t *F,
                            int32_t R, int32_t *perm, const float *beta, int64_t n_sweeps,
                            uint64_t seed, uint64_t sweep_offset, int init_best, int64_t *E,
                            int64_t *E_best, int32_t *perm_best, int64_t *counters, char *err,
                            int32_t err_len);

#ifdef __cplusplus
}
#endif

#endif /* PDIT_H */
