// pdit_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pdit.h"
#include "pt_common.h"
#include "sweep_common.h"

namespace pdit {

// Per-instance data summary computed on the device (step "instance prep").
struct InstanceStats {
    int32_t max_abs_d;      // max |D_ij|
    int32_t max_abs_f;      // max |F_ij|
    int64_t max_rowsum_d;   // max_i sum_j |D_ij|
    int64_t max_colsum_f;   // max_c sum_j |F_jc|
    int32_t asym_d;         // number of (i, j) with D_ij != D_ji
    int32_t asym_f;
    int32_t bad_perm_rows;  // rows of perm that are not permutations
    int32_t bad_beta;       // beta values that are NaN, infinite or negative
    int32_t diag_nz_d;      // nonzero diagonal entries of D
    int32_t diag_nz_f;      // nonzero diagonal entries of F
    int32_t bad_slots;      // parallel tempering: sets whose slots are not a permutation of
                            // 0..L-1, or whose pass counter is negative
    int32_t bad_grid;       // beta selection: grid values <= 0 or not above the previous one
    int32_t clique_bad;     // entries of F that break F[a][b] = c(a) c(b) (a != b), F[a][a] = 0
    int32_t clique_size;    // facilities with c(a) = 1
    int32_t int_min;        // entries of D or F equal to INT32_MIN (their magnitude needs 32 bits)
    int32_t neg_d;          // negative entries of D
    int32_t neg_f;          // negative entries of F
};

// Exact bound on |H_ik| for any permutation: |sum_j D_ij F_{p(j)p(k)}| <=
// min(max|D| * max col-sum |F|, max|F| * max row-sum |D|).
inline int64_t h_bound(const InstanceStats &s) {
    const int64_t b1 = (int64_t)s.max_abs_d * s.max_colsum_f;
    const int64_t b2 = (int64_t)s.max_abs_f * s.max_rowsum_d;
    return b1 < b2 ? b1 : b2;
}

// Bound on |dE| = |2 (H_rs + H_sr - H_rr - H_ss) + (D_rr + D_ss - 2 D_rs)
// (F_aa + F_bb - 2 F_ab)|.
inline int64_t delta_bound(const InstanceStats &s) {
    return 8 * h_bound(s) + 16 * (int64_t)s.max_abs_d * s.max_abs_f;
}

// Per-replica state buffers owned by the context (device memory).
struct ReplicaState {
    int n_inst = 0;
    std::vector<int32_t> Ns, Rs;      // shape signature of the last run
    int64_t R_total = 0;
    int64_t perm_total = 0;           // sum R_n * N_n
    int64_t *E = nullptr;             // [R_total]
    int64_t *E_best = nullptr;        // [R_total]
    int32_t *perm_best = nullptr;     // [perm_total]
    int64_t *counters = nullptr;      // [R_total * 3]
    bool best_valid = false;
};

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace pdit

struct pdit_ctx {
    pdit_opts opts;
    hipStream_t stream = nullptr;
    uint64_t sweep_offset = 0;
    std::string last_error;
    pdit::ReplicaState st;
    pdit::DeviceBuffer h_buf;         // H of all replicas (int32 or int64)
    pdit::DeviceBuffer tstate;        // table-kernel states between parallel-tempering periods
    pdit::DeviceBuffer pt_buf;        // fused parallel tempering: published energy words
    pdit::DeviceBuffer trial_buf;     // beta selection: trial permutations and their slots
    pdit::DeviceBuffer clique_buf;    // clique flows: membership of each facility
    pdit::DeviceBuffer large_buf;     // the large kernel's padded copies of D and F
    int coop = 0;                     // the device supports cooperative launches
    int wall_clock_khz = 0;
    pdit::DeviceBuffer scratch;       // small per-call scratch (stats, flags)
    pdit::DeviceBuffer check_buf;     // paranoid rechecks: recomputed energies, H and counts
    pdit::DeviceBuffer conv_buf;      // H recompute on MFMA: D and F in operand format
    pdit::DeviceBuffer cupim_buf;     // GPU-CUPIM beyond the on-chip kernel: S, diag H, draws
    // the instances of the last run (N, R, D, F, perm as given), for the
    // debug exports on the context's replica state
    std::vector<pdit_instance> last_insts;
    pdit::InstanceStats *stats_host = nullptr;  // pinned host mirror
    int32_t *err_dev = nullptr;       // deferred device error word
    int32_t *flag_host = nullptr;     // pinned: fused parallel tempering's wait flag
    int32_t *rec_choices = nullptr;   // recording buffers for the next run
    int64_t *rec_trace = nullptr;
    int64_t last_updates = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // before recompute, before sweep, after sweep
    bool timed = false;                               // events of the last run are recorded
    // batched runs: descriptors, work items, queues and per-call parameters
    pdit::DeviceBuffer batch_buf;
    hipStream_t capture_stream = nullptr;             // graphs are captured here, launched on `stream`
    // batched runs: one stream per group of the captured graph (forked from
    // and joined back to the capture stream, default priority) and the fork
    // and join events
    std::vector<hipStream_t> group_streams;
    std::vector<hipEvent_t> group_events;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<char> graph_sig;                      // what the captured graph was built for
    int num_cus = 0;
    int last_sweep = 0, last_class = 0, last_mode = 0;  // plan of the last single-instance run
    bool noalloc = false;  // borrowed buffers only (pdit_run_sweeps_noalloc): never allocate
};

namespace pdit {

// ---- launchers (each returns a hipError_t) --------------------------------
// Parallel tempering: slot validation (into out->bad_slots) and the exchange
// pass of every set after a period.
hipError_t launch_pt_check(hipStream_t s, int n_sets, int L, const int32_t *slot,
                           const int32_t *since_top, InstanceStats *out);
hipError_t launch_pt_exchange(hipStream_t s, int n_sets, int L, const int64_t *E, int32_t *slot,
                              int32_t *since_top, int32_t timeout);
hipError_t launch_grid_check(hipStream_t s, int G, const float *grid, InstanceStats *out);
// out[0 .. n-1] = 0 by a kernel (no memset node in code a caller may capture)
hipError_t launch_zero_i64(hipStream_t s, int64_t *out, int64_t n);
// clique flows: member[a] = c(a) (facility a has a nonzero flow), and the
// count of entries of F that break F = c c^T off the diagonal, 0 on it
hipError_t launch_clique_check(hipStream_t s, int N, const int32_t *F, int32_t *member,
                               InstanceStats *out);
// beta-range selection: trial replicas (perm rows repeated per grid value,
// slot = grid index), summed ending energies per grid value, the range rule
hipError_t launch_trial_setup(hipStream_t s, int N, int R, int G, const int32_t *perm,
                              int32_t *trial_perm, int32_t *slot);
hipError_t launch_group_sums(hipStream_t s, int R, int G, const int64_t *E, int64_t *E_sum);
hipError_t launch_instance_stats(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                                 int R, const int32_t *perm, const float *beta, int64_t T,
                                 InstanceStats *out_dev);
// paranoid rechecks: rows of perm (R x N) that are not permutations of
// 0..N-1, added to *bad; entries where two arrays of n elements of
// elem_bytes (4 or 8) bytes differ, added to *count
hipError_t launch_perm_rows_check(hipStream_t s, int N, int R, const int32_t *perm, int32_t *bad);
hipError_t launch_count_diff(hipStream_t s, int64_t n, int elem_bytes, const void *a,
                             const void *b, int32_t *count);

// g_layout: G = D F[p,:] (columns by facility, for the register sweep kernel)
// instead of H = D F[p,p]
hipError_t launch_h_recompute_plain(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                                    int R, const int32_t *perm, void *H, bool h64,
                                    int64_t *E, bool g_layout = false);
// operands: device work space of mfma_operand_bytes(mode, N) bytes for D and
// F in the MFMA operand format (rewritten by every call)
size_t mfma_operand_bytes(int mode, int N);
hipError_t launch_h_recompute_mfma(hipStream_t s, int mode, int N, const int32_t *D,
                                   const int32_t *F, int R, const int32_t *perm, void *H,
                                   bool h64, int64_t *E, bool g_layout, void *operands);
hipError_t launch_widen_h(hipStream_t s, int64_t count, const int32_t *src, int64_t *dst);

struct SweepArgs {
    int N;
    int R;
    const int32_t *D;
    const int32_t *F;
    int32_t *perm;           // [R][N] in/out
    void *H;                 // [R][N][N] int32 or int64, initial H (overwritten by plain)
    int64_t *E;              // [R] in: initial energies; out: final
    int64_t *E_best;         // [R] in/out
    int32_t *perm_best;      // [R][N] in/out
    int64_t *counters;       // [R][3] out
    const float *beta;       // [T]
    int64_t T;
    uint64_t seed;
    uint64_t sweep_offset;
    uint32_t inst_id;
    int32_t *choices;        // optional [R][T][N]
    int64_t *E_trace;        // optional [R][T]
    int seq_threshold;
    bool zero_diag;          // D and F have zero diagonals
    // parallel tempering: replica k runs every sweep of the launch at
    // beta[slot[k]] (null: the schedule beta[t])
    const int32_t *slot;
    int32_t *tstate;         // table kernel: [R][table_state_words(N)] replica state between launches
    uint32_t flags;          // kLoadState | kSaveState | kAccumCounters
    int32_t *err;            // deferred device error word (set to 1 on an internal wait's timeout), or null
};

// Launch flags of the sweep kernels (parallel-tempering periods).
constexpr uint32_t kLoadState = 1;      // resume from the saved state (table kernel: tstate)
constexpr uint32_t kSaveState = 2;      // save the state at the end (table: tstate; H kernels: H; large: diag H)
constexpr uint32_t kAccumCounters = 4;  // add to the counters instead of overwriting them
// int32 words of one replica's saved table state: the table (NMAX x (NMAX+4))
// and diag H (NMAX) of its size class
// Row pitch (int32) of the table kernel's table: N + 4 keeps a row quarter
// on distinct banks; at 96 the unpadded pitch already does (rows of 96 words
// start 32 banks apart), and it keeps two replicas of that class per CU.
__host__ __device__ constexpr int table_pitch(int nmax) { return nmax == 96 ? 96 : nmax + 4; }
__host__ __device__ inline int64_t table_state_words(int nmax) {
    return (int64_t)nmax * table_pitch(nmax) + nmax;
}

constexpr int kFastNMax = 256;            // largest N of the on-chip kernel
// Accepted moves in a sweep above which the fast kernels run the next sweep
// one update at a time.  On the table classes (N <= 128) a speculative pass
// plus an accepted move costs about a tenth of a sequential sweep, so the
// switch pays only for hot sweeps; the large classes switch early.
inline int default_seq_threshold(int nmax, int N) {
    if (nmax <= 128) return N / 4 > 4 ? N / 4 : 4;
    return 3;
}

// GPU-CUPIM (concurrent updates): one replica per workgroup, N <= 128,
// |D|, |F| <= 127; the kernel computes its own H and E.
struct CupimArgs {
    int N;
    int R;
    const int32_t *D;
    const int32_t *F;
    int32_t *perm;           // [R][N] in/out
    int64_t *E;              // [R] out
    int64_t *E_best;         // [R] in/out
    int32_t *perm_best;      // [R][N] in/out
    int64_t *counters;       // [R][3] out
    const float *beta;       // [T]
    int64_t T;
    uint64_t seed;
    uint64_t sweep_offset;
    uint32_t inst_id;
    bool zero_diag;
    int init_best;           // start the best state from the initial one
    const int32_t *slot;     // parallel tempering: replica k runs at beta[slot[k]] (else beta[t])
    int accumulate;          // add to the counters instead of overwriting them
};
struct CupimJob {
    int N;
    const int32_t *D;
    const int32_t *F;
    int32_t *perm;
    int64_t *E;
    int64_t *E_best;
    int32_t *perm_best;
    int64_t *counters;
    const float *beta;       // beta of iteration t is beta[t * beta_stride]
    int64_t beta_stride;
    int64_t T;
    uint64_t seed;
    uint64_t sweep_offset;
    uint32_t rep;
    uint32_t inst;
    int init_best;
    int accumulate;
};
// size class (16, 32, 64, 128) of the CUPIM kernel, 0 when it does not apply
inline int cupim_class(int N, const InstanceStats &st) {
    if (st.max_abs_d > 127 || st.max_abs_f > 127) return 0;
    return N <= 16 ? 16 : N <= 32 ? 32 : N <= 64 ? 64 : N <= 128 ? 128 : 0;
}
hipError_t launch_cupim(hipStream_t s, int nmax, const CupimArgs &c);

// GPU-CUPIM with the snapshot in device memory (any N <= PDIT_NMAX, entries
// beyond 8 bits): one iteration is draw, resolve, the H recompute into H,
// S = H + H^T with diag H, and the best state.
struct CupimLargeArgs {
    int N;
    int R;
    const int32_t *D;
    const int32_t *F;
    int32_t *perm;           // [R][N] in/out
    const int64_t *S;        // [R][N][N] H + H^T of the snapshot
    const int64_t *hd;       // [R][N] diag H
    int32_t *sel;            // [R][N] each location's draw
    int64_t *dsel;           // [R][N] its snapshot dE
    int32_t *tie;            // [R][N] the draw's threshold fell in the tie band
    int64_t *counters;       // [R][3] (updates, accepted, ties), added to
    const float *beta;       // [T] one value per iteration
    uint64_t seed;
    uint32_t inst_id;
    bool zero_diag;
};
hipError_t launch_cupim_large_draw(hipStream_t s, const CupimLargeArgs &c, int64_t t, uint32_t g);
hipError_t launch_cupim_large_resolve(hipStream_t s, const CupimLargeArgs &c);
hipError_t launch_cupim_large_sym(hipStream_t s, int N, int R, const void *H, bool h64,
                                  int64_t *S, int64_t *hd);
hipError_t launch_cupim_large_best(hipStream_t s, int N, int R, const int32_t *perm,
                                   const int64_t *E, int64_t *E_best, int32_t *perm_best);

// The sweep specialised to clique flows (one wave per replica, N <= 512).
struct CliqueArgs {
    int N;
    int R;
    const int32_t *D;
    const int32_t *member;   // [N] c(a) of each facility
    int32_t *perm;           // [R][N] in/out
    int64_t *E;              // [R] out
    int64_t *E_best;         // [R] in/out
    int32_t *perm_best;      // [R][N] in/out
    int64_t *counters;       // [R][3] out
    const float *beta;       // [T]
    int64_t T;
    uint64_t seed;
    uint64_t sweep_offset;
    uint32_t inst;
    int init_best;
    int32_t *choices;        // optional [R][T][N]
    int64_t *E_trace;        // optional [R][T]
};
constexpr int kCliqueNMax = 512;
// the clique kernel applies: F is a 0/1 clique, D has a zero diagonal, and
// every energy change 2 (g(s) - g(r) - D[r][s]) stays below 2^30 in magnitude
inline bool clique_fits(int N, const InstanceStats &st) {
    return N <= kCliqueNMax && st.clique_bad == 0 && st.diag_nz_d == 0 &&
           (4 * (int64_t)N + 2) * st.max_abs_d < (int64_t)(1 << 30) - 1;
}
hipError_t launch_sweep_clique(hipStream_t s, const CliqueArgs &a);

hipError_t launch_sweep_plain(hipStream_t s, const SweepArgs &a, bool h64);
// The kernel that stores no H (any N <= kLargeNMax, 512 threads per replica):
// reads diag H of the initial p from a.H (int64 when h64); with kSaveState it
// writes the final diag H there (the state between tempering periods) and
// leaves the rest of a.H stale.
// Its products read padded copies of D and F made by launch_large_copy.
constexpr int kLargeNMax = 512;
struct LargePlan {
    bool narrow = false;  // int32 partial sums of 24-bit products
    int elem = 4;         // bytes per element of the copies (2: int16, 1: int8 planes)
    bool planes = false;  // int8 hi/lo planes for the MFMA products (|D|, |F| <= 16383)
    int rows = 0;         // rows of each copy: int32, N rounded up to 32 plus 16 zero
                          // rows; int16 pairs, word rows N64 / 2 + 4; planes, N16
    size_t bytes = 0;     // both copies
};
struct LargeCopies {
    const void *D = nullptr;
    const void *F = nullptr;
};
LargePlan large_plan(int N, const InstanceStats &st);
hipError_t launch_large_copy(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                             const LargePlan &pl, void *buf, LargeCopies *out);
hipError_t launch_sweep_large(hipStream_t s, const SweepArgs &a, bool h64, const LargePlan &pl,
                              const LargeCopies &c);
struct BatchArgs;
hipError_t launch_sweep_large_persistent(hipStream_t s, const LargePlan &pl, bool h64,
                                         const BatchArgs &b, int grid);
int large_blocks_per_cu(const LargePlan &pl);
// size class of the on-chip kernel that runs an instance (16, 32, 64, 96, 128,
// 160 or 256), or 0 when its data do not fit that kernel's exact arithmetic
int fast_class(int N, const InstanceStats &st);
hipError_t launch_sweep_fast(hipStream_t s, int nmax, const SweepArgs &a);
// the kernel with G = D F[p,:] in registers (128 < N <= 256, 8-bit D and F,
// |H| <= 32767): 1 for unsigned copies, 2 for signed, 0 when it does not fit
int reg_class(int N, const InstanceStats &st);
hipError_t launch_sweep_reg(hipStream_t s, int cls, const SweepArgs &a);
hipError_t launch_sweep_fast_persistent(hipStream_t s, int nmax, bool zero_diag, const BatchArgs &b,
                                        int grid);
int fast_blocks_per_cu(int nmax);
// the N <= 128 classes (table of energy changes on chip), called by the above
hipError_t launch_sweep_table(hipStream_t s, int nmax, const SweepArgs &a);
hipError_t launch_sweep_table_persistent(hipStream_t s, int nmax, bool zero_diag, const BatchArgs &b,
                                         int grid);
int table_blocks_per_cu(int nmax);
// fused parallel tempering on the table classes: cooperative launches of as
// many whole sets as are resident at once
hipError_t launch_sweep_table_pt(hipStream_t s, int nmax, const SweepArgs &a, const PtFusedArgs &p,
                                 int num_cus);
hipError_t launch_sweep_plain_persistent(hipStream_t s, bool h64, const BatchArgs &b, int grid);
hipError_t launch_queue_reset(hipStream_t s, int *queue, int n);
int plain_blocks_per_cu(bool h64);

hipError_t launch_debug_delta(hipStream_t s, int N, const int32_t *D, const int32_t *F, int R,
                              const int32_t *perm, const int64_t *H, int r, int64_t *out);
hipError_t launch_debug_choice(hipStream_t s, int N, int M, const int64_t *delta,
                               const float *beta, const uint32_t *u24, int32_t *choice,
                               int32_t *tie);
hipError_t launch_debug_uniform24(hipStream_t s, int M, const uint32_t *ctr, uint64_t seed,
                                  uint32_t *out);

}  // namespace pdit
