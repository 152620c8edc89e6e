// api.hip -- the C ABI (include/pdit.h): validation, exact-width and mode
// selection, buffer management and kernel sequencing on the caller's stream.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>

#include "pdit_internal.h"

#include <cmath>

using pdit::InstanceStats;

namespace {

int fail(pdit_t *ctx, int code, const char *msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

// The last run's instances, for the debug exports.
void remember(pdit_t *ctx, int32_t N, int32_t R, const int32_t *D, const int32_t *F,
              int32_t *perm) {
    pdit_instance x{};
    x.N = N;
    x.R = R;
    x.D = D;
    x.F = F;
    x.perm = perm;
    ctx->last_insts.assign(1, x);
}

int fail_hip(pdit_t *ctx, hipError_t e, const char *where) {
    if (ctx) {
        ctx->last_error = std::string(where) + ": " + hipGetErrorString(e);
    }
    (void)hipGetLastError();  // clear the sticky-free error state
    return e == hipErrorOutOfMemory ? PDIT_ENOMEM : PDIT_EDEVICE;
}

#define PDIT_HIP(ctx, expr)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return fail_hip(ctx, e_, #expr); \
    } while (0)

// The step timers; a context made by the no-allocation entry point has none.
hipError_t record_event(pdit_t *ctx, int i) {
    return ctx->ev[i] ? hipEventRecord(ctx->ev[i], ctx->stream) : hipSuccess;
}

int ensure(pdit_t *ctx, pdit::DeviceBuffer &b, size_t bytes) {
    if (b.bytes >= bytes && b.ptr) return PDIT_OK;
    if (ctx->noalloc)
        return fail(ctx, PDIT_ENOMEM,
                    "the run needs more device memory than the no-allocation scratch holds "
                    "(PDIT_NOALLOC_SCRATCH_BYTES)");
    if (b.ptr) {
        PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        PDIT_HIP(ctx, hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 256);
    PDIT_HIP(ctx, hipMalloc(&b.ptr, want));
    b.bytes = want;
    return PDIT_OK;
}

void free_state(pdit::ReplicaState &s) {
    hipFree(s.E);
    hipFree(s.E_best);
    hipFree(s.perm_best);
    hipFree(s.counters);
    s.E = s.E_best = s.counters = nullptr;
    s.perm_best = nullptr;
    s.R_total = s.perm_total = 0;
    s.n_inst = 0;
    s.Ns.clear();
    s.Rs.clear();
    s.best_valid = false;
}

// (Re)shape the replica state for a run; returns PDIT_OK and sets *fresh when
// the best state has to start from the initial one.
int shape_state(pdit_t *ctx, const std::vector<int32_t> &Ns, const std::vector<int32_t> &Rs,
                bool *fresh) {
    pdit::ReplicaState &s = ctx->st;
    if (ctx->noalloc) {  // the caller's output buffers, set up for this one run
        *fresh = !s.best_valid;
        return PDIT_OK;
    }
    const bool same = s.E && s.Ns == Ns && s.Rs == Rs;
    if (!same) {
        PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        free_state(s);
        int64_t R_total = 0, perm_total = 0;
        for (size_t k = 0; k < Ns.size(); ++k) {
            R_total += Rs[k];
            perm_total += (int64_t)Rs[k] * Ns[k];
        }
        PDIT_HIP(ctx, hipMalloc(&s.E, sizeof(int64_t) * R_total));
        PDIT_HIP(ctx, hipMalloc(&s.E_best, sizeof(int64_t) * R_total));
        PDIT_HIP(ctx, hipMalloc(&s.perm_best, sizeof(int32_t) * perm_total));
        PDIT_HIP(ctx, hipMalloc(&s.counters, sizeof(int64_t) * 3 * R_total));
        s.Ns = Ns;
        s.Rs = Rs;
        s.n_inst = (int)Ns.size();
        s.R_total = R_total;
        s.perm_total = perm_total;
        s.best_valid = false;
    }
    *fresh = !s.best_valid;
    return PDIT_OK;
}

// Reads the instance summary (one host synchronisation) and validates.
int instance_prep(pdit_t *ctx, int N, const int32_t *D, const int32_t *F, int R,
                  const int32_t *perm, const float *beta, int64_t T, InstanceStats *st,
                  const pdit_pt *pt = nullptr, bool beta_is_grid = false,
                  int32_t *clique_member = nullptr) {
    int rc = ensure(ctx, ctx->scratch, sizeof(InstanceStats));
    if (rc) return rc;
    InstanceStats *dev = (InstanceStats *)ctx->scratch.ptr;
    PDIT_HIP(ctx, pdit::launch_instance_stats(ctx->stream, N, D, F, R, perm, beta, T, dev));
    if (pt)
        PDIT_HIP(ctx, pdit::launch_pt_check(ctx->stream, R / pt->L, pt->L, pt->slot,
                                            pt->since_top, dev));
    if (beta_is_grid) PDIT_HIP(ctx, pdit::launch_grid_check(ctx->stream, (int)T, beta, dev));
    if (clique_member)
        PDIT_HIP(ctx, pdit::launch_clique_check(ctx->stream, N, F, clique_member, dev));
    PDIT_HIP(ctx, hipMemcpyAsync(ctx->stats_host, dev, sizeof(InstanceStats),
                                 hipMemcpyDeviceToHost, ctx->stream));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *st = *ctx->stats_host;
    if (st->asym_d || st->asym_f) return fail(ctx, PDIT_ENOTSYM, "D or F is not symmetric");
    if (st->int_min)
        return fail(ctx, PDIT_EOVERFLOW, "D and F entries must be greater than INT32_MIN");
    if (st->bad_perm_rows)
        return fail(ctx, PDIT_EBADPERM, "a row of perm is not a permutation of 0..N-1");
    if (st->bad_beta) return fail(ctx, PDIT_EBETA, "an inverse temperature is NaN, infinite or negative");
    if (st->bad_grid)
        return fail(ctx, PDIT_EBETA, "the beta grid must be > 0 and strictly ascending");
    if (st->bad_slots)
        return fail(ctx, PDIT_EINVAL,
                    "the slots of a parallel-tempering set are not a permutation of 0..L-1, or its "
                    "pass counter is negative");
    // |H| <= bound, |dE| <= 8 bound + 16 max|D| max|F| must stay far inside int64
    const __int128 b1 = (__int128)st->max_abs_d * st->max_colsum_f;
    const __int128 b2 = (__int128)st->max_abs_f * st->max_rowsum_d;
    const __int128 b = b1 < b2 ? b1 : b2;
    if (b > ((__int128)1 << 58))
        return fail(ctx, PDIT_EOVERFLOW, "the exact bound on H exceeds the int64 range of the sweeps");
    return PDIT_OK;
}

bool recompute_exact(int mode, const InstanceStats &st, int64_t bound) {
    const int32_t mx = std::max(st.max_abs_d, st.max_abs_f);
    switch (mode) {
        case PDIT_RECOMPUTE_PLAIN: return true;
        case PDIT_RECOMPUTE_I8: return mx <= 127 && bound <= INT32_MAX;
        case PDIT_RECOMPUTE_BF16: return mx <= 256 && bound < (1 << 24);
        case PDIT_RECOMPUTE_SPLIT: return mx < (1 << 14);
        default: return false;
    }
}

int pick_recompute(pdit_t *ctx, const InstanceStats &st, int64_t bound, int requested, int *mode) {
    if (requested == PDIT_RECOMPUTE_AUTO) {
        for (int m : {PDIT_RECOMPUTE_I8, PDIT_RECOMPUTE_BF16, PDIT_RECOMPUTE_SPLIT, PDIT_RECOMPUTE_PLAIN})
            if (recompute_exact(m, st, bound)) {
                *mode = m;
                return PDIT_OK;
            }
    }
    if (requested < PDIT_RECOMPUTE_PLAIN || requested > PDIT_RECOMPUTE_SPLIT)
        return fail(ctx, PDIT_EINVAL, "unknown recompute mode");
    if (!recompute_exact(requested, st, bound))
        return fail(ctx, PDIT_EOVERFLOW, "the requested recompute mode is not exact for this data");
    *mode = requested;
    return PDIT_OK;
}

hipError_t run_recompute(pdit_t *ctx, int mode, int N, const int32_t *D, const int32_t *F, int R,
                         const int32_t *perm, void *H, bool h64, int64_t *E,
                         bool g_layout = false) {
    if (mode == PDIT_RECOMPUTE_PLAIN)
        return pdit::launch_h_recompute_plain(ctx->stream, N, D, F, R, perm, H, h64, E, g_layout);
    // (a failure here leaves its message and reads as out of memory)
    if (ensure(ctx, ctx->conv_buf, pdit::mfma_operand_bytes(mode, N)) != PDIT_OK)
        return hipErrorOutOfMemory;
    return pdit::launch_h_recompute_mfma(ctx->stream, mode, N, D, F, R, perm, H, h64, E, g_layout,
                                         ctx->conv_buf.ptr);
}

}  // namespace

extern "C" {

void pdit_default_opts(pdit_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->recompute = PDIT_RECOMPUTE_AUTO;
    o->sweep = PDIT_SWEEP_AUTO;
    o->blocks_per_cu = 0;
    o->seq_threshold = -1;
    o->paranoid = 0;
}

int pdit_create(pdit_t **out, const pdit_opts *opts) {
    if (!out) return PDIT_EINVAL;
    *out = nullptr;
    pdit_t *ctx = new (std::nothrow) pdit_ctx();
    if (!ctx) return PDIT_ENOMEM;
    if (opts)
        ctx->opts = *opts;
    else
        pdit_default_opts(&ctx->opts);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ctx->opts.device < 0 || ctx->opts.device >= ndev) {
        (void)hipGetLastError();
        delete ctx;
        return PDIT_EDEVICE;
    }
    if (hipSetDevice(ctx->opts.device) != hipSuccess) {
        delete ctx;
        return PDIT_EDEVICE;
    }
    // NULL is the device's null stream, which is also torch's default stream
    ctx->stream = (hipStream_t)ctx->opts.stream;
    for (auto &e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            pdit_destroy(ctx);
            return PDIT_EDEVICE;
        }
    }
    if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount,
                              ctx->opts.device) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->coop, hipDeviceAttributeCooperativeLaunch, ctx->opts.device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&ctx->wall_clock_khz, hipDeviceAttributeWallClockRate,
                              ctx->opts.device) != hipSuccess) {
        pdit_destroy(ctx);
        return PDIT_EDEVICE;
    }
    if (hipHostMalloc((void **)&ctx->stats_host, sizeof(InstanceStats), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc((void **)&ctx->err_dev, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->flag_host, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        pdit_destroy(ctx);
        return PDIT_ENOMEM;
    }
    if (hipMemset(ctx->err_dev, 0, sizeof(int32_t)) != hipSuccess) {
        pdit_destroy(ctx);
        return PDIT_EDEVICE;
    }
    *out = ctx;
    return PDIT_OK;
}

int pdit_destroy(pdit_t *ctx) {
    if (!ctx) return PDIT_OK;
    hipSetDevice(ctx->opts.device);
    hipStreamSynchronize(ctx->stream);
    free_state(ctx->st);
    hipFree(ctx->h_buf.ptr);
    hipFree(ctx->tstate.ptr);
    hipFree(ctx->pt_buf.ptr);
    hipFree(ctx->trial_buf.ptr);
    hipFree(ctx->clique_buf.ptr);
    hipFree(ctx->large_buf.ptr);
    hipFree(ctx->scratch.ptr);
    hipFree(ctx->check_buf.ptr);
    hipFree(ctx->conv_buf.ptr);
    hipFree(ctx->cupim_buf.ptr);
    hipFree(ctx->err_dev);
    for (auto &e : ctx->ev)
        if (e) hipEventDestroy(e);
    if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
    hipFree(ctx->batch_buf.ptr);
    if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
    for (auto st : ctx->group_streams) hipStreamDestroy(st);
    for (auto ev : ctx->group_events) hipEventDestroy(ev);
    if (ctx->stats_host) hipHostFree(ctx->stats_host);
    if (ctx->flag_host) hipHostFree(ctx->flag_host);
    delete ctx;
    return PDIT_OK;
}

// The clique-flow sweep (validated by the caller): no H; the kernel builds
// its own state from D, the facility membership and p.
int run_clique(pdit_t *ctx, int32_t N, const int32_t *D, int32_t R, int32_t *perm,
               const float *beta, int64_t n_sweeps, uint64_t seed) {
    bool fresh = false;
    int rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;
    pdit::CliqueArgs a{};
    a.N = N;
    a.R = R;
    a.D = D;
    a.member = (const int32_t *)ctx->clique_buf.ptr;
    a.perm = perm;
    a.E = S.E;
    a.E_best = S.E_best;
    a.perm_best = S.perm_best;
    a.counters = S.counters;
    a.beta = beta;
    a.T = n_sweeps;
    a.seed = seed;
    a.sweep_offset = ctx->sweep_offset;
    a.inst = 0;
    a.init_best = fresh ? 1 : 0;
    a.choices = ctx->rec_choices;
    a.E_trace = ctx->rec_trace;
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, record_event(ctx, 1));
    PDIT_HIP(ctx, pdit::launch_sweep_clique(ctx->stream, a));
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->rec_choices = nullptr;
    ctx->rec_trace = nullptr;
    ctx->sweep_offset += (uint64_t)n_sweeps;
    ctx->last_updates = (int64_t)R * N * n_sweeps;
    ctx->last_sweep = PDIT_SWEEP_CLIQUE;
    ctx->last_class = 0;
    ctx->last_mode = 0;
    S.best_valid = true;
    return PDIT_OK;
}

}  // extern "C"

// Paranoid mode of pdit_run_sweeps: one launch per sweep (the later ones
// adding to the counters), then every replica checked against its exact
// recomputation from p (Eq. 1): both permutations, E and E_best, and H
// itself where the kernel keeps it in device memory (plain).  For the other
// kernels the recompute of p is written to the H buffer, which is what the
// next launch starts from.
template <typename Launch>
int paranoid_sweeps(pdit_t *ctx, const pdit::SweepArgs &a, Launch &&launch, int mode, bool h64,
                    bool g_layout, bool h_resident) {
    const int N = a.N, R = a.R;
    const size_t hbytes = (size_t)R * N * N * (h64 ? 8 : 4);
    const size_t head = 256 + 2 * sizeof(int64_t) * (size_t)R;
    int rc = ensure(ctx, ctx->check_buf, head + (h_resident ? hbytes : 0));
    if (rc) return rc;
    char *base = (char *)ctx->check_buf.ptr;
    int32_t *counts = (int32_t *)base;   // bad perm rows, bad best rows, E, E_best, H
    int64_t *E_chk = (int64_t *)(base + 256);
    int64_t *Eb_chk = E_chk + R;
    void *Hc = h_resident ? (void *)(base + head) : ctx->h_buf.ptr;
    pdit::ReplicaState &S = ctx->st;
    for (int64_t t = 0; t < a.T; ++t) {
        pdit::SweepArgs x = a;
        x.beta = a.beta + t;
        x.T = 1;
        x.sweep_offset = a.sweep_offset + (uint64_t)t;
        x.flags = t ? pdit::kAccumCounters : 0u;
        PDIT_HIP(ctx, launch(x));
        PDIT_HIP(ctx, pdit::launch_zero_i64(ctx->stream, (int64_t *)counts, 4));
        PDIT_HIP(ctx, pdit::launch_perm_rows_check(ctx->stream, N, R, a.perm, &counts[0]));
        PDIT_HIP(ctx, pdit::launch_perm_rows_check(ctx->stream, N, R, S.perm_best, &counts[1]));
        int32_t host[5] = {0, 0, 0, 0, 0};
        PDIT_HIP(ctx, hipMemcpyAsync(host, counts, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                     ctx->stream));
        PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const uint64_t g = x.sweep_offset;
        if (host[0] || host[1]) {
            char msg[160];
            snprintf(msg, sizeof msg,
                     "paranoid recheck after sweep %llu: %d rows of perm and %d of perm_best are "
                     "not permutations", (unsigned long long)g, host[0], host[1]);
            return fail(ctx, PDIT_ECHECK, msg);
        }
        // the best states first, so that the H buffer ends with H of p
        PDIT_HIP(ctx, run_recompute(ctx, mode, N, a.D, a.F, R, S.perm_best, Hc, h64, Eb_chk,
                                    g_layout));
        PDIT_HIP(ctx, pdit::launch_count_diff(ctx->stream, R, 8, Eb_chk, S.E_best, &counts[3]));
        PDIT_HIP(ctx, run_recompute(ctx, mode, N, a.D, a.F, R, a.perm, Hc, h64, E_chk, g_layout));
        PDIT_HIP(ctx, pdit::launch_count_diff(ctx->stream, R, 8, E_chk, S.E, &counts[2]));
        if (h_resident)
            PDIT_HIP(ctx, pdit::launch_count_diff(ctx->stream, (int64_t)R * N * N, h64 ? 8 : 4, Hc,
                                                  ctx->h_buf.ptr, &counts[4]));
        PDIT_HIP(ctx, hipMemcpyAsync(host, counts, sizeof host, hipMemcpyDeviceToHost,
                                     ctx->stream));
        PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (host[2] || host[3] || host[4]) {
            char msg[200];
            snprintf(msg, sizeof msg,
                     "paranoid recheck after sweep %llu: %d replicas' energies and %d best "
                     "energies differ from Eq. 1, %d entries of H from D F[p,p]",
                     (unsigned long long)g, host[2], host[3], host[4]);
            return fail(ctx, PDIT_ECHECK, msg);
        }
    }
    return PDIT_OK;
}

extern "C" {

int pdit_run_sweeps(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                    int32_t *perm, const float *beta, int64_t n_sweeps, uint64_t seed) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || (!beta && n_sweeps > 0))
        return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 2 || N > PDIT_NMAX) return fail(ctx, PDIT_EINVAL, "N must be in [2, PDIT_NMAX]");
    if (R < 1) return fail(ctx, PDIT_EINVAL, "R must be >= 1");
    if (n_sweeps < 0) return fail(ctx, PDIT_EINVAL, "n_sweeps must be >= 0");
    if (ctx->opts.sweep < PDIT_SWEEP_AUTO || ctx->opts.sweep > PDIT_SWEEP_REG)
        return fail(ctx, PDIT_EINVAL, "unknown sweep kernel");
    const bool paranoid = ctx->opts.paranoid != 0;
    if (paranoid && (ctx->rec_choices || ctx->rec_trace))
        return fail(ctx, PDIT_EINVAL, "recording is not available with paranoid rechecks");
    if (paranoid && ctx->noalloc)
        return fail(ctx, PDIT_EINVAL, "paranoid rechecks need buffers: not without allocation");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));

    // clique flows are looked for where the table kernel does not apply
    const bool try_clique = ctx->opts.sweep == PDIT_SWEEP_CLIQUE ||
                            (ctx->opts.sweep == PDIT_SWEEP_AUTO && N > 128);
    int rc = PDIT_OK;
    if (try_clique) {
        rc = ensure(ctx, ctx->clique_buf, sizeof(int32_t) * (size_t)N);
        if (rc) return rc;
    }
    InstanceStats st;
    rc = instance_prep(ctx, N, D, F, R, perm, beta, n_sweeps, &st, nullptr, false,
                       try_clique ? (int32_t *)ctx->clique_buf.ptr : nullptr);
    if (rc) return rc;
    if (try_clique && pdit::clique_fits(N, st) && !paranoid) {
        rc = run_clique(ctx, N, D, R, perm, beta, n_sweeps, seed);
        if (rc == PDIT_OK) remember(ctx, N, R, D, F, perm);
        return rc;
    }
    if (paranoid && ctx->opts.sweep == PDIT_SWEEP_CLIQUE)
        return fail(ctx, PDIT_EINVAL, "the clique kernel has no paranoid rechecks");
    if (ctx->opts.sweep == PDIT_SWEEP_CLIQUE)
        return fail(ctx, PDIT_EINVAL,
                    "the clique kernel needs F = c c^T off the diagonal (0/1, a facility subset), "
                    "zero diagonals, N <= 512 and (4N + 2) max|D| < 2^30");
    const int64_t bound = pdit::h_bound(st);
    const bool h64 = bound > INT32_MAX;
    // the register kernel (G in registers, 8-bit D and F in LDS) where it fits
    const int rclass = pdit::reg_class(N, st);
    if (ctx->opts.sweep == PDIT_SWEEP_REG && !rclass)
        return fail(ctx, PDIT_EOVERFLOW,
                    "the register sweep kernel needs 128 < N <= 256, |H| <= 32767 and D, F in "
                    "[0, 255] or in [-128, 127]");
    const bool use_reg = rclass != 0 && (ctx->opts.sweep == PDIT_SWEEP_REG ||
                                         ctx->opts.sweep == PDIT_SWEEP_AUTO);
    // the on-chip kernel's size class, 0 if the data do not fit its exact arithmetic
    const int fclass = use_reg ? 0 : pdit::fast_class(N, st);
    bool use_fast = false;
    if (ctx->opts.sweep == PDIT_SWEEP_FAST) {
        if (!fclass)
            return fail(ctx, PDIT_EOVERFLOW,
                        "the fast sweep kernel needs N <= 256, |dE| < 2^30 and, by size, "
                        "|D|, |F| <= 32767 (N <= 128) or |2H| <= 32767 (N > 160)");
        use_fast = true;
    } else if (ctx->opts.sweep == PDIT_SWEEP_AUTO) {
        use_fast = fclass != 0;
    }
    // without a fast class the kernel that stores no H replaces the plain one
    const bool use_large = !use_reg && (ctx->opts.sweep == PDIT_SWEEP_LARGE ||
                                        (ctx->opts.sweep == PDIT_SWEEP_AUTO && !use_fast));
    int mode = 0;
    rc = pick_recompute(ctx, st, bound, ctx->opts.recompute, &mode);
    if (rc) return rc;

    rc = ensure(ctx, ctx->h_buf, (size_t)R * N * N * (h64 ? 8 : 4));
    if (rc) return rc;
    const pdit::LargePlan lplan = use_large ? pdit::large_plan(N, st) : pdit::LargePlan{};
    if (use_large) {
        rc = ensure(ctx, ctx->large_buf, lplan.bytes);
        if (rc) return rc;
    }
    bool fresh = false;
    rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;

    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    // the register kernel takes G = D F[p,:] (its tile rows read contiguously)
    PDIT_HIP(ctx, run_recompute(ctx, mode, N, D, F, R, perm, ctx->h_buf.ptr, h64, S.E, use_reg));
    pdit::LargeCopies lcopy;
    if (use_large)
        PDIT_HIP(ctx, pdit::launch_large_copy(ctx->stream, N, D, F, lplan, ctx->large_buf.ptr,
                                              &lcopy));
    if (fresh) {
        PDIT_HIP(ctx, hipMemcpyAsync(S.E_best, S.E, sizeof(int64_t) * R, hipMemcpyDeviceToDevice,
                                     ctx->stream));
        PDIT_HIP(ctx, hipMemcpyAsync(S.perm_best, perm, sizeof(int32_t) * (size_t)R * N,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    }
    pdit::SweepArgs a{};
    a.N = N;
    a.R = R;
    a.D = D;
    a.F = F;
    a.perm = perm;
    a.H = ctx->h_buf.ptr;
    a.E = S.E;
    a.E_best = S.E_best;
    a.perm_best = S.perm_best;
    a.counters = S.counters;
    a.beta = beta;
    a.T = n_sweeps;
    a.seed = seed;
    a.sweep_offset = ctx->sweep_offset;
    a.inst_id = 0;
    a.choices = ctx->rec_choices;
    a.E_trace = ctx->rec_trace;
    a.seq_threshold = ctx->opts.seq_threshold;
    a.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    a.err = ctx->err_dev;
    PDIT_HIP(ctx, record_event(ctx, 1));
    auto launch = [&](const pdit::SweepArgs &x) -> hipError_t {
        if (use_reg) return pdit::launch_sweep_reg(ctx->stream, rclass, x);
        if (use_fast) return pdit::launch_sweep_fast(ctx->stream, fclass, x);
        if (use_large) return pdit::launch_sweep_large(ctx->stream, x, h64, lplan, lcopy);
        return pdit::launch_sweep_plain(ctx->stream, x, h64);
    };
    if (n_sweeps > 0 && paranoid) {
        rc = paranoid_sweeps(ctx, a, launch, mode, h64, use_reg,
                             !use_reg && !use_fast && !use_large);
        if (rc) return rc;
    } else if (n_sweeps > 0) {
        PDIT_HIP(ctx, launch(a));
    } else {
        PDIT_HIP(ctx, pdit::launch_zero_i64(ctx->stream, S.counters, 3 * (int64_t)R));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->rec_choices = nullptr;
    ctx->rec_trace = nullptr;
    ctx->sweep_offset += (uint64_t)n_sweeps;
    ctx->last_updates = (int64_t)R * N * n_sweeps;
    ctx->last_sweep = use_reg    ? PDIT_SWEEP_REG
                      : use_fast ? PDIT_SWEEP_FAST
                      : use_large ? PDIT_SWEEP_LARGE
                                  : PDIT_SWEEP_PLAIN;
    ctx->last_class = use_fast ? fclass : use_reg ? 256 : 0;
    ctx->last_mode = mode;
    S.best_valid = true;
    remember(ctx, N, R, D, F, perm);
    return PDIT_OK;
}

// Parallel tempering with concurrent updates: one CUPIM launch per period
// (each replica at its rung's beta; the kernel rebuilds its snapshot from p,
// so nothing is saved between periods), then the exchange pass.
int run_pt_cupim(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                 int32_t *perm, const pdit_pt *pt, int64_t n_periods, uint64_t seed,
                 const InstanceStats &st) {
    const int cls = pdit::cupim_class(N, st);
    if (!cls)
        return fail(ctx, PDIT_EOVERFLOW,
                    "parallel tempering with concurrent updates needs N <= 128 and |D|, |F| <= "
                    "127 (the on-chip kernel)");
    bool fresh = false;
    int rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;
    pdit::CupimArgs c{};
    c.N = N;
    c.R = R;
    c.D = D;
    c.F = F;
    c.perm = perm;
    c.E = S.E;
    c.E_best = S.E_best;
    c.perm_best = S.perm_best;
    c.counters = S.counters;
    c.beta = pt->beta;
    c.slot = pt->slot;
    c.T = pt->period_sweeps;
    c.seed = seed;
    c.inst_id = 0;
    c.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, record_event(ctx, 1));
    // with no period, one launch of no iterations still yields E and zero counters
    const int64_t launches = n_periods > 0 ? n_periods : 1;
    for (int64_t per = 0; per < launches; ++per) {
        c.T = n_periods > 0 ? pt->period_sweeps : 0;
        c.sweep_offset = ctx->sweep_offset + (uint64_t)(per * pt->period_sweeps);
        c.init_best = (fresh && per == 0) ? 1 : 0;
        c.accumulate = per > 0 ? 1 : 0;
        PDIT_HIP(ctx, pdit::launch_cupim(ctx->stream, cls, c));
        if (n_periods > 0)
            PDIT_HIP(ctx, pdit::launch_pt_exchange(ctx->stream, R / pt->L, pt->L, S.E, pt->slot,
                                                   pt->since_top, pt->timeout));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->sweep_offset += (uint64_t)(n_periods * pt->period_sweeps);
    ctx->last_updates = (int64_t)R * N * n_periods * pt->period_sweeps;
    ctx->last_sweep = PDIT_SWEEP_FAST;
    ctx->last_class = cls;
    ctx->last_mode = 0;
    S.best_valid = true;
    remember(ctx, N, R, D, F, perm);
    return PDIT_OK;
}

int pdit_run_pt(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                int32_t *perm, const pdit_pt *pt, int64_t n_periods, uint64_t seed) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || !pt || !pt->beta || !pt->slot || !pt->since_top)
        return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 2 || N > PDIT_NMAX) return fail(ctx, PDIT_EINVAL, "N must be in [2, PDIT_NMAX]");
    if (pt->L < 1 || pt->L > PDIT_PT_MAXL)
        return fail(ctx, PDIT_EINVAL, "L must be in [1, PDIT_PT_MAXL]");
    if (R < 1 || R % pt->L) return fail(ctx, PDIT_EINVAL, "R must be a positive multiple of L");
    if (n_periods < 0 || pt->period_sweeps < 0)
        return fail(ctx, PDIT_EINVAL, "n_periods and period_sweeps must be >= 0");
    if (pt->schedule < PDIT_PT_AUTO || pt->schedule > PDIT_PT_FUSED)
        return fail(ctx, PDIT_EINVAL, "unknown parallel-tempering schedule");
    if (pt->dynamics != PDIT_PT_SEQUENTIAL && pt->dynamics != PDIT_PT_CUPIM)
        return fail(ctx, PDIT_EINVAL, "unknown parallel-tempering dynamics");
    if (pt->dynamics == PDIT_PT_CUPIM && pt->schedule == PDIT_PT_FUSED)
        return fail(ctx, PDIT_EINVAL, "concurrent-update tempering runs on the periodic schedule");
    if (ctx->rec_choices || ctx->rec_trace)
        return fail(ctx, PDIT_EINVAL, "recording is not available for parallel tempering");
    if (ctx->opts.sweep < PDIT_SWEEP_AUTO || ctx->opts.sweep > PDIT_SWEEP_LARGE ||
        ctx->opts.sweep == PDIT_SWEEP_CLIQUE)
        return fail(ctx, PDIT_EINVAL,
                    ctx->opts.sweep == PDIT_SWEEP_CLIQUE
                        ? "the clique kernel runs only in pdit_run_sweeps"
                        : "unknown sweep kernel");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));

    InstanceStats st;
    int rc = instance_prep(ctx, N, D, F, R, perm, pt->beta, pt->L, &st, pt);
    if (rc) return rc;
    if (pt->dynamics == PDIT_PT_CUPIM) return run_pt_cupim(ctx, N, D, F, R, perm, pt, n_periods, seed, st);
    const int64_t bound = pdit::h_bound(st);
    const bool h64 = bound > INT32_MAX;
    const int fclass = pdit::fast_class(N, st);
    bool use_fast = false;
    if (ctx->opts.sweep == PDIT_SWEEP_FAST) {
        if (!fclass)
            return fail(ctx, PDIT_EOVERFLOW, "the data do not fit the fast sweep kernel");
        use_fast = true;
    } else if (ctx->opts.sweep == PDIT_SWEEP_AUTO) {
        use_fast = fclass != 0;
    }
    // without a fast class the kernel that stores no H replaces the plain one
    const bool use_large = ctx->opts.sweep == PDIT_SWEEP_LARGE ||
                           (ctx->opts.sweep == PDIT_SWEEP_AUTO && !use_fast);
    const bool table = use_fast && fclass <= 128;
    // fused: the table kernel, cooperative launches, energies inside the
    // published word (|E| <= N max|H| < 2^35; the table classes imply it)
    const bool can_fuse = table && ctx->coop && ctx->wall_clock_khz > 0 &&
                          (int64_t)N * bound < ((int64_t)1 << (pdit::kPtEBits - 1));
    if (pt->schedule == PDIT_PT_FUSED && !can_fuse)
        return fail(ctx, PDIT_EINVAL,
                    "the fused schedule needs N <= 128, data that fit the fast kernel and a "
                    "device with cooperative launches");
    const bool fused = can_fuse && pt->schedule != PDIT_PT_PERIODIC && n_periods > 0;
    int mode = 0;
    rc = pick_recompute(ctx, st, bound, ctx->opts.recompute, &mode);
    if (rc) return rc;
    rc = ensure(ctx, ctx->h_buf, (size_t)R * N * N * (h64 ? 8 : 4));
    if (rc) return rc;
    if (fused) {
        rc = ensure(ctx, ctx->pt_buf, sizeof(uint64_t) * 2 * (size_t)R + sizeof(int32_t));
        if (rc) return rc;
    } else if (table) {
        rc = ensure(ctx, ctx->tstate, sizeof(int32_t) * (size_t)R * pdit::table_state_words(fclass));
        if (rc) return rc;
    }
    const pdit::LargePlan lplan = use_large ? pdit::large_plan(N, st) : pdit::LargePlan{};
    if (use_large) {
        rc = ensure(ctx, ctx->large_buf, lplan.bytes);
        if (rc) return rc;
    }
    bool fresh = false;
    rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;

    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, run_recompute(ctx, mode, N, D, F, R, perm, ctx->h_buf.ptr, h64, S.E));
    pdit::LargeCopies lcopy;
    if (use_large)
        PDIT_HIP(ctx, pdit::launch_large_copy(ctx->stream, N, D, F, lplan, ctx->large_buf.ptr,
                                              &lcopy));
    if (fresh) {
        PDIT_HIP(ctx, hipMemcpyAsync(S.E_best, S.E, sizeof(int64_t) * R, hipMemcpyDeviceToDevice,
                                     ctx->stream));
        PDIT_HIP(ctx, hipMemcpyAsync(S.perm_best, perm, sizeof(int32_t) * (size_t)R * N,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    }
    pdit::SweepArgs a{};
    a.N = N;
    a.R = R;
    a.D = D;
    a.F = F;
    a.perm = perm;
    a.H = ctx->h_buf.ptr;
    a.E = S.E;
    a.E_best = S.E_best;
    a.perm_best = S.perm_best;
    a.counters = S.counters;
    a.beta = pt->beta;
    a.slot = pt->slot;
    a.T = pt->period_sweeps;
    a.seed = seed;
    a.inst_id = 0;
    a.seq_threshold = ctx->opts.seq_threshold;
    a.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    a.tstate = table ? (int32_t *)ctx->tstate.ptr : nullptr;
    PDIT_HIP(ctx, record_event(ctx, 1));
    if (!fused && (pt->period_sweeps == 0 || n_periods == 0))
        PDIT_HIP(ctx, hipMemsetAsync(S.counters, 0, sizeof(int64_t) * 3 * R, ctx->stream));
    if (fused) {
        // every period in one launch per group of resident sets
        uint64_t *Epub = (uint64_t *)ctx->pt_buf.ptr;
        int32_t *err = (int32_t *)(Epub + 2 * (size_t)R);
        PDIT_HIP(ctx, hipMemsetAsync(Epub, 0, sizeof(uint64_t) * 2 * (size_t)R + sizeof(int32_t),
                                     ctx->stream));
        pdit::PtFusedArgs p{};
        p.L = pt->L;
        p.ladder = pt->beta;
        p.slot = pt->slot;
        p.since_top = pt->since_top;
        p.n_periods = n_periods;
        p.period_sweeps = pt->period_sweeps;
        p.timeout = pt->timeout;
        p.Epub = Epub;
        p.err = err;
        p.R = R;
        p.min_wait = (uint64_t)ctx->wall_clock_khz * 1000u * 20u;
        a.sweep_offset = ctx->sweep_offset;
        a.flags = 0;
        a.tstate = nullptr;
        PDIT_HIP(ctx, pdit::launch_sweep_table_pt(ctx->stream, fclass, a, p, ctx->num_cus));
        PDIT_HIP(ctx, hipMemcpyAsync(ctx->flag_host, err, sizeof(int32_t), hipMemcpyDeviceToHost,
                                     ctx->stream));
    }
    // each period: the sweeps of every replica at its rung's beta (resuming
    // from the state the previous period saved), then one exchange pass per set
    for (int64_t per = 0; per < n_periods && !fused; ++per) {
        if (pt->period_sweeps > 0) {
            a.sweep_offset = ctx->sweep_offset + (uint64_t)(per * pt->period_sweeps);
            a.flags = pdit::kSaveState | (per > 0 ? pdit::kLoadState | pdit::kAccumCounters : 0u);
            if (use_fast)
                PDIT_HIP(ctx, pdit::launch_sweep_fast(ctx->stream, fclass, a));
            else if (use_large)
                PDIT_HIP(ctx, pdit::launch_sweep_large(ctx->stream, a, h64, lplan, lcopy));
            else
                PDIT_HIP(ctx, pdit::launch_sweep_plain(ctx->stream, a, h64));
        }
        PDIT_HIP(ctx, pdit::launch_pt_exchange(ctx->stream, R / pt->L, pt->L, S.E, pt->slot,
                                               pt->since_top, pt->timeout));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    if (fused) {
        PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (*ctx->flag_host)
            return fail(ctx, PDIT_EDEVICE,
                        "a parallel-tempering set did not meet within the wait bound (members "
                        "not resident together); the outputs are undefined");
    }
    ctx->sweep_offset += (uint64_t)(n_periods * pt->period_sweeps);
    ctx->last_updates = (int64_t)R * N * n_periods * pt->period_sweeps;
    ctx->last_sweep = use_fast ? PDIT_SWEEP_FAST : use_large ? PDIT_SWEEP_LARGE : PDIT_SWEEP_PLAIN;
    ctx->last_class = use_fast ? fclass : 0;
    ctx->last_mode = mode;
    S.best_valid = true;
    remember(ctx, N, R, D, F, perm);
    return PDIT_OK;
}

}  // extern "C"

// GPU-CUPIM where the on-chip kernel does not fit (N > 128 or entries beyond
// 8 bits): the snapshot S = H + H^T in device memory, one kernel per step of
// an iteration (validated by the caller).
int run_cupim_large(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                    int32_t *perm, const float *beta, int64_t n_sweeps, uint64_t seed,
                    const InstanceStats &st) {
    const int64_t bound = pdit::h_bound(st);
    // snapshot energy changes |dE| <= 8 bound + 16 max|D| max|F| must pack
    // with the location index into the 64-bit proposal key
    const __int128 dmax = (__int128)8 * bound + (__int128)16 * st.max_abs_d * st.max_abs_f;
    if (dmax >= ((__int128)1 << 53))
        return fail(ctx, PDIT_EOVERFLOW,
                    "concurrent updates need 8 |H| + 16 max|D| max|F| < 2^53");
    const bool h64 = bound > INT32_MAX;
    int mode = 0;
    int rc = pick_recompute(ctx, st, bound, ctx->opts.recompute, &mode);
    if (rc) return rc;
    rc = ensure(ctx, ctx->h_buf, (size_t)R * N * N * (h64 ? 8 : 4));
    if (rc) return rc;
    const size_t n1 = (size_t)R * N, n2 = n1 * N;
    rc = ensure(ctx, ctx->cupim_buf, 8 * n2 + 16 * n1 + 8 * n1);
    if (rc) return rc;
    bool fresh = false;
    rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &St = ctx->st;
    char *b = (char *)ctx->cupim_buf.ptr;
    pdit::CupimLargeArgs c{};
    c.N = N;
    c.R = R;
    c.D = D;
    c.F = F;
    c.perm = perm;
    int64_t *Sbuf = (int64_t *)b;
    int64_t *hd = Sbuf + n2;
    c.S = Sbuf;
    c.hd = hd;
    c.dsel = hd + n1;
    c.sel = (int32_t *)(c.dsel + n1);
    c.tie = c.sel + n1;
    c.counters = St.counters;
    c.beta = beta;
    c.seed = seed;
    c.inst_id = 0;
    c.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    auto refresh = [&]() -> hipError_t {
        hipError_t e = run_recompute(ctx, mode, N, D, F, R, perm, ctx->h_buf.ptr, h64, St.E);
        if (e == hipSuccess) e = pdit::launch_cupim_large_sym(ctx->stream, N, R, ctx->h_buf.ptr, h64, Sbuf, hd);
        return e;
    };
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, refresh());
    if (fresh) {
        PDIT_HIP(ctx, hipMemcpyAsync(St.E_best, St.E, sizeof(int64_t) * R, hipMemcpyDeviceToDevice,
                                     ctx->stream));
        PDIT_HIP(ctx, hipMemcpyAsync(St.perm_best, perm, sizeof(int32_t) * (size_t)R * N,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    }
    PDIT_HIP(ctx, pdit::launch_zero_i64(ctx->stream, St.counters, 3 * (int64_t)R));
    PDIT_HIP(ctx, record_event(ctx, 1));
    for (int64_t t = 0; t < n_sweeps; ++t) {
        const uint32_t g = (uint32_t)(ctx->sweep_offset + (uint64_t)t);
        PDIT_HIP(ctx, pdit::launch_cupim_large_draw(ctx->stream, c, t, g));
        PDIT_HIP(ctx, pdit::launch_cupim_large_resolve(ctx->stream, c));
        PDIT_HIP(ctx, refresh());
        PDIT_HIP(ctx, pdit::launch_cupim_large_best(ctx->stream, N, R, perm, St.E, St.E_best,
                                                    St.perm_best));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->sweep_offset += (uint64_t)n_sweeps;
    ctx->last_updates = (int64_t)R * N * n_sweeps;
    ctx->last_sweep = PDIT_SWEEP_LARGE;
    ctx->last_class = 0;
    ctx->last_mode = mode;
    St.best_valid = true;
    remember(ctx, N, R, D, F, perm);
    return PDIT_OK;
}

extern "C" {

int pdit_run_cupim(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                   int32_t *perm, const float *beta, int64_t n_sweeps, uint64_t seed) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || (!beta && n_sweeps > 0))
        return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 2 || N > PDIT_NMAX) return fail(ctx, PDIT_EINVAL, "N must be in [2, PDIT_NMAX]");
    if (R < 1) return fail(ctx, PDIT_EINVAL, "R must be >= 1");
    if (n_sweeps < 0) return fail(ctx, PDIT_EINVAL, "n_sweeps must be >= 0");
    if (ctx->rec_choices || ctx->rec_trace)
        return fail(ctx, PDIT_EINVAL, "recording is not available for concurrent updates");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    InstanceStats st;
    int rc = instance_prep(ctx, N, D, F, R, perm, beta, n_sweeps, &st);
    if (rc) return rc;
    const int cls = pdit::cupim_class(N, st);
    if (!cls) return run_cupim_large(ctx, N, D, F, R, perm, beta, n_sweeps, seed, st);
    bool fresh = false;
    rc = shape_state(ctx, {N}, {R}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;
    pdit::CupimArgs c{};
    c.N = N;
    c.R = R;
    c.D = D;
    c.F = F;
    c.perm = perm;
    c.E = S.E;
    c.E_best = S.E_best;
    c.perm_best = S.perm_best;
    c.counters = S.counters;
    c.beta = beta;
    c.T = n_sweeps;
    c.seed = seed;
    c.sweep_offset = ctx->sweep_offset;
    c.inst_id = 0;
    c.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    c.init_best = fresh ? 1 : 0;
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, record_event(ctx, 1));
    PDIT_HIP(ctx, pdit::launch_cupim(ctx->stream, cls, c));
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->sweep_offset += (uint64_t)n_sweeps;
    ctx->last_updates = (int64_t)R * N * n_sweeps;
    ctx->last_sweep = PDIT_SWEEP_FAST;
    ctx->last_class = cls;
    ctx->last_mode = 0;
    S.best_valid = true;
    remember(ctx, N, R, D, F, perm);
    return PDIT_OK;
}

int pdit_beta_select(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, const float *grid, int32_t G, int64_t trial_sweeps,
                     uint64_t seed, int32_t L, int32_t level_pct, int64_t *E_sum, float *ladder,
                     int32_t *range) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || !grid || !E_sum || !ladder || !range)
        return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (level_pct < 0 || level_pct > 100)
        return fail(ctx, PDIT_EINVAL, "level_pct must be in [0, 100]");
    if (N < 2 || N > PDIT_NMAX) return fail(ctx, PDIT_EINVAL, "N must be in [2, PDIT_NMAX]");
    if (R < 1 || G < 1 || (int64_t)R * G > INT32_MAX)
        return fail(ctx, PDIT_EINVAL, "R and G must be >= 1 with R * G < 2^31");
    if (L < 2) return fail(ctx, PDIT_EINVAL, "the ladder needs L >= 2 rungs");
    if (trial_sweeps < 0) return fail(ctx, PDIT_EINVAL, "trial_sweeps must be >= 0");
    if (ctx->rec_choices || ctx->rec_trace)
        return fail(ctx, PDIT_EINVAL, "recording is not available for beta selection");
    if (ctx->opts.sweep < PDIT_SWEEP_AUTO || ctx->opts.sweep > PDIT_SWEEP_LARGE ||
        ctx->opts.sweep == PDIT_SWEEP_CLIQUE)
        return fail(ctx, PDIT_EINVAL,
                    ctx->opts.sweep == PDIT_SWEEP_CLIQUE
                        ? "the clique kernel runs only in pdit_run_sweeps"
                        : "unknown sweep kernel");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));

    InstanceStats st;
    int rc = instance_prep(ctx, N, D, F, R, perm, grid, G, &st, nullptr, true);
    if (rc) return rc;
    const int64_t bound = pdit::h_bound(st);
    // |E| <= N bound; the rule adds up to 5 sums of R energies exactly in int64
    if ((__int128)R * N * bound >= ((__int128)1 << 59))
        return fail(ctx, PDIT_EOVERFLOW, "R * N * (bound on |H|) must stay below 2^59");
    const bool h64 = bound > INT32_MAX;
    const int fclass = pdit::fast_class(N, st);
    bool use_fast = false;
    if (ctx->opts.sweep == PDIT_SWEEP_FAST) {
        if (!fclass) return fail(ctx, PDIT_EOVERFLOW, "the data do not fit the fast sweep kernel");
        use_fast = true;
    } else if (ctx->opts.sweep == PDIT_SWEEP_AUTO) {
        use_fast = fclass != 0;
    }
    // without a fast class the kernel that stores no H replaces the plain one
    const bool use_large = ctx->opts.sweep == PDIT_SWEEP_LARGE ||
                           (ctx->opts.sweep == PDIT_SWEEP_AUTO && !use_fast);
    int mode = 0;
    rc = pick_recompute(ctx, st, bound, ctx->opts.recompute, &mode);
    if (rc) return rc;
    const int RT = R * G;  // trial replicas: row g R + k is replica k at grid[g]
    rc = ensure(ctx, ctx->h_buf, (size_t)RT * N * N * (h64 ? 8 : 4));
    if (rc) return rc;
    rc = ensure(ctx, ctx->trial_buf, sizeof(int32_t) * (size_t)RT * (N + 1));
    if (rc) return rc;
    const pdit::LargePlan lplan = use_large ? pdit::large_plan(N, st) : pdit::LargePlan{};
    if (use_large) {
        rc = ensure(ctx, ctx->large_buf, lplan.bytes);
        if (rc) return rc;
    }
    int32_t *tperm = (int32_t *)ctx->trial_buf.ptr;
    int32_t *tslot = tperm + (size_t)RT * N;
    ctx->st.best_valid = false;  // the trials start their own best states
    bool fresh = false;
    rc = shape_state(ctx, {N}, {RT}, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;

    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, pdit::launch_trial_setup(ctx->stream, N, R, G, perm, tperm, tslot));
    PDIT_HIP(ctx, run_recompute(ctx, mode, N, D, F, RT, tperm, ctx->h_buf.ptr, h64, S.E));
    pdit::LargeCopies lcopy;
    if (use_large)
        PDIT_HIP(ctx, pdit::launch_large_copy(ctx->stream, N, D, F, lplan, ctx->large_buf.ptr,
                                              &lcopy));
    PDIT_HIP(ctx, hipMemcpyAsync(S.E_best, S.E, sizeof(int64_t) * RT, hipMemcpyDeviceToDevice,
                                 ctx->stream));
    PDIT_HIP(ctx, hipMemcpyAsync(S.perm_best, tperm, sizeof(int32_t) * (size_t)RT * N,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    pdit::SweepArgs a{};
    a.N = N;
    a.R = RT;
    a.D = D;
    a.F = F;
    a.perm = tperm;
    a.H = ctx->h_buf.ptr;
    a.E = S.E;
    a.E_best = S.E_best;
    a.perm_best = S.perm_best;
    a.counters = S.counters;
    a.beta = grid;
    a.slot = tslot;
    a.T = trial_sweeps;
    a.seed = seed;
    a.sweep_offset = 0;  // every trial starts at sweep 0
    a.inst_id = 0;
    a.seq_threshold = ctx->opts.seq_threshold;
    a.zero_diag = st.diag_nz_d == 0 && st.diag_nz_f == 0;
    PDIT_HIP(ctx, record_event(ctx, 1));
    if (trial_sweeps > 0) {
        if (use_fast)
            PDIT_HIP(ctx, pdit::launch_sweep_fast(ctx->stream, fclass, a));
        else if (use_large)
            PDIT_HIP(ctx, pdit::launch_sweep_large(ctx->stream, a, h64, lplan, lcopy));
        else
            PDIT_HIP(ctx, pdit::launch_sweep_plain(ctx->stream, a, h64));
    } else {
        PDIT_HIP(ctx, hipMemsetAsync(S.counters, 0, sizeof(int64_t) * 3 * RT, ctx->stream));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    PDIT_HIP(ctx, pdit::launch_group_sums(ctx->stream, R, G, S.E, E_sum));
    ctx->timed = true;
    // the rule on the G sums, on the host: integers compared exactly in 128
    // bits, the geometric ladder in double
    std::vector<int64_t> sums(G);
    std::vector<float> gv(G);
    PDIT_HIP(ctx, hipMemcpyAsync(sums.data(), E_sum, sizeof(int64_t) * G, hipMemcpyDeviceToHost,
                                 ctx->stream));
    PDIT_HIP(ctx, hipMemcpyAsync(gv.data(), grid, sizeof(float) * G, hipMemcpyDeviceToHost,
                                 ctx->stream));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    int64_t smax = sums[0], smin = sums[0];
    int gmin = 0;
    for (int g = 1; g < G; ++g) {
        if (sums[g] > smax) smax = sums[g];
        if (sums[g] < smin) {
            smin = sums[g];
            gmin = g;
        }
    }
    const __int128 level = (__int128)level_pct * smax + (__int128)(100 - level_pct) * smin;
    int32_t rng[2] = {0, gmin + 2 < G ? gmin + 2 : G - 1};
    while (rng[0] < G - 1 && (__int128)100 * sums[rng[0]] > level) ++rng[0];  // Smin meets it
    std::vector<float> lad(L);
    const double b0 = gv[rng[0]], b1 = gv[rng[1]];
    const double lr = log(b1 / b0);
    for (int i = 1; i + 1 < L; ++i) lad[i] = (float)(b0 * exp(lr * (double)i / (double)(L - 1)));
    lad[0] = gv[rng[0]];
    lad[L - 1] = gv[rng[1]];
    PDIT_HIP(ctx, hipMemcpyAsync(range, rng, sizeof(rng), hipMemcpyHostToDevice, ctx->stream));
    PDIT_HIP(ctx, hipMemcpyAsync(ladder, lad.data(), sizeof(float) * L, hipMemcpyHostToDevice,
                                 ctx->stream));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->last_updates = (int64_t)RT * N * trial_sweeps;
    ctx->last_sweep = use_fast ? PDIT_SWEEP_FAST : use_large ? PDIT_SWEEP_LARGE : PDIT_SWEEP_PLAIN;
    ctx->last_class = use_fast ? fclass : 0;
    ctx->last_mode = mode;
    S.best_valid = true;
    ctx->last_insts.clear();   // the trial replicas are the library's own
    return PDIT_OK;
}

int pdit_run_sweeps_batch(pdit_t *ctx, int32_t n_inst, const pdit_instance *inst,
                          int64_t n_sweeps, uint64_t seed) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!inst || n_inst < 1) return fail(ctx, PDIT_EINVAL, "empty or null instance list");
    if (n_sweeps < 0) return fail(ctx, PDIT_EINVAL, "n_sweeps must be >= 0");
    if (ctx->rec_choices || ctx->rec_trace)
        return fail(ctx, PDIT_EINVAL,
                    "pdit_set_recording applies to single-instance runs: batched runs record "
                    "through the instances' choices and E_trace pointers");
    if (ctx->opts.sweep < PDIT_SWEEP_AUTO || ctx->opts.sweep > PDIT_SWEEP_LARGE ||
        ctx->opts.sweep == PDIT_SWEEP_CLIQUE)
        return fail(ctx, PDIT_EINVAL,
                    ctx->opts.sweep == PDIT_SWEEP_CLIQUE
                        ? "the clique kernel runs only in pdit_run_sweeps"
                        : "unknown sweep kernel");
    for (int k = 0; k < n_inst; ++k) {
        const pdit_instance &in = inst[k];
        if (in.N < 2 || in.N > PDIT_NMAX || in.R < 1)
            return fail(ctx, PDIT_EINVAL, "an instance has N outside [2, PDIT_NMAX] or R < 1");
        if (!in.D || !in.F || !in.perm || (!in.beta && n_sweeps > 0))
            return fail(ctx, PDIT_EINVAL, "null pointer in an instance");
    }
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));

    // ---- instance prep for every instance, one host synchronisation ----
    int rc = ensure(ctx, ctx->scratch, sizeof(InstanceStats) * (size_t)n_inst);
    if (rc) return rc;
    InstanceStats *dev_st = (InstanceStats *)ctx->scratch.ptr;
    for (int k = 0; k < n_inst; ++k)
        PDIT_HIP(ctx, pdit::launch_instance_stats(ctx->stream, inst[k].N, inst[k].D, inst[k].F,
                                                  inst[k].R, inst[k].perm, inst[k].beta, n_sweeps,
                                                  dev_st + k));
    std::vector<InstanceStats> st(n_inst);
    PDIT_HIP(ctx, hipMemcpyAsync(st.data(), dev_st, sizeof(InstanceStats) * n_inst,
                                 hipMemcpyDeviceToHost, ctx->stream));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));

    struct Plan {
        int mode;
        int fclass;
        bool h64, fast, large, zd;
        int64_t hoff;  // byte offset of replica 0's H
        pdit::LargePlan lp;
        size_t coff;   // large kernel: byte offset of the instance's copies
    };
    std::vector<Plan> plan(n_inst);
    size_t hbytes = 0, cbytes = 0;
    for (int k = 0; k < n_inst; ++k) {
        const InstanceStats &q = st[k];
        if (q.asym_d || q.asym_f) return fail(ctx, PDIT_ENOTSYM, "D or F of an instance is not symmetric");
        if (q.int_min)
            return fail(ctx, PDIT_EOVERFLOW, "an instance has an entry equal to INT32_MIN");
        if (q.bad_perm_rows)
            return fail(ctx, PDIT_EBADPERM, "a row of an instance's perm is not a permutation");
        if (q.bad_beta)
            return fail(ctx, PDIT_EBETA, "an instance's inverse temperature is NaN, infinite or negative");
        const __int128 b1 = (__int128)q.max_abs_d * q.max_colsum_f;
        const __int128 b2 = (__int128)q.max_abs_f * q.max_rowsum_d;
        if ((b1 < b2 ? b1 : b2) > ((__int128)1 << 58))
            return fail(ctx, PDIT_EOVERFLOW, "an instance's exact bound on H exceeds the int64 range");
        const int64_t bound = pdit::h_bound(q);
        Plan &pl = plan[k];
        pl.h64 = bound > INT32_MAX;
        pl.fclass = pdit::fast_class(inst[k].N, q);
        if (ctx->opts.sweep == PDIT_SWEEP_FAST && !pl.fclass)
            return fail(ctx, PDIT_EOVERFLOW, "an instance does not fit the fast sweep kernel");
        pl.fast = (ctx->opts.sweep == PDIT_SWEEP_AUTO || ctx->opts.sweep == PDIT_SWEEP_FAST) &&
                  pl.fclass != 0;
        // without a fast class the kernel that stores no H replaces the plain one
        pl.large = !pl.fast && ctx->opts.sweep != PDIT_SWEEP_PLAIN;
        pl.zd = q.diag_nz_d == 0 && q.diag_nz_f == 0;
        rc = pick_recompute(ctx, q, bound, ctx->opts.recompute, &pl.mode);
        if (rc) return rc;
        const size_t elem = pl.h64 ? 8 : 4;
        hbytes = (hbytes + 7) & ~(size_t)7;
        pl.hoff = (int64_t)hbytes;
        hbytes += (size_t)inst[k].R * inst[k].N * inst[k].N * elem;
        if (pl.large) {
            pl.lp = pdit::large_plan(inst[k].N, q);
            cbytes = (cbytes + 255) & ~(size_t)255;
            pl.coff = cbytes;
            cbytes += pl.lp.bytes;
        }
    }
    rc = ensure(ctx, ctx->h_buf, hbytes);
    if (rc) return rc;
    if (cbytes) {
        rc = ensure(ctx, ctx->large_buf, cbytes);
        if (rc) return rc;
    }
    std::vector<int32_t> Ns(n_inst), Rs(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        Ns[k] = inst[k].N;
        Rs[k] = inst[k].R;
    }
    bool fresh = false;
    rc = shape_state(ctx, Ns, Rs, &fresh);
    if (rc) return rc;
    pdit::ReplicaState &S = ctx->st;

    // ---- descriptors ----
    std::vector<pdit::BatchInstance> desc(n_inst);
    int64_t rep_base = 0, perm_off = 0;
    bool rec = false;
    for (int k = 0; k < n_inst; ++k) {
        pdit::BatchInstance &d = desc[k];
        d.N = inst[k].N;
        d.R = inst[k].R;
        d.D = inst[k].D;
        d.F = inst[k].F;
        d.perm = inst[k].perm;
        d.beta = inst[k].beta;
        d.h_off = plan[k].hoff / (plan[k].h64 ? 8 : 4);
        d.rep_base = rep_base;
        d.perm_off = perm_off;
        d.zero_diag = plan[k].zd ? 1 : 0;
        d.inst_id = k;
        d.choices = inst[k].choices;
        d.E_trace = inst[k].E_trace;
        if (d.choices || d.E_trace) rec = true;
        if (plan[k].large) {
            d.cD = (const char *)ctx->large_buf.ptr + plan[k].coff;
            d.cF = (const char *)d.cD + plan[k].lp.bytes / 2;
        }
        rep_base += inst[k].R;
        perm_off += (int64_t)inst[k].R * inst[k].N;
    }

    // ---- H recompute and fresh best state ----
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    for (int k = 0; k < n_inst; ++k)
        PDIT_HIP(ctx, run_recompute(ctx, plan[k].mode, inst[k].N, inst[k].D, inst[k].F, inst[k].R,
                                    inst[k].perm, (char *)ctx->h_buf.ptr + plan[k].hoff,
                                    plan[k].h64, S.E + desc[k].rep_base));
    for (int k = 0; k < n_inst; ++k)
        if (plan[k].large) {
            pdit::LargeCopies lc;
            PDIT_HIP(ctx, pdit::launch_large_copy(ctx->stream, inst[k].N, inst[k].D, inst[k].F,
                                                  plan[k].lp, (char *)ctx->large_buf.ptr +
                                                  plan[k].coff, &lc));
        }
    if (fresh) {
        PDIT_HIP(ctx, hipMemcpyAsync(S.E_best, S.E, sizeof(int64_t) * S.R_total,
                                     hipMemcpyDeviceToDevice, ctx->stream));
        for (int k = 0; k < n_inst; ++k)
            PDIT_HIP(ctx, hipMemcpyAsync(S.perm_best + desc[k].perm_off, inst[k].perm,
                                         sizeof(int32_t) * (size_t)inst[k].R * inst[k].N,
                                         hipMemcpyDeviceToDevice, ctx->stream));
    }
    PDIT_HIP(ctx, record_event(ctx, 1));

    if (n_sweeps > 0) {
        // ---- groups of work items: (kernel, size class, diagonal mode), largest N first ----
        struct Group {
            bool fast, zd, h64;
            int nmax;
            std::vector<int2> items;
            int grid;
            bool large;
            pdit::LargePlan lp;  // large kernel: copy layout and product width of the group
        };
        std::vector<Group> groups;
        std::vector<int> order(n_inst);
        for (int k = 0; k < n_inst; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return inst[x].N > inst[y].N; });
        for (int k : order) {
            const Plan &pl = plan[k];
            const int nmax = pl.fast ? pl.fclass : 0;
            Group *g = nullptr;
            for (auto &gg : groups)
                if (gg.fast == pl.fast && gg.large == pl.large && gg.nmax == nmax &&
                    (pl.fast ? gg.zd == pl.zd : gg.h64 == pl.h64) &&
                    (!pl.large || (gg.lp.elem == pl.lp.elem && gg.lp.narrow == pl.lp.narrow)))
                    g = &gg;
            if (!g) {
                groups.push_back(Group{pl.fast, pl.fast && pl.zd, !pl.fast && pl.h64, nmax, {}, 0,
                                       pl.large, pl.lp});
                g = &groups.back();
            }
            for (int r = 0; r < inst[k].R; ++r) g->items.push_back(make_int2(k, r));
        }
        for (auto &g : groups) {
            int bpc = g.fast    ? pdit::fast_blocks_per_cu(g.nmax)
                      : g.large ? pdit::large_blocks_per_cu(g.lp)
                                : pdit::plain_blocks_per_cu(g.h64);
            if (ctx->opts.blocks_per_cu > 0 && ctx->opts.blocks_per_cu < bpc) bpc = ctx->opts.blocks_per_cu;
            const int64_t want = (int64_t)bpc * std::max(ctx->num_cus, 1);
            g.grid = (int)std::min<int64_t>(want, (int64_t)g.items.size());
        }

        // ---- device blob: descriptors, items, queues, parameters ----
        auto align = [](size_t x) { return (x + 15) & ~(size_t)15; };
        const size_t off_desc = 0;
        size_t off = align(sizeof(pdit::BatchInstance) * n_inst);
        std::vector<size_t> off_items(groups.size());
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            off_items[gi] = off;
            off = align(off + sizeof(int2) * groups[gi].items.size());
        }
        const size_t off_queue = off;
        off = align(off + sizeof(int) * groups.size());
        const size_t off_params = off;
        const size_t blob_bytes = align(off + sizeof(pdit::BatchParams));
        std::vector<char> blob(blob_bytes, 0);
        memcpy(blob.data() + off_desc, desc.data(), sizeof(pdit::BatchInstance) * n_inst);
        for (size_t gi = 0; gi < groups.size(); ++gi)
            memcpy(blob.data() + off_items[gi], groups[gi].items.data(),
                   sizeof(int2) * groups[gi].items.size());
        pdit::BatchParams params{seed, ctx->sweep_offset};

        // signature of the captured graph: the blob without the parameters,
        // the launch shapes and every buffer address the kernels receive
        const int seq_thr = ctx->opts.seq_threshold;  // < 0: each kernel's default
        std::vector<char> sig(blob.begin(), blob.begin() + off_params);
        auto push = [&](const void *p, size_t n) {
            sig.insert(sig.end(), (const char *)p, (const char *)p + n);
        };
        rc = ensure(ctx, ctx->batch_buf, blob_bytes);
        if (rc) return rc;
        void *ptrs[7] = {ctx->batch_buf.ptr, ctx->h_buf.ptr, S.E, S.E_best, S.perm_best, S.counters,
                         (void *)ctx->stream};
        push(ptrs, sizeof(ptrs));
        push(&n_sweeps, sizeof(n_sweeps));
        push(&seq_thr, sizeof(seq_thr));
        push(&rec, sizeof(rec));
        for (auto &g : groups) push(&g.grid, sizeof(g.grid));

        char *dbuf = (char *)ctx->batch_buf.ptr;
        if (sig != ctx->graph_sig || !ctx->graph_exec) {
            // descriptors and items change only with the signature
            PDIT_HIP(ctx, hipMemcpyAsync(dbuf, blob.data(), off_params, hipMemcpyHostToDevice,
                                         ctx->stream));
            PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->graph_exec) {
                PDIT_HIP(ctx, hipGraphExecDestroy(ctx->graph_exec));
                ctx->graph_exec = nullptr;
            }
            ctx->graph_sig.clear();
            // the groups run as independent nodes of the graph: each on a
            // stream of its own, forked from the capture stream after the
            // queue reset and joined back to it (their persistent kernels
            // share no queue and never wait for each other)
            const size_t ng = groups.size();
            const bool fork = ng > 1;
            while (fork && ctx->group_streams.size() < ng) {
                hipStream_t st = nullptr;
                PDIT_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
                ctx->group_streams.push_back(st);
            }
            while (fork && ctx->group_events.size() < ng + 1) {
                hipEvent_t ev = nullptr;
                PDIT_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                ctx->group_events.push_back(ev);
            }
            hipStream_t cs = ctx->capture_stream;
            PDIT_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t cap = pdit::launch_queue_reset(cs, (int *)(dbuf + off_queue), (int)ng);
            if (fork && cap == hipSuccess) cap = hipEventRecord(ctx->group_events[ng], cs);
            for (size_t gi = 0; gi < ng && cap == hipSuccess; ++gi) {
                const auto &g = groups[gi];
                hipStream_t gs = fork ? ctx->group_streams[gi] : cs;
                if (fork) cap = hipStreamWaitEvent(gs, ctx->group_events[ng], 0);
                if (cap != hipSuccess) break;
                pdit::BatchArgs b{};
                b.inst = (const pdit::BatchInstance *)(dbuf + off_desc);
                b.items = (const int2 *)(dbuf + off_items[gi]);
                b.n_items = (int)g.items.size();
                b.queue = (int *)(dbuf + off_queue) + gi;
                b.params = (const pdit::BatchParams *)(dbuf + off_params);
                b.H = ctx->h_buf.ptr;
                b.E = S.E;
                b.E_best = S.E_best;
                b.perm_best = S.perm_best;
                b.counters = S.counters;
                b.T = n_sweeps;
                b.seq_threshold = seq_thr >= 0 ? seq_thr : pdit::default_seq_threshold(g.nmax, g.nmax);
                b.rec = rec ? 1 : 0;
                cap = g.fast    ? pdit::launch_sweep_fast_persistent(gs, g.nmax, g.zd, b, g.grid)
                      : g.large ? pdit::launch_sweep_large_persistent(gs, g.lp, g.h64, b, g.grid)
                                : pdit::launch_sweep_plain_persistent(gs, g.h64, b, g.grid);
                if (fork && cap == hipSuccess) cap = hipEventRecord(ctx->group_events[gi], gs);
            }
            for (size_t gi = 0; fork && gi < ng && cap == hipSuccess; ++gi)
                cap = hipStreamWaitEvent(cs, ctx->group_events[gi], 0);
            hipGraph_t graph = nullptr;
            const hipError_t end = hipStreamEndCapture(cs, &graph);
            if (cap != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return fail_hip(ctx, cap, "persistent launch during capture");
            }
            PDIT_HIP(ctx, end);
            const hipError_t inst_rc = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            PDIT_HIP(ctx, inst_rc);
            ctx->graph_sig = sig;
        }
        PDIT_HIP(ctx, hipMemcpyAsync(dbuf + off_params, &params, sizeof(params),
                                     hipMemcpyHostToDevice, ctx->stream));
        PDIT_HIP(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    } else {
        PDIT_HIP(ctx, hipMemsetAsync(S.counters, 0, sizeof(int64_t) * 3 * S.R_total, ctx->stream));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->sweep_offset += (uint64_t)n_sweeps;
    ctx->last_updates = 0;
    for (int k = 0; k < n_inst; ++k) ctx->last_updates += (int64_t)inst[k].R * inst[k].N * n_sweeps;
    S.best_valid = true;
    ctx->last_insts.assign(inst, inst + n_inst);
    return PDIT_OK;
}

int pdit_autotune(pdit_t *ctx, int32_t n_inst, const pdit_instance *inst, int64_t n_trial_sweeps,
                  uint64_t seed, pdit_tuning *out) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!inst || n_inst < 1 || n_trial_sweeps < 1)
        return fail(ctx, PDIT_EINVAL, "bad instance list or trial length");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    // the cache file, keyed by architecture, CU count and the batch's shape
    const char *cache = getenv("PDIT_AUTOTUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        hipDeviceProp_t prop;
        PDIT_HIP(ctx, hipGetDeviceProperties(&prop, ctx->opts.device));
        key = std::string(prop.gcnArchName) + "/cu" + std::to_string(ctx->num_cus);
        for (int k = 0; k < n_inst; ++k) {
            if (!inst[k].perm || inst[k].N < 2 || inst[k].N > PDIT_NMAX || inst[k].R < 1)
                return fail(ctx, PDIT_EINVAL, "bad instance descriptor");
            InstanceStats st;
            const int prc = instance_prep(ctx, inst[k].N, inst[k].D, inst[k].F, inst[k].R,
                                          inst[k].perm, nullptr, 0, &st);
            if (prc) return prc;
            const int32_t mx = std::max(st.max_abs_d, st.max_abs_f);
            key += "/" + std::to_string(inst[k].N) + "x" + std::to_string(inst[k].R) + "w" +
                   (mx <= 127 ? "8" : mx <= 32767 ? "16" : "32");
        }
        for (char &c : key)
            if (c == ' ' || c == '\t' || c == '\n') c = '_';
        if (FILE *f = fopen(cache, "r")) {
            char line[8192];
            pdit_tuning hit{0, 0, 0.0, 0};
            while (fgets(line, sizeof line, f)) {
                char k2[4096];
                int bpc = 0, thr = 0;
                double ms = 0.0;
                if (sscanf(line, "%4095s %d %d %lf", k2, &bpc, &thr, &ms) == 4 && key == k2 &&
                    bpc > 0)
                    hit = pdit_tuning{bpc, thr, ms, 1};
            }
            fclose(f);
            if (hit.cached) {
                ctx->opts.blocks_per_cu = hit.blocks_per_cu;
                ctx->opts.seq_threshold = hit.seq_threshold;
                if (out) *out = hit;
                return PDIT_OK;
            }
        }
    }
    // private copies of the permutations: trials must not touch the caller's state
    std::vector<pdit_instance> trial(inst, inst + n_inst);
    std::vector<int32_t *> copies(n_inst, nullptr);
    int rc = PDIT_OK;
    pdit_t *tmp = nullptr;
    for (int k = 0; k < n_inst && rc == PDIT_OK; ++k) {
        if (!inst[k].perm || inst[k].N < 2 || inst[k].R < 1) rc = PDIT_EINVAL;
        else if (hipMalloc(&copies[k], sizeof(int32_t) * (size_t)inst[k].R * inst[k].N) != hipSuccess)
            rc = PDIT_ENOMEM;
        trial[k].perm = copies[k];
        trial[k].choices = nullptr;  // trials record nothing
        trial[k].E_trace = nullptr;
    }
    pdit_opts o = ctx->opts;
    if (rc == PDIT_OK) rc = pdit_create(&tmp, &o);
    // resident workgroups per CU to try: up to the most any kernel of the batch allows
    int max_bpc = pdit::plain_blocks_per_cu(false);
    for (int nmax : {16, 32, 64, 96, 128, 160, 256}) max_bpc = std::max(max_bpc, pdit::fast_blocks_per_cu(nmax));
    max_bpc = std::min(max_bpc, 4);
    pdit_tuning best{0, 0, 1e300, 0};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == PDIT_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = PDIT_EDEVICE;
    const int thresholds[3] = {3, 12, 40};
    for (int bpc = 1; bpc <= max_bpc && rc == PDIT_OK; ++bpc) {
        for (int ti = 0; ti < 3 && rc == PDIT_OK; ++ti) {
            for (int k = 0; k < n_inst; ++k)
                if (hipMemcpyAsync(copies[k], inst[k].perm, sizeof(int32_t) * (size_t)inst[k].R * inst[k].N,
                                   hipMemcpyDeviceToDevice, tmp->stream) != hipSuccess)
                    rc = PDIT_EDEVICE;
            tmp->opts.blocks_per_cu = bpc;
            tmp->opts.seq_threshold = thresholds[ti];
            tmp->sweep_offset = ctx->sweep_offset;
            pdit_reset(tmp);
            // first run captures the graph for this setting; the timed run replays it
            if (rc == PDIT_OK) rc = pdit_run_sweeps_batch(tmp, n_inst, trial.data(), n_trial_sweeps, seed);
            for (int k = 0; k < n_inst && rc == PDIT_OK; ++k)
                if (hipMemcpyAsync(copies[k], inst[k].perm, sizeof(int32_t) * (size_t)inst[k].R * inst[k].N,
                                   hipMemcpyDeviceToDevice, tmp->stream) != hipSuccess)
                    rc = PDIT_EDEVICE;
            tmp->sweep_offset = ctx->sweep_offset;
            if (rc == PDIT_OK && hipEventRecord(e0, tmp->stream) != hipSuccess) rc = PDIT_EDEVICE;
            if (rc == PDIT_OK) rc = pdit_run_sweeps_batch(tmp, n_inst, trial.data(), n_trial_sweeps, seed);
            if (rc == PDIT_OK && (hipEventRecord(e1, tmp->stream) != hipSuccess ||
                                  hipEventSynchronize(e1) != hipSuccess))
                rc = PDIT_EDEVICE;
            float ms = 0.f;
            if (rc == PDIT_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PDIT_EDEVICE;
            if (rc == PDIT_OK && ms < best.best_ms) best = pdit_tuning{bpc, thresholds[ti], (double)ms};
        }
    }
    if (rc != PDIT_OK && tmp && !tmp->last_error.empty()) ctx->last_error = tmp->last_error;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    pdit_destroy(tmp);
    for (auto *c : copies) hipFree(c);
    if (rc != PDIT_OK) {
        if (ctx->last_error.empty()) ctx->last_error = "autotune trial failed";
        return rc;
    }
    ctx->opts.blocks_per_cu = best.blocks_per_cu;
    ctx->opts.seq_threshold = best.seq_threshold;
    if (cache && *cache && key.size() < 4096) {
        if (FILE *f = fopen(cache, "a")) {
            fprintf(f, "%s %d %d %.6f\n", key.c_str(), best.blocks_per_cu, best.seq_threshold,
                    best.best_ms);
            fclose(f);
        }
    }
    best.cached = 0;
    if (out) *out = best;
    return PDIT_OK;
}

int pdit_energy(pdit_t *ctx, int64_t *E_out) {
    if (!ctx || !E_out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (!ctx->st.E || !ctx->st.best_valid) return fail(ctx, PDIT_ESTATE, "no run yet");
    PDIT_HIP(ctx, hipMemcpyAsync(E_out, ctx->st.E, sizeof(int64_t) * ctx->st.R_total,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    return PDIT_OK;
}

int pdit_best(pdit_t *ctx, int64_t *E_best, int32_t *perm_best) {
    if (!ctx || (!E_best && !perm_best)) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (!ctx->st.E || !ctx->st.best_valid) return fail(ctx, PDIT_ESTATE, "no run yet");
    if (E_best)
        PDIT_HIP(ctx, hipMemcpyAsync(E_best, ctx->st.E_best, sizeof(int64_t) * ctx->st.R_total,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    if (perm_best)
        PDIT_HIP(ctx, hipMemcpyAsync(perm_best, ctx->st.perm_best,
                                     sizeof(int32_t) * ctx->st.perm_total,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    return PDIT_OK;
}

int pdit_replica_counters(pdit_t *ctx, int64_t *out) {
    if (!ctx || !out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (!ctx->st.counters || !ctx->st.best_valid) return fail(ctx, PDIT_ESTATE, "no run yet");
    PDIT_HIP(ctx, hipMemcpyAsync(out, ctx->st.counters, sizeof(int64_t) * 3 * ctx->st.R_total,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    return PDIT_OK;
}

int pdit_counters(pdit_t *ctx, pdit_counters_t *out) {
    if (!ctx || !out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (!ctx->st.counters || !ctx->st.best_valid) return fail(ctx, PDIT_ESTATE, "no run yet");
    std::vector<int64_t> h(3 * ctx->st.R_total);
    PDIT_HIP(ctx, hipMemcpyAsync(h.data(), ctx->st.counters, sizeof(int64_t) * h.size(),
                                 hipMemcpyDeviceToHost, ctx->stream));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out->updates = out->accepted = out->ties = 0;
    for (int64_t k = 0; k < ctx->st.R_total; ++k) {
        out->updates += h[3 * k];
        out->accepted += h[3 * k + 1];
        out->ties += h[3 * k + 2];
    }
    return PDIT_OK;
}

int pdit_set_sweep_offset(pdit_t *ctx, uint64_t offset) {
    if (!ctx) return PDIT_EINVAL;
    ctx->sweep_offset = offset;
    return PDIT_OK;
}

int pdit_get_sweep_offset(pdit_t *ctx, uint64_t *offset) {
    if (!ctx || !offset) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    *offset = ctx->sweep_offset;
    return PDIT_OK;
}

int pdit_reset(pdit_t *ctx) {
    if (!ctx) return PDIT_EINVAL;
    ctx->st.best_valid = false;
    return PDIT_OK;
}

int pdit_sync(pdit_t *ctx) {
    if (!ctx) return PDIT_EINVAL;
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    PDIT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->err_dev) {
        int32_t e = 0;
        PDIT_HIP(ctx, hipMemcpy(&e, ctx->err_dev, sizeof(e), hipMemcpyDeviceToHost));
        if (e) {
            PDIT_HIP(ctx, hipMemset(ctx->err_dev, 0, sizeof(int32_t)));
            return fail(ctx, PDIT_EDEVICE, "a sweep kernel's internal wait gave up (its results are undefined)");
        }
    }
    return PDIT_OK;
}

const char *pdit_last_error(const pdit_t *ctx) {
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

int pdit_set_recording(pdit_t *ctx, int32_t *choices, int64_t *E_trace) {
    if (!ctx) return PDIT_EINVAL;
    ctx->rec_choices = choices;
    ctx->rec_trace = E_trace;
    return PDIT_OK;
}

int pdit_h_recompute(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, int mode, int64_t *H_out, int64_t *E_out) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || !E_out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 2 || N > PDIT_NMAX || R < 1) return fail(ctx, PDIT_EINVAL, "bad N or R");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    InstanceStats st;
    int rc = instance_prep(ctx, N, D, F, R, perm, nullptr, 0, &st);
    if (rc) return rc;
    const int64_t bound = pdit::h_bound(st);
    const bool h64 = bound > INT32_MAX;
    int m = 0;
    rc = pick_recompute(ctx, st, bound, mode, &m);
    if (rc) return rc;
    rc = ensure(ctx, ctx->h_buf, (size_t)R * N * N * (h64 ? 8 : 4));
    if (rc) return rc;
    // pdit_last_timing: the recompute (H and its trace), then the copy to H_out
    ctx->timed = false;
    PDIT_HIP(ctx, record_event(ctx, 0));
    PDIT_HIP(ctx, run_recompute(ctx, m, N, D, F, R, perm, ctx->h_buf.ptr, h64, E_out));
    PDIT_HIP(ctx, record_event(ctx, 1));
    if (H_out) {
        const int64_t count = (int64_t)R * N * N;
        if (h64)
            PDIT_HIP(ctx, hipMemcpyAsync(H_out, ctx->h_buf.ptr, sizeof(int64_t) * count,
                                         hipMemcpyDeviceToDevice, ctx->stream));
        else
            PDIT_HIP(ctx, pdit::launch_widen_h(ctx->stream, count, (const int32_t *)ctx->h_buf.ptr,
                                               H_out));
    }
    PDIT_HIP(ctx, record_event(ctx, 2));
    ctx->timed = true;
    ctx->last_mode = m;
    return PDIT_OK;
}

int pdit_debug_delta(pdit_t *ctx, int32_t N, const int32_t *D, const int32_t *F, int32_t R,
                     const int32_t *perm, int32_t r, int64_t *delta_out) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!D || !F || !perm || !delta_out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 2 || N > PDIT_NMAX || R < 1 || r < 0 || r >= N)
        return fail(ctx, PDIT_EINVAL, "bad N, R or r");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    InstanceStats st;
    int rc = instance_prep(ctx, N, D, F, R, perm, nullptr, 0, &st);
    if (rc) return rc;
    rc = ensure(ctx, ctx->h_buf, (size_t)R * N * N * 8 + sizeof(int64_t) * R);
    if (rc) return rc;
    int64_t *H = (int64_t *)ctx->h_buf.ptr;
    int64_t *E = H + (size_t)R * N * N;
    PDIT_HIP(ctx, pdit::launch_h_recompute_plain(ctx->stream, N, D, F, R, perm, H, true, E));
    PDIT_HIP(ctx, pdit::launch_debug_delta(ctx->stream, N, D, F, R, perm, H, r, delta_out));
    return PDIT_OK;
}

// replica `replica` of instance `inst` of the last run: its N, D, F and row
// of perm, validated
static int last_replica(pdit_t *ctx, int32_t inst, int32_t replica, pdit_instance *x,
                        const int32_t **prow) {
    if (ctx->last_insts.empty()) return fail(ctx, PDIT_ESTATE, "no run yet");
    if (inst < 0 || inst >= (int32_t)ctx->last_insts.size())
        return fail(ctx, PDIT_EINVAL, "inst out of range");
    *x = ctx->last_insts[inst];
    if (replica < 0 || replica >= x->R) return fail(ctx, PDIT_EINVAL, "replica out of range");
    if (!x->D || !x->F || !x->perm) return fail(ctx, PDIT_ESTATE, "the last run kept no data");
    *prow = x->perm + (int64_t)replica * x->N;
    return PDIT_OK;
}

int pdit_debug_H(pdit_t *ctx, int32_t inst, int32_t replica, int64_t *H_out) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!H_out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    pdit_instance x;
    const int32_t *prow = nullptr;
    int rc = last_replica(ctx, inst, replica, &x, &prow);
    if (rc) return rc;
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    rc = ensure(ctx, ctx->check_buf, 256);
    if (rc) return rc;
    PDIT_HIP(ctx, pdit::launch_h_recompute_plain(ctx->stream, x.N, x.D, x.F, 1, prow, H_out, true,
                                                 (int64_t *)ctx->check_buf.ptr));
    return PDIT_OK;
}

int pdit_debug_delta_replica(pdit_t *ctx, int32_t inst, int32_t replica, int32_t r,
                             int64_t *delta_out) {
    if (!ctx) return PDIT_EINVAL;
    ctx->last_error.clear();
    if (!delta_out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    pdit_instance x;
    const int32_t *prow = nullptr;
    int rc = last_replica(ctx, inst, replica, &x, &prow);
    if (rc) return rc;
    if (r < 0 || r >= x.N) return fail(ctx, PDIT_EINVAL, "r out of range");
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    rc = ensure(ctx, ctx->check_buf, 256 + sizeof(int64_t) * (size_t)x.N * x.N);
    if (rc) return rc;
    int64_t *H = (int64_t *)((char *)ctx->check_buf.ptr + 256);
    PDIT_HIP(ctx, pdit::launch_h_recompute_plain(ctx->stream, x.N, x.D, x.F, 1, prow, H, true,
                                                 (int64_t *)ctx->check_buf.ptr));
    PDIT_HIP(ctx, pdit::launch_debug_delta(ctx->stream, x.N, x.D, x.F, 1, prow, H, r, delta_out));
    return PDIT_OK;
}

int pdit_debug_choice(pdit_t *ctx, int32_t N, int32_t M, const int64_t *delta, const float *beta,
                      const uint32_t *u24, int32_t *choice, int32_t *tie) {
    if (!ctx) return PDIT_EINVAL;
    if (!delta || !beta || !u24 || !choice) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (N < 1 || N > PDIT_NMAX || M < 0) return fail(ctx, PDIT_EINVAL, "bad N or M");
    if (M == 0) return PDIT_OK;
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    PDIT_HIP(ctx, pdit::launch_debug_choice(ctx->stream, N, M, delta, beta, u24, choice, tie));
    return PDIT_OK;
}

int pdit_last_timing(pdit_t *ctx, double *recompute_ms, double *sweep_ms) {
    if (!ctx) return PDIT_EINVAL;
    if (!ctx->timed) return fail(ctx, PDIT_ESTATE, "no timed run yet");
    PDIT_HIP(ctx, hipEventSynchronize(ctx->ev[2]));
    float a = 0.f, b = 0.f;
    PDIT_HIP(ctx, hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
    PDIT_HIP(ctx, hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
    if (recompute_ms) *recompute_ms = a;
    if (sweep_ms) *sweep_ms = b;
    return PDIT_OK;
}

int pdit_last_plan(pdit_t *ctx, int *sweep, int *size_class, int *recompute) {
    if (!ctx) return PDIT_EINVAL;
    if (!ctx->last_sweep) return fail(ctx, PDIT_ESTATE, "no single-instance run yet");
    if (sweep) *sweep = ctx->last_sweep;
    if (size_class) *size_class = ctx->last_class;
    if (recompute) *recompute = ctx->last_mode;
    return PDIT_OK;
}

int pdit_debug_uniform24(pdit_t *ctx, int32_t M, const uint32_t *ctr, uint64_t seed,
                         uint32_t *out) {
    if (!ctx) return PDIT_EINVAL;
    if (!ctr || !out) return fail(ctx, PDIT_EINVAL, "null pointer argument");
    if (M < 0) return fail(ctx, PDIT_EINVAL, "bad M");
    if (M == 0) return PDIT_OK;
    PDIT_HIP(ctx, hipSetDevice(ctx->opts.device));
    PDIT_HIP(ctx, pdit::launch_debug_uniform24(ctx->stream, M, ctr, seed, out));
    return PDIT_OK;
}

// ---------------------------------------------------------------------------
// The no-allocation variant of pdit_run_sweeps.  Its device work space (the
// instance summary, the clique membership, the large kernel's copies and the
// initial H) lives in `scratch`, a file-scope device array that each GPU the
// library runs on holds until the process ends; host code reaches it only
// through the per-device address hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kNoAllocScratch = (size_t)PDIT_NOALLOC_SCRATCH_BYTES;
constexpr size_t kNoAllocStats = 4096;             // instance summary
constexpr size_t kNoAllocClique = 4096;            // clique membership, N <= 512 words
constexpr size_t kNoAllocCopies = (size_t)4 << 20;  // large kernel copies, any N <= 512
constexpr size_t kNoAllocConv = (size_t)1 << 20;    // MFMA operand copies of D and F, N <= 512
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::atomic<void *> g_scratch_addr[kNoAllocDevices];
InstanceStats g_noalloc_stats[kNoAllocDevices];  // host copies of the summary

// Address of `scratch` on the current device (looked up once per device).
hipError_t noalloc_scratch(int device, void **out) {
    void *p = g_scratch_addr[device].load(std::memory_order_acquire);
    if (!p) {
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device].store(p, std::memory_order_release);
    }
    *out = p;
    return hipSuccess;
}

void copy_error(const char *msg, char *err, int32_t err_len) {
    if (!err || err_len < 1) return;
    snprintf(err, (size_t)err_len, "%s", msg);
}

}  // namespace

extern "C" {

int pdit_run_sweeps_noalloc(const pdit_opts *opts, int32_t N, const int32_t *D, const int32_t *F,
                            int32_t R, int32_t *perm, const float *beta, int64_t n_sweeps,
                            uint64_t seed, uint64_t sweep_offset, int init_best, int64_t *E,
                            int64_t *E_best, int32_t *perm_best, int64_t *counters, char *err,
                            int32_t err_len) {
    copy_error("", err, err_len);
    pdit_opts o;
    if (opts)
        o = *opts;
    else
        pdit_default_opts(&o);
    if (!E || !E_best || !perm_best || !counters) {
        copy_error("null output pointer", err, err_len);
        return PDIT_EINVAL;
    }
    if (o.device < 0 || o.device >= kNoAllocDevices) {
        copy_error("device ordinal outside the supported range", err, err_len);
        return PDIT_EINVAL;
    }
    if (hipSetDevice(o.device) != hipSuccess) {
        (void)hipGetLastError();
        copy_error("hipSetDevice failed", err, err_len);
        return PDIT_EDEVICE;
    }
    void *base = nullptr;
    const hipError_t se = noalloc_scratch(o.device, &base);
    if (se != hipSuccess) {
        (void)hipGetLastError();
        copy_error("hipGetSymbolAddress of the scratch array failed", err, err_len);
        return PDIT_EDEVICE;
    }
    pdit_ctx c;
    c.opts = o;
    c.stream = (hipStream_t)o.stream;
    c.noalloc = true;
    c.sweep_offset = sweep_offset;
    c.stats_host = &g_noalloc_stats[o.device];
    char *b = (char *)base;
    c.scratch = {b, kNoAllocStats};
    c.clique_buf = {b + kNoAllocStats, kNoAllocClique};
    c.large_buf = {b + kNoAllocStats + kNoAllocClique, kNoAllocCopies};
    c.conv_buf = {b + kNoAllocStats + kNoAllocClique + kNoAllocCopies, kNoAllocConv};
    const size_t used = kNoAllocStats + kNoAllocClique + kNoAllocCopies + kNoAllocConv;
    c.h_buf = {b + used, kNoAllocScratch - used};
    pdit::ReplicaState &S = c.st;
    S.n_inst = 1;
    S.Ns = {N};
    S.Rs = {R};
    S.R_total = R;
    S.perm_total = (int64_t)R * N;
    S.E = E;
    S.E_best = E_best;
    S.perm_best = perm_best;
    S.counters = counters;
    S.best_valid = init_best == 0;
    const int rc = pdit_run_sweeps(&c, N, D, F, R, perm, beta, n_sweeps, seed);
    copy_error(c.last_error.c_str(), err, err_len);
    // the context borrowed every buffer: nothing to free
    S.E = S.E_best = S.counters = nullptr;
    S.perm_best = nullptr;
    return rc;
}

}  // extern "C"
