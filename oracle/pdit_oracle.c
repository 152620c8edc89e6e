/*
 * pdit_oracle.c -- plain CPU reference for the p-dit probabilistic Ising
 * machine on the quadratic assignment problem (Duffee, Burling-Smith et al.,
 * "P-dit Probabilistic Ising Machine for Solving the Quadratic Assignment
 * Problem").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * library itself never links, loads or calls it, and it shares no code,
 * header, table or constant with the GPU sources.
 *
 * What it follows:
 *   - Eq. 1 (Introduction): E(p) = sum_i sum_j D_ij F_{p(i) p(j)}.
 *   - Eq. 2 (Results, "Implementation"): influence of the other p-dits on
 *     location i towards facility a,
 *       I_i^a = - sum_j ( D_ij F_{a,p(j)} + D_ji F_{p(j),a} ),
 *     the sum running over every location j (reading of the garbled bounds).
 *   - Eq. 3: energy change of swapping the facilities a = p(i), b = p(j),
 *       dE = -[ I_i^b - I_i^a + I_j^a - I_j^b
 *               - (D_ii + D_jj - D_ij - D_ji)(F_aa + F_bb - F_ab - F_ba) ].
 *     Eq. 4 (the same without the bracketed correction) is kept only so a
 *     test can show it differs from the true change by 4 D_ij F_ab on
 *     symmetric zero-diagonal data.
 *   - Eq. 5: the update of p-dit i picks candidate k among all N locations
 *     (k = i meaning "stay") with probability exp(-beta dE_k) / sum.
 *   - "every p-dit initiates an update once" per iteration: a sweep visits
 *     locations 0..N-1 in ascending order; only swaps are proposed, so the
 *     state stays a permutation.
 *   - Methods, "CPU-PIM Algorithm": I is kept up to date incrementally after
 *     each accepted swap rather than recomputed.
 *
 * Readings where the paper is silent (the random source and the sampling
 * arithmetic are not specified):
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (lo32(seed), hi32(seed)), counter = (r, g, replica, instance)
 *     for the update of location r in global sweep g; word 0 shifted right
 *     by 8 gives a 24-bit uniform u24, u = u24 * 2^-24 (exact in double);
 *   - Eq. 5 is evaluated in double precision: with m = min_k dE_k (a no-op
 *     for the probabilities that keeps exp from overflowing),
 *     w_k = exp(-beta (dE_k - m)) with the C library's exp, the running sum
 *     C_k = w_0 + ... + w_k taken in ascending k, Z = C_{N-1},
 *     tau = u Z, and the chosen candidate is the first k with C_k > tau;
 *   - a "tie" is a draw whose tau lies within 2^-20 Z (about 1e-6 of the
 *     total) of a boundary C_k that separates two candidates of nonzero
 *     weight (0 < C_k < Z): a different but equally valid evaluation of the
 *     weights (single precision, another exp) may move such a draw to the
 *     neighbouring candidate, so ties are counted and logged.
 *
 * Integer arithmetic is int64 throughout; the only floating point is the
 * double-precision evaluation of Eq. 5 above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PO_OK 0
#define PO_EINVAL (-1)
#define PO_EMISMATCH (-2)
#define PO_EBADPERM (-3)
#define PO_ENOMEM (-4)

#define IDX(i, j) ((int64_t)(i) * N + (j))

/* ------------------------------------------------------------------ */
/* Eq. 1                                                               */
/* ------------------------------------------------------------------ */
int64_t po_energy(int N, const int32_t *D, const int32_t *F, const int32_t *p)
{
    int64_t E = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            E += (int64_t)D[IDX(i, j)] * (int64_t)F[IDX(p[i], p[j])];
    return E;
}

/* ------------------------------------------------------------------ */
/* Eq. 2: I[i*N + a] = influence on location i towards facility a      */
/* ------------------------------------------------------------------ */
void po_influence(int N, const int32_t *D, const int32_t *F, const int32_t *p, int64_t *I)
{
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < N; ++a) {
            int64_t s = 0;
            for (int j = 0; j < N; ++j)
                s += (int64_t)D[IDX(i, j)] * F[IDX(a, p[j])] + (int64_t)D[IDX(j, i)] * F[IDX(p[j], a)];
            I[IDX(i, a)] = -s;
        }
}

/* ------------------------------------------------------------------ */
/* Eq. 3 (exact) and Eq. 4 (as printed)                                */
/* ------------------------------------------------------------------ */
int64_t po_delta_eq3(int N, const int32_t *D, const int32_t *F, const int32_t *p,
                     const int64_t *I, int i, int j)
{
    const int a = p[i], b = p[j];
    const int64_t dterm = (int64_t)D[IDX(i, i)] + D[IDX(j, j)] - D[IDX(i, j)] - D[IDX(j, i)];
    const int64_t fterm = (int64_t)F[IDX(a, a)] + F[IDX(b, b)] - F[IDX(a, b)] - F[IDX(b, a)];
    return -(I[IDX(i, b)] - I[IDX(i, a)] + I[IDX(j, a)] - I[IDX(j, b)] - dterm * fterm);
}

int64_t po_delta_eq4(int N, const int32_t *D, const int32_t *F, const int32_t *p,
                     const int64_t *I, int i, int j)
{
    (void)D; (void)F;
    const int a = p[i], b = p[j];
    return -(I[IDX(i, b)] - I[IDX(i, a)] + I[IDX(j, a)] - I[IDX(j, b)]);
}

/* Energy changes of every candidate for the update of p-dit r (Eq. 3 with
 * I computed afresh from Eq. 2). */
int po_delta_row(int N, const int32_t *D, const int32_t *F, const int32_t *p, int r, int64_t *out)
{
    if (N < 1 || r < 0 || r >= N) return PO_EINVAL;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * N);
    if (!I) return PO_ENOMEM;
    po_influence(N, D, F, p, I);
    for (int s = 0; s < N; ++s) out[s] = po_delta_eq3(N, D, F, p, I, r, s);
    free(I);
    return PO_OK;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 S-box, */
/* the key bumped by the Weyl constants between rounds.                */
/* ------------------------------------------------------------------ */
void po_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t prod0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t prod1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        const uint32_t y0 = hi1 ^ x1 ^ k0;
        const uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t po_uniform24(uint64_t seed, uint32_t r, uint32_t g, uint32_t rep, uint32_t inst)
{
    const uint32_t ctr[4] = {r, g, rep, inst};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    po_philox4x32_10(ctr, key, out);
    return out[0] >> 8;
}

/* ------------------------------------------------------------------ */
/* Eq. 5: Gibbs choice among the N candidates, in double precision      */
/* ------------------------------------------------------------------ */
#define PO_TIE_BAND 9.5367431640625e-07 /* 2^-20, relative to Z */

/*
 * Chosen candidate of one update with energy changes dE[0..N-1] at inverse
 * temperature beta and uniform u24 (returns PO_ENOMEM on allocation
 * failure).  *tie (optional) is set when tau = u Z lies within 2^-20 Z of a
 * boundary between two candidates of nonzero weight; *margin (optional)
 * receives the distance of tau to the nearest such boundary divided by Z
 * (HUGE_VAL when there is none).
 */
int po_gibbs_choice(int N, const int64_t *dE, float beta, uint32_t u24, int *tie, double *margin)
{
    if (N < 1 || !dE) return PO_EINVAL;
    double *C = (double *)malloc(sizeof(double) * (size_t)N);
    if (!C) return PO_ENOMEM;
    int64_t m = dE[0];
    for (int s = 1; s < N; ++s)
        if (dE[s] < m) m = dE[s];
    const double b = (double)beta;
    double acc = 0.0;
    for (int s = 0; s < N; ++s) {
        const double x = b * (double)(dE[s] - m);
        /* exp(-x) is exactly 0 in double beyond x = 745.2; skip the call */
        acc += x > 746.0 ? 0.0 : exp(-x);
        C[s] = acc;
    }
    const double Z = acc;
    const double tau = ((double)u24 / 16777216.0) * Z;
    int sel = N - 1;
    for (int s = 0; s < N; ++s)
        if (C[s] > tau) {
            sel = s;
            break;
        }
    double near = HUGE_VAL;
    if (sel > 0 && C[sel - 1] > 0.0) near = tau - C[sel - 1];
    if (C[sel] < Z && C[sel] - tau < near) near = C[sel] - tau;
    if (tie) *tie = near < PO_TIE_BAND * Z;
    if (margin) *margin = near == HUGE_VAL ? HUGE_VAL : near / Z;
    free(C);
    return sel;
}

/* po_gibbs_choice on M rows: row i has energy changes dE[i*N .. i*N+N-1],
 * inverse temperature beta[i] and uniform u24[i]; sel, tie (optional) and
 * margin (optional) receive one value per row. */
int po_gibbs_rows(int64_t M, int N, const int64_t *dE, const float *beta, const uint32_t *u24,
                  int32_t *sel, int32_t *tie, double *margin)
{
    if (M < 0 || N < 1 || !dE || !beta || !u24 || !sel) return PO_EINVAL;
    for (int64_t i = 0; i < M; ++i) {
        int t = 0;
        double mg = 0.0;
        const int k = po_gibbs_choice(N, dE + i * N, beta[i], u24[i], &t, &mg);
        if (k < 0) return k;
        sel[i] = k;
        if (tie) tie[i] = t;
        if (margin) margin[i] = mg;
    }
    return PO_OK;
}

/* Draw M updates of p-dit r from the fixed energy-change row dE, with the
 * counters (r, g0 + m, rep, inst) for m = 0..M-1; counts[k] += 1 for each
 * draw of candidate k. */
int po_sample_choices(int N, const int64_t *dE, float beta, uint64_t seed, uint32_t r,
                      uint32_t g0, uint32_t rep, uint32_t inst, int64_t M, int64_t *counts)
{
    for (int64_t m = 0; m < M; ++m) {
        const uint32_t u24 = po_uniform24(seed, r, g0 + (uint32_t)m, rep, inst);
        const int k = po_gibbs_choice(N, dE, beta, u24, NULL, NULL);
        if (k < 0) return k;
        counts[k] += 1;
    }
    return PO_OK;
}

/* ------------------------------------------------------------------ */
/* The sweep engine                                                    */
/* ------------------------------------------------------------------ */
static int is_permutation(int N, const int32_t *p, unsigned char *seen)
{
    memset(seen, 0, (size_t)N);
    for (int i = 0; i < N; ++i) {
        if (p[i] < 0 || p[i] >= N || seen[p[i]]) return 0;
        seen[p[i]] = 1;
    }
    return 1;
}

/*
 * Run T sweeps on each of R replicas of one instance.
 *
 *   perm       [R*N] in/out, each row a permutation (facility at location i)
 *   rep_ids    [R] replica index of each row inside its instance (Philox)
 *   inst_id    instance index (Philox)
 *   beta       [T] inverse temperature of each sweep
 *   sweep_off  global index of the first sweep (Philox)
 *   E          [R] out: energy of the final state
 *   E_best     [R] in/out, perm_best [R*N] in/out: lowest energy seen and
 *              the first state that reached it; when init_best != 0 they
 *              start from the initial state
 *   counters   [R*3] out: updates, accepted swaps, ties
 *   tie_log    optional [cap*3]: (row, sweep, location) of each tie
 *   choices    optional [R*T*N]: the chosen candidate of every update
 *   E_trace    optional [R*T]: the energy after every sweep
 *   paranoid   after every sweep, check I against Eq. 2 and E against Eq. 1
 *   forced     optional [R*T*N]: draws made by another evaluation of the
 *              same dynamics (for parity checks).  Where forced differs from
 *              this oracle's own choice, the draw must be a tie: the oracle
 *              then takes the forced candidate (so it follows the other
 *              trajectory from there on) and counts it in excused[row];
 *              otherwise the run stops with PO_EMISMATCH and fail_at =
 *              (row, t, r, own choice, forced choice).
 *   excused    optional [R] out (with forced): adopted draws per row
 *   fail_at    optional [5] out (with forced): first disagreement off a tie
 */
int po_run(int N, const int32_t *D, const int32_t *F, int R, const int32_t *rep_ids,
           int32_t inst_id, int32_t *perm, const float *beta, int64_t T, uint64_t seed,
           uint64_t sweep_off, int64_t *E, int64_t *E_best, int32_t *perm_best, int init_best,
           int64_t *counters, int32_t *tie_log, int64_t tie_cap, int64_t *tie_n,
           int32_t *choices, int64_t *E_trace, int paranoid, const int32_t *forced,
           int64_t *excused, int64_t *fail_at)
{
    if (N < 2 || R < 1 || T < 0 || !D || !F || !perm || !beta || !E || !E_best || !perm_best ||
        !counters)
        return PO_EINVAL;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * N);
    int64_t *I2 = paranoid ? (int64_t *)malloc(sizeof(int64_t) * (size_t)N * N) : NULL;
    int64_t *dE = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    unsigned char *seen = (unsigned char *)malloc((size_t)N);
    int rc = PO_OK;
    if (!I || !dE || !seen || (paranoid && !I2)) {
        rc = PO_ENOMEM;
        goto done;
    }
    if (tie_n) *tie_n = 0;
    if (forced && excused) memset(excused, 0, sizeof(int64_t) * (size_t)R);

    for (int row = 0; row < R; ++row) {
        int32_t *p = perm + (int64_t)row * N;
        int32_t *pb = perm_best + (int64_t)row * N;
        const uint32_t rep = rep_ids ? (uint32_t)rep_ids[row] : (uint32_t)row;
        if (!is_permutation(N, p, seen)) {
            rc = PO_EBADPERM;
            goto done;
        }
        po_influence(N, D, F, p, I);
        int64_t e = po_energy(N, D, F, p);
        if (init_best) {
            E_best[row] = e;
            memcpy(pb, p, sizeof(int32_t) * (size_t)N);
        }
        int64_t n_upd = 0, n_acc = 0, n_tie = 0;
        for (int64_t t = 0; t < T; ++t) {
            const uint32_t g = (uint32_t)(sweep_off + (uint64_t)t);
            const float b = beta[t];
            for (int r = 0; r < N; ++r) {
                for (int s = 0; s < N; ++s) dE[s] = po_delta_eq3(N, D, F, p, I, r, s);
                const uint32_t u24 = po_uniform24(seed, (uint32_t)r, g, rep, (uint32_t)inst_id);
                int tie = 0;
                int k = po_gibbs_choice(N, dE, b, u24, &tie, NULL);
                if (k < 0) {
                    rc = k;
                    goto done;
                }
                if (forced) {
                    const int32_t kf = forced[((int64_t)row * T + t) * N + r];
                    if (kf < 0 || kf >= N) {
                        rc = PO_EINVAL;
                        goto done;
                    }
                    if (kf != k) {
                        if (!tie) {
                            if (fail_at) {
                                fail_at[0] = row;
                                fail_at[1] = t;
                                fail_at[2] = r;
                                fail_at[3] = k;
                                fail_at[4] = kf;
                            }
                            rc = PO_EMISMATCH;
                            goto done;
                        }
                        k = kf;
                        if (excused) ++excused[row];
                    }
                }
                ++n_upd;
                if (tie) {
                    ++n_tie;
                    if (tie_log && tie_n && *tie_n < tie_cap) {
                        tie_log[3 * *tie_n + 0] = row;
                        tie_log[3 * *tie_n + 1] = (int32_t)g;
                        tie_log[3 * *tie_n + 2] = r;
                        ++*tie_n;
                    }
                }
                if (choices) choices[((int64_t)row * T + t) * N + r] = k;
                if (k == r) continue;
                /* accept: energy, then influence of the moved facilities */
                ++n_acc;
                e += dE[k];
                const int a = p[r], bfac = p[k];
                for (int i = 0; i < N; ++i) {
                    const int64_t du = (int64_t)D[IDX(i, r)] - D[IDX(i, k)];
                    const int64_t dv = (int64_t)D[IDX(r, i)] - D[IDX(k, i)];
                    for (int c = 0; c < N; ++c) {
                        const int64_t fu = (int64_t)F[IDX(c, bfac)] - F[IDX(c, a)];
                        const int64_t fv = (int64_t)F[IDX(bfac, c)] - F[IDX(a, c)];
                        I[IDX(i, c)] -= du * fu + dv * fv;
                    }
                }
                p[r] = bfac;
                p[k] = a;
                if (e < E_best[row]) {
                    E_best[row] = e;
                    memcpy(pb, p, sizeof(int32_t) * (size_t)N);
                }
            }
            if (E_trace) E_trace[(int64_t)row * T + t] = e;
            if (paranoid) {
                po_influence(N, D, F, p, I2);
                if (memcmp(I, I2, sizeof(int64_t) * (size_t)N * N) != 0 ||
                    e != po_energy(N, D, F, p)) {
                    rc = PO_EMISMATCH;
                    goto done;
                }
            }
        }
        E[row] = e;
        counters[3 * row + 0] = n_upd;
        counters[3 * row + 1] = n_acc;
        counters[3 * row + 2] = n_tie;
    }
done:
    free(I);
    free(I2);
    free(dE);
    free(seen);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Parallel tempering (Results, "Implementation"; Methods, "CPU-PIM      */
/* Algorithm").  A set holds L replicas at L inverse temperatures, slot */
/* 0 the lowest.  After every period of sweeps the slots are visited    */
/* from the lowest beta up: when the replica in slot i+1 has an energy  */
/* greater than or equal to the one in slot i, the two configurations   */
/* change places, so a low-energy configuration can travel to the       */
/* highest beta in one pass.  If the highest slot has not changed hands */
/* for `timeout` passes, it changes places with the lowest slot.        */
/* Configurations changing places is represented by the two replicas    */
/* exchanging slots; each replica keeps its own random stream.          */
/* ------------------------------------------------------------------ */

/*
 * One exchange pass over a set.  E[k]: energy of replica k of the set;
 * slot_of[k] in/out: its slot; since_top in/out: passes since the highest
 * slot last changed hands (timeout <= 0: never forced).  Returns 1 when the
 * highest slot changed hands.
 */
int po_pt_exchange(int L, const int64_t *E, int32_t *slot_of, int32_t *since_top, int32_t timeout)
{
    if (L < 1 || L > 4096 || !E || !slot_of || !since_top) return PO_EINVAL;
    int32_t who[4096];
    for (int i = 0; i < L; ++i) who[i] = -1;
    for (int k = 0; k < L; ++k) {
        if (slot_of[k] < 0 || slot_of[k] >= L || who[slot_of[k]] >= 0) return PO_EINVAL;
        who[slot_of[k]] = k;
    }
    int top = 0;
    for (int i = 0; i + 1 < L; ++i) {
        const int32_t lo = who[i], hi = who[i + 1];
        if (E[hi] >= E[lo]) {
            who[i] = hi;
            who[i + 1] = lo;
            if (i + 1 == L - 1) top = 1;
        }
    }
    if (top) {
        *since_top = 0;
    } else if (timeout > 0 && ++*since_top >= timeout) {
        const int32_t w = who[L - 1];
        who[L - 1] = who[0];
        who[0] = w;
        *since_top = 0;
        top = L > 1;
    }
    for (int i = 0; i < L; ++i) slot_of[who[i]] = i;
    return top;
}

int po_run_cupim(int N, const int32_t *D, const int32_t *F, int R, const int32_t *rep_ids,
                 int32_t inst_id, int32_t *perm, const float *beta, int64_t T, uint64_t seed,
                 uint64_t sweep_off, int64_t *E, int64_t *E_best, int32_t *perm_best,
                 int init_best, int64_t *counters, int32_t *choices, unsigned char *won);

/*
 * n_periods periods of `period_sweeps` sweeps, each followed by an exchange
 * pass in every set; replica k (set k / L) runs its sweeps at
 * ladder[slot_of[k]], with the sequential sweep (method 0) or the GPU-CUPIM
 * iteration (method 1; Methods, "GPU-CUPIM Algorithm": the same exchange
 * rules).  The arguments are those of po_run, plus:
 *   L          replicas per set (R a multiple of L)
 *   ladder     [L] inverse temperatures of the slots, lowest first
 *   slot_of    [R] in/out: slot of each replica within its set
 *   since_top  [R/L] in/out: exchange passes since the set's highest slot
 *              last changed hands
 *   counters   [R*3] out: totals over all periods
 */
int po_run_pt(int N, const int32_t *D, const int32_t *F, int R, int L, int32_t *perm,
              const float *ladder, int32_t *slot_of, int32_t *since_top, int64_t n_periods,
              int64_t period_sweeps, int32_t timeout, uint64_t seed, uint64_t sweep_off,
              int32_t inst_id, int64_t *E, int64_t *E_best, int32_t *perm_best, int init_best,
              int64_t *counters, int method)
{
    if (N < 2 || R < 1 || L < 1 || R % L || n_periods < 0 || period_sweeps < 0 || !ladder ||
        (method != 0 && method != 1) ||
        !slot_of || !since_top || !E || !E_best || !perm_best || !counters)
        return PO_EINVAL;
    float *b = (float *)malloc(sizeof(float) * (size_t)(period_sweeps > 0 ? period_sweeps : 1));
    if (!b) return PO_ENOMEM;
    int rc = PO_OK;
    memset(counters, 0, sizeof(int64_t) * 3 * (size_t)R);
    for (int64_t per = 0; per < n_periods && rc == PO_OK; ++per) {
        for (int k = 0; k < R && rc == PO_OK; ++k) {
            const int32_t sl = slot_of[k];
            if (sl < 0 || sl >= L) {
                rc = PO_EINVAL;
                break;
            }
            for (int64_t t = 0; t < period_sweeps; ++t) b[t] = ladder[sl];
            int64_t cnt[3];
            const int32_t rep = k;
            if (method == 0)
                rc = po_run(N, D, F, 1, &rep, inst_id, perm + (int64_t)k * N, b, period_sweeps,
                            seed, sweep_off + (uint64_t)(per * period_sweeps), E + k, E_best + k,
                            perm_best + (int64_t)k * N, init_best && per == 0, cnt, NULL, 0, NULL,
                            NULL, NULL, 0, NULL, NULL, NULL);
            else
                rc = po_run_cupim(N, D, F, 1, &rep, inst_id, perm + (int64_t)k * N, b,
                                  period_sweeps, seed, sweep_off + (uint64_t)(per * period_sweeps),
                                  E + k, E_best + k, perm_best + (int64_t)k * N,
                                  init_best && per == 0, cnt, NULL, NULL);
            for (int c = 0; c < 3; ++c) counters[3 * k + c] += cnt[c];
        }
        for (int s = 0; s < R / L && rc == PO_OK; ++s) {
            const int x = po_pt_exchange(L, E + (int64_t)s * L, slot_of + (int64_t)s * L,
                                         since_top + s, timeout);
            if (x < 0) rc = x;
        }
    }
    free(b);
    return rc;
}

/* ------------------------------------------------------------------ */
/* GPU-CUPIM (Results, "GPU Implementations"; Methods, "GPU-CUPIM      */
/* Algorithm"): every p-dit of an iteration draws from a snapshot of   */
/* the energy changes taken at the iteration's start; overlapping      */
/* proposals are resolved, and the winners are applied together.      */
/* ------------------------------------------------------------------ */
/*
 * Conflict resolution.  Location r proposes exchanging its facility with
 * location sel[r] (sel[r] == r: no proposal) at snapshot energy change
 * dE[r].  A proposal's key is (dE[r], r), smaller first: the larger energy
 * decrease wins, a tie goes to the lower proposing index.  A proposal wins
 * when no other proposal touching either of its two locations has a
 * smaller key; losers do not move.  Winners are pairwise disjoint.
 * win[r] = 1 for a winning proposal, else 0; returns the number of winners.
 */
int po_cupim_resolve(int N, const int32_t *sel, const int64_t *dE, unsigned char *win)
{
    if (N < 1 || !sel || !dE || !win) return PO_EINVAL;
    int n = 0;
    for (int r = 0; r < N; ++r) {
        win[r] = 0;
        const int s = sel[r];
        if (s < 0 || s >= N) return PO_EINVAL;
        if (s == r) continue;
        int ok = 1;
        for (int q = 0; q < N && ok; ++q) {
            const int u = sel[q];
            if (q == r || u == q) continue;
            if (q != r && q != s && u != r && u != s) continue; /* shares no location */
            if (dE[q] < dE[r] || (dE[q] == dE[r] && q < r)) ok = 0;
        }
        if (ok) {
            win[r] = 1;
            ++n;
        }
    }
    return n;
}

/*
 * T iterations of the concurrent update.  Per iteration g (global sweep
 * sweep_off + t) and replica: the snapshot row of every location r (Eq. 3 on
 * the iteration's starting permutation), the Gibbs choice of each row (Eq. 5,
 * uniform from the Philox counter (r, g, replica, instance) as in po_run),
 * the resolution above, every winning exchange applied, then I and E
 * recomputed from Eq. 2 and Eq. 1.  The best state is checked once per
 * iteration (strict improvement).  counters: updates (N per iteration),
 * accepted (winning exchanges), ties (draws within the tie band).  choices
 * (optional, [R][T][N]): every draw; won (optional, [R][T][N]): the winners.
 */
int po_run_cupim(int N, const int32_t *D, const int32_t *F, int R, const int32_t *rep_ids,
                 int32_t inst_id, int32_t *perm, const float *beta, int64_t T, uint64_t seed,
                 uint64_t sweep_off, int64_t *E, int64_t *E_best, int32_t *perm_best,
                 int init_best, int64_t *counters, int32_t *choices, unsigned char *won)
{
    if (N < 2 || R < 1 || T < 0 || !D || !F || !perm || !beta || !E || !E_best || !perm_best ||
        !counters)
        return PO_EINVAL;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * N);
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *dsel = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    unsigned char *win = (unsigned char *)malloc((size_t)N);
    unsigned char *seen = (unsigned char *)malloc((size_t)N);
    int rc = PO_OK;
    if (!I || !row || !dsel || !sel || !win || !seen) {
        rc = PO_ENOMEM;
        goto done;
    }
    for (int k = 0; k < R; ++k) {
        int32_t *p = perm + (int64_t)k * N;
        int32_t *pb = perm_best + (int64_t)k * N;
        const uint32_t rep = rep_ids ? (uint32_t)rep_ids[k] : (uint32_t)k;
        if (!is_permutation(N, p, seen)) {
            rc = PO_EBADPERM;
            goto done;
        }
        int64_t e = po_energy(N, D, F, p);
        if (init_best) {
            E_best[k] = e;
            memcpy(pb, p, sizeof(int32_t) * (size_t)N);
        }
        int64_t n_acc = 0, n_tie = 0;
        for (int64_t t = 0; t < T; ++t) {
            const uint32_t g = (uint32_t)(sweep_off + (uint64_t)t);
            po_influence(N, D, F, p, I); /* the snapshot */
            for (int r = 0; r < N; ++r) {
                for (int s = 0; s < N; ++s) row[s] = po_delta_eq3(N, D, F, p, I, r, s);
                const uint32_t u24 = po_uniform24(seed, (uint32_t)r, g, rep, (uint32_t)inst_id);
                int tie = 0;
                const int c = po_gibbs_choice(N, row, beta[t], u24, &tie, NULL);
                if (c < 0) {
                    rc = c;
                    goto done;
                }
                n_tie += tie;
                sel[r] = c;
                dsel[r] = row[c];
                if (choices) choices[((int64_t)k * T + t) * N + r] = c;
            }
            n_acc += po_cupim_resolve(N, sel, dsel, win);
            for (int r = 0; r < N; ++r) {
                if (won) won[((int64_t)k * T + t) * N + r] = win[r];
                if (!win[r]) continue;
                const int32_t a = p[r];
                p[r] = p[sel[r]];
                p[sel[r]] = a;
            }
            e = po_energy(N, D, F, p);
            if (e < E_best[k]) {
                E_best[k] = e;
                memcpy(pb, p, sizeof(int32_t) * (size_t)N);
            }
        }
        E[k] = e;
        counters[3 * k + 0] = (int64_t)N * T;
        counters[3 * k + 1] = n_acc;
        counters[3 * k + 2] = n_tie;
    }
done:
    free(I);
    free(row);
    free(dsel);
    free(sel);
    free(win);
    free(seen);
    return rc;
}

/* ------------------------------------------------------------------ */
/* beta-range selection (Results, "Implementation"; Methods, "CPU-PIM   */
/* Algorithm"): short fixed-beta trials on a grid, then the range rule. */
/* ------------------------------------------------------------------ */
/*
 * The rule, on the summed ending energies of the trials (E_sum[g] = sum of
 * the R trial replicas' energies at grid[g], the mean times R, so exact):
 * with Smax and Smin the largest and smallest sums, the low end lo is the
 * first g (lowest beta first) whose sum is at most the level that lies
 * level_pct percent of Smax - Smin above Smin,
 *   100 E_sum[g] <= level_pct Smax + (100 - level_pct) Smin
 * (exact in 128-bit integers).  The paper puts the level at about 40% of the
 * range between the minimum and the maximum: level_pct = 40; the other
 * reading of its wording, a drop of 40% from the maximum, is level_pct = 60.
 * The high end is two grid steps past the first g holding Smin, at most
 * G - 1.  The ladder of L >= 2 rungs is geometric between grid[lo] and
 * grid[hi]: ladder[i] = fl32(grid[lo] * exp(log(grid[hi] / grid[lo]) * i /
 * (L - 1))) in double, with both ends exactly the grid values.
 * lo_hi[0] = lo, lo_hi[1] = hi.  Sums must stay below 2^59 in magnitude and
 * level_pct lie in [0, 100].
 */
int po_beta_rule(int G, const int64_t *E_sum, const float *grid, int L, int level_pct,
                 float *ladder, int32_t *lo_hi)
{
    if (G < 1 || L < 2 || !E_sum || !grid || !ladder || !lo_hi || level_pct < 0 ||
        level_pct > 100)
        return PO_EINVAL;
    const int64_t lim = (int64_t)1 << 59;
    int64_t smax = E_sum[0], smin = E_sum[0];
    int gmin = 0;
    for (int g = 0; g < G; ++g) {
        if (E_sum[g] >= lim || E_sum[g] <= -lim) return PO_EINVAL;
        if (E_sum[g] > smax) smax = E_sum[g];
        if (E_sum[g] < smin) {
            smin = E_sum[g];
            gmin = g;
        }
    }
    const __int128 level = (__int128)level_pct * smax + (__int128)(100 - level_pct) * smin;
    int lo = -1;
    for (int g = 0; g < G && lo < 0; ++g)
        if ((__int128)100 * E_sum[g] <= level) lo = g;
    int hi = gmin + 2 < G ? gmin + 2 : G - 1;
    lo_hi[0] = lo;
    lo_hi[1] = hi;
    const double b0 = grid[lo], b1 = grid[hi];
    for (int i = 0; i < L; ++i)
        ladder[i] = (float)(b0 * exp(log(b1 / b0) * (double)i / (double)(L - 1)));
    ladder[0] = grid[lo];
    ladder[L - 1] = grid[hi];
    return PO_OK;
}

/*
 * The trials: for each beta of the grid (finite, > 0, strictly ascending),
 * R replicas start from the given permutations and run trial_sweeps sweeps
 * at that fixed beta with no exchanges; trial replica k of grid point g
 * draws with Philox replica id g R + k, instance inst_id, from sweep 0.
 * E_trial (optional, [G*R]) receives every ending energy; then the rule
 * with the given level.
 */
int po_beta_select(int N, const int32_t *D, const int32_t *F, int R, const int32_t *perm,
                   const float *grid, int G, int64_t trial_sweeps, uint64_t seed, int32_t inst_id,
                   int L, int level_pct, int64_t *E_sum, float *ladder, int32_t *lo_hi,
                   int64_t *E_trial)
{
    if (N < 2 || R < 1 || G < 1 || trial_sweeps < 0 || !D || !F || !perm || !grid || !E_sum)
        return PO_EINVAL;
    for (int g = 0; g < G; ++g)
        if (!(grid[g] > 0.0f) || !isfinite(grid[g]) || (g > 0 && !(grid[g] > grid[g - 1])))
            return PO_EINVAL;
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)N * R);
    int32_t *pb = (int32_t *)malloc(sizeof(int32_t) * (size_t)N * R);
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int64_t *Eb = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)R);
    float *b = (float *)malloc(sizeof(float) * (size_t)(trial_sweeps > 0 ? trial_sweeps : 1));
    int rc = PO_OK;
    if (!p || !pb || !ids || !E || !Eb || !cnt || !b) {
        rc = PO_ENOMEM;
        goto done;
    }
    for (int g = 0; g < G && rc == PO_OK; ++g) {
        memcpy(p, perm, sizeof(int32_t) * (size_t)N * R);
        for (int k = 0; k < R; ++k) ids[k] = g * R + k;
        for (int64_t t = 0; t < trial_sweeps; ++t) b[t] = grid[g];
        rc = po_run(N, D, F, R, ids, inst_id, p, b, trial_sweeps, seed, 0, E, Eb, pb, 1, cnt, NULL,
                    0, NULL, NULL, NULL, 0, NULL, NULL, NULL);
        int64_t sum = 0;
        for (int k = 0; k < R; ++k) {
            sum += E[k];
            if (E_trial) E_trial[(int64_t)g * R + k] = E[k];
        }
        E_sum[g] = sum;
    }
    if (rc == PO_OK && ladder && lo_hi)
        rc = po_beta_rule(G, E_sum, grid, L, level_pct, ladder, lo_hi);
done:
    free(p);
    free(pb);
    free(ids);
    free(E);
    free(Eb);
    free(cnt);
    free(b);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Exhaustive minimum of Eq. 1 (small N): all permutations with p[0] =  */
/* first (or all of them when first < 0), enumerated by Heap's method. */
/* ------------------------------------------------------------------ */
int64_t po_brute_min(int N, const int32_t *D, const int32_t *F, int first, int32_t *best_perm)
{
    int32_t p[32], rest[32], c[32];
    if (N < 1 || N > 16) return INT64_MIN;
    int off = 0, m = 0;
    if (first >= 0) {
        p[0] = first;
        off = 1;
        for (int v = 0; v < N; ++v)
            if (v != first) rest[m++] = v;
    } else {
        for (int v = 0; v < N; ++v) rest[m++] = v;
    }
    for (int k = 0; k < m; ++k) {
        p[off + k] = rest[k];
        c[k] = 0;
    }
    int64_t best = po_energy(N, D, F, p);
    if (best_perm) memcpy(best_perm, p, sizeof(int32_t) * (size_t)N);
    int k = 1;
    while (k < m) {
        if (c[k] < k) {
            const int j = (k % 2 == 0) ? 0 : c[k];
            const int32_t tmp = p[off + j];
            p[off + j] = p[off + k];
            p[off + k] = tmp;
            const int64_t e = po_energy(N, D, F, p);
            if (e < best) {
                best = e;
                if (best_perm) memcpy(best_perm, p, sizeof(int32_t) * (size_t)N);
            }
            ++c[k];
            k = 1;
        } else {
            c[k] = 0;
            ++k;
        }
    }
    return best;
}
