// sweep_fast.hip -- the sweep kernel with H on chip.
//
// One workgroup owns one replica and keeps its H = D F[p,p] (stored doubled)
// in LDS for the whole run.  The method's order of updates (locations 0..N-1
// per sweep, each a Gibbs choice among N candidates; Results,
// "Implementation", Eq. 3 and Eq. 5) is kept exactly.  The workgroup has
// NMAX/16 waves; wave w owns the 16 locations 16w..16w+15 and the lanes of a
// quad split the candidates of one location four ways.
//
// Size classes (N <= 128 runs on the table kernel, sweep_table.hip; this
// file also holds the class choice and the dispatch):
//   NMAX = 160 (2H int32) and 256 (2H int16, for instances whose exact bound
//     allows it): only H and per-location arrays in LDS, D and F read from
//     device memory (shared by all replicas, so they stay in L2).
//
// Two schedules give the same result:
//
//  * speculative rows (cold sweeps).  An update that keeps its facility
//    ("stay") leaves H unchanged, so the choices of locations pos..N-1 can be
//    evaluated all at once from the current H.  The rows up to the first one
//    that swaps are exactly what the sequential method would do; that swap is
//    applied and evaluation restarts after it.  A sweep with k swaps costs
//    k + 1 such passes.
//
//  * one update at a time (hot sweeps).  Lanes hold the candidates of the
//    current location; the minimum and the running weight sum are wave
//    reductions, computed redundantly by every wave of the replica.  Used for
//    a sweep when the previous one accepted more than `seq_threshold` swaps.
//
// The Gibbs weights are exact integers (q = rint(w 2^25)) summed exactly (in
// 32 bits for N <= 64, in 64 bits beyond), so both schedules, whatever their
// summation order, select the same candidate.  A candidate whose distance d to the row minimum
// satisfies d >= dthr has q = 0 and skips the exponential; d = 0 gives 2^25.
//
// The energy change of swapping the facilities of locations l and s is
//   dE = 2 (H_ls + H_sl - H_ll - H_ss) + (D_ll + D_ss - 2 D_ls)(Fp_ll + Fp_ss - 2 Fp_ls)
// (Eq. 3 with I = -2H); with zero diagonals the last term is 4 D_ls Fp_ls.
// Keeping 2H and 4D makes it two adds and a 24-bit multiply-add.
#include "device_common.h"
#include "pdit_internal.h"
#include "sweep_common.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int32_t kBig = (1 << 30) - 1;  // excluded candidates (|dE| < 2^30 is guaranteed)
constexpr uint32_t kOne = kWeightOne;    // weight of the row minimum

template <int NMAX, bool LARGE, typename HT>
struct FastSmem {
    // padded H rows: column reads are bank-conflict-free
    static constexpr int P = sizeof(HT) == 4 ? NMAX + 1 : NMAX + 2;
    static constexpr int PF = NMAX + 2;  // Fp row pitch (int16)
    HT Hs[NMAX * P];                     // 2 H
    int16_t Ds[LARGE ? 2 : NMAX * NMAX];  // D, times 4 with zero diagonals
    int16_t Fp[LARGE ? 2 : NMAX * PF];    // F[p,p]
    int32_t hdv[NMAX];                   // 2 H[l][l]
    int32_t ddv[NMAX];                   // D[l][l]
    int32_t fdv[NMAX];                   // Fp[l][l]
    int32_t pv[NMAX];                    // p(l)
    int32_t sel_row[2][NMAX];
    int32_t flag_row[2][NMAX];           // bit 0: the row swaps, bit 1: tie
    int32_t seq_msg[2][2];               // one update at a time: wave 0's choice, energy change
    int32_t vswap[NMAX];                 // accepted swap: Fp[r][src] - Fp[s][src] by column
};

// Runs one replica's sweeps with the whole workgroup (NMAX/16 waves).
template <int NMAX, bool ZD, bool EXACT, bool LARGE, typename HT>
__device__ __forceinline__ void fast_replica(const ReplicaJob &a, FastSmem<NMAX, LARGE, HT> &sm) {
    constexpr int WPR = NMAX / 16;         // waves per replica
    constexpr int K = NMAX / 4;            // candidates per lane in a speculative pass
    constexpr int CPL = (NMAX + 63) / 64;  // locations per lane in row-vector work
    constexpr int P = FastSmem<NMAX, LARGE, HT>::P;
    constexpr int PF = FastSmem<NMAX, LARGE, HT>::PF;
    // LDS classes keep 4 D with zero diagonals; large classes read D as is and
    // scale the product instead
    constexpr int kDScale = (ZD && !LARGE) ? 4 : 1;
    constexpr int kProdScale = (ZD && LARGE) ? 4 : 1;
    // CDF type: a lane's partial sum of at most 64 weights of 2^25 fits 32
    // bits; a row's total fits 32 bits only for N <= 64
    using CT = typename std::conditional<(NMAX <= 64), uint32_t, uint64_t>::type;
    HT *Hs = sm.Hs;
    int16_t *Ds = sm.Ds;
    int16_t *Fp = sm.Fp;
    int32_t *hdv = sm.hdv;
    int32_t *ddv = sm.ddv;
    int32_t *fdv = sm.fdv;
    int32_t *pv = sm.pv;

    const int N = EXACT ? NMAX : a.N;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int32_t *__restrict__ Dg = a.D;
    const int32_t *__restrict__ Fg = a.F;

    // D[i][j] and Fp[i][j] = F[p(i)][p(j)]; in the large classes from device
    // memory with indices clamped into the N x N matrices (padding rows and
    // candidates beyond N are computed and discarded)
    auto d_at = [&](int i, int j) -> int32_t {
        if (LARGE) return Dg[(int64_t)min(i, N - 1) * N + min(j, N - 1)];
        return Ds[i * NMAX + j];
    };
    auto fp_at = [&](int i, int j) -> int32_t {
        if (LARGE) return Fg[(int64_t)pv[i] * N + pv[j]];
        return Fp[i * PF + j];
    };

    // ---- stage p, 2H (and D, F[p,p] in the LDS classes); zero outside N ----
    for (int e = tid; e < NMAX; e += 64 * WPR) pv[e] = e < N ? a.perm[e] : 0;
    if (!LARGE) {
        for (int e = tid; e < NMAX * NMAX; e += 64 * WPR) {
            const int i = e / NMAX, j = e % NMAX;
            Ds[e] = (int16_t)((i < N && j < N) ? kDScale * Dg[(int64_t)i * N + j] : 0);
        }
    }
    {
        const int32_t *Hg = (const int32_t *)a.H;
        for (int e = tid; e < NMAX * P; e += 64 * WPR) {
            const int i = e / P, k = e % P;
            Hs[e] = (HT)((i < N && k < N) ? 2 * Hg[(int64_t)i * N + k] : 0);
        }
    }
    __syncthreads();
    if (!LARGE) {
        for (int e = tid; e < NMAX * PF; e += 64 * WPR) {
            const int i = e / PF, k = e % PF;
            Fp[e] = (int16_t)((i < N && k < N) ? Fg[(int64_t)pv[i] * N + pv[k]] : 0);
        }
        __syncthreads();
    }
    for (int e = tid; e < NMAX; e += 64 * WPR) {
        hdv[e] = Hs[e * P + e];
        ddv[e] = (ZD || e >= N) ? 0 : d_at(e, e);
        fdv[e] = (ZD || e >= N) ? 0 : fp_at(e, e);
    }
    __syncthreads();

    int64_t E = *a.E;
    int64_t E_best = *a.E_best;
    int64_t n_acc = 0, n_tie = 0;
    int parity = 0;
    int seq_slot = 0;
    bool seq_mode = false;

    // speculative layout: this lane's location and candidate quarter
    const int rl = lane >> 2, cq = lane & 3;
    const int rr = 16 * wv + rl;  // location of this lane's row

    // energy change of the (uniform) pair r, s
    auto pair_delta = [&](int r, int s) -> int32_t {
        const int32_t h2 = (int32_t)Hs[r * P + s] + (int32_t)Hs[s * P + r] - hdv[r] - hdv[s];
        const int32_t dv = d_at(s, r), fv = fp_at(s, r);
        if (ZD) return h2 + kProdScale * dv * fv;
        return h2 + (ddv[r] + ddv[s] - 2 * dv) * (fdv[r] + fdv[s] - 2 * fv);
    };

    // ---- apply an accepted swap of locations r and s; every wave calls it ----
    auto apply_swap = [&](int r, int s, int64_t dE) {
        E += dE;
        ++n_acc;
        // column k of the new H is column src(k) of H + u v^T, with
        // u_i = D[i][s] - D[i][r] and v_src = Fp[r][src] - Fp[s][src]
        // padding rows (i >= N) get u = 0 and padding columns v = 0, so the
        // update leaves them as they are and the loop below needs no bound
        // test per row or column (such tests made it a chain of branches
        // that waited for every row's LDS reads)
        int src[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int k = (lane + 64 * c) < NMAX ? lane + 64 * c : 0;
            src[c] = k == r ? s : k == s ? r : k;
        }
        // v of every column, gathered once (waves 0..CPL-1, one column per
        // lane) into LDS for all waves after the barrier below: every wave
        // gathering all N columns itself had the scattered loads queue in the
        // CU's load path.  Gathered unconditionally (padding entries of pv
        // are 0, so every address is valid), then zeroed.
        if (wv < CPL) {
            const int k = 64 * wv + lane;
            if (k < NMAX) {
                const int sk = k == r ? s : k == s ? r : k;
                const int32_t dv = fp_at(r, sk) - fp_at(s, sk);
                sm.vswap[k] = (EXACT || k < N) ? dv : 0;
            }
        }
        // 2 u_i of the wave's 16 rows, lane l for row 16 wv + l: one round of
        // loads beside the v gathers instead of one per row in the loop below
        // (d_at clamps its indices, so lanes 16..63 load valid entries too)
        const int iu = 16 * wv + (lane & 15);
        const int32_t du = d_at(s, iu) - d_at(r, iu);
        const int32_t u2l = (lane < 16 && (EXACT || iu < N)) ? (kDScale == 4 ? du / 2 : 2 * du) : 0;
        __syncthreads();  // every read of H, Fp and the per-location arrays is done
        int32_t v[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) v[c] = (lane + 64 * c) < NMAX ? sm.vswap[lane + 64 * c] : 0;
        // RG rows at a time: every read of the group before its writes, so
        // one LDS round trip serves RG rows (two in the largest class, whose
        // 128 registers per lane would otherwise spill)
        constexpr int RG = CPL > 3 ? 2 : 4;
        for (int i0 = 16 * wv; i0 < 16 * wv + 16; i0 += RG) {
            int32_t x[RG][CPL];
#pragma unroll
            for (int q = 0; q < RG; ++q)
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (64 * c + 64 <= NMAX || lane + 64 * c < NMAX)
                        x[q][c] = Hs[(i0 + q) * P + src[c]];
#pragma unroll
            for (int q = 0; q < RG; ++q) {
                const int32_t u2 = __builtin_amdgcn_readlane(u2l, i0 - 16 * wv + q);  // 2 u_i
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (64 * c + 64 <= NMAX || lane + 64 * c < NMAX)
                        Hs[(i0 + q) * P + lane + 64 * c] = (HT)(x[q][c] + u2 * v[c]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < 16 && (EXACT || 16 * wv + lane < N)) {
            const int i = 16 * wv + lane;
            hdv[i] = Hs[i * P + i];
        }
        if (wv == 0) {
            if (!LARGE) {
                // Fp <- Fp with rows r, s and then columns r, s exchanged
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int k = lane + 64 * c;
                    if (k < N) {
                        const int16_t fr = Fp[r * PF + k], fs = Fp[s * PF + k];
                        Fp[r * PF + k] = fs;
                        Fp[s * PF + k] = fr;
                    }
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int k = lane + 64 * c;
                    if (k < N) {
                        const int16_t cr = Fp[k * PF + r], cs = Fp[k * PF + s];
                        Fp[k * PF + r] = cs;
                        Fp[k * PF + s] = cr;
                    }
                }
            }
            if (lane == 0) {
                const int32_t fa = pv[r], fb = pv[s];
                pv[r] = fb;
                pv[s] = fa;
                if (!ZD) {
                    const int32_t t0 = fdv[r];
                    fdv[r] = fdv[s];
                    fdv[s] = t0;
                }
            }
        }
        __syncthreads();
        if (E < E_best) {
            E_best = E;
            if (wv == 0) {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (lane + 64 * c < N) a.perm_best[lane + 64 * c] = pv[lane + 64 * c];
            }
        }
    };

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = a.beta[t * a.beta_stride];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        const int64_t acc_before = n_acc;
        int32_t *ch = (a.choices && wv == 0) ? a.choices + t * N : nullptr;

        if (!seq_mode) {
            // ============ speculative rows: 16 locations per wave, 4 lanes each ============
            const uint32_t u24 = uniform24(a.seed, (uint32_t)rr, g, a.rep, a.inst);
            int pos = 0;
            while (pos < N) {
                const bool rowv = rr < N && rr >= pos;
                int sel = rr;
                bool tie = false, swaps = false;
                if (__ballot(rowv)) {
                    const int32_t nhdr = -hdv[rr];
                    const int32_t ddr = ddv[rr], fdr = fdv[rr];
                    const int32_t prr = pv[rr];
                    const int64_t rrc = min(rr, N - 1);
                    // energy change of candidate cq*K + j of this lane's row
                    auto cand = [&](int j) -> int32_t {
                        const int s = cq * K + j;
                        const int32_t x = (int32_t)Hs[rr * P + s] + (int32_t)Hs[s * P + rr] + nhdr - hdv[s];
                        int32_t dv, fv;
                        if (LARGE) {
                            dv = Dg[(int64_t)min(s, N - 1) * N + rrc];
                            fv = Fg[(int64_t)pv[s] * N + prr];
                        } else {
                            dv = Ds[s * NMAX + rr];
                            fv = Fp[s * PF + rr];
                        }
                        int32_t v;
                        if (ZD) {
                            v = kProdScale * __mul24(dv, fv) + x;
                        } else {
                            v = x + __mul24(ddr + ddv[s] - 2 * dv, fdr + fdv[s] - 2 * fv);
                        }
                        if (!EXACT && s >= N) v = kBig;
                        return v;
                    };
                    // weight of a candidate at distance d from the row minimum:
                    // d = 0 -> 2^25; 0 < d < dthr -> expf; d >= dthr -> 0
                    auto weight = [&](int j, int32_t d) -> uint32_t {
                        const bool zero = d == 0;
                        uint32_t q = zero ? kOne : 0u;
                        const bool need = d < dthr && !zero;
                        if (__ballot(need)) {
                            if (need) q = gibbs_weight(beta, (float)d);
                        }
                        if (!EXACT && cq * K + j >= N) q = 0;
                        return q;
                    };
                    // the small classes keep the row in registers; the large
                    // ones recompute it in each pass instead
                    constexpr int KR = LARGE ? 1 : K;
                    int32_t dl[KR];
                    uint32_t ql[KR];
                    int32_t mn = kBig;
#pragma unroll(LARGE ? 4 : K)
                    for (int j = 0; j < K; ++j) {
                        const int32_t v = cand(j);
                        if (!LARGE) dl[j % KR] = v;
                        mn = min(mn, v);
                    }
                    mn = min(mn, quad<kQuadXor1>(mn));
                    mn = min(mn, quad<kQuadXor2>(mn));
                    uint32_t Zc = 0;
                    int am = -1;
#pragma unroll(LARGE ? 4 : K)
                    for (int j = 0; j < K; ++j) {
                        const int32_t d = (LARGE ? cand(j) : dl[j % KR]) - mn;
                        const uint32_t q = weight(j, d);
                        am = d == 0 ? cq * K + j : am;
                        if (!LARGE) ql[j % KR] = q;
                        Zc += q;
                    }
                    // quarters before this one, and the row total
                    const CT p1 = quadu<kQuadPrev1>(Zc), p2 = quadu<kQuadPrev2>(Zc),
                             p3 = quadu<kQuadPrev3>(Zc);
                    const CT off = (cq >= 1 ? p1 : 0) + (cq >= 2 ? p2 : 0) + (cq >= 3 ? p3 : 0);
                    const CT Z = quadu<kQuadLast>((CT)(off + Zc));
                    am = max(am, quad<kQuadXor1>(am));
                    am = max(am, quad<kQuadXor2>(am));
                    sel = am;
                    // a row whose only nonzero weight is its minimum (Z = 2^25)
                    // picks the minimum; otherwise locate the threshold by
                    // counting: the first s with C_s > thr is #{s : C_s <= thr},
                    // and a tie is a boundary thr_lo < C_s <= thr_hi (the band
                    // around the threshold, with 0 < C_s < Z)
                    if (__ballot(rowv && Z != kOne)) {
                        const uint64_t target = (uint64_t)u24 * Z;
                        const uint64_t band = (uint64_t)Z << 4;
                        const CT thr = (CT)(target >> 24);
                        const CT thr_lo = target >= band ? (CT)((target - band) >> 24) : 0;
                        const CT thr_hi = (CT)min((target + band) >> 24, (uint64_t)(Z - 1));
                        const CT lo1 = thr_lo + 1;
                        const CT width = thr_hi >= lo1 ? thr_hi - thr_lo : 0;
                        CT C = off;
                        int n_sel = 0, n_band = 0;
#pragma unroll(LARGE ? 4 : K)
                        for (int j = 0; j < K; ++j) {
                            C += LARGE ? weight(j, cand(j) - mn) : ql[j % KR];
                            n_sel += C <= thr;
                            n_band += (C - lo1) < width;
                        }
                        n_sel += quad<kQuadXor1>(n_sel);
                        n_sel += quad<kQuadXor2>(n_sel);
                        n_band += quad<kQuadXor1>(n_band);
                        n_band += quad<kQuadXor2>(n_band);
                        if (Z != kOne) {
                            sel = n_sel;
                            tie = n_band > 0;
                        }
                    }
                    swaps = rowv && sel != rr;
                }
                if (cq == 0) {
                    sm.sel_row[parity][rr] = sel;
                    sm.flag_row[parity][rr] = (swaps ? 1 : 0) | (rowv && tie ? 2 : 0);
                }
                __syncthreads();
                // every wave reads the same flags: first swapping row from pos
                int last = N - 1;
                bool found = false;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int row = lane + 64 * c;
                    const int32_t fl = row < NMAX ? sm.flag_row[parity][row] : 0;
                    const uint64_t acc_mask = __ballot(fl & 1);
                    if (!found && acc_mask) {
                        last = 64 * c + __ffsll((unsigned long long)acc_mask) - 1;
                        found = true;
                    }
                }
                if (wv == 0) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const int row = lane + 64 * c;
                        const int32_t fl = row < NMAX ? sm.flag_row[parity][row] : 0;
                        const bool committed = row >= pos && row <= last && row < N;
                        n_tie += __popcll(__ballot(committed && (fl & 2)));
                        if (ch && committed) ch[row] = sm.sel_row[parity][row];
                    }
                }
                if (found) {
                    const int s = sm.sel_row[parity][last];
                    apply_swap(last, s, (int64_t)pair_delta(last, s));
                }
                parity ^= 1;
                pos = last + 1;
            }
        } else {
            // ============ one update at a time: lane = candidate ============
            uint32_t u24l[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                u24l[c] = uniform24(a.seed, (uint32_t)(lane + 64 * c), g, a.rep, a.inst);
            for (int r = 0; r < N; ++r) {
                // wave 0 draws; the other waves take its choice at the barrier
                // (slots alternate per update, so one barrier per update suffices)
                if (wv == 0) {
                    int32_t v[CPL];
                    uint32_t q[CPL];
                    int32_t lmin = kBig;
                    const int32_t pr = pv[r];
    #pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const int ls = lane + 64 * c;
                        v[c] = kBig;
                        if (ls < N) {
                            const int32_t x = (int32_t)Hs[r * P + ls] + (int32_t)Hs[ls * P + r] - hdv[r] - hdv[ls];
                            int32_t dv, fv;
                            if (LARGE) {
                                dv = Dg[(int64_t)r * N + ls];
                                fv = Fg[(int64_t)pr * N + pv[ls]];
                            } else {
                                dv = Ds[r * NMAX + ls];
                                fv = Fp[r * PF + ls];
                            }
                            if (ZD) {
                                v[c] = kProdScale * __mul24(dv, fv) + x;
                            } else {
                                v[c] = x + __mul24(ddv[r] + ddv[ls] - 2 * dv, fdv[r] + fdv[ls] - 2 * fv);
                            }
                        }
                        lmin = min(lmin, v[c]);
                    }
                    const int32_t mn = wave_min_i32(lmin);
                    CT C[CPL];
                    CT base = 0;
    #pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const bool valid = lane + 64 * c < N;
                        const int32_t d = valid ? v[c] - mn : 0;
                        q[c] = d == 0 ? kOne : 0u;
                        if (d > 0 && d < dthr) q[c] = gibbs_weight(beta, (float)d);
                        if (!valid) q[c] = 0;
                        // one chunk of 64 weights sums to at most 2^31
                        C[c] = base + (CT)wave_scan_u32(q[c]);
                        base = (CT)readlane_u64((uint64_t)C[c], 63);
                    }
                    const CT Z = base;
                    uint32_t ur24 = 0;
    #pragma unroll
                    for (int c = 0; c < CPL; ++c)
                        if ((r >> 6) == c) ur24 = (uint32_t)__builtin_amdgcn_readlane((int32_t)u24l[c], r & 63);
                    const CT thr = (CT)(((uint64_t)ur24 * Z) >> 24);
                    int s = -1;
    #pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const uint64_t hit = __ballot(C[c] > thr);
                        if (s < 0 && hit) s = 64 * c + __ffsll((unsigned long long)hit) - 1;
                    }
                    if (s < 0 || s >= N) s = r;  // unreachable: location N-1 holds C = Z > thr
                    const int sl = s & 63;
                    CT csel = 0;
                    uint32_t qsel = 0;
                    int32_t vsel = 0;
    #pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        if ((s >> 6) == c) {
                            csel = (CT)readlane_u64((uint64_t)C[c], sl);
                            qsel = (uint32_t)__builtin_amdgcn_readlane((int32_t)q[c], sl);
                            vsel = __builtin_amdgcn_readlane(v[c], sl);
                        }
                    }
                    if (wv == 0) n_tie += is_tie(csel - qsel, csel, Z, ur24) ? 1 : 0;
                    if (ch && lane == 0) ch[r] = s;
                    if (lane == 0) {
                        sm.seq_msg[seq_slot][0] = s;
                        sm.seq_msg[seq_slot][1] = vsel;
                    }
                }
                __syncthreads();
                const int s = sm.seq_msg[seq_slot][0];
                const int32_t vsel = sm.seq_msg[seq_slot][1];
                seq_slot ^= 1;
                if (s != r) apply_swap(r, s, (int64_t)vsel);
            }
        }
        seq_mode = (n_acc - acc_before) > a.seq_threshold;
        if (a.E_trace && tid == 0) a.E_trace[t] = E;
    }

    if (a.flags & kSaveState) {
        // H of the final state back to device memory (the next launch resumes from it)
        __syncthreads();
        int32_t *Hout = (int32_t *)const_cast<void *>(a.H);
        for (int e = tid; e < N * N; e += 64 * WPR) {
            const int i = e / N, k = e % N;
            Hout[e] = (int32_t)Hs[i * P + k] / 2;
        }
    }
    if (wv == 0) {
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (lane + 64 * c < N) a.perm[lane + 64 * c] = pv[lane + 64 * c];
        if (lane == 0) {
            *a.E = E;
            *a.E_best = E_best;
            const bool acc = (a.flags & kAccumCounters) != 0;
            a.counters[0] = (acc ? a.counters[0] : 0) + (int64_t)N * a.T;
            a.counters[1] = (acc ? a.counters[1] : 0) + n_acc;
            a.counters[2] = (acc ? a.counters[2] : 0) + n_tie;
        }
    }
}

// Waves per SIMD each class runs at (one replica's waves spread over the
// CU's four SIMDs): four replicas of N <= 64 per CU, one replica otherwise.
template <int NMAX>
constexpr int fast_waves_per_eu() {
    return NMAX <= 64 ? 4 : NMAX == 128 ? 2 : NMAX == 160 ? 3 : 4;
}

// H element type of each class.
template <int NMAX>
using FastH = typename std::conditional<NMAX == 256, int16_t, int32_t>::type;
template <int NMAX>
constexpr bool fast_large() { return NMAX > 128; }

// One replica per workgroup (single-instance runs).
template <int NMAX, bool ZD, bool EXACT>
__global__ void __launch_bounds__(64 * (NMAX / 16))
__attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<NMAX>())))
sweep_fast_kernel(SweepArgs a) {
    __shared__ FastSmem<NMAX, fast_large<NMAX>(), FastH<NMAX>> sm;
    const int64_t rep = blockIdx.x;
    ReplicaJob j;
    j.N = a.N;
    j.D = a.D;
    j.F = a.F;
    j.perm = a.perm + rep * a.N;
    j.H = (const int32_t *)a.H + rep * (int64_t)a.N * a.N;
    j.E = a.E + rep;
    j.E_best = a.E_best + rep;
    j.perm_best = a.perm_best + rep * a.N;
    j.counters = a.counters + 3 * rep;
    job_beta(j, a.beta, a.slot, rep);
    j.T = a.T;
    j.seed = a.seed;
    j.sweep_offset = a.sweep_offset;
    j.rep = (uint32_t)rep;
    j.inst = a.inst_id;
    j.choices = a.choices ? a.choices + rep * a.T * a.N : nullptr;
    j.E_trace = a.E_trace ? a.E_trace + rep * a.T : nullptr;
    j.seq_threshold = a.seq_threshold;
    j.zero_diag = ZD;
    j.tstate = nullptr;
    j.flags = a.flags;
    fast_replica<NMAX, ZD, EXACT, fast_large<NMAX>(), FastH<NMAX>>(j, sm);
}

// Persistent: each workgroup takes (instance, replica) items from a queue
// until it is exhausted; items come largest N first.  Every workgroup
// reaches the exit: the queue only grows, so each one reads an item index
// >= n_items after at most n_items increments.
template <int NMAX, bool ZD>
__global__ void __launch_bounds__(64 * (NMAX / 16))
__attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<NMAX>())))
sweep_fast_persistent(BatchArgs b) {
    __shared__ FastSmem<NMAX, fast_large<NMAX>(), FastH<NMAX>> sm;
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(item_sh);  // wave-uniform
        __syncthreads();
        if (item >= b.n_items) break;
        fast_replica<NMAX, ZD, false, fast_large<NMAX>(), FastH<NMAX>>(
            batch_job(b, item, sizeof(int32_t)), sm);
        __syncthreads();
    }
}

template <int NMAX, bool ZD, bool EXACT>
hipError_t launch_fast(hipStream_t s, const SweepArgs &a) {
    sweep_fast_kernel<NMAX, ZD, EXACT><<<a.R, 64 * (NMAX / 16), 0, s>>>(a);
    return hipGetLastError();
}

template <int NMAX>
hipError_t launch_nmax(hipStream_t s, const SweepArgs &a) {
    const bool exact = a.N == NMAX;
    if (a.zero_diag)
        return exact ? launch_fast<NMAX, true, true>(s, a) : launch_fast<NMAX, true, false>(s, a);
    return exact ? launch_fast<NMAX, false, true>(s, a) : launch_fast<NMAX, false, false>(s, a);
}

template <int NMAX>
hipError_t launch_persistent_nmax(hipStream_t s, bool zd, const BatchArgs &b, int grid) {
    if (zd)
        sweep_fast_persistent<NMAX, true><<<grid, 64 * (NMAX / 16), 0, s>>>(b);
    else
        sweep_fast_persistent<NMAX, false><<<grid, 64 * (NMAX / 16), 0, s>>>(b);
    return hipGetLastError();
}

template <int NMAX>
int persistent_blocks_per_cu() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, sweep_fast_persistent<NMAX, true>, 64 * (NMAX / 16), 0);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

int fast_class(int N, const InstanceStats &st) {
    if (N < 2 || N > kFastNMax) return 0;
    const int64_t bound = h_bound(st);
    // H and dE in int32 with |dE| < 2^30 - 1 (below the excluded-candidate
    // sentinel), 24-bit products
    if (bound > INT32_MAX || delta_bound(st) >= (int64_t)(1 << 30) - 1) return 0;
    if (st.max_abs_d >= (1 << 21) || st.max_abs_f >= (1 << 21)) return 0;
    if (N <= 128) {
        // D and F[p,p] in int16
        if (st.max_abs_d > 32767 || st.max_abs_f > 32767) return 0;
        return N <= 16 ? 16 : N <= 32 ? 32 : N <= 64 ? 64 : N <= 96 ? 96 : 128;
    }
    if (N <= 160) return 160;
    // 2H in int16
    return 2 * bound <= 32767 ? 256 : 0;
}

hipError_t launch_sweep_fast(hipStream_t s, int nmax, const SweepArgs &a0) {
    SweepArgs a = a0;
    if (a.seq_threshold < 0) a.seq_threshold = default_seq_threshold(nmax, a.N);
    if (nmax <= 128) return launch_sweep_table(s, nmax, a);
    switch (nmax) {
        case 160: return launch_nmax<160>(s, a);
        case 256: return launch_nmax<256>(s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_fast_persistent(hipStream_t s, int nmax, bool zd, const BatchArgs &b,
                                        int grid) {
    if (nmax <= 128) return launch_sweep_table_persistent(s, nmax, zd, b, grid);
    switch (nmax) {
        case 160: return launch_persistent_nmax<160>(s, zd, b, grid);
        case 256: return launch_persistent_nmax<256>(s, zd, b, grid);
        default: return hipErrorInvalidValue;
    }
}

int fast_blocks_per_cu(int nmax) {
    if (nmax <= 128) return table_blocks_per_cu(nmax);
    switch (nmax) {
        case 160: return persistent_blocks_per_cu<160>();
        case 256: return persistent_blocks_per_cu<256>();
        default: return 1;
    }
}

}  // namespace pdit
