// sweep_fast.hip -- the sweep kernel with H on chip.
//
// One workgroup owns one replica.  Its H = D F[p,p] (int32, stored doubled)
// and its permuted flows Fp = F[p,p] (int16), with D (int16), live in LDS for
// the whole run; N <= 64.  The method's order of updates (locations 0..N-1 per
// sweep, each a Gibbs choice among N candidates; Results, "Implementation",
// Eq. 3 and Eq. 5) is kept exactly.  The workgroup has NMAX/16 waves; wave w
// owns the 16 locations 16w..16w+15 and the lanes of a quad split the
// candidates of one location four ways, so a replica keeps NMAX/16 waves
// busy and four replicas of N = 64 share a CU with four waves per SIMD.
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
// The Gibbs weights are exact integers (q = rint(w 2^25)); for N <= 64 their
// sums fit 32 bits, so both schedules, whatever their summation order, select
// the same candidate.  A candidate whose distance d to the row minimum
// satisfies d >= dthr has q = 0 and skips the exponential; d = 0 gives 2^25.
//
// The energy change of swapping the facilities of locations l and s is
//   dE = 2 (H_ls + H_sl - H_ll - H_ss) + (D_ll + D_ss - 2 D_ls)(Fp_ll + Fp_ss - 2 Fp_ls)
// (Eq. 3 with I = -2H); with zero diagonals the last term is 4 D_ls Fp_ls.
// Keeping 2H and 4D makes it two adds and a 24-bit multiply-add.
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

constexpr int32_t kBig = (1 << 30) - 1;  // excluded candidates (|dE| < 2^30 is guaranteed)
constexpr uint32_t kOne = kWeightOne;    // weight of the row minimum

// quad_perm DPP selectors (lane i of each quad reads lane sel[i])
constexpr int kQuadXor1 = 0xB1;   // [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // [2,3,0,1]
constexpr int kQuadPrev1 = 0x90;  // [0,0,1,2]
constexpr int kQuadPrev2 = 0x40;  // [0,0,0,1]
constexpr int kQuadPrev3 = 0x00;  // [0,0,0,0]
constexpr int kQuadLast = 0xFF;   // [3,3,3,3]

template <int CTRL>
__device__ __forceinline__ int32_t quad(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint32_t quadu(uint32_t v) {
    return (uint32_t)quad<CTRL>((int32_t)v);
}

// four replicas of N = 64 per CU need four waves per SIMD: at most 128 VGPRs
template <int NMAX, bool ZD, bool EXACT>
__global__ void __launch_bounds__(64 * (NMAX / 16)) __attribute__((amdgpu_waves_per_eu(4)))
sweep_fast_kernel(SweepArgs a) {
    constexpr int WPR = NMAX / 16;  // waves per replica
    constexpr int K = NMAX / 4;     // candidates per lane in a speculative pass
    constexpr int P = NMAX + 1;     // H row pitch (int32): column reads are conflict-free
    constexpr int PF = NMAX + 2;    // Fp row pitch (int16)
    constexpr int kDScale = ZD ? 4 : 1;  // Ds holds 4 D with zero diagonals

    __shared__ int32_t Hs[NMAX * P];  // 2 H
    __shared__ int16_t Ds[NMAX * NMAX];
    __shared__ int16_t Fp[NMAX * PF];
    __shared__ int32_t hdv[NMAX];  // 2 H[l][l]
    __shared__ int32_t ddv[NMAX];  // D[l][l]
    __shared__ int32_t fdv[NMAX];  // Fp[l][l]
    __shared__ int32_t pv[NMAX];   // p(l)
    __shared__ int32_t sel_row[2][NMAX];
    __shared__ int32_t flag_row[2][NMAX];  // bit 0: the row swaps, bit 1: tie

    const int N = EXACT ? NMAX : a.N;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t rep = blockIdx.x;

    // ---- stage D, p, 2H and F[p,p] (zero outside N) ----
    for (int e = tid; e < NMAX * NMAX; e += 64 * WPR) {
        const int i = e / NMAX, j = e % NMAX;
        Ds[e] = (int16_t)((i < N && j < N) ? kDScale * a.D[(int64_t)i * N + j] : 0);
    }
    for (int e = tid; e < NMAX; e += 64 * WPR) pv[e] = e < N ? a.perm[rep * N + e] : 0;
    {
        const int32_t *Hg = (const int32_t *)a.H + rep * (int64_t)N * N;
        for (int e = tid; e < NMAX * P; e += 64 * WPR) {
            const int i = e / P, k = e % P;
            Hs[e] = (i < N && k < N) ? 2 * Hg[(int64_t)i * N + k] : 0;
        }
    }
    __syncthreads();
    for (int e = tid; e < NMAX * PF; e += 64 * WPR) {
        const int i = e / PF, k = e % PF;
        Fp[e] = (int16_t)((i < N && k < N) ? a.F[(int64_t)pv[i] * N + pv[k]] : 0);
    }
    __syncthreads();
    for (int e = tid; e < NMAX; e += 64 * WPR) {
        hdv[e] = Hs[e * P + e];
        ddv[e] = ZD ? 0 : Ds[e * NMAX + e];
        fdv[e] = ZD ? 0 : Fp[e * PF + e];
    }
    __syncthreads();

    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0, n_tie = 0;
    int parity = 0;
    bool seq_mode = false;

    // speculative layout: this lane's location and candidate quarter
    const int rl = lane >> 2, cq = lane & 3;
    const int rr = 16 * wv + rl;  // location of this lane's row
    // candidate layout for one-update-at-a-time (lanes >= NMAX are idle)
    const int ls = lane < NMAX ? lane : 0;

    // energy change of the (uniform) pair r, s, from LDS
    auto pair_delta = [&](int r, int s) -> int32_t {
        const int32_t h2 = Hs[r * P + s] + Hs[s * P + r] - hdv[r] - hdv[s];
        const int32_t dv = Ds[s * NMAX + r], fv = Fp[s * PF + r];
        if (ZD) return h2 + dv * fv;
        return h2 + (ddv[r] + ddv[s] - 2 * dv) * (fdv[r] + fdv[s] - 2 * fv);
    };

    // ---- apply an accepted swap of locations r and s; every wave calls it ----
    auto apply_swap = [&](int r, int s, int64_t dE) {
        E += dE;
        ++n_acc;
        // column k of the new H is column src(k) of H + u v^T, with
        // u_i = D[i][s] - D[i][r] and v_src = Fp[r][src] - Fp[s][src]
        const int src = ls == r ? s : ls == s ? r : ls;
        const int32_t v = (int32_t)Fp[r * PF + src] - (int32_t)Fp[s * PF + src];
        __syncthreads();  // every read of H, Fp and the per-location arrays is done
#pragma unroll 4
        for (int ii = 0; ii < 16; ++ii) {
            const int i = 16 * wv + ii;
            if (EXACT || i < N) {
                const int32_t du = (int32_t)Ds[s * NMAX + i] - (int32_t)Ds[r * NMAX + i];
                const int32_t u2 = ZD ? du / 2 : 2 * du;  // 2 u_i
                const int32_t x = Hs[i * P + src];
                if (lane < N) Hs[i * P + lane] = x + u2 * v;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < 16 && (EXACT || 16 * wv + lane < N)) {
            const int i = 16 * wv + lane;
            hdv[i] = Hs[i * P + i];
        }
        if (wv == 0) {
            // Fp <- Fp with rows r, s and then columns r, s exchanged
            if (lane < N) {
                const int16_t fr = Fp[r * PF + lane], fs = Fp[s * PF + lane];
                Fp[r * PF + lane] = fs;
                Fp[s * PF + lane] = fr;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < N) {
                const int16_t cr = Fp[lane * PF + r], cs = Fp[lane * PF + s];
                Fp[lane * PF + r] = cs;
                Fp[lane * PF + s] = cr;
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
            if (wv == 0 && lane < N) a.perm_best[rep * N + lane] = pv[lane];
        }
    };

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = a.beta[t];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        const int64_t acc_before = n_acc;
        int32_t *ch = (a.choices && wv == 0) ? a.choices + (rep * a.T + t) * N : nullptr;

        if (!seq_mode) {
            // ============ speculative rows: 16 locations per wave, 4 lanes each ============
            const uint32_t u24 = uniform24(a.seed, (uint32_t)rr, g, (uint32_t)rep, a.inst_id);
            int pos = 0;
            while (pos < N) {
                const bool rowv = rr < N && rr >= pos;
                int sel = rr;
                bool tie = false, swaps = false;
                if (__ballot(rowv)) {
                    const int32_t nhdr = -hdv[rr];
                    const int32_t ddr = ddv[rr], fdr = fdv[rr];
                    int32_t dl[K];
                    int32_t mn = kBig;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const int s = cq * K + j;
                        const int32_t x = Hs[rr * P + s] + Hs[s * P + rr] + nhdr - hdv[s];
                        const int32_t dv = Ds[s * NMAX + rr];
                        const int32_t fv = Fp[s * PF + rr];
                        int32_t v;
                        if (ZD) {
                            v = __mul24(dv, fv) + x;
                        } else {
                            v = x + __mul24(ddr + ddv[s] - 2 * dv, fdr + fdv[s] - 2 * fv);
                        }
                        if (!EXACT && s >= N) v = kBig;
                        dl[j] = v;
                        mn = min(mn, v);
                    }
                    mn = min(mn, quad<kQuadXor1>(mn));
                    mn = min(mn, quad<kQuadXor2>(mn));
                    // weights: d = 0 -> 2^25; 0 < d < dthr -> expf; d >= dthr -> 0
                    uint32_t ql[K];
                    uint32_t Zc = 0;
                    int am = -1;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const int32_t d = dl[j] - mn;
                        const bool zero = d == 0;
                        uint32_t q = zero ? kOne : 0u;
                        am = zero ? cq * K + j : am;
                        const bool need = d < dthr && !zero;
                        if (__ballot(need)) {
                            if (need) q = gibbs_weight(beta, (float)d);
                        }
                        if (!EXACT && cq * K + j >= N) q = 0;
                        ql[j] = q;
                        Zc += q;
                    }
                    // quarters before this one, and the row total
                    const uint32_t p1 = quadu<kQuadPrev1>(Zc), p2 = quadu<kQuadPrev2>(Zc),
                                   p3 = quadu<kQuadPrev3>(Zc);
                    const uint32_t off = (cq >= 1 ? p1 : 0u) + (cq >= 2 ? p2 : 0u) + (cq >= 3 ? p3 : 0u);
                    const uint32_t Z = quadu<kQuadLast>(off + Zc);
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
                        const uint32_t thr = (uint32_t)(target >> 24);
                        const uint32_t thr_lo = target >= band ? (uint32_t)((target - band) >> 24) : 0u;
                        const uint32_t thr_hi = (uint32_t)min((target + band) >> 24, (uint64_t)(Z - 1));
                        const uint32_t lo1 = thr_lo + 1;
                        const uint32_t width = thr_hi >= lo1 ? thr_hi - thr_lo : 0u;
                        uint32_t C = off;
                        int n_sel = 0, n_band = 0;
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            C += ql[j];
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
                    sel_row[parity][rr] = sel;
                    flag_row[parity][rr] = (swaps ? 1 : 0) | (rowv && tie ? 2 : 0);
                }
                __syncthreads();
                // every wave reads the same flags: first swapping row from pos
                const int32_t fl = lane < NMAX ? flag_row[parity][lane] : 0;
                const uint64_t acc_mask = __ballot(fl & 1);
                const int last = acc_mask ? __ffsll((unsigned long long)acc_mask) - 1 : N - 1;
                const bool committed = lane >= pos && lane <= last && lane < N;
                if (wv == 0) {
                    n_tie += __popcll(__ballot(committed && (fl & 2)));
                    if (ch && committed) ch[lane] = sel_row[parity][lane];
                }
                if (acc_mask) {
                    const int s = sel_row[parity][last];
                    apply_swap(last, s, (int64_t)pair_delta(last, s));
                }
                parity ^= 1;
                pos = last + 1;
            }
        } else {
            // ============ one update at a time: lane = candidate ============
            const uint32_t u24l = uniform24(a.seed, (uint32_t)ls, g, (uint32_t)rep, a.inst_id);
            const bool lv = lane < N;
            for (int r = 0; r < N; ++r) {
                int32_t v = kBig;
                if (lv) {
                    const int32_t x = Hs[r * P + ls] + Hs[ls * P + r] - hdv[r] - hdv[ls];
                    const int32_t dv = Ds[r * NMAX + ls];
                    const int32_t fv = Fp[r * PF + ls];
                    if (ZD) {
                        v = __mul24(dv, fv) + x;
                    } else {
                        v = x + __mul24(ddv[r] + ddv[ls] - 2 * dv, fdv[r] + fdv[ls] - 2 * fv);
                    }
                }
                const int32_t mn = wave_min_i32(v);
                const int32_t d = lv ? v - mn : 0;
                uint32_t q = d == 0 ? kOne : 0u;
                if (d > 0 && d < dthr) q = gibbs_weight(beta, (float)d);
                if (!lv) q = 0;
                const uint32_t C = wave_scan_u32(q);
                const uint32_t Z = (uint32_t)__builtin_amdgcn_readlane((int32_t)C, 63);
                const uint32_t ur24 = (uint32_t)__builtin_amdgcn_readlane((int32_t)u24l, r);
                const uint32_t thr = (uint32_t)(((uint64_t)ur24 * Z) >> 24);
                const uint64_t hit = __ballot(C > thr);
                int s = __ffsll((unsigned long long)hit) - 1;
                if (s < 0 || s >= N) s = r;  // unreachable: lane N-1 holds C = Z > thr
                const uint32_t csel = (uint32_t)__builtin_amdgcn_readlane((int32_t)C, s);
                const uint32_t cprev = csel - (uint32_t)__builtin_amdgcn_readlane((int32_t)q, s);
                if (wv == 0) n_tie += is_tie(cprev, csel, Z, ur24) ? 1 : 0;
                if (ch && lane == 0) ch[r] = s;
                if (s != r) apply_swap(r, s, (int64_t)__builtin_amdgcn_readlane(v, s));
            }
        }
        seq_mode = (n_acc - acc_before) > a.seq_threshold;
        if (a.E_trace && tid == 0) a.E_trace[rep * a.T + t] = E;
    }

    if (wv == 0) {
        if (lane < N) a.perm[rep * N + lane] = pv[lane];
        if (lane == 0) {
            a.E[rep] = E;
            a.E_best[rep] = E_best;
            a.counters[rep * 3 + 0] = (int64_t)N * a.T;
            a.counters[rep * 3 + 1] = n_acc;
            a.counters[rep * 3 + 2] = n_tie;
        }
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

}  // namespace

bool sweep_fast_supports(int N) { return N >= 2 && N <= 64; }

hipError_t launch_sweep_fast(hipStream_t s, const SweepArgs &a0) {
    SweepArgs a = a0;
    if (a.seq_threshold < 0) a.seq_threshold = 3;
    if (a.N <= 16) return launch_nmax<16>(s, a);
    if (a.N <= 32) return launch_nmax<32>(s, a);
    return launch_nmax<64>(s, a);
}

}  // namespace pdit
