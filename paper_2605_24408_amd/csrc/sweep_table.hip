// sweep_table.hip -- the sweep kernel for N <= 128, with the table of swap
// energy changes on chip.
//
// One workgroup owns one replica.  For the whole run it keeps in LDS the
// N x N table T[l][s] = energy change of exchanging the facilities of
// locations l and s (Eq. 3, with I = -2H for symmetric D and F), the
// distances D and the permuted flows Fp = F[p,p] (int16), and the diagonal
// of H = D Fp.  The method's order of updates (locations 0..N-1 per sweep,
// each a Gibbs choice among N candidates including the stay, Eq. 5) is kept
// exactly; the table only changes how a candidate's energy change is
// obtained: one quarter of a 16-byte LDS load instead of five loads and
// five operations on H, D and Fp.
//
// After an accepted exchange of locations r and t (Fp' is Fp with rows and
// columns r, t exchanged), with a_x = D[x][r] - D[x][t] and
// c_x = Fp[x][t] - Fp[x][r]:
//   T'[l][s] = T[l][s] + (a_s - a_l)(2 c_l - 2 c_s)   for l, s not in {r, t}
//   H'[x][x] = H[x][x] + a_x c_x                        for x not in {r, t}
// and rows and columns r and t follow from Eq. 3 with the four vectors
// H'[r][.], H'[t][.], H'[.][r], H'[.][t], each the product of a row of D or
// Fp' with the other (symmetric) matrix, as int16 dot products.  That is
// O(N^2) per accepted move, the order of the method's own H update.  All
// table arithmetic is integer modulo 2^32 and every stored value is a true
// energy change of magnitude below 2^30, so the table is exact.
//
// Two schedules give the same result:
//
//  * speculative rows (cold sweeps).  A stay leaves the table unchanged, so
//    the choices of locations pos..N-1 can be drawn all at once; the rows up
//    to the first one that swaps are what the sequential method does, that
//    swap is applied and the pass restarts after it.  16 locations per
//    wave, the four lanes of a quad splitting a location's candidates.
//
//  * one update at a time (hot sweeps, after a sweep with more than
//    `seq_threshold` accepted moves): lanes hold the candidates of the
//    current location; minimum and running weight sum are wave reductions,
//    done redundantly by every wave of the replica.
//
// Weights are the integers q = rint(expf(-fl32(beta fl32(d))) 2^25) of the
// distance d >= 0 to the row minimum, summed exactly (32 bits for N <= 64,
// 64 bits beyond), so the schedules agree whatever their summation order.
// A candidate with d >= dthr has q = 0.  The stay's energy change is 0, so
// the table's diagonal holds a sentinel (kBig) instead and the smallest
// entry m of a row is its best move: m >= dthr puts all the row's weight on
// the stay, whose draw then keeps the facility whatever the uniform; such a
// row evaluates no weights, and no uniform (a pure function of location and
// sweep).
#include "device_common.h"
#include "pdit_internal.h"
#include "sweep_common.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int32_t kBig = (1 << 30) - 1;  // excluded candidates (|dE| < 2^30 is guaranteed)
constexpr uint32_t kOne = kWeightOne;    // weight of the row minimum

typedef short short2v __attribute__((ext_vector_type(2)));

// acc + x.lo * y.lo + x.hi * y.hi over signed 16-bit halves, modulo 2^32
__device__ __forceinline__ int32_t dot2(uint32_t x, uint32_t y, int32_t acc) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, x), __builtin_bit_cast(short2v, y),
                                  acc, false);
}

template <int NMAX>
struct TableSmem {
    static constexpr int PT = NMAX + 4;  // table row pitch (int32), rows 16-byte aligned
    static constexpr int PD = NMAX + 8;  // D and Fp row pitch (int16), rows 16-byte aligned
    int32_t T[NMAX * PT];                // T[l][s]; kBig on the diagonal and outside N x N
    int16_t Ds[NMAX * PD];               // D
    int16_t Fp[NMAX * PD];               // F[p,p]
    int32_t hd[NMAX];                    // H[x][x]
    int32_t pv[NMAX];                    // p(x)
    int32_t av[NMAX];                    // a_x of the exchange being applied
    int32_t cv2[NMAX];                   // 2 c_x
    int32_t hv[4][NMAX];                 // H'[r][x], H'[t][x], H'[x][r], H'[x][t]
    // per wave and pass: 0, or 2^30 | first swapping row << 16 | its choice
    __align__(16) int32_t summ[2][NMAX / 16 < 4 ? 4 : NMAX / 16];
    int64_t tie_sum[NMAX / 16];
};

// Runs one replica's sweeps with the whole workgroup (NMAX/16 waves).  REC:
// the job records choices and/or the energy trace.
template <int NMAX, bool ZD, bool EXACT, bool REC>
__device__ __forceinline__ void table_replica(const ReplicaJob &a, TableSmem<NMAX> &sm) {
    constexpr int WPR = NMAX / 16;         // waves per replica
    constexpr int NT = 64 * WPR;           // threads: 4 NMAX
    constexpr int K = NMAX / 4;            // candidates per lane in a speculative pass
    constexpr int CPL = (NMAX + 63) / 64;  // candidates per lane in a sequential update
    constexpr int PT = TableSmem<NMAX>::PT;
    constexpr int PD = TableSmem<NMAX>::PD;
    // CDF type: a lane's partial sum of at most 64 weights of 2^25 fits 32
    // bits; a row's total fits 32 bits only for N <= 64
    using CT = typename std::conditional<(NMAX <= 64), uint32_t, uint64_t>::type;
    int32_t *T = sm.T;
    int16_t *Ds = sm.Ds;
    int16_t *Fp = sm.Fp;
    int32_t *hd = sm.hd;
    int32_t *pv = sm.pv;
    int32_t *av = sm.av;
    int32_t *cv2 = sm.cv2;

    const int N = EXACT ? NMAX : a.N;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;

    // Eq. 3 for locations l, s from H[l][s], H[s][l], H[l][l], H[s][s] and the
    // D and Fp in LDS, modulo 2^32
    auto eq3 = [&](int l, int s, int32_t hls, int32_t hsl, int32_t hll, int32_t hss) -> int32_t {
        const uint32_t h = 2u * ((uint32_t)hls + (uint32_t)hsl - (uint32_t)hll - (uint32_t)hss);
        const int32_t dls = Ds[l * PD + s], fls = Fp[l * PD + s];
        uint32_t corr;
        if (ZD) {
            corr = 4u * (uint32_t)(dls * fls);
        } else {
            const int32_t dd = (int32_t)Ds[l * PD + l] + (int32_t)Ds[s * PD + s] - 2 * dls;
            const int32_t ff = (int32_t)Fp[l * PD + l] + (int32_t)Fp[s * PD + s] - 2 * fls;
            corr = (uint32_t)dd * (uint32_t)ff;
        }
        return (int32_t)(h + corr);
    };

    // ---- stage p, D, F[p,p], diag(H) and the table (zero / kBig outside N) ----
    for (int e = tid; e < NMAX; e += NT) pv[e] = e < N ? a.perm[e] : 0;
    for (int e = tid; e < NMAX * PD; e += NT) {
        const int i = e / PD, k = e % PD;
        Ds[e] = (int16_t)((i < N && k < N) ? a.D[(int64_t)i * N + k] : 0);
    }
    const int32_t *Hg = (const int32_t *)a.H;
    for (int e = tid; e < NMAX; e += NT) hd[e] = e < N ? Hg[(int64_t)e * N + e] : 0;
    __syncthreads();
    for (int e = tid; e < NMAX * PD; e += NT) {
        const int i = e / PD, k = e % PD;
        Fp[e] = (int16_t)((i < N && k < N) ? a.F[(int64_t)pv[i] * N + pv[k]] : 0);
    }
    __syncthreads();
    for (int e = tid; e < NMAX * PT; e += NT) {
        const int l = e / PT, s = e % PT;
        int32_t v = kBig;
        if (l < N && s < N && l != s)
            v = eq3(l, s, Hg[(int64_t)l * N + s], Hg[(int64_t)s * N + l], hd[l], hd[s]);
        T[e] = v;
    }
    __syncthreads();

    int64_t E = *a.E;
    int64_t E_best = *a.E_best;
    int64_t n_acc = 0, n_tie = 0;
    int parity = 0;
    bool seq_mode = false;

    // speculative layout: this lane's location and candidate quarter
    const int rl = lane >> 2, cq = lane & 3;
    const int rr = 16 * wv + rl;

    // ---- apply the exchange of locations r and t; every thread calls it ----
    auto apply_swap = [&](int r, int t, int32_t dE) {
        E += dE;
        ++n_acc;
        // (1) a and 2c from the flows before the exchange.  Nothing writes D
        // or Fp before barrier (2), and av / cv2 were last read before the
        // previous exchange's barrier (3).
        for (int x = tid; x < NMAX; x += NT) {
            const bool in = x < N;
            av[x] = in ? (int32_t)Ds[x * PD + r] - (int32_t)Ds[x * PD + t] : 0;
            cv2[x] = in ? 2 * ((int32_t)Fp[x * PD + t] - (int32_t)Fp[x * PD + r]) : 0;
        }
        __syncthreads();  // also: every read of the table for this update is done
        // (2) every table entry off rows/columns r, t (those are rewritten in
        // (4)); wave 0 exchanges rows and columns r, t of Fp and p(r), p(t)
        if (rr < N) {
            const int32_t al = av[rr], cl2 = cv2[rr];
            int32_t *row = T + rr * PT + cq * K;
#pragma unroll
            for (int j = 0; j < K; j += 4) {
                int4 x = *reinterpret_cast<int4 *>(row + j);
                const int4 as = *reinterpret_cast<const int4 *>(av + cq * K + j);
                const int4 cs = *reinterpret_cast<const int4 *>(cv2 + cq * K + j);
                const int s0 = cq * K + j;
                const int32_t n0 = __mul24(as.x - al, cl2 - cs.x) + x.x;
                const int32_t n1 = __mul24(as.y - al, cl2 - cs.y) + x.y;
                const int32_t n2 = __mul24(as.z - al, cl2 - cs.z) + x.z;
                const int32_t n3 = __mul24(as.w - al, cl2 - cs.w) + x.w;
                x.x = (EXACT || s0 + 0 < N) ? n0 : x.x;
                x.y = (EXACT || s0 + 1 < N) ? n1 : x.y;
                x.z = (EXACT || s0 + 2 < N) ? n2 : x.z;
                x.w = (EXACT || s0 + 3 < N) ? n3 : x.w;
                *reinterpret_cast<int4 *>(row + j) = x;
            }
        }
        if (wv == 0) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = lane + 64 * c;
                if (k < N) {
                    const int16_t fr = Fp[r * PD + k], ft = Fp[t * PD + k];
                    Fp[r * PD + k] = ft;
                    Fp[t * PD + k] = fr;
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = lane + 64 * c;
                if (k < N) {
                    const int16_t cr = Fp[k * PD + r], ct = Fp[k * PD + t];
                    Fp[k * PD + r] = ct;
                    Fp[k * PD + t] = cr;
                }
            }
            if (lane == 0) {
                const int32_t fa = pv[r], fb = pv[t];
                pv[r] = fb;
                pv[t] = fa;
            }
        }
        __syncthreads();
        // (3) the four H' vectors, one (vector, x) per thread, and diag(H')
        // off r, t
        {
            const int vec = tid / NMAX, x = tid % NMAX;
            if (x < N) {
                const int16_t *pl = (vec < 2 ? Fp : Ds) + x * PD;
                const int16_t *pu = vec == 0 ? Ds + r * PD
                                  : vec == 1 ? Ds + t * PD
                                  : vec == 2 ? Fp + r * PD
                                             : Fp + t * PD;
                int32_t acc = 0;
#pragma unroll
                for (int k = 0; k < NMAX; k += 8) {
                    const uint4 xl = *reinterpret_cast<const uint4 *>(pl + k);
                    const uint4 xu = *reinterpret_cast<const uint4 *>(pu + k);
                    acc = dot2(xl.x, xu.x, acc);
                    acc = dot2(xl.y, xu.y, acc);
                    acc = dot2(xl.z, xu.z, acc);
                    acc = dot2(xl.w, xu.w, acc);
                }
                sm.hv[vec][x] = acc;
            }
            if (tid < N && tid != r && tid != t)
                hd[tid] = (int32_t)((uint32_t)hd[tid] + (uint32_t)av[tid] * (uint32_t)(cv2[tid] >> 1));
        }
        __syncthreads();
        // (4) rows and columns r and t from Eq. 3
        if (tid < 2 * NMAX) {
            const int vr = tid < NMAX ? 0 : 1;
            const int w = vr == 0 ? r : t;
            const int x = tid % NMAX;
            if (x < N) {
                const int32_t hww = sm.hv[vr][w];
                const int32_t hxx = x == r ? sm.hv[0][r] : x == t ? sm.hv[1][t] : hd[x];
                const int32_t v =
                    x == w ? kBig : eq3(w, x, sm.hv[vr][x], sm.hv[vr + 2][x], hww, hxx);
                T[w * PT + x] = v;
                T[x * PT + w] = v;
            }
        } else if (tid == 2 * NMAX) {
            hd[r] = sm.hv[0][r];
            hd[t] = sm.hv[1][t];
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

    // beta and the zero-weight distance of 64 sweeps at a time, lane i
    // holding sweep t0 + i
    float bcache = 0.0f;
    int32_t dcache = 0;
    for (int64_t t = 0; t < a.T; ++t) {
        const int slot = (int)(t & 63);
        if (slot == 0) {
            const int64_t tt = t + lane < a.T ? t + lane : a.T - 1;
            bcache = a.beta[tt];
            dcache = zero_weight_distance(bcache);
        }
        const float beta = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bcache), slot));
        const int32_t dthr = __builtin_amdgcn_readlane(dcache, slot);
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int64_t acc_before = n_acc;
        int32_t *ch = (REC && a.choices) ? a.choices + t * N : nullptr;

        if (!seq_mode) {
            // ============ speculative rows: 16 locations per wave, 4 lanes each ============
            bool have_u = false;  // wave-uniform
            uint32_t u24 = 0;
            int pos = 0;
            while (pos < N) {
                const bool rowv = rr < N && rr >= pos;
                int sel = rr;
                bool tie = false;
                if (__ballot(rowv)) {
                    int32_t dl[K];
                    const int32_t *row = T + rr * PT + cq * K;
#pragma unroll
                    for (int j = 0; j < K; j += 4) {
                        const int4 x = *reinterpret_cast<const int4 *>(row + j);
                        dl[j] = x.x;
                        dl[j + 1] = x.y;
                        dl[j + 2] = x.z;
                        dl[j + 3] = x.w;
                    }
                    // best move of the row (the diagonal holds the sentinel)
                    int32_t m = kBig;
#pragma unroll
                    for (int j = 0; j < K; j += 2) m = min(m, min(dl[j], dl[j + 1]));
                    m = min(m, quad<kQuadXor1>(m));
                    m = min(m, quad<kQuadXor2>(m));
                    const bool stays = m >= dthr;
                    if (__ballot(rowv && !stays)) {
                        if (!have_u) {
                            // kept inside the branch: the uniform is only
                            // evaluated by passes that draw
                            uint32_t row = (uint32_t)rr;
                            asm volatile("" : "+v"(row));
                            u24 = uniform24(a.seed, row, g, a.rep, a.inst);
                            have_u = true;
                        }
                        const int js = rr - cq * K;  // this lane's slot of the stay, if any
                        const int32_t mn = min(m, 0);
                        // weights: d = 0 -> 2^25; 0 < d < dthr -> expf; d >= dthr -> 0
                        uint32_t ql[K];
                        uint32_t Zc = 0;
                        int am = -1;
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            const int32_t d = (j == js ? 0 : dl[j]) - mn;
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
                    }
                }
                const bool swaps = rowv && sel != rr;
                // this wave's first swapping row and its choice, one word per wave
                const uint64_t swm = __ballot(swaps);
                int32_t word = 0;
                if (swm) {
                    const int fl = __ffsll((unsigned long long)swm) - 1;  // lane 4 rl + cq
                    const int32_t sv = __builtin_amdgcn_readlane(sel, fl);
                    word = (int32_t)(0x40000000u | ((uint32_t)(16 * wv + (fl >> 2)) << 16) |
                                     (uint32_t)sv);
                }
                if (lane == 0) sm.summ[parity][wv] = word;
                __syncthreads();
                // the first swapping row of the pass, from the waves in order
                int last = N - 1, s_last = 0;
                bool found = false;
#pragma unroll
                for (int w = 0; w < WPR; ++w) {
                    const int32_t x = __builtin_amdgcn_readfirstlane(sm.summ[parity][w]);
                    if (!found && x != 0) {
                        found = true;
                        last = (x >> 16) & 0x3fff;
                        s_last = x & 0xffff;
                    }
                }
                // rows pos..last are committed: each wave counts (and
                // records) its own
                const bool committed = rowv && rr <= last;
                n_tie += __popcll(__ballot(committed && tie && cq == 0));
                if (REC && ch && committed && cq == 0) ch[rr] = sel;
                if (found) apply_swap(last, s_last, T[last * PT + s_last]);
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
                int32_t v[CPL];
                uint32_t q[CPL];
                int32_t lmin = kBig;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int ls = lane + 64 * c;
                    v[c] = ls < N ? (ls == r ? 0 : T[r * PT + ls]) : kBig;
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
                if (REC && ch && tid == 0) ch[r] = s;
                if (s != r) apply_swap(r, s, vsel);
            }
        }
        seq_mode = (n_acc - acc_before) > a.seq_threshold;
        if (REC && a.E_trace && tid == 0) a.E_trace[t] = E;
    }

    if (lane == 0) sm.tie_sum[wv] = n_tie;
    __syncthreads();
    if (wv == 0) {
        if (lane == 0) {
#pragma unroll
            for (int w = 1; w < WPR; ++w) n_tie += sm.tie_sum[w];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (lane + 64 * c < N) a.perm[lane + 64 * c] = pv[lane + 64 * c];
        if (lane == 0) {
            *a.E = E;
            *a.E_best = E_best;
            a.counters[0] = (int64_t)N * a.T;
            a.counters[1] = n_acc;
            a.counters[2] = n_tie;
        }
    }
}

// Waves per SIMD: four replicas of N <= 64 share a CU (one wave per SIMD
// each at N = 64), one replica of N = 128 fills a CU's LDS.
template <int NMAX>
constexpr int table_waves_per_eu() {
    return NMAX <= 64 ? 4 : 2;
}

// One replica per workgroup (single-instance runs).
template <int NMAX, bool ZD, bool EXACT, bool REC>
__global__ void __launch_bounds__(4 * NMAX)
__attribute__((amdgpu_waves_per_eu(table_waves_per_eu<NMAX>())))
sweep_table_kernel(SweepArgs a) {
    __shared__ __align__(16) TableSmem<NMAX> sm;
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
    j.beta = a.beta;
    j.T = a.T;
    j.seed = a.seed;
    j.sweep_offset = a.sweep_offset;
    j.rep = (uint32_t)rep;
    j.inst = a.inst_id;
    j.choices = a.choices ? a.choices + rep * a.T * a.N : nullptr;
    j.E_trace = a.E_trace ? a.E_trace + rep * a.T : nullptr;
    j.seq_threshold = a.seq_threshold;
    j.zero_diag = ZD;
    table_replica<NMAX, ZD, EXACT, REC>(j, sm);
}

// Persistent: each workgroup takes (instance, replica) items from a queue
// until it is exhausted; items come largest N first.  Every workgroup
// reaches the exit: the queue only grows, so each one reads an item index
// >= n_items after at most n_items increments.
template <int NMAX, bool ZD>
__global__ void __launch_bounds__(4 * NMAX)
__attribute__((amdgpu_waves_per_eu(table_waves_per_eu<NMAX>())))
sweep_table_persistent(BatchArgs b) {
    __shared__ __align__(16) TableSmem<NMAX> sm;
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= b.n_items) break;
        table_replica<NMAX, ZD, false, false>(batch_job(b, item, sizeof(int32_t)), sm);
        __syncthreads();
    }
}

template <int NMAX, bool ZD, bool EXACT>
hipError_t launch_one(hipStream_t s, const SweepArgs &a) {
    if (a.choices || a.E_trace)
        sweep_table_kernel<NMAX, ZD, EXACT, true><<<a.R, 4 * NMAX, 0, s>>>(a);
    else
        sweep_table_kernel<NMAX, ZD, EXACT, false><<<a.R, 4 * NMAX, 0, s>>>(a);
    return hipGetLastError();
}

template <int NMAX>
hipError_t launch_nmax(hipStream_t s, const SweepArgs &a) {
    const bool exact = a.N == NMAX;
    if (a.zero_diag)
        return exact ? launch_one<NMAX, true, true>(s, a) : launch_one<NMAX, true, false>(s, a);
    return exact ? launch_one<NMAX, false, true>(s, a) : launch_one<NMAX, false, false>(s, a);
}

template <int NMAX>
hipError_t launch_persistent_nmax(hipStream_t s, bool zd, const BatchArgs &b, int grid) {
    if (zd)
        sweep_table_persistent<NMAX, true><<<grid, 4 * NMAX, 0, s>>>(b);
    else
        sweep_table_persistent<NMAX, false><<<grid, 4 * NMAX, 0, s>>>(b);
    return hipGetLastError();
}

template <int NMAX>
int persistent_blocks_per_cu() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, sweep_table_persistent<NMAX, true>, 4 * NMAX, 0);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_sweep_table(hipStream_t s, int nmax, const SweepArgs &a) {
    switch (nmax) {
        case 16: return launch_nmax<16>(s, a);
        case 32: return launch_nmax<32>(s, a);
        case 64: return launch_nmax<64>(s, a);
        case 128: return launch_nmax<128>(s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_table_persistent(hipStream_t s, int nmax, bool zd, const BatchArgs &b,
                                         int grid) {
    switch (nmax) {
        case 16: return launch_persistent_nmax<16>(s, zd, b, grid);
        case 32: return launch_persistent_nmax<32>(s, zd, b, grid);
        case 64: return launch_persistent_nmax<64>(s, zd, b, grid);
        case 128: return launch_persistent_nmax<128>(s, zd, b, grid);
        default: return hipErrorInvalidValue;
    }
}

int table_blocks_per_cu(int nmax) {
    switch (nmax) {
        case 16: return persistent_blocks_per_cu<16>();
        case 32: return persistent_blocks_per_cu<32>();
        case 64: return persistent_blocks_per_cu<64>();
        case 128: return persistent_blocks_per_cu<128>();
        default: return 1;
    }
}

}  // namespace pdit
