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
    static constexpr int PT = table_pitch(NMAX);  // table row pitch (int32), rows 16-byte aligned
    static constexpr int PD = NMAX + 8;  // D and Fp row pitch (int16), rows 16-byte aligned
    int32_t T[NMAX * PT];                // T[l][s]; kBig on the diagonal and outside N x N
    int16_t Ds[NMAX * PD];               // D
    int16_t Fp[NMAX * PD];               // F[p,p]
    int32_t hd[NMAX];                    // H[x][x]
    int32_t pv[NMAX];                    // p(x)
    int32_t av[NMAX];                    // a_x of the exchange being applied
    int32_t cv2[NMAX];                   // 2 c_x
    int32_t hv[4][NMAX];                 // H'[r][x], H'[t][x], H'[x][r], H'[x][t]
    int32_t fnew[2][NMAX];               // rows r and t of Fp'
    int32_t fdn[NMAX];                   // diag Fp' (nonzero diagonals only)
    // per wave and pass: 0, or 2^30 | first swapping row << 16 | its choice
    __align__(16) int32_t summ[2][NMAX / 16 < 4 ? 4 : NMAX / 16];
    int64_t tie_sum[NMAX / 16];
};

// Per-workgroup state of fused parallel tempering: the set's energies and
// rung assignment (identical in every member), this replica's rung.
struct PtSmem {
    int64_t E[kPtMaxL];      // energy of each member at the end of the period
    int32_t who[kPtMaxL];    // member on each rung
    int32_t rung;            // this replica's rung
    int32_t since;           // passes since the top rung changed hands
    int32_t abort;           // a wait exceeded its bound
    uint64_t tper;           // wall clock at the start of the period
};

// Runs one replica's sweeps with the whole workgroup (NMAX/16 waves).  REC:
// the job records choices and/or the energy trace.  PTF: fused parallel
// tempering -- pf->n_periods periods of pf->period_sweeps sweeps at the
// beta of the replica's rung, each followed by a meeting of the set's
// members and the exchange pass (replica `rep` is member rep % L of set
// rep / L).
template <int NMAX, bool ZD, bool EXACT, bool REC, bool PTF = false>
__device__ __forceinline__ void table_replica(const ReplicaJob &a, TableSmem<NMAX> &sm,
                                              const PtFusedArgs *pf = nullptr,
                                              PtSmem *ps = nullptr, int64_t rep = 0) {
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
    if (PTF) {
        // the set's rung assignment and pass counter, read before this
        // replica's first arrival (no member writes them before the last)
        const int L = pf->L;
        const int64_t set = rep / L;
        if (tid < L) ps->who[pf->slot[set * L + tid]] = tid;
        if (tid == 0) {
            ps->since = pf->since_top[set];
            ps->rung = pf->slot[rep];
            ps->abort = 0;
            ps->tper = wall_clock64();
        }
    }
    for (int e = tid; e < NMAX; e += NT) pv[e] = e < N ? a.perm[e] : 0;
    for (int e = tid; e < NMAX * PD; e += NT) {
        const int i = e / PD, k = e % PD;
        Ds[e] = (int16_t)((i < N && k < N) ? a.D[(int64_t)i * N + k] : 0);
    }
    // a resumed replica (parallel-tempering periods) reloads its table and
    // diag H; otherwise both come from the recomputed H
    const bool resume = (a.flags & kLoadState) && a.tstate;
    const int32_t *Hg = (const int32_t *)a.H;
    if (resume) {
        for (int e = tid; e < NMAX * PT / 4; e += NT)
            reinterpret_cast<int4 *>(T)[e] = reinterpret_cast<const int4 *>(a.tstate)[e];
        for (int e = tid; e < NMAX; e += NT) hd[e] = a.tstate[NMAX * PT + e];
    } else {
        for (int e = tid; e < NMAX; e += NT) hd[e] = e < N ? Hg[(int64_t)e * N + e] : 0;
    }
    __syncthreads();
    for (int e = tid; e < NMAX * PD; e += NT) {
        const int i = e / PD, k = e % PD;
        Fp[e] = (int16_t)((i < N && k < N) ? a.F[(int64_t)pv[i] * N + pv[k]] : 0);
    }
    __syncthreads();
    if (!resume) {
        for (int e = tid; e < NMAX * PT; e += NT) {
            const int l = e / PT, s = e % PT;
            int32_t v = kBig;
            if (l < N && s < N && l != s)
                v = eq3(l, s, Hg[(int64_t)l * N + s], Hg[(int64_t)s * N + l], hd[l], hd[s]);
            T[e] = v;
        }
        __syncthreads();
    }

    int64_t E = *a.E;
    int64_t E_best = *a.E_best;
    int64_t n_acc = 0, n_tie = 0;
    int parity = 0;
    bool seq_mode = false;

    // speculative layout: this lane's location and candidate quarter
    const int rl = lane >> 2, cq = lane & 3;
    const int rr = 16 * wv + rl;

    // ---- apply the exchange of locations r and t; every thread calls it ----
    // Phase A reads only the state before the exchange (D, Fp, diag H) and
    // fills a, 2c, the four H' vectors, diag H' and the new rows r, t of Fp';
    // phase B rewrites the table, then Fp and p.  With pi the exchange of r
    // and t and Fp' = Fp[pi, pi]:
    //   H'[w][x] = dot(D[w], Fp[pi x]) + (D[w][t] - D[w][r])(Fp[pi x][r] - Fp[pi x][t])
    //   H'[x][w] = dot(D[x], Fp[pi w]) + (D[x][t] - D[x][r])(Fp[pi w][r] - Fp[pi w][t])
    auto apply_swap = [&](int r, int t, int32_t dE) {
        E += dE;
        ++n_acc;
        {
            // phase A: every LDS read first, then the arithmetic
            const int vec = tid / NMAX, x = tid % NMAX;  // one (vector, x) per thread
            const int px = x == r ? t : x == t ? r : x;
            const int urow = vec == 0 ? r : vec == 1 ? t : x;
            const int frow = vec < 2 ? px : vec == 2 ? t : r;
            const int16_t *pu = Ds + urow * PD;
            const int16_t *pf = Fp + frow * PD;
            // the two rows in chunks of at most 8 x 16 bytes (up to 64 VGPRs
            // in flight: all of a row at N <= 64)
            constexpr int NK = NMAX / 8;
            constexpr int CH = NK < 8 ? NK : 8;
            uint4 xu[CH], xf[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                xu[k] = *reinterpret_cast<const uint4 *>(pu + 8 * k);
                xf[k] = *reinterpret_cast<const uint4 *>(pf + 8 * k);
            }
            const int32_t du = (int32_t)pu[t] - (int32_t)pu[r];
            const int32_t df = (int32_t)pf[r] - (int32_t)pf[t];
            const int32_t ax = (int32_t)Ds[x * PD + r] - (int32_t)Ds[x * PD + t];
            const int32_t cx = (int32_t)Fp[x * PD + t] - (int32_t)Fp[x * PD + r];
            const int32_t fsrc = Fp[(vec == 0 ? t : r) * PD + px];  // Fp'[r][x] or Fp'[t][x]
            const int32_t fdg = ZD ? 0 : Fp[px * PD + px];        // Fp'[x][x]
            const int32_t hdx = hd[x];
            int32_t acc = 0;
#pragma unroll
            for (int k0 = 0; k0 < NK; k0 += CH) {
                if (k0 > 0) {
#pragma unroll
                    for (int k = 0; k < CH && k0 + k < NK; ++k) {
                        xu[k] = *reinterpret_cast<const uint4 *>(pu + 8 * (k0 + k));
                        xf[k] = *reinterpret_cast<const uint4 *>(pf + 8 * (k0 + k));
                    }
                }
#pragma unroll
                for (int k = 0; k < CH && k0 + k < NK; ++k) {
                    acc = dot2(xu[k].x, xf[k].x, acc);
                    acc = dot2(xu[k].y, xf[k].y, acc);
                    acc = dot2(xu[k].z, xf[k].z, acc);
                    acc = dot2(xu[k].w, xf[k].w, acc);
                }
            }
            const int32_t h = (int32_t)((uint32_t)acc + (uint32_t)du * (uint32_t)df);
            if (x < N) {
                sm.hv[vec][x] = h;
                if (vec == 0) {
                    av[x] = ax;
                    cv2[x] = 2 * cx;
                    sm.fnew[0][x] = fsrc;
                    if (x == r)
                        hd[x] = h;
                    else if (x != t)
                        hd[x] = (int32_t)((uint32_t)hdx + (uint32_t)ax * (uint32_t)cx);
                } else if (vec == 1) {
                    sm.fnew[1][x] = fsrc;
                    if (x == t) hd[x] = h;
                } else if (vec == 2 && !ZD) {
                    sm.fdn[x] = fdg;
                }
            } else if (vec == 0) {
                av[x] = 0;
                cv2[x] = 0;
            }
        }
        __syncthreads();  // also: every read of the table for this update is done
        // Phase B.  Entries off rows/columns r, t: T += (a_s - a_l)(2c_l - 2c_s).
        // Columns r and t from Eq. 3, written with their transposes (rows r and
        // t) by the owner of row l; T[r][t] = T[t][r] = -dE (the way back).
        if (rr < N && rr != r && rr != t) {
            const int l = rr;
            int32_t *row = T + l * PT + cq * K;
            int4 xs[K / 4], as4[K / 4], cs4[K / 4];
#pragma unroll
            for (int j = 0; j < K / 4; ++j) {
                xs[j] = *reinterpret_cast<const int4 *>(row + 4 * j);
                as4[j] = *reinterpret_cast<const int4 *>(av + cq * K + 4 * j);
                cs4[j] = *reinterpret_cast<const int4 *>(cv2 + cq * K + 4 * j);
            }
            const int32_t al = av[l], cl2 = cv2[l];
            // inputs of Eq. 3 for the entries (l, r) and (l, t)
            const int32_t sr = (int32_t)((uint32_t)sm.hv[2][l] + (uint32_t)sm.hv[0][l]);
            const int32_t st = (int32_t)((uint32_t)sm.hv[3][l] + (uint32_t)sm.hv[1][l]);
            const int32_t hdl = hd[l], hdr = hd[r], hdt = hd[t];
            const int32_t dlr = Ds[l * PD + r], dlt = Ds[l * PD + t];
            const int32_t flr = sm.fnew[0][l], flt = sm.fnew[1][l];
            int32_t dll = 0, drr = 0, dtt = 0, fll = 0, frr = 0, ftt = 0;
            if (!ZD) {
                dll = Ds[l * PD + l];
                drr = Ds[r * PD + r];
                dtt = Ds[t * PD + t];
                fll = sm.fdn[l];
                frr = sm.fdn[r];
                ftt = sm.fdn[t];
            }
#pragma unroll
            for (int j = 0; j < K / 4; ++j) {
                int4 x = xs[j];
                const int4 as = as4[j], cs = cs4[j];
                const int s0 = cq * K + 4 * j;
                const int32_t n0 = __mul24(as.x - al, cl2 - cs.x) + x.x;
                const int32_t n1 = __mul24(as.y - al, cl2 - cs.y) + x.y;
                const int32_t n2 = __mul24(as.z - al, cl2 - cs.z) + x.z;
                const int32_t n3 = __mul24(as.w - al, cl2 - cs.w) + x.w;
                x.x = (EXACT || s0 + 0 < N) ? n0 : x.x;
                x.y = (EXACT || s0 + 1 < N) ? n1 : x.y;
                x.z = (EXACT || s0 + 2 < N) ? n2 : x.z;
                x.w = (EXACT || s0 + 3 < N) ? n3 : x.w;
                *reinterpret_cast<int4 *>(row + 4 * j) = x;
            }
#pragma unroll
            for (int wi = 0; wi < 2; ++wi) {
                const int w = wi == 0 ? r : t;
                if (w >= cq * K && w < cq * K + K) {
                    const uint32_t h = 2u * ((uint32_t)(wi == 0 ? sr : st) - (uint32_t)hdl -
                                             (uint32_t)(wi == 0 ? hdr : hdt));
                    const int32_t dlw = wi == 0 ? dlr : dlt, flw = wi == 0 ? flr : flt;
                    uint32_t corr;
                    if (ZD) {
                        corr = 4u * (uint32_t)(dlw * flw);
                    } else {
                        const int32_t dd = dll + (wi == 0 ? drr : dtt) - 2 * dlw;
                        const int32_t ff = fll + (wi == 0 ? frr : ftt) - 2 * flw;
                        corr = (uint32_t)dd * (uint32_t)ff;
                    }
                    const int32_t v = (int32_t)(h + corr);
                    T[l * PT + w] = v;
                    T[w * PT + l] = v;
                }
            }
        }
        if (tid == 0) {
            T[r * PT + t] = -dE;
            T[t * PT + r] = -dE;
        }
        // Fp' rows and columns r, t from the buffer, one store per thread
        // across all waves (where a row and a column meet they carry the same
        // value: Fp' is symmetric); p(r) <-> p(t)
        for (int e = tid; e < 4 * N; e += NT) {
            const int kind = e / N, x = e - kind * N;
            const int16_t v = (int16_t)sm.fnew[kind >> 1][x];
            const int w = kind < 2 ? r : t;
            if (kind & 1)
                Fp[x * PD + w] = v;
            else
                Fp[w * PD + x] = v;
        }
        if (tid == 0) {
            const int32_t fa = pv[r], fb = pv[t];
            pv[r] = fb;
            pv[t] = fa;
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

    uint32_t u4 = 0, u4_g = 0;  // cached uniforms (wave-uniform validity)
    bool u4_valid = false;
    // beta and the zero-weight distance of 64 sweeps at a time, lane i
    // holding sweep t0 + i
    float bcache = 0.0f;
    int32_t dcache = 0;
    const int64_t n_per = PTF ? pf->n_periods : 1;
    const int64_t T_per = PTF ? pf->period_sweeps : a.T;
    const float *bsrc = a.beta;
    int64_t bstride = a.beta_stride;
    uint64_t t_done = 0;  // sweeps of the earlier periods
    for (int64_t per = 0; per < n_per; ++per, t_done += (uint64_t)T_per) {
    if (PTF) {
        bsrc = pf->ladder + __builtin_amdgcn_readfirstlane(ps->rung);
        bstride = 0;
    }
    for (int64_t t = 0; t < T_per; ++t) {
        const int slot = (int)(t & 63);
        if (slot == 0) {
            const int64_t tt = t + lane < T_per ? t + lane : T_per - 1;
            bcache = bsrc[tt * bstride];
            dcache = zero_weight_distance(bcache);
        }
        const float beta = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bcache), slot));
        const int32_t dthr = __builtin_amdgcn_readlane(dcache, slot);
        const uint32_t g = (uint32_t)(a.sweep_offset + t_done + (uint64_t)t);
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
                            // the uniforms of four sweeps at a time: lane cq of
                            // a quad holds sweep u4_g + cq of its row (kept
                            // inside the branch: only passes that draw need them)
                            if (!u4_valid || g - u4_g >= 4u) {
                                uint32_t row = (uint32_t)rr;
                                asm volatile("" : "+v"(row));
                                u4 = uniform24(a.seed, row, g + (uint32_t)cq, a.rep, a.inst);
                                u4_g = g;
                                u4_valid = true;
                            }
                            const uint32_t k = g - u4_g;
                            u24 = k == 0   ? quadu<0x00>(u4)
                                  : k == 1 ? quadu<0x55>(u4)
                                  : k == 2 ? quadu<0xAA>(u4)
                                           : quadu<0xFF>(u4);
                            have_u = true;
                        }
                        const int js = rr - cq * K;  // this lane's slot of the stay, if any
                        const int32_t mn = min(m, 0);
                        // candidates whose weight may be nonzero: d = v - mn < dthr,
                        // i.e. v < lim (the sentinel never qualifies); the stay
                        // (v = 0) by its own test
                        const int32_t lim = (int32_t)min((int64_t)mn + (int64_t)dthr, (int64_t)kBig);
                        uint32_t near = 0;
#pragma unroll
                        for (int j = 0; j < K; ++j) near |= (dl[j] < lim ? 1u : 0u) << j;
                        if (js >= 0 && js < K && 0 < lim) near |= 1u << js;
                        // sparse draw: up to S such candidates per lane, in order
                        constexpr int S = 4;
                        uint32_t qs[S];
                        int jx[S];
                        uint32_t rest = near;
                        uint32_t Zc = 0;
#pragma unroll
                        for (int it = 0; it < S; ++it) {
                            qs[it] = 0;
                            jx[it] = -1;
                            if (!__ballot(rest != 0)) continue;
                            const bool has = rest != 0;
                            const int j = has ? (int)__builtin_ctz(rest) : 0;
                            rest &= rest - 1;
                            const int32_t v = j == js ? 0 : T[rr * PT + cq * K + j];
                            const int32_t d = v - mn;
                            uint32_t q = (has && d == 0) ? kOne : 0u;
                            const bool need = has && d != 0;
                            if (__ballot(need)) {
                                if (need) q = gibbs_weight(beta, (float)d);
                            }
                            qs[it] = q;
                            jx[it] = has ? cq * K + j : -1;
                            Zc += q;
                        }
                        if (!__ballot(rest != 0)) {
                            // quarters before this one, the row total, and the
                            // candidate where the running sum crosses the
                            // threshold; a tie is a sum thr_lo < C <= thr_hi (the
                            // band around it, with 0 < C < Z)
                            const CT p1 = quadu<kQuadPrev1>(Zc), p2 = quadu<kQuadPrev2>(Zc),
                                     p3 = quadu<kQuadPrev3>(Zc);
                            const CT off = (cq >= 1 ? p1 : 0) + (cq >= 2 ? p2 : 0) + (cq >= 3 ? p3 : 0);
                            const CT Z = quadu<kQuadLast>((CT)(off + Zc));
                            const uint64_t target = (uint64_t)u24 * Z;
                            const uint64_t band = (uint64_t)Z << 4;
                            const CT thr = (CT)(target >> 24);
                            const CT thr_lo = target >= band ? (CT)((target - band) >> 24) : 0;
                            const CT thr_hi = (CT)min((target + band) >> 24, (uint64_t)(Z - 1));
                            const CT lo1 = thr_lo + 1;
                            const CT width = thr_hi >= lo1 ? thr_hi - thr_lo : 0;
                            CT C = off;
                            int selx = 0x7fffffff, n_band = 0;
#pragma unroll
                            for (int it = 0; it < S; ++it) {
                                const CT Cp = C;
                                C += qs[it];
                                if (jx[it] >= 0 && Cp <= thr && C > thr) selx = jx[it];
                                n_band += (jx[it] >= 0 && (C - lo1) < width) ? 1 : 0;
                            }
                            selx = min(selx, quad<kQuadXor1>(selx));
                            selx = min(selx, quad<kQuadXor2>(selx));
                            n_band += quad<kQuadXor1>(n_band);
                            n_band += quad<kQuadXor2>(n_band);
                            sel = selx;
                            tie = n_band > 0;
                        } else {
                            // more than S such candidates in some lane: every
                            // candidate's weight, d = 0 -> 2^25; 0 < d < dthr ->
                            // expf; d >= dthr -> 0
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
    if (PTF) {
        // ---- meet the set's other members, then the exchange pass ----
        // Each member publishes one 64-bit word, the period number (28
        // bits) over its energy (36 bits, two's complement; the table
        // classes bound |E| below 2^35), with a device-scope store, and
        // reads its set's words until every tag is this period's.  One
        // atomic word carries both the value and its validity, so no
        // cache-wide release or acquire is needed.  Words alternate between
        // two buffers by period parity: a member can be at most one period
        // ahead of the slowest reader of its set.
        const int L = pf->L;
        const int64_t set = rep / L;
        const int32_t m = (int32_t)(rep - set * L);
        uint64_t *pub = pf->Epub + (per & 1) * pf->R;
        if (wv == 0) {
            const uint64_t tag = (uint64_t)(per + 1) & kPtTagMask;
            const uint64_t mine = (tag << kPtEBits) | ((uint64_t)E & kPtEMask);
            if (lane == 0) __hip_atomic_store(pub + rep, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // every wait ends: the members are resident together and each
            // publishes after its own sweeps; the bound (1000 times this
            // member's period, at least pf->min_wait ticks) only guards
            // against a launch that broke that premise, and once one member
            // gave up every other waiter stops at its next poll
            const uint64_t w0 = wall_clock64();
            const uint64_t own = w0 - ps->tper;
            const uint64_t bound = own * 1000 > pf->min_wait ? own * 1000 : pf->min_wait;
            uint64_t w = mine;
            bool ready = lane >= L || lane == m;
            int32_t ab = 0;
            for (;;) {
                if (!ready) {
                    w = __hip_atomic_load(pub + set * L + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ready = (w >> kPtEBits) == tag;
                }
                if (__ballot(!ready) == 0) break;
                __builtin_amdgcn_s_sleep(2);
                const int32_t e = __hip_atomic_load(pf->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__builtin_amdgcn_readfirstlane(e) != 0 || wall_clock64() - w0 > bound) {
                    ab = 1;
                    break;
                }
            }
            if (lane < L) ps->E[lane] = (int64_t)(w << (64 - kPtEBits)) >> (64 - kPtEBits);
            if (lane == 0) {
                if (ab) __hip_atomic_store(pf->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ps->abort = ab;
            }
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(ps->abort)) break;
        if (tid == 0) {
            int32_t c = ps->since;
            pt_pass(L, ps->E, ps->who, c, pf->timeout);
            ps->since = c;
            for (int i = 0; i < L; ++i)
                if (ps->who[i] == m) ps->rung = i;
            ps->tper = wall_clock64();
        }
        __syncthreads();
    }
    }

    if (lane == 0) sm.tie_sum[wv] = n_tie;
    __syncthreads();
    if ((a.flags & kSaveState) && a.tstate) {
        for (int e = tid; e < NMAX * PT / 4; e += NT)
            reinterpret_cast<int4 *>(a.tstate)[e] = reinterpret_cast<const int4 *>(T)[e];
        for (int e = tid; e < NMAX; e += NT) a.tstate[NMAX * PT + e] = hd[e];
    }
    if (wv == 0) {
        if (lane == 0) {
#pragma unroll
            for (int w = 1; w < WPR; ++w) n_tie += sm.tie_sum[w];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (lane + 64 * c < N) a.perm[lane + 64 * c] = pv[lane + 64 * c];
        if (lane == 0) {
            if (PTF) {
                pf->slot[rep] = ps->rung;
                if (rep % pf->L == 0) pf->since_top[rep / pf->L] = ps->since;
            }
            *a.E = E;
            *a.E_best = E_best;
            const bool acc = (a.flags & kAccumCounters) != 0;
            a.counters[0] = (acc ? a.counters[0] : 0) + (int64_t)N * a.T;
            a.counters[1] = (acc ? a.counters[1] : 0) + n_acc;
            a.counters[2] = (acc ? a.counters[2] : 0) + n_tie;
        }
    }
}

// Waves per SIMD: four replicas of N <= 64 share a CU (one wave per SIMD
// each at N = 64), two of N <= 96 (six waves each), one of N = 128 fills a
// CU's LDS.
template <int NMAX>
constexpr int table_waves_per_eu() {
    return NMAX <= 64 ? 4 : NMAX <= 96 ? 3 : 2;
}

// Replica rep's job in a single-instance launch.
template <int NMAX, bool ZD>
__device__ __forceinline__ ReplicaJob table_job(const SweepArgs &a, int64_t rep) {
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
    j.tstate = a.tstate ? a.tstate + rep * table_state_words(NMAX) : nullptr;
    j.flags = a.flags;
    return j;
}

// One replica per workgroup (single-instance runs).
template <int NMAX, bool ZD, bool EXACT, bool REC>
__global__ void __launch_bounds__(4 * NMAX)
__attribute__((amdgpu_waves_per_eu(table_waves_per_eu<NMAX>())))
sweep_table_kernel(SweepArgs a) {
    __shared__ __align__(16) TableSmem<NMAX> sm;
    table_replica<NMAX, ZD, EXACT, REC>(table_job<NMAX, ZD>(a, blockIdx.x), sm);
}

// Fused parallel tempering: replicas rep0 .. rep0 + gridDim.x - 1 (whole
// sets), every period in one cooperative launch.
template <int NMAX, bool ZD, bool EXACT>
__global__ void __launch_bounds__(4 * NMAX)
__attribute__((amdgpu_waves_per_eu(table_waves_per_eu<NMAX>())))
sweep_table_pt(SweepArgs a, PtFusedArgs p, int64_t rep0) {
    __shared__ __align__(16) TableSmem<NMAX> sm;
    __shared__ PtSmem ps;
    const int64_t rep = rep0 + blockIdx.x;
    ReplicaJob j = table_job<NMAX, ZD>(a, rep);
    j.beta = p.ladder;
    j.beta_stride = 0;
    j.T = p.n_periods * p.period_sweeps;
    j.tstate = nullptr;
    j.flags = 0;
    table_replica<NMAX, ZD, EXACT, false, true>(j, sm, &p, &ps, rep);
}

// Persistent: each workgroup takes (instance, replica) items from a queue
// until it is exhausted; items come largest N first.  Every workgroup
// reaches the exit: the queue only grows, so each one reads an item index
// >= n_items after at most n_items increments.
template <int NMAX, bool ZD, bool REC>
__global__ void __launch_bounds__(4 * NMAX)
__attribute__((amdgpu_waves_per_eu(table_waves_per_eu<NMAX>())))
sweep_table_persistent(BatchArgs b) {
    __shared__ __align__(16) TableSmem<NMAX> sm;
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(item_sh);  // wave-uniform
        __syncthreads();
        if (item >= b.n_items) break;
        table_replica<NMAX, ZD, false, REC>(batch_job(b, item, sizeof(int32_t)), sm);
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
    if (b.rec) {
        if (zd)
            sweep_table_persistent<NMAX, true, true><<<grid, 4 * NMAX, 0, s>>>(b);
        else
            sweep_table_persistent<NMAX, false, true><<<grid, 4 * NMAX, 0, s>>>(b);
    } else if (zd) {
        sweep_table_persistent<NMAX, true, false><<<grid, 4 * NMAX, 0, s>>>(b);
    } else {
        sweep_table_persistent<NMAX, false, false><<<grid, 4 * NMAX, 0, s>>>(b);
    }
    return hipGetLastError();
}

// Cooperative launches of whole sets, as many per launch as fit the device
// at once (the members of a set must all be resident to meet).
template <int NMAX, bool ZD, bool EXACT>
hipError_t launch_pt_one(hipStream_t s, const SweepArgs &a, const PtFusedArgs &p, int num_cus) {
    const void *kern = reinterpret_cast<const void *>(&sweep_table_pt<NMAX, ZD, EXACT>);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_table_pt<NMAX, ZD, EXACT>,
                                                                4 * NMAX, 0);
    if (e != hipSuccess) return e;
    const int64_t sets_per_launch = (int64_t)per_cu * num_cus / p.L;
    if (sets_per_launch < 1) return hipErrorCooperativeLaunchTooLarge;
    const int64_t n_sets = a.R / p.L;
    for (int64_t s0 = 0; s0 < n_sets; s0 += sets_per_launch) {
        const int64_t ns = n_sets - s0 < sets_per_launch ? n_sets - s0 : sets_per_launch;
        SweepArgs aa = a;
        PtFusedArgs pp = p;
        int64_t rep0 = s0 * p.L;
        void *args[] = {&aa, &pp, &rep0};
        e = hipLaunchCooperativeKernel(kern, dim3((unsigned)(ns * p.L)), dim3(4 * NMAX), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int NMAX>
hipError_t launch_pt_nmax(hipStream_t s, const SweepArgs &a, const PtFusedArgs &p, int num_cus) {
    const bool exact = a.N == NMAX;
    if (a.zero_diag)
        return exact ? launch_pt_one<NMAX, true, true>(s, a, p, num_cus)
                     : launch_pt_one<NMAX, true, false>(s, a, p, num_cus);
    return exact ? launch_pt_one<NMAX, false, true>(s, a, p, num_cus)
                 : launch_pt_one<NMAX, false, false>(s, a, p, num_cus);
}

template <int NMAX>
int persistent_blocks_per_cu() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, sweep_table_persistent<NMAX, true, false>, 4 * NMAX, 0);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_sweep_table(hipStream_t s, int nmax, const SweepArgs &a) {
    switch (nmax) {
        case 16: return launch_nmax<16>(s, a);
        case 32: return launch_nmax<32>(s, a);
        case 64: return launch_nmax<64>(s, a);
        case 96: return launch_nmax<96>(s, a);
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
        case 96: return launch_persistent_nmax<96>(s, zd, b, grid);
        case 128: return launch_persistent_nmax<128>(s, zd, b, grid);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_table_pt(hipStream_t s, int nmax, const SweepArgs &args, const PtFusedArgs &p,
                                 int num_cus) {
    if (p.L < 1 || p.L > kPtMaxL || args.R % p.L) return hipErrorInvalidValue;
    SweepArgs a = args;
    if (a.seq_threshold < 0) a.seq_threshold = default_seq_threshold(nmax, a.N);
    switch (nmax) {
        case 16: return launch_pt_nmax<16>(s, a, p, num_cus);
        case 32: return launch_pt_nmax<32>(s, a, p, num_cus);
        case 64: return launch_pt_nmax<64>(s, a, p, num_cus);
        case 96: return launch_pt_nmax<96>(s, a, p, num_cus);
        case 128: return launch_pt_nmax<128>(s, a, p, num_cus);
        default: return hipErrorInvalidValue;
    }
}

int table_blocks_per_cu(int nmax) {
    switch (nmax) {
        case 16: return persistent_blocks_per_cu<16>();
        case 32: return persistent_blocks_per_cu<32>();
        case 64: return persistent_blocks_per_cu<64>();
        case 96: return persistent_blocks_per_cu<96>();
        case 128: return persistent_blocks_per_cu<128>();
        default: return 1;
    }
}

}  // namespace pdit
