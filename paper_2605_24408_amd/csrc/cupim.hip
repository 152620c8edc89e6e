// cupim.hip -- GPU-CUPIM: concurrent p-dit updates (Results, "GPU
// Implementations"; Methods, "GPU-CUPIM Algorithm").
//
// An iteration draws every location at once from a snapshot of the swap
// energy changes taken at its start (Eq. 3, Eq. 5), resolves overlapping
// proposals, applies all winners together and refreshes the snapshot.
// Conflict rule: location r proposing the exchange with s != r has the key
// (snapshot dE, r), smaller first (the larger energy decrease, then the lower
// proposing index); a proposal wins when it holds the smallest key at both
// of its locations; losers stay.  Winners are disjoint, so they commute.
//
// One workgroup (N/16 waves, 4 NMAX threads) per replica, N <= 128 and
// |D|, |F| <= 127.  LDS holds the snapshot table T[l][s] (int32; the stay's
// slot on the diagonal holds a sentinel), int8 copies of D, F and F[p,p],
// and p.  After an iteration with winners the table is rebuilt from
// S = D F[p,p] + F[p,p] D on 16x16x64 int8 MFMAs, each lane turning its own
// accumulator entries into table entries (Eq. 3 with I = -2H, H + H^T = S);
// E = trace H.  An iteration without winners leaves the snapshot valid and
// skips the refresh.
// Draws use the same integer weights, CDF and Philox stream as the
// sequential kernels: q = rint(expf(-fl32(beta fl32(d))) 2^25) of the
// distance d to the row minimum, the first s with C_s 2^24 > u24 Z, u24 from
// counter (r, g, replica, instance).
#include "device_common.h"
#include "pdit_internal.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int32_t kBig = (1 << 30) - 1;  // sentinel: the stay on the diagonal, rows/columns >= N
constexpr uint32_t kOne = kWeightOne;

typedef int v4i __attribute__((ext_vector_type(4)));

template <int NMAX>
struct CupimSmem {
    static constexpr int PT = NMAX + 4;               // table row pitch (int32)
    static constexpr int KP = NMAX < 64 ? 64 : NMAX;  // K extent of the int8 rows (MFMA K = 64)
    static constexpr int P8 = KP + 16;                // int8 row pitch (bytes), 16-byte aligned
    int32_t TH[NMAX * PT];                            // T (pitch padding never read)
    int8_t D8[NMAX * P8];                             // D, zero outside N x N
    int8_t Fp8[NMAX * P8];                            // F[p,p], zero outside N x N
    int8_t F8[NMAX * NMAX];                           // F
    int32_t pv[NMAX];                                 // p(x)
    int32_t hd[NMAX];                                 // H[x][x]
    unsigned long long key[NMAX];                     // smallest proposal key at each location
    int32_t nwin[NMAX / 16];                          // winners per wave
    long long esum;                                   // trace of H
};

// Rebuilds the snapshot from S = D F[p,p] + F[p,p] D = H + H^T (both
// operands symmetric): two 16x16x64 int8 MFMA products per output tile, so
// each lane holds S[l][s] for its own (l, s) and turns it into
// T[l][s] = 2 (S[l][s] - H[l][l] - H[s][s]) + correction (Eq. 3 with
// I = -2H) in registers; H[x][x] = S[x][x] / 2 comes from the diagonal
// tiles through LDS.  Returns E = trace H.  Every thread calls it; the table
// must not be read concurrently.
template <int NMAX, bool ZD>
__device__ __forceinline__ int64_t cupim_refresh(CupimSmem<NMAX> &sm, int N) {
    constexpr int PT = CupimSmem<NMAX>::PT;
    constexpr int P8 = CupimSmem<NMAX>::P8;
    constexpr int KC = CupimSmem<NMAX>::KP / 64;  // K chunks
    constexpr int NJ = NMAX / 16;                 // column tiles
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // wave wv owns rows 16 wv .. 16 wv + 15 and all NJ column tiles; element
    // e of tile j is S[16 wv + 4 (lane / 16) + e][16 j + lane % 16]
    v4i acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = v4i{0, 0, 0, 0};
    const int arow = 16 * wv + (lane & 15);
    const int kb = (lane >> 4) * 16;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const v4i ad = *reinterpret_cast<const v4i *>(&sm.D8[arow * P8 + kc * 64 + kb]);
        const v4i af = *reinterpret_cast<const v4i *>(&sm.Fp8[arow * P8 + kc * 64 + kb]);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int brow = (16 * j + (lane & 15)) * P8 + kc * 64 + kb;
            const v4i bf = *reinterpret_cast<const v4i *>(&sm.Fp8[brow]);
            const v4i bd = *reinterpret_cast<const v4i *>(&sm.D8[brow]);
            acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ad, bf, acc[j], 0, 0, 0);  // D Fp
            acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bd, acc[j], 0, 0, 0);  // Fp D
        }
    }
    const int r0 = 16 * wv + 4 * (lane >> 4);
    const int c0 = lane & 15;
    if (tid == 0) sm.esum = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        if (j == wv)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (r0 + e == 16 * j + c0) sm.hd[r0 + e] = r0 + e < N ? acc[j][e] / 2 : 0;
    __syncthreads();
    if (tid < N) atomicAdd(reinterpret_cast<unsigned long long *>(&sm.esum),
                           (unsigned long long)(long long)sm.hd[tid]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int l = r0 + e;
        const int32_t hl = sm.hd[l];
        int32_t dll = 0, fll = 0;
        if (!ZD) {
            dll = sm.D8[l * P8 + l];
            fll = sm.Fp8[l * P8 + l];
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int c = 16 * j + c0;
            int32_t v = kBig;
            if (l < N && c < N && l != c) {
                const uint32_t h = 2u * ((uint32_t)acc[j][e] - (uint32_t)hl - (uint32_t)sm.hd[c]);
                const int32_t dls = sm.D8[l * P8 + c], fls = sm.Fp8[l * P8 + c];
                uint32_t corr;
                if (ZD) {
                    corr = 4u * (uint32_t)(dls * fls);
                } else {
                    const int32_t dd = dll + (int32_t)sm.D8[c * P8 + c] - 2 * dls;
                    const int32_t ff = fll + (int32_t)sm.Fp8[c * P8 + c] - 2 * fls;
                    corr = (uint32_t)(dd * ff);
                }
                v = (int32_t)(h + corr);
            }
            sm.TH[l * PT + c] = v;
        }
    }
    __syncthreads();
    return (int64_t)sm.esum;
}

// F[p,p] from F and p, four bytes per store (zero beyond N).
template <int NMAX>
__device__ __forceinline__ void cupim_gather_fp(CupimSmem<NMAX> &sm, int N) {
    constexpr int P8 = CupimSmem<NMAX>::P8;
    constexpr int NT = 4 * NMAX;
    const int n4 = (N + 3) / 4;
    for (int e = threadIdx.x; e < N * n4; e += NT) {
        const int i = e / n4, c = 4 * (e % n4);
        const int8_t *frow = sm.F8 + sm.pv[i] * NMAX;
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (c + b < N) w |= (uint32_t)(uint8_t)frow[sm.pv[c + b]] << (8 * b);
        *reinterpret_cast<uint32_t *>(&sm.Fp8[i * P8 + c]) = w;
    }
}

// One replica's run: T iterations of the concurrent update.
template <int NMAX, bool ZD>
__device__ __forceinline__ void cupim_replica(const CupimJob &a, CupimSmem<NMAX> &sm) {
    constexpr int WPR = NMAX / 16;
    constexpr int NT = 64 * WPR;
    constexpr int K = NMAX / 4;  // candidates per lane of a row's quad
    constexpr int PT = CupimSmem<NMAX>::PT;
    constexpr int P8 = CupimSmem<NMAX>::P8;
    using CT = typename std::conditional<(NMAX <= 64), uint32_t, uint64_t>::type;
    const int N = a.N;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    // ---- stage D, F, p, F[p,p] (int8, zero padding) ----
    for (int x = tid; x < NMAX; x += NT) sm.pv[x] = x < N ? a.perm[x] : 0;
    for (int e = tid; e < NMAX * P8; e += NT) {
        const int i = e / P8, k = e % P8;
        sm.D8[e] = (int8_t)((i < N && k < N) ? a.D[i * N + k] : 0);
    }
    for (int e = tid; e < NMAX * NMAX; e += NT) {
        const int i = e / NMAX, k = e % NMAX;
        sm.F8[e] = (int8_t)((i < N && k < N) ? a.F[i * N + k] : 0);
    }
    for (int e = tid; e < NMAX * P8; e += NT) sm.Fp8[e] = 0;
    __syncthreads();
    cupim_gather_fp<NMAX>(sm, N);
    __syncthreads();
    int64_t E = cupim_refresh<NMAX, ZD>(sm, N);
    int64_t E_best = a.init_best ? E : *a.E_best;
    if (a.init_best && wv == 0)
        for (int x = lane; x < N; x += 64) a.perm_best[x] = sm.pv[x];

    int64_t n_acc = 0, n_tie = 0;
    const int rl = lane >> 2, cq = lane & 3;
    const int rr = 16 * wv + rl;  // this quad's location
    const bool rowv = rr < N;
    uint32_t u4 = 0, u4_g = 0;
    bool u4_valid = false;
    float bcache = 0.0f;
    int32_t dcache = 0;
    for (int64_t t = 0; t < a.T; ++t) {
        const int slot = (int)(t & 63);
        if (slot == 0) {
            const int64_t tt = t + lane < a.T ? t + lane : a.T - 1;
            bcache = a.beta[tt * a.beta_stride];
            dcache = zero_weight_distance(bcache);
        }
        const float beta = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bcache), slot));
        const int32_t dthr = __builtin_amdgcn_readlane(dcache, slot);
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);

        // ---- 1. every location draws from the snapshot (quad per row) ----
        int32_t dl[K];
        const int32_t *row = sm.TH + rr * PT + cq * K;
#pragma unroll
        for (int j = 0; j < K; j += 4) {
            const int4 x = rowv ? *reinterpret_cast<const int4 *>(row + j) : int4{kBig, kBig, kBig, kBig};
            dl[j] = x.x;
            dl[j + 1] = x.y;
            dl[j + 2] = x.z;
            dl[j + 3] = x.w;
        }
        int32_t m = kBig;
#pragma unroll
        for (int j = 0; j < K; j += 2) m = min(m, min(dl[j], dl[j + 1]));
        m = min(m, quad<kQuadXor1>(m));
        m = min(m, quad<kQuadXor2>(m));
        int sel = rr;
        bool tie = false;
        if (__ballot(rowv && m < dthr)) {
            // uniforms of four iterations at a time: lane cq of a quad holds
            // iteration u4_g + cq of its row
            if (!u4_valid || g - u4_g >= 4u) {
                uint32_t r32 = (uint32_t)rr;
                asm volatile("" : "+v"(r32));
                u4 = uniform24(a.seed, r32, g + (uint32_t)cq, a.rep, a.inst);
                u4_g = g;
                u4_valid = true;
            }
            const uint32_t k4 = g - u4_g;
            const uint32_t u24 = k4 == 0   ? quadu<0x00>(u4)
                                 : k4 == 1 ? quadu<0x55>(u4)
                                 : k4 == 2 ? quadu<0xAA>(u4)
                                           : quadu<0xFF>(u4);
            const int js = rr - cq * K;  // this lane's slot of the stay, if any
            const int32_t mn = min(m, 0);
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
                ql[j] = q;
                Zc += q;
            }
            const CT p1 = quadu<kQuadPrev1>((CT)Zc), p2 = quadu<kQuadPrev2>((CT)Zc),
                     p3 = quadu<kQuadPrev3>((CT)Zc);
            const CT off = (cq >= 1 ? p1 : 0) + (cq >= 2 ? p2 : 0) + (cq >= 3 ? p3 : 0);
            const CT Z = quadu<kQuadLast>((CT)(off + Zc));
            am = max(am, quad<kQuadXor1>(am));
            am = max(am, quad<kQuadXor2>(am));
            if (rowv && m < dthr) {
                sel = am;
                if (Z != kOne) {
                    // first s with C_s > thr is #{s : C_s <= thr}; a tie is a
                    // boundary thr_lo < C_s <= thr_hi (0 < C_s < Z)
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
                    sel = n_sel;
                    tie = n_band > 0;
                }
            }
        }
        n_tie += __popcll(__ballot(rowv && tie && cq == 0));

        // ---- 2. proposals and the conflict rule ----
        const bool prop = rowv && cq == 0 && sel != rr;
        unsigned long long mykey = ~0ull;
        if (prop) {
            const int32_t dE = sm.TH[rr * PT + sel];
            mykey = ((unsigned long long)(uint32_t)(dE + (1 << 30)) << 8) | (unsigned)rr;
        }
        for (int x = tid; x < NMAX; x += NT) sm.key[x] = ~0ull;
        __syncthreads();
        if (prop) {
            atomicMin(&sm.key[rr], mykey);
            atomicMin(&sm.key[sel], mykey);
        }
        __syncthreads();
        const bool win = prop && sm.key[rr] == mykey && sm.key[sel] == mykey;
        const int nw = __popcll(__ballot(win));
        if (lane == 0) sm.nwin[wv] = nw;
        // winners are disjoint: each exchanges its own two entries of p
        if (win) {
            const int32_t fa = sm.pv[rr], fb = sm.pv[sel];
            sm.pv[rr] = fb;
            sm.pv[sel] = fa;
        }
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int w = 0; w < WPR; ++w) total += __builtin_amdgcn_readfirstlane(sm.nwin[w]);
        if (total == 0) continue;  // the snapshot stays valid
        n_acc += total;

        // ---- 3. refresh: F[p,p], then S, E, T ----
        cupim_gather_fp<NMAX>(sm, N);
        __syncthreads();
        E = cupim_refresh<NMAX, ZD>(sm, N);
        if (E < E_best) {
            E_best = E;
            if (wv == 0)
                for (int x = lane; x < N; x += 64) a.perm_best[x] = sm.pv[x];
        }
    }

    // n_tie is per wave; gather through the winners' slots
    __syncthreads();
    if (lane == 0) sm.nwin[wv] = (int32_t)n_tie;
    __syncthreads();
    if (wv == 0) {
        for (int x = lane; x < N; x += 64) a.perm[x] = sm.pv[x];
        if (lane == 0) {
            int64_t ties = 0;
#pragma unroll
            for (int w = 0; w < WPR; ++w) ties += sm.nwin[w];
            *a.E = E;
            *a.E_best = E_best;
            const int64_t keep = a.accumulate ? 1 : 0;  // parallel-tempering periods add up
            a.counters[0] = keep * a.counters[0] + (int64_t)N * a.T;
            a.counters[1] = keep * a.counters[1] + n_acc;
            a.counters[2] = keep * a.counters[2] + ties;
        }
    }
}

template <int NMAX, bool ZD>
__global__ void __launch_bounds__(4 * NMAX) __attribute__((amdgpu_waves_per_eu(NMAX <= 64 ? 4 : 2)))
cupim_kernel(CupimArgs c) {
    __shared__ __align__(16) CupimSmem<NMAX> sm;
    const int64_t rep = blockIdx.x;
    CupimJob j;
    j.N = c.N;
    j.D = c.D;
    j.F = c.F;
    j.perm = c.perm + rep * c.N;
    j.E = c.E + rep;
    j.E_best = c.E_best + rep;
    j.perm_best = c.perm_best + rep * c.N;
    j.counters = c.counters + 3 * rep;
    // parallel tempering: every iteration at the rung's beta
    j.beta = c.slot ? c.beta + c.slot[rep] : c.beta;
    j.beta_stride = c.slot ? 0 : 1;
    j.accumulate = c.accumulate;
    j.T = c.T;
    j.seed = c.seed;
    j.sweep_offset = c.sweep_offset;
    j.rep = (uint32_t)rep;
    j.inst = c.inst_id;
    j.init_best = c.init_best;
    cupim_replica<NMAX, ZD>(j, sm);
}

template <int NMAX>
hipError_t launch_cupim_nmax(hipStream_t s, const CupimArgs &c) {
    if (c.zero_diag)
        cupim_kernel<NMAX, true><<<c.R, 4 * NMAX, 0, s>>>(c);
    else
        cupim_kernel<NMAX, false><<<c.R, 4 * NMAX, 0, s>>>(c);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cupim(hipStream_t s, int nmax, const CupimArgs &c) {
    switch (nmax) {
        case 16: return launch_cupim_nmax<16>(s, c);
        case 32: return launch_cupim_nmax<32>(s, c);
        case 64: return launch_cupim_nmax<64>(s, c);
        case 128: return launch_cupim_nmax<128>(s, c);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pdit
