// cupim_large.hip -- GPU-CUPIM (concurrent p-dit updates; Results, "GPU
// Implementations"; Methods, "GPU-CUPIM Algorithm") where the snapshot does
// not fit a CU: N up to PDIT_NMAX and entries of D and F beyond 8 bits.
//
// The iteration is the one of cupim.hip, with the replica state in device
// memory and one kernel per step:
//   draw     every location r draws from the snapshot (Eq. 3 with I = -2H,
//            Eq. 5): one wave per location, dE_rs = 2 (S_rs - H_rr - H_ss)
//            + (D_rr + D_ss - 2 D_rs)(F_aa + F_bb - 2 F_ab) with S = H + H^T,
//            a = p(r), b = p(s), int64 throughout; the integer Gibbs weights,
//            their exact 64-bit CDF in location order and the Philox uniform
//            of (r, g, replica, instance), as in every sweep kernel;
//   resolve  the proposal of r to exchange with s != r has the key
//            (snapshot dE, r), smaller first, and wins when it holds the
//            smallest key at both of its locations; the winners, disjoint,
//            exchange their facilities together;
//   refresh  H = D F[p,p] recomputed exactly (the H recompute step, any of
//            its modes), E = tr H, then S = H + H^T and diag H (this file),
//            and the best state.
// An iteration without winners recomputes the same snapshot, so the result
// equals the on-chip kernel's (which skips that refresh).
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

constexpr int kKMax = PDIT_NMAX / 64;  // candidates per lane of a location's wave

// exact signed/unsigned 64-bit wave reductions and scans (lane order)
__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// inclusive prefix sum over the lanes
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t w = __shfl_up(v, o);
        if (lane >= o) v += w;
    }
    return v;
}

// One wave per location r of one replica: the draw from the snapshot.
template <bool ZD>
__global__ void __launch_bounds__(256) cupim_draw_kernel(CupimLargeArgs c, int64_t t,
                                                         uint32_t g) {
    const int N = c.N;
    const float beta = c.beta[t];
    const int64_t dthr = zero_weight_distance64(beta);
    const int lane = threadIdx.x & 63;
    const int locs = (N + 3) / 4;  // blocks per replica, four locations each
    const int64_t rep = blockIdx.x / locs;
    const int r = (int)(blockIdx.x % locs) * 4 + (threadIdx.x >> 6);
    if (r >= N) return;
    const int32_t *p = c.perm + rep * N;
    const int64_t *Srow = c.S + (rep * N + r) * (int64_t)N;
    const int64_t *hd = c.hd + rep * N;
    const int a = p[r];
    const int64_t hrr = hd[r];
    const int64_t drr = ZD ? 0 : c.D[(int64_t)r * N + r];
    const int64_t faa = ZD ? 0 : c.F[(int64_t)a * N + a];
    // lane l holds the candidates s = l K .. l K + K - 1 (K = ceil(N / 64))
    const int K = (N + 63) / 64;
    int64_t dl[kKMax];
    int64_t m = INT64_MAX;
#pragma unroll
    for (int j = 0; j < kKMax; ++j) {
        const int s = lane * K + j;
        dl[j] = INT64_MAX;
        if (j < K && s < N && s != r) {
            const int b = p[s];
            const int64_t drs = c.D[(int64_t)r * N + s];
            const int64_t fab = c.F[(int64_t)a * N + b];
            int64_t corr;
            if (ZD) {
                corr = 4 * drs * fab;
            } else {
                const int64_t dss = c.D[(int64_t)s * N + s];
                const int64_t fbb = c.F[(int64_t)b * N + b];
                corr = (drr + dss - 2 * drs) * (faa + fbb - 2 * fab);
            }
            dl[j] = 2 * (Srow[s] - hrr - hd[s]) + corr;
            m = dl[j] < m ? dl[j] : m;
        }
    }
    m = wave_min_i64(m);
    int sel = r, tie = 0;
    int64_t dsel = 0;
    if (m < dthr) {
        // weights of the distances to min(m, 0) (the stay's dE is 0)
        const int64_t mn = m < 0 ? m : 0;
        uint32_t q[kKMax];
        uint64_t lsum = 0;
#pragma unroll
        for (int j = 0; j < kKMax; ++j) {
            const int s = lane * K + j;
            q[j] = 0;
            if (j < K && s < N) {
                const int64_t d = (s == r ? 0 : dl[j]) - mn;
                q[j] = d == 0 ? kWeightOne : d < dthr ? gibbs_weight(beta, (float)d) : 0u;
            }
            lsum += q[j];
        }
        const uint64_t incl = wave_scan_u64(lsum, lane);
        const uint64_t Z = __shfl(incl, 63);
        const uint32_t u24 = uniform24(c.seed, (uint32_t)r, g, (uint32_t)rep, c.inst_id);
        // the first s with C_s 2^24 > u24 Z is the number of s with C_s <= thr;
        // a tie: some C_s with 0 < C_s < Z in (thr_lo, thr_hi]
        const uint64_t target = (uint64_t)u24 * Z;
        const uint64_t band = Z << 4;
        const uint64_t thr = target >> 24;
        const uint64_t thr_lo = target >= band ? (target - band) >> 24 : 0;
        uint64_t thr_hi = (target + band) >> 24;
        if (thr_hi > Z - 1) thr_hi = Z - 1;
        uint64_t C = incl - lsum;
        int n_sel = 0, n_band = 0;
#pragma unroll
        for (int j = 0; j < kKMax; ++j) {
            if (j < K) {
                C += q[j];
                n_sel += C <= thr;
                n_band += (C > thr_lo && C <= thr_hi) ? 1 : 0;
            }
        }
        sel = wave_sum_i32(n_sel);
        tie = Z != kWeightOne && wave_sum_i32(n_band) > 0;
        // dE of the drawn candidate, from the lane that holds it
        const int owner = sel / K, js = sel % K;
        int64_t mine = 0;
#pragma unroll
        for (int j = 0; j < kKMax; ++j)
            if (j == js) mine = dl[j];
        dsel = __shfl(mine, owner);
        if (sel == r) dsel = 0;
    }
    if (lane == 0) {
        c.sel[rep * N + r] = sel;
        c.dsel[rep * N + r] = dsel;
        c.tie[rep * N + r] = tie;
    }
}

// One block per replica: the conflict rule, the winners' exchanges and the
// counters of the iteration.
__global__ void __launch_bounds__(PDIT_NMAX) cupim_resolve_kernel(CupimLargeArgs c) {
    __shared__ unsigned long long key[PDIT_NMAX];
    __shared__ int nwin, nties;
    const int N = c.N;
    const int64_t rep = blockIdx.x;
    const int x = threadIdx.x;
    int32_t *p = c.perm + rep * N;
    if (x < N) key[x] = ~0ull;
    if (x == 0) {
        nwin = 0;
        nties = 0;
    }
    __syncthreads();
    int sel = x;
    unsigned long long mine = ~0ull;
    if (x < N) {
        sel = c.sel[rep * N + x];
        if (c.tie[rep * N + x]) atomicAdd(&nties, 1);
        if (sel != x) {
            // (dE, r) in one word: |dE| < 2^53 (checked by the host), r < 2^10
            const uint64_t d = (uint64_t)(c.dsel[rep * N + x] + ((int64_t)1 << 53));
            mine = (d << 10) | (uint64_t)x;
            atomicMin(&key[x], mine);
            atomicMin(&key[sel], mine);
        }
    }
    __syncthreads();
    const bool win = x < N && sel != x && key[x] == mine && key[sel] == mine;
    int32_t fa = 0, fb = 0;
    if (win) {
        fa = p[x];
        fb = p[sel];
        atomicAdd(&nwin, 1);
    }
    __syncthreads();
    // winners are disjoint: each writes its own two entries of p
    if (win) {
        p[x] = fb;
        p[sel] = fa;
    }
    if (x == 0) {
        int64_t *cnt = c.counters + 3 * rep;
        cnt[0] += N;
        cnt[1] += nwin;
        cnt[2] += nties;
    }
}

// S = H + H^T and diag H, 32 x 32 tiles of one replica through LDS.
template <typename HT>
__global__ void __launch_bounds__(256) cupim_sym_kernel(int N, int tiles, const HT *__restrict__ H,
                                                        int64_t *__restrict__ S,
                                                        int64_t *__restrict__ hd) {
    __shared__ int64_t t[32][33];
    const int64_t per = (int64_t)tiles * tiles;
    const int64_t rep = blockIdx.x / per;
    const int ti = (int)(blockIdx.x % per) / tiles, tk = (int)(blockIdx.x % per) % tiles;
    const HT *Hr = H + rep * N * (int64_t)N;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    // H[tk*32 + y][ti*32 + x] into t[y][x]
    for (int y = ty; y < 32; y += 8) {
        const int i = tk * 32 + y, k = ti * 32 + tx;
        t[y][tx] = (i < N && k < N) ? (int64_t)Hr[(int64_t)i * N + k] : 0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int i = ti * 32 + y, k = tk * 32 + tx;
        if (i < N && k < N) {
            const int64_t h = (int64_t)Hr[(int64_t)i * N + k];
            S[(rep * N + i) * (int64_t)N + k] = h + t[tx][y];   // + H[k][i]
            if (i == k) hd[rep * N + i] = h;
        }
    }
}

// The best state after an iteration: E_best and perm_best where E improved.
__global__ void __launch_bounds__(256) cupim_best_kernel(int N, const int32_t *__restrict__ perm,
                                                         const int64_t *__restrict__ E,
                                                         int64_t *__restrict__ E_best,
                                                         int32_t *__restrict__ perm_best) {
    const int64_t rep = blockIdx.x;
    if (!(E[rep] < E_best[rep])) return;
    for (int x = threadIdx.x; x < N; x += blockDim.x)
        perm_best[rep * N + x] = perm[rep * N + x];
    __syncthreads();
    if (threadIdx.x == 0) E_best[rep] = E[rep];
}

}  // namespace

hipError_t launch_cupim_large_draw(hipStream_t s, const CupimLargeArgs &c, int64_t t, uint32_t g) {
    const int64_t blocks = (int64_t)c.R * ((c.N + 3) / 4);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (c.zero_diag)
        cupim_draw_kernel<true><<<(unsigned)blocks, 256, 0, s>>>(c, t, g);
    else
        cupim_draw_kernel<false><<<(unsigned)blocks, 256, 0, s>>>(c, t, g);
    return hipGetLastError();
}

hipError_t launch_cupim_large_resolve(hipStream_t s, const CupimLargeArgs &c) {
    cupim_resolve_kernel<<<c.R, PDIT_NMAX, 0, s>>>(c);
    return hipGetLastError();
}

hipError_t launch_cupim_large_sym(hipStream_t s, int N, int R, const void *H, bool h64,
                                  int64_t *S, int64_t *hd) {
    const int tiles = (N + 31) / 32;
    const int64_t blocks = (int64_t)R * tiles * tiles;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (h64)
        cupim_sym_kernel<int64_t><<<(unsigned)blocks, 256, 0, s>>>(N, tiles, (const int64_t *)H, S, hd);
    else
        cupim_sym_kernel<int32_t><<<(unsigned)blocks, 256, 0, s>>>(N, tiles, (const int32_t *)H, S, hd);
    return hipGetLastError();
}

hipError_t launch_cupim_large_best(hipStream_t s, int N, int R, const int32_t *perm,
                                   const int64_t *E, int64_t *E_best, int32_t *perm_best) {
    cupim_best_kernel<<<R, 256, 0, s>>>(N, perm, E, E_best, perm_best);
    return hipGetLastError();
}

}  // namespace pdit
