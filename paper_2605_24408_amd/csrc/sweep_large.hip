// sweep_large.hip -- the p-dit sweep without a stored H (any N <= 512; the
// kernel of choice above the on-chip size classes).
//
// The update of location r needs, from H = D F[p,p] (Eq. 3 with I = -2H),
// only row r, column r and the diagonal.  D and F are symmetric, so
//   H[k][r] = sum_j D[j][k] F[p(r)][p(j)]                 (rows j of D)
//   H[r][k] = G[p(k)],  G[c] = sum_b F[b][c] D[r][q(b)]   (rows b of F;
//             q = p^-1 maps a facility to its location)
// and the diagonal is kept in LDS and moved in O(N) per accepted exchange:
// with u = D[.][t] - D[.][r] and v = F[p(r)][p(.)] - F[p(t)][p(.)] (the
// permuted flows before the exchange), the new H is H + u v^T with columns r
// and t exchanged, so H'[x][x] = H[x][x] + u[x] v[x] for x not in {r, t},
// H'[r][r] = H[r][t] + u[r] v[t] and H'[t][t] = H[t][r] + u[t] v[r].
// An update costs 2 N^2 multiply-adds over rows of D and F that every replica
// reads through the same L2 (one coalesced row per wave and row index); an
// accepted exchange costs O(N), where the plain kernel rewrites the N^2
// entries of H in device memory.  The dynamics are those of every other
// sweep kernel: locations 0..N-1 in order, Eq. 5 over the N candidates with
// the same integer weights, CDF and Philox stream.
//
// One workgroup of 512 threads (8 waves) per replica: thread k owns location
// k in the draw and column k of both products.  The products read padded
// copies of D and F whose rows N..N32+15 (N32 = N rounded up to 32) are
// zero, so blocks of 16 rows run in pairs without a tail and the next block
// is always loadable.  When |D|, |F| <= 32767 the copies hold int16 values in row
// pairs (one 32-bit word = rows 2i and 2i+1 of a column) and a block is 8
// word loads and 8 `v_dot2_i32_i16` per matrix, each exact in int32; else
// they are int32 rows with 24-bit (|D|, |F| < 2^23) or int64 products.
// Narrow instances (16 max|D| max|F| < 2^31) sum a block in int32 before the
// int64 total.
#include <algorithm>

#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

constexpr int kLargeThreads = 512;
constexpr int kLargeWaves = kLargeThreads / 64;
constexpr int kRowBlock = 16;  // rows per block of the two products

struct LargeSmem {
    alignas(16) int32_t f[kLargeNMax];    // F[p(r)][p(.)], zero beyond N
    alignas(16) int32_t dq[kLargeNMax];   // D[r][q(.)] (row r of D by facility), zero beyond N
    alignas(16) int16_t f16[kLargeNMax];  // the same as int16 (paired copies)
    alignas(16) int16_t dq16[kLargeNMax];
    int32_t p[kLargeNMax];                // facility at each location
    int32_t d[kLargeNMax];                // D[r][.]
    int32_t ddiag[kLargeNMax];            // D[x][x]
    int32_t fdiag[kLargeNMax];            // F[c][c]
    int64_t G[kLargeNMax];                // H[r][.] by facility
    int64_t hd[kLargeNMax];               // H[x][x]
    int64_t hcol[kLargeNMax];             // H[.][r]
    int32_t u[kLargeNMax], v[kLargeNMax];
    int64_t wmin[kLargeWaves];
    uint64_t wsum[kLargeWaves];
    int32_t wsel[kLargeWaves];
    int32_t tie;
};

typedef short short2v __attribute__((ext_vector_type(2)));

// acc + x.lo * y.lo + x.hi * y.hi over signed 16-bit halves (exact in int32
// for int16 operands when acc is 0, modulo 2^32 otherwise)
__device__ __forceinline__ int32_t dot2(uint32_t x, uint32_t y, int32_t acc) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, x), __builtin_bit_cast(short2v, y),
                                  acc, false);
}

// Buffer descriptor of a padded copy (raw buffer, GFX9 format word).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t copy_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// Words of one block per lane: 8 row pairs (int16 copies) or 16 rows (int32).
template <bool PAIRS>
struct Block {
    static constexpr int W = PAIRS ? kRowBlock / 2 : kRowBlock;
};

// The lane's words of a block: its offsets (column k of each word row of a
// block) stay in vector registers for the whole kernel and the block's row
// offset is wave-uniform, so a load is one instruction.
template <int W>
__device__ __forceinline__ void load_block(__amdgpu_buffer_rsrc_t rs, const uint32_t (&voff)[W],
                                           uint32_t soff, uint32_t (&x)[W]) {
#pragma unroll
    for (int u = 0; u < W; ++u) x[u] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff[u], soff, 0);
}

// Adds the products of one block (the lane's words x1, x2 of rows j0..j0+15)
// with entries j0..j0+15 of a and b to acc1, acc2.
template <bool PAIRS, bool NARROW>
__device__ __forceinline__ void block_products(const uint32_t (&x1)[Block<PAIRS>::W],
                                               const uint32_t (&x2)[Block<PAIRS>::W],
                                               const void *a, const void *b, int j0,
                                               int64_t &acc1, int64_t &acc2) {
    if constexpr (PAIRS) {
        // 16 int16 entries of a and b = 8 packed words each
        const uint4 *a4 = (const uint4 *)((const int16_t *)a + j0);
        const uint4 *b4 = (const uint4 *)((const int16_t *)b + j0);
        const uint4 aw0 = a4[0], aw1 = a4[1], bw0 = b4[0], bw1 = b4[1];
        const uint32_t aw[8] = {aw0.x, aw0.y, aw0.z, aw0.w, aw1.x, aw1.y, aw1.z, aw1.w};
        const uint32_t bw[8] = {bw0.x, bw0.y, bw0.z, bw0.w, bw1.x, bw1.y, bw1.z, bw1.w};
        if (NARROW) {
            int32_t s1 = 0, s2 = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s1 = dot2(x1[u], aw[u], s1);
                s2 = dot2(x2[u], bw[u], s2);
            }
            acc1 += s1;
            acc2 += s2;
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc1 += dot2(x1[u], aw[u], 0);
                acc2 += dot2(x2[u], bw[u], 0);
            }
        }
    } else {
        const int4 *a4 = (const int4 *)((const int32_t *)a + j0);
        const int4 *b4 = (const int4 *)((const int32_t *)b + j0);
        if (NARROW) {
            int32_t s1 = 0, s2 = 0;
#pragma unroll
            for (int q = 0; q < kRowBlock / 4; ++q) {
                const int4 av = a4[q], bv = b4[q];
                s1 = __mul24((int32_t)x1[4 * q + 0], av.x) + s1;
                s1 = __mul24((int32_t)x1[4 * q + 1], av.y) + s1;
                s1 = __mul24((int32_t)x1[4 * q + 2], av.z) + s1;
                s1 = __mul24((int32_t)x1[4 * q + 3], av.w) + s1;
                s2 = __mul24((int32_t)x2[4 * q + 0], bv.x) + s2;
                s2 = __mul24((int32_t)x2[4 * q + 1], bv.y) + s2;
                s2 = __mul24((int32_t)x2[4 * q + 2], bv.z) + s2;
                s2 = __mul24((int32_t)x2[4 * q + 3], bv.w) + s2;
            }
            acc1 += s1;
            acc2 += s2;
        } else {
#pragma unroll
            for (int q = 0; q < kRowBlock / 4; ++q) {
                const int4 av = a4[q], bv = b4[q];
                acc1 += (int64_t)(int32_t)x1[4 * q + 0] * av.x +
                        (int64_t)(int32_t)x1[4 * q + 1] * av.y +
                        (int64_t)(int32_t)x1[4 * q + 2] * av.z +
                        (int64_t)(int32_t)x1[4 * q + 3] * av.w;
                acc2 += (int64_t)(int32_t)x2[4 * q + 0] * bv.x +
                        (int64_t)(int32_t)x2[4 * q + 1] * bv.y +
                        (int64_t)(int32_t)x2[4 * q + 2] * bv.z +
                        (int64_t)(int32_t)x2[4 * q + 3] * bv.w;
            }
        }
    }
}

// hkr = sum_j M1[j][k] a[j], gk = sum_j M2[j][k] b[j] over rows 0..N32-1
// (N32 = N rounded up to 32; a, b: int16 vectors for paired copies, int32
// otherwise, zero beyond N).  Two blocks per iteration in alternating
// registers: the loads of one block are in flight while the other's
// products run, with no register copies that would wait for them.
template <bool PAIRS, bool NARROW>
__device__ __forceinline__ void two_products(__amdgpu_buffer_rsrc_t M1, __amdgpu_buffer_rsrc_t M2,
                                             const uint32_t (&voff)[Block<PAIRS>::W],
                                             uint32_t block_bytes, const void *a, const void *b,
                                             int N32, int64_t &hkr, int64_t &gk) {
    constexpr int W = Block<PAIRS>::W;
    uint32_t xa1[W], xa2[W], xb1[W], xb2[W];
    load_block<W>(M1, voff, 0, xa1);
    load_block<W>(M2, voff, 0, xa2);
    int64_t acc1 = 0, acc2 = 0;
    uint32_t soff = 0;
    for (int j0 = 0; j0 < N32; j0 += 2 * kRowBlock) {
        soff += block_bytes;
        load_block<W>(M1, voff, soff, xb1);
        load_block<W>(M2, voff, soff, xb2);
        block_products<PAIRS, NARROW>(xa1, xa2, a, b, j0, acc1, acc2);
        // the block after the last one is the zero pad block: always in range
        soff += block_bytes;
        load_block<W>(M1, voff, soff, xa1);
        load_block<W>(M2, voff, soff, xa2);
        block_products<PAIRS, NARROW>(xb1, xb2, a, b, j0 + kRowBlock, acc1, acc2);
    }
    hkr = acc1;
    gk = acc2;
}

template <bool PAIRS, bool NARROW, typename HT>
__global__ void __launch_bounds__(kLargeThreads) sweep_large_kernel(SweepArgs a, LargeCopies c) {
    __shared__ LargeSmem sm;
    const int N = a.N;
    const int N32 = (N + 2 * kRowBlock - 1) / (2 * kRowBlock) * (2 * kRowBlock);
    const int64_t rep = blockIdx.x;
    const int k = threadIdx.x, lane = k & 63, wv = k >> 6;
    const bool own = k < N;
    const int32_t *__restrict__ D = a.D;
    const int32_t *__restrict__ F = a.F;
    // word rows of a copy: row pairs (int16) or rows (int32), N words each
    constexpr int W = Block<PAIRS>::W;
    const uint32_t pitch = (uint32_t)N * 4;
    const uint32_t copy_bytes = (uint32_t)(N32 + kRowBlock) * (PAIRS ? 2 : 4) * N;
    const __amdgpu_buffer_rsrc_t Dc = copy_rsrc(c.D, copy_bytes);
    const __amdgpu_buffer_rsrc_t Fc = copy_rsrc(c.F, copy_bytes);
    // lanes past N read column 0 (results unused): every offset stays inside
    // the copy even for the prefetch of the zero block
    const uint32_t col = own ? (uint32_t)k : 0u;
    uint32_t voff[W];
#pragma unroll
    for (int u = 0; u < W; ++u) voff[u] = col * 4 + u * pitch;
    int32_t *perm = a.perm + rep * N;
    int32_t *pbest = a.perm_best + rep * N;
    HT *H0 = (HT *)a.H + rep * (int64_t)N * N;  // diag H of the initial p; kSaveState writes it back
    const float *beta_p = a.slot ? a.beta + a.slot[rep] : a.beta;
    const int64_t beta_stride = a.slot ? 0 : 1;

    if (own) {
        sm.p[k] = perm[k];
        sm.ddiag[k] = D[(int64_t)k * N + k];
        sm.fdiag[k] = F[(int64_t)k * N + k];
        sm.hd[k] = (int64_t)H0[(int64_t)k * N + k];
    } else {
        sm.f[k] = 0;  // the products' zero pad
        sm.dq[k] = 0;
        sm.f16[k] = 0;
        sm.dq16[k] = 0;
    }
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0, n_tie = 0;
    __syncthreads();

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = beta_p[t * beta_stride];
        const int64_t dthr = zero_weight_distance64(beta);
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        for (int r = 0; r < N; ++r) {
            const int pr = sm.p[r];
            // ---- row r of D, by location and by facility, and of the permuted flows ----
            if (own) {
                const int pk = sm.p[k];
                const int32_t drk = D[(int64_t)r * N + k];
                const int32_t fk = F[(int64_t)pr * N + pk];
                sm.d[k] = drk;
                sm.f[k] = fk;
                if (PAIRS) {
                    sm.dq16[pk] = (int16_t)drk;
                    sm.f16[k] = (int16_t)fk;
                } else {
                    sm.dq[pk] = drk;
                }
            }
            __syncthreads();
            // ---- column r of H (location k) and row r of H by facility (facility k) ----
            int64_t hkr = 0, gk = 0;
            if (wv * 64 < N) {  // waves with no location skip the products
                if constexpr (PAIRS)
                    two_products<true, NARROW>(Dc, Fc, voff, W * pitch, sm.f16, sm.dq16, N32, hkr,
                                               gk);
                else
                    two_products<false, NARROW>(Dc, Fc, voff, W * pitch, sm.f, sm.dq, N32, hkr,
                                                gk);
                if (own) {
                    sm.G[k] = gk;
                    sm.hcol[k] = hkr;
                }
            }
            __syncthreads();
            // ---- energy change of candidate k (Eq. 3) ----
            int64_t v = INT64_MAX;
            if (own) {
                const int64_t hrk = sm.G[sm.p[k]];
                const int64_t h = hrk + hkr - sm.hd[r] - sm.hd[k];
                const int64_t dd = (int64_t)sm.ddiag[r] + sm.ddiag[k] - 2 * (int64_t)sm.d[k];
                const int64_t ff = (int64_t)sm.fdiag[pr] + sm.fdiag[sm.p[k]] - 2 * (int64_t)sm.f[k];
                v = k == r ? 0 : 2 * h + dd * ff;
            }
            // ---- block minimum ----
            int64_t m = v;
            for (int off = 32; off > 0; off >>= 1) m = min(m, (int64_t)__shfl_xor(m, off));
            if (lane == 0) sm.wmin[wv] = m;
            __syncthreads();
            m = sm.wmin[0];
#pragma unroll
            for (int w = 1; w < kLargeWaves; ++w) m = min(m, sm.wmin[w]);
            // ---- integer weights, running sums, the draw (Eq. 5) ----
            uint32_t qk = 0;
            if (own) {
                const int64_t dk = v - m;
                qk = dk < dthr ? gibbs_weight(beta, (float)dk) : 0u;
            }
            const uint64_t cw = (uint64_t)wave_scan_u32(qk);  // at most 64 x 2^25 = 2^31
            if (lane == 63) sm.wsum[wv] = cw;
            __syncthreads();
            uint64_t off = 0, Z = 0;
#pragma unroll
            for (int w = 0; w < kLargeWaves; ++w) {
                const uint64_t x = sm.wsum[w];
                off += w < wv ? x : 0;
                Z += x;
            }
            const uint64_t C = off + cw;
            const uint32_t u24 = uniform24(a.seed, (uint32_t)r, g, (uint32_t)rep, a.inst_id);
            const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
            // the first candidate whose running sum exceeds the threshold
            const uint64_t hit = __ballot(own && C > thr);
            if (lane == 0) sm.wsel[wv] = hit ? 64 * wv + __ffsll((unsigned long long)hit) - 1 : 0x7fffffff;
            __syncthreads();
            int s = 0x7fffffff;
#pragma unroll
            for (int w = 0; w < kLargeWaves; ++w) s = min(s, sm.wsel[w]);
            if (s >= N) s = r;  // unreachable: location N-1 holds C = Z > thr
            if (k == s) sm.tie = is_tie(C - qk, C, Z, u24) ? 1 : 0;
            __syncthreads();
            n_tie += sm.tie;
            if (a.choices && k == 0) a.choices[(rep * a.T + t) * N + r] = s;
            if (s == r) continue;
            // ---- accepted exchange of r and s: E, diag H, p ----
            ++n_acc;
            const int ps = sm.p[s];
            if (own) {
                sm.u[k] = D[(int64_t)s * N + k] - sm.d[k];          // D[k][s] - D[k][r]
                sm.v[k] = sm.f[k] - F[(int64_t)ps * N + sm.p[k]];   // Fp[r][k] - Fp[s][k]
            }
            const int64_t h_rs = sm.G[ps], h_sr = sm.hcol[s];
            const int64_t dE = 2 * (h_rs + h_sr - sm.hd[r] - sm.hd[s]) +
                               ((int64_t)sm.ddiag[r] + sm.ddiag[s] - 2 * (int64_t)sm.d[s]) *
                                   ((int64_t)sm.fdiag[pr] + sm.fdiag[ps] - 2 * (int64_t)sm.f[s]);
            __syncthreads();
            E += dE;
            if (own) {
                const int64_t uk = sm.u[k];
                if (k == r)
                    sm.hd[k] = h_rs + uk * sm.v[s];
                else if (k == s)
                    sm.hd[k] = h_sr + uk * sm.v[r];
                else
                    sm.hd[k] += uk * sm.v[k];
            }
            if (k == 0) {
                sm.p[r] = ps;
                sm.p[s] = pr;
            }
            __syncthreads();
            if (E < E_best) {
                E_best = E;
                if (own) pbest[k] = sm.p[k];
            }
        }
        if (a.E_trace && k == 0) a.E_trace[rep * a.T + t] = E;
    }
    if (own) {
        perm[k] = sm.p[k];
        if (a.flags & kSaveState) H0[(int64_t)k * N + k] = (HT)sm.hd[k];
    }
    if (k == 0) {
        a.E[rep] = E;
        a.E_best[rep] = E_best;
        const bool acc = (a.flags & kAccumCounters) != 0;
        a.counters[3 * rep + 0] = (acc ? a.counters[3 * rep + 0] : 0) + (int64_t)N * a.T;
        a.counters[3 * rep + 1] = (acc ? a.counters[3 * rep + 1] : 0) + n_acc;
        a.counters[3 * rep + 2] = (acc ? a.counters[3 * rep + 2] : 0) + n_tie;
    }
}

// Padded int32 copies: rows 0..N-1 of D (then F), the other rows zero.
__global__ void large_copy32_kernel(int N, int rows, const int32_t *D, const int32_t *F,
                                    int32_t *Dc, int32_t *Fc) {
    const int64_t total = (int64_t)rows * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const bool in = e < (int64_t)N * N;
        Dc[e] = in ? D[e] : 0;
        Fc[e] = in ? F[e] : 0;
    }
}

// Paired int16 copies: word (i, k) = M[2i][k] | M[2i+1][k] << 16 (rows beyond
// N zero); the host checks |D|, |F| <= 32767.
__global__ void large_copy16_kernel(int N, int rows, const int32_t *D, const int32_t *F,
                                    uint32_t *Dc, uint32_t *Fc) {
    const int64_t total = (int64_t)(rows / 2) * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N, k = e - i * N;
        const int64_t lo = 2 * i * N + k, hi = lo + N;
        const bool in_lo = 2 * i < N, in_hi = 2 * i + 1 < N;
        Dc[e] = (uint32_t)(uint16_t)(in_lo ? D[lo] : 0) | (uint32_t)(uint16_t)(in_hi ? D[hi] : 0) << 16;
        Fc[e] = (uint32_t)(uint16_t)(in_lo ? F[lo] : 0) | (uint32_t)(uint16_t)(in_hi ? F[hi] : 0) << 16;
    }
}

}  // namespace

LargePlan large_plan(int N, const InstanceStats &st) {
    LargePlan pl;
    const int32_t mx = st.max_abs_d > st.max_abs_f ? st.max_abs_d : st.max_abs_f;
    pl.narrow = mx < (1 << 23) &&
                (int64_t)kRowBlock * st.max_abs_d * st.max_abs_f < ((int64_t)1 << 31);
    pl.elem = mx <= 32767 ? 2 : 4;
    pl.rows = (N + 2 * kRowBlock - 1) / (2 * kRowBlock) * (2 * kRowBlock) + kRowBlock;
    pl.bytes = 2 * (size_t)pl.rows * N * pl.elem;
    return pl;
}

hipError_t launch_large_copy(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                             const LargePlan &pl, void *buf, LargeCopies *out) {
    const size_t one = (size_t)pl.rows * N * pl.elem;
    out->D = buf;
    out->F = (char *)buf + one;
    const int64_t total = (int64_t)pl.rows * N;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 1024);
    if (pl.elem == 2)
        large_copy16_kernel<<<grid, 256, 0, s>>>(N, pl.rows, D, F, (uint32_t *)out->D,
                                                 (uint32_t *)out->F);
    else
        large_copy32_kernel<<<grid, 256, 0, s>>>(N, pl.rows, D, F, (int32_t *)out->D,
                                                 (int32_t *)out->F);
    return hipGetLastError();
}

hipError_t launch_sweep_large(hipStream_t s, const SweepArgs &a, bool h64, const LargePlan &pl,
                              const LargeCopies &c) {
    if (a.N > kLargeNMax || a.N < 2) return hipErrorInvalidValue;
#define PDIT_LARGE(PAIRS, NARROW)                                                               \
    do {                                                                                    \
        if (h64)                                                                            \
            sweep_large_kernel<PAIRS, NARROW, int64_t><<<a.R, kLargeThreads, 0, s>>>(a, c);     \
        else                                                                                \
            sweep_large_kernel<PAIRS, NARROW, int32_t><<<a.R, kLargeThreads, 0, s>>>(a, c);     \
    } while (0)
    if (pl.elem == 2 && pl.narrow)
        PDIT_LARGE(true, true);
    else if (pl.elem == 2)
        PDIT_LARGE(true, false);
    else if (pl.narrow)
        PDIT_LARGE(false, true);
    else
        PDIT_LARGE(false, false);
#undef PDIT_LARGE
    return hipGetLastError();
}

}  // namespace pdit
