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
// One workgroup of 512 threads (8 waves) per replica; thread k owns location
// k in the draw.  The products read library copies of D and F:
// * |D|, |F| <= 16383: two int8 planes per matrix,
//   x = 128 hi + lo, in MFMA operand order; a pass over eight locations is
//   the product of the copies with the locations' permuted rows, four
//   `v_mfma_i32_16x16x64_i8` per tile and chunk (plane_products), in
//   single launches and in the persistent batch kernel.
// * |D|, |F| <= 32767: int16 row pairs, one 32-bit word = rows 2i and 2i+1
//   of a column, rows padded with zeros to N64 (N rounded up to 64) and
//   columns to N4 (rounded up to 4), plus 4 zero word rows.  Each lane takes
//   four adjacent columns with one 16-byte load per word row and matrix and
//   `v_dot2_i32_i16` (exact in int32 per word); the two waves of pair q take
//   word rows [q N64/8, (q+1) N64/8) for 256 columns each, and the four
//   quarter sums meet in LDS.  Wide 16-byte loads matter: one-column 4-byte
//   loads ran at half the per-CU rate from L2.  One pass over the copies
//   serves several consecutive locations (three, two in the persistent
//   kernel): their products are taken under the p at the start of the pass
//   and an accepted exchange corrects the later rows' sums by rank-1 terms
//   (pair_replica), which costs O(N) where a new pass would cost 2 N^2.
// * otherwise: int32 rows (N32 = N rounded up to 32, plus 16 zero rows), one
//   column per lane, 24-bit (|D|, |F| < 2^23) or int64 products.
// Narrow instances (16 max|D| max|F| < 2^31) sum each block in int32 before
// the int64 total.  A load's lane offsets live in registers for the whole
// kernel and its row offset is wave-uniform; two blocks per iteration in
// alternating registers keep the next block's loads in flight while one
// block's products run.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "pdit_internal.h"
#include "sweep_common.h"

namespace pdit {
namespace {

constexpr int kLargeThreads = 512;
constexpr int kLargeWaves = kLargeThreads / 64;
constexpr int kRowBlock = 16;  // rows per block of the two products
// locations per pass over the int16 pairs: three where one replica runs per
// workgroup, two in the persistent kernel (three would spill registers there)
constexpr int kRowsSingle = 3, kRowsBatch = 2;
constexpr int kRowsPlanes = 8;  // locations per pass on the int8 plane copies (MFMA products)

struct LargeSmem {
    alignas(16) int32_t f[kLargeNMax];    // F[p(r)][p(.)], zero beyond N
    alignas(16) int32_t dq[kLargeNMax];   // D[r][q(.)] (row r of D by facility), zero beyond N
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
    int32_t wtie[kLargeWaves];     // tie flag of each wave's first hit
    uint32_t u24s[kLargeNMax];     // the sweep's uniforms, one per location
    int32_t xf[2];  // prefetched next-row flows of locations r and s (accepted exchange)
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

// Minimum of a 64-bit value over the wave: DPP shifts within rows of 16
// lanes (neutral INT64_MAX shifted in), then the four row results.
__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#define PDIT_MIN_STEP(K)                                                               \
    {                                                                                  \
        const uint32_t tl = (uint32_t)dpp_row_shr<K>(-1, (int32_t)(uint32_t)v);        \
        const uint32_t th = (uint32_t)dpp_row_shr<K>(INT32_MAX, (int32_t)(v >> 32));   \
        const int64_t t = (int64_t)((uint64_t)th << 32 | tl);                          \
        v = t < v ? t : v;                                                             \
    }
    PDIT_MIN_STEP(1)
    PDIT_MIN_STEP(2)
    PDIT_MIN_STEP(4)
    PDIT_MIN_STEP(8)
#undef PDIT_MIN_STEP
    const int64_t a = readlane_i64(v, 15), b = readlane_i64(v, 31);
    const int64_t c = readlane_i64(v, 47), d = readlane_i64(v, 63);
    const int64_t ab = a < b ? a : b, cd = c < d ? c : d;
    return ab < cd ? ab : cd;
}

// The lane's entries of a block of int32 rows: its offsets (column k of each
// row of a block) stay in vector registers for the whole kernel and the
// block's row offset is wave-uniform, so a load is one instruction.
template <int W>
__device__ __forceinline__ void load_block(__amdgpu_buffer_rsrc_t rs, const uint32_t (&voff)[W],
                                           uint32_t soff, uint32_t (&x)[W]) {
#pragma unroll
    for (int u = 0; u < W; ++u) x[u] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff[u], soff, 0);
}

// Adds the products of one block of int32 rows (the lane's entries x1, x2 of
// rows j0..j0+15) with entries j0..j0+15 of a and b to acc1, acc2.
template <bool NARROW>
__device__ __forceinline__ void block_products(const uint32_t (&x1)[kRowBlock],
                                               const uint32_t (&x2)[kRowBlock], const int32_t *a,
                                               const int32_t *b, int j0, int64_t &acc1,
                                               int64_t &acc2) {
    const int4 *a4 = (const int4 *)(a + j0);
    const int4 *b4 = (const int4 *)(b + j0);
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
            acc1 += (int64_t)(int32_t)x1[4 * q + 0] * av.x + (int64_t)(int32_t)x1[4 * q + 1] * av.y +
                    (int64_t)(int32_t)x1[4 * q + 2] * av.z + (int64_t)(int32_t)x1[4 * q + 3] * av.w;
            acc2 += (int64_t)(int32_t)x2[4 * q + 0] * bv.x + (int64_t)(int32_t)x2[4 * q + 1] * bv.y +
                    (int64_t)(int32_t)x2[4 * q + 2] * bv.z + (int64_t)(int32_t)x2[4 * q + 3] * bv.w;
        }
    }
}

// Paired copies, four adjacent columns per lane (one 16-byte load per word
// row and matrix), one quarter of the word rows per wave pair: partial sums
// of the quarter for columns c0..c0+3 and each of the K rows of a pass
// (a[i], b[i]: the int16 vectors of row i).  Every loaded word meets the K
// rows' words, so one pass over the copies serves K rows.  Word rows
// q0 .. q0+Q-1, blocks of 4.
template <int K, bool NARROW>
__device__ __forceinline__ void quarter_products(__amdgpu_buffer_rsrc_t M1,
                                                 __amdgpu_buffer_rsrc_t M2, uint32_t pitchB,
                                                 uint32_t voff0, int q0, int Q,
                                                 const int16_t (*a)[kLargeNMax],
                                                 const int16_t (*b)[kLargeNMax],
                                                 int64_t (&acc1)[K][4], int64_t (&acc2)[K][4]) {
    constexpr int B = 4;  // word rows per block
    uint32_t voff[B];
#pragma unroll
    for (int u = 0; u < B; ++u) voff[u] = voff0 + u * pitchB;
    uint4 xa1[B], xa2[B], xb1[B], xb2[B];
    uint32_t soff = (uint32_t)q0 * pitchB;
    const uint32_t block_bytes = B * pitchB;
#pragma unroll
    for (int u = 0; u < B; ++u) {
        xa1[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M1, voff[u], soff, 0));
        xa2[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M2, voff[u], soff, 0));
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc1[i][c] = acc2[i][c] = 0;
    // products of one block (word rows w0..w0+3) added to s1, s2: int32 partial
    // sums of at most 16 products (two blocks) when NARROW, else each word's
    // pair of products (exact in int32) straight into the int64 totals
    auto block = [&](const uint4 (&x1)[B], const uint4 (&x2)[B], int w0, int32_t (&s1)[K][4],
                     int32_t (&s2)[K][4]) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint4 aw = *(const uint4 *)(a[i] + 2 * w0);
            const uint4 bw = *(const uint4 *)(b[i] + 2 * w0);
            const uint32_t av[4] = {aw.x, aw.y, aw.z, aw.w};
            const uint32_t bv[4] = {bw.x, bw.y, bw.z, bw.w};
#pragma unroll
            for (int u = 0; u < B; ++u) {
                if (NARROW) {
                    s1[i][0] = dot2(x1[u].x, av[u], s1[i][0]);
                    s1[i][1] = dot2(x1[u].y, av[u], s1[i][1]);
                    s1[i][2] = dot2(x1[u].z, av[u], s1[i][2]);
                    s1[i][3] = dot2(x1[u].w, av[u], s1[i][3]);
                    s2[i][0] = dot2(x2[u].x, bv[u], s2[i][0]);
                    s2[i][1] = dot2(x2[u].y, bv[u], s2[i][1]);
                    s2[i][2] = dot2(x2[u].z, bv[u], s2[i][2]);
                    s2[i][3] = dot2(x2[u].w, bv[u], s2[i][3]);
                } else {
                    acc1[i][0] += dot2(x1[u].x, av[u], 0);
                    acc1[i][1] += dot2(x1[u].y, av[u], 0);
                    acc1[i][2] += dot2(x1[u].z, av[u], 0);
                    acc1[i][3] += dot2(x1[u].w, av[u], 0);
                    acc2[i][0] += dot2(x2[u].x, bv[u], 0);
                    acc2[i][1] += dot2(x2[u].y, bv[u], 0);
                    acc2[i][2] += dot2(x2[u].z, bv[u], 0);
                    acc2[i][3] += dot2(x2[u].w, bv[u], 0);
                }
            }
        }
    };
    for (int w = q0; w < q0 + Q; w += 2 * B) {
        soff += block_bytes;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            xb1[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M1, voff[u], soff, 0));
            xb2[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M2, voff[u], soff, 0));
        }
        int32_t s1[K][4], s2[K][4];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) s1[i][c] = s2[i][c] = 0;
        block(xa1, xa2, w, s1, s2);
        // the block after a quarter's last is the next quarter's first, or the pad block
        soff += block_bytes;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            xa1[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M1, voff[u], soff, 0));
            xa2[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(M2, voff[u], soff, 0));
        }
        block(xb1, xb2, w + B, s1, s2);
        if (NARROW) {
#pragma unroll
            for (int i = 0; i < K; ++i)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc1[i][c] += s1[i][c];
                    acc2[i][c] += s2[i][c];
                }
        }
    }
}

// int32 copies, one column per lane: hkr = sum_j M1[j][k] a[j], gk =
// sum_j M2[j][k] b[j] over rows 0..N32-1 (N32 = N rounded up to 32; a, b zero
// beyond N).  Two blocks per iteration in alternating registers: the loads
// of one block are in flight while the other's products run, with no
// register copies that would wait for them.
template <bool NARROW>
__device__ __forceinline__ void column_products(__amdgpu_buffer_rsrc_t M1,
                                                __amdgpu_buffer_rsrc_t M2,
                                                const uint32_t (&voff)[kRowBlock],
                                                uint32_t block_bytes, const int32_t *a,
                                                const int32_t *b, int N32, int64_t &hkr,
                                                int64_t &gk) {
    uint32_t xa1[kRowBlock], xa2[kRowBlock], xb1[kRowBlock], xb2[kRowBlock];
    load_block<kRowBlock>(M1, voff, 0, xa1);
    load_block<kRowBlock>(M2, voff, 0, xa2);
    int64_t acc1 = 0, acc2 = 0;
    uint32_t soff = 0;
    for (int j0 = 0; j0 < N32; j0 += 2 * kRowBlock) {
        soff += block_bytes;
        load_block<kRowBlock>(M1, voff, soff, xb1);
        load_block<kRowBlock>(M2, voff, soff, xb2);
        block_products<NARROW>(xa1, xa2, a, b, j0, acc1, acc2);
        // the block after the last one is the zero pad block: always in range
        soff += block_bytes;
        load_block<kRowBlock>(M1, voff, soff, xa1);
        load_block<kRowBlock>(M2, voff, soff, xa2);
        block_products<NARROW>(xb1, xb2, a, b, j0 + kRowBlock, acc1, acc2);
    }
    hkr = acc1;
    gk = acc2;
}

typedef int mf_v4i __attribute__((ext_vector_type(4)));
// row pitch of the int8 plane vectors in LDS: 16 bytes beyond a multiple of
// 512, so the 16 rows one B operand reads start in different banks
constexpr int kPlanePitch = kLargeNMax + 16;

// MFMA products of one pass over the int8 plane copies: for the K rows of the
// pass, S1[k][i] = sum_j D[k][j] f_i[j] and S2[c][i] = sum_b F[c][b] dq_i[b]
// (D and F symmetric, so rows stand for columns).  Every operand is split as
// x = 128 hi + lo with hi signed and lo in [0, 127] (|x| <= 16383), so a
// product is four `v_mfma_i32_16x16x64_i8`: hi hi, the two cross terms in one
// accumulator, lo lo, each exact in int32 for N <= 512 (at most 512 terms of
// 2^14).  A operand: rows 16 t .. 16 t + 15 of a copy; B operand: the pass's
// rows as columns, zero beyond K.  Wave w takes tiles w, w + 8, ...; the next
// chunk's copy rows are loaded while the current chunk's products run.
template <int K>
__device__ __forceinline__ void plane_products(__amdgpu_buffer_rsrc_t Dp,
                                               __amdgpu_buffer_rsrc_t Fp, uint32_t plane,
                                               int N, int N16, int N64, int wv, int lane,
                                               const int8_t (*fh)[kPlanePitch],
                                               const int8_t (*fl)[kPlanePitch],
                                               const int8_t (*dh)[kPlanePitch],
                                               const int8_t (*dl)[kPlanePitch],
                                               int64_t (*out1)[1][kLargeNMax],
                                               int64_t (*out2)[1][kLargeNMax]) {
    static_assert(K <= 16, "one 16-column B tile");
    const int n = lane & 15;          // row of the A tile and column of B
    const int kq = (lane >> 4) * 16;  // this lane's 16 bytes of the 64-wide chunk
    const int NT = N16 / 16, NC = N64 / 64;
    const int steps = ((NT - wv + kLargeWaves - 1) / kLargeWaves) * NC;  // (tile, chunk) pairs
    if (wv >= NT) return;
    // (tile, chunk) of the next load and of the next step, advanced by
    // counting (a division by the runtime NC per step costs more than the step)
    int lt = wv, lc = 0, st = wv, sc = 0;
    auto load = [&](mf_v4i (&a)[4]) {
        // past the wave's last step the ring reloads its first: always in range
        if (lt >= NT) {
            lt = wv;
            lc = 0;
        }
        // the copies hold each operand in lane order: 1 KB per tile and chunk
        const uint32_t off = (uint32_t)(((lt * NC + lc) * 64 + lane) * 16);
        if (++lc == NC) {
            lc = 0;
            lt += kLargeWaves;
        }
        a[0] = __builtin_bit_cast(mf_v4i, __builtin_amdgcn_raw_buffer_load_b128(Dp, off, 0, 0));
        a[1] = __builtin_bit_cast(mf_v4i, __builtin_amdgcn_raw_buffer_load_b128(Dp, off, plane, 0));
        a[2] = __builtin_bit_cast(mf_v4i, __builtin_amdgcn_raw_buffer_load_b128(Fp, off, 0, 0));
        a[3] = __builtin_bit_cast(mf_v4i, __builtin_amdgcn_raw_buffer_load_b128(Fp, off, plane, 0));
    };
    const mf_v4i z = {0, 0, 0, 0};
    mf_v4i h1 = z, x1 = z, l1 = z, h2 = z, x2 = z, l2 = z;
    // products of the next step from the operands in a
    auto step = [&](const mf_v4i (&a)[4]) {
        const int c = sc;
        mf_v4i bfh = z, bfl = z, bdh = z, bdl = z;
        if (n < K) {
            bfh = *(const mf_v4i *)&fh[n][64 * c + kq];
            bfl = *(const mf_v4i *)&fl[n][64 * c + kq];
            bdh = *(const mf_v4i *)&dh[n][64 * c + kq];
            bdl = *(const mf_v4i *)&dl[n][64 * c + kq];
        }
        h1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], bfh, h1, 0, 0, 0);
        h2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[2], bdh, h2, 0, 0, 0);
        x1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], bfl, x1, 0, 0, 0);
        x2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[2], bdl, x2, 0, 0, 0);
        l1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], bfl, l1, 0, 0, 0);
        l2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[3], bdl, l2, 0, 0, 0);
        x1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], bfh, x1, 0, 0, 0);
        x2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[3], bdh, x2, 0, 0, 0);
        if (c == NC - 1) {
            // element e: row 16 t + 4 (lane / 16) + e of the tile, column n
            const int t = st;
            if (n < K) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * t + 4 * (lane >> 4) + e;
                    if (k < N) {
                        out1[n][0][k] = 16384 * (int64_t)h1[e] + 128 * (int64_t)x1[e] + l1[e];
                        out2[n][0][k] = 16384 * (int64_t)h2[e] + 128 * (int64_t)x2[e] + l2[e];
                    }
                }
            }
            h1 = x1 = l1 = h2 = x2 = l2 = z;
        }
        if (++sc == NC) {
            sc = 0;
            st += kLargeWaves;
        }
    };
    // a ring of four operand sets, three steps in flight, no register copies
    // (a copy would wait for its loads)
    mf_v4i a0[4], a1[4], a2[4], a3[4];
    load(a0);
    load(a1);
    load(a2);
    for (int q = 0; q < steps; q += 4) {
        load(a3);
        step(a0);
        load(a0);
        if (q + 1 < steps) step(a1);
        load(a1);
        if (q + 2 < steps) step(a2);
        load(a2);
        if (q + 3 < steps) step(a3);
    }
}

// LDS of the multi-location passes (int16 pairs or int8 planes): the
// vectors and partial sums of the K rows of a products pass, and the state
// shared by all rows.
template <int K, bool MF>
struct PairSmem {
    static constexpr int K16 = MF ? 1 : K;  // rows of the int16 vectors (dot2 products)
    static constexpr int K8 = MF ? K : 1;   // rows of the int8 planes (MFMA products)
    static constexpr int QN = MF ? 1 : 4;   // partial sums per row and column
    alignas(16) int16_t f16[K16][kLargeNMax];   // F[p(x)][p(.)] (row x of the pass), zero beyond N
    alignas(16) int16_t dq16[K16][kLargeNMax];  // D[x][q(.)] by facility, zero beyond N
    alignas(16) int8_t fh[K8][kPlanePitch];     // the same two as int8 planes, hi and lo
    alignas(16) int8_t fl[K8][kPlanePitch];
    alignas(16) int8_t dh[K8][kPlanePitch];
    alignas(16) int8_t dl[K8][kPlanePitch];
    int64_t part1[K][QN][kLargeNMax];  // partial sums: H[.][x] by location
    int64_t part2[K][QN][kLargeNMax];  // partial sums: H[x][.] by facility
    int32_t fr[K][kLargeNMax];        // F[p(x)][p(k)] under the current p
    int32_t dr[K][kLargeNMax];        // D[x][k]
    int32_t p[kLargeNMax];                     // facility at each location
    int32_t ddiag[kLargeNMax];                 // D[x][x]
    int32_t fdiag[kLargeNMax];                 // F[c][c]
    int64_t hd[kLargeNMax];                    // H[x][x]
    int32_t v[kLargeNMax];
    int64_t wmin[kLargeWaves];
    uint64_t wsum[kLargeWaves];
    int32_t wsel[kLargeWaves];
    int32_t wtie[kLargeWaves];     // tie flag of each wave's first hit
    uint32_t u24s[kLargeNMax];     // the sweep's uniforms, one per location
    int32_t xf[K][2];     // prefetched next-pass flows of locations r and s (accepted exchange)
};

// One replica's sweeps on the int16 pairs (MF false) or the int8 planes (MF
// true), K locations per pass over the copies.  The pass takes the products of its rows under the p at
// its start; an accepted exchange of r and s (p -> p tau, tau exchanging r
// and s) moves the sums of a later row x of the pass by rank-1 terms:
//   H'[k][x] = H[k][x] + (D[r][k] - D[s][k]) (F[p(x)][p(s)] - F[p(x)][p(r)])
// for x != s, and for x = s (p'(s) = p(r)) the sums of row r itself:
//   H'[k][s] = H[k][r] + (D[r][k] - D[s][k]) (F[p(r)][p(s)] - F[p(r)][p(r)]);
// by facility, G'[c] = G[c] + (F[p(r)][c] - F[p(s)][c]) (D[x][s] - D[x][r])
// in both cases.  A stay changes nothing.  So every row of a pass is drawn
// exactly as if its products had been taken just before its update.
template <int K, bool MF, bool NARROW, typename HT>
__device__ void pair_replica(const ReplicaJob &j, PairSmem<K, MF> &sm) {
    constexpr int QN = PairSmem<K, MF>::QN;
    const int N = j.N;
    const int k = threadIdx.x, lane = k & 63;
    const int wv = __builtin_amdgcn_readfirstlane(k >> 6);  // wave-uniform, as the compiler must see
    const bool own = k < N;
    const int32_t *__restrict__ D = j.D;
    const int32_t *__restrict__ F = j.F;
    // word rows of a copy: row pairs, N4 = N rounded up to 4 words, N64 / 2 + 4 word rows
    const int N4 = (N + 3) & ~3;
    const int N64 = (N + 63) & ~63;
    const uint32_t pitch = (uint32_t)N4 * 4;
    // plane copies: N16 x N64 bytes per plane, hi then lo
    const int N16 = (N + 15) & ~15;
    const uint32_t plane = (uint32_t)N16 * (uint32_t)N64;
    const uint32_t copy_bytes = MF ? 2 * plane : (uint32_t)(N64 / 2 + 4) * pitch;
    const __amdgpu_buffer_rsrc_t Dc = copy_rsrc(j.cD, copy_bytes);
    const __amdgpu_buffer_rsrc_t Fc = copy_rsrc(j.cF, copy_bytes);
    int32_t *perm = j.perm;
    int32_t *pbest = j.perm_best;
    // diag H of the initial p; kSaveState writes the final one back (the
    // library's H buffer, writable)
    HT *H0 = (HT *)const_cast<void *>(j.H);
    const float *beta_p = j.beta;
    const int64_t beta_stride = j.beta_stride;
    // the next pass's rows are loaded during the products (int16 pairs),
    // unless the pass wraps onto itself (N <= K); on the planes, with eight
    // locations per pass, each pass loads its rows at its start: permuting
    // eight prefetched rows after every accepted exchange cost more than
    // that load
    const bool pre = !MF && N > K;

    if (own) {
        sm.p[k] = perm[k];
        sm.ddiag[k] = D[(int64_t)k * N + k];
        sm.fdiag[k] = F[(int64_t)k * N + k];
        sm.hd[k] = (int64_t)H0[(int64_t)k * N + k];
    } else {
        // the products' zero pad
        if constexpr (MF) {
#pragma unroll
            for (int i = 0; i < K; ++i) sm.fh[i][k] = sm.fl[i][k] = sm.dh[i][k] = sm.dl[i][k] = 0;
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i) sm.f16[i][k] = sm.dq16[i][k] = 0;
        }
    }
    int64_t E = *j.E;
    int64_t E_best = *j.E_best;
    int64_t n_acc = 0, n_tie = 0;
    __syncthreads();
    // this lane's own location: facility, D[k][k], F[p(k)][p(k)] and H[k][k]
    // in registers (LDS keeps them for the other lanes)
    int32_t myp = own ? sm.p[k] : 0;
    const int32_t ddk = own ? sm.ddiag[k] : 0;
    int32_t fdk = own ? sm.fdiag[myp] : 0;
    int64_t hdk = own ? sm.hd[k] : 0;
    // location k's entries of the pass's rows: D[x][k] and F[p(x)][p(k)]
    int32_t pd[K], pf[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        pd[i] = pf[i] = 0;
        if (pre && own) {
            pd[i] = D[(int64_t)i * N + k];
            pf[i] = F[(int64_t)sm.p[i] * N + myp];
        }
    }

    for (int64_t t = 0; t < j.T; ++t) {
        const float beta = beta_p[t * beta_stride];
        const int64_t dthr = zero_weight_distance64(beta);
        const uint32_t g = (uint32_t)(j.sweep_offset + (uint64_t)t);
        // the sweep's N uniforms at once, lane k for location k (ordered
        // before their first use by the first barrier of the first pass)
        if (own) sm.u24s[k] = uniform24(j.seed, (uint32_t)k, g, j.rep, j.inst);
        for (int r0 = 0; r0 < N; r0 += K) {
            const int kb = N - r0 < K ? N - r0 : K;  // rows of this pass
            // ---- the pass's rows: by location, by facility, and as int16 ----
            if (own) {
                const int pk = myp;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    int32_t dx = pd[i], fx = pf[i];
                    if (!pre) {
                        dx = fx = 0;
                        if (i < kb) {
                            dx = D[(int64_t)(r0 + i) * N + k];
                            fx = F[(int64_t)sm.p[r0 + i] * N + pk];
                        }
                    }
                    sm.dr[i][k] = dx;
                    sm.fr[i][k] = fx;
                    if constexpr (MF) {
                        sm.fh[i][k] = (int8_t)(fx >> 7);
                        sm.fl[i][k] = (int8_t)(fx & 127);
                        sm.dh[i][pk] = (int8_t)(dx >> 7);
                        sm.dl[i][pk] = (int8_t)(dx & 127);
                    } else {
                        sm.f16[i][k] = (int16_t)fx;
                        sm.dq16[i][pk] = (int16_t)dx;
                    }
                }
            }
            __syncthreads();
            // the next pass's rows under the current p; accepted exchanges of
            // this pass permute them afterwards
            const int nb = r0 + K < N ? r0 + K : 0;
            if (pre) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    pd[i] = pf[i] = 0;
                    if (own && nb + i < N) {
                        pd[i] = D[(int64_t)(nb + i) * N + k];
                        pf[i] = F[(int64_t)sm.p[nb + i] * N + myp];
                    }
                }
            }
            // ---- products: columns x of H and rows x of H by facility, x in the pass ----
            if constexpr (MF) {
                plane_products<K>(Dc, Fc, plane, N, N16, N64, wv, lane, sm.fh, sm.fl, sm.dh, sm.dl,
                                  sm.part1, sm.part2);
            } else {
                // wave pair rq takes word rows [rq Q, (rq + 1) Q), wave ch of the
                // pair columns 256 ch + 4 lane .. + 3
                const int rq = wv >> 1, ch = wv & 1;
                const int c0 = 256 * ch + 4 * lane;
                const bool act = c0 < N4;
                const int Q = N64 / 8;  // a multiple of 8 word rows: whole block pairs
                if (256 * ch < N4) {
                    int64_t p1[K][4], p2[K][4];
                    quarter_products<K, NARROW>(Dc, Fc, pitch, act ? (uint32_t)c0 * 4 : 0u,
                                                rq * Q, Q, sm.f16, sm.dq16, p1, p2);
                    if (act) {
#pragma unroll
                        for (int i = 0; i < K; ++i)
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                sm.part1[i][rq][c0 + c] = p1[i][c];
                                sm.part2[i][rq][c0 + c] = p2[i][c];
                            }
                    }
                }
            }
            __syncthreads();
            // H[y][x] and H[x][y] (= G at facility p(y)) for row i of the pass:
            // the sums of the partial sums, read where they lie
            auto hcol_at = [&](int i, int y) -> int64_t {
                int64_t a = sm.part1[i][0][y];
#pragma unroll
                for (int q = 1; q < QN; ++q) a += sm.part1[i][q][y];
                return a;
            };
            auto g_at = [&](int i, int c) -> int64_t {
                int64_t a = sm.part2[i][0][c];
#pragma unroll
                for (int q = 1; q < QN; ++q) a += sm.part2[i][q][c];
                return a;
            };
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (i >= kb) break;
                const int r = r0 + i;
                const int pr = sm.p[r];
                // ---- energy change of candidate k (Eq. 3) ----
                int64_t v = INT64_MAX;
                if (own) {
                    const int64_t hkr = hcol_at(i, k);
                    const int64_t hrk = g_at(i, myp);
                    const int64_t h = hrk + hkr - sm.hd[r] - hdk;
                    const int64_t dd = (int64_t)sm.ddiag[r] + ddk - 2 * (int64_t)sm.dr[i][k];
                    const int64_t ff = (int64_t)sm.fdiag[pr] + fdk - 2 * (int64_t)sm.fr[i][k];
                    v = k == r ? 0 : 2 * h + dd * ff;
                }
                // ---- block minimum ----
                const int64_t m0 = wave_min_i64(v);
                if (lane == 0) sm.wmin[wv] = m0;
                __syncthreads();
                int64_t m = sm.wmin[0];
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
                const uint32_t u24 = sm.u24s[r];
                const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
                // the first candidate whose running sum exceeds the threshold: each
                // wave publishes its first hit and that candidate's tie flag
                const uint64_t hit = __ballot(own && C > thr);
                const int first = hit ? __ffsll((unsigned long long)hit) - 1 : -1;  // wave-uniform
                if (first < 0) {
                    if (lane == 0) sm.wsel[wv] = 0x7fffffff;
                } else if (lane == first) {
                    sm.wsel[wv] = 64 * wv + first;
                    sm.wtie[wv] = is_tie(C - qk, C, Z, u24) ? 1 : 0;
                }
                __syncthreads();
                int s = 0x7fffffff;
#pragma unroll
                for (int w = 0; w < kLargeWaves; ++w) s = min(s, sm.wsel[w]);
                int tie = 0;
                if (s >= N)
                    s = r;  // unreachable: location N-1 holds C = Z > thr
                else
                    tie = sm.wtie[s >> 6];
                n_tie += tie;
                if (j.choices && k == 0) j.choices[t * N + r] = s;
                if (s == r) continue;
                // ---- accepted exchange of r and s: E, diag H, p, the later rows ----
                ++n_acc;
                const int ps = sm.p[s];
                int32_t uk = 0, wk = 0;
                if (own) {
                    uk = D[(int64_t)s * N + k] - sm.dr[i][k];             // D[k][s] - D[k][r]
                    sm.v[k] = sm.fr[i][k] - F[(int64_t)ps * N + myp];  // Fp[r][k] - Fp[s][k]
                    wk = F[(int64_t)pr * N + k] - F[(int64_t)ps * N + k];  // F[p(r)][c] - F[p(s)][c], c = k
                    if (pre) {
#pragma unroll
                        for (int i2 = 0; i2 < K; ++i2) {
                            if (k == r) sm.xf[i2][0] = pf[i2];
                            if (k == s) sm.xf[i2][1] = pf[i2];
                        }
                    }
                }
                // later rows' factors, read before anything moves
                int32_t frr[K], frs[K], ddl[K];
#pragma unroll
                for (int i2 = 0; i2 < K; ++i2) {
                    frr[i2] = frs[i2] = ddl[i2] = 0;
                    if (i2 > i && i2 < kb) {
                        frr[i2] = sm.fr[i2][r];
                        frs[i2] = sm.fr[i2][s];
                        ddl[i2] = sm.dr[i2][s] - sm.dr[i2][r];
                    }
                }
                const int32_t dfr = sm.fr[i][s] - sm.fr[i][r];
                const int64_t h_rs = g_at(i, ps), h_sr = hcol_at(i, s);
                const int64_t dE = 2 * (h_rs + h_sr - sm.hd[r] - sm.hd[s]) +
                                   ((int64_t)sm.ddiag[r] + sm.ddiag[s] - 2 * (int64_t)sm.dr[i][s]) *
                                       ((int64_t)sm.fdiag[pr] + sm.fdiag[ps] - 2 * (int64_t)sm.fr[i][s]);
                __syncthreads();
                E += dE;
                const int tk = k == r ? s : k == s ? r : k;
                if (own) {
                    if (k == r)
                        hdk = h_rs + (int64_t)uk * sm.v[s];
                    else if (k == s)
                        hdk = h_sr + (int64_t)uk * sm.v[r];
                    else
                        hdk += (int64_t)uk * sm.v[k];
                    sm.hd[k] = hdk;
                    if (k == r || k == s) {
                        myp = k == r ? ps : pr;
                        fdk = sm.fdiag[myp];
                    }
                    // the later rows of the pass
#pragma unroll
                    for (int i2 = 0; i2 < K; ++i2) {
                        if (i2 <= i || i2 >= kb) continue;
                        if (r0 + i2 == s) {
                            sm.part1[i2][0][k] = hcol_at(i, k) - (int64_t)uk * dfr;
#pragma unroll
                            for (int q = 1; q < QN; ++q) sm.part1[i2][q][k] = 0;
                            sm.fr[i2][k] = sm.fr[i][tk];
                        } else {
                            sm.part1[i2][0][k] -= (int64_t)uk * (frs[i2] - frr[i2]);
                            if (k == r) sm.fr[i2][k] = frs[i2];
                            if (k == s) sm.fr[i2][k] = frr[i2];
                        }
                        sm.part2[i2][0][k] += (int64_t)wk * ddl[i2];
                    }
                }
                if (k == 0) {
                    sm.p[r] = ps;
                    sm.p[s] = pr;
                }
                // the next pass's rows after the exchange: D as prefetched;
                // F[p'(y)][p'(k)] = F[p(y)][p(tau k)], the prefetched row at
                // tau k, or, when y = s (p'(s) = p(r)), row r's at tau k
                if (pre && own) {
#pragma unroll
                    for (int i2 = 0; i2 < K; ++i2) {
                        if (nb + i2 >= N) continue;
                        if (nb + i2 == s)
                            pf[i2] = sm.fr[i][tk];
                        else if (k == r)
                            pf[i2] = sm.xf[i2][1];
                        else if (k == s)
                            pf[i2] = sm.xf[i2][0];
                    }
                }
                __syncthreads();
                if (E < E_best) {
                    E_best = E;
                    if (own) pbest[k] = myp;
                }
            }
        }
        if (j.E_trace && k == 0) j.E_trace[t] = E;
    }
    if (own) {
        perm[k] = myp;
        if (j.flags & kSaveState) H0[(int64_t)k * N + k] = (HT)hdk;
    }
    if (k == 0) {
        *j.E = E;
        *j.E_best = E_best;
        const bool acc = (j.flags & kAccumCounters) != 0;
        j.counters[0] = (acc ? j.counters[0] : 0) + (int64_t)N * j.T;
        j.counters[1] = (acc ? j.counters[1] : 0) + n_acc;
        j.counters[2] = (acc ? j.counters[2] : 0) + n_tie;
    }
}

// One replica's sweeps on the int32 copies, one location at a time.
template <bool NARROW, typename HT>
__device__ void large_replica(const ReplicaJob &j, LargeSmem &sm) {
    const int N = j.N;
    const int N32 = (N + 2 * kRowBlock - 1) / (2 * kRowBlock) * (2 * kRowBlock);
    const int k = threadIdx.x, lane = k & 63;
    const int wv = __builtin_amdgcn_readfirstlane(k >> 6);  // wave-uniform, as the compiler must see
    const bool own = k < N;
    const int32_t *__restrict__ D = j.D;
    const int32_t *__restrict__ F = j.F;
    // rows of a copy: N words, N32 + 16 rows
    const uint32_t pitch = (uint32_t)N * 4;
    const uint32_t copy_bytes = (uint32_t)(N32 + kRowBlock) * pitch;
    const __amdgpu_buffer_rsrc_t Dc = copy_rsrc(j.cD, copy_bytes);
    const __amdgpu_buffer_rsrc_t Fc = copy_rsrc(j.cF, copy_bytes);
    // lanes past N read column 0 (results unused): every offset stays inside
    // the copy even for the prefetch of the zero block
    const uint32_t col = own ? (uint32_t)k : 0u;
    uint32_t voff[kRowBlock];  // int32 copies: column k of the rows of a block
#pragma unroll
    for (int u = 0; u < kRowBlock; ++u) voff[u] = col * 4 + u * pitch;
    int32_t *perm = j.perm;
    int32_t *pbest = j.perm_best;
    // diag H of the initial p; kSaveState writes the final one back (the
    // library's H buffer, writable)
    HT *H0 = (HT *)const_cast<void *>(j.H);
    const float *beta_p = j.beta;
    const int64_t beta_stride = j.beta_stride;

    if (own) {
        sm.p[k] = perm[k];
        sm.ddiag[k] = D[(int64_t)k * N + k];
        sm.fdiag[k] = F[(int64_t)k * N + k];
        sm.hd[k] = (int64_t)H0[(int64_t)k * N + k];
    } else {
        sm.f[k] = 0;  // the products' zero pad
        sm.dq[k] = 0;
    }
    int64_t E = *j.E;
    int64_t E_best = *j.E_best;
    int64_t n_acc = 0, n_tie = 0;
    __syncthreads();
    // location k's entries of the current row: D[r][k] and F[p(r)][p(k)],
    // loaded for row 0, then prefetched during the previous update
    int32_t drk = 0, fk = 0;
    if (own) {
        drk = D[k];
        fk = F[(int64_t)sm.p[0] * N + sm.p[k]];
    }

    for (int64_t t = 0; t < j.T; ++t) {
        const float beta = beta_p[t * beta_stride];
        const int64_t dthr = zero_weight_distance64(beta);
        const uint32_t g = (uint32_t)(j.sweep_offset + (uint64_t)t);
        // the sweep's N uniforms at once, lane k for location k (ordered
        // before their first use by the first barrier of update 0)
        if (own) sm.u24s[k] = uniform24(j.seed, (uint32_t)k, g, j.rep, j.inst);
        for (int r = 0; r < N; ++r) {
            const int pr = sm.p[r];
            // ---- row r of D, by location and by facility, and of the permuted flows ----
            if (own) {
                const int pk = sm.p[k];
                sm.d[k] = drk;
                sm.f[k] = fk;
                sm.dq[pk] = drk;
            }
            __syncthreads();
            // prefetch of the next location's rows under the current p; an
            // accepted exchange of r and s permutes the flows afterwards
            const int rn = r + 1 < N ? r + 1 : 0;
            int32_t dn = 0, fn = 0;
            if (own) {
                dn = D[(int64_t)rn * N + k];
                fn = F[(int64_t)sm.p[rn] * N + sm.p[k]];
            }
            // ---- column r of H (location k) and row r of H by facility (facility k) ----
            int64_t hkr = 0, gk = 0;
            if (wv * 64 < N) {  // waves with no location skip the products
                column_products<NARROW>(Dc, Fc, voff, kRowBlock * pitch, sm.f, sm.dq, N32, hkr,
                                        gk);
                if (own) {
                    sm.G[k] = gk;
                    sm.hcol[k] = hkr;
                }
            }
            __syncthreads();
            // H[x][r] and H[r][x] (= G at facility p(x))
            auto hcol_at = [&](int x) -> int64_t { return sm.hcol[x]; };
            auto g_at = [&](int c) -> int64_t { return sm.G[c]; };
            // ---- energy change of candidate k (Eq. 3) ----
            int64_t v = INT64_MAX;
            if (own) {
                const int64_t hrk = g_at(sm.p[k]);
                const int64_t h = hrk + hkr - sm.hd[r] - sm.hd[k];
                const int64_t dd = (int64_t)sm.ddiag[r] + sm.ddiag[k] - 2 * (int64_t)sm.d[k];
                const int64_t ff = (int64_t)sm.fdiag[pr] + sm.fdiag[sm.p[k]] - 2 * (int64_t)sm.f[k];
                v = k == r ? 0 : 2 * h + dd * ff;
            }
            // ---- block minimum ----
            const int64_t m0 = wave_min_i64(v);
            if (lane == 0) sm.wmin[wv] = m0;
            __syncthreads();
            int64_t m = sm.wmin[0];
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
            const uint32_t u24 = sm.u24s[r];
            const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
            // the first candidate whose running sum exceeds the threshold: each
            // wave publishes its first hit and that candidate's tie flag
            const uint64_t hit = __ballot(own && C > thr);
            const int first = hit ? __ffsll((unsigned long long)hit) - 1 : -1;  // wave-uniform
            if (first < 0) {
                if (lane == 0) sm.wsel[wv] = 0x7fffffff;
            } else if (lane == first) {
                sm.wsel[wv] = 64 * wv + first;
                sm.wtie[wv] = is_tie(C - qk, C, Z, u24) ? 1 : 0;
            }
            __syncthreads();
            int s = 0x7fffffff;
#pragma unroll
            for (int w = 0; w < kLargeWaves; ++w) s = min(s, sm.wsel[w]);
            int tie = 0;
            if (s >= N)
                s = r;  // unreachable: location N-1 holds C = Z > thr
            else
                tie = sm.wtie[s >> 6];
            n_tie += tie;
            if (j.choices && k == 0) j.choices[t * N + r] = s;
            if (s == r) {
                drk = dn;
                fk = fn;
                continue;
            }
            // ---- accepted exchange of r and s: E, diag H, p ----
            ++n_acc;
            const int ps = sm.p[s];
            if (own) {
                sm.u[k] = D[(int64_t)s * N + k] - drk;              // D[k][s] - D[k][r]
                sm.v[k] = fk - F[(int64_t)ps * N + sm.p[k]];        // Fp[r][k] - Fp[s][k]
                if (k == r) sm.xf[0] = fn;
                if (k == s) sm.xf[1] = fn;
            }
            const int64_t h_rs = g_at(ps), h_sr = hcol_at(s);
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
            // the next row after the exchange (tau swaps r and s): D[rn][k] as
            // prefetched; F[p'(rn)][p'(k)] = F[p(rn)][p(tau k)], the prefetched
            // row at tau k, or, when rn = s (p'(s) = p(r)), the current row at tau k
            drk = dn;
            if (own) {
                const int tk = k == r ? s : k == s ? r : k;
                fk = rn == s ? sm.f[tk] : k == r ? sm.xf[1] : k == s ? sm.xf[0] : fn;
            }
            __syncthreads();
            if (E < E_best) {
                E_best = E;
                if (own) pbest[k] = sm.p[k];
            }
        }
        if (j.E_trace && k == 0) j.E_trace[t] = E;
    }
    if (own) {
        perm[k] = sm.p[k];
        if (j.flags & kSaveState) H0[(int64_t)k * N + k] = (HT)sm.hd[k];
    }
    if (k == 0) {
        *j.E = E;
        *j.E_best = E_best;
        const bool acc = (j.flags & kAccumCounters) != 0;
        j.counters[0] = (acc ? j.counters[0] : 0) + (int64_t)N * j.T;
        j.counters[1] = (acc ? j.counters[1] : 0) + n_acc;
        j.counters[2] = (acc ? j.counters[2] : 0) + n_tie;
    }
}

template <bool PAIRS, bool NARROW, typename HT, bool MF>
__global__ void __launch_bounds__(kLargeThreads) sweep_large_kernel(SweepArgs a, LargeCopies c) {
    const int64_t rep = blockIdx.x;
    ReplicaJob j;
    j.N = a.N;
    j.D = a.D;
    j.F = a.F;
    j.cD = c.D;
    j.cF = c.F;
    j.perm = a.perm + rep * a.N;
    j.H = (HT *)a.H + rep * (int64_t)a.N * a.N;
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
    j.zero_diag = a.zero_diag;
    j.tstate = nullptr;
    j.flags = a.flags;
    if constexpr (MF) {
        __shared__ PairSmem<kRowsPlanes, true> sp;
        pair_replica<kRowsPlanes, true, NARROW, HT>(j, sp);
    } else if constexpr (PAIRS) {
        __shared__ PairSmem<kRowsSingle, false> sp;
        pair_replica<kRowsSingle, false, NARROW, HT>(j, sp);
    } else {
        __shared__ LargeSmem sm;
        large_replica<NARROW, HT>(j, sm);
    }
}

// Persistent: each workgroup takes (instance, replica) items of one group
// (same copy layout and H width) from a queue until it is exhausted.
template <bool PAIRS, bool NARROW, typename HT, bool MF>
__global__ void __launch_bounds__(kLargeThreads) sweep_large_persistent(BatchArgs b) {
    using Smem = typename std::conditional<
        MF, PairSmem<kRowsPlanes, true>,
        typename std::conditional<PAIRS, PairSmem<kRowsBatch, false>, LargeSmem>::type>::type;
    __shared__ Smem sm;
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(item_sh);  // wave-uniform
        __syncthreads();
        if (item >= b.n_items) break;
        if constexpr (MF)
            pair_replica<kRowsPlanes, true, NARROW, HT>(batch_job(b, item, sizeof(HT)), sm);
        else if constexpr (PAIRS)
            pair_replica<kRowsBatch, false, NARROW, HT>(batch_job(b, item, sizeof(HT)), sm);
        else
            large_replica<NARROW, HT>(batch_job(b, item, sizeof(HT)), sm);
        __syncthreads();
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

// Paired int16 copies: word (i, c) = M[2i][c] | M[2i+1][c] << 16 for
// c < N4 (N rounded up to 4), entries outside N x N zero; the host checks
// |D|, |F| <= 32767.
__global__ void large_copy16_kernel(int N, int wrows, const int32_t *D, const int32_t *F,
                                    uint32_t *Dc, uint32_t *Fc) {
    const int N4 = (N + 3) & ~3;
    const int64_t total = (int64_t)wrows * N4;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N4, c = e - i * N4;
        const int64_t lo = 2 * i * N + c, hi = lo + N;
        const bool in_c = c < N;
        const bool in_lo = in_c && 2 * i < N, in_hi = in_c && 2 * i + 1 < N;
        Dc[e] = (uint32_t)(uint16_t)(in_lo ? D[lo] : 0) | (uint32_t)(uint16_t)(in_hi ? D[hi] : 0) << 16;
        Fc[e] = (uint32_t)(uint16_t)(in_lo ? F[lo] : 0) | (uint32_t)(uint16_t)(in_hi ? F[hi] : 0) << 16;
    }
}

// int8 plane copies for the MFMA products: for M = D then F, plane hi then
// plane lo of M[k][j] (x = 128 hi + lo, lo in [0, 127]) for k < N16 (N
// rounded up to 16), j < N64 (rounded up to 64), zero outside N x N; the
// host checks |D|, |F| <= 16383.  Stored in MFMA operand order: block
// (t, c) of 1 KB holds rows 16 t .. 16 t + 15 and columns 64 c .. 64 c + 63,
// lane l's 16 bytes (row 16 t + l % 16, columns 64 c + 16 (l / 16) ..) at
// 16 l, so one operand load per wave is one contiguous 1 KB read.
__global__ void large_copy8_kernel(int N, int N16, int N64, const int32_t *D, const int32_t *F,
                                   int8_t *out) {
    const int64_t plane = (int64_t)N16 * N64;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * plane;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = e < plane ? e : e - plane;
        const int64_t blk = w >> 10, l = (w >> 4) & 63, byte = w & 15;
        const int64_t NC = N64 / 64, t = blk / NC, c = blk - t * NC;
        const int64_t k = 16 * t + (l & 15), jj = 64 * c + 16 * (l >> 4) + byte;
        const int32_t *M = e < plane ? D : F;
        const int32_t x = (k < N && jj < N) ? M[k * N + jj] : 0;
        int8_t *base = out + (e < plane ? 0 : 2 * plane);
        base[w] = (int8_t)(x >> 7);
        base[plane + w] = (int8_t)(x & 127);
    }
}

}  // namespace

LargePlan large_plan(int N, const InstanceStats &st) {
    LargePlan pl;
    const int32_t mx = st.max_abs_d > st.max_abs_f ? st.max_abs_d : st.max_abs_f;
    pl.narrow = mx < (1 << 23) &&
                (int64_t)kRowBlock * st.max_abs_d * st.max_abs_f < ((int64_t)1 << 31);
    pl.elem = mx <= 32767 ? 2 : 4;
    pl.planes = mx <= 16383;
    if (pl.planes) {
        pl.elem = 1;
        pl.rows = (N + 15) & ~15;  // rows of a plane, N64 bytes each
        pl.bytes = 4 * (size_t)pl.rows * ((N + 63) & ~63);
    } else if (pl.elem == 2) {
        pl.rows = ((N + 63) & ~63) / 2 + 4;  // word rows
        pl.bytes = 2 * (size_t)pl.rows * ((N + 3) & ~3) * 4;
    } else {
        pl.rows = (N + 2 * kRowBlock - 1) / (2 * kRowBlock) * (2 * kRowBlock) + kRowBlock;
        pl.bytes = 2 * (size_t)pl.rows * N * 4;
    }
    return pl;
}

hipError_t launch_large_copy(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                             const LargePlan &pl, void *buf, LargeCopies *out) {
    const size_t one = pl.bytes / 2;
    out->D = buf;
    out->F = (char *)buf + one;
    const int64_t total = (int64_t)pl.rows * ((N + 3) & ~3);
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 1024);
    if (pl.planes)
        large_copy8_kernel<<<grid, 256, 0, s>>>(N, pl.rows, (N + 63) & ~63, D, F, (int8_t *)buf);
    else if (pl.elem == 2)
        large_copy16_kernel<<<grid, 256, 0, s>>>(N, pl.rows, D, F, (uint32_t *)out->D,
                                                 (uint32_t *)out->F);
    else
        large_copy32_kernel<<<grid, 256, 0, s>>>(N, pl.rows, D, F, (int32_t *)out->D,
                                                 (int32_t *)out->F);
    return hipGetLastError();
}

hipError_t launch_sweep_large_persistent(hipStream_t s, const LargePlan &pl, bool h64,
                                         const BatchArgs &b, int grid) {
#define PDIT_LARGE_P(PAIRS, NARROW)                                                          \
    do {                                                                                     \
        if (h64)                                                                             \
            sweep_large_persistent<PAIRS, NARROW, int64_t, false><<<grid, kLargeThreads, 0, s>>>(b); \
        else                                                                                 \
            sweep_large_persistent<PAIRS, NARROW, int32_t, false><<<grid, kLargeThreads, 0, s>>>(b); \
    } while (0)
    if (pl.planes) {
        if (h64)
            sweep_large_persistent<true, true, int64_t, true><<<grid, kLargeThreads, 0, s>>>(b);
        else
            sweep_large_persistent<true, true, int32_t, true><<<grid, kLargeThreads, 0, s>>>(b);
    } else if (pl.elem == 2 && pl.narrow)
        PDIT_LARGE_P(true, true);
    else if (pl.elem == 2)
        PDIT_LARGE_P(true, false);
    else if (pl.narrow)
        PDIT_LARGE_P(false, true);
    else
        PDIT_LARGE_P(false, false);
#undef PDIT_LARGE_P
    return hipGetLastError();
}

int large_blocks_per_cu(const LargePlan &pl) {
    int n = 0;
    const hipError_t e =
        pl.planes      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &n, sweep_large_persistent<true, true, int64_t, true>, kLargeThreads, 0)
        : pl.elem == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &n, sweep_large_persistent<true, true, int64_t, false>, kLargeThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &n, sweep_large_persistent<false, true, int64_t, false>, kLargeThreads, 0);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_sweep_large(hipStream_t s, const SweepArgs &a, bool h64, const LargePlan &pl,
                              const LargeCopies &c) {
    if (a.N > kLargeNMax || a.N < 2) return hipErrorInvalidValue;
#define PDIT_LARGE(PAIRS, NARROW)                                                               \
    do {                                                                                    \
        if (h64)                                                                            \
            sweep_large_kernel<PAIRS, NARROW, int64_t, false><<<a.R, kLargeThreads, 0, s>>>(a, c); \
        else                                                                                \
            sweep_large_kernel<PAIRS, NARROW, int32_t, false><<<a.R, kLargeThreads, 0, s>>>(a, c); \
    } while (0)
    if (pl.planes) {
        if (h64)
            sweep_large_kernel<true, true, int64_t, true><<<a.R, kLargeThreads, 0, s>>>(a, c);
        else
            sweep_large_kernel<true, true, int32_t, true><<<a.R, kLargeThreads, 0, s>>>(a, c);
    } else if (pl.elem == 2 && pl.narrow)
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
