// h_recompute.hip -- step "H recompute": for every replica, the influence
// matrix H = D F[p,p] (H_ik = sum_j D_ij F_{p(j) p(k)}; for symmetric data
// the influence of Eq. 2 is I_i^{p(k)} = -2 H_ik) and the energy
// E = trace(H) = Eq. 1.  The G layout (for the register sweep kernel) keeps
// the columns by facility instead: G = D F[p,:], G_ic = sum_j D_ij
// F_{p(j) c}, so H_ik = G_{i p(k)} and E = sum_i G_{i p(i)}.
//
// Variants (all exact for the data they accept):
//   plain  vector ALU, int64 accumulation;
//   i8     int8 MFMA (v_mfma_i32_16x16x64_i8), int32 accumulation;
//          needs |D|, |F| <= 127 and |H| < 2^31;
//   bf16   bf16 MFMA (v_mfma_f32_16x16x32_bf16), fp32 accumulation; integers
//          up to 256 are exact in bf16 and every partial sum stays below 2^24,
//          so the float sums are exact integers in any order;
//   split  7-bit byte planes x = 128 x_hi + x_lo (x_lo in [0,127], x_hi in
//          [-128,127]), four int8 MFMA products accumulated in int32
//          (|sum| <= N * 128 * 127 < 2^31 for N <= 512), combined in int64 as
//          2^14 hi*hi + 2^7 (hi*lo + lo*hi) + lo*lo.
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

// ---------------------------------------------------------------------------
// plain: one block per (row i, replica); threads over columns k.
// ---------------------------------------------------------------------------
template <typename HT, bool GL>
__global__ void __launch_bounds__(256) h_plain_kernel(int N, const int32_t *__restrict__ D,
                                                      const int32_t *__restrict__ F,
                                                      const int32_t *__restrict__ perm,
                                                      HT *__restrict__ H) {
    __shared__ int32_t p[PDIT_NMAX];
    __shared__ int32_t drow[PDIT_NMAX];
    const int i = blockIdx.x;
    const int64_t rep = blockIdx.y;
    const int32_t *pr = perm + rep * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        p[j] = pr[j];
        drow[j] = D[(int64_t)i * N + j];
    }
    __syncthreads();
    HT *out = H + (rep * N + i) * (int64_t)N;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const int pk = GL ? k : p[k];
        int64_t acc = 0;
        for (int j = 0; j < N; ++j) acc += (int64_t)drow[j] * F[(int64_t)p[j] * N + pk];
        out[k] = (HT)acc;
    }
}

// E[rep] = sum_i H[rep][i][i] (G layout: sum_i G[rep][i][p(i)]); one block
// per replica.
template <typename HT, bool GL>
__global__ void __launch_bounds__(256) trace_kernel(int N, const HT *__restrict__ H,
                                                    const int32_t *__restrict__ perm,
                                                    int64_t *__restrict__ E) {
    __shared__ int64_t part[256];
    const int64_t rep = blockIdx.x;
    int64_t s = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        s += (int64_t)H[(rep * N + i) * N + (GL ? perm[rep * N + i] : i)];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[rep] = part[0];
}

__global__ void widen_kernel(int64_t count, const int32_t *__restrict__ src,
                             int64_t *__restrict__ dst) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

// ---------------------------------------------------------------------------
// MFMA.  With F symmetric, H_ik = sum_m D'_im F_{p(k) m} where D'_im =
// D_{i p^-1(m)} (m = p(j)), and G_ic = sum_m D'_im F_{c m}: the second operand
// is whole rows of F (row p(k) for H, row c for G), read 16 bytes at a time,
// and only the first is gathered, inside rows of D.  D and F are first
// converted once per call to the operand format (bf16 bits, int8, or for
// split the 7-bit planes: D as (lo, hi) byte pairs, F as two planes), with
// rows padded with zeros to a pitch ld = N rounded up to 64.
//
// One block (4 waves) computes a 64 x TN tile of one replica; wave w owns
// rows 16w..16w+15 and the TN/16 column subtiles; K runs in chunks of 64
// staged in LDS as [row][k].  Operand layout of the 16x16 MFMAs: lane l
// supplies row (l % 16) of A and column (l % 16) of B, each with the same
// group of k values selected by l / 16; the result holds C[4 (l / 16) + e]
// [l % 16] in element e.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kTile = 64;  // rows of a block's tile
constexpr int kKC = 64;    // k of one staged chunk
constexpr int kPad = 16;   // bytes of padding per LDS row

enum { kModeI8 = 0, kModeBF16 = 1, kModeSplit = 2 };

__device__ __forceinline__ int8_t lo7(int32_t x) { return (int8_t)(x & 127); }
__device__ __forceinline__ int8_t hi7(int32_t x) { return (int8_t)(x >> 7); }  // floor(x / 128)
__device__ __forceinline__ uint16_t bf16_bits(int32_t x) {  // exact for |x| <= 256
    return __builtin_bit_cast(uint16_t, (__bf16)(float)x);
}

inline int64_t operand_pitch(int N) { return ((int64_t)N + 63) / 64 * 64; }

// D and F in operand format (layout above): bf16 D then F (2 bytes each);
// i8 D then F; split D pairs (2 bytes), then F's low and high planes
template <int MODE>
__global__ void __launch_bounds__(256) operand_prep_kernel(int N, int ld,
                                                           const int32_t *__restrict__ D,
                                                           const int32_t *__restrict__ F,
                                                           unsigned char *__restrict__ out) {
    const int64_t n2 = (int64_t)ld * ld;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), j = (int)(e % ld);
        const bool in = i < N && j < N;
        const int32_t d = in ? D[(int64_t)i * N + j] : 0;
        const int32_t f = in ? F[(int64_t)i * N + j] : 0;
        if constexpr (MODE == kModeBF16) {
            ((uint16_t *)out)[e] = bf16_bits(d);
            ((uint16_t *)out)[n2 + e] = bf16_bits(f);
        } else if constexpr (MODE == kModeI8) {
            ((int8_t *)out)[e] = (int8_t)d;
            ((int8_t *)out)[n2 + e] = (int8_t)f;
        } else {
            ((uint16_t *)out)[e] = (uint16_t)((uint8_t)lo7(d) | ((uint16_t)(uint8_t)hi7(d) << 8));
            ((int8_t *)out)[2 * n2 + e] = lo7(f);
            ((int8_t *)out)[3 * n2 + e] = hi7(f);
        }
    }
}

template <int MODE, typename HT, bool GL, int TN>
__global__ void __launch_bounds__(256) h_mfma_kernel(int N, int ld, int mtiles, int ntiles,
                                                     const unsigned char *__restrict__ ops,
                                                     const int32_t *__restrict__ perm,
                                                     HT *__restrict__ H) {
    constexpr int kElem = MODE == kModeBF16 ? 2 : 1;   // bytes per element of a plane
    constexpr int kPlanes = MODE == kModeSplit ? 2 : 1;
    constexpr int kRow = kKC * kElem + kPad;           // LDS row pitch (bytes)
    constexpr int kSub = TN / 16;                      // column subtiles per wave
    __shared__ __attribute__((aligned(16))) unsigned char As[kPlanes][kTile * kRow];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[kPlanes][TN * kRow];
    __shared__ int32_t p[PDIT_NMAX];
    __shared__ int32_t pinv[PDIT_NMAX];

    const int64_t per_rep = (int64_t)mtiles * ntiles;
    const int64_t rep = blockIdx.x / per_rep;
    const int t = (int)(blockIdx.x % per_rep);
    const int tm = t / ntiles, tn = t % ntiles;
    const int32_t *pr = perm + rep * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) p[j] = pr[j];
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) pinv[p[j]] = j;

    const int64_t n2 = (int64_t)ld * ld;
    const unsigned char *Fb = ops + (MODE == kModeI8 ? n2 : 2 * n2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int kAcc = MODE == kModeSplit ? 3 : 1;   // split: lo*lo, lo*hi + hi*lo, hi*hi
    v4i acc_i[kAcc][kSub];
    v4f acc_f[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
        acc_f[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kAcc; ++q) acc_i[q][j] = v4i{0, 0, 0, 0};
    }
    // A staging: D symmetric makes D'[i][m] = D[p^-1(m)][i], so a chunk of A
    // is 64 rows p^-1(m) of D read along the tile's rows i (16 bytes at a
    // time: kAP pieces per thread) and transposed into [i][m] as it is
    // written to LDS; B staging: kBU 16-byte pieces of rows of F per thread
    constexpr int kAE = MODE == kModeI8 ? 1 : 2;       // bytes per element of D in memory
    constexpr int kAPR = kTile * kAE / 16;             // 16-byte pieces per row of the A chunk
    constexpr int kAP = kKC * kAPR / 256;              // ... per thread
    constexpr int kUnits = kKC * kElem / 16;           // 16-byte pieces per B row and plane
    constexpr int kBU = TN * kUnits * kPlanes / 256;
    static_assert(TN * kUnits * kPlanes % 256 == 0 && kKC * kAPR % 256 == 0, "pieces per thread");
    v4i aw[kAP];
    v4i bw[kBU];
    // chunk kc of A and B into registers
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int w = 0; w < kAP; ++w) {
            const int u = tid + 256 * w;
            const int mr = u / kAPR, pc = u % kAPR;
            const int m = kc * kKC + mr;
            v4i x = v4i{0, 0, 0, 0};
            if (m < N)
                x = *(const v4i *)(ops + ((int64_t)pinv[m] * ld + tm * kTile) * kAE + pc * 16);
            aw[w] = x;
        }
#pragma unroll
        for (int w = 0; w < kBU; ++w) {
            const int u = tid + 256 * w;
            const int pl = u / (TN * kUnits);
            const int rem = u % (TN * kUnits);
            const int rr = rem / kUnits, pc = rem % kUnits;
            const int n = tn * TN + rr;
            v4i x = v4i{0, 0, 0, 0};
            if (n < N) {
                const int q = GL ? n : p[n];
                x = *(const v4i *)(Fb + pl * n2 + ((int64_t)q * ld + kc * kKC) * kElem + pc * 16);
            }
            bw[w] = x;
        }
    };
    auto store_chunk = [&]() {
        // element e of piece (mr, pc) is D'[i][m] for i = pc * 16 / kAE + e
#pragma unroll
        for (int w = 0; w < kAP; ++w) {
            const int u = tid + 256 * w;
            const int mr = u / kAPR, pc = u % kAPR;
            const uint32_t word[4] = {(uint32_t)aw[w].x, (uint32_t)aw[w].y, (uint32_t)aw[w].z,
                                      (uint32_t)aw[w].w};
            if constexpr (MODE == kModeI8) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    As[0][(pc * 16 + e) * kRow + mr] = (unsigned char)(word[e >> 2] >> (8 * (e & 3)));
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t v = (word[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                    const int i = pc * 8 + e;
                    if constexpr (MODE == kModeBF16) {
                        *(uint16_t *)&As[0][i * kRow + 2 * mr] = (uint16_t)v;
                    } else {   // split: (lo, hi) byte pair to the two planes
                        As[0][i * kRow + mr] = (unsigned char)(v & 0xFF);
                        As[1][i * kRow + mr] = (unsigned char)(v >> 8);
                    }
                }
            }
        }
#pragma unroll
        for (int w = 0; w < kBU; ++w) {
            const int u = tid + 256 * w;
            const int pl = u / (TN * kUnits);
            const int rem = u % (TN * kUnits);
            const int rr = rem / kUnits, pc = rem % kUnits;
            *(v4i *)&Bs[pl][rr * kRow + pc * 16] = bw[w];
        }
    };

    const int nk = ld / kKC;
    __syncthreads();   // pinv complete
    load_chunk(0);
    for (int kc = 0; kc < nk; ++kc) {
        __syncthreads();   // the previous chunk's products have read the LDS tiles
        store_chunk();
        __syncthreads();
        // the next chunk's loads are in flight during this chunk's products
        if (kc + 1 < nk) load_chunk(kc + 1);
        const int arow = wave * 16 + (lane & 15);
        const int grp = lane >> 4;
        if constexpr (MODE == kModeBF16) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                // k values [half*32 + grp*8, +8)
                const int kb = (half * 32 + grp * 8) * 2;
                const v8bf a = *reinterpret_cast<const v8bf *>(&As[0][arow * kRow + kb]);
#pragma unroll
                for (int j = 0; j < kSub; ++j) {
                    const int brow = j * 16 + (lane & 15);
                    const v8bf b = *reinterpret_cast<const v8bf *>(&Bs[0][brow * kRow + kb]);
                    acc_f[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc_f[j], 0, 0, 0);
                }
            }
        } else {
            const int kb = grp * 16;  // k values [grp*16, +16)
            v4i a[kPlanes];
#pragma unroll
            for (int q = 0; q < kPlanes; ++q)
                a[q] = *reinterpret_cast<const v4i *>(&As[q][arow * kRow + kb]);
#pragma unroll
            for (int j = 0; j < kSub; ++j) {
                const int brow = j * 16 + (lane & 15);
                v4i b[kPlanes];
#pragma unroll
                for (int q = 0; q < kPlanes; ++q)
                    b[q] = *reinterpret_cast<const v4i *>(&Bs[q][brow * kRow + kb]);
                if constexpr (MODE == kModeI8) {
                    acc_i[0][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[0], acc_i[0][j], 0, 0, 0);
                } else {
                    // planes: 0 = lo, 1 = hi; |lo*hi + hi*lo| summed over k <= 2 N 127 128 < 2^31
                    acc_i[0][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[0], acc_i[0][j], 0, 0, 0);
                    acc_i[1][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[1], acc_i[1][j], 0, 0, 0);
                    acc_i[1][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], b[0], acc_i[1][j], 0, 0, 0);
                    acc_i[2][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], b[1], acc_i[2][j], 0, 0, 0);
                }
            }
        }
    }

    // write back: element e of subtile j is C[4*(lane/16) + e][lane % 16]
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = tm * kTile + wave * 16 + 4 * (lane >> 4) + e;
            const int gk = tn * TN + j * 16 + (lane & 15);
            if (gi < N && gk < N) {
                int64_t v;
                if constexpr (MODE == kModeI8) {
                    v = acc_i[0][j][e];
                } else if constexpr (MODE == kModeSplit) {
                    v = (int64_t)acc_i[0][j][e] + (int64_t)acc_i[1][j][e] * 128 +
                        (int64_t)acc_i[2][j][e] * 16384;
                } else {
                    v = (int64_t)acc_f[j][e];
                }
                H[(rep * N + gi) * (int64_t)N + gk] = (HT)v;
            }
        }
    }
}

}  // namespace

hipError_t launch_h_recompute_plain(hipStream_t s, int N, const int32_t *D, const int32_t *F,
                                    int R, const int32_t *perm, void *H, bool h64, int64_t *E,
                                    bool g_layout) {
    dim3 grid(N, R);
#define PDIT_LAUNCH(HT, GL)                                                            \
    {                                                                                  \
        h_plain_kernel<HT, GL><<<grid, 256, 0, s>>>(N, D, F, perm, (HT *)H);           \
        trace_kernel<HT, GL><<<R, 256, 0, s>>>(N, (const HT *)H, perm, E);             \
    }
    if (h64) {
        if (g_layout) PDIT_LAUNCH(int64_t, true) else PDIT_LAUNCH(int64_t, false)
    } else {
        if (g_layout) PDIT_LAUNCH(int32_t, true) else PDIT_LAUNCH(int32_t, false)
    }
#undef PDIT_LAUNCH
    return hipGetLastError();
}

size_t mfma_operand_bytes(int mode, int N) {
    if (mode == PDIT_RECOMPUTE_PLAIN) return 0;
    const int64_t ld = operand_pitch(N);
    return (size_t)(mode == PDIT_RECOMPUTE_I8 ? 2 : 4) * (size_t)(ld * ld);
}

hipError_t launch_h_recompute_mfma(hipStream_t s, int mode, int N, const int32_t *D,
                                   const int32_t *F, int R, const int32_t *perm, void *H,
                                   bool h64, int64_t *E, bool g_layout, void *operands) {
    int kmode;
    if (mode == PDIT_RECOMPUTE_I8) kmode = kModeI8;
    else if (mode == PDIT_RECOMPUTE_BF16) kmode = kModeBF16;
    else if (mode == PDIT_RECOMPUTE_SPLIT) kmode = kModeSplit;
    else return hipErrorInvalidValue;
    if (!operands) return hipErrorInvalidValue;
    const int ld = (int)operand_pitch(N);
    // the column tile: the whole padded row up to 256 (128 in split mode,
    // whose three accumulator sets would not fit 256; 64 measured no faster)
    const int cap = kmode == kModeSplit ? 128 : 256;
    const int tn = ld < cap ? ld : cap;           // 64, 128 or 256 (ld is a multiple of 64)
    const int width = tn == 192 ? 256 : tn;
    const int mtiles = (N + kTile - 1) / kTile;
    const int ntiles = (N + width - 1) / width;
    const int64_t blocks = (int64_t)R * mtiles * ntiles;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    unsigned char *ops = (unsigned char *)operands;
    {
        const int64_t n2 = (int64_t)ld * ld;
        const int g = (int)((n2 + 255) / 256 < 4096 ? (n2 + 255) / 256 : 4096);
        if (kmode == kModeI8) operand_prep_kernel<kModeI8><<<g, 256, 0, s>>>(N, ld, D, F, ops);
        else if (kmode == kModeBF16) operand_prep_kernel<kModeBF16><<<g, 256, 0, s>>>(N, ld, D, F, ops);
        else operand_prep_kernel<kModeSplit><<<g, 256, 0, s>>>(N, ld, D, F, ops);
    }
#define PDIT_LAUNCH(MODE, HT, GL, TN)                                                  \
    h_mfma_kernel<MODE, HT, GL, TN><<<(unsigned)blocks, 256, 0, s>>>(N, ld, mtiles, ntiles, ops, \
                                                                    perm, (HT *)H)
#define PDIT_LAUNCH_TN(MODE, HT, GL)                                                   \
    {                                                                                  \
        if (width == 64) PDIT_LAUNCH(MODE, HT, GL, 64);                                \
        else if (width == 128) PDIT_LAUNCH(MODE, HT, GL, 128);                         \
        else if (MODE != kModeSplit) PDIT_LAUNCH(MODE, HT, GL, (MODE == kModeSplit ? 128 : 256)); \
    }
#define PDIT_LAUNCH_MODES(HT, GL)                                                      \
    {                                                                                  \
        if (kmode == kModeI8) PDIT_LAUNCH_TN(kModeI8, HT, GL)                          \
        else if (kmode == kModeBF16) PDIT_LAUNCH_TN(kModeBF16, HT, GL)                 \
        else PDIT_LAUNCH_TN(kModeSplit, HT, GL)                                        \
        trace_kernel<HT, GL><<<R, 256, 0, s>>>(N, (const HT *)H, perm, E);             \
    }
    if (h64) {
        if (g_layout) PDIT_LAUNCH_MODES(int64_t, true) else PDIT_LAUNCH_MODES(int64_t, false)
    } else {
        if (g_layout) PDIT_LAUNCH_MODES(int32_t, true) else PDIT_LAUNCH_MODES(int32_t, false)
    }
#undef PDIT_LAUNCH_MODES
#undef PDIT_LAUNCH_TN
#undef PDIT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_widen_h(hipStream_t s, int64_t count, const int32_t *src, int64_t *dst) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    widen_kernel<<<(unsigned)blocks, 256, 0, s>>>(count, src, dst);
    return hipGetLastError();
}

}  // namespace pdit
