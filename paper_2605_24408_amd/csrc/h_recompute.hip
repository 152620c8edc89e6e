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
// MFMA: one block (4 waves) per 64x64 tile of one replica's H; K in chunks of
// 64.  Both operands are staged in LDS as [index][k] rows: A = D (rows i),
// B = F[p,p] (rows k of the output; F[p,p] is symmetric, so its rows are the
// columns the product needs).  Each wave owns 16 output rows and the 4
// 16-column subtiles of the tile.
//
// Operand layout of the 16x16 MFMAs: lane l supplies row (l % 16) of A and
// column (l % 16) of B, each with the same group of k values selected by
// l / 16; the result holds C[4 (l / 16) + e][l % 16] in element e.  The order
// of k inside a group is immaterial as long as A and B use the same one.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kTile = 64;
constexpr int kPad = 16;  // bytes of padding per LDS row

enum { kModeI8 = 0, kModeBF16 = 1, kModeSplit = 2 };

__device__ __forceinline__ int8_t lo7(int32_t x) { return (int8_t)(x & 127); }
__device__ __forceinline__ int8_t hi7(int32_t x) { return (int8_t)(x >> 7); }  // floor(x / 128)

template <int MODE, typename HT, bool GL>
__global__ void __launch_bounds__(256) h_mfma_kernel(int N, int tiles, const int32_t *__restrict__ D,
                                                     const int32_t *__restrict__ F,
                                                     const int32_t *__restrict__ perm,
                                                     HT *__restrict__ H) {
    // element size of one staged operand row: int8 (i8, split planes) or bf16
    constexpr int kElem = MODE == kModeBF16 ? 2 : 1;
    constexpr int kRow = kTile * kElem + kPad;
    constexpr int kPlanes = MODE == kModeSplit ? 2 : 1;
    __shared__ __attribute__((aligned(16))) unsigned char As[kPlanes][kTile * kRow];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[kPlanes][kTile * kRow];
    __shared__ int32_t p[PDIT_NMAX];

    const int64_t blk = blockIdx.x;
    const int tiles2 = tiles * tiles;
    const int64_t rep = blk / tiles2;
    const int tm = (int)(blk % tiles2) / tiles, tn = (int)(blk % tiles2) % tiles;
    const int32_t *pr = perm + rep * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) p[j] = pr[j];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kAcc = MODE == kModeSplit ? 4 : 1;
    v4i acc_i[kAcc][4];
    v4f acc_f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        acc_f[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kAcc; ++q) acc_i[q][j] = v4i{0, 0, 0, 0};
    }

    const int kchunks = (N + kTile - 1) / kTile;
    for (int kc = 0; kc < kchunks; ++kc) {
        __syncthreads();
        // stage 64 x 64 of A (D rows tm*64.., k cols kc*64..) and B (F[p,p]
        // rows tn*64.., k cols kc*64..)
        for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
            const int r = e / kTile, c = e % kTile;
            const int gi = tm * kTile + r, gn = tn * kTile + r, gk = kc * kTile + c;
            const bool kin = gk < N;
            const int32_t a = (gi < N && kin) ? D[(int64_t)gi * N + gk] : 0;
            const int32_t b = (gn < N && kin) ? F[(int64_t)(GL ? gn : p[gn]) * N + p[gk]] : 0;
            if constexpr (MODE == kModeI8) {
                As[0][r * kRow + c] = (unsigned char)(int8_t)a;
                Bs[0][r * kRow + c] = (unsigned char)(int8_t)b;
            } else if constexpr (MODE == kModeSplit) {
                As[0][r * kRow + c] = (unsigned char)lo7(a);
                As[1][r * kRow + c] = (unsigned char)hi7(a);
                Bs[0][r * kRow + c] = (unsigned char)lo7(b);
                Bs[1][r * kRow + c] = (unsigned char)hi7(b);
            } else {
                reinterpret_cast<__bf16 *>(&As[0][r * kRow])[c] = (__bf16)(float)a;
                reinterpret_cast<__bf16 *>(&Bs[0][r * kRow])[c] = (__bf16)(float)b;
            }
        }
        __syncthreads();
        const int arow = wave * 16 + (lane & 15);
        const int grp = lane >> 4;
        if constexpr (MODE == kModeBF16) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                // k values [half*32 + grp*8, +8)
                const int kb = (half * 32 + grp * 8) * 2;
                const v8bf a = *reinterpret_cast<const v8bf *>(&As[0][arow * kRow + kb]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
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
            for (int j = 0; j < 4; ++j) {
                const int brow = j * 16 + (lane & 15);
                v4i b[kPlanes];
#pragma unroll
                for (int q = 0; q < kPlanes; ++q)
                    b[q] = *reinterpret_cast<const v4i *>(&Bs[q][brow * kRow + kb]);
                if constexpr (MODE == kModeI8) {
                    acc_i[0][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[0], acc_i[0][j], 0, 0, 0);
                } else {
                    // planes: 0 = lo, 1 = hi; acc 0 = lo*lo, 1 = lo*hi, 2 = hi*lo, 3 = hi*hi
                    acc_i[0][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[0], acc_i[0][j], 0, 0, 0);
                    acc_i[1][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[1], acc_i[1][j], 0, 0, 0);
                    acc_i[2][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], b[0], acc_i[2][j], 0, 0, 0);
                    acc_i[3][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], b[1], acc_i[3][j], 0, 0, 0);
                }
            }
        }
    }

    // write back: element e of subtile j is C[4*(lane/16) + e][lane % 16]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = tm * kTile + wave * 16 + 4 * (lane >> 4) + e;
            const int gk = tn * kTile + j * 16 + (lane & 15);
            if (gi < N && gk < N) {
                int64_t v;
                if constexpr (MODE == kModeI8) {
                    v = acc_i[0][j][e];
                } else if constexpr (MODE == kModeSplit) {
                    v = (int64_t)acc_i[0][j][e] + ((int64_t)acc_i[1][j][e] + acc_i[2][j][e]) * 128 +
                        (int64_t)acc_i[3][j][e] * 16384;
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

hipError_t launch_h_recompute_mfma(hipStream_t s, int mode, int N, const int32_t *D,
                                   const int32_t *F, int R, const int32_t *perm, void *H,
                                   bool h64, int64_t *E, bool g_layout) {
    const int tiles = (N + kTile - 1) / kTile;
    const int64_t blocks = (int64_t)R * tiles * tiles;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    int kmode;
    if (mode == PDIT_RECOMPUTE_I8) kmode = kModeI8;
    else if (mode == PDIT_RECOMPUTE_BF16) kmode = kModeBF16;
    else if (mode == PDIT_RECOMPUTE_SPLIT) kmode = kModeSplit;
    else return hipErrorInvalidValue;
#define PDIT_LAUNCH(MODE, HT, GL) \
    h_mfma_kernel<MODE, HT, GL><<<(unsigned)blocks, 256, 0, s>>>(N, tiles, D, F, perm, (HT *)H)
#define PDIT_LAUNCH_MODES(HT, GL)                                                      \
    {                                                                                  \
        if (kmode == kModeI8) PDIT_LAUNCH(kModeI8, HT, GL);                            \
        else if (kmode == kModeBF16) PDIT_LAUNCH(kModeBF16, HT, GL);                   \
        else PDIT_LAUNCH(kModeSplit, HT, GL);                                          \
        trace_kernel<HT, GL><<<R, 256, 0, s>>>(N, (const HT *)H, perm, E);             \
    }
    if (h64) {
        if (g_layout) PDIT_LAUNCH_MODES(int64_t, true) else PDIT_LAUNCH_MODES(int64_t, false)
    } else {
        if (g_layout) PDIT_LAUNCH_MODES(int32_t, true) else PDIT_LAUNCH_MODES(int32_t, false)
    }
#undef PDIT_LAUNCH_MODES
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
