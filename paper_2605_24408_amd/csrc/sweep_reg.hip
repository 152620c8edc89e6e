// sweep_reg.hip -- the sweep kernel that keeps a replica's state in
// registers, for 128 < N <= 256 with D and F held as 8-bit copies.
//
// The state is G = D F[p,:] (location x facility): G[i][c] = sum_j D[i][j]
// F[p(j)][c], so H = D F[p,p] is H[i][k] = G[i][p(k)].  An accepted exchange
// of the facilities a = p(r) and b = p(s) changes G by one rank-1 term and
// moves no column (Methods, "CPU-PIM Algorithm": the influence is kept
// incrementally; with symmetric data I = -2H, Eq. 2):
//   G'[i][c] = G[i][c] + u_i w_c,  u_i = D[i][r] - D[i][s],
//                                   w_c = F[b][c] - F[a][c].
//
// A replica has four waves.  Lane j of wave w holds the 4 x 64 tile of G at
// rows 4j .. 4j + 3 and facilities 64w .. 64w + 63, as packed int16 pairs
// (exact while |H| <= 32767): 128 registers, and an accepted exchange costs
// 128 packed multiply-adds per lane, with w read for the wave's 64
// facilities only.
//
// The update of location r (Results, "Implementation": locations 0..N-1 in
// order; Eq. 3 and Eq. 5) needs row r of G (H[r][k] = G[r][p(k)]) and the
// column of G at a = p(r) (H[k][r] = G[k][a]).  Before each update the waves
// publish exactly these two vectors to LDS (the lane holding row r writes
// its 64 entries in every wave; the wave holding facility a writes the
// column) and wait for each other: that is the only exchange between waves.
// Then every wave evaluates all N candidates itself, four consecutive
// locations per lane,
//   dE_k = 2 (H[r][k] - H[r][r] + H[k][r] - H[k][k])
//          + (D_rr + D_kk - 2 D_rk)(F_aa + F_cc - 2 F_ac),  c = p(k),
// with H[k][k], p and the diagonals of D and F kept per candidate in its
// registers, takes the row minimum, the integer Gibbs weights
// q = rint(expf(-beta d) 2^25) and their exact 64-bit CDF in location
// order, as the other sweep kernels do, and draws the same candidate: the
// four waves reach the same decision with no message.  A row whose only
// nonzero weight is its own stay (every other candidate lies at or beyond the
// zero-weight distance above 0) keeps its facility without weights or scan.
//
// Batches.  An update that keeps its facility changes nothing, so when few
// exchanges are accepted the updates of locations r0 .. r0 + 11 can all be
// evaluated on the same state: the waves publish the 12 rows and columns
// together, each wave evaluates three of the updates, and the stays up to
// the first exchange are committed.  The update with that exchange then runs
// as a single update on the batch's row and column (it draws the same
// candidate, the state being the one it was evaluated on) and the next batch
// starts after it.  Every draw is the sequential one; a sweep runs in
// batches when the sweep before it accepted at most kRSpecAcc exchanges.
//
// Two replicas share a workgroup (eight waves, each SIMD holding one wave of
// each) and its LDS: D and F as 8-bit copies (64 KB each, unsigned in
// [0, 255] or signed in [-128, 127]), so every read of D and F on the path
// is an LDS read.  The replicas wait only for their own waves.
#include "device_common.h"
#include "pdit_internal.h"
#include "sweep_common.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int kRN = 256;          // locations (and facilities) per replica
constexpr int kRWaves = 4;        // waves per replica
constexpr int kRReps = 2;         // replicas per workgroup
constexpr int kRThreads = 64 * kRWaves * kRReps;
constexpr int32_t kRBig = (1 << 30) - 1;  // padding candidates (|dE| < 2^30 - 1)
// Batches: kRSpec consecutive updates evaluated on one state (kRSpec / kRWaves
// per wave) when the previous sweep accepted at most kRSpecAcc exchanges
constexpr int kRSpec = 12;
constexpr int kRSpecAcc = 48;
// spins of a replica's wait before it gives up (about 0.1 s): reached only
// if a wave of the replica stopped taking part, which the kernel's uniform
// control flow excludes; the call then reports PDIT_EDEVICE at pdit_sync
constexpr uint32_t kRSpinLimit = 1u << 22;

typedef int v32i __attribute__((ext_vector_type(32)));
typedef short v64s __attribute__((ext_vector_type(64)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

struct alignas(16) RegRep {
    union {
        struct {                               // one update at a time
            alignas(16) int16_t prow[2][kRN];  // row r of G by facility (by update parity)
            alignas(16) int16_t pcol[2][kRN];  // column p(r) of G by location
        } sq;
        struct {                               // a batch of kRSpec updates
            alignas(16) int16_t brow[kRSpec][kRN];
            alignas(16) int16_t bcol[kRSpec][kRN];
        } sp;
        alignas(16) int16_t stage[kRWaves][16][64];  // set-up: rows of G on their way to the tiles
    } u;
    alignas(16) int16_t w[kRWaves][kRN];       // per wave: the accepted exchange's w, by facility
    alignas(16) v4i outc[kRSpec];              // batch: per update its draw s and tie flag
    alignas(16) uint32_t sync[kRWaves];        // per wave: the last step it finished
};

template <bool SGN>
struct RegSmem {
    using E8 = typename std::conditional<SGN, int8_t, uint8_t>::type;
    E8 D[kRN * kRN];             // D, zero outside N x N
    E8 F[kRN * kRN];             // F, zero outside N x N
    RegRep rep[kRReps];
};

__device__ __forceinline__ uint32_t pack16(int32_t lo, int32_t hi) {
    return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
}

// byte t of a packed word of four 8-bit entries, widened
template <bool SGN>
__device__ __forceinline__ int32_t byte_at(uint32_t x, int t) {
    return SGN ? (int32_t)(int8_t)(x >> (8 * t)) : (int32_t)((x >> (8 * t)) & 0xFFu);
}

// g += u w elementwise on int16 lanes (modulo 2^16; the true values fit)
__device__ __forceinline__ v32i rank1(v32i g, short u, v32i w) {
    const v64s gs = __builtin_bit_cast(v64s, g);
    const v64s ws = __builtin_bit_cast(v64s, w);
    return __builtin_bit_cast(v32i, gs + (v64s)u * ws);
}

// entry (uniform) facility c of a tile row: register c / 2, half c % 2
__device__ __forceinline__ int32_t tile_entry(const v32i &g, int m, int half) {
    const int word = g[__builtin_amdgcn_readfirstlane(m)];
    return half ? (word >> 16) : (int32_t)(int16_t)(word & 0xFFFF);
}

// value of the candidate slot of location k (uniform): lane k / 4, slot k % 4
__device__ __forceinline__ int32_t pick(const int32_t (&v)[4], int k) {
    const int t = k & 3;
    const int32_t x = t == 0 ? v[0] : t == 1 ? v[1] : t == 2 ? v[2] : v[3];
    return __builtin_amdgcn_readlane(x, k >> 2);
}

typedef __attribute__((address_space(3))) volatile v4i lds_v4i;
typedef __attribute__((address_space(3))) char lds_char;

// LDS byte address of a pointer into the kernel's shared memory
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const lds_char *)p;
}

// 128-byte store of a tile row to LDS (eight 16-byte writes).  Each call site
// passes its own tag, so that the stores of different rows stay separate
// instructions and no copy of a row is formed to merge them.
#define PDIT_REG_STORE_ROW(addr, g, tag)                                                   \
    __asm__ volatile("; tile row " tag "\n\t"                                              \
                     "ds_write_b128 %0, %1\n\t"                                            \
                     "ds_write_b128 %0, %2 offset:16\n\t"                                  \
                     "ds_write_b128 %0, %3 offset:32\n\t"                                  \
                     "ds_write_b128 %0, %4 offset:48\n\t"                                  \
                     "ds_write_b128 %0, %5 offset:64\n\t"                                  \
                     "ds_write_b128 %0, %6 offset:80\n\t"                                  \
                     "ds_write_b128 %0, %7 offset:96\n\t"                                  \
                     "ds_write_b128 %0, %8 offset:112"                                     \
                     :                                                                     \
                     : "v"(addr), "v"((g).s0123), "v"((g).s4567), "v"((g).s89ab),          \
                       "v"((g).scdef), "v"((g).hi.s0123), "v"((g).hi.s4567),               \
                       "v"((g).hi.s89ab), "v"((g).hi.scdef)                                \
                     : "memory")

// Inclusive prefix sum of a 32-bit value across the wave (lane order):
// shifts within rows of 16, then the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ uint32_t scan_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// The waves of a replica meet through one LDS word per wave, not workgroup
// barriers, so the two replicas of a workgroup run independently.  The LDS
// operations of one wave are carried out in the order it issues them, so
// (1) a wave's flag store lands after its publication stores, and (2) a
// read issued after a poll that found every flag set returns the published
// data: a wave issues its poll and the publication's reads back to back and
// pays one LDS round trip for both.
__device__ __forceinline__ void rep_signal(uint32_t *slots, int w, uint32_t seq) {
    __asm__ volatile("" ::: "memory");
    __hip_atomic_store(&slots[w], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ const lds_v4i *rep_flags(uint32_t *slots) {
    return (const lds_v4i *)(__attribute__((address_space(3))) uint32_t *)slots;
}

// every wave of the replica has finished step seq (uniform)
__device__ __forceinline__ bool rep_done(v4i v, uint32_t seq) {
    const bool done = (int32_t)(v.x - seq) >= 0 && (int32_t)(v.y - seq) >= 0 &&
                      (int32_t)(v.z - seq) >= 0 && (int32_t)(v.w - seq) >= 0;
    return __builtin_amdgcn_readfirstlane((int)done) != 0;
}

// Polls until every wave has finished step seq; false when the wait gave up
// (kRSpinLimit).
__device__ __forceinline__ bool rep_spin(const lds_v4i *ps, uint32_t seq) {
    for (uint32_t it = 0; it < kRSpinLimit; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (rep_done(*ps, seq)) {
            __asm__ volatile("" ::: "memory");
            return true;
        }
    }
    return false;
}

template <bool SGN, bool ZD>
__global__ void __launch_bounds__(kRThreads)
sweep_reg_kernel(SweepArgs a) {
    using E8 = typename RegSmem<SGN>::E8;
    __shared__ __align__(16) RegSmem<SGN> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane((tid >> 6) % kRWaves);  // wave in the replica
    const int qr = __builtin_amdgcn_readfirstlane((tid >> 6) / kRWaves);  // replica slot
    const int N = a.N;
    int64_t rep = (int64_t)kRReps * blockIdx.x + qr;
    // an odd last replica: the second slot repeats the first and writes nothing
    const bool live = rep < a.R;
    if (!live) rep = (int64_t)kRReps * blockIdx.x;
    RegRep &rs = sm.rep[qr];
    const uint32_t *D32 = (const uint32_t *)sm.D;
    const uint32_t *F32 = (const uint32_t *)sm.F;

    // ---- D and F copies (both replicas) ----
    for (int e = tid; e < kRN * kRN; e += kRThreads) {
        const int i = e >> 8, j = e & 255;
        const bool in = i < N && j < N;
        sm.D[e] = (E8)(in ? a.D[(int64_t)i * N + j] : 0);
        sm.F[e] = (E8)(in ? a.F[(int64_t)i * N + j] : 0);
    }
    // ---- candidates 4 lane + t: p (padding locations hold the padding facilities) ----
    int32_t pk[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * lane + t;
        pk[t] = k < N ? a.perm[rep * N + k] : k;
    }
    if (lane < kRWaves && wv == 0) rs.sync[lane] = 0;

    // ---- the tile: G[4 lane + t][64 wv + c], from G = D F[p,:] (row k of a
    // replica's N x N block, columns by facility).  Rows 16 q .. 16 q + 15 of
    // the wave's 64 facilities are read along the rows (lane c takes column
    // 64 wv + c), staged in the wave's part of LDS as int16, and
    // read back by the four lanes that hold them; LDS accesses of one wave
    // complete in order, so the wave needs no barrier. ----
    v32i g0, g1, g2, g3;
    {
        const int32_t *Gb = (const int32_t *)a.H + rep * N * (int64_t)N;
        int16_t *stage = rs.u.stage[wv][0];     // 16 rows x 64 facilities
        const int c = 64 * wv + lane;
        for (int q = 0; q < kRN / 16; ++q) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int k = 16 * q + i;
                stage[i * 64 + lane] = (int16_t)((k < N && c < N) ? Gb[k * (int64_t)N + c] : 0);
            }
            __asm__ volatile("" ::: "memory");
            if ((lane >> 2) == q) {
                const v32i *src = (const v32i *)&stage[(4 * (lane & 3)) * 64];
                g0 = src[0];
                g1 = src[1];
                g2 = src[2];
                g3 = src[3];
            }
            __asm__ volatile("" ::: "memory");
        }
    }
    // the D and F copies and the flags are complete before the first reads
    __syncthreads();
    // per candidate: H[k][k] = G[k][p(k)], D[k][k], F[p(k)][p(k)]
    int32_t dg[4], ddk[4], fdk[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * lane + t;
        dg[t] = k < N ? ((const int32_t *)a.H)[(rep * N + k) * (int64_t)N + pk[t]] : 0;
        ddk[t] = ZD ? 0 : (int32_t)sm.D[k * kRN + k];
        fdk[t] = ZD ? 0 : (int32_t)sm.F[pk[t] * kRN + pk[t]];
    }
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0;
    int32_t n_tie = 0;
    int32_t *ch_base = (a.choices && live && wv == 0) ? a.choices + rep * a.T * N : nullptr;
    const float *bp = a.slot ? a.beta + a.slot[rep] : a.beta;
    const int64_t bstride = a.slot ? 0 : 1;
    const bool writer = live && wv == 0;   // wave 0 writes the replica's outputs


    // ---------------- publication ----------------
    // the column of G at facility an, for this lane's four locations, to dst
#define PDIT_REG_STORE_COL(an, dst)                                                        \
    {                                                                                      \
        const int an_ = __builtin_amdgcn_readfirstlane(an);                                \
        if (wv == (an_ >> 6)) {                                                            \
            const int m_ = (an_ & 63) >> 1, h_ = an_ & 1;                                  \
            v2i x_;                                                                        \
            x_.x = (int)pack16(tile_entry(g0, m_, h_), tile_entry(g1, m_, h_));            \
            x_.y = (int)pack16(tile_entry(g2, m_, h_), tile_entry(g3, m_, h_));            \
            *(v2i *)&(dst)[4 * lane] = x_;                                                 \
        }                                                                                  \
    }
    // row nr (the wave's 64 facilities) and the column at facility an, into buffer par
#define PDIT_REG_PUBLISH(nr, an, par)                                                      \
    {                                                                                      \
        const int nr_ = __builtin_amdgcn_readfirstlane(nr);                                \
        if (lane == (nr_ >> 2)) {                                                          \
            const uint32_t dst_ = lds_addr(&rs.u.sq.prow[(par)][64 * wv]);                 \
            const int t_ = nr_ & 3;                                                        \
            if (t_ == 0) PDIT_REG_STORE_ROW(dst_, g0, "0");                                \
            else if (t_ == 1) PDIT_REG_STORE_ROW(dst_, g1, "1");                           \
            else if (t_ == 2) PDIT_REG_STORE_ROW(dst_, g2, "2");                           \
            else PDIT_REG_STORE_ROW(dst_, g3, "3");                                        \
        }                                                                                  \
        PDIT_REG_STORE_COL(an, rs.u.sq.pcol[(par)])                                        \
    }
    // rows r0 .. r0 + nb - 1 and their columns, into the batch buffers
#define PDIT_REG_PUBLISH_BATCH(r0, nb)                                                     \
    {                                                                                      \
        const int row_ = 4 * lane - (r0);                                                  \
        const uint32_t dst_ = lds_addr(&rs.u.sp.brow[0][64 * wv]) + 2 * kRN * row_;        \
        if (row_ >= 0 && row_ < (nb)) PDIT_REG_STORE_ROW(dst_, g0, "b0");                  \
        if (row_ + 1 >= 0 && row_ + 1 < (nb)) PDIT_REG_STORE_ROW(dst_ + 2 * kRN, g1, "b1");\
        if (row_ + 2 >= 0 && row_ + 2 < (nb)) PDIT_REG_STORE_ROW(dst_ + 4 * kRN, g2, "b2");\
        if (row_ + 3 >= 0 && row_ + 3 < (nb)) PDIT_REG_STORE_ROW(dst_ + 6 * kRN, g3, "b3");\
        for (int j_ = 0; j_ < (nb); ++j_) PDIT_REG_STORE_COL(pick(pk, (r0) + j_), rs.u.sp.bcol[j_]) \
    }

    // ---------------- one update's candidates ----------------
    // LDS reads for the update of location R (a = AF) from row PROW and column PCOL
    int32_t hrr_v, d_rr_v, f_aa_v, hr[4], fak[4];
    v2i hc2;
    uint32_t drw;
#define PDIT_REG_READS(PROW, PCOL, R, AF)                                                  \
    {                                                                                      \
        hrr_v = (PROW)[AF];                                                                \
        hc2 = *(const v2i *)&(PCOL)[4 * lane];                                             \
        drw = D32[(R) * (kRN / 4) + lane]; /* D[r][4 lane + t] */                          \
        d_rr_v = ZD ? 0 : (int32_t)sm.D[(R) * kRN + (R)];                                  \
        f_aa_v = ZD ? 0 : (int32_t)sm.F[(AF) * kRN + (AF)];                                \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                    \
            hr[i] = (PROW)[pk[i]];                                                         \
            fak[i] = (int32_t)sm.F[(AF) * kRN + pk[i]];                                    \
        }                                                                                  \
    }
    int32_t hrr, d_rr, f_aa, hc[4], drk[4], dv[4], m2;
    // dE of the N candidates (four per lane) and the minimum over k != R
#define PDIT_REG_DELTA(R)                                                                  \
    {                                                                                      \
        hrr = __builtin_amdgcn_readfirstlane(hrr_v);                                       \
        d_rr = __builtin_amdgcn_readfirstlane(d_rr_v);                                     \
        f_aa = __builtin_amdgcn_readfirstlane(f_aa_v);                                     \
        hc[0] = (int32_t)(int16_t)(hc2.x & 0xFFFF);                                        \
        hc[1] = hc2.x >> 16;                                                               \
        hc[2] = (int32_t)(int16_t)(hc2.y & 0xFFFF);                                        \
        hc[3] = hc2.y >> 16;                                                               \
        m2 = kRBig;                                                                        \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                    \
            const int k = 4 * lane + i;                                                    \
            drk[i] = byte_at<SGN>(drw, i);                                                 \
            const int32_t x = 2 * (hr[i] - hrr + hc[i] - dg[i]);                           \
            const int32_t y = ZD ? 4 * __mul24(drk[i], fak[i])                             \
                                 : __mul24(d_rr + ddk[i] - 2 * drk[i], f_aa + fdk[i] - 2 * fak[i]); \
            dv[i] = k >= N ? kRBig : k == (R) ? 0 : x + y;                                 \
            m2 = min(m2, k == (R) ? kRBig : dv[i]);                                        \
        }                                                                                  \
        m2 = wave_min_i32(m2);                                                             \
    }
    // the draw of the update of location R: S (R for a stay) and whether its
    // threshold fell within the tie band (TIE)
#define PDIT_REG_DRAW(R, S, TIE)                                                           \
    {                                                                                      \
        S = (R);                                                                           \
        TIE = 0;                                                                           \
        if (m2 < dthr) {                                                                   \
            const int32_t mn = min(m2, 0);                                                 \
            uint32_t q[4];                                                                 \
            int32_t dd[4];                                                                 \
            bool any = false;                                                              \
            _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                \
                dd[i] = dv[i] - mn; /* >= 0 */                                             \
                const bool valid = 4 * lane + i < N;                                       \
                q[i] = (valid && dd[i] == 0) ? kWeightOne : 0u;                            \
                any = any || (valid && dd[i] > 0 && dd[i] < dthr);                         \
            }                                                                              \
            if (__ballot(any)) {                                                           \
                _Pragma("unroll") for (int i = 0; i < 4; ++i) {                            \
                    const bool need = 4 * lane + i < N && dd[i] > 0 && dd[i] < dthr;       \
                    const uint32_t wq = gibbs_weight(beta, (float)dd[i]);                  \
                    q[i] = need ? wq : q[i];                                               \
                }                                                                          \
            }                                                                              \
            /* exact running sums: the lane's four weights (< 2^27) scanned as */          \
            /* 16-bit halves, each half's wave sum within 32 bits */                       \
            const uint32_t qs = q[0] + q[1] + q[2] + q[3];                                 \
            const uint32_t slo = scan_u32(qs & 0xFFFFu);                                   \
            const uint32_t shi = scan_u32(qs >> 16);                                       \
            const uint64_t C = ((uint64_t)shi << 16) + slo;                                \
            const uint64_t Z =                                                             \
                ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)shi, 63) << 16) +      \
                (uint32_t)__builtin_amdgcn_readlane((int)slo, 63);                         \
            const uint32_t ur = (uint32_t)pick(uu, (R));                                   \
            const uint64_t thr = ((uint64_t)ur * Z) >> 24; /* first C > thr */             \
            const uint64_t hit = __ballot(C > thr);                                        \
            const int sl = __ffsll((unsigned long long)hit) - 1;                           \
            const uint64_t c0 = C - qs + q[0], c1 = c0 + q[1], c2 = c1 + q[2];             \
            const bool b0 = c0 > thr, b1 = c1 > thr, b2 = c2 > thr;                        \
            const int sel = b0 ? 0 : b1 ? 1 : b2 ? 2 : 3;                                  \
            const uint64_t csel = b0 ? c0 : b1 ? c1 : b2 ? c2 : C;                         \
            const uint32_t qsel = b0 ? q[0] : b1 ? q[1] : b2 ? q[2] : q[3];                \
            const int ssel = __builtin_amdgcn_readlane(sel, sl);                           \
            const uint64_t cs = readlane_u64(csel, sl);                                    \
            const uint32_t qq = (uint32_t)__builtin_amdgcn_readlane((int32_t)qsel, sl);    \
            TIE = is_tie(cs - qq, cs, Z, ur) ? 1 : 0;                                      \
            S = 4 * sl + ssel;                                                             \
        }                                                                                  \
    }
    // the accepted exchange of R and S (a = AF): dE DES; G[R][b] from row PROW,
    // hc_s = G[S][a]; drk, fak and f_aa hold the update's D and F reads
#define PDIT_REG_ACCEPT(R, S, AF, DES, PROW, HC_S)                                         \
    {                                                                                      \
        const int bf = pick(pk, (S)); /* b = p(s) */                                       \
        const int32_t h_rb_v = (int32_t)(PROW)[bf];                                        \
        E += (DES);                                                                        \
        ++n_acc;                                                                           \
        const uint32_t dsw = D32[(S) * (kRN / 4) + lane]; /* D[s][4 lane + t] */           \
        const uint32_t fb4 = F32[bf * (kRN / 4) + lane];  /* F[b][4 lane + t] */           \
        const uint32_t fa4 = F32[(AF) * (kRN / 4) + lane];                                 \
        const int32_t f_ba_v = (int32_t)sm.F[bf * kRN + (AF)];                             \
        const int32_t f_bb_v = (int32_t)sm.F[bf * kRN + bf];                               \
        const int32_t f_ab_v = (int32_t)sm.F[(AF) * kRN + bf];                             \
        int32_t fbk[4];                                                                    \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) fbk[i] = (int32_t)sm.F[bf * kRN + pk[i]]; \
        /* w of facilities 4 lane .. 4 lane + 3, to this wave's copy */                    \
        int16_t *wl = rs.w[wv];                                                            \
        {                                                                                  \
            v2i x;                                                                         \
            x.x = (int)pack16(byte_at<SGN>(fb4, 0) - byte_at<SGN>(fa4, 0),                 \
                              byte_at<SGN>(fb4, 1) - byte_at<SGN>(fa4, 1));                \
            x.y = (int)pack16(byte_at<SGN>(fb4, 2) - byte_at<SGN>(fa4, 2),                 \
                              byte_at<SGN>(fb4, 3) - byte_at<SGN>(fa4, 3));                \
            *(v2i *)&wl[4 * lane] = x;                                                     \
        }                                                                                  \
        /* LDS accesses of one wave complete in order: this read sees the */               \
        /* whole wave's writes */                                                          \
        __asm__ volatile("" ::: "memory");                                                 \
        const v32i wt = *(const v32i *)&wl[64 * wv]; /* w of the wave's facilities */      \
        int32_t u[4];                                                                      \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) u[i] = drk[i] - byte_at<SGN>(dsw, i); \
        const int32_t f_bb = __builtin_amdgcn_readfirstlane(f_bb_v);                       \
        const int32_t h_rb = __builtin_amdgcn_readfirstlane(h_rb_v);                       \
        const int32_t w_a = __builtin_amdgcn_readfirstlane(f_ba_v) - f_aa; /* F[b][a] - F[a][a] */ \
        const int32_t w_b = f_bb - __builtin_amdgcn_readfirstlane(f_ab_v); /* F[b][b] - F[a][b] */ \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                    \
            const int k = 4 * lane + i;                                                    \
            const int32_t wp = fbk[i] - fak[i]; /* w at p(k) */                            \
            const bool is_r = k == (R), is_s = k == (S);                                   \
            dg[i] = is_r ? h_rb + __mul24(u[i], w_b)        /* G'[r][b] */                 \
                  : is_s ? (HC_S) + __mul24(u[i], w_a)      /* G'[s][a] */                 \
                         : dg[i] + __mul24(u[i], wp);                                      \
            if (!ZD) fdk[i] = is_r ? f_bb : is_s ? f_aa : fdk[i];                          \
            pk[i] = is_r ? bf : is_s ? (AF) : pk[i];                                       \
        }                                                                                  \
        /* the tile: G += u w over the wave's 64 facilities */                             \
        g0 = rank1(g0, (short)u[0], wt);                                                   \
        g1 = rank1(g1, (short)u[1], wt);                                                   \
        g2 = rank1(g2, (short)u[2], wt);                                                   \
        g3 = rank1(g3, (short)u[3], wt);                                                   \
        if (E < E_best) {                                                                  \
            E_best = E;                                                                    \
            if (writer) {                                                                  \
                _Pragma("unroll") for (int i = 0; i < 4; ++i) {                            \
                    const int k = 4 * lane + i;                                            \
                    if (k < N) a.perm_best[rep * N + k] = pk[i];                           \
                }                                                                          \
            }                                                                              \
        }                                                                                  \
    }

    const lds_v4i *flags = rep_flags(rs.sync);
    uint32_t seq = 0;      // steps of this replica's waits
    PDIT_REG_PUBLISH(0, pick(pk, 0), 0)
    rep_signal(rs.sync, wv, ++seq);
    bool ok = true;        // every wait completed
    bool batch = false;    // this sweep runs in batches

    for (int64_t t = 0; t < a.T && ok; ++t) {
        const float beta = bp[t * bstride];
        const uint32_t gsw = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        int32_t *ch = ch_base ? ch_base + t * N : nullptr;
        int32_t uu[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            uu[i] = (int32_t)uniform24(a.seed, (uint32_t)(4 * lane + i), gsw, (uint32_t)rep,
                                       a.inst_id);
        const int64_t acc0 = n_acc;
        // the next sweep runs in batches when this one accepts few exchanges
#define PDIT_REG_NEXT_BATCH() (t + 1 < a.T && n_acc - acc0 <= kRSpecAcc)

        // Steps: one update, which every wave evaluates, or in a batch sweep a
        // batch of kRSpec updates evaluated on one state, kRSpec / kRWaves per
        // wave.  A batch commits its stays up to the first exchange; the update
        // with the exchange then runs as a single update on the batch's row and
        // column, which draws the same candidate.
        if (batch && !rep_done(*flags, seq)) ok = rep_spin(flags, seq);  // buffers free
        bool replayed = false;                  // batch: the last step was a single update
        int r0 = 0;
        while (r0 < N && ok) {
            const int16_t *prow, *pcol;
            bool fresh = true;                  // the row and column were just published
            if (batch) {
                // ============ a batch: rows r0 .. r0 + nb - 1 ============
                if (replayed && !rep_done(*flags, seq)) {  // every wave left that update
                    ok = rep_spin(flags, seq);
                    if (!ok) break;
                }
                const int nb = min(kRSpec, N - r0);
                PDIT_REG_PUBLISH_BATCH(r0, nb)
                rep_signal(rs.sync, wv, ++seq);
                // this wave's updates j = wv, wv + kRWaves, ...: the draw and its tie
                // flag to the outcome slots
                for (int j = wv; j < nb; j += kRWaves) {
                    const int rj = r0 + j;
                    const int af = pick(pk, rj);
                    const int16_t *brow = rs.u.sp.brow[j];
                    {
                        const v4i fl = *flags;
                        __asm__ volatile("" ::: "memory");
                        PDIT_REG_READS(brow, rs.u.sp.bcol[j], rj, af)
                        if (j == wv && !rep_done(fl, seq)) {
                            ok = rep_spin(flags, seq);
                            if (!ok) break;
                            PDIT_REG_READS(brow, rs.u.sp.bcol[j], rj, af)
                        }
                    }
                    PDIT_REG_DELTA(rj)
                    int sj, tie;
                    PDIT_REG_DRAW(rj, sj, tie)
                    if (lane == 0) rs.outc[j] = v4i{sj, tie, 0, 0};
                }
                if (!ok) break;
                rep_signal(rs.sync, wv, ++seq);
                // the outcomes: the first exchange ends the batch
                v4i o;
                {
                    const v4i fl = *flags;
                    __asm__ volatile("" ::: "memory");
                    o = rs.outc[lane < nb ? lane : 0];
                    if (!rep_done(fl, seq)) {
                        ok = rep_spin(flags, seq);
                        if (!ok) break;
                        o = rs.outc[lane < nb ? lane : 0];
                    }
                }
                const uint64_t moves = __ballot(lane < nb && o.x != r0 + lane);
                const int jm = moves ? __ffsll((unsigned long long)moves) - 1 : nb;
                n_tie += __popcll(__ballot(lane < jm && o.y != 0));
                if (ch && lane < jm) ch[r0 + lane] = o.x;
                replayed = false;
                if (jm == nb) {
                    r0 += nb;
                    continue;
                }
                r0 += jm;
                prow = rs.u.sp.brow[jm];
                pcol = rs.u.sp.bcol[jm];
                fresh = false;
            } else {
                const int par = (seq - 1) & 1;  // the buffer that holds row r0, column p(r0)
                prow = rs.u.sq.prow[par];
                pcol = rs.u.sq.pcol[par];
            }
            // ============ one update: location r0 ============
            const int r = r0;
            const int af = pick(pk, r);         // a = p(r)
            // the flags and the publication in one LDS round trip
            {
                const v4i fl = *flags;
                __asm__ volatile("" ::: "memory");
                PDIT_REG_READS(prow, pcol, r, af)
                if (fresh && !rep_done(fl, seq)) {
                    ok = rep_spin(flags, seq);
                    if (!ok) break;
                    PDIT_REG_READS(prow, pcol, r, af)
                }
            }
            PDIT_REG_DELTA(r)
            int s, tie;
            PDIT_REG_DRAW(r, s, tie)
            n_tie += tie;
            if (ch && lane == 0) ch[r] = s;
            if (s != r) PDIT_REG_ACCEPT(r, s, af, pick(dv, s), prow, pick(hc, s))
            ++r0;
            if (!batch) {
                // the next update's row and column (the next sweep's first, unless
                // it runs in batches)
                if (r0 < N || !PDIT_REG_NEXT_BATCH()) {
                    const int nr = r0 < N ? r0 : 0;
                    PDIT_REG_PUBLISH(nr, pick(pk, nr), seq & 1)
                }
            } else {
                replayed = true;
            }
            rep_signal(rs.sync, wv, ++seq);
        }
        if (ok && batch && !PDIT_REG_NEXT_BATCH()) {
            // the next sweep goes one update at a time: its first row and column,
            // once every wave has left the batch buffers they share
            if (replayed && !rep_done(*flags, seq)) ok = rep_spin(flags, seq);
            PDIT_REG_PUBLISH(0, pick(pk, 0), seq & 1)
            rep_signal(rs.sync, wv, ++seq);
        }
        batch = PDIT_REG_NEXT_BATCH();
#undef PDIT_REG_NEXT_BATCH
        if (a.E_trace && writer && lane == 0) a.E_trace[rep * a.T + t] = E;
    }
#undef PDIT_REG_STORE_COL
#undef PDIT_REG_PUBLISH
#undef PDIT_REG_PUBLISH_BATCH
#undef PDIT_REG_READS
#undef PDIT_REG_DELTA
#undef PDIT_REG_DRAW
#undef PDIT_REG_ACCEPT

    // ---- outputs ----
    if (!ok && a.err) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (writer) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * lane + i;
            if (k < N) a.perm[rep * N + k] = pk[i];
        }
        if (lane == 0) {
            a.E[rep] = E;
            a.E_best[rep] = E_best;
            const bool accum = (a.flags & kAccumCounters) != 0;
            a.counters[3 * rep + 0] = (accum ? a.counters[3 * rep + 0] : 0) + (int64_t)N * a.T;
            a.counters[3 * rep + 1] = (accum ? a.counters[3 * rep + 1] : 0) + n_acc;
            a.counters[3 * rep + 2] = (accum ? a.counters[3 * rep + 2] : 0) + n_tie;
        }
    }
}

template <bool SGN, bool ZD>
hipError_t launch_reg_one(hipStream_t s, const SweepArgs &a) {
    const unsigned blocks = (unsigned)((a.R + kRReps - 1) / kRReps);
    sweep_reg_kernel<SGN, ZD><<<blocks, kRThreads, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

int reg_class(int N, const InstanceStats &st) {
    if (N <= 128 || N > kRN) return 0;
    // G = H permuted, packed int16; |dE| below the padding sentinel
    if (h_bound(st) > 32767 || delta_bound(st) >= (int64_t)kRBig) return 0;
    const bool u8 = st.neg_d == 0 && st.neg_f == 0 && st.max_abs_d <= 255 && st.max_abs_f <= 255;
    const bool s8 = st.max_abs_d <= 127 && st.max_abs_f <= 127;
    return u8 ? 1 : s8 ? 2 : 0;
}

hipError_t launch_sweep_reg(hipStream_t s, int cls, const SweepArgs &a) {
    if (a.flags & (kLoadState | kSaveState)) return hipErrorInvalidValue;
    if (cls == 1) return a.zero_diag ? launch_reg_one<false, true>(s, a) : launch_reg_one<false, false>(s, a);
    if (cls == 2) return a.zero_diag ? launch_reg_one<true, true>(s, a) : launch_reg_one<true, false>(s, a);
    return hipErrorInvalidValue;
}

}  // namespace pdit
