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
// column) and wait for each other.  Lane j of wave w then evaluates the one
// candidate k = 64w + j,
//   dE_k = 2 (H[r][k] - H[r][r] + H[k][r] - H[k][k])
//          + (D_rr + D_kk - 2 D_rk)(F_aa + F_cc - 2 F_ac),  c = p(k),
// with H[k][k], p(k) and the diagonals of D and F kept in its registers.
// The waves meet twice more: for the row minimum over k != r (a row whose
// only nonzero weight is its own stay, every other candidate lying at or
// beyond the zero-weight distance above 0, keeps its facility without
// weights or scan), and for the running sums of the integer Gibbs weights
// q = rint(expf(-beta d) 2^25), each wave's exact within 32 bits, from which
// every wave reads the same 64-bit CDF in location order and draws the same
// candidate, as the other sweep kernels do.
//
// Batches.  An update that keeps its facility changes nothing, so when few
// exchanges are accepted the updates of locations r0 .. r0 + nb - 1 can all
// be evaluated on the same state: the waves publish the nb rows and columns
// together, and each wave takes up to three of the updates whole, on all N
// candidates at four consecutive locations per lane (their p and H[k][k]
// read from LDS), with its own minimum and draw; the draws (candidate, dE,
// its facility) meet in LDS and the stays up to the first exchange are
// committed.  That exchange is applied as in a single update, and the next
// batch starts after it.  Every draw is the sequential one.  A sweep runs in
// batches when the sweep before it accepted at most kRAcc4 exchanges, with
// nb = 12, 8 or 4 as that count falls below kRAcc12, kRAcc8 or kRAcc4: a
// batch is cut at its first exchange, so the more exchanges, the shorter
// the batch that pays.
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
// Batches: after a sweep that accepted at most kRAcc4 exchanges the next
// sweep evaluates consecutive updates on one state, kRSpec of them when it
// accepted at most kRAcc12, 8 up to kRAcc8, else 4
constexpr int kRSpec = 12;
constexpr int kRAcc12 = 24;
constexpr int kRAcc8 = 48;
constexpr int kRAcc4 = 112;
// polls of a replica's wait before it gives up (a fraction of a second): reached only
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
            alignas(16) v2i cd[kRWaves][64];   // per candidate: its wave's running weight sum, dE
        } sq;
        struct {                               // a batch of kRSpec updates
            alignas(16) int16_t brow[kRSpec][kRN];
            alignas(16) int16_t bcol[kRSpec][kRN];
        } sp;
        alignas(16) int16_t stage[kRWaves][16][64];  // set-up: rows of G on their way to the tiles
    } u;
    alignas(16) int16_t w[kRN];              // accepted exchange: F[b][c] - F[a][c] (wave w: c in its 64)
    alignas(16) int32_t pv[kRN];             // p by location
    alignas(16) int32_t dga[kRN];            // batch: H[k][k] by location
    alignas(16) uint32_t u24[kRN];           // the sweep's uniforms by location
    alignas(16) v4i outc[kRSpec];              // batch: per update its draw s, tie flag, dE_s, p(s)
    alignas(16) int32_t smin[kRWaves];       // one update: per wave, min dE over k != r
    alignas(16) uint32_t sync[kRWaves];      // per wave: the last step it finished
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

// every wave of the replica has finished step seq (uniform: every lane reads
// the same four flags, so the ballot is all lanes or none)
__device__ __forceinline__ bool rep_done(v4i v, uint32_t seq) {
    const int32_t d = min(min((int32_t)(v.x - seq), (int32_t)(v.y - seq)),
                          min((int32_t)(v.z - seq), (int32_t)(v.w - seq)));
    return __builtin_amdgcn_ballot_w64(d >= 0) != 0;
}

// Polls until every wave has finished step seq; false when the wait gave up
// (kRSpinLimit).  Each poll is one LDS round trip; a sleep between polls
// (s_sleep 1) made the hot sweeps of the N=256 workload 1.3% slower.
__device__ __forceinline__ bool rep_spin(const lds_v4i *ps, uint32_t seq) {
    for (uint32_t it = 0; it < kRSpinLimit; ++it) {
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
    const int k = 64 * wv + lane;     // this lane's candidate location
    const bool kval = k < N;

    // ---- D and F copies (both replicas) ----
    for (int e = tid; e < kRN * kRN; e += kRThreads) {
        const int i = e >> 8, j = e & 255;
        const bool in = i < N && j < N;
        sm.D[e] = (E8)(in ? a.D[(int64_t)i * N + j] : 0);
        sm.F[e] = (E8)(in ? a.F[(int64_t)i * N + j] : 0);
    }
    // ---- p (padding locations hold the padding facilities) ----
    int32_t pk = kval ? a.perm[rep * N + k] : k;
    rs.pv[k] = pk;
    if (lane < kRWaves && wv == 0) rs.sync[lane] = 0;

    // ---- the tile: G[4 lane + t][64 wv + c], from G = D F[p,:] (row k of a
    // replica's N x N block, columns by facility).  Rows 16 q .. 16 q + 15 of
    // the wave's 64 facilities are read along the rows (lane c takes column
    // 64 wv + c), staged in the wave's part of LDS as int16, and read back by
    // the four lanes that hold them; LDS accesses of one wave complete in
    // order, so the wave needs no barrier. ----
    v32i g0, g1, g2, g3;
    {
        const int32_t *Gb = (const int32_t *)a.H + rep * N * (int64_t)N;
        int16_t *stage = rs.u.stage[wv][0];     // 16 rows x 64 facilities
        const int c = 64 * wv + lane;
        for (int q = 0; q < kRN / 16; ++q) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int kr = 16 * q + i;
                stage[i * 64 + lane] = (int16_t)((kr < N && c < N) ? Gb[kr * (int64_t)N + c] : 0);
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
    // the D and F copies, p and the flags are complete before the first reads
    __syncthreads();
    // the candidate's H[k][k] = G[k][p(k)], D[k][k], F[p(k)][p(k)]
    int32_t dg = kval ? ((const int32_t *)a.H)[(rep * N + k) * (int64_t)N + pk] : 0;
    const int32_t ddk = ZD ? 0 : (int32_t)sm.D[k * kRN + k];
    int32_t fdk = ZD ? 0 : (int32_t)sm.F[pk * kRN + pk];
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0;
    int32_t n_tie = 0;
    int32_t *ch_base = (a.choices && live && wv == 0) ? a.choices + rep * a.T * N : nullptr;
    const float *bp = a.slot ? a.beta + a.slot[rep] : a.beta;
    const int64_t bstride = a.slot ? 0 : 1;
    const bool writer = live && wv == 0;   // wave 0 writes the replica's scalar outputs

    // ---------------- publication ----------------
    // the column of G at facility an, for this lane's four tile rows, to dst
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

    // ---------------- one update's candidates (this wave's 64) ----------------
    int32_t hrr_v, d_rr_v, f_aa_v, hr_v, hc_v, drk_v, fak_v;
    // LDS reads for the update of location R (a = AF) from row PROW and column PCOL
#define PDIT_REG_READS(PROW, PCOL, R, AF)                                                  \
    {                                                                                      \
        hrr_v = (PROW)[AF];                                                                \
        hr_v = (PROW)[pk];                                                                 \
        hc_v = (PCOL)[k];                                                                  \
        drk_v = (int32_t)sm.D[(R) * kRN + k];                                              \
        fak_v = (int32_t)sm.F[(AF) * kRN + pk];                                            \
        d_rr_v = ZD ? 0 : (int32_t)sm.D[(R) * (kRN + 1)];                                  \
        f_aa_v = ZD ? 0 : (int32_t)sm.F[(AF) * (kRN + 1)];                                 \
    }
    int32_t f_aa, dv, mw;
    // dE of this lane's candidate and the wave's minimum over k != R
#define PDIT_REG_DELTA(R)                                                                  \
    {                                                                                      \
        const int32_t hrr = __builtin_amdgcn_readfirstlane(hrr_v);                         \
        const int32_t d_rr = __builtin_amdgcn_readfirstlane(d_rr_v);                       \
        f_aa = __builtin_amdgcn_readfirstlane(f_aa_v);                                     \
        const int32_t x = 2 * (hr_v - hrr + hc_v - dg);                                    \
        const int32_t y = ZD ? 4 * __mul24(drk_v, fak_v)                                   \
                             : __mul24(d_rr + ddk - 2 * drk_v, f_aa + fdk - 2 * fak_v);    \
        dv = !kval ? kRBig : k == (R) ? 0 : x + y;                                         \
        mw = wave_min_i32(k == (R) ? kRBig : dv);                                          \
    }
    // the accepted exchange of R and S (a = AF, b = BF): dE DES; G[R][b] from
    // row PROW; hc_v, drk_v, fak_v and f_aa hold the update's reads
#define PDIT_REG_ACCEPT(R, S, AF, BF, DES, PROW)                                           \
    {                                                                                      \
        E += (DES);                                                                        \
        ++n_acc;                                                                           \
        const int32_t h_rb_v = (int32_t)(PROW)[BF];                                        \
        const uint32_t drw = D32[(R) * (kRN / 4) + lane]; /* D[r][4 lane + t] */           \
        const uint32_t dsw = D32[(S) * (kRN / 4) + lane]; /* D[s][4 lane + t] */           \
        const int32_t dsk = (int32_t)sm.D[(S) * kRN + k];                                  \
        const int32_t fbk = (int32_t)sm.F[(BF) * kRN + pk];                                \
        const int32_t fbc = (int32_t)sm.F[(BF) * kRN + 64 * wv + lane];                    \
        const int32_t fac = (int32_t)sm.F[(AF) * kRN + 64 * wv + lane];                    \
        const int32_t f_ba_v = (int32_t)sm.F[(BF) * kRN + (AF)];                           \
        const int32_t f_bb_v = (int32_t)sm.F[(BF) * (kRN + 1)];                            \
        const int32_t f_ab_v = (int32_t)sm.F[(AF) * kRN + (BF)];                           \
        /* w of this wave's facilities 64 wv + lane */                                     \
        rs.w[64 * wv + lane] = (int16_t)(fbc - fac);                                       \
        /* LDS accesses of one wave complete in order: this read sees the */               \
        /* whole wave's writes */                                                          \
        __asm__ volatile("" ::: "memory");                                                 \
        const v32i wt = *(const v32i *)&rs.w[64 * wv];                                     \
        const int32_t h_rb = __builtin_amdgcn_readfirstlane(h_rb_v);                       \
        const int32_t f_bb = __builtin_amdgcn_readfirstlane(f_bb_v);                       \
        const int32_t w_a = __builtin_amdgcn_readfirstlane(f_ba_v) - f_aa; /* F[b][a] - F[a][a] */ \
        const int32_t w_b = f_bb - __builtin_amdgcn_readfirstlane(f_ab_v); /* F[b][b] - F[a][b] */ \
        const int32_t uk = drk_v - dsk;                 /* D[k][r] - D[k][s] */             \
        const bool is_r = k == (R), is_s = k == (S);                                       \
        dg = is_r ? h_rb + __mul24(uk, w_b)            /* G'[r][b] */                      \
           : is_s ? hc_v + __mul24(uk, w_a)            /* G'[s][a] */                      \
                  : dg + __mul24(uk, fbk - fak_v);     /* + u_k (F[b][p(k)] - F[a][p(k)]) */ \
        if (!ZD) fdk = is_r ? f_bb : is_s ? f_aa : fdk;                                    \
        if (is_r || is_s) {                                                                \
            pk = is_r ? (BF) : (AF);                                                       \
            rs.pv[k] = pk;                                                                 \
        }                                                                                  \
        /* the tile: G += u w over the wave's 64 facilities */                             \
        g0 = rank1(g0, (short)(byte_at<SGN>(drw, 0) - byte_at<SGN>(dsw, 0)), wt);          \
        g1 = rank1(g1, (short)(byte_at<SGN>(drw, 1) - byte_at<SGN>(dsw, 1)), wt);          \
        g2 = rank1(g2, (short)(byte_at<SGN>(drw, 2) - byte_at<SGN>(dsw, 2)), wt);          \
        g3 = rank1(g3, (short)(byte_at<SGN>(drw, 3) - byte_at<SGN>(dsw, 3)), wt);          \
        if (E < E_best) {                                                                  \
            E_best = E;                                                                    \
            if (live && kval) a.perm_best[rep * N + k] = pk;                               \
        }                                                                                  \
    }

#define PDIT_REG_POLL(READS)                                                               \
    {                                                                                      \
        const v4i fl_ = *flags;                                                            \
        __asm__ volatile("" ::: "memory");                                                 \
        READS                                                                              \
        if (!rep_done(fl_, seq)) {                                                         \
            ok = rep_spin(flags, seq);                                                     \
            if (!ok) break;                                                                \
            READS                                                                          \
        }                                                                                  \
    }

    // p of candidates lane, 64 + lane, 128 + lane, 192 + lane (read in a meeting
    // before any exchange can change them)
    int32_t pw0 = 0, pw1 = 0, pw2 = 0, pw3 = 0;
    // The draw of the update of location R whose minimum over k != R is M2
    // (< dthr) and whose dE on this lane's candidate is DVJ, uniform UR:
    // weights, this wave's running sums (64 weights of at most 2^25: 32
    // bits), a meeting, and the first candidate whose running sum over all N
    // exceeds the threshold.  Sets S, TIE, DES (dE_S) and BF (p(S)).
#define PDIT_REG_DRAW(R, DVJ, M2, UR, S, TIE, DES, BF)                                     \
    {                                                                                      \
        const int32_t mn_ = min((M2), 0);                                                  \
        const int32_t d_ = (DVJ) - mn_; /* >= 0 */                                         \
        uint32_t q_ = (kval && d_ == 0) ? kWeightOne : 0u;                                 \
        const bool need_ = kval && d_ > 0 && d_ < dthr;                                    \
        if (__ballot(need_)) {                                                             \
            const uint32_t wq_ = gibbs_weight(beta, (float)d_);                            \
            q_ = need_ ? wq_ : q_;                                                         \
        }                                                                                  \
        const uint32_t C_ = scan_u32(q_);                                                  \
        rs.u.sq.cd[wv][lane] = v2i{(int)C_, (DVJ)};                                        \
        rep_signal(rs.sync, wv, ++seq);                                                    \
        v2i c0_, c1_, c2_, c3_;                                                            \
        PDIT_REG_POLL({                                                                    \
            c0_ = rs.u.sq.cd[0][lane];                                                     \
            c1_ = rs.u.sq.cd[1][lane];                                                     \
            c2_ = rs.u.sq.cd[2][lane];                                                     \
            c3_ = rs.u.sq.cd[3][lane];                                                     \
        })                                                                                 \
        const uint64_t T0_ = (uint32_t)__builtin_amdgcn_readlane(c0_.x, 63);               \
        const uint64_t T1_ = (uint32_t)__builtin_amdgcn_readlane(c1_.x, 63);               \
        const uint64_t T2_ = (uint32_t)__builtin_amdgcn_readlane(c2_.x, 63);               \
        const uint64_t T3_ = (uint32_t)__builtin_amdgcn_readlane(c3_.x, 63);               \
        const uint64_t o1_ = T0_, o2_ = T0_ + T1_, o3_ = T0_ + T1_ + T2_;                  \
        const uint64_t Z_ = o3_ + T3_;                                                     \
        const uint32_t ur_ = (uint32_t)__builtin_amdgcn_readfirstlane((int)(UR));          \
        const uint64_t thr_ = ((uint64_t)ur_ * Z_) >> 24; /* first C > thr */              \
        const int ws_ = thr_ < o1_ ? 0 : thr_ < o2_ ? 1 : thr_ < o3_ ? 2 : 3;              \
        const uint64_t off_ = ws_ == 0 ? 0 : ws_ == 1 ? o1_ : ws_ == 2 ? o2_ : o3_;        \
        const v2i cw_ = ws_ == 0 ? c0_ : ws_ == 1 ? c1_ : ws_ == 2 ? c2_ : c3_;            \
        const int32_t pwv_ = ws_ == 0 ? pw0 : ws_ == 1 ? pw1 : ws_ == 2 ? pw2 : pw3;       \
        const uint64_t cg_ = off_ + (uint32_t)cw_.x;                                       \
        const uint64_t hit_ = __ballot(cg_ > thr_);                                        \
        const int sl_ = __ffsll((unsigned long long)hit_) - 1;                             \
        const uint64_t csel_ = readlane_u64(cg_, sl_);                                     \
        const uint64_t cprev_ = sl_ > 0 ? readlane_u64(cg_, sl_ > 0 ? sl_ - 1 : 0) : off_; \
        TIE = is_tie(cprev_, csel_, Z_, ur_) ? 1 : 0;                                      \
        S = 64 * ws_ + sl_;                                                                \
        DES = __builtin_amdgcn_readlane(cw_.y, sl_);                                       \
        BF = __builtin_amdgcn_readlane(pwv_, sl_);                                         \
    }

    const lds_v4i *flags = rep_flags(rs.sync);
    uint32_t seq = 0;      // steps of this replica's waits
    int a_next = __builtin_amdgcn_readfirstlane(rs.pv[0]);  // p of the next single update's row
    // the buffer (of two) that holds the next single update's row and column;
    // it alternates per update, whatever the number of meetings in between, so
    // that the next publication never overwrites the row a slower wave may
    // still read in its accept
    int pbuf = 0;
    PDIT_REG_PUBLISH(0, a_next, 0)
    rep_signal(rs.sync, wv, ++seq);
    bool ok = true;        // every wait completed
    int nbat = 0;          // updates per batch in this sweep (0: one update at a time)

    for (int64_t t = 0; t < a.T && ok; ++t) {
        const float beta = bp[t * bstride];
        const uint32_t gsw = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        int32_t *ch = ch_base ? ch_base + t * N : nullptr;
        // the sweep's uniforms by location; every read of them follows the
        // first minimum meeting of the sweep, which follows this store
        rs.u24[k] = uniform24(a.seed, (uint32_t)k, gsw, (uint32_t)rep, a.inst_id);
        const int64_t acc0 = n_acc;
        // the next sweep runs in batches when this one accepts few exchanges
#define PDIT_REG_NEXT_BATCH() (t + 1 < a.T && n_acc - acc0 <= kRAcc4)

        // Steps: one update, evaluated by the four waves on 64 candidates each
        // (meetings: the row and column, the minimum, the running sums), or in
        // a batch sweep a batch of nbat updates evaluated on one state: their
        // energy changes and minima, then the draws of the updates that can
        // move, in order, until one exchanges; the stays before it are
        // committed and the exchange is applied.
        if (nbat && !rep_done(*flags, seq)) ok = rep_spin(flags, seq);  // buffers free
        bool replayed = false;                  // batch: the last step ended in an exchange
        int r0 = 0;
        while (r0 < N && ok) {
            // the step's exchange, if any: r, s, a, b, dE and the row of G[r][b]
            int r = r0, s = r0, af = 0, bf = 0, nxt = 0;
            int32_t des = 0;
            const int16_t *prow = rs.u.sq.prow[0];
            if (nbat) {
                // ============ a batch: rows r0 .. r0 + nb - 1 ============
                if (replayed && !rep_done(*flags, seq)) {  // every wave left the exchange
                    ok = rep_spin(flags, seq);
                    if (!ok) break;
                }
                const int nb = min(nbat, N - r0);
                const int ab = rs.pv[r0 + (lane < nb ? lane : 0)];  // p of the batch's rows
                rs.dga[k] = dg;
                {
                    const int row_ = 4 * lane - r0;
                    const uint32_t dst_ = lds_addr(&rs.u.sp.brow[0][64 * wv]) + 2 * kRN * row_;
                    if (row_ >= 0 && row_ < nb) PDIT_REG_STORE_ROW(dst_, g0, "b0");
                    if (row_ + 1 >= 0 && row_ + 1 < nb) PDIT_REG_STORE_ROW(dst_ + 2 * kRN, g1, "b1");
                    if (row_ + 2 >= 0 && row_ + 2 < nb) PDIT_REG_STORE_ROW(dst_ + 4 * kRN, g2, "b2");
                    if (row_ + 3 >= 0 && row_ + 3 < nb) PDIT_REG_STORE_ROW(dst_ + 6 * kRN, g3, "b3");
                    for (int j = 0; j < nb; ++j)
                        PDIT_REG_STORE_COL(__builtin_amdgcn_readlane(ab, j), rs.u.sp.bcol[j])
                }
                rep_signal(rs.sync, wv, ++seq);
                // this wave's updates j = wv, wv + 4, wv + 8, each on all N
                // candidates, four consecutive locations per lane: their p and
                // H[k][k] from LDS (fixed until the batch's exchange)
                v4i pk4v, dg4v;
                PDIT_REG_POLL({
                    pk4v = *(const v4i *)&rs.pv[4 * lane];
                    dg4v = *(const v4i *)&rs.dga[4 * lane];
                })
                const int32_t pk4[4] = {pk4v.x, pk4v.y, pk4v.z, pk4v.w};
                const int32_t dg4[4] = {dg4v.x, dg4v.y, dg4v.z, dg4v.w};
                int32_t dd4[4], fd4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    dd4[i] = ZD ? 0 : (int32_t)sm.D[(4 * lane + i) * (kRN + 1)];
                    fd4[i] = ZD ? 0 : (int32_t)sm.F[pk4[i] * (kRN + 1)];
                }
#pragma unroll
                for (int jj = 0; jj < kRSpec / kRWaves; ++jj) {
                    const int j = wv + kRWaves * jj;
                    if (j >= nb) break;
                    const int rj = r0 + j;
                    const int aj = __builtin_amdgcn_readlane(ab, j);
                    const int16_t *brow = rs.u.sp.brow[j];
                    const v2i hc2 = *(const v2i *)&rs.u.sp.bcol[j][4 * lane];
                    const uint32_t drw = D32[rj * (kRN / 4) + lane];
                    const int32_t hrr_j = brow[aj];
                    const int32_t drr_j = ZD ? 0 : (int32_t)sm.D[rj * (kRN + 1)];
                    const int32_t faa_j = ZD ? 0 : (int32_t)sm.F[aj * (kRN + 1)];
                    const uint32_t ur_j = rs.u24[rj];
                    int32_t hr4[4], fa4[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        hr4[i] = brow[pk4[i]];
                        fa4[i] = (int32_t)sm.F[aj * kRN + pk4[i]];
                    }
                    const int32_t hrr = __builtin_amdgcn_readfirstlane(hrr_j);
                    const int32_t d_rr = __builtin_amdgcn_readfirstlane(drr_j);
                    const int32_t f_a = __builtin_amdgcn_readfirstlane(faa_j);
                    const int32_t hc4[4] = {(int32_t)(int16_t)(hc2.x & 0xFFFF), hc2.x >> 16,
                                            (int32_t)(int16_t)(hc2.y & 0xFFFF), hc2.y >> 16};
                    int32_t dv4[4], mj = kRBig;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int kk = 4 * lane + i;
                        const int32_t dr = byte_at<SGN>(drw, i);
                        const int32_t x = 2 * (hr4[i] - hrr + hc4[i] - dg4[i]);
                        const int32_t y = ZD ? 4 * __mul24(dr, fa4[i])
                                             : __mul24(d_rr + dd4[i] - 2 * dr, f_a + fd4[i] - 2 * fa4[i]);
                        dv4[i] = kk >= N ? kRBig : kk == rj ? 0 : x + y;
                        mj = min(mj, kk == rj ? kRBig : dv4[i]);
                    }
                    mj = wave_min_i32(mj);
                    // the draw, when a candidate lies within the zero-weight
                    // distance: weights, the exact 64-bit running sums (the
                    // lane's four weights, < 2^27, scanned as 16-bit halves)
                    int sj = rj, tj = 0, dj = 0, bj = aj;
                    if (mj < dthr) {
                        const int32_t mn = min(mj, 0);
                        uint32_t q[4];
                        int32_t dd[4];
                        bool any = false;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            dd[i] = dv4[i] - mn;
                            const bool valid = 4 * lane + i < N;
                            q[i] = (valid && dd[i] == 0) ? kWeightOne : 0u;
                            any = any || (valid && dd[i] > 0 && dd[i] < dthr);
                        }
                        if (__ballot(any)) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const bool need = 4 * lane + i < N && dd[i] > 0 && dd[i] < dthr;
                                const uint32_t wq = gibbs_weight(beta, (float)dd[i]);
                                q[i] = need ? wq : q[i];
                            }
                        }
                        const uint32_t qs = q[0] + q[1] + q[2] + q[3];
                        const uint32_t slo = scan_u32(qs & 0xFFFFu);
                        const uint32_t shi = scan_u32(qs >> 16);
                        const uint64_t C = ((uint64_t)shi << 16) + slo;
                        const uint64_t Z =
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)shi, 63) << 16) +
                            (uint32_t)__builtin_amdgcn_readlane((int)slo, 63);
                        const uint32_t ur = (uint32_t)__builtin_amdgcn_readfirstlane((int)ur_j);
                        const uint64_t thr = ((uint64_t)ur * Z) >> 24;   // first C > thr
                        const uint64_t hit = __ballot(C > thr);
                        const int sl = __ffsll((unsigned long long)hit) - 1;
                        const uint64_t cc0 = C - qs + q[0], cc1 = cc0 + q[1], cc2 = cc1 + q[2];
                        const bool b0 = cc0 > thr, b1 = cc1 > thr, b2 = cc2 > thr;
                        const int sel = b0 ? 0 : b1 ? 1 : b2 ? 2 : 3;
                        const uint64_t csel = b0 ? cc0 : b1 ? cc1 : b2 ? cc2 : C;
                        const uint32_t qsel = b0 ? q[0] : b1 ? q[1] : b2 ? q[2] : q[3];
                        const int32_t dsel = b0 ? dv4[0] : b1 ? dv4[1] : b2 ? dv4[2] : dv4[3];
                        const int32_t psel = b0 ? pk4[0] : b1 ? pk4[1] : b2 ? pk4[2] : pk4[3];
                        const int ssel = __builtin_amdgcn_readlane(sel, sl);
                        const uint64_t cs = readlane_u64(csel, sl);
                        const uint32_t qq = (uint32_t)__builtin_amdgcn_readlane((int32_t)qsel, sl);
                        tj = is_tie(cs - qq, cs, Z, ur) ? 1 : 0;
                        sj = 4 * sl + ssel;
                        dj = __builtin_amdgcn_readlane(dsel, sl);
                        bj = __builtin_amdgcn_readlane(psel, sl);
                    }
                    if (lane == 0) rs.outc[j] = v4i{sj, tj, dj, bj};
                }
                if (!ok) break;
                rep_signal(rs.sync, wv, ++seq);
                // the outcomes: the stays up to the first exchange are committed
                v4i o;
                PDIT_REG_POLL(o = rs.outc[lane < nb ? lane : 0];)
                const uint64_t moves = __ballot(lane < nb && o.x != r0 + lane);
                const int jm = moves ? __ffsll((unsigned long long)moves) - 1 : nb;
                n_tie += __popcll(__ballot(lane < nb && lane <= jm && o.y != 0));
                if (ch && lane < jm) ch[r0 + lane] = r0 + lane;
                replayed = false;
                if (jm == nb) {
                    r0 += nb;
                    continue;
                }
                // the exchange: this wave's reads of its row and column
                r = r0 + jm;
                s = __builtin_amdgcn_readlane(o.x, jm);
                des = __builtin_amdgcn_readlane(o.z, jm);
                bf = __builtin_amdgcn_readlane(o.w, jm);
                af = __builtin_amdgcn_readlane(ab, jm);
                prow = rs.u.sp.brow[jm];
                PDIT_REG_READS(prow, rs.u.sp.bcol[jm], r, af)
                f_aa = ZD ? 0 : __builtin_amdgcn_readfirstlane(f_aa_v);
                if (ch && lane == 0) ch[r] = s;
            } else {
            // ============ one update: location r = r0 ============
            prow = rs.u.sq.prow[pbuf];           // row r, column p(r)
            const int16_t *pcol = rs.u.sq.pcol[pbuf];
            af = a_next;                        // a = p(r)
            const int nr = r + 1 < N ? r + 1 : 0;
            int nxt_v;                          // p(nr) before this update
            PDIT_REG_POLL({ PDIT_REG_READS(prow, pcol, r, af) nxt_v = rs.pv[nr]; })
            PDIT_REG_DELTA(r)
            if (lane == 0) rs.smin[wv] = mw;
            rep_signal(rs.sync, wv, ++seq);
            // the minimum over k != r; with it the uniform of r and p of every
            // candidate (nothing writes them before the next meeting)
            v4i mv;
            uint32_t ur_v;
            PDIT_REG_POLL({
                mv = *(const v4i *)rs.smin;
                ur_v = rs.u24[r];
                pw0 = rs.pv[lane];
                pw1 = rs.pv[64 + lane];
                pw2 = rs.pv[128 + lane];
                pw3 = rs.pv[192 + lane];
            })
            const int32_t m2 = __builtin_amdgcn_readfirstlane(min(min(mv.x, mv.y), min(mv.z, mv.w)));
            int tie = 0;
            bf = af;
            if (m2 < dthr) PDIT_REG_DRAW(r, dv, m2, ur_v, s, tie, des, bf)
            if (!ok) break;
            n_tie += tie;
            if (ch && lane == 0) ch[r] = s;
            nxt = __builtin_amdgcn_readfirstlane(nxt_v);
            }
            // ============ the accepted exchange (the step's only one) ============
            if (s != r) PDIT_REG_ACCEPT(r, s, af, bf, des, prow)
            r0 = r + 1;
            if (nbat) {
                replayed = true;
            } else {
                // p(r + 1) after this update, and the next update's row and column
                // (the next sweep's first, unless it runs in batches)
                const int nr = r + 1 < N ? r + 1 : 0;
                a_next = (s != r && s == nr) ? af : nxt;
                if (r0 < N || !PDIT_REG_NEXT_BATCH()) {
                    pbuf ^= 1;
                    PDIT_REG_PUBLISH(nr, a_next, pbuf)
                }
            }
            rep_signal(rs.sync, wv, ++seq);
        }
        if (ok && nbat && !PDIT_REG_NEXT_BATCH()) {
            // the next sweep goes one update at a time: its first row and column,
            // once every wave has left the batch buffers they share
            if (!rep_done(*flags, seq)) ok = rep_spin(flags, seq);
            a_next = __builtin_amdgcn_readfirstlane(rs.pv[0]);
            pbuf ^= 1;
            PDIT_REG_PUBLISH(0, a_next, pbuf)
            rep_signal(rs.sync, wv, ++seq);
        }
        nbat = !PDIT_REG_NEXT_BATCH()      ? 0
             : n_acc - acc0 <= kRAcc12 ? kRSpec
             : n_acc - acc0 <= kRAcc8  ? 8
                                       : 4;
#undef PDIT_REG_NEXT_BATCH
        if (a.E_trace && writer && lane == 0) a.E_trace[rep * a.T + t] = E;
    }
#undef PDIT_REG_POLL
#undef PDIT_REG_DRAW
#undef PDIT_REG_STORE_COL
#undef PDIT_REG_PUBLISH
#undef PDIT_REG_READS
#undef PDIT_REG_DELTA
#undef PDIT_REG_ACCEPT

    // ---- outputs ----
    if (!ok && a.err) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (live && kval) a.perm[rep * N + k] = pk;
    if (writer && lane == 0) {
        a.E[rep] = E;
        a.E_best[rep] = E_best;
        const bool accum = (a.flags & kAccumCounters) != 0;
        a.counters[3 * rep + 0] = (accum ? a.counters[3 * rep + 0] : 0) + (int64_t)N * a.T;
        a.counters[3 * rep + 1] = (accum ? a.counters[3 * rep + 1] : 0) + n_acc;
        a.counters[3 * rep + 2] = (accum ? a.counters[3 * rep + 2] : 0) + n_tie;
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
