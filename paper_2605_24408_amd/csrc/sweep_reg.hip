// sweep_reg.hip -- the sweep kernel that keeps a replica's state in
// registers, for 128 < N <= 256 with D and F held as 8-bit copies.
//
// The state is G = D F[p,:] (location x facility): G[i][c] = sum_j D[i][j]
// F[p(j)][c], so H = D F[p,p] is H[i][k] = G[i][p(k)].  Lane l of a
// replica's 256 lanes (four waves) owns location l and keeps row l of G in
// 128 registers as packed int16 pairs (exact while |H| <= 32767), and diag
// H[l][l].  An accepted exchange of the facilities a = p(r) and b = p(s)
// changes G by one rank-1 term and moves no column (Methods, "CPU-PIM
// Algorithm": the influence is kept incrementally; with symmetric data
// I = -2H, Eq. 2):
//   G'[i][c] = G[i][c] + (D[i][r] - D[i][s]) (F[b][c] - F[a][c]),
// 128 packed multiply-adds per lane.
//
// The update of location r (Results, "Implementation": locations 0..N-1 in
// order; Eq. 3 and Eq. 5) needs row r of H, H[r][k] = G[r][p(k)] (lane r
// writes its row to LDS, lane k reads entry p(k)), column r, H[k][r] =
// G[k][p(r)] (each lane reads its own register at the uniform index p(r)),
// and the diagonal.  Then
//   dE_k = 2 (H[r][k] - H[r][r] + H[k][r] - H[k][k])
//          + (D_rr + D_kk - 2 D_rk)(F_aa + F_cc - 2 F_ac),  c = p(k),
// the row minimum, the integer Gibbs weights q = rint(expf(-beta d) 2^25)
// and their exact 64-bit CDF, as in the other sweep kernels, so every kernel
// draws the same candidate.  A row whose only nonzero weight is its own
// stay (the minimum is 0 and every other candidate lies beyond the
// zero-weight distance) keeps its facility without weights or scan.
//
// Two replicas share a workgroup (eight waves) and its LDS: D and F as 8-bit
// copies (64 KB each, unsigned in [0, 255] or signed in [-128, 127]), so
// every read of D and F on the path is an LDS read.  The two replicas move
// in step: an update takes four workgroup barriers whatever happens in it.
#include "device_common.h"
#include "pdit_internal.h"
#include "sweep_common.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int kRN = 256;          // locations (lanes) per replica
constexpr int kRWaves = 4;        // waves per replica
constexpr int kRReps = 2;         // replicas per workgroup
constexpr int kRThreads = 64 * kRWaves * kRReps;
constexpr int kRBlock = 16;       // rows of G copied to LDS together
constexpr int32_t kRBig = (1 << 30) - 1;  // padding candidates (|dE| < 2^30 - 1)
// spins of a replica's wait before it gives up (about 0.1 s): reached only
// if a wave of the replica stopped taking part, which the kernel's uniform
// control flow excludes; the call then reports PDIT_EDEVICE at pdit_sync
constexpr uint32_t kRSpinLimit = 1u << 22;

typedef int v32i __attribute__((ext_vector_type(32)));
typedef short v64s __attribute__((ext_vector_type(64)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));

struct alignas(16) RegRep {
    alignas(16) int16_t blk[kRBlock][kRN];  // rows 16 b .. 16 b + 15 of G, by facility
    alignas(16) uint32_t w[kRN / 2];        // accepted exchange: F[b][c] - F[a][c], int16 pairs
    alignas(16) uint32_t sync[kRWaves];     // per wave: the last step it finished
    int32_t pv[kRN];                        // p(l)
    uint32_t u24[2][kRN];                   // the sweep's uniforms by location, by sweep parity
    int32_t xmin[2][kRWaves][2];            // per wave: minimum, minimum over l != r (update parity)
    uint64_t xz[kRWaves];                   // per wave: sum of the weights
    uint64_t xr[2];                         // the wave of r: exclusive sum at r, weight of r
    int32_t msg[3];                         // accepted: s, dE, p(s)
    int16_t ublk[kRBlock];                  // accepted: u of the block's rows
    int32_t ties[kRWaves];
};

template <bool SGN>
struct RegSmem {
    using E8 = typename std::conditional<SGN, int8_t, uint8_t>::type;
    E8 D[kRN * kRN];             // D, zero outside N x N
    E8 F[kRN * kRN];             // F, zero outside N x N
    RegRep rep[kRReps];
};

// Entry c of a row of 256 int16 values packed in four 32-register vectors;
// c is wave-uniform, so each read is a relative register move.
__device__ __forceinline__ int32_t row_entry(const v32i &g0, const v32i &g1, const v32i &g2,
                                             const v32i &g3, int c) {
    const int cu = __builtin_amdgcn_readfirstlane(c);
    const int k = cu >> 1;
    const int lo = k & 31;
    const int v0 = g0[lo], v1 = g1[lo], v2 = g2[lo], v3 = g3[lo];
    const int hi = k >> 5;
    const int word = hi == 0 ? v0 : hi == 1 ? v1 : hi == 2 ? v2 : v3;
    return (cu & 1) ? (word >> 16) : (int32_t)(int16_t)(word & 0xFFFF);
}

__device__ __forceinline__ uint32_t pack16(int32_t lo, int32_t hi) {
    return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
}

// g += u w elementwise on int16 lanes (modulo 2^16; the true values fit)
__device__ __forceinline__ v32i rank1(v32i g, short u, v32i w) {
    const v64s gs = __builtin_bit_cast(v64s, g);
    const v64s ws = __builtin_bit_cast(v64s, w);
    return __builtin_bit_cast(v32i, gs + (v64s)u * ws);
}

// Wait of the kRWaves waves of one replica (the other replica of the
// workgroup goes on): wave w records that it finished step `seq`, after its
// LDS writes have completed, and waits until every wave of the replica has.
// Returns false when the wait gave up (kRSpinLimit).
__device__ __forceinline__ bool rep_wait(uint32_t *slots, int w, uint32_t seq) {
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __hip_atomic_store(&slots[w], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (uint32_t it = 0; it < kRSpinLimit; ++it) {
        const v4i v = *(volatile const v4i *)slots;
        const bool done = (int32_t)(v.x - seq) >= 0 && (int32_t)(v.y - seq) >= 0 &&
                          (int32_t)(v.z - seq) >= 0 && (int32_t)(v.w - seq) >= 0;
        if (__builtin_amdgcn_readfirstlane((int)done)) {
            __asm__ volatile("" ::: "memory");
            return true;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

template <bool SGN, bool ZD>
__global__ void __launch_bounds__(kRThreads)
sweep_reg_kernel(SweepArgs a) {
    __shared__ __align__(16) RegSmem<SGN> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int qr = wv / kRWaves;       // replica slot of this wave in the workgroup
    const int w = wv % kRWaves;        // wave within the replica
    const int l = 64 * w + lane;       // this lane's location
    const int N = a.N;
    int64_t rep = (int64_t)kRReps * blockIdx.x + qr;
    // an odd last replica: the second slot repeats the first and writes nothing
    const bool live = rep < a.R;
    if (!live) rep = (int64_t)kRReps * blockIdx.x;
    RegRep &rs = sm.rep[qr];
    const bool valid = l < N;

    // ---- D and F copies (both replicas) ----
    for (int e = tid; e < kRN * kRN; e += kRThreads) {
        const int i = e >> 8, j = e & 255;
        const bool in = i < N && j < N;
        sm.D[e] = (typename RegSmem<SGN>::E8)(in ? a.D[(int64_t)i * N + j] : 0);
        sm.F[e] = (typename RegSmem<SGN>::E8)(in ? a.F[(int64_t)i * N + j] : 0);
    }
    // ---- p, p^-1 (padding locations hold the padding facilities) ----
    int p_l = valid ? a.perm[rep * N + l] : l;
    rs.pv[l] = p_l;
    rs.u24[0][p_l] = (uint32_t)l;
    if (lane < kRWaves && w == 0) rs.sync[lane] = 0;
    __syncthreads();

    // ---- row l of G = row l of H reordered by facility: G[l][c] = H[l][p^-1(c)] ----
    const int32_t *Hl = (const int32_t *)a.H + (rep * N + (valid ? l : 0)) * (int64_t)N;
    v32i g0, g1, g2, g3;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
#define PDIT_G_AT(c) ((valid && (c) < N) ? Hl[rs.u24[0][(c)]] : 0)
        g0[k] = (int)pack16(PDIT_G_AT(2 * k), PDIT_G_AT(2 * k + 1));
        g1[k] = (int)pack16(PDIT_G_AT(64 + 2 * k), PDIT_G_AT(64 + 2 * k + 1));
        g2[k] = (int)pack16(PDIT_G_AT(128 + 2 * k), PDIT_G_AT(128 + 2 * k + 1));
        g3[k] = (int)pack16(PDIT_G_AT(192 + 2 * k), PDIT_G_AT(192 + 2 * k + 1));
#undef PDIT_G_AT
    }
    int32_t diag = valid ? Hl[l] : 0;                    // H[l][l]
    const int32_t dd_l = ZD ? 0 : (int32_t)sm.D[l * kRN + l];
    int32_t fd_l = ZD ? 0 : (int32_t)sm.F[p_l * kRN + p_l];
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0;
    int32_t n_tie = 0;
    int32_t *ch_base = (a.choices && live) ? a.choices + rep * a.T * N : nullptr;
    const float *bp = a.slot ? a.beta + a.slot[rep] : a.beta;
    const int64_t bstride = a.slot ? 0 : 1;
    uint32_t seq = 0;      // steps of this replica's waits
    bool ok = true;        // every wait completed
    __syncthreads();       // every read of p^-1 is done before the uniforms reuse the buffer

    for (int64_t t = 0; t < a.T && ok; ++t) {
        const float beta = bp[t * bstride];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        int32_t *ch = ch_base ? ch_base + t * N : nullptr;
        uint32_t *u24 = rs.u24[t & 1];
        u24[l] = uniform24(a.seed, (uint32_t)l, g, (uint32_t)rep, a.inst_id);

        for (int r = 0; r < N && ok; ++r) {
            const int rb = r & (kRBlock - 1);
            if (rb == 0) {
                // rows r .. r + 15 of G to LDS (their lanes are in one wave)
                if ((l & ~(kRBlock - 1)) == r) {
                    v32i *dst = (v32i *)rs.blk[l - r];
                    dst[0] = g0;
                    dst[1] = g1;
                    dst[2] = g2;
                    dst[3] = g3;
                }
                ok = rep_wait(rs.sync, w, ++seq);
            }
            // ================= energy changes of the N candidates =================
            const int af = rs.pv[r];
            const int16_t *hrow = rs.blk[rb];      // H[r][k] = G[r][p(k)]
            int32_t dv = kRBig;
            if (valid) {
                const int32_t hrs = hrow[p_l];
                const int32_t hrr = hrow[af];
                const int32_t hsr = row_entry(g0, g1, g2, g3, af);
                const int32_t x = 2 * (hrs - hrr + hsr - diag);
                const int32_t d_rl = sm.D[r * kRN + l];
                const int32_t f_al = sm.F[af * kRN + p_l];
                if (ZD) {
                    dv = x + 4 * d_rl * f_al;
                } else {
                    const int32_t d_rr = sm.D[r * kRN + r];
                    const int32_t f_aa = sm.F[af * kRN + af];
                    dv = x + (d_rr + dd_l - 2 * d_rl) * (f_aa + fd_l - 2 * f_al);
                }
            }
            {
                const int32_t m1 = wave_min_i32(dv);
                const int32_t m2 = wave_min_i32(l == r ? kRBig : dv);
                if (lane == 0) {
                    rs.xmin[r & 1][w][0] = m1;
                    rs.xmin[r & 1][w][1] = m2;
                }
            }
            ok = ok && rep_wait(rs.sync, w, ++seq);

            // ================= weights and their CDF =================
            int32_t mn = rs.xmin[r & 1][0][0], mn2 = rs.xmin[r & 1][0][1];
#pragma unroll
            for (int k = 1; k < kRWaves; ++k) {
                mn = min(mn, rs.xmin[r & 1][k][0]);
                mn2 = min(mn2, rs.xmin[r & 1][k][1]);
            }
            // only the stay (dE = 0) carries weight: the draw keeps r
            if (mn == 0 && mn2 >= dthr) {
                if (ch && w == 0 && lane == 0) ch[r] = r;
                continue;
            }
            uint32_t qw = 0;
            {
                const int32_t d = dv - mn;
                const bool need = valid && d > 0 && d < dthr;
                if (valid && d == 0) qw = kWeightOne;
                if (__ballot(need)) {
                    if (need) qw = gibbs_weight(beta, (float)d);
                }
            }
            const uint64_t C = wave_scan_u64((uint64_t)qw);
            if (lane == 63) rs.xz[w] = C;
            if (l == r) {
                rs.xr[0] = C - qw;
                rs.xr[1] = qw;
            }
            ok = ok && rep_wait(rs.sync, w, ++seq);

            // ================= the draw =================
            uint64_t off = 0, Z = 0, off_r = 0;
#pragma unroll
            for (int k = 0; k < kRWaves; ++k) {
                const uint64_t zk = rs.xz[k];
                if (k < w) off += zk;
                if (k < (r >> 6)) off_r += zk;
                Z += zk;
            }
            const uint32_t ur = u24[r];
            const uint64_t thr = ((uint64_t)ur * Z) >> 24;  // first C > thr
            const uint64_t c_prev = off_r + rs.xr[0];
            const bool stay = c_prev <= thr && thr < c_prev + rs.xr[1];
            const uint64_t zw = rs.xz[w];
            if (off <= thr && thr < off + zw) {  // the wave holding the threshold
                const uint64_t cg = off + C;
                const uint64_t hit = __ballot(valid && cg > thr);
                const int sl = __ffsll((unsigned long long)hit) - 1;
                const int s = 64 * w + sl;
                const uint64_t csel = readlane_u64(cg, sl);
                const uint32_t qsel = (uint32_t)__builtin_amdgcn_readlane((int32_t)qw, sl);
                n_tie += is_tie(csel - qsel, csel, Z, ur) ? 1 : 0;
                if (ch && lane == 0) ch[r] = s;
                if (s != r) {
                    const int32_t dsel = __builtin_amdgcn_readlane(dv, sl);
                    const int bf = rs.pv[s];
                    // F[b][c] - F[a][c] for c = 4 lane .. 4 lane + 3, as two int16 pairs
                    const uint32_t fa4 = ((const uint32_t *)sm.F)[af * (kRN / 4) + lane];
                    const uint32_t fb4 = ((const uint32_t *)sm.F)[bf * (kRN / 4) + lane];
                    int32_t dw[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int32_t xa = SGN ? (int32_t)(int8_t)(fa4 >> (8 * k))
                                               : (int32_t)((fa4 >> (8 * k)) & 0xFF);
                        const int32_t xb = SGN ? (int32_t)(int8_t)(fb4 >> (8 * k))
                                               : (int32_t)((fb4 >> (8 * k)) & 0xFF);
                        dw[k] = xb - xa;
                    }
                    rs.w[2 * lane] = pack16(dw[0], dw[1]);
                    rs.w[2 * lane + 1] = pack16(dw[2], dw[3]);
                    if (lane < kRBlock) {
                        // u of the block's rows: D[i][r] - D[i][s], i = 16 (r / 16) + lane
                        const int i = (r & ~(kRBlock - 1)) + lane;
                        rs.ublk[lane] = (int16_t)((int32_t)sm.D[r * kRN + i] -
                                                  (int32_t)sm.D[s * kRN + i]);
                    }
                    if (lane == 0) {
                        rs.msg[0] = s;
                        rs.msg[1] = dsel;
                        rs.msg[2] = bf;
                    }
                }
            }
            if (stay) continue;
            ok = ok && rep_wait(rs.sync, w, ++seq);

            // ================= accepted exchange of r and s =================
            {
                const int s = rs.msg[0];
                const int bf = rs.msg[2];
                E += rs.msg[1];
                ++n_acc;
                // u_l = D[l][r] - D[l][s] (rows r and s of the symmetric D)
                const int32_t u = valid ? (int32_t)sm.D[r * kRN + l] - (int32_t)sm.D[s * kRN + l] : 0;
                const v32i *wv32 = (const v32i *)rs.w;
                g0 = rank1(g0, (short)u, wv32[0]);
                g1 = rank1(g1, (short)u, wv32[1]);
                g2 = rank1(g2, (short)u, wv32[2]);
                g3 = rank1(g3, (short)u, wv32[3]);
                // the block's copy of rows 16 (r / 16) + i: lane (i, j) moves
                // columns 16 j .. 16 j + 15 of row i
                {
                    const int i = l >> 4, j = l & 15;
                    const short ui = rs.ublk[i];
                    v8s *bp8 = (v8s *)&rs.blk[i][16 * j];
                    const v8s *wp8 = (const v8s *)&rs.w[8 * j];
                    const v8s b0 = bp8[0], b1 = bp8[1];
                    bp8[0] = b0 + (v8s)ui * wp8[0];
                    bp8[1] = b1 + (v8s)ui * wp8[1];
                }
                // diag H: H'[l][l] = G'[l][p'(l)]; off {r, s} p(l) stays and
                // the change is u_l (F[b][p(l)] - F[a][p(l)])
                const int32_t at_b = row_entry(g0, g1, g2, g3, bf);
                const int32_t at_a = row_entry(g0, g1, g2, g3, af);
                if (l == r) {
                    p_l = bf;
                    diag = at_b;
                } else if (l == s) {
                    p_l = af;
                    diag = at_a;
                } else {
                    diag += u * (int32_t)((const int16_t *)rs.w)[p_l];
                }
                if (!ZD && (l == r || l == s)) fd_l = (int32_t)sm.F[p_l * kRN + p_l];
                if (l == r || l == s) rs.pv[l] = p_l;
                if (E < E_best) {
                    E_best = E;
                    if (live && valid) a.perm_best[rep * N + l] = p_l;
                }
            }
            ok = ok && rep_wait(rs.sync, w, ++seq);
        }
        if (a.E_trace && live && l == 0) a.E_trace[rep * a.T + t] = E;
    }

    // ---- outputs ----
    if (!ok && a.err) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) rs.ties[w] = n_tie;
    __syncthreads();
    if (live) {
        if (valid) a.perm[rep * N + l] = p_l;
        if (l == 0) {
            int64_t ties = 0;
#pragma unroll
            for (int k = 0; k < kRWaves; ++k) ties += rs.ties[k];
            a.E[rep] = E;
            a.E_best[rep] = E_best;
            const bool accum = (a.flags & kAccumCounters) != 0;
            a.counters[3 * rep + 0] = (accum ? a.counters[3 * rep + 0] : 0) + (int64_t)N * a.T;
            a.counters[3 * rep + 1] = (accum ? a.counters[3 * rep + 1] : 0) + n_acc;
            a.counters[3 * rep + 2] = (accum ? a.counters[3 * rep + 2] : 0) + ties;
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
