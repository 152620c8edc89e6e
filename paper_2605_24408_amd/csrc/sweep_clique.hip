// sweep_clique.hip -- the p-dit sweep specialised to clique flows (Methods,
// "CPU-PIM Algorithm", the tai256c instance): F[a][b] = 1 for two distinct
// facilities of a clique C and 0 otherwise, D symmetric with a zero diagonal.
//
// Eq. 1 then depends only on the set S of locations holding clique
// facilities: E = sum over i, j in S of D[i][j].  With g(x) = sum_{j in S}
// D[x][j], the energy change of exchanging locations r and s (Eq. 3) is 0
// when both are in S or both outside, 2 (g(s) - g(r) - D[r][s]) when r is in
// S and s is not, and 2 (g(r) - g(s) - D[r][s]) the other way round.  An
// accepted exchange across the classes moves S and changes g by
// +-(D[x][s] - D[x][r]); one inside a class only exchanges two entries of p.
// So a candidate costs O(1) and an accepted move O(N) instead of O(N^2): the
// simplification the paper describes.  The dynamics (order of updates,
// candidates, weights, CDF, Philox stream, best tracking) are exactly those
// of the general sweep.
//
// One wave per replica, every location's state in registers: lane l holds
// locations l, l + 64, ... (p, class bit, g); D rows are read from device
// memory (shared by all replicas, so L2-resident).  An exchange inside a
// class changes no energy change of any row, so rows are drawn a few at a
// time from one state and committed in order up to the first exchange across
// the classes.
#include "device_common.h"
#include "pdit_internal.h"

#include <type_traits>

namespace pdit {
namespace {

constexpr int32_t kExcluded = (1 << 30) - 1;  // lanes beyond N
constexpr uint32_t kOne = kWeightOne;

// element c of a register array, c wave-uniform
template <int CPL, typename T>
__device__ __forceinline__ T pick(const T (&v)[CPL], int c) {
    T out = v[0];
#pragma unroll
    for (int k = 1; k < CPL; ++k)
        if (c == k) out = v[k];
    return out;
}

template <int CPL, int RB, bool REC>
__global__ void __launch_bounds__(64 * RB) sweep_clique_kernel(CliqueArgs a) {
    using CT = typename std::conditional<(CPL == 1), uint32_t, uint64_t>::type;
    __shared__ int32_t sm_sel[2][RB], sm_v[2][RB], sm_tie[2][RB];
    const int N = a.N;
    const int64_t rep = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    int par = 0;
    const int32_t *D = a.D;
    int32_t *perm = a.perm + rep * N;
    int32_t *pbest = a.perm_best + rep * N;

    int32_t pv[CPL], g[CPL];
    bool in[CPL], valid[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int x = lane + 64 * c;
        valid[c] = x < N;
        pv[c] = valid[c] ? perm[x] : 0;
        in[c] = valid[c] && a.member[pv[c]] != 0;
        g[c] = 0;
    }
    // g(x) = sum over j in S of D[j][x] (D symmetric), row by row
    for (int j = 0; j < N; ++j) {
        const bool inj = __builtin_amdgcn_readlane((int)pick<CPL>(in, j >> 6), j & 63) != 0;
        if (!inj) continue;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (valid[c]) g[c] += D[(int64_t)j * N + lane + 64 * c];
    }
    int64_t E = 0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) E += in[c] ? (int64_t)g[c] : 0;
    for (int off = 32; off > 0; off >>= 1) E += __shfl_xor(E, off);
    int64_t E_best = a.init_best ? E : a.E_best[rep];
    if (a.init_best && wv == 0)
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            if (valid[c]) pbest[lane + 64 * c] = pv[c];
    int64_t n_acc = 0, n_tie = 0;

    float bcache = 0.0f;
    int32_t dcache = 0;
    for (int64_t t = 0; t < a.T; ++t) {
        const int slot = (int)(t & 63);
        if (slot == 0) {
            const int64_t tt = t + lane < a.T ? t + lane : a.T - 1;
            bcache = a.beta[tt];
            dcache = zero_weight_distance(bcache);
        }
        const float beta = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bcache), slot));
        const int32_t dthr = __builtin_amdgcn_readlane(dcache, slot);
        const uint32_t gs = (uint32_t)(a.sweep_offset + (uint64_t)t);
        uint32_t u24l[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            u24l[c] = uniform24(a.seed, (uint32_t)(lane + 64 * c), gs, (uint32_t)rep, a.inst);
        int32_t *ch = (REC && a.choices) ? a.choices + (rep * a.T + t) * N : nullptr;
        // Rows are drawn RB at a time, one per wave, from the same state: a
        // draw depends only on g and the class bits, which an exchange inside
        // a class leaves unchanged, so the rows of a batch up to its first
        // exchange across the classes are exactly what the one-at-a-time sweep
        // draws.  Every wave commits them in order on its own copy of the
        // state; the next batch starts after that exchange.  Results pass
        // through LDS by batch parity (a wave is at most one batch ahead).
        int r0 = 0;
        while (r0 < N) {
            const int r = r0 + wv;
            if (r < N) {
                const int cr = r >> 6, lr = r & 63;
                int32_t Drow[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    Drow[c] = valid[c] ? D[(int64_t)r * N + lane + 64 * c] : 0;
                const int32_t gr = __builtin_amdgcn_readlane(pick<CPL>(g, cr), lr);
                const bool inr = __builtin_amdgcn_readlane((int)pick<CPL>(in, cr), lr) != 0;
                // energy change of every candidate (the stay's and same-class ones are 0)
                int32_t v[CPL];
                int32_t lmin = kExcluded;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    int32_t d = 0;
                    if (in[c] != inr)
                        d = inr ? 2 * (g[c] - gr - Drow[c]) : 2 * (gr - g[c] - Drow[c]);
                    v[c] = valid[c] ? d : kExcluded;
                    lmin = min(lmin, v[c]);
                }
                const int32_t mn = wave_min_i32(lmin);
                CT C[CPL];
                uint32_t q[CPL];
                CT base = 0;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int32_t d = valid[c] ? v[c] - mn : 0;
                    q[c] = d == 0 ? kOne : 0u;
                    if (d > 0 && d < dthr) q[c] = gibbs_weight(beta, (float)d);
                    if (!valid[c]) q[c] = 0;
                    // one chunk of 64 weights sums to at most 2^31
                    C[c] = base + (CT)wave_scan_u32(q[c]);
                    base = (CT)readlane_u64((uint64_t)C[c], 63);
                }
                const CT Z = base;
                const uint32_t ur24 =
                    (uint32_t)__builtin_amdgcn_readlane((int32_t)pick<CPL>(u24l, cr), lr);
                const CT thr = (CT)(((uint64_t)ur24 * Z) >> 24);
                int sb = -1;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const uint64_t hit = __ballot(C[c] > thr);
                    if (sb < 0 && hit) sb = 64 * c + __ffsll((unsigned long long)hit) - 1;
                }
                if (sb < 0 || sb >= N) sb = r;  // unreachable: location N-1 holds C = Z > thr
                const int cs = sb >> 6, ls = sb & 63;
                const CT csel = (CT)readlane_u64((uint64_t)pick<CPL>(C, cs), ls);
                const uint32_t qsel = (uint32_t)__builtin_amdgcn_readlane((int32_t)pick<CPL>(q, cs), ls);
                const int32_t vs = __builtin_amdgcn_readlane(pick<CPL>(v, cs), ls);
                const bool tie = is_tie(csel - qsel, csel, Z, ur24);
                if (lane == 0) {
                    sm_sel[par][wv] = sb;
                    sm_v[par][wv] = vs;
                    sm_tie[par][wv] = tie ? 1 : 0;
                }
            }
            __syncthreads();
            // commit in order, up to and including the first exchange across the classes
            int next = r0 + RB;
            for (int b = 0; b < RB; ++b) {
                const int rb = r0 + b;
                if (rb >= N || rb >= next) break;
                const int sb = __builtin_amdgcn_readfirstlane(sm_sel[par][b]);
                n_tie += __builtin_amdgcn_readfirstlane(sm_tie[par][b]);
                if (REC && ch && wv == 0 && lane == 0) ch[rb] = sb;
                if (sb == rb) continue;
                ++n_acc;
                const int cr = rb >> 6, lr = rb & 63, cs = sb >> 6, ls = sb & 63;
                const bool inr = __builtin_amdgcn_readlane((int)pick<CPL>(in, cr), lr) != 0;
                const bool ins = __builtin_amdgcn_readlane((int)pick<CPL>(in, cs), ls) != 0;
                const int32_t pr = __builtin_amdgcn_readlane(pick<CPL>(pv, cr), lr);
                const int32_t ps = __builtin_amdgcn_readlane(pick<CPL>(pv, cs), ls);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int x = lane + 64 * c;
                    if (x == rb) {
                        pv[c] = ps;
                        in[c] = ins;
                    } else if (x == sb) {
                        pv[c] = pr;
                        in[c] = inr;
                    }
                }
                if (ins == inr) continue;  // inside a class: E, S and g unchanged
                // across the classes: r in S: S loses r, gains s, g += D[.][s] - D[.][r];
                // else the reverse
                E += __builtin_amdgcn_readfirstlane(sm_v[par][b]);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int32_t drx = valid[c] ? D[(int64_t)rb * N + lane + 64 * c] : 0;
                    const int32_t dsx = valid[c] ? D[(int64_t)sb * N + lane + 64 * c] : 0;
                    g[c] += inr ? dsx - drx : drx - dsx;
                }
                if (E < E_best) {
                    E_best = E;
                    if (wv == 0)
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            if (valid[c]) pbest[lane + 64 * c] = pv[c];
                }
                next = rb + 1;
            }
            r0 = next;
            par ^= 1;
        }
        if (REC && a.E_trace && wv == 0 && lane == 0) a.E_trace[rep * a.T + t] = E;
    }
    if (wv != 0) return;  // every wave holds the same state
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        if (valid[c]) perm[lane + 64 * c] = pv[c];
    if (lane == 0) {
        a.E[rep] = E;
        a.E_best[rep] = E_best;
        a.counters[3 * rep + 0] = (int64_t)N * a.T;
        a.counters[3 * rep + 1] = n_acc;
        a.counters[3 * rep + 2] = n_tie;
    }
}

template <int CPL>
hipError_t launch_cpl(hipStream_t s, const CliqueArgs &a) {
    constexpr int RB = 4;  // rows drawn together, one wave each
    if (a.choices || a.E_trace)
        sweep_clique_kernel<CPL, RB, true><<<a.R, 64 * RB, 0, s>>>(a);
    else
        sweep_clique_kernel<CPL, RB, false><<<a.R, 64 * RB, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_clique(hipStream_t s, const CliqueArgs &a) {
    switch ((a.N + 63) / 64) {
        case 1: return launch_cpl<1>(s, a);
        case 2: return launch_cpl<2>(s, a);
        case 3: return launch_cpl<3>(s, a);
        case 4: return launch_cpl<4>(s, a);
        case 5: return launch_cpl<5>(s, a);
        case 6: return launch_cpl<6>(s, a);
        case 7: return launch_cpl<7>(s, a);
        case 8: return launch_cpl<8>(s, a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pdit
