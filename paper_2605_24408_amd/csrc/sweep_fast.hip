// sweep_fast.hip -- the sweep kernel with H on chip.
//
// One wave64 owns one replica; its H (int32, N <= 64) lives in LDS for the
// whole run, D and F are staged once per workgroup, and the sweep order of
// the method (locations 0..N-1, each a Gibbs choice among N candidates,
// Results "Implementation", Eq. 3 and Eq. 5) is kept exactly.
//
// Two schedules give the same result:
//
//  * speculative rows (cold sweeps).  An update that keeps its facility
//    ("stay") leaves H unchanged, so the choices of locations pos..N-1 can be
//    evaluated all at once from the current H, lane l computing row l (its N
//    candidates in ascending order).  The rows up to the first lane that
//    swaps are exactly what the sequential method would do; that swap is
//    applied and evaluation restarts after it.  A sweep with k swaps costs
//    k + 1 such passes.
//
//  * one update at a time (hot sweeps).  Lanes hold the N candidates of the
//    current location; the minimum and the running weight sum are wave
//    reductions.  Used for a sweep when the previous one accepted more than
//    `seq_threshold` swaps.
//
// The Gibbs weights are exact integers (q = rint(w 2^30)) summed in 64 bits,
// so both schedules, whatever their summation order, select the same
// candidate.  Candidates whose distance to the row minimum makes w < 2^-31
// have q = 0 and skip the exponential.
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

struct LaneAux {  // per-location data broadcast from LDS
    int32_t fac;  // p(l)
    int32_t hd;   // H[l][l]
    int32_t dd;   // D[l][l]
    int32_t fd;   // F[p(l)][p(l)]
};

template <int NMAX, int W>
__global__ void __launch_bounds__(64 * W) sweep_fast_kernel(SweepArgs a) {
    constexpr int P = NMAX + 1;  // padded H row: column reads are conflict-free
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    int32_t *Ds = reinterpret_cast<int32_t *>(smem);                 // [NMAX][NMAX]
    int32_t *Fs = Ds + NMAX * NMAX;                                   // [NMAX][NMAX]
    LaneAux *Ua = reinterpret_cast<LaneAux *>(Fs + NMAX * NMAX);      // [W][NMAX]
    int32_t *Hall = reinterpret_cast<int32_t *>(Ua + W * NMAX);       // [W][NMAX][P]

    const int N = a.N;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t rep = (int64_t)blockIdx.x * W + w;

    // ---- stage D, F (zero outside N) and this wave's H ----
    for (int e = threadIdx.x; e < NMAX * NMAX; e += 64 * W) {
        const int i = e / NMAX, j = e % NMAX;
        const bool in = i < N && j < N;
        Ds[e] = in ? a.D[(int64_t)i * N + j] : 0;
        Fs[e] = in ? a.F[(int64_t)i * N + j] : 0;
    }
    int32_t *Hs = Hall + w * NMAX * P;
    LaneAux *U = Ua + w * NMAX;
    const bool active = rep < a.R;
    if (active) {
        const int32_t *Hg = (const int32_t *)a.H + rep * (int64_t)N * N;
        for (int e = lane; e < NMAX * P; e += 64) {
            const int i = e / P, k = e % P;
            Hs[e] = (i < N && k < N) ? Hg[(int64_t)i * N + k] : 0;
        }
    }
    __syncthreads();
    if (!active) return;

    const bool lv = lane < N;
    // lanes >= NMAX (small templates) address location 0 so that every LDS
    // access stays inside this wave's arrays; their results are never used
    const int ll = lane < NMAX ? lane : 0;
    int32_t p = lv ? a.perm[rep * N + lane] : 0;
    const int32_t dd = lv ? Ds[ll * NMAX + ll] : 0;
    int32_t fd = Fs[p * NMAX + p];
    int32_t hd = Hs[ll * P + ll];
    if (lane < NMAX) U[lane] = LaneAux{p, hd, dd, fd};
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0, n_tie = 0;
    const int seq_thr = a.seq_threshold;
    bool seq_mode = false;

    // ---- apply an accepted swap of locations r and s (energy change dE) ----
    auto apply_swap = [&](int r, int s, int64_t dE) {
        E += dE;
        ++n_acc;
        const int32_t fa = __builtin_amdgcn_readlane(p, r);
        const int32_t fb = __builtin_amdgcn_readlane(p, s);
        // u_i = D[i][s] - D[i][r]; column k of the new H is column src(k) of
        // H + u v^T, with v_src = F[a][p(src)] - F[b][p(src)]
        const int32_t u = Ds[s * NMAX + ll] - Ds[r * NMAX + ll];
        const int src = lane == r ? s : lane == s ? r : ll;
        const int32_t cf = lane == r ? fb : lane == s ? fa : p;
        const int32_t v = Fs[fa * NMAX + cf] - Fs[fb * NMAX + cf];
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i < N) {
                const int32_t ui = __builtin_amdgcn_readlane(u, i);
                const int32_t x = Hs[i * P + src];
                if (lv) Hs[i * P + lane] = x + ui * v;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == r) {
            p = fb;
        } else if (lane == s) {
            p = fa;
        }
        fd = Fs[p * NMAX + p];
        hd = Hs[ll * P + ll];
        if (lane < NMAX) U[lane] = LaneAux{p, hd, dd, fd};
        __builtin_amdgcn_wave_barrier();
        if (E < E_best) {
            E_best = E;
            if (lv) a.perm_best[rep * N + lane] = p;
        }
    };

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = a.beta[t];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        const uint32_t u24 = uniform24(a.seed, (uint32_t)lane, g, (uint32_t)rep, a.inst_id);
        const int64_t acc_before = n_acc;
        int32_t *ch = a.choices ? a.choices + (rep * a.T + t) * N : nullptr;

        if (!seq_mode) {
            // ================= speculative rows: lane = location =================
            int pos = 0;
            while (pos < N) {
                const bool rowv = lv && lane >= pos;
                int32_t dl[NMAX];
                int32_t mn = INT32_MAX;
                int am = 0;
#pragma unroll
                for (int s = 0; s < NMAX; ++s) {
                    if (s < N) {
                        const LaneAux us = U[s];
                        const int32_t h = Hs[ll * P + s] + Hs[s * P + ll] - hd - us.hd;
                        const int32_t dv = Ds[s * NMAX + ll];
                        const int32_t fv = Fs[us.fac * NMAX + p];
                        const int32_t v = 2 * h + (dd + us.dd - 2 * dv) * (fd + us.fd - 2 * fv);
                        dl[s] = v;
                        if (v < mn) {
                            mn = v;
                            am = s;
                        }
                    } else {
                        dl[s] = 0;
                    }
                }
                // weights: d = 0 -> 2^30 exactly; d >= dthr -> 0; else expf
                uint32_t ql[NMAX];
                uint64_t Z = 0;
                int nlive = 0;
#pragma unroll
                for (int s = 0; s < NMAX; ++s) {
                    if (s < N) {
                        const int32_t d = dl[s] - mn;
                        uint32_t q = d == 0 ? (1u << 30) : 0u;
                        const bool need = d > 0 && d < dthr;
                        if (__ballot(need)) {
                            if (need) q = gibbs_weight(beta, (float)d);
                        }
                        ql[s] = q;
                        Z += q;
                        nlive += q != 0;
                    } else {
                        ql[s] = 0;
                    }
                }
                int sel = am;
                int32_t dsel = mn;
                bool tie = false;
                if (__ballot(rowv && nlive > 1)) {
                    const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
                    uint64_t C = 0, cprev = 0, csel = 0;
                    bool found = false;
#pragma unroll
                    for (int s = 0; s < NMAX; ++s) {
                        if (s < N) {
                            const uint64_t c0 = C;
                            C += ql[s];
                            const bool hit = !found && C > thr;
                            if (hit) {
                                sel = s;
                                dsel = dl[s];
                                cprev = c0;
                                csel = C;
                            }
                            found = found || hit;
                        }
                    }
                    if (nlive > 1) tie = is_tie(cprev, csel, Z, u24);
                }
                const uint64_t acc_mask = __ballot(rowv && sel != lane);
                const int last = acc_mask ? __ffsll((unsigned long long)acc_mask) - 1 : N - 1;
                const bool committed = rowv && lane <= last;
                n_tie += __popcll(__ballot(committed && tie));
                if (ch && committed) ch[lane] = sel;
                if (acc_mask) {
                    const int s = __builtin_amdgcn_readlane(sel, last);
                    const int32_t dE = __builtin_amdgcn_readlane(dsel, last);
                    apply_swap(last, s, (int64_t)dE);
                }
                pos = last + 1;
            }
        } else {
            // ================= one update at a time: lane = candidate =================
            for (int r = 0; r < N; ++r) {
                const LaneAux ur = U[r];
                int32_t v = INT32_MAX;
                if (lv) {
                    const int32_t h = Hs[r * P + lane] + Hs[lane * P + r] - ur.hd - hd;
                    const int32_t dv = Ds[r * NMAX + lane];
                    const int32_t fv = Fs[ur.fac * NMAX + p];
                    v = 2 * h + (ur.dd + dd - 2 * dv) * (ur.fd + fd - 2 * fv);
                }
                const int32_t mn = wave_min_i32(v);
                const int32_t d = lv ? v - mn : 0;
                uint32_t q = 0;
                if (lv) {
                    q = d == 0 ? (1u << 30) : 0u;
                    if (d > 0 && d < dthr) q = gibbs_weight(beta, (float)d);
                }
                const uint64_t C = wave_scan_u64(q);
                const uint64_t Z = readlane_u64(C, 63);
                const uint32_t ur24 = (uint32_t)__builtin_amdgcn_readlane((int32_t)u24, r);
                const uint64_t thr = ((uint64_t)ur24 * Z) >> 24;
                const uint64_t hit = __ballot(C > thr);
                int s = __ffsll((unsigned long long)hit) - 1;
                if (s < 0 || s >= N) s = r;  // unreachable: lane N-1 holds C = Z > thr
                const uint64_t csel = readlane_u64(C, s);
                const uint64_t cprev = csel - (uint32_t)__builtin_amdgcn_readlane((int32_t)q, s);
                n_tie += is_tie(cprev, csel, Z, ur24) ? 1 : 0;
                if (ch && lane == 0) ch[r] = s;
                if (s != r) apply_swap(r, s, (int64_t)__builtin_amdgcn_readlane(v, s));
            }
        }
        seq_mode = (n_acc - acc_before) > seq_thr;
        if (a.E_trace && lane == 0) a.E_trace[rep * a.T + t] = E;
    }

    if (lv) a.perm[rep * N + lane] = p;
    if (lane == 0) {
        a.E[rep] = E;
        a.E_best[rep] = E_best;
        a.counters[rep * 3 + 0] = (int64_t)N * a.T;
        a.counters[rep * 3 + 1] = n_acc;
        a.counters[rep * 3 + 2] = n_tie;
    }
}

template <int NMAX, int W>
hipError_t launch_fast(hipStream_t s, const SweepArgs &a) {
    constexpr size_t kLds = sizeof(int32_t) * 2 * NMAX * NMAX + sizeof(LaneAux) * W * NMAX +
                            sizeof(int32_t) * W * NMAX * (NMAX + 1);
    const unsigned blocks = (unsigned)((a.R + W - 1) / W);
    hipError_t e = hipFuncSetAttribute((const void *)sweep_fast_kernel<NMAX, W>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
    if (e != hipSuccess) return e;
    sweep_fast_kernel<NMAX, W><<<blocks, 64 * W, kLds, s>>>(a);
    return hipGetLastError();
}

}  // namespace

bool sweep_fast_supports(int N) { return N >= 2 && N <= 64; }

hipError_t launch_sweep_fast(hipStream_t s, const SweepArgs &a0) {
    SweepArgs a = a0;
    if (a.seq_threshold < 0) a.seq_threshold = 3;
    if (a.N <= 16) return launch_fast<16, 4>(s, a);
    if (a.N <= 32) return launch_fast<32, 4>(s, a);
    return launch_fast<64, 4>(s, a);
}

}  // namespace pdit
