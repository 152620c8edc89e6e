// sweep_plain.hip -- the straightforward sweep kernel: one workgroup per
// replica, H kept in device memory (int32 or int64), LDS tree reductions.
//
// Per update of location r (Results, "Implementation"; Eq. 3 and Eq. 5):
//   dE_s = 2 (H_rs + H_sr - H_rr - H_ss) + (D_rr + D_ss - 2 D_rs)
//          (F_aa + F_cc - 2 F_ac),  a = p(r), c = p(s)          (Eq. 3, I = -2H)
//   Gibbs choice among s = 0..N-1 (s = r is "stay")            (Eq. 5)
//   on a swap of r and s*, with b = p(s*):
//     H_ik += (D_is* - D_ir) (F_a,p(k) - F_b,p(k)), then columns r and s* of
//     H are exchanged, which gives D F[p',p'] for the new permutation p'.
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const int64_t m = red[0];
    __syncthreads();
    return m;
}

template <typename HT>
__global__ void __launch_bounds__(kBlock) sweep_plain_kernel(SweepArgs a) {
    __shared__ int32_t p[PDIT_NMAX];
    __shared__ int64_t dE[PDIT_NMAX];
    __shared__ uint64_t C[PDIT_NMAX];
    __shared__ uint64_t Ctmp[PDIT_NMAX];
    __shared__ int32_t uvec[PDIT_NMAX];
    __shared__ int32_t vvec[PDIT_NMAX];
    __shared__ int64_t red[kBlock];
    __shared__ int32_t sel_sh, tie_sh;

    const int N = a.N;
    const int64_t rep = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int32_t *__restrict__ D = a.D;
    const int32_t *__restrict__ F = a.F;
    HT *__restrict__ H = (HT *)a.H + rep * (int64_t)N * N;

    for (int s = tid; s < N; s += nt) p[s] = a.perm[rep * N + s];
    int64_t E = a.E[rep];
    int64_t E_best = a.E_best[rep];
    int64_t n_acc = 0, n_tie = 0;
    __syncthreads();

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = a.beta[t];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int32_t dthr = zero_weight_distance(beta);
        for (int r = 0; r < N; ++r) {
            // ---- energy change of every candidate (Eq. 3) ----
            const int fa = p[r];
            const int64_t hrr = H[(int64_t)r * N + r];
            const int64_t drr = D[(int64_t)r * N + r];
            const int64_t faa = F[(int64_t)fa * N + fa];
            int64_t lmin = INT64_MAX;
            for (int s = tid; s < N; s += nt) {
                const int c = p[s];
                const int64_t h = (int64_t)H[(int64_t)r * N + s] + (int64_t)H[(int64_t)s * N + r] -
                                  hrr - (int64_t)H[(int64_t)s * N + s];
                const int64_t dd = drr + D[(int64_t)s * N + s] - 2 * (int64_t)D[(int64_t)r * N + s];
                const int64_t ff = faa + F[(int64_t)c * N + c] - 2 * (int64_t)F[(int64_t)fa * N + c];
                const int64_t v = 2 * h + dd * ff;
                dE[s] = v;
                lmin = min(lmin, v);
            }
            const int64_t m = block_min_i64(lmin, red);
            if (tid == 0) {
                sel_sh = r;  // overwritten below: exactly one candidate holds the threshold
                tie_sh = 0;
            }
            // ---- Gibbs weights and their running sum (Eq. 5) ----
            for (int s = tid; s < N; s += nt) {
                const int64_t d = dE[s] - m;
                C[s] = d < (int64_t)dthr ? gibbs_weight(beta, (float)d) : 0u;
            }
            __syncthreads();
            for (int off = 1; off < N; off <<= 1) {
                for (int s = tid; s < N; s += nt) Ctmp[s] = C[s] + (s >= off ? C[s - off] : 0);
                __syncthreads();
                for (int s = tid; s < N; s += nt) C[s] = Ctmp[s];
                __syncthreads();
            }
            const uint64_t Z = C[N - 1];
            const uint32_t u24 = uniform24(a.seed, (uint32_t)r, g, (uint32_t)rep, a.inst_id);
            const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
            for (int s = tid; s < N; s += nt) {
                const uint64_t prev = s > 0 ? C[s - 1] : 0;
                if (prev <= thr && C[s] > thr) {
                    sel_sh = s;
                    tie_sh = is_tie(prev, C[s], Z, u24) ? 1 : 0;
                }
            }
            __syncthreads();
            const int ss = sel_sh;
            n_tie += tie_sh;
            if (a.choices && tid == 0) a.choices[(rep * a.T + t) * N + r] = ss;
            if (ss != r) {
                // ---- accepted swap: energy, rank-1 update of H, column exchange ----
                ++n_acc;
                E += dE[ss];
                const int fb = p[ss];
                for (int i = tid; i < N; i += nt) {
                    uvec[i] = D[(int64_t)i * N + ss] - D[(int64_t)i * N + r];
                    const int c = p[i];
                    vvec[i] = F[(int64_t)fa * N + c] - F[(int64_t)fb * N + c];
                }
                __syncthreads();
                for (int64_t e = tid; e < (int64_t)N * N; e += nt) {
                    const int i = (int)(e / N), k = (int)(e % N);
                    H[e] += (HT)((int64_t)uvec[i] * vvec[k]);
                }
                __syncthreads();
                for (int i = tid; i < N; i += nt) {
                    const HT x = H[(int64_t)i * N + r];
                    H[(int64_t)i * N + r] = H[(int64_t)i * N + ss];
                    H[(int64_t)i * N + ss] = x;
                }
                if (tid == 0) {
                    p[r] = fb;
                    p[ss] = fa;
                }
                __syncthreads();
                if (E < E_best) {
                    E_best = E;
                    for (int s = tid; s < N; s += nt) a.perm_best[rep * N + s] = p[s];
                }
            }
            __syncthreads();
        }
        if (a.E_trace && tid == 0) a.E_trace[rep * a.T + t] = E;
    }
    for (int s = tid; s < N; s += nt) a.perm[rep * N + s] = p[s];
    if (tid == 0) {
        a.E[rep] = E;
        a.E_best[rep] = E_best;
        a.counters[rep * 3 + 0] = (int64_t)N * a.T;
        a.counters[rep * 3 + 1] = n_acc;
        a.counters[rep * 3 + 2] = n_tie;
    }
}

}  // namespace

hipError_t launch_sweep_plain(hipStream_t s, const SweepArgs &a, bool h64) {
    const int threads = a.N <= 64 ? 64 : a.N <= 128 ? 128 : kBlock;
    if (h64)
        sweep_plain_kernel<int64_t><<<a.R, threads, 0, s>>>(a);
    else
        sweep_plain_kernel<int32_t><<<a.R, threads, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace pdit
