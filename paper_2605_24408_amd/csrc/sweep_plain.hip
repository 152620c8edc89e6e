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
#include "sweep_common.h"

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

struct PlainSmem {
    int32_t p[PDIT_NMAX];
    int64_t dE[PDIT_NMAX];
    uint64_t C[PDIT_NMAX];
    uint64_t Ctmp[PDIT_NMAX];
    int32_t uvec[PDIT_NMAX];
    int32_t vvec[PDIT_NMAX];
    int64_t red[kBlock];
    int32_t sel_sh, tie_sh;
};

// Runs one replica's sweeps with the whole workgroup.  H (this replica's
// N x N, int32 or int64) is updated in place in device memory.
template <typename HT>
__device__ void plain_replica(const ReplicaJob &a, PlainSmem &sm) {
    int32_t *p = sm.p;
    int64_t *dE = sm.dE;
    uint64_t *C = sm.C;
    uint64_t *Ctmp = sm.Ctmp;
    const int N = a.N;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int32_t *__restrict__ D = a.D;
    const int32_t *__restrict__ F = a.F;
    HT *__restrict__ H = (HT *)a.H;

    for (int s = tid; s < N; s += nt) p[s] = a.perm[s];
    int64_t E = *a.E;
    int64_t E_best = *a.E_best;
    int64_t n_acc = 0, n_tie = 0;
    __syncthreads();

    for (int64_t t = 0; t < a.T; ++t) {
        const float beta = a.beta[t * a.beta_stride];
        const uint32_t g = (uint32_t)(a.sweep_offset + (uint64_t)t);
        const int64_t dthr = zero_weight_distance64(beta);
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
            const int64_t m = block_min_i64(lmin, sm.red);
            if (tid == 0) {
                sm.sel_sh = r;  // overwritten below: exactly one candidate holds the threshold
                sm.tie_sh = 0;
            }
            // ---- Gibbs weights and their running sum (Eq. 5) ----
            for (int s = tid; s < N; s += nt) {
                const int64_t d = dE[s] - m;
                C[s] = d < dthr ? gibbs_weight(beta, (float)d) : 0u;
            }
            __syncthreads();
            for (int off = 1; off < N; off <<= 1) {
                for (int s = tid; s < N; s += nt) Ctmp[s] = C[s] + (s >= off ? C[s - off] : 0);
                __syncthreads();
                for (int s = tid; s < N; s += nt) C[s] = Ctmp[s];
                __syncthreads();
            }
            const uint64_t Z = C[N - 1];
            const uint32_t u24 = uniform24(a.seed, (uint32_t)r, g, a.rep, a.inst);
            const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
            for (int s = tid; s < N; s += nt) {
                const uint64_t prev = s > 0 ? C[s - 1] : 0;
                if (prev <= thr && C[s] > thr) {
                    sm.sel_sh = s;
                    sm.tie_sh = is_tie(prev, C[s], Z, u24) ? 1 : 0;
                }
            }
            __syncthreads();
            const int ss = sm.sel_sh;
            n_tie += sm.tie_sh;
            if (a.choices && tid == 0) a.choices[t * N + r] = ss;
            if (ss != r) {
                // ---- accepted swap: energy, rank-1 update of H, column exchange ----
                ++n_acc;
                E += dE[ss];
                const int fb = p[ss];
                for (int i = tid; i < N; i += nt) {
                    sm.uvec[i] = D[(int64_t)i * N + ss] - D[(int64_t)i * N + r];
                    const int c = p[i];
                    sm.vvec[i] = F[(int64_t)fa * N + c] - F[(int64_t)fb * N + c];
                }
                __syncthreads();
                // rows by wave, columns by lane (coalesced); four rows are
                // read before any is written back, so that their loads are in
                // flight together
                const int nw = nt >> 6, wv = tid >> 6, ln = tid & 63;
                for (int i0 = 4 * wv; i0 < N; i0 += 4 * nw) {
                    const int nr = min(4, N - i0);
                    HT *row = H + (int64_t)i0 * N;
                    for (int k = ln; k < N; k += 64) {
                        HT x[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (j < nr) x[j] = row[(int64_t)j * N + k];
                        const int64_t vk = sm.vvec[k];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (j < nr) row[(int64_t)j * N + k] = x[j] + (HT)(sm.uvec[i0 + j] * vk);
                    }
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
                    for (int s = tid; s < N; s += nt) a.perm_best[s] = p[s];
                }
            }
            __syncthreads();
        }
        if (a.E_trace && tid == 0) a.E_trace[t] = E;
    }
    for (int s = tid; s < N; s += nt) a.perm[s] = p[s];
    if (tid == 0) {
        *a.E = E;
        *a.E_best = E_best;
        const bool acc = (a.flags & kAccumCounters) != 0;
        a.counters[0] = (acc ? a.counters[0] : 0) + (int64_t)N * a.T;
        a.counters[1] = (acc ? a.counters[1] : 0) + n_acc;
        a.counters[2] = (acc ? a.counters[2] : 0) + n_tie;
    }
}

template <typename HT>
__global__ void __launch_bounds__(kBlock) sweep_plain_kernel(SweepArgs a) {
    __shared__ PlainSmem sm;
    const int64_t rep = blockIdx.x;
    ReplicaJob j;
    j.N = a.N;
    j.D = a.D;
    j.F = a.F;
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
    plain_replica<HT>(j, sm);
}

// Persistent: each workgroup takes (instance, replica) items from a queue
// until it is exhausted (every workgroup reaches the exit: the queue only
// grows).
template <typename HT>
__global__ void __launch_bounds__(kBlock) sweep_plain_persistent(BatchArgs b) {
    __shared__ PlainSmem sm;
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(item_sh);  // wave-uniform
        __syncthreads();
        if (item >= b.n_items) break;
        plain_replica<HT>(batch_job(b, item, sizeof(HT)), sm);
        __syncthreads();
    }
}

// Clears the work queues before a persistent launch (a kernel, not a memset,
// so that the sequence can be captured in a graph).
__global__ void queue_reset_kernel(int *queue, int n) {
    const int i = threadIdx.x;
    if (i < n) queue[i] = 0;
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

namespace pdit {

hipError_t launch_sweep_plain_persistent(hipStream_t s, bool h64, const BatchArgs &b, int grid) {
    if (h64)
        sweep_plain_persistent<int64_t><<<grid, kBlock, 0, s>>>(b);
    else
        sweep_plain_persistent<int32_t><<<grid, kBlock, 0, s>>>(b);
    return hipGetLastError();
}

int plain_blocks_per_cu(bool h64) {
    int n = 0;
    const hipError_t e =
        h64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_plain_persistent<int64_t>, kBlock, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_plain_persistent<int32_t>, kBlock, 0);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_queue_reset(hipStream_t s, int *queue, int n) {
    queue_reset_kernel<<<1, 64, 0, s>>>(queue, n);
    return hipGetLastError();
}

}  // namespace pdit
