// prep.hip -- step "instance prep": data summary used to choose exact
// integer widths and the recompute mode, plus validation of the inputs
// (symmetry of D and F, permutation rows, inverse temperatures).
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

__global__ void zero_stats_kernel(InstanceStats *s) {
    if (threadIdx.x == 0) {
        s->max_abs_d = 0;
        s->max_abs_f = 0;
        s->max_rowsum_d = 0;
        s->max_colsum_f = 0;
        s->asym_d = 0;
        s->asym_f = 0;
        s->bad_perm_rows = 0;
        s->bad_beta = 0;
        s->diag_nz_d = 0;
        s->diag_nz_f = 0;
        s->bad_slots = 0;
        s->bad_grid = 0;
        s->clique_bad = 0;
        s->clique_size = 0;
        s->int_min = 0;
        s->neg_d = 0;
        s->neg_f = 0;
    }
}

// One thread per row i (D row sums, D symmetry/max) and per column c (F).
__global__ void matrix_stats_kernel(int N, const int32_t *__restrict__ D,
                                    const int32_t *__restrict__ F, InstanceStats *s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * N) return;
    const bool isD = t < N;
    const int i = isD ? t : t - N;
    const int32_t *M = isD ? D : F;
    int64_t sum = 0;
    int32_t mx = 0, asym = 0, int_min = 0, neg = 0;
    for (int j = 0; j < N; ++j) {
        // row i of D; column i of F (sum over the row index j)
        const int32_t v = isD ? M[(int64_t)i * N + j] : M[(int64_t)j * N + i];
        // |INT32_MIN| does not fit int32: counted (and refused by the host)
        // instead of folded into the maximum
        const int64_t a = v < 0 ? -(int64_t)v : (int64_t)v;
        int_min += v == INT32_MIN;
        neg += v < 0;
        sum += a;
        mx = max(mx, (int32_t)min(a, (int64_t)INT32_MAX));
        if (j > i && M[(int64_t)i * N + j] != M[(int64_t)j * N + i]) ++asym;
    }
    if (int_min) atomicAdd(&s->int_min, int_min);
    if (neg) atomicAdd(isD ? &s->neg_d : &s->neg_f, neg);
    const bool diag_nz = M[(int64_t)i * N + i] != 0;
    if (isD) {
        if (diag_nz) atomicAdd(&s->diag_nz_d, 1);
        atomicMax(&s->max_abs_d, mx);
        atomicMax((unsigned long long *)&s->max_rowsum_d, (unsigned long long)sum);
        if (asym) atomicAdd(&s->asym_d, asym);
    } else {
        if (diag_nz) atomicAdd(&s->diag_nz_f, 1);
        atomicMax(&s->max_abs_f, mx);
        atomicMax((unsigned long long *)&s->max_colsum_f, (unsigned long long)sum);
        if (asym) atomicAdd(&s->asym_f, asym);
    }
}

// One block per permutation row (grid-stride): every value in [0, N) seen once.
__global__ void perm_check_kernel(int N, int R, const int32_t *__restrict__ perm,
                                  int32_t *bad_rows) {
    __shared__ int32_t seen[PDIT_NMAX];
    for (int row = blockIdx.x; row < R; row += gridDim.x) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) seen[i] = 0;
        __syncthreads();
        int bad = 0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const int32_t v = perm[(int64_t)row * N + i];
            if (v < 0 || v >= N)
                bad = 1;
            else
                atomicAdd(&seen[v], 1);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += blockDim.x)
            if (seen[i] != 1) bad = 1;
        bad = __syncthreads_or(bad);
        if (bad && threadIdx.x == 0) atomicAdd(bad_rows, 1);
        __syncthreads();
    }
}

__global__ void beta_check_kernel(int64_t T, const float *__restrict__ beta, InstanceStats *s) {
    int bad = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < T;
         t += (int64_t)gridDim.x * blockDim.x) {
        const float b = beta[t];
        if (!(b >= 0.0f) || !isfinite(b)) ++bad;
    }
    if (bad) atomicAdd(&s->bad_beta, bad);
}

// A beta grid for trials: every value > 0 and above the one before it.
__global__ void grid_check_kernel(int G, const float *__restrict__ grid, InstanceStats *s) {
    int bad = 0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x)
        if (!(grid[g] > 0.0f) || (g > 0 && !(grid[g] > grid[g - 1]))) ++bad;
    if (bad) atomicAdd(&s->bad_grid, bad);
}

// member[a] = 1 when facility a has a nonzero flow to another facility.
__global__ void clique_member_kernel(int N, const int32_t *__restrict__ F,
                                     int32_t *__restrict__ member) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int32_t c = 0;
    for (int b = 0; b < N; ++b)
        if (b != a && F[(int64_t)a * N + b] != 0) c = 1;
    member[a] = c;
}

// Entries that break F[a][b] = member[a] member[b] (a != b), F[a][a] = 0.
__global__ void clique_check_kernel(int N, const int32_t *__restrict__ F,
                                    const int32_t *__restrict__ member, InstanceStats *s) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int bad = 0;
    for (int b = 0; b < N; ++b) {
        const int32_t want = b == a ? 0 : member[a] * member[b];
        bad += F[(int64_t)a * N + b] != want;
    }
    if (bad) atomicAdd(&s->clique_bad, bad);
    if (member[a]) atomicAdd(&s->clique_size, 1);
}

// One thread per parallel-tempering set: its L slots are distinct values in
// [0, L) and its pass counter is not negative.
__global__ void pt_check_kernel(int n_sets, int L, const int32_t *__restrict__ slot,
                                const int32_t *__restrict__ since_top, InstanceStats *s) {
    const int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets) return;
    uint64_t seen = 0;
    bool bad = since_top[set] < 0;
    for (int k = 0; k < L; ++k) {
        const int32_t v = slot[(int64_t)set * L + k];
        if (v < 0 || v >= L || ((seen >> v) & 1))
            bad = true;
        else
            seen |= 1ull << v;
    }
    if (bad) atomicAdd(&s->bad_slots, 1);
}

}  // namespace

hipError_t launch_pt_check(hipStream_t st, int n_sets, int L, const int32_t *slot,
                           const int32_t *since_top, InstanceStats *out) {
    if (L < 1 || L > kPtMaxL) return hipErrorInvalidValue;
    pt_check_kernel<<<(n_sets + 255) / 256, 256, 0, st>>>(n_sets, L, slot, since_top, out);
    return hipGetLastError();
}

hipError_t launch_grid_check(hipStream_t st, int G, const float *grid, InstanceStats *out) {
    grid_check_kernel<<<(G + 255) / 256 < 64 ? (G + 255) / 256 : 64, 256, 0, st>>>(G, grid, out);
    return hipGetLastError();
}

hipError_t launch_clique_check(hipStream_t st, int N, const int32_t *F, int32_t *member,
                               InstanceStats *out) {
    clique_member_kernel<<<(N + 255) / 256, 256, 0, st>>>(N, F, member);
    clique_check_kernel<<<(N + 255) / 256, 256, 0, st>>>(N, F, member, out);
    return hipGetLastError();
}

namespace {
__global__ void zero_i64_kernel(int64_t *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = 0;
}

// entries where a and b (n elements of T) differ, added to *count
template <typename T>
__global__ void count_diff_kernel(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                                  int32_t *count) {
    int diff = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        diff += a[i] != b[i];
    // one atomic per wave
    for (int o = 32; o > 0; o >>= 1) diff += __shfl_xor(diff, o);
    if ((threadIdx.x & 63) == 0 && diff) atomicAdd(count, diff);
}
}  // namespace

hipError_t launch_zero_i64(hipStream_t s, int64_t *out, int64_t n) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    zero_i64_kernel<<<(int)(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(out, n);
    return hipGetLastError();
}

hipError_t launch_perm_rows_check(hipStream_t s, int N, int R, const int32_t *perm, int32_t *bad) {
    if (R <= 0) return hipSuccess;
    perm_check_kernel<<<R < 2048 ? R : 2048, 256, 0, s>>>(N, R, perm, bad);
    return hipGetLastError();
}

hipError_t launch_count_diff(hipStream_t s, int64_t n, int elem_bytes, const void *a,
                             const void *b, int32_t *count) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    const int grid = (int)(blocks < 2048 ? blocks : 2048);
    if (elem_bytes == 8)
        count_diff_kernel<int64_t><<<grid, 256, 0, s>>>(n, (const int64_t *)a, (const int64_t *)b,
                                                        count);
    else
        count_diff_kernel<int32_t><<<grid, 256, 0, s>>>(n, (const int32_t *)a, (const int32_t *)b,
                                                        count);
    return hipGetLastError();
}

hipError_t launch_instance_stats(hipStream_t st, int N, const int32_t *D, const int32_t *F,
                                 int R, const int32_t *perm, const float *beta, int64_t T,
                                 InstanceStats *out) {
    zero_stats_kernel<<<1, 64, 0, st>>>(out);
    matrix_stats_kernel<<<(2 * N + 255) / 256, 256, 0, st>>>(N, D, F, out);
    if (perm && R > 0) {
        const int grid = R < 2048 ? R : 2048;
        perm_check_kernel<<<grid, 256, 0, st>>>(N, R, perm, &out->bad_perm_rows);
    }
    if (beta && T > 0) {
        const int64_t blocks = (T + 255) / 256;
        beta_check_kernel<<<(int)(blocks < 1024 ? blocks : 1024), 256, 0, st>>>(T, beta, out);
    }
    return hipGetLastError();
}

}  // namespace pdit
