// beta_select.hip -- beta-range selection (Results, "Implementation";
// Methods, "CPU-PIM Algorithm"): short trials at fixed beta on a grid, with
// no exchanges, averaged over their ending energies, then the range rule.
//
// The trials themselves run on the sweep kernels (replica k of grid point g
// is row g R + k of one batch, at beta grid[g] through its slot); this file
// holds their set-up, the per-grid-point sums and the rule:
//   with Smax, Smin the largest and smallest sums of ending energies, the
//   low end is the first grid point whose sum has come down from Smax by at
//   least 40% of Smax - Smin (5 S <= 3 Smax + 2 Smin, exact in integers);
//   the high end is two grid points past the first that holds Smin (at
//   most the last); the ladder is geometric between them, computed in
//   double and rounded to float, both ends exactly the grid values.
#include "pdit_internal.h"

namespace pdit {
namespace {

// trial_perm[g R + k] = perm[k]; slot[g R + k] = g
__global__ void trial_setup_kernel(int N, int R, int G, const int32_t *__restrict__ perm,
                                   int32_t *__restrict__ trial_perm, int32_t *__restrict__ slot) {
    const int64_t total = (int64_t)G * R * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / N;
        trial_perm[e] = perm[(row % R) * N + e % N];
        if (e % N == 0) slot[row] = (int32_t)(row / R);
    }
}

// One block per grid point: exact int64 sum of its R ending energies.
__global__ void __launch_bounds__(256)
group_sum_kernel(int R, const int64_t *__restrict__ E, int64_t *__restrict__ E_sum) {
    __shared__ int64_t part[256];
    const int g = blockIdx.x;
    int64_t acc = 0;
    for (int k = threadIdx.x; k < R; k += 256) acc += E[(int64_t)g * R + k];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) E_sum[g] = part[0];
}

// One thread: the rule on G sums (|sum| < 2^59, checked by the caller).
__global__ void beta_rule_kernel(int G, const int64_t *__restrict__ E_sum,
                                 const float *__restrict__ grid, int L, float *__restrict__ ladder,
                                 int32_t *__restrict__ range) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t smax = E_sum[0], smin = E_sum[0];
    int gmin = 0;
    for (int g = 1; g < G; ++g) {
        const int64_t v = E_sum[g];
        if (v > smax) smax = v;
        if (v < smin) {
            smin = v;
            gmin = g;
        }
    }
    const int64_t level = 3 * smax + 2 * smin;
    int lo = 0;
    while (lo < G - 1 && 5 * E_sum[lo] > level) ++lo;  // E_sum[gmin] meets the level
    const int hi = gmin + 2 < G ? gmin + 2 : G - 1;
    range[0] = lo;
    range[1] = hi;
    const double b0 = grid[lo], b1 = grid[hi];
    const double lr = log(b1 / b0);
    for (int i = 1; i + 1 < L; ++i) ladder[i] = (float)(b0 * exp(lr * (double)i / (double)(L - 1)));
    ladder[0] = grid[lo];
    ladder[L - 1] = grid[hi];
}

}  // namespace

hipError_t launch_trial_setup(hipStream_t s, int N, int R, int G, const int32_t *perm,
                              int32_t *trial_perm, int32_t *slot) {
    const int64_t total = (int64_t)G * R * N;
    const int64_t blocks = (total + 255) / 256;
    trial_setup_kernel<<<(int)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(N, R, G, perm,
                                                                            trial_perm, slot);
    return hipGetLastError();
}

hipError_t launch_group_sums(hipStream_t s, int R, int G, const int64_t *E, int64_t *E_sum) {
    group_sum_kernel<<<G, 256, 0, s>>>(R, E, E_sum);
    return hipGetLastError();
}

hipError_t launch_beta_rule(hipStream_t s, int G, const int64_t *E_sum, const float *grid, int L,
                            float *ladder, int32_t *range) {
    if (G < 1 || L < 2) return hipErrorInvalidValue;
    beta_rule_kernel<<<1, 64, 0, s>>>(G, E_sum, grid, L, ladder, range);
    return hipGetLastError();
}

}  // namespace pdit
