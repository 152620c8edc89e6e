// beta_select.hip -- beta-range selection (Results, "Implementation";
// Methods, "CPU-PIM Algorithm"): short trials at fixed beta on a grid, with
// no exchanges, averaged over their ending energies, then the range rule.
//
// The trials themselves run on the sweep kernels (replica k of grid point g
// is row g R + k of one batch, at beta grid[g] through its slot); this file
// holds their set-up and the per-grid-point sums.  The range rule and the
// ladder act on G sums and run on the host (api.hip), so that no floating
// point beyond the sampling's single precision runs on the device.
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

}  // namespace pdit
