// pt.hip -- parallel tempering: the stand-alone exchange pass between sweep
// periods, for the kernels that run one period per launch (the pass itself
// is in pt_common.h).
#include "pdit_internal.h"

namespace pdit {
namespace {

// One wave per set (L <= kPtMaxL; the slots were validated as a permutation
// of 0..L-1 and the pass keeps them one): lanes load the set's slots and
// energies together, lane 0 runs the pass on LDS, lanes write the new slots.
__global__ void __launch_bounds__(64)
pt_exchange_kernel(int n_sets, int L, const int64_t *__restrict__ E, int32_t *__restrict__ slot,
                   int32_t *__restrict__ since_top, int32_t timeout) {
    __shared__ int64_t Es[kPtMaxL];
    __shared__ int32_t who[kPtMaxL];
    const int set = blockIdx.x;
    const int k = threadIdx.x;
    const int64_t base = (int64_t)set * L;
    if (k < L) {
        Es[k] = E[base + k];
        who[slot[base + k]] = k;
    }
    __syncthreads();
    if (k == 0) {
        int32_t c = since_top[set];
        pt_pass(L, Es, who, c, timeout);
        since_top[set] = c;
    }
    __syncthreads();
    if (k < L) slot[base + who[k]] = k;
}

}  // namespace

hipError_t launch_pt_exchange(hipStream_t s, int n_sets, int L, const int64_t *E, int32_t *slot,
                              int32_t *since_top, int32_t timeout) {
    if (L < 1 || L > kPtMaxL) return hipErrorInvalidValue;
    if (n_sets < 1) return hipSuccess;
    pt_exchange_kernel<<<n_sets, 64, 0, s>>>(n_sets, L, E, slot, since_top, timeout);
    return hipGetLastError();
}

}  // namespace pdit
