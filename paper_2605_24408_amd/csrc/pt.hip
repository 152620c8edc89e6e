// pt.hip -- parallel tempering: the exchange pass between sweep periods
// (Results, "Implementation"; Methods, "CPU-PIM Algorithm").
//
// A set holds L replicas (rows set*L .. set*L+L-1 of the batch) on an
// ascending ladder of inverse temperatures; slot[k] is the rung replica k
// sits on.  After each period of sweeps the rungs are visited from the
// lowest beta up: when the replica on rung i+1 has an energy greater than or
// equal to the one on rung i, the two configurations change rungs, so a
// low-energy configuration can climb the whole ladder in one pass.  If the
// top rung has not changed hands for `timeout` passes it trades with the
// bottom rung.  Replicas keep their states and random streams; only the
// rung assignment moves.
#include "pdit_internal.h"

namespace pdit {
namespace {

// One thread per set (L <= kPtMaxL; the slots were validated as a
// permutation of 0..L-1 and the kernel keeps them one).
__global__ void pt_exchange_kernel(int n_sets, int L, const int64_t *__restrict__ E,
                                   int32_t *__restrict__ slot, int32_t *__restrict__ since_top,
                                   int32_t timeout) {
    const int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets) return;
    const int64_t base = (int64_t)set * L;
    int32_t who[kPtMaxL];  // replica (within the set) on each rung
    for (int i = 0; i < L; ++i) who[i] = i;
    for (int k = 0; k < L; ++k) {
        const int32_t v = slot[base + k];
        if (v >= 0 && v < L) who[v] = k;
    }
    bool top = false;
    for (int i = 0; i + 1 < L; ++i) {
        const int32_t lo = who[i], hi = who[i + 1];
        if (E[base + hi] >= E[base + lo]) {
            who[i] = hi;
            who[i + 1] = lo;
            if (i + 1 == L - 1) top = true;
        }
    }
    int32_t c = since_top[set];
    if (top) {
        c = 0;
    } else if (timeout > 0 && ++c >= timeout) {
        const int32_t w = who[L - 1];
        who[L - 1] = who[0];
        who[0] = w;
        c = 0;
    }
    since_top[set] = c;
    for (int i = 0; i < L; ++i) slot[base + who[i]] = i;
}

}  // namespace

hipError_t launch_pt_exchange(hipStream_t s, int n_sets, int L, const int64_t *E, int32_t *slot,
                              int32_t *since_top, int32_t timeout) {
    if (L < 1 || L > kPtMaxL) return hipErrorInvalidValue;
    pt_exchange_kernel<<<(n_sets + 63) / 64, 64, 0, s>>>(n_sets, L, E, slot, since_top, timeout);
    return hipGetLastError();
}

}  // namespace pdit
