// debug.hip -- kernels behind the test/debug entry points: the energy-change
// row of one update, the Gibbs choice on its own, and Philox uniforms.
#include "device_common.h"
#include "pdit_internal.h"

namespace pdit {
namespace {

// One block per replica; threads over candidates s.  H is int64 [R][N][N].
__global__ void delta_row_kernel(int N, const int32_t *__restrict__ D,
                                 const int32_t *__restrict__ F, const int32_t *__restrict__ perm,
                                 const int64_t *__restrict__ H, int r, int64_t *__restrict__ out) {
    const int64_t rep = blockIdx.x;
    const int32_t *p = perm + rep * N;
    const int64_t *Hr = H + rep * (int64_t)N * N;
    const int fa = p[r];
    const int64_t hrr = Hr[(int64_t)r * N + r];
    for (int s = threadIdx.x; s < N; s += blockDim.x) {
        const int c = p[s];
        const int64_t h = Hr[(int64_t)r * N + s] + Hr[(int64_t)s * N + r] - hrr - Hr[(int64_t)s * N + s];
        const int64_t dd = (int64_t)D[(int64_t)r * N + r] + D[(int64_t)s * N + s] - 2 * (int64_t)D[(int64_t)r * N + s];
        const int64_t ff = (int64_t)F[(int64_t)fa * N + fa] + F[(int64_t)c * N + c] - 2 * (int64_t)F[(int64_t)fa * N + c];
        out[rep * N + s] = 2 * h + dd * ff;
    }
}

// One wave per row.  Lane l owns the J consecutive candidates [l*J, l*J + J);
// lane partial sums are scanned across the wave, then each lane locates the
// threshold inside its own run.
__global__ void __launch_bounds__(64) choice_kernel(int N, const int64_t *__restrict__ delta,
                                                    const float *__restrict__ beta,
                                                    const uint32_t *__restrict__ u24v,
                                                    int32_t *__restrict__ choice,
                                                    int32_t *__restrict__ tie) {
    const int64_t row = blockIdx.x;
    const int lane = threadIdx.x;
    const int J = (N + kWave - 1) / kWave;
    const int64_t *dr = delta + row * N;
    // row minimum: lane minimum, then a butterfly over the wave
    int64_t lmin = INT64_MAX;
    for (int j = 0; j < J; ++j) {
        const int s = lane * J + j;
        if (s < N) lmin = min(lmin, dr[s]);
    }
    for (int off = 32; off > 0; off >>= 1) lmin = min(lmin, (int64_t)__shfl_xor(lmin, off));
    const int64_t m = lmin;
    const float b = beta[row];
    const int64_t dthr = zero_weight_distance64(b);
    uint64_t part = 0;
    for (int j = 0; j < J; ++j) {
        const int s = lane * J + j;
        if (s < N) {
            const int64_t d = dr[s] - m;
            part += d < dthr ? gibbs_weight(b, (float)d) : 0u;
        }
    }
    const uint64_t incl = wave_scan_u64(part);
    const uint64_t Z = readlane_u64(incl, 63);
    const uint32_t u24 = u24v[row];
    const uint64_t thr = ((uint64_t)u24 * Z) >> 24;
    uint64_t C = incl - part;
    for (int j = 0; j < J; ++j) {
        const int s = lane * J + j;
        if (s < N) {
            const int64_t d = dr[s] - m;
            const uint64_t q = d < dthr ? gibbs_weight(b, (float)d) : 0u;
            const uint64_t prev = C;
            C += q;
            if (prev <= thr && C > thr) {
                choice[row] = s;
                if (tie) tie[row] = is_tie(prev, C, Z, u24) ? 1 : 0;
            }
        }
    }
}

__global__ void uniform24_kernel(int M, const uint32_t *__restrict__ ctr, uint64_t seed,
                                 uint32_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    out[i] = philox_word0(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                          (uint32_t)seed, (uint32_t)(seed >> 32)) >> 8;
}

}  // namespace

hipError_t launch_debug_delta(hipStream_t s, int N, const int32_t *D, const int32_t *F, int R,
                              const int32_t *perm, const int64_t *H, int r, int64_t *out) {
    delta_row_kernel<<<R, 256, 0, s>>>(N, D, F, perm, H, r, out);
    return hipGetLastError();
}

hipError_t launch_debug_choice(hipStream_t s, int N, int M, const int64_t *delta,
                               const float *beta, const uint32_t *u24, int32_t *choice,
                               int32_t *tie) {
    choice_kernel<<<M, 64, 0, s>>>(N, delta, beta, u24, choice, tie);
    return hipGetLastError();
}

hipError_t launch_debug_uniform24(hipStream_t s, int M, const uint32_t *ctr, uint64_t seed,
                                  uint32_t *out) {
    uniform24_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, ctr, seed, out);
    return hipGetLastError();
}

}  // namespace pdit
