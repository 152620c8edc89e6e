// sweep_common.h -- descriptors shared by the sweep kernels and the host
// runtime: one replica's job, and the device-side description of a batched
// run of instances of uneven size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdit {

// Everything one replica's run needs; pointers address this replica's own
// slots.
struct ReplicaJob {
    int N;
    const int32_t *D;        // [N][N]
    const int32_t *F;        // [N][N]
    const void *cD, *cF;     // large kernel: padded copies of D and F (else null)
    int32_t *perm;           // [N] in/out
    const void *H;           // [N][N] initial H (int32, or int64 on the plain kernel)
    int64_t *E;              // in: initial energy, out: final
    int64_t *E_best;         // in/out
    int32_t *perm_best;      // [N] in/out
    int64_t *counters;       // [3] out: updates, accepted, ties
    const float *beta;       // beta of sweep t is beta[t * beta_stride]
    int64_t beta_stride;     // 1: a schedule; 0: one beta for every sweep
    int64_t T;
    uint64_t seed;
    uint64_t sweep_offset;
    uint32_t rep;            // replica index inside its instance (Philox word 2)
    uint32_t inst;           // instance index (Philox word 3)
    int32_t *choices;        // [T][N] or null
    int64_t *E_trace;        // [T] or null
    int seq_threshold;
    bool zero_diag;
    int32_t *tstate;         // table kernel: this replica's saved state, or null
    uint32_t flags;          // kLoadState | kSaveState | kAccumCounters
};

// Beta of the replica's sweeps: beta[slot[rep]] for every sweep when a slot
// array is given, else the schedule.
__device__ __forceinline__ void job_beta(ReplicaJob &j, const float *beta, const int32_t *slot,
                                         int64_t rep) {
    j.beta = slot ? beta + slot[rep] : beta;
    j.beta_stride = slot ? 0 : 1;
}

// One instance of a batched run (device memory).
struct BatchInstance {
    int32_t N;
    int32_t R;
    const int32_t *D;
    const int32_t *F;
    int32_t *perm;           // [R][N]
    const void *cD, *cF;     // large kernel: the instance's padded copies of D and F (else null)
    const float *beta;       // [T]
    int64_t h_off;           // element offset of replica 0's H in the H buffer
    int64_t rep_base;        // index of replica 0 in the per-replica state arrays
    int64_t perm_off;        // offset of replica 0's row in perm_best
    int32_t zero_diag;
    int32_t inst_id;
    int32_t *choices;        // [R][T][N] recorded draws, or null
    int64_t *E_trace;        // [R][T] recorded energies, or null
};

// Values that change from call to call, read by the kernels from device
// memory so that a captured graph can be replayed.
struct BatchParams {
    uint64_t seed;
    uint64_t sweep_offset;
};

struct BatchArgs {
    const BatchInstance *inst;
    const int2 *items;       // (instance, replica) work items, largest N first
    int n_items;
    int *queue;              // next item to hand out
    const BatchParams *params;
    void *H;                 // H buffer (int32 for the fast kernel; plain: per h64)
    int64_t *E;
    int64_t *E_best;
    int32_t *perm_best;
    int64_t *counters;
    int64_t T;
    int seq_threshold;
    int rec;                 // some instance records (selects the recording kernels)
};

__device__ __forceinline__ ReplicaJob batch_job(const BatchArgs &b, int item, size_t hsize) {
    const int2 it = b.items[item];
    const BatchInstance &in = b.inst[it.x];
    const int64_t r = it.y;
    ReplicaJob j;
    j.N = in.N;
    j.D = in.D;
    j.F = in.F;
    j.cD = in.cD;
    j.cF = in.cF;
    j.perm = in.perm + r * in.N;
    j.H = (const char *)b.H + (in.h_off + r * (int64_t)in.N * in.N) * hsize;
    j.E = b.E + in.rep_base + r;
    j.E_best = b.E_best + in.rep_base + r;
    j.perm_best = b.perm_best + in.perm_off + r * in.N;
    j.counters = b.counters + 3 * (in.rep_base + r);
    j.beta = in.beta;
    j.beta_stride = 1;
    j.T = b.T;
    j.seed = b.params->seed;
    j.sweep_offset = b.params->sweep_offset;
    j.rep = (uint32_t)r;
    j.inst = (uint32_t)in.inst_id;
    j.choices = in.choices ? in.choices + r * b.T * in.N : nullptr;
    j.E_trace = in.E_trace ? in.E_trace + r * b.T : nullptr;
    j.seq_threshold = b.seq_threshold;
    j.zero_diag = in.zero_diag != 0;
    j.tstate = nullptr;
    j.flags = 0;
    return j;
}

}  // namespace pdit
