// pt_common.h -- parallel tempering: the exchange pass shared by the
// stand-alone exchange kernel and the fused table kernel, and the arguments
// of the fused kernel (Results, "Implementation"; Methods, "CPU-PIM
// Algorithm").
//
// A set holds L replicas (consecutive rows of the batch) on an ascending
// ladder of inverse temperatures, rung 0 the hottest.  After each period of
// sweeps the rungs are visited from the lowest beta up: when the replica on
// rung i+1 has an energy greater than or equal to the one on rung i, the two
// configurations change rungs, so a low-energy configuration can climb the
// whole ladder in one pass.  If the top rung has not changed hands for
// `timeout` passes it trades with the bottom rung.  Replicas keep their
// states and random streams; only the rung assignment moves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdit {

constexpr int kPtMaxL = 64;  // rungs per set

// One exchange pass over a set, by one thread.  E[k]: energy of member k;
// who[i]: member on rung i (a permutation of 0..L-1, kept one); since:
// passes since the top rung last changed hands.
__device__ __forceinline__ void pt_pass(int L, const int64_t *E, int32_t *who, int32_t &since,
                                        int32_t timeout) {
    bool top = false;
    for (int i = 0; i + 1 < L; ++i) {
        const int32_t lo = who[i], hi = who[i + 1];
        if (E[hi] >= E[lo]) {
            who[i] = hi;
            who[i + 1] = lo;
            top = top || i + 2 == L;
        }
    }
    if (top) {
        since = 0;
    } else if (timeout > 0 && ++since >= timeout) {
        const int32_t w = who[L - 1];
        who[L - 1] = who[0];
        who[0] = w;
        since = 0;
    }
}

// Fused parallel tempering (table kernel): every period of every set in one
// launch whose workgroups are all resident at once.  After each period every
// member publishes a word holding the period number and its energy, and
// waits until it has read that period's word from every member of its set;
// all members then run the same pass on the same energies, so all hold the
// same rung assignment.
constexpr int kPtEBits = 36;                                  // energy field of a word
constexpr uint64_t kPtEMask = (uint64_t(1) << kPtEBits) - 1;
constexpr uint64_t kPtTagMask = (uint64_t(1) << (64 - kPtEBits)) - 1;

struct PtFusedArgs {
    int L;
    const float *ladder;     // [L] beta of each rung, ascending
    int32_t *slot;           // [R] in/out: rung of each replica
    int32_t *since_top;      // [R / L] in/out
    int64_t n_periods;
    int64_t period_sweeps;
    int32_t timeout;
    uint64_t *Epub;          // [2][R] published words (by period parity), zero at launch
    int32_t *err;            // set to 1 when a wait exceeds its bound, zero at launch
    int64_t R;               // replicas of the run (stride of Epub)
    uint64_t min_wait;       // least bound on one wait, in wall-clock ticks
};

}  // namespace pdit
