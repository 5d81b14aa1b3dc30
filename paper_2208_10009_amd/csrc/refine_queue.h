// refine_queue.h -- the precise algorithm as one persistent launch fed by a
// device work queue of sub-rays (refine.hip); shared with the host
// orchestration (api.hip); not part of the public ABI.
#pragma once
#include "internal.h"

namespace sbr {

// Per-path state between iterations: the current axis, the cone radius of
// the iteration being evaluated (i), the reported error and iteration, the
// flags, and the sub-rays of iteration i still being traced.
struct QState {
    double axis[3];
    double rho, tan;
    int32_t i, iters;
    uint32_t flags;
    int32_t pending;
};
static_assert(sizeof(QState) == 56, "QState layout");

// Result of one traced sub-ray (slot 8 p + s).
struct QSlot {
    double tan, D, Llast;
    int32_t ok, pad;
};
static_assert(sizeof(QSlot) == 32, "QSlot layout");

// Device buffers of a queue refinement over at most U_max paths whose jobs
// run at most max_iters iterations: state [U_max], slots [U_max][8], the
// item array [cap] (0 = not yet pushed; zeroed by the caller with the three
// counters head, tail, done).
struct RefineQueue {
    QState* state;
    QSlot* slot;
    unsigned long long* items;
    int64_t cap;
    uint32_t* ctr;  // [0] items handed out, [1] items pushed, [2] paths done
};

inline int64_t refine_queue_cap(int64_t U_max, int32_t max_iters)
{
    return U_max * 8 * (int64_t)(max_iters > 0 ? max_iters : 1);
}

// The precise algorithm for uniq[0 .. min(U_max, *n_dev)): an init launch
// (start of every path, first iteration's sub-rays pushed) and one
// persistent launch of `blocks` workgroups whose lanes take sub-rays from the
// queue; the lane that finishes an iteration's last sub-ray picks its winner
// and pushes the next iteration's.  Same RefineOut as launch_refine; no path
// geometry is stored (launch_solve with replay traces the final axis).
hipError_t launch_refine_queue(const CallDev& call, const sbr_candidate* uniq, int64_t U_max,
                               const int32_t* n_dev, const RefineQueue& Q, int blocks,
                               RefineOut* out, int32_t* err, hipStream_t s);

}  // namespace sbr
