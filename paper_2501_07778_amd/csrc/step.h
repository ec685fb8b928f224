// The hot step y = round(A x) as a launch sequence, shared by the eager
// call (qtt_matvec_round, capi.cpp) and its graph form (graph.cpp).
#ifndef QTT_STEP_H
#define QTT_STEP_H

#include "internal.h"

namespace qtt {

// the product train and the rounding workspace, carved from the caller's ws
struct MatvecRoundPlan {
  TTDesc t;
  RoundWs w;
};

// every argument check of qtt_matvec_round except the workspace's size
qtt_status check_matvec_round_args(const qtt_tt *A, const qtt_tt *x, const qtt_tt *y,
                                   qtt_dtype compute, int32_t ell, double eps);

// Carves the step's buffers from ws and enqueues every launch of the step
// on s up to the rounded train in the workspace (device ranks p.t.v.rk,
// norm and squared error in p.w.scal).  The ranks of A and x travel as
// kernel arguments, so the sequence holds no host synchronisation, no
// host-to-device copy and no memset, and can be captured into a graph.
qtt_status enqueue_matvec_round(const qtt_tt *A, const qtt_tt *x, qtt_dtype compute,
                                int32_t ell, uint64_t seed, double eps, int32_t rmax, void *ws,
                                size_t ws_bytes, hipStream_t s, MatvecRoundPlan &p);

// true while qtt_kernel_timing records events (ktimer.cpp)
bool ktimer_active();

}  // namespace qtt

#endif
