// Persistent batched forward kernels, one kernel per (kind, p) class (see
// qbx_batched.hip).  This file is compiled twice, with QBX_FWD_MODE 0 (values
// only) and 1 (values and the tape), so that the two sets of 3 x 25 template
// instances build in parallel.
#include "qbx_batched.h"

#ifndef QBX_FWD_MODE
#error "compile with -DQBX_FWD_MODE=0 (values) or -DQBX_FWD_MODE=1 (values and the tape)"
#endif
#define QBX_CAT2(a, b) a##b
#define QBX_CAT(a, b) QBX_CAT2(a, b)
#define QBX_FWD_KERNEL QBX_CAT(k_forward_batched_, QBX_FWD_MODE)
#define QBX_FWD_LAUNCH QBX_CAT(launch_forward_batched_, QBX_FWD_MODE)

namespace qbx {

template <int P, int KIND>
__global__ __launch_bounds__(256) void QBX_FWD_KERNEL(BatchTasks t,
                                                      const double4* __restrict__ geo,
                                                      const double2* __restrict__ densw,
                                                      const CenterRec* __restrict__ ctr,
                                                      const double* __restrict__ jtab,
                                                      double* __restrict__ out,
                                                      double2* __restrict__ tape) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    // every lane takes part in the atomic (lane 0 adds 1, the others 0): a
    // divergent `if (lane == 0)` here could be merged by the compiler with the
    // lane-0 stores that end the previous task, letting the other lanes reach
    // the shuffle below without lane 0
    int task = atomicAdd(t.counter, lane == 0 ? 1 : 0);
    task = __builtin_amdgcn_readfirstlane(__shfl(task, 0));
    if (task >= t.n_tasks) break;   // every wave leaves once the counter passes the end
    const int slot = find_slot(t.pre, t.n, task);
    const BatchItemDev& B = t.items[t.order[slot]];
    forward_task<QBX_FWD_MODE, P, KIND>(B, (int)(task - t.pre[slot]), lane, geo, densw, ctr,
                                        jtab, out, tape);
  }
}

template <int P>
static hipError_t launch_p(int kind, const BatchTasks& t, const double4* geo,
                           const double2* densw, const CenterRec* ctr, const double* jtab,
                           double* out, double2* tape, double grid_scale, hipStream_t s) {
  static int per_cu[4] = {0, 0, 0, 0};
#define QBX_LAUNCH(KD)                                                                        \
  {                                                                                           \
    const unsigned g = persistent_grid(QBX_FWD_KERNEL<P, KD>, &per_cu[KD], 256, t.n_tasks,     \
                                       grid_scale);                                           \
    hipLaunchKernelGGL((QBX_FWD_KERNEL<P, KD>), dim3(g), dim3(256), 0, s, t, geo, densw, ctr,  \
                       jtab, out, tape);                                                      \
  }
  if (kind == 1)
    QBX_LAUNCH(1)
  else if (kind == 2)
    QBX_LAUNCH(2)
  else
    QBX_LAUNCH(3)
#undef QBX_LAUNCH
  return hipGetLastError();
}

hipError_t QBX_FWD_LAUNCH(int kind, int p, const BatchTasks& t, const double4* geo,
                          const double2* densw, const CenterRec* ctr, const double* jtab,
                          double* out, double2* tape, double grid_scale, hipStream_t s) {
  QBX_P_SWITCH(p, launch_p, kind, t, geo, densw, ctr, jtab, out, tape, grid_scale, s)
}

}  // namespace qbx
