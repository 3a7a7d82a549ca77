// Persistent batched adjoint source pass, one kernel per (kind, p) class (see
// qbx_batched.hip).
#include "qbx_batched.h"

namespace qbx {

template <int P, int KIND>
__global__ __launch_bounds__(256) void k_adjoint_batched(BatchTasks t,
                                                         const double4* __restrict__ geo,
                                                         const double2* __restrict__ densw,
                                                         const CenterRec* __restrict__ ctr,
                                                         const double* __restrict__ jtab,
                                                         const double2* __restrict__ G,
                                                         double2* __restrict__ spart) {
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
    adjoint_task<P, KIND>(B, (int)(task - t.pre[slot]), lane, geo, densw, ctr, jtab, G, spart);
  }
}

template <int P>
static hipError_t launch_p(int kind, const BatchTasks& t, const double4* geo,
                           const double2* densw, const CenterRec* ctr, const double* jtab,
                           const double2* G, double2* spart, double grid_scale, hipStream_t s) {
  static int per_cu[4] = {0, 0, 0, 0};
#define QBX_LAUNCH(KD)                                                                        \
  {                                                                                           \
    const unsigned g = persistent_grid(k_adjoint_batched<P, KD>, &per_cu[KD], 256, t.n_tasks, \
                                       grid_scale);                                           \
    hipLaunchKernelGGL((k_adjoint_batched<P, KD>), dim3(g), dim3(256), 0, s, t, geo, densw,   \
                       ctr, jtab, G, spart);                                                  \
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

hipError_t launch_adjoint_batched(int kind, int p, const BatchTasks& t, const double4* geo,
                                  const double2* densw, const CenterRec* ctr, const double* jtab,
                                  const double2* G, double2* spart, double grid_scale,
                                  hipStream_t s) {
  QBX_P_SWITCH(p, launch_p, kind, t, geo, densw, ctr, jtab, G, spart, grid_scale, s)
}

}  // namespace qbx
