// Persistent batched adjoint source pass (see qbx_batched.hip).
#include "qbx_batched.h"

namespace qbx {

__global__ __launch_bounds__(256) void k_adjoint_batched(
    const BatchItemDev* __restrict__ items, const int* __restrict__ order,
    const long long* __restrict__ pre, int n, long long n_tasks, int* __restrict__ counter,
    const double4* __restrict__ geo, const CenterRec* __restrict__ ctr,
    const double* __restrict__ jtab, const double2* __restrict__ G,
    double2* __restrict__ spart) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= n_tasks) break;
    const int slot = find_slot(pre, n, t);
    const BatchItemDev& B = items[order[slot]];
    const int chunk = (int)(t - pre[slot]);
    const int key = __builtin_amdgcn_readfirstlane(B.d.kind * 32 + B.d.p);
    switch (key) {
#define QBX_ADJ_CASE(K, PP)                                                                   \
  case K * 32 + PP:                                                                           \
    adjoint_task<PP, K>(B, chunk, lane, geo, ctr, jtab, G, spart);                            \
    break;
      QBX_BATCH_CASES(QBX_ADJ_CASE, 1)
      QBX_BATCH_CASES(QBX_ADJ_CASE, 2)
      QBX_BATCH_CASES(QBX_ADJ_CASE, 3)
#undef QBX_ADJ_CASE
      default:
        break;
    }
  }
}

hipError_t launch_adjoint_batched(dim3 grid, const BatchItemDev* items, const int* order,
                                  const long long* pre, int n, long long n_tasks, int* counter,
                                  const double4* geo, const CenterRec* ctr, const double* jtab,
                                  const double2* G, double2* spart, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_batched, grid, dim3(256), 0, s, items, order, pre, n, n_tasks,
                     counter, geo, ctr, jtab, G, spart);
  return hipGetLastError();
}

}  // namespace qbx
