// Persistent batched forward kernel (see qbx_batched.hip).
#include "qbx_batched.h"

namespace qbx {

template <int MODE>
__global__ __launch_bounds__(256) void k_forward_batched(
    const BatchItemDev* __restrict__ items, const int* __restrict__ order,
    const long long* __restrict__ pre, int n, long long n_tasks, int* __restrict__ counter,
    const double4* __restrict__ geo, const double2* __restrict__ densw,
    const CenterRec* __restrict__ ctr, const double* __restrict__ jtab, double* __restrict__ out,
    double2* __restrict__ tape) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= n_tasks) break;
    const int slot = find_slot(pre, n, t);
    const BatchItemDev& B = items[order[slot]];
    const int ci = (int)(t - pre[slot]);
    const int key = __builtin_amdgcn_readfirstlane(B.d.kind * 32 + B.d.p);
    switch (key) {
#define QBX_FWD_CASE(K, PP)                                                                   \
  case K * 32 + PP:                                                                           \
    forward_task<MODE, PP, K>(B, ci, lane, geo, densw, ctr, jtab, out, tape);                 \
    break;
      QBX_BATCH_CASES(QBX_FWD_CASE, 1)
      QBX_BATCH_CASES(QBX_FWD_CASE, 2)
      QBX_BATCH_CASES(QBX_FWD_CASE, 3)
#undef QBX_FWD_CASE
      default:
        break;
    }
  }
}

hipError_t launch_forward_batched_0(dim3 grid, const BatchItemDev* items, const int* order,
                                       const long long* pre, int n, long long n_tasks,
                                       int* counter, const double4* geo, const double2* densw,
                                       const CenterRec* ctr, const double* jtab, double* out,
                                       double2* tape, hipStream_t s) {
  hipLaunchKernelGGL((k_forward_batched<0>), grid, dim3(256), 0, s, items, order, pre, n,
                     n_tasks, counter, geo, densw, ctr, jtab, out, tape);
  return hipGetLastError();
}

}  // namespace qbx
