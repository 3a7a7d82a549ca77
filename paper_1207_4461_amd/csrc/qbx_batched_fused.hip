// Persistent batched fused adjoint, one kernel per (kind, p) class (see
// qbx_batched.hip): workgroups take (contour, center block, source block) tiles
// from the class's counter and run the fused tile body of the per-contour
// kernel (fused_tile in qbx_pair.h).
#include "qbx_batched.h"

namespace qbx {

template <int P, int KIND>
__global__ __launch_bounds__(256) void k_adjoint_fused_batched(BatchTasks t,
                                                               const double4* __restrict__ geo,
                                                               const double2* __restrict__ densw,
                                                               const CenterRec* __restrict__ ctr,
                                                               const double* __restrict__ jtab,
                                                               const double2* __restrict__ G,
                                                               double2* __restrict__ spart,
                                                               double* __restrict__ cpart) {
  constexpr int NA = src_slots(KIND);
  __shared__ double acc[4 * fused_centers(KIND) * 4];
  __shared__ long long s_task;
  for (;;) {
    // one task per workgroup: thread 0 takes it, the barrier hands it to all
    if (threadIdx.x == 0) s_task = atomicAdd(t.counter, 1);
    __syncthreads();
    const long long task = s_task;
    __syncthreads();   // every thread has read s_task before the next fetch
    if (task >= t.n_tasks) break;   // the same value in every thread: the whole group leaves
    const int slot = find_slot(t.pre, t.n, task);
    const BatchItemDev& B = t.items[t.order[slot]];
    const Dims& d = B.d;
    const int local = (int)(task - t.pre[slot]);
    const int cb = local / d.n_sb;
    const int sb = local - cb * d.n_sb;
    const int i0 = cb * d.fused_cblock;
    const int ch0 = sb * d.chunks_per_sb;
    fused_tile<P, KIND>(geo + B.src_off, densw + B.densw_off, d.N, ctr + B.ctr_off,
                        jtab + B.jtab_off, d.NJ, G + B.G_off, d.Mc, i0,
                        min(d.fused_cblock, d.Mc - i0), ch0, min(ch0 + d.chunks_per_sb, d.chunks),
                        d.k, spart + B.spart_off + (size_t)cb * NA * d.N,
                        cpart + B.cpart_off + (size_t)sb * d.Mc * 4, acc);
  }
}

template <int P>
static hipError_t launch_p(int kind, const BatchTasks& t, const double4* geo,
                           const double2* densw, const CenterRec* ctr, const double* jtab,
                           const double2* G, double2* spart, double* cpart, double grid_scale,
                           hipStream_t s) {
  static int per_cu[4] = {0, 0, 0, 0};
  // persistent_grid counts wavefront tasks: a tile task occupies four waves
#define QBX_LAUNCH(KD)                                                                        \
  {                                                                                           \
    const unsigned g = persistent_grid(k_adjoint_fused_batched<P, KD>, &per_cu[KD], 256,       \
                                       t.n_tasks * 4, grid_scale);                            \
    hipLaunchKernelGGL((k_adjoint_fused_batched<P, KD>), dim3(g), dim3(256), 0, s, t, geo,     \
                       densw, ctr, jtab, G, spart, cpart);                                    \
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

hipError_t launch_adjoint_fused_batched(int kind, int p, const BatchTasks& t, const double4* geo,
                                        const double2* densw, const CenterRec* ctr,
                                        const double* jtab, const double2* G, double2* spart,
                                        double* cpart, double grid_scale, hipStream_t s) {
  QBX_P_SWITCH(p, launch_p, kind, t, geo, densw, ctr, jtab, G, spart, cpart, grid_scale, s)
}

}  // namespace qbx
