// Shared pieces of the batched kernels (qbx_batched*.hip): the per-contour
// descriptor, the task lookup and the per-task bodies of the persistent kernels.
#pragma once

#include "qbx_pair.h"
#include "qbx_panel.h"

namespace qbx {

struct BatchItemDev {
  Dims d;
  long long node_off;    // doubles into nodes (and grad_nodes)
  long long din_off;     // doubles into density (and grad_density)
  long long out_off;     // doubles into out (and cotangent)
  long long src_off;     // sources into geo / wgt, sources * 8 into sg
  long long densw_off;   // double2 into the weighted source densities
  long long ctr_off;     // centers into ctr, centers * 8 into cg
  long long jtab_off;    // doubles into jtab
  long long tape_off;    // double2 into tape
  long long G_off;       // double2 into G
  long long spart_off;   // double2 into the source-pass sums
  long long panel_off;   // first panel of this contour in the batch
  long long cpart_off;   // doubles into the fused adjoint's center-side partial sums
};

__device__ __forceinline__ int find_slot(const long long* __restrict__ pre, int n, long long t) {
  int lo = 0, hi = n;   // pre[lo] <= t < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Arguments of one persistent launch: the contours of one (kind, p) class in
// decreasing cost order (order[0..n)), the prefix sums of their task counts
// (pre[0..n]) and the class's task counter.
struct BatchTasks {
  const BatchItemDev* items;
  const int* order;
  const long long* pre;
  int n;
  long long n_tasks;
  int* counter;
};

// ---------------------------------------------------------------------------
// persistent forward: MODE 0 writes out, MODE 1 writes out and the tape
// ---------------------------------------------------------------------------
template <int MODE, int P, int KIND>
__device__ __forceinline__ void forward_task(const BatchItemDev& B, int ci, int lane,
                                             const double4* __restrict__ geo,
                                             const double2* __restrict__ densw,
                                             const CenterRec* __restrict__ ctr,
                                             const double* __restrict__ jtab,
                                             double* __restrict__ out, double2* __restrict__ tape) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const Dims& d = B.d;
  const int si = ci / d.T, t = ci - si * d.T;
  double* o = out ? out + B.out_off : nullptr;
  if (MODE == 0) {
    Cplx S, Dd;
    forward_center<P, KIND>(geo + B.src_off, densw + B.densw_off, d.N, ctr + B.ctr_off + ci,
                            jtab + B.jtab_off + (size_t)ci * d.NJ, d.k, 0, d.chunks, lane, S, Dd);
    if (lane == 0) {
      int kk = 0;
      if (kS) {
        const size_t q = ((size_t)si * NK + kk++) * d.T + t;
        o[2 * q] = -0.25 * S.i;
        o[2 * q + 1] = 0.25 * S.r;
      }
      if (kD) {
        const size_t q = ((size_t)si * NK + kk) * d.T + t;
        o[2 * q] = -0.25 * d.k * Dd.i;
        o[2 * q + 1] = 0.25 * d.k * Dd.r;
      }
    }
  } else {
    Cplx A[2][5];
    tape_center<P, KIND>(geo + B.src_off, densw + B.densw_off, d.N, ctr + B.ctr_off + ci,
                         jtab + B.jtab_off + (size_t)ci * d.NJ, d.NJ, d.k, 0, d.chunks, lane, A);
    if (lane == 0) {
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const size_t q = ((size_t)si * NK + kk) * d.T + t;
        if (out) {
          o[2 * q] = -0.25 * A[kk][0].i;
          o[2 * q + 1] = 0.25 * A[kk][0].r;
        }
        double2* tp = tape + B.tape_off + ((size_t)ci * NK + kk) * 4;
#pragma unroll
        for (int b = 0; b < 4; ++b) tp[b] = make_double2(A[kk][b + 1].r, A[kk][b + 1].i);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// persistent adjoint source pass: one task = 64 sources of one contour against
// one split of its centers; tasks are split-major, so neighbouring wavefronts
// read the same centers
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void adjoint_task(const BatchItemDev& B, int task, int lane,
                                             const double4* __restrict__ geo,
                                             const double2* __restrict__ densw,
                                             const CenterRec* __restrict__ ctr,
                                             const double* __restrict__ jtab,
                                             const double2* __restrict__ G,
                                             double2* __restrict__ spart) {
  constexpr int NA = src_slots(KIND);
  constexpr int NK = KIND == 3 ? 2 : 1;
  const Dims& d = B.d;
  const int sp = task / d.chunks;
  const int j = (task - sp * d.chunks) * kWave + lane;
  if (j >= d.N) return;
  const int c0 = sp * d.centers_per_split;
  const int c1 = min(c0 + d.centers_per_split, d.Mc);
  double2 q[2];
  q[0] = densw[B.densw_off + j];
  q[1] = densw[B.densw_off + (size_t)(NK - 1) * d.N + j];
  Cplx A[NA];
  adjoint_source<P, KIND>(geo[B.src_off + j], q, ctr + B.ctr_off, jtab + B.jtab_off, d.NJ,
                          G + B.G_off, d.Mc, c0, c1, d.k, A);
  double2* out = spart + B.spart_off + (size_t)sp * NA * d.N;
#pragma unroll
  for (int b = 0; b < NA; ++b) out[(size_t)b * d.N + j] = make_double2(A[b].r, A[b].i);
}

// launchers of the persistent kernels of one (kind, p) class (one translation
// unit each); `grid_scale` multiplies the resident-block count of the kernel.
hipError_t launch_forward_batched(int mode, int kind, int p, const BatchTasks& t,
                                  const double4* geo, const double2* densw, const CenterRec* ctr,
                                  const double* jtab, double* out, double2* tape, double grid_scale,
                                  hipStream_t s);
hipError_t launch_adjoint_batched(int kind, int p, const BatchTasks& t, const double4* geo,
                                  const double2* densw, const CenterRec* ctr, const double* jtab,
                                  const double2* G, double2* spart, double grid_scale,
                                  hipStream_t s);
// fused adjoint (no tape): persistent workgroups over (contour, center block,
// source block) tiles of one (kind, p) class
hipError_t launch_adjoint_fused_batched(int kind, int p, const BatchTasks& t, const double4* geo,
                                        const double2* densw, const CenterRec* ctr,
                                        const double* jtab, const double2* G, double2* spart,
                                        double* cpart, double grid_scale, hipStream_t s);

// number of workgroups of `block` threads of `kernel` resident on the whole
// device (the per-CU figure is cached by the caller in *per_cu), times
// grid_scale, and at most what `n_tasks` wavefront tasks need
template <typename K>
inline unsigned persistent_grid(K kernel, int* per_cu, int block, long long n_tasks,
                                double grid_scale) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  if (*per_cu < 1) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kernel, block, 0) != hipSuccess || v < 1)
      v = 1;
    *per_cu = v;
  }
  double g = (double)cus * *per_cu * (grid_scale > 0.0 ? grid_scale : 1.0);
  const long long need = (n_tasks * kWave + block - 1) / block;
  if (g > (double)need) g = (double)need;
  return g < 1.0 ? 1u : (unsigned)g;
}

}  // namespace qbx
