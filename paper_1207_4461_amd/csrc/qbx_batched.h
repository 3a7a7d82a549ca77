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

// ---------------------------------------------------------------------------
// persistent forward: MODE 0 writes out, MODE 1 writes out and the tape
// ---------------------------------------------------------------------------
// Not inlined: each (kind, p) body is compiled as its own function (one task is
// a whole center or source chunk, so the call costs nothing measurable).
template <int MODE, int P, int KIND>
__device__ __attribute__((noinline)) void forward_task(const BatchItemDev& B, int ci, int lane,
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
// persistent adjoint source pass: one task = 64 sources of one contour
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __attribute__((noinline)) void adjoint_task(const BatchItemDev& B, int chunk, int lane,
                                             const double4* __restrict__ geo,
                                             const CenterRec* __restrict__ ctr,
                                             const double* __restrict__ jtab,
                                             const double2* __restrict__ G,
                                             double2* __restrict__ spart) {
  constexpr int NA = ((KIND & 1) ? 3 : 0) + ((KIND & 2) ? 4 : 0);
  const Dims& d = B.d;
  const int j = chunk * kWave + lane;
  if (j >= d.N) return;
  Cplx A[NA];
  adjoint_source<P, KIND>(geo[B.src_off + j], ctr + B.ctr_off, jtab + B.jtab_off, d.NJ,
                          G + B.G_off, d.Mc, 0, d.Mc, d.k, A);
  double2* q = spart + B.spart_off;
#pragma unroll
  for (int b = 0; b < NA; ++b) q[(size_t)b * d.N + j] = make_double2(A[b].r, A[b].i);
}

#define QBX_BATCH_CASES(X, K)                                                                \
  X(K, 0) X(K, 1) X(K, 2) X(K, 3) X(K, 4) X(K, 5) X(K, 6) X(K, 7) X(K, 8) X(K, 9) X(K, 10)  \
  X(K, 11) X(K, 12) X(K, 13) X(K, 14) X(K, 15) X(K, 16) X(K, 17) X(K, 18) X(K, 19)           \
  X(K, 20) X(K, 21) X(K, 22) X(K, 23) X(K, 24)


// launchers of the persistent kernels (one translation unit each)
hipError_t launch_forward_batched(int mode, dim3 grid, const BatchItemDev* items, const int* order,
                                  const long long* pre, int n, long long n_tasks, int* counter,
                                  const double4* geo, const double2* densw, const CenterRec* ctr,
                                  const double* jtab, double* out, double2* tape, hipStream_t s);
hipError_t launch_adjoint_batched(dim3 grid, const BatchItemDev* items, const int* order,
                                  const long long* pre, int n, long long n_tasks, int* counter,
                                  const double4* geo, const CenterRec* ctr, const double* jtab,
                                  const double2* G, double2* spart, hipStream_t s);

}  // namespace qbx
