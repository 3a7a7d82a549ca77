// Forward kernels of libqbx: the per-contour launch of the pair loop
// (forward_center in qbx_pair.h, where the formulas are derived), the split
// reduction, and the principal-value post-step of Section 3.2.
#include "qbx_pair.h"

namespace qbx {

template <int P, int KIND>
__global__ __launch_bounds__(256) void k_forward(const double4* __restrict__ geo,
                                                 const double2* __restrict__ dens, int N,
                                                 const CenterRec* __restrict__ ctr,
                                                 const double* __restrict__ jtab, int NJ, int Mc,
                                                 int n_split, int chunks, int chunks_per_split,
                                                 double k, double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int ci = gw / n_split;
  const int sp = gw - ci * n_split;
  if (ci >= Mc) return;
  const int c0 = sp * chunks_per_split;
  const int c1 = min(c0 + chunks_per_split, chunks);
  Cplx S, Dd;
  forward_center<P, KIND>(geo, dens, N, ctr + ci, jtab + (size_t)ci * NJ, k, c0, c1, lane, S, Dd);
  const double accS_r = S.r, accS_i = S.i, accD_r = Dd.r, accD_i = Dd.i;
  if (lane == 0) {
    int kk = 0;
    if (kS) partial[((size_t)sp * NK + kk++) * Mc + ci] = make_double2(accS_r, accS_i);
    if (kD) partial[((size_t)sp * NK + kk) * Mc + ci] = make_double2(k * accD_r, k * accD_i);
  }
}

template <int P>
static hipError_t launch_forward_p(const Dims& d, const double4* geo, const double2* dens,
                                   const CenterRec* ctr, const double* jtab, double2* partial,
                                   hipStream_t s) {
  const long waves = (long)d.Mc * d.n_split;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
  switch (d.kind) {
    case 1:
      hipLaunchKernelGGL((k_forward<P, 1>), grid, block, 0, s, geo, dens, d.N, ctr, jtab, d.NJ,
                         d.Mc, d.n_split, d.chunks, d.chunks_per_split, d.k, partial);
      break;
    case 2:
      hipLaunchKernelGGL((k_forward<P, 2>), grid, block, 0, s, geo, dens, d.N, ctr, jtab, d.NJ,
                         d.Mc, d.n_split, d.chunks, d.chunks_per_split, d.k, partial);
      break;
    default:
      hipLaunchKernelGGL((k_forward<P, 3>), grid, block, 0, s, geo, dens, d.N, ctr, jtab, d.NJ,
                         d.Mc, d.n_split, d.chunks, d.chunks_per_split, d.k, partial);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const Dims& d, const double4* geo, const double2* dens,
                          const CenterRec* ctr, const double* jtab, double2* partial,
                          hipStream_t s) {
  switch (d.p) {
#define QBX_CASE(PP) \
  case PP:           \
    return launch_forward_p<PP>(d, geo, dens, ctr, jtab, partial, s);
    QBX_CASE(0) QBX_CASE(1) QBX_CASE(2) QBX_CASE(3) QBX_CASE(4) QBX_CASE(5) QBX_CASE(6)
    QBX_CASE(7) QBX_CASE(8) QBX_CASE(9) QBX_CASE(10) QBX_CASE(11) QBX_CASE(12) QBX_CASE(13)
    QBX_CASE(14) QBX_CASE(15) QBX_CASE(16) QBX_CASE(17) QBX_CASE(18) QBX_CASE(19) QBX_CASE(20)
    QBX_CASE(21) QBX_CASE(22) QBX_CASE(23) QBX_CASE(24)
#undef QBX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// out[si][kk][t] = (i/4) * sum over splits (fixed order)
__global__ __launch_bounds__(256) void k_finalize(int Mc, int T, int nk, int n_split,
                                                  const double2* __restrict__ partial,
                                                  double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Mc * nk) return;
  const int kk = e / Mc, ci = e - kk * Mc;
  double r = 0.0, im = 0.0;
  for (int sp = 0; sp < n_split; ++sp) {
    const double2 v = partial[((size_t)sp * nk + kk) * Mc + ci];
    r += v.x;
    im += v.y;
  }
  const int si = ci / T, t = ci - si * T;
  const size_t o = ((size_t)si * nk + kk) * T + t;
  out[2 * o] = -0.25 * im;   // (i/4)(r + i im)
  out[2 * o + 1] = 0.25 * r;
}

// principal value: average of both limits, or one limit minus the D jump
__global__ __launch_bounds__(256) void k_principal_value(int T, int nk, int side, int kind,
                                                         const double2* __restrict__ out,
                                                         const double2* __restrict__ density,
                                                         double2* __restrict__ pv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * nk) return;
  const int kk = e / T, t = e - kk * T;
  const bool isD = (kind == 2) || (kind == 3 && kk == 1);
  double2 v;
  if (side == 0) {
    const double2 a = out[(size_t)kk * T + t], b = out[((size_t)nk + kk) * T + t];
    v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
  } else {
    v = out[(size_t)kk * T + t];
    if (isD) {
      const double2 mu = density[(size_t)kk * T + t];
      const double s = side > 0 ? 0.5 : -0.5;
      v = make_double2(v.x - s * mu.x, v.y - s * mu.y);
    }
  }
  pv[e] = v;
}

hipError_t launch_principal_value(int T, int nk, int side, int kind, const double* out,
                                  const double* density, double* pv, hipStream_t s) {
  const int n = T * nk;
  hipLaunchKernelGGL(k_principal_value, dim3((n + 255) / 256), dim3(256), 0, s, T, nk, side, kind,
                     reinterpret_cast<const double2*>(out),
                     reinterpret_cast<const double2*>(density), reinterpret_cast<double2*>(pv));
  return hipGetLastError();
}

hipError_t launch_finalize(const Dims& d, const double2* partial, double* out, hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk,
                     d.n_split, partial, out);
  return hipGetLastError();
}

}  // namespace qbx
