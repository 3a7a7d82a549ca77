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

// On-surface derivatives from one-sided limits (Section 3.2): with both sides the
// average of the two limits; with one side s (+1 exterior, -1 interior) the
// limit minus its jump,
//   grad S = grad S^s + s n sigma / 2,   S' = S'^s + s sigma / 2,
//   grad D = grad D^s - s t dmu/ds / 2,  D' = D'^s,
// with n the target's outward unit normal and t = (-n_y, n_x) the
// counter-clockwise tangent, both from the 16-node derivative X'(tau) as for the
// centers, and dmu/ds = (dmu/dtau) / |X'(tau)|.
__global__ __launch_bounds__(256) void k_gradient_principal_value(
    int T, int nk, int side, int kind, NodeDiff D, const double* __restrict__ nodes,
    const double2* __restrict__ density, const double2* __restrict__ grad,
    const double2* __restrict__ dn, double2* __restrict__ grad_pv, double2* __restrict__ dn_pv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * nk) return;
  const int kk = e / T, t = e - kk * T;
  if (side == 0) {
    const size_t a = (size_t)kk * T + t, b = ((size_t)nk + kk) * T + t;
    if (grad_pv) {
      for (int c = 0; c < 2; ++c) {
        const double2 u = grad[2 * a + c], v = grad[2 * b + c];
        grad_pv[2 * a + c] = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y + v.y));
      }
    }
    if (dn_pv) {
      const double2 u = dn[a], v = dn[b];
      dn_pv[a] = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y + v.y));
    }
    return;
  }
  const double s = side > 0 ? 1.0 : -1.0;
  const bool isD = (kind == 2) || (kind == 3 && kk == 1);
  const int m = t / kQ, row = t - m * kQ;
  const double* X = nodes + (size_t)m * 2 * kQ;
  double dx = 0.0, dy = 0.0;
  for (int a = 0; a < kQ; ++a) {
    dx = fma(D.d[row][a], X[2 * a], dx);
    dy = fma(D.d[row][a], X[2 * a + 1], dy);
  }
  const double inv = 1.0 / sqrt(dx * dx + dy * dy);
  const double tx = dx * inv, ty = dy * inv;   // t = X' / |X'|; n = (t_y, -t_x)
  const size_t o = (size_t)kk * T + t;
  if (!isD) {
    const double2 sig = density[o];
    if (grad_pv) {
      const double nx = ty, ny = -tx;
      const double2 gx = grad[2 * o], gy = grad[2 * o + 1];
      grad_pv[2 * o] = make_double2(fma(0.5 * s * nx, sig.x, gx.x), fma(0.5 * s * nx, sig.y, gx.y));
      grad_pv[2 * o + 1] =
          make_double2(fma(0.5 * s * ny, sig.x, gy.x), fma(0.5 * s * ny, sig.y, gy.y));
    }
    if (dn_pv) {
      const double2 v = dn[o];
      dn_pv[o] = make_double2(fma(0.5 * s, sig.x, v.x), fma(0.5 * s, sig.y, v.y));
    }
    return;
  }
  if (grad_pv) {
    const double2* mu = density + (size_t)kk * T + (size_t)m * kQ;
    double dr = 0.0, di = 0.0;
    for (int a = 0; a < kQ; ++a) {
      dr = fma(D.d[row][a], mu[a].x, dr);
      di = fma(D.d[row][a], mu[a].y, di);
    }
    dr *= inv;
    di *= inv;
    const double2 gx = grad[2 * o], gy = grad[2 * o + 1];
    grad_pv[2 * o] = make_double2(fma(-0.5 * s * tx, dr, gx.x), fma(-0.5 * s * tx, di, gx.y));
    grad_pv[2 * o + 1] = make_double2(fma(-0.5 * s * ty, dr, gy.x), fma(-0.5 * s * ty, di, gy.y));
  }
  if (dn_pv) dn_pv[o] = dn[o];
}

hipError_t launch_gradient_principal_value(int T, int nk, int side, int kind, const NodeDiff& D,
                                           const double* nodes, const double* density,
                                           const double* grad, const double* dn,
                                           double* grad_pv, double* dn_pv, hipStream_t s) {
  const int n = T * nk;
  hipLaunchKernelGGL(k_gradient_principal_value, dim3((n + 255) / 256), dim3(256), 0, s, T, nk,
                     side, kind, D, nodes, reinterpret_cast<const double2*>(density),
                     reinterpret_cast<const double2*>(grad), reinterpret_cast<const double2*>(dn),
                     reinterpret_cast<double2*>(grad_pv), reinterpret_cast<double2*>(dn_pv));
  return hipGetLastError();
}

hipError_t launch_finalize(const Dims& d, const double2* partial, double* out, hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk,
                     d.n_split, partial, out);
  return hipGetLastError();
}

}  // namespace qbx
