// Geometry kernels of libqbx: quadrature/interpolation tables, the oversampled
// source grid, expansion centers with their Bessel J tables, and checks.
//
//  * Section 4.1: a panel is the degree-15 polynomial through its 16 nodes at
//    the Gauss-Legendre abscissae of the panel parameter tau in [-1, 1].
//  * Section 3.4.2: the density is interpolated from the 16 nodes (target
//    grid) to the q_s = 16*oversample point Gauss-Legendre rule of the same
//    panel (source grid); source weights w = omega |dX/dtau|, outward normal
//    n = (y', -x') / |X'| for a counter-clockwise curve (Section 3.2).
//  * Section 3.3 step 4(a): c = x + s r h_m n with h_m the panel length,
//    radius R = r h_m, and theta = arg(x - c) = arg(-s n).
#include "qbx_internal.h"
#include "qbx_panel.h"
#include "qbx_special.h"

namespace qbx {

// ---------------------------------------------------------------------------
// tables: GL rules (16 and q_s points), Lagrange value / derivative maps from
// the 16 nodes to the q_s source nodes, and the 16x16 differentiation matrix.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tables(int qs, double* __restrict__ tab) {
  const TableLayout L = table_layout(qs);
  __shared__ double t16[kQ], w16[kQ], tq[128], wq[128], bw[kQ];
  const int t = threadIdx.x;
  if (t < kQ) gauss_legendre_node(kQ, t, &t16[t], &w16[t]);
  if (t < qs) gauss_legendre_node(qs, t, &tq[t], &wq[t]);
  __syncthreads();
  if (t < kQ) {  // barycentric weights 1 / prod_{c != a} (tau_a - tau_c)
    double prod = 1.0;
    for (int c = 0; c < kQ; ++c)
      if (c != t) prod *= (t16[t] - t16[c]);
    bw[t] = 1.0 / prod;
  }
  __syncthreads();
  if (t < kQ) {
    tab[L.tau16 + t] = t16[t];
    tab[L.w16 + t] = w16[t];
  }
  if (t < qs) {
    tab[L.taus + t] = tq[t];
    tab[L.ws + t] = wq[t];
  }
  for (int e = t; e < qs * kQ; e += blockDim.x) {
    const int b = e / kQ, a = e % kQ;
    const double tau = tq[b];
    double val = 1.0;
    for (int c = 0; c < kQ; ++c)
      if (c != a) val *= (tau - t16[c]);
    double der = 0.0;  // d/dtau of prod_{c != a}(tau - tau_c): drop one factor at a time
    for (int e2 = 0; e2 < kQ; ++e2) {
      if (e2 == a) continue;
      double pr = 1.0;
      for (int c = 0; c < kQ; ++c)
        if (c != a && c != e2) pr *= (tau - t16[c]);
      der += pr;
    }
    tab[L.V + e] = bw[a] * val;
    tab[L.Vd + e] = bw[a] * der;
  }
  for (int e = t; e < kQ * kQ; e += blockDim.x) {
    const int b = e / kQ, a = e % kQ;  // row: node b, column: basis a
    double v;
    if (a != b) {
      v = (bw[a] / bw[b]) / (t16[b] - t16[a]);
    } else {
      v = 0.0;
      for (int c = 0; c < kQ; ++c)
        if (c != b) v += 1.0 / (t16[b] - t16[c]);
    }
    tab[L.Dn + e] = v;
  }
}

hipError_t launch_tables(const Dims& d, double* tables, hipStream_t s) {
  hipLaunchKernelGGL(k_tables, dim3(1), dim3(256), 0, s, d.qs, tables);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_order_weighted(int Mc, int NJ, double* __restrict__ jtab) {
  const int nj = NJ / 2;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Mc * nj) return;
  const size_t ci = e / nj;
  const int l = (int)(e - ci * nj);
  jtab[(size_t)Mc * NJ + e] = (double)l * jtab[ci * NJ + l];
}

hipError_t launch_order_weighted(const Dims& d, double* jtab, hipStream_t s) {
  const size_t n = (size_t)d.Mc * (d.NJ / 2);
  hipLaunchKernelGGL(k_order_weighted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d.Mc,
                     d.NJ, jtab);
  return hipGetLastError();
}

__global__ __launch_bounds__(128) void k_upsample(Dims d, const double* __restrict__ nodes,
                                                  const double* __restrict__ density,
                                                  const double* __restrict__ tab,
                                                  double4* __restrict__ geo,
                                                  double2* __restrict__ dens,
                                                  double* __restrict__ wgt,
                                                  double* __restrict__ hpan,
                                                  CenterRec* __restrict__ ctr,
                                                  double* __restrict__ jtab) {
  upsample_panel(d, blockIdx.x, nodes, density, tab, geo, dens, wgt, hpan, ctr, jtab);
}

hipError_t launch_upsample(const Dims& d, const double* nodes, const double* density,
                           const double* tables, double4* geo, double2* dens, double* wgt,
                           double* h, CenterRec* ctr, double* jtab, hipStream_t s) {
  hipLaunchKernelGGL(k_upsample, dim3(d.P), dim3(128), 0, s, d, nodes, density, tables, geo, dens,
                     wgt, h, ctr, jtab);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// checks: signed area and Graf's condition |x'-c| >= R for every pair.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_check_ratio(int N, int Mc, const double4* __restrict__ geo,
                                                     const CenterRec* __restrict__ ctr,
                                                     double* __restrict__ ratio) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ci = blockIdx.x * 4 + wave;
  if (ci >= Mc) return;
  const double cx = ctr[ci].cx, cy = ctr[ci].cy, R = ctr[ci].R;
  double m2 = 1e300;
  for (int j = lane; j < N; j += kWave) {
    const double4 g = geo[j];
    const double vx = g.x - cx, vy = g.y - cy;
    m2 = fmin(m2, vx * vx + vy * vy);
  }
  for (int off = 32; off > 0; off >>= 1) m2 = fmin(m2, __shfl_xor(m2, off));
  if (lane == 0) ratio[ci] = sqrt(m2) / R;
}

__global__ __launch_bounds__(256) void k_check_reduce(int N, int Mc, const double4* __restrict__ geo,
                                                      const double* __restrict__ wgt,
                                                      const double* __restrict__ ratio,
                                                      double* __restrict__ out) {
  __shared__ double ra[256], rm[256];
  const int t = threadIdx.x;
  double area = 0.0, mn = 1e300;
  for (int j = t; j < N; j += 256) {
    const double4 g = geo[j];
    area += 0.5 * wgt[j] * (g.x * g.z + g.y * g.w);
  }
  for (int i = t; i < Mc; i += 256) mn = fmin(mn, ratio[i]);
  ra[t] = area;
  rm[t] = mn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      ra[t] += ra[t + off];
      rm[t] = fmin(rm[t], rm[t + off]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = ra[0];
    out[1] = rm[0];
  }
}

hipError_t launch_check(const Dims& d, const double4* geo, const double* wgt, const CenterRec* ctr,
                        double* scratch, hipStream_t s) {
  // per-center ratios go after the two result slots
  double* ratio = scratch + 16;
  hipLaunchKernelGGL(k_check_ratio, dim3((d.Mc + 3) / 4), dim3(256), 0, s, d.N, d.Mc, geo, ctr,
                     ratio);
  hipLaunchKernelGGL(k_check_reduce, dim3(1), dim3(256), 0, s, d.N, d.Mc, geo, wgt, ratio, scratch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// debug hooks for the special functions
// ---------------------------------------------------------------------------
__global__ void k_debug_hankel01(const double* __restrict__ z, int n, double* __restrict__ h0,
                                 double* __restrict__ h1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const H01 h = hankel01(z[i], 1.0 / z[i], g_seed_table);
  h0[2 * i] = h.h0r;
  h0[2 * i + 1] = h.h0i;
  h1[2 * i] = h.h1r;
  h1[2 * i + 1] = h.h1i;
}

__global__ void k_debug_besselj(const double* __restrict__ x, int n, int L, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bessel_j_miller(x[i], L, out + (size_t)i * (L + 1));
}

hipError_t launch_debug_hankel01(const double* z, int n, double* h0, double* h1, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_debug_hankel01, dim3((n + 255) / 256), dim3(256), 0, s, z, n, h0, h1);
  return hipGetLastError();
}

hipError_t launch_debug_besselj(const double* x, int n, int L, double* out, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_debug_besselj, dim3((n + 255) / 256), dim3(256), 0, s, x, n, L, out);
  return hipGetLastError();
}

}  // namespace qbx
