// Forward pair kernels of libqbx: the hot loop of QBX.
//
// For center c_i with target x_i (theta_i = arg(x_i - c_i), R_i = |x_i - c_i|)
// and source x'_j (rho = |x'_j - c_i|, theta' = arg(x'_j - c_i)), the
// expansion of Section 2 (eq. graf-coefficient) evaluated at the target
// (Section 3.3 step 4(c)) is, summed over -p..p and paired l <-> -l with
// H_{-l} = (-1)^l H_l, J_{-l} = (-1)^l J_l,
//
//   K_S = H_0 J_0 + 2 sum_{l=1}^{p} H_l(k rho) J_l(k R) cos(l Delta),
//   Delta = theta_i - theta',
//
// and u_S(x_i) = (i/4) sum_j w_j sigma_j K_S.  The double layer
// (eq. graf-coefficient-dlp) uses d/dn' f_l = (k/2)(conj(nu) f_{l-1} - nu f_{l+1})
// with nu = n'_x + i n'_y; regrouped the same way,
//
//   K_D = k [ H_0 J_1 cos(psi) + sum_{m=1}^{p-1} H_m J_{m+1} cos(m Delta + psi)
//                              - sum_{m=1}^{p+1} H_m J_{m-1} cos(m Delta - psi) ],
//   psi = theta_i - arg(nu).
//
// The storage-free variant of the paper's algorithm (each source adds its
// contribution to u directly; the coefficients need not be stored) is what
// the loop computes: one complex accumulator per kind and lane.  H_l comes from
// the upward recurrence H_{l+1} = (2l/z) H_l - H_{l-1} from the seeds H_0, H_1;
// cos(l Delta +- psi) from the Chebyshev recurrence c_{l+1} = 2 cos(Delta) c_l - c_{l-1};
// J_l(k R_i) is a per-center table (Miller's recurrence), read as wave-uniform
// scalars.
//
// Mapping: one wavefront per (center, source split); lanes stride over the
// split's sources in chunks of 64 (coalesced double4 loads); a butterfly
// reduction over the 64 lanes at the end; partial sums per split are added
// in a fixed order by k_finalize (deterministic).
#include "qbx_internal.h"
#include "qbx_special.h"

namespace qbx {

template <int P, int KIND>
__device__ __forceinline__ void pair_kernel(double z, double iz, double cd, double sd, double cps,
                                            double sps, const double* __restrict__ J,
                                            const double* __restrict__ cf, double& s_r,
                                            double& s_i, double& d_r, double& d_i) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int LMAX = kD ? P + 1 : P;
  const H01 h = hankel01(z, iz, cf);
  double hm_r = h.h0r, hm_i = h.h0i;  // H_{l-1}
  double hc_r = h.h1r, hc_i = h.h1i;  // H_l
  const double tz = 2.0 * iz;
  double tl = tz;                     // 2l/z
  const double two_cd = 2.0 * cd;
  // l = 0 terms
  double a0r = 0.0, a0i = 0.0, sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
  if (kS) {
    a0r = J[0] * hm_r;
    a0i = J[0] * hm_i;
  }
  if (kD) {
    const double f = J[1] * cps;
    dr = f * hm_r;
    di = f * hm_i;
  }
  double c_m = 1.0, c_c = cd;                            // cos((l-1)D), cos(lD)
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);       // cos((l-1)D + psi), cos(lD + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);        // cos((l-1)D - psi), cos(lD - psi)
#pragma unroll
  for (int l = 1; l <= LMAX; ++l) {
    if (kS && l <= P) {
      const double f = J[l] * c_c;
      sr = fma(f, hc_r, sr);
      si = fma(f, hc_i, si);
    }
    if (kD) {
      double f = -J[l - 1] * b_c;
      if (l <= P - 1) f = fma(J[l + 1], a_c, f);
      dr = fma(f, hc_r, dr);
      di = fma(f, hc_i, di);
    }
    if (l < LMAX) {
      const double hn_r = fma(tl, hc_r, -hm_r);
      const double hn_i = fma(tl, hc_i, -hm_i);
      hm_r = hc_r;
      hm_i = hc_i;
      hc_r = hn_r;
      hc_i = hn_i;
      tl += tz;
      if (kS) {
        const double cn = fma(two_cd, c_c, -c_m);
        c_m = c_c;
        c_c = cn;
      }
      if (kD) {
        const double an = fma(two_cd, a_c, -a_m);
        a_m = a_c;
        a_c = an;
        const double bn = fma(two_cd, b_c, -b_m);
        b_m = b_c;
        b_c = bn;
      }
    }
  }
  s_r = fma(2.0, sr, a0r);
  s_i = fma(2.0, si, a0i);
  d_r = dr;
  d_i = di;
}

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
  const double cx = ctr[ci].cx, cy = ctr[ci].cy, ct = ctr[ci].ct, st = ctr[ci].st;
  const double inv_k = 1.0 / k;
  const double* Jtab = jtab + (size_t)ci * NJ;
  double accS_r = 0.0, accS_i = 0.0, accD_r = 0.0, accD_i = 0.0;
  const int c0 = sp * chunks_per_split;
  const int c1 = min(c0 + chunks_per_split, chunks);
  for (int c = c0; c < c1; ++c) {
    const int j = c * kWave + lane;
    if (j < N) {
      // uniform tables re-read (scalar cache) every iteration, see opaque_zero()
      const int z0 = opaque_zero();
      const double* __restrict__ J = Jtab + z0;
      const double* __restrict__ cf = g_seed_table + z0;
      const double4 g = geo[j];
      const double vx = g.x - cx, vy = g.y - cy;
      const double rho = sqrt(fma(vx, vx, vy * vy));
      const double ir = 1.0 / rho;
      const double cd = (ct * vx + st * vy) * ir;   // cos(theta_i - theta')
      const double sd = (st * vx - ct * vy) * ir;   // sin(theta_i - theta')
      double cps = 0.0, sps = 0.0;
      if (kD) {
        cps = ct * g.z + st * g.w;                   // cos(theta_i - arg nu)
        sps = st * g.z - ct * g.w;                   // sin(theta_i - arg nu)
      }
      double s_r, s_i, d_r, d_i;
      pair_kernel<P, KIND>(k * rho, ir * inv_k, cd, sd, cps, sps, J, cf, s_r, s_i, d_r, d_i);
      if (kS) {
        const double2 w = dens[j];
        accS_r = fma(w.x, s_r, fma(-w.y, s_i, accS_r));
        accS_i = fma(w.x, s_i, fma(w.y, s_r, accS_i));
      }
      if (kD) {
        const double2 w = dens[(kS ? (size_t)N : 0) + j];
        accD_r = fma(w.x, d_r, fma(-w.y, d_i, accD_r));
        accD_i = fma(w.x, d_i, fma(w.y, d_r, accD_i));
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    if (kS) {
      accS_r += __shfl_xor(accS_r, off);
      accS_i += __shfl_xor(accS_i, off);
    }
    if (kD) {
      accD_r += __shfl_xor(accD_r, off);
      accD_i += __shfl_xor(accD_i, off);
    }
  }
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

hipError_t launch_finalize(const Dims& d, const double2* partial, double* out, hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk,
                     d.n_split, partial, out);
  return hipGetLastError();
}

}  // namespace qbx
