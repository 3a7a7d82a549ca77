// Stored local expansions (Section 5: one local expansion serving several nearby
// targets).  The coefficients a_l, l = -p..p, of every center (Section 2, eq.
// graf-coefficient; Section 3.2, eq. graf-coefficient-dlp) are formed once and
// kept; any target inside a center's disk is then evaluated from them by Section
// 3.3 step 4(c), with its own distance and angle from the center.
//
//  * k_coef<M>: lanes are 64 centers, the sources of a source split are
//    wave-uniform (scalar loads).  Per pair, with v = x' - c, rho = |v| and
//    E = e^{-i arg v}, the source factors f_m = H_m(k rho) E^m and
//    f_{-m} = (-1)^m H_m(k rho) conj(E)^m, |m| <= M, are added with a complex
//    weight q_j into 2M + 1 complex sums per lane, all in registers (one
//    template instance per M).  One launch per weight.
//  * The single layer takes q = w sigma and M = p.  The double layer uses the
//    ladder d/dn' f_l = (k/2)(conj(nu) f_{l-1} - nu f_{l+1}), nu = n_x + i n_y:
//    two launches with q = w mu conj(nu) and q = w mu nu at M = p + 1 give sums
//    alpha_m, beta_m, and a^D_l = (k/2)(alpha_{l-1} - beta_{l+1}) (k_coef_finalize).
//  * k_evaluate_expansions: one thread per target,
//    u = (i/4) sum_l a_l J_l(k|x - c|) e^{i l arg(x - c)} with J_l by Miller's
//    recurrence (J_{-l} = (-1)^l J_l).
//  * k_assign_centers: one wave per target, the nearest center whose disk holds
//    it (ties to the lower index), or -1.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/qbx.h"
#include "qbx_internal.h"
#include "qbx_panel.h"
#include "qbx_special.h"

namespace qbx {

// the D weights w mu conj(nu) and w mu nu per source: qd[0][j], qd[1][j]
__global__ __launch_bounds__(256) void k_dlp_weights(int N, const double4* __restrict__ geo,
                                                     const double2* __restrict__ densD,
                                                     double2* __restrict__ qd) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double4 g = geo[j];
  const double2 w = densD[j];
  // (w_r + i w_i)(n_x -+ i n_y)
  qd[j] = make_double2(fma(w.x, g.z, w.y * g.w), fma(w.y, g.z, -w.x * g.w));
  qd[(size_t)N + j] = make_double2(fma(w.x, g.z, -w.y * g.w), fma(w.y, g.z, w.x * g.w));
}

// partial[sp][m + M][ci]: sum over the sources of split sp of q_j f_m(x'_j - c_ci)
template <int M>
__global__ __launch_bounds__(256) void k_coef(const double4* __restrict__ geo,
                                              const double2* __restrict__ q, int N,
                                              const CenterRec* __restrict__ ctr, int Mc,
                                              int n_cb, int n_sp, int src_per_split, double k,
                                              double2* __restrict__ partial) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int sp = gw / n_cb;
  const int cb = gw - sp * n_cb;
  const int ci = cb * kWave + lane;
  if (sp >= n_sp) return;   // past the last split (whole waves); an empty split writes zeros
  const int j0 = sp * src_per_split;
  const int j1 = min(N, j0 + src_per_split);
  const bool valid = ci < Mc;
  const CenterRec c = ctr[valid ? ci : Mc - 1];
  const double inv_k = 1.0 / k;
  double ar[2 * M + 1], ai[2 * M + 1];
#pragma unroll
  for (int m = 0; m <= 2 * M; ++m) ar[m] = ai[m] = 0.0;
  for (int j = j0; j < j1; ++j) {
    const int z0 = opaque_zero();
    const double* __restrict__ cf = g_seed_table + z0;
    const double4 g = geo[j];
    const double2 w = q[j];
    const double vx = g.x - c.cx, vy = g.y - c.cy;
    const double rho2 = fma(vx, vx, vy * vy);
    const double ir = rsqrt_refined(rho2);
    const double z = k * (rho2 * ir), iz = ir * inv_k;
    const H01 h = hankel01(z, iz, cf);
    const double e1r = vx * ir, e1i = -vy * ir;   // E = e^{-i theta'}
    // m = 0
    ar[M] = fma(w.x, h.h0r, fma(-w.y, h.h0i, ar[M]));
    ai[M] = fma(w.x, h.h0i, fma(w.y, h.h0r, ai[M]));
    double hpr = h.h0r, hpi = h.h0i, hr = h.h1r, hi = h.h1i;   // H_{m-1}, H_m
    double er = e1r, ei = e1i;                                 // E^m
#pragma unroll
    for (int m = 1; m <= M; ++m) {
      // f = H_m E^m, g = H_m conj(E)^m from the four shared products
      const double rr = hr * er, ii = hi * ei, ri = hr * ei, ir2 = hi * er;
      const double fr = rr - ii, fi = ri + ir2;
      const double gr = rr + ii, gi = ir2 - ri;
      ar[M + m] = fma(w.x, fr, fma(-w.y, fi, ar[M + m]));
      ai[M + m] = fma(w.x, fi, fma(w.y, fr, ai[M + m]));
      // f_{-m} = (-1)^m H_m conj(E)^m
      const double s = (m & 1) ? -1.0 : 1.0;
      ar[M - m] = fma(s * w.x, gr, fma(-s * w.y, gi, ar[M - m]));
      ai[M - m] = fma(s * w.x, gi, fma(s * w.y, gr, ai[M - m]));
      if (m < M) {
        // H_{m+1} = (2m/z) H_m - H_{m-1};  E^{m+1} = E^m E
        const double t = 2.0 * m * iz;
        const double nr = fma(t, hr, -hpr), ni = fma(t, hi, -hpi);
        hpr = hr;
        hpi = hi;
        hr = nr;
        hi = ni;
        const double tr = fma(er, e1r, -ei * e1i);
        ei = fma(er, e1i, ei * e1r);
        er = tr;
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int m = 0; m <= 2 * M; ++m)
      partial[((size_t)sp * (2 * M + 1) + m) * Mc + ci] = make_double2(ar[m], ai[m]);
  }
}

// coef[kk][ci][l + p] from the split sums: S straight (a_l), D by the ladder
// (k/2)(alpha_{l-1} - beta_{l+1}); pS: [n_sp][2p+1][Mc], pa, pb: [n_sp][2p+3][Mc]
__global__ __launch_bounds__(256) void k_coef_finalize(int Mc, int p, int kind, int n_sp,
                                                       double k,
                                                       const double2* __restrict__ pS,
                                                       const double2* __restrict__ pa,
                                                       const double2* __restrict__ pb,
                                                       double* __restrict__ coef) {
  const int L = 2 * p + 1;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nk = kind == 3 ? 2 : 1;
  if (e >= (long long)nk * Mc * L) return;
  const int kk = (int)(e / ((long long)Mc * L));
  const int rem = (int)(e - (long long)kk * Mc * L);
  const int ci = rem / L, li = rem - ci * L;   // li = l + p
  const bool isD = (kind == 2) || (kind == 3 && kk == 1);
  double r = 0.0, im = 0.0;
  if (!isD) {
    for (int sp = 0; sp < n_sp; ++sp) {
      const double2 v = pS[((size_t)sp * L + li) * Mc + ci];
      r += v.x;
      im += v.y;
    }
  } else {
    const int LD = L + 2;   // orders -(p+1)..(p+1)
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    for (int sp = 0; sp < n_sp; ++sp) {
      // alpha_{l-1} at index (l - 1) + (p + 1) = li; beta_{l+1} at li + 2
      const double2 a = pa[((size_t)sp * LD + li) * Mc + ci];
      const double2 b = pb[((size_t)sp * LD + li + 2) * Mc + ci];
      ar += a.x;
      ai += a.y;
      br += b.x;
      bi += b.y;
    }
    r = 0.5 * k * (ar - br);
    im = 0.5 * k * (ai - bi);
  }
  const size_t o = ((size_t)kk * Mc + ci) * L + li;
  coef[2 * o] = r;
  coef[2 * o + 1] = im;
}

// ctr_xy [Mc][2], ctr_r [Mc] from the center records (either may be NULL)
__global__ __launch_bounds__(256) void k_center_out(int Mc, const CenterRec* __restrict__ ctr,
                                                    double* __restrict__ xy,
                                                    double* __restrict__ rad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mc) return;
  const CenterRec c = ctr[i];
  if (xy) {
    xy[2 * (size_t)i] = c.cx;
    xy[2 * (size_t)i + 1] = c.cy;
  }
  if (rad) rad[i] = c.R;
}

// out[kk][t] = (i/4) sum_{l=-p..p} a_l J_l(k R) e^{i l theta}, R e^{i theta} = x_t - c;
// a center index outside [0, Mc) gives NaN
__global__ __launch_bounds__(256) void k_evaluate_expansions(
    int Mc, const double* __restrict__ ctr_xy, const double2* __restrict__ coef, double k,
    int p, int nk, int n_t, const double* __restrict__ tgt, const int32_t* __restrict__ idx,
    double2* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  const int ci = idx[t];
  if (ci < 0 || ci >= Mc) {
    for (int kk = 0; kk < nk; ++kk) out[(size_t)kk * n_t + t] = make_double2(NAN, NAN);
    return;
  }
  const int L = 2 * p + 1;
  const double dx = tgt[2 * (size_t)t] - ctr_xy[2 * (size_t)ci];
  const double dy = tgt[2 * (size_t)t + 1] - ctr_xy[2 * (size_t)ci + 1];
  const double R = sqrt(dx * dx + dy * dy);
  const double c1 = R > 0.0 ? dx / R : 1.0, s1 = R > 0.0 ? dy / R : 0.0;
  double J[kPMax + 1];
  bessel_j_miller(k * R, p, J);
  for (int kk = 0; kk < nk; ++kk) {
    const double2* a = coef + ((size_t)kk * Mc + ci) * L;
    const double2 a0 = a[p];
    double ur = a0.x * J[0], ui = a0.y * J[0];
    double er = 1.0, ei = 0.0;   // e^{i l theta}
    for (int l = 1; l <= p; ++l) {
      const double tr = er * c1 - ei * s1;
      ei = er * s1 + ei * c1;
      er = tr;
      const double2 ap = a[p + l], am = a[p - l];
      const double jl = J[l], jm = (l & 1) ? -J[l] : J[l];   // J_{-l} = (-1)^l J_l
      // a_l J_l e^{il theta} + a_{-l} J_{-l} e^{-il theta}
      ur += jl * (ap.x * er - ap.y * ei) + jm * (am.x * er + am.y * ei);
      ui += jl * (ap.x * ei + ap.y * er) + jm * (am.y * er - am.x * ei);
    }
    out[(size_t)kk * n_t + t] = make_double2(-0.25 * ui, 0.25 * ur);   // (i/4) u
  }
}

// the nearest center with |x_t - c| <= slack R_c, ties to the lower index; -1 if none.
// Every product and sum is rounded on its own (no contraction), so any IEEE double
// evaluation of the same formula takes the same decisions.
__global__ __launch_bounds__(256) void k_assign_centers(int Mc, const double* __restrict__ ctr_xy,
                                                        const double* __restrict__ ctr_r,
                                                        double slack, int n_t,
                                                        const double* __restrict__ tgt,
                                                        int32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + wave;
  if (t >= n_t) return;
  const double tx = tgt[2 * (size_t)t], ty = tgt[2 * (size_t)t + 1];
  double best = INFINITY;
  int bi = -1;
  for (int i = lane; i < Mc; i += kWave) {
    const double dx = tx - ctr_xy[2 * (size_t)i], dy = ty - ctr_xy[2 * (size_t)i + 1];
    const double d2 = dx * dx + dy * dy;
    const double rr = slack * ctr_r[i];
    if (d2 <= rr * rr && d2 < best) {   // lanes visit their centers in increasing order
      best = d2;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ob < best || (ob == best && oi >= 0 && (bi < 0 || oi < bi))) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) idx[t] = bi;
}

namespace {

template <int M>
hipError_t launch_coef_m(const double4* geo, const double2* q, int N, const CenterRec* ctr,
                         int Mc, int n_cb, int n_sp, int src_per_split, double k,
                         double2* partial, hipStream_t s) {
  const long waves = (long)n_cb * n_sp;
  hipLaunchKernelGGL((k_coef<M>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, geo, q, N,
                     ctr, Mc, n_cb, n_sp, src_per_split, k, partial);
  return hipGetLastError();
}

hipError_t launch_coef(int M, const double4* geo, const double2* q, int N, const CenterRec* ctr,
                       int Mc, int n_cb, int n_sp, int src_per_split, double k,
                       double2* partial, hipStream_t s) {
  switch (M) {
#define QBX_CASE(MM) \
  case MM:           \
    return launch_coef_m<MM>(geo, q, N, ctr, Mc, n_cb, n_sp, src_per_split, k, partial, s);
    QBX_CASE(0) QBX_CASE(1) QBX_CASE(2) QBX_CASE(3) QBX_CASE(4) QBX_CASE(5) QBX_CASE(6)
    QBX_CASE(7) QBX_CASE(8) QBX_CASE(9) QBX_CASE(10) QBX_CASE(11) QBX_CASE(12) QBX_CASE(13)
    QBX_CASE(14) QBX_CASE(15) QBX_CASE(16) QBX_CASE(17) QBX_CASE(18) QBX_CASE(19) QBX_CASE(20)
    QBX_CASE(21) QBX_CASE(22) QBX_CASE(23) QBX_CASE(24) QBX_CASE(25)
#undef QBX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// source splits of the coefficient pass: enough waves (64 centers each) to fill
// the device about four times, at most 8 splits (the split sums take
// n_sp x (2M + 1) x Mc x 16 bytes per weight)
int coef_splits(const Dims& d) {
  const int n_cb = (d.Mc + kWave - 1) / kWave;
  int n_sp = (4096 + n_cb - 1) / n_cb;
  if (n_sp > 8) n_sp = 8;
  const int chunks = (d.N + kWave - 1) / kWave;
  if (n_sp > chunks) n_sp = chunks;
  return n_sp < 1 ? 1 : n_sp;
}

struct ExpLayout {
  Layout base;          // tables .. partial of make_forward_layout (partial unused)
  size_t qd, pS, pa, pb, total;
};

ExpLayout make_expansion_layout(const Dims& d) {
  ExpLayout E;
  E.base = make_forward_layout(d);
  size_t o = E.base.total;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t n_sp = (size_t)coef_splits(d);
  const bool hasS = d.kind & 1, hasD = d.kind & 2;
  E.qd = take(hasD ? sizeof(double2) * 2 * (size_t)d.N : 0);
  E.pS = take(hasS ? sizeof(double2) * n_sp * (2 * d.p + 1) * d.Mc : 0);
  E.pa = take(hasD ? sizeof(double2) * n_sp * (2 * d.p + 3) * d.Mc : 0);
  E.pb = take(hasD ? sizeof(double2) * n_sp * (2 * d.p + 3) * d.Mc : 0);
  E.total = o;
  return E;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

}  // namespace
}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_expansion_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                     int kind) {
  Dims d;
  if (!make_dims(n_panels, q, p, oversample, side, kind, 1.0, 0.5, &d)) return 0;
  return make_expansion_layout(d).total;
}

int qbx_expansion_coefficients(const qbx_geometry* g, const double* density, double k, int p,
                               double r, int oversample, int side, int kind, double* coef,
                               double* ctr_xy, double* ctr_r, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!coef) return fail(QBX_EINVAL, "coef is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const ExpLayout E = make_expansion_layout(d);
  if (ws_bytes < E.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, E.total);
  const Layout& L = E.base;
  hipError_t e = launch_tables(d, at<double>(ws, L.tables), stream);
  if (e != hipSuccess) return device_fail(e, "tables kernel");
  e = launch_upsample(d, g->nodes, density, at<double>(ws, L.tables), at<double4>(ws, L.geo),
                      at<double2>(ws, L.dens), at<double>(ws, L.wgt), at<double>(ws, L.h),
                      at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab), stream);
  if (e != hipSuccess) return device_fail(e, "upsample kernel");
  const int n_cb = (d.Mc + kWave - 1) / kWave;
  const int n_sp = coef_splits(d);
  const int per = (d.N + n_sp - 1) / n_sp;
  const double4* geo = at<double4>(ws, L.geo);
  const CenterRec* ctr = at<CenterRec>(ws, L.ctr);
  const double2* dens = at<double2>(ws, L.dens);
  if (d.kind & 1) {
    e = launch_coef(d.p, geo, dens, d.N, ctr, d.Mc, n_cb, n_sp, per, d.k, at<double2>(ws, E.pS),
                    stream);
    if (e != hipSuccess) return device_fail(e, "coefficient kernel (S)");
  }
  if (d.kind & 2) {
    const double2* densD = dens + ((d.kind & 1) ? (size_t)d.N : 0);
    double2* qd = at<double2>(ws, E.qd);
    hipLaunchKernelGGL(k_dlp_weights, dim3((d.N + 255) / 256), dim3(256), 0, stream, d.N, geo,
                       densD, qd);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = launch_coef(d.p + 1, geo, qd, d.N, ctr, d.Mc, n_cb, n_sp, per, d.k,
                      at<double2>(ws, E.pa), stream);
    if (e == hipSuccess)
      e = launch_coef(d.p + 1, geo, qd + d.N, d.N, ctr, d.Mc, n_cb, n_sp, per, d.k,
                      at<double2>(ws, E.pb), stream);
    if (e != hipSuccess) return device_fail(e, "coefficient kernels (D)");
  }
  const long long n = (long long)d.nk * d.Mc * (2 * d.p + 1);
  hipLaunchKernelGGL(k_coef_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     d.Mc, d.p, d.kind, n_sp, d.k, at<double2>(ws, E.pS), at<double2>(ws, E.pa),
                     at<double2>(ws, E.pb), coef);
  if (ctr_xy || ctr_r)
    hipLaunchKernelGGL(k_center_out, dim3((d.Mc + 255) / 256), dim3(256), 0, stream, d.Mc, ctr,
                       ctr_xy, ctr_r);
  e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "coefficient finalize kernels");
}

int qbx_evaluate_expansions(int n_ctr, const double* ctr_xy, const double* coef, double k,
                            int p, int kind, int n_targets, const double* target_xy,
                            const int32_t* center_index, double* out, hipStream_t stream) {
  if (n_ctr < 1 || n_targets < 0) return fail(QBX_EINVAL, "n_ctr = %d, n_targets = %d", n_ctr,
                                                n_targets);
  if (p < 0 || p > kPMax) return fail(QBX_EINVAL, "order p = %d outside [0, %d]", p, kPMax);
  if (!(k > 0.0) || !std::isfinite(k)) return fail(QBX_EINVAL, "wavenumber k = %g must be > 0", k);
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D))
    return fail(QBX_EINVAL, "kind = %d is not 1 (S), 2 (D) or 3 (S|D)", kind);
  if (n_targets == 0) return QBX_OK;
  if (!ctr_xy || !coef || !target_xy || !center_index || !out)
    return fail(QBX_EINVAL, "NULL array argument");
  const int nk = kind == 3 ? 2 : 1;
  hipLaunchKernelGGL(k_evaluate_expansions, dim3((n_targets + 255) / 256), dim3(256), 0, stream,
                     n_ctr, ctr_xy, reinterpret_cast<const double2*>(coef), k, p, nk, n_targets,
                     target_xy, center_index, reinterpret_cast<double2*>(out));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "expansion evaluation kernel");
}

int qbx_assign_centers(int n_ctr, const double* ctr_xy, const double* ctr_r, int n_targets,
                       const double* target_xy, double slack, int32_t* center_index,
                       hipStream_t stream) {
  if (n_ctr < 1 || n_targets < 0) return fail(QBX_EINVAL, "n_ctr = %d, n_targets = %d", n_ctr,
                                                n_targets);
  if (!(slack > 0.0) || !std::isfinite(slack))
    return fail(QBX_EINVAL, "slack = %g must be > 0", slack);
  if (n_targets == 0) return QBX_OK;
  if (!ctr_xy || !ctr_r || !target_xy || !center_index)
    return fail(QBX_EINVAL, "NULL array argument");
  hipLaunchKernelGGL(k_assign_centers, dim3((unsigned)(((long)n_targets + 3) / 4)), dim3(256), 0,
                     stream, n_ctr, ctr_xy, ctr_r, slack, n_targets, target_xy, center_index);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "center assignment kernel");
}

}  // extern "C"
