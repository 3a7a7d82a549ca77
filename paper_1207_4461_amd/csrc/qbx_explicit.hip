// Kernel-level entry points: the QBX pair sums for caller-given sources and
// expansion centers (qbx_apply_explicit / qbx_apply_explicit_adjoint).  No
// panels and no interpolation: the caller supplies the source points, normals
// and weighted densities of the smooth rule, and each center's position,
// radius and target direction (Section 2, eqs. graf-coefficient and
// graf-addition; Section 3.2, eq. graf-coefficient-dlp; Section 3.3 step 4(c)).
// The pair loops, the tape and the source-major adjoint pass are those of the
// per-contour path; only the packing of the inputs and the last per-element
// steps of the gradients differ.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/qbx.h"
#include "qbx_internal.h"
#include "qbx_panel.h"

namespace qbx {

// sources: geo = {x, y, n_x, n_y} (the normal as given; zero for S only),
// dens[kind][j] = q_j
__global__ __launch_bounds__(256) void k_explicit_sources(int N, int nk,
                                                          const double* __restrict__ src_xy,
                                                          const double* __restrict__ src_nu,
                                                          const double* __restrict__ src_q,
                                                          double4* __restrict__ geo,
                                                          double2* __restrict__ dens) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double nx = src_nu ? src_nu[2 * (size_t)j] : 0.0;
  const double ny = src_nu ? src_nu[2 * (size_t)j + 1] : 0.0;
  geo[j] = make_double4(src_xy[2 * (size_t)j], src_xy[2 * (size_t)j + 1], nx, ny);
  for (int kk = 0; kk < nk; ++kk) {
    const size_t o = (size_t)kk * N + j;
    dens[o] = make_double2(src_q[2 * o], src_q[2 * o + 1]);
  }
}

// centers: CenterRec {c, R, e^{i theta}, target x = c + R e^{i theta}} and the
// J_l(kR), J'_l(kR) table
__global__ __launch_bounds__(256) void k_explicit_centers(int Mc, int NJ, double k,
                                                          const double* __restrict__ ctr_xy,
                                                          const double* __restrict__ ctr_r,
                                                          const double* __restrict__ ctr_dir,
                                                          CenterRec* __restrict__ ctr,
                                                          double* __restrict__ jtab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mc) return;
  CenterRec c;
  c.cx = ctr_xy[2 * (size_t)i];
  c.cy = ctr_xy[2 * (size_t)i + 1];
  c.R = ctr_r[i];
  c.ct = ctr_dir[2 * (size_t)i];
  c.st = ctr_dir[2 * (size_t)i + 1];
  c.x = fma(c.R, c.ct, c.cx);
  c.y = fma(c.R, c.st, c.cy);
  c.pad = 0.0;
  ctr[i] = c;
  center_bessel_table(k * c.R, NJ / 2, jtab + (size_t)i * NJ);
}

// per source, from the source-major partial sums (the src_slots layout):
//   grad_q[kind][j]  = sum_i conj(G_i K_ij)                      (complex)
//   grad_src_xy[j]   = sum_i Re G_i q_j grad_v K_ij, over the kinds
//   grad_src_nu[j]   = sum_i Re G_i q_j dK_ij/d(n_x, n_y)  (D)
// K_D is linear in the normal: K = cps a + sps b with (cps, sps) the normal in
// the frame of the target direction, so dK/dn = (K n_x + K_psi n_y,
// K n_y - K_psi n_x) / |n|^2 with K_psi = dK/dpsi; n is per source, so the
// factor comes out of the sum over centers.
__global__ __launch_bounds__(256) void k_explicit_source_grads(
    int N, int kind, int n_csplit, const double4* __restrict__ geo,
    const double2* __restrict__ dens, const double2* __restrict__ partial,
    double* __restrict__ grad_q, double* __restrict__ grad_src_xy,
    double* __restrict__ grad_src_nu) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const bool hasS = kind & 1, hasD = kind & 2;
  const int nk = hasS && hasD ? 2 : 1;
  const int NA = src_slots(kind);
  double s[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int cs = 0; cs < n_csplit; ++cs)
    for (int b = 0; b < NA; ++b) {
      const double2 v = partial[((size_t)cs * NA + b) * N + j];
      s[b][0] += v.x;
      s[b][1] += v.y;
    }
  if (grad_q) {
    for (int kk = 0; kk < nk; ++kk) {
      const size_t o = (size_t)kk * N + j;
      grad_q[2 * o] = s[kk][0];
      grad_q[2 * o + 1] = s[kk][1];
    }
  }
  if (hasD && grad_src_nu) {
    // s[nk - 1] = conj(sum G K): Re(q sum G K) = Re(q conj(s[nk - 1]))
    const double2 w = dens[(size_t)(nk - 1) * N + j];
    const double A = w.x * s[nk - 1][0] + w.y * s[nk - 1][1];
    const double B = s[nk + 1][0];
    const double4 g = geo[j];
    const double n2 = fma(g.z, g.z, g.w * g.w);
    const double inv = n2 > 0.0 ? 1.0 / n2 : 0.0;
    grad_src_nu[2 * (size_t)j] = fma(g.z, A, g.w * B) * inv;
    grad_src_nu[2 * (size_t)j + 1] = fma(g.w, A, -g.z * B) * inv;
  }
  if (grad_src_xy) {
    grad_src_xy[2 * (size_t)j] = s[nk][0];
    grad_src_xy[2 * (size_t)j + 1] = s[nk][1];
  }
}

// per center, from the tape (sum_j q_j of dK/dR, dK/dtheta, grad_v K):
//   grad_ctr_xy = -Re G grad_v-sum (the target offset R e^{i theta} is an input,
//   so moving c moves the target with it), grad_ctr_r = Re G dK/dR-sum,
//   grad_ctr_theta = Re G dK/dtheta-sum, summed over kinds
__global__ __launch_bounds__(256) void k_explicit_center_grads(
    int Mc, int nk, const double2* __restrict__ tape, const double2* __restrict__ G,
    double* __restrict__ grad_ctr_xy, double* __restrict__ grad_ctr_r,
    double* __restrict__ grad_ctr_theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mc) return;
  double dR = 0.0, dt = 0.0, gvx = 0.0, gvy = 0.0;
  for (int kk = 0; kk < nk; ++kk) {
    const double2 g = G[(size_t)kk * Mc + i];
    const double2* tp = tape + ((size_t)i * nk + kk) * 4;
    dR += g.x * tp[0].x - g.y * tp[0].y;
    dt += g.x * tp[1].x - g.y * tp[1].y;
    gvx += g.x * tp[2].x - g.y * tp[2].y;
    gvy += g.x * tp[3].x - g.y * tp[3].y;
  }
  if (grad_ctr_xy) {
    grad_ctr_xy[2 * (size_t)i] = -gvx;
    grad_ctr_xy[2 * (size_t)i + 1] = -gvy;
  }
  if (grad_ctr_r) grad_ctr_r[i] = dR;
  if (grad_ctr_theta) grad_ctr_theta[i] = dt;
}

namespace {

bool explicit_dims(int n_src, int n_ctr, int p, int kind, double k, Dims* d) {
  if (n_src < 1 || n_ctr < 1 || p < 0 || p > kPMax) return false;
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D)) return false;
  if (!(k > 0.0) || !std::isfinite(k)) return false;
  if ((long)n_src > (1L << 30) || (long)n_ctr > (1L << 28)) return false;
  // one "panel" of 16 nodes keeps the shared workspace layout valid; the
  // panel tables and lengths are not used here
  d->P = 1;
  d->qs = kQ;
  d->T = n_ctr;
  d->N = n_src;
  d->n_sides = 1;
  d->nk = kind == 3 ? 2 : 1;
  d->p = p;
  d->Mc = n_ctr;
  d->NJ = 2 * (p + 4);
  d->side = QBX_EXTERIOR;
  d->kind = kind;
  d->k = k;
  d->r = 0.0;
  set_launch_shape(d);
  return true;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int explicit_validate(int n_src, const double* src_xy, const double* src_nu, const double* src_q,
                      int n_ctr, const double* ctr_xy, const double* ctr_r, const double* ctr_dir,
                      double k, int p, int kind, void* ws, size_t ws_bytes, Dims* d, Layout* L) {
  if (!explicit_dims(n_src, n_ctr, p, kind, k, d))
    return fail(QBX_EINVAL,
                "invalid explicit problem (n_src = %d, n_ctr = %d, p = %d, kind = %d, k = %g)",
                n_src, n_ctr, p, kind, k);
  if (!src_xy || !src_q || !ctr_xy || !ctr_r || !ctr_dir)
    return fail(QBX_EINVAL, "NULL source or center array");
  if ((kind & QBX_D) && !src_nu) return fail(QBX_EINVAL, "src_nu is needed for the double layer");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  *L = make_layout(*d);
  if (ws_bytes < L->total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L->total);
  return QBX_OK;
}

int explicit_prepare(const Dims& d, const Layout& L, const double* src_xy, const double* src_nu,
                     const double* src_q, const double* ctr_xy, const double* ctr_r,
                     const double* ctr_dir, void* ws, hipStream_t s) {
  hipLaunchKernelGGL(k_explicit_sources, dim3((d.N + 255) / 256), dim3(256), 0, s, d.N, d.nk,
                     src_xy, (d.kind & QBX_D) ? src_nu : nullptr, src_q, at<double4>(ws, L.geo),
                     at<double2>(ws, L.dens));
  hipLaunchKernelGGL(k_explicit_centers, dim3((d.Mc + 255) / 256), dim3(256), 0, s, d.Mc, d.NJ,
                     d.k, ctr_xy, ctr_r, ctr_dir, at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "explicit input kernels");
}

}  // namespace
}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_explicit_workspace_bytes(int n_src, int n_ctr, int p, int kind) {
  Dims d;
  if (!explicit_dims(n_src, n_ctr, p, kind, 1.0, &d)) return 0;
  return make_layout(d).total;
}

size_t qbx_explicit_tape_bytes(int n_ctr, int kind) {
  if (n_ctr < 1 || (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D))) return 0;
  return sizeof(double2) * (size_t)n_ctr * (kind == 3 ? 2 : 1) * 4;
}

int qbx_apply_explicit(int n_src, const double* src_xy, const double* src_nu, const double* src_q,
                       int n_ctr, const double* ctr_xy, const double* ctr_r, const double* ctr_dir,
                       double k, int p, int kind, double* out, double* tape, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  Dims d;
  Layout L;
  int rc = explicit_validate(n_src, src_xy, src_nu, src_q, n_ctr, ctr_xy, ctr_r, ctr_dir, k, p,
                             kind, ws, ws_bytes, &d, &L);
  if (rc) return rc;
  if (!out) return fail(QBX_EINVAL, "out is NULL");
  rc = explicit_prepare(d, L, src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, ws, stream);
  if (rc) return rc;
  hipError_t e;
  if (tape) {
    timer_begin(3, stream);
    e = launch_forward_tape(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                            at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                            at<double2>(ws, L.partial), stream);
    timer_end(3, stream);
    if (e != hipSuccess) return device_fail(e, "explicit forward (tape) kernel");
    e = launch_finalize_tape(d, at<double2>(ws, L.partial), out, reinterpret_cast<double2*>(tape),
                             stream);
    return e == hipSuccess ? QBX_OK : device_fail(e, "explicit finalize (tape) kernel");
  }
  timer_begin(0, stream);
  e = launch_forward(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens), at<CenterRec>(ws, L.ctr),
                     at<double>(ws, L.jtab), at<double2>(ws, L.partial), stream);
  timer_end(0, stream);
  if (e != hipSuccess) return device_fail(e, "explicit forward kernel");
  e = launch_finalize(d, at<double2>(ws, L.partial), out, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "explicit finalize kernel");
}

int qbx_apply_explicit_gradient(int n_src, const double* src_xy, const double* src_nu,
                                const double* src_q, int n_ctr, const double* ctr_xy,
                                const double* ctr_r, const double* ctr_dir, double k, int p,
                                int kind, double* grad, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  Dims d;
  Layout L;
  int rc = explicit_validate(n_src, src_xy, src_nu, src_q, n_ctr, ctr_xy, ctr_r, ctr_dir, k, p,
                             kind, ws, ws_bytes, &d, &L);
  if (rc) return rc;
  if (!grad) return fail(QBX_EINVAL, "grad is NULL");
  rc = explicit_prepare(d, L, src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, ws, stream);
  if (rc) return rc;
  hipError_t e = launch_order_weighted(d, at<double>(ws, L.jtab), stream);
  if (e != hipSuccess) return device_fail(e, "explicit order-weighted table kernel");
  timer_begin(5, stream);
  e = launch_forward_grad(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                          at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                          at<double2>(ws, L.partial), stream);
  timer_end(5, stream);
  if (e != hipSuccess) return device_fail(e, "explicit target-derivative kernel");
  // one side and T = n_ctr: out[kind][center][2] = the gradient at the target
  e = launch_finalize_gradient(d, at<CenterRec>(ws, L.ctr), at<double2>(ws, L.partial), grad,
                               nullptr, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "explicit gradient finalize kernel");
}

int qbx_apply_explicit_adjoint(int n_src, const double* src_xy, const double* src_nu,
                               const double* src_q, int n_ctr, const double* ctr_xy,
                               const double* ctr_r, const double* ctr_dir, double k, int p,
                               int kind, const double* cotangent, const double* tape,
                               double* grad_q, double* grad_src_xy, double* grad_src_nu,
                               double* grad_ctr_xy, double* grad_ctr_r, double* grad_ctr_theta,
                               void* ws, size_t ws_bytes, hipStream_t stream) {
  Dims d;
  Layout L;
  int rc = explicit_validate(n_src, src_xy, src_nu, src_q, n_ctr, ctr_xy, ctr_r, ctr_dir, k, p,
                             kind, ws, ws_bytes, &d, &L);
  if (rc) return rc;
  if (!cotangent) return fail(QBX_EINVAL, "cotangent is NULL");
  if (!(kind & QBX_D)) grad_src_nu = nullptr;
  const bool want_src = grad_q || grad_src_xy || grad_src_nu;
  const bool want_ctr = grad_ctr_xy || grad_ctr_r || grad_ctr_theta;
  if (!want_src && !want_ctr) return QBX_OK;
  rc = explicit_prepare(d, L, src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, ws, stream);
  if (rc) return rc;
  hipError_t e = launch_make_G(d, cotangent, at<double2>(ws, L.G), stream);
  if (e != hipSuccess) return device_fail(e, "explicit cotangent kernel");
  if (want_ctr) {
    const double2* tp = reinterpret_cast<const double2*>(tape);
    if (!tp) {
      timer_begin(3, stream);
      e = launch_forward_tape(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                              at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                              at<double2>(ws, L.partial), stream);
      timer_end(3, stream);
      if (e != hipSuccess) return device_fail(e, "explicit forward (tape) kernel");
      e = launch_finalize_tape(d, at<double2>(ws, L.partial), nullptr, at<double2>(ws, L.tape),
                               stream);
      if (e != hipSuccess) return device_fail(e, "explicit finalize (tape) kernel");
      tp = at<double2>(ws, L.tape);
    }
    hipLaunchKernelGGL(k_explicit_center_grads, dim3((d.Mc + 255) / 256), dim3(256), 0, stream,
                       d.Mc, d.nk, tp, at<double2>(ws, L.G), grad_ctr_xy, grad_ctr_r,
                       grad_ctr_theta);
    e = hipGetLastError();
    if (e != hipSuccess) return device_fail(e, "explicit center gradient kernel");
  }
  if (want_src) {
    timer_begin(1, stream);
    e = launch_adjoint_src(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                           at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                           at<double2>(ws, L.G), at<double2>(ws, L.spart), stream);
    timer_end(1, stream);
    if (e != hipSuccess) return device_fail(e, "explicit adjoint source pass");
    hipLaunchKernelGGL(k_explicit_source_grads, dim3((d.N + 255) / 256), dim3(256), 0, stream,
                       d.N, d.kind, d.n_csplit, at<double4>(ws, L.geo),
                       at<double2>(ws, L.dens), at<double2>(ws, L.spart), grad_q, grad_src_xy,
                       grad_src_nu);
    e = hipGetLastError();
    if (e != hipSuccess) return device_fail(e, "explicit source gradient kernel");
  }
  return QBX_OK;
}

}  // extern "C"
