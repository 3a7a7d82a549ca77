// Nystrom solve of the Dirichlet problem (Section 4.3) with the combined-field
// representation u = -D sigma + alpha S sigma:
//     -+ sigma/2 + alpha S sigma - D sigma = f           (eq. dirichlet-inteq)
// (upper sign: the exterior problem), S and D the principal values.  Both are
// taken as the averages of the two one-sided QBX limits (eq. dlp-twosided):
// Section 3.5 shows that the one-sided limit of D damps high-frequency densities
// but not the sigma/2 of its jump, so that its discrete spectrum loses the
// clustering of the continuous operator and GMRES stalls at the discretization
// error, while the average keeps it.  One matrix-vector product is therefore
// one S+D call of the forward (qbx_layer_potential, or
// qbx_layer_potential_split) for both sides, with the density sigma for both
// kinds.
//
// As the paper does (after Bremer), the unknowns are tau = sqrt(w) sigma, w the
// 16-point rule's weight at the node, so that the l2 product of the iteration
// approximates the L2 product on the curve: GMRES solves
// W^{1/2} A W^{-1/2} tau = W^{1/2} f.  GMRES(m): Arnoldi with classical
// Gram-Schmidt and one re-orthogonalisation, Givens rotations and the small
// least-squares problem on the host; every vector operation in the kernels
// below, every reduction in a fixed order (the solve is deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "../../include/qbx.h"
#include "qbx_internal.h"

namespace qbx {

using cplx = std::complex<double>;
constexpr int kDotBlocks = 256;      // first-stage blocks of the multi-dot
constexpr int kMaxRestart = 1000;   // Krylov vectors kept (16 B x nodes each)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// sw[t] = sqrt(w_t), w_t = omega_a |X'(tau_a)| at node t = 16 m + a: the 16-point
// rule on the panel's parameter interval, X' from the 16-node derivative matrix
__global__ __launch_bounds__(256) void k_sqrt_weights(int T, int qs, const double* __restrict__ nodes,
                                                      const double* __restrict__ tab,
                                                      double* __restrict__ sw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const TableLayout L = table_layout(qs);
  const int m = t / kQ, a = t - m * kQ;
  const double* X = nodes + (size_t)m * 2 * kQ;
  const double* Dr = tab + L.Dn + a * kQ;
  double tx = 0.0, ty = 0.0;
  for (int c = 0; c < kQ; ++c) {
    tx = fma(Dr[c], X[2 * c], tx);
    ty = fma(Dr[c], X[2 * c + 1], ty);
  }
  sw[t] = sqrt(tab[L.w16 + a] * sqrt(tx * tx + ty * ty));
}

// y = x * sw (inv = 0) or x / sw (inv = 1)
__global__ __launch_bounds__(256) void k_scale_weights(int T, const double2* __restrict__ x,
                                                       const double* __restrict__ sw, int inv,
                                                       double2* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double s = inv ? 1.0 / sw[t] : sw[t];
  y[t] = make_double2(x[t].x * s, x[t].y * s);
}

// the density of both kinds for the forward: sigma = v / sw
__global__ __launch_bounds__(256) void k_to_density(int T, const double2* __restrict__ v,
                                                    const double* __restrict__ sw,
                                                    double2* __restrict__ dens) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double s = 1.0 / sw[t];
  const double2 d = make_double2(v[t].x * s, v[t].y * s);
  dens[t] = d;
  dens[T + t] = d;
}

// y = half v + sw (alpha S sigma - D sigma), sigma = v / sw, with S and D the
// averages of out = [S+, D+, S-, D-] (exterior limits first)
__global__ __launch_bounds__(256) void k_combine(int T, const double2* __restrict__ v,
                                                 const double* __restrict__ sw,
                                                 const double2* __restrict__ out, double half,
                                                 double2 alpha, double2* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double2 sp = out[t], dp = out[T + t], sm = out[2 * T + t], dm = out[3 * T + t];
  const double2 S = make_double2(0.5 * (sp.x + sm.x), 0.5 * (sp.y + sm.y));
  const double2 a = cmul(alpha, S);
  const double dx = 0.5 * (dp.x + dm.x), dy = 0.5 * (dp.y + dm.y);
  y[t] = make_double2(fma(half, v[t].x, sw[t] * (a.x - dx)), fma(half, v[t].y, sw[t] * (a.y - dy)));
}

// partial[b][i] = sum over block b's slice of conj(V_i[t]) w[t], i < nv
__global__ __launch_bounds__(256) void k_dots_partial(int T, const double2* __restrict__ V, int nv,
                                                      const double2* __restrict__ w,
                                                      double2* __restrict__ partial) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  for (int i = 0; i < nv; ++i) {
    const double2* vi = V + (size_t)i * T;
    double re = 0.0, im = 0.0;
    for (int t = blockIdx.x * 256 + tid; t < T; t += gridDim.x * 256) {
      const double2 a = vi[t], b = w[t];
      re = fma(a.x, b.x, fma(a.y, b.y, re));     // conj(a) b
      im = fma(a.x, b.y, fma(-a.y, b.x, im));
    }
    red[0][tid] = re;
    red[1][tid] = im;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) {
        red[0][tid] += red[0][tid + off];
        red[1][tid] += red[1][tid + off];
      }
      __syncthreads();
    }
    if (tid == 0) partial[(size_t)blockIdx.x * nv + i] = make_double2(red[0][0], red[1][0]);
    __syncthreads();
  }
}

// h[i] = sum over blocks, in block order
__global__ __launch_bounds__(256) void k_dots_final(int nblk, int nv,
                                                    const double2* __restrict__ partial,
                                                    double2* __restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2 v = partial[(size_t)b * nv + i];
    re += v.x;
    im += v.y;
  }
  h[i] = make_double2(re, im);
}

// w -= sum_i h[i] V_i
__global__ __launch_bounds__(256) void k_subtract(int T, const double2* __restrict__ V, int nv,
                                                  const double2* __restrict__ h,
                                                  double2* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double2 acc = w[t];
  for (int i = 0; i < nv; ++i) {
    const double2 c = h[i], v = V[(size_t)i * T + t];
    acc.x -= c.x * v.x - c.y * v.y;
    acc.y -= c.x * v.y + c.y * v.x;
  }
  w[t] = acc;
}

// y = s x (s real), or y = b - x when diff != 0; y may be x (in place)
__global__ __launch_bounds__(256) void k_axpby(int T, double s, const double2* x, int diff,
                                               const double2* b, double2* y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  y[t] = diff ? make_double2(b[t].x - x[t].x, b[t].y - x[t].y)
              : make_double2(s * x[t].x, s * x[t].y);
}

// adjoint products: cot[si][kk][t] = u_t / 2 for both sides and kinds, u = sw v
__global__ __launch_bounds__(256) void k_adj_cot(int T, const double2* __restrict__ v,
                                                 const double* __restrict__ sw,
                                                 double2* __restrict__ cot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double h = 0.5 * sw[t];
  const double2 u = make_double2(h * v[t].x, h * v[t].y);
  cot[t] = u;
  cot[T + t] = u;
  cot[2 * T + t] = u;
  cot[3 * T + t] = u;
}

// y = (half u + conj(alpha) S^H u - D^H u) / sw, u = sw v, gd = [S^H u; D^H u] (averaged
// over the sides by the cotangent's halves)
__global__ __launch_bounds__(256) void k_adj_combine(int T, const double2* __restrict__ v,
                                                     const double* __restrict__ sw,
                                                     const double2* __restrict__ gd, double half,
                                                     double2 alpha, double2* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double2 a = cmul(make_double2(alpha.x, -alpha.y), gd[t]);
  const double2 d = gd[T + t];
  const double inv = 1.0 / sw[t];
  y[t] = make_double2(fma(half, v[t].x, inv * (a.x - d.x)), fma(half, v[t].y, inv * (a.y - d.y)));
}

// node gradient of the solve: dens = [sigma; sigma] and, on both sides,
// cot[si][0] = -conj(alpha) lambda / 2 (S) and cot[si][1] = lambda / 2 (D), the
// cotangents whose layer-potential node adjoint is -grad_x Re <lambda, A(x) sigma>
__global__ __launch_bounds__(256) void k_node_cot(int T, const double2* __restrict__ sigma,
                                                  const double2* __restrict__ lambda,
                                                  double2 alpha, double2* __restrict__ dens,
                                                  double2* __restrict__ cot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double2 sg = sigma[t], lm = lambda[t];
  dens[t] = sg;
  dens[T + t] = sg;
  const double2 ca = cmul(make_double2(alpha.x, -alpha.y), lm);
  const double2 cs = make_double2(-0.5 * ca.x, -0.5 * ca.y);
  const double2 cd = make_double2(0.5 * lm.x, 0.5 * lm.y);
  cot[t] = cs;
  cot[T + t] = cd;
  cot[2 * T + t] = cs;
  cot[3 * T + t] = cd;
}

__global__ __launch_bounds__(256) void k_zero(int n, double2* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = make_double2(0.0, 0.0);
}

struct SolveLayout {
  size_t fws, fws_bytes, tables, sw, dens, out, V, w, b, x, partial, h, total;
};

static SolveLayout make_solve_layout(const Dims& d, int restart) {
  SolveLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t T = (size_t)d.T;
  L.fws_bytes = make_layout(d).total;
  L.fws = take(L.fws_bytes);
  L.tables = take(sizeof(double) * table_layout(d.qs).total);
  L.sw = take(sizeof(double) * T);
  L.dens = take(sizeof(double2) * 6 * T);   // density [2][T], then adjoint cotangent [4][T]
  L.out = take(sizeof(double2) * 4 * T);
  L.V = take(sizeof(double2) * (size_t)(restart + 1) * T);
  L.w = take(sizeof(double2) * T);
  L.b = take(sizeof(double2) * T);
  L.x = take(sizeof(double2) * T);
  L.partial = take(sizeof(double2) * kDotBlocks * (size_t)(restart + 1));
  L.h = take(sizeof(double2) * (size_t)(restart + 1));
  L.total = o;
  return L;
}

// the iteration's state and its device calls
struct Gmres {
  const qbx_geometry* g;
  const Dims& d;
  SolveLayout L;
  char* ws;
  hipStream_t s;
  double k, r, gamma;
  int p, oversample;
  double half;     // -1/2 for the exterior problem, +1/2 for the interior one
  double2 alpha;
  bool adjoint;    // products by A^H instead of A
  int T, grid;

  template <typename X>
  X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
  double2* V(int i) const { return at<double2>(L.V) + (size_t)i * T; }

  int check(hipError_t e, const char* what) const {
    return e == hipSuccess ? QBX_OK : device_fail(e, what);
  }
  // y = W^{1/2} (-+ 1/2 + alpha S - D) W^{-1/2} v, or for the adjoint system
  // y = W^{-1/2} (-+ 1/2 + conj(alpha) S^H - D^H) W^{1/2} v
  int matvec(const double2* v, double2* y) const {
    if (adjoint) return matvec_adjoint(v, y);
    hipLaunchKernelGGL(k_to_density, dim3(grid), dim3(256), 0, s, T, v, at<double>(L.sw),
                       at<double2>(L.dens));
    int rc = check(hipGetLastError(), "solve density kernel");
    if (rc) return rc;
    double* out = at<double>(L.out);
    const double* dens = at<double>(L.dens);
    if (gamma > 0.0)
      rc = qbx_layer_potential_split(g, dens, k, p, r, oversample, QBX_BOTH, 3, gamma, out,
                                     ws + L.fws, L.fws_bytes, s);
    else
      rc = qbx_layer_potential(g, dens, k, p, r, oversample, QBX_BOTH, 3, out, nullptr,
                               ws + L.fws, L.fws_bytes, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_combine, dim3(grid), dim3(256), 0, s, T, v, at<double>(L.sw),
                       at<double2>(L.out), half, alpha, y);
    return check(hipGetLastError(), "solve combine kernel");
  }
  int matvec_adjoint(const double2* v, double2* y) const {
    double2* cot = at<double2>(L.dens) + 2 * (size_t)T;
    hipLaunchKernelGGL(k_adj_cot, dim3(grid), dim3(256), 0, s, T, v, at<double>(L.sw), cot);
    int rc = check(hipGetLastError(), "solve cotangent kernel");
    if (rc) return rc;
    double* gd = at<double>(L.out);
    const double* dens = at<double>(L.dens);   // zeros: the density gradient does not read it
    const double* c = reinterpret_cast<const double*>(cot);
    if (gamma > 0.0)
      rc = qbx_layer_potential_split_adjoint(g, dens, k, p, r, oversample, QBX_BOTH, 3, gamma, c,
                                             gd, nullptr, ws + L.fws, L.fws_bytes, s);
    else
      rc = qbx_layer_potential_adjoint(g, dens, k, p, r, oversample, QBX_BOTH, 3, c, nullptr, gd,
                                       nullptr, ws + L.fws, L.fws_bytes, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_adj_combine, dim3(grid), dim3(256), 0, s, T, v, at<double>(L.sw),
                       at<double2>(L.out), half, alpha, y);
    return check(hipGetLastError(), "solve adjoint combine kernel");
  }
  // h[0..nv) = V_i^H w on the device, and a host copy
  int dots(const double2* Vb, int nv, const double2* w, cplx* host) const {
    hipLaunchKernelGGL(k_dots_partial, dim3(kDotBlocks), dim3(256), 0, s, T, Vb, nv, w,
                       at<double2>(L.partial));
    hipLaunchKernelGGL(k_dots_final, dim3((nv + 255) / 256), dim3(256), 0, s, kDotBlocks, nv,
                       at<double2>(L.partial), at<double2>(L.h));
    int rc = check(hipGetLastError(), "solve dot kernels");
    if (rc) return rc;
    rc = check(hipMemcpyAsync(host, at<double2>(L.h), sizeof(double2) * nv,
                              hipMemcpyDeviceToHost, s), "solve dot copy");
    if (rc) return rc;
    return check(hipStreamSynchronize(s), "solve dot sync");
  }
  // w -= sum_i h_i V_i with h already on the device
  int subtract(int nv, double2* w) const {
    hipLaunchKernelGGL(k_subtract, dim3(grid), dim3(256), 0, s, T, at<double2>(L.V), nv,
                       at<double2>(L.h), w);
    return check(hipGetLastError(), "solve update kernel");
  }
  int norm(const double2* w, double* n) const {
    cplx h;
    const int rc = dots(w, 1, w, &h);
    *n = std::sqrt(std::max(h.real(), 0.0));
    return rc;
  }
  int axpby(double sc, const double2* x, int diff, const double2* b, double2* y) const {
    hipLaunchKernelGGL(k_axpby, dim3(grid), dim3(256), 0, s, T, sc, x, diff, b, y);
    return check(hipGetLastError(), "solve vector kernel");
  }
};

}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_solve_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                 int restart) {
  Dims d;
  if ((side != QBX_EXTERIOR && side != QBX_INTERIOR) || restart < 1 || restart > kMaxRestart)
    return 0;
  if (!make_dims(n_panels, q, p, oversample, QBX_BOTH, 3, 1.0, 0.5, &d)) return 0;
  return make_solve_layout(d, restart).total;
}

}  // extern "C"

namespace qbx {

// GMRES on the scaled system (adjoint = false: A sigma = f, b = W^{1/2} f and
// sigma = W^{-1/2} x; adjoint = true: A^H lambda = f, b = W^{-1/2} f and
// lambda = W^{1/2} x)
static int solve(const qbx_geometry* g, const double* f, double k, int p, double r,
                 int oversample, int side, double alpha_re, double alpha_im, double gamma,
                 double tol, int restart, int max_iter, bool adjoint, double* sigma,
                 int* iterations, double* residual, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  if (side != QBX_EXTERIOR && side != QBX_INTERIOR)
    return fail(QBX_EINVAL, "side = %d must be -1 (interior) or 1 (exterior)", side);
  Dims d;   // of the forward, which takes both one-sided limits
  int rc = validate(g, p, k, r, oversample, QBX_BOTH, 3, &d);
  if (rc) return rc;
  if (!f || !sigma) return fail(QBX_EINVAL, "right-hand side or solution is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(QBX_EINVAL, "tol = %g must be > 0", tol);
  if (restart < 1 || restart > kMaxRestart)
    return fail(QBX_EINVAL, "restart = %d outside [1, %d]", restart, kMaxRestart);
  if (max_iter < 1) return fail(QBX_EINVAL, "max_iter = %d < 1", max_iter);
  if (!(gamma >= 0.0)) return fail(QBX_EINVAL, "gamma = %g must be >= 0", gamma);
  if (!std::isfinite(alpha_re) || !std::isfinite(alpha_im))
    return fail(QBX_EINVAL, "alpha is not finite");
  const SolveLayout L = make_solve_layout(d, restart);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  Gmres G{g, d, L, static_cast<char*>(ws), stream, k, r, gamma, p, oversample,
          side == QBX_EXTERIOR ? -0.5 : 0.5, make_double2(alpha_re, alpha_im), adjoint, d.T,
          (d.T + 255) / 256};
  const int T = d.T, m = restart;
  double2* b = G.at<double2>(L.b);
  double2* x = G.at<double2>(L.x);
  double2* w = G.at<double2>(L.w);
  double* sw = G.at<double>(L.sw);
  // weights and the scaled right-hand side
  hipError_t e = launch_tables(d, G.at<double>(L.tables), stream);
  if (e != hipSuccess) return device_fail(e, "tables kernel");
  hipLaunchKernelGGL(k_sqrt_weights, dim3(G.grid), dim3(256), 0, stream, T, d.qs, g->nodes,
                     G.at<double>(L.tables), sw);
  hipLaunchKernelGGL(k_scale_weights, dim3(G.grid), dim3(256), 0, stream, T,
                     reinterpret_cast<const double2*>(f), sw, adjoint ? 1 : 0, b);
  hipLaunchKernelGGL(k_zero, dim3(G.grid), dim3(256), 0, stream, T, x);
  if (adjoint)
    hipLaunchKernelGGL(k_zero, dim3((2 * T + 255) / 256), dim3(256), 0, stream, 2 * T,
                       G.at<double2>(L.dens));
  if ((rc = G.check(hipGetLastError(), "solve set-up kernels"))) return rc;
  double bnorm;
  if ((rc = G.norm(b, &bnorm))) return rc;
  int it = 0;
  double res = 0.0;
  if (bnorm > 0.0) {
    std::vector<cplx> H((size_t)(m + 1) * m), gv(m + 1), cs(m), sn(m), y(m), h1(m + 1), h2(m + 1);
    auto Hs = [&](int i, int j) -> cplx& { return H[(size_t)i * m + j]; };
    bool done = false;
    while (!done) {
      // r = b - A x (x = 0 at the start)
      if (it == 0) {
        rc = G.axpby(1.0, b, 0, nullptr, G.V(0));
      } else {
        if ((rc = G.matvec(x, w))) return rc;
        rc = G.axpby(0.0, w, 1, b, G.V(0));
      }
      if (rc) return rc;
      double beta;
      if ((rc = G.norm(G.V(0), &beta))) return rc;
      res = beta / bnorm;
      if (res <= tol || it >= max_iter) break;
      if ((rc = G.axpby(1.0 / beta, G.V(0), 0, nullptr, G.V(0)))) return rc;
      std::fill(gv.begin(), gv.end(), cplx(0.0));
      gv[0] = beta;
      int jj = 0;
      for (int j = 0; j < m; ++j) {
        if ((rc = G.matvec(G.V(j), w))) return rc;
        // classical Gram-Schmidt, twice
        if ((rc = G.dots(G.V(0), j + 1, w, h1.data()))) return rc;
        if ((rc = G.subtract(j + 1, w))) return rc;
        if ((rc = G.dots(G.V(0), j + 1, w, h2.data()))) return rc;
        if ((rc = G.subtract(j + 1, w))) return rc;
        for (int i = 0; i <= j; ++i) Hs(i, j) = h1[i] + h2[i];
        double hn;
        if ((rc = G.norm(w, &hn))) return rc;
        // previous rotations, then the new one
        for (int i = 0; i < j; ++i) {
          const cplx a = Hs(i, j), bb = Hs(i + 1, j);
          Hs(i, j) = cs[i] * a + sn[i] * bb;
          Hs(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * bb;
        }
        const cplx a = Hs(j, j);
        const double aa = std::abs(a);
        if (aa == 0.0) {
          cs[j] = 0.0;
          sn[j] = 1.0;
          Hs(j, j) = hn;
        } else {
          const double rr = std::hypot(aa, hn);
          const cplx ph = a / aa;
          cs[j] = aa / rr;
          sn[j] = ph * hn / rr;
          Hs(j, j) = ph * rr;
        }
        gv[j + 1] = -std::conj(sn[j]) * gv[j];
        gv[j] = cs[j] * gv[j];
        ++it;
        jj = j + 1;
        res = std::abs(gv[j + 1]) / bnorm;
        if (res <= tol || it >= max_iter || hn == 0.0) {
          done = true;
          break;
        }
        if ((rc = G.axpby(1.0 / hn, w, 0, nullptr, G.V(j + 1)))) return rc;
      }
      // x += V y, H y = g (upper triangular).  A zero pivot (the operator
      // singular on the Krylov space: w = 0 with nothing left to rotate) takes
      // y_i = 0, so the update stays finite and the true residual below shows it
      for (int i = jj - 1; i >= 0; --i) {
        cplx acc = gv[i];
        for (int l = i + 1; l < jj; ++l) acc -= Hs(i, l) * y[l];
        y[i] = Hs(i, i) == cplx(0.0) ? cplx(0.0) : acc / Hs(i, i);
      }
      std::vector<double2> ny(jj);
      for (int i = 0; i < jj; ++i) ny[i] = make_double2(-y[i].real(), -y[i].imag());
      if ((rc = G.check(hipMemcpyAsync(G.at<double2>(L.h), ny.data(), sizeof(double2) * jj,
                                       hipMemcpyHostToDevice, stream), "solve copy"))) return rc;
      if ((rc = G.subtract(jj, x))) return rc;
      if ((rc = G.check(hipStreamSynchronize(stream), "solve sync"))) return rc;
    }
    // the true residual of the returned solution
    if ((rc = G.matvec(x, w))) return rc;
    if ((rc = G.axpby(0.0, w, 1, b, w))) return rc;
    double rn;
    if ((rc = G.norm(w, &rn))) return rc;
    res = rn / bnorm;
  }
  hipLaunchKernelGGL(k_scale_weights, dim3(G.grid), dim3(256), 0, stream, T, x, sw,
                     adjoint ? 0 : 1, reinterpret_cast<double2*>(sigma));
  if ((rc = G.check(hipGetLastError(), "solve output kernel"))) return rc;
  if ((rc = G.check(hipStreamSynchronize(stream), "solve sync"))) return rc;
  if (iterations) *iterations = it;
  if (residual) *residual = res;
  return QBX_OK;
}

}  // namespace qbx

extern "C" {

int qbx_solve_dirichlet(const qbx_geometry* g, const double* f, double k, int p, double r,
                        int oversample, int side, double alpha_re, double alpha_im, double gamma,
                        double tol, int restart, int max_iter, double* sigma, int* iterations,
                        double* residual, void* ws, size_t ws_bytes, hipStream_t stream) {
  return solve(g, f, k, p, r, oversample, side, alpha_re, alpha_im, gamma, tol, restart, max_iter,
               false, sigma, iterations, residual, ws, ws_bytes, stream);
}

size_t qbx_solve_node_gradient_workspace_bytes(int n_panels, int q, int p, int oversample) {
  Dims d;
  if (!make_dims(n_panels, q, p, oversample, QBX_BOTH, 3, 1.0, 0.5, &d)) return 0;
  return align256(make_layout(d).total) + align256(sizeof(double2) * 2 * (size_t)d.T) +
         align256(sizeof(double2) * 4 * (size_t)d.T);
}

int qbx_solve_dirichlet_node_gradient(const qbx_geometry* g, const double* sigma,
                                      const double* lambda, double k, int p, double r,
                                      int oversample, int side, double alpha_re, double alpha_im,
                                      double gamma, double* grad_nodes, void* ws,
                                      size_t ws_bytes, hipStream_t stream) {
  if (side != QBX_EXTERIOR && side != QBX_INTERIOR)
    return fail(QBX_EINVAL, "side = %d: the Dirichlet problem takes 1 or -1", side);
  Dims d;
  int rc = validate(g, p, k, r, oversample, QBX_BOTH, 3, &d);
  if (rc) return rc;
  if (!sigma || !lambda || !grad_nodes) return fail(QBX_EINVAL, "NULL array argument");
  if (!std::isfinite(alpha_re) || !std::isfinite(alpha_im))
    return fail(QBX_EINVAL, "alpha is not finite");
  if (!(gamma >= 0.0)) return fail(QBX_EINVAL, "near-panel factor gamma = %g must be >= 0", gamma);
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const size_t fws = make_layout(d).total;
  const size_t o_dens = align256(fws), o_cot = o_dens + align256(sizeof(double2) * 2 * (size_t)d.T);
  const size_t need = o_cot + align256(sizeof(double2) * 4 * (size_t)d.T);
  if (ws_bytes < need)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  char* w = static_cast<char*>(ws);
  double2* dens = reinterpret_cast<double2*>(w + o_dens);
  double2* cot = reinterpret_cast<double2*>(w + o_cot);
  hipLaunchKernelGGL(k_node_cot, dim3((d.T + 255) / 256), dim3(256), 0, stream, d.T,
                     reinterpret_cast<const double2*>(sigma),
                     reinterpret_cast<const double2*>(lambda), make_double2(alpha_re, alpha_im),
                     dens, cot);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return device_fail(e, "node-gradient cotangent kernel");
  const double* dp = reinterpret_cast<const double*>(dens);
  const double* cp = reinterpret_cast<const double*>(cot);
  if (gamma > 0.0)
    return qbx_layer_potential_split_adjoint(g, dp, k, p, r, oversample, QBX_BOTH, 3, gamma, cp,
                                             nullptr, grad_nodes, ws, fws, stream);
  return qbx_layer_potential_adjoint(g, dp, k, p, r, oversample, QBX_BOTH, 3, cp, nullptr, nullptr,
                                     grad_nodes, ws, fws, stream);
}

int qbx_solve_dirichlet_adjoint(const qbx_geometry* g, const double* rhs, double k, int p,
                                double r, int oversample, int side, double alpha_re,
                                double alpha_im, double gamma, double tol, int restart,
                                int max_iter, double* lambda, int* iterations, double* residual,
                                void* ws, size_t ws_bytes, hipStream_t stream) {
  return solve(g, rhs, k, p, r, oversample, side, alpha_re, alpha_im, gamma, tol, restart,
               max_iter, true, lambda, iterations, residual, ws, ws_bytes, stream);
}

}  // extern "C"
