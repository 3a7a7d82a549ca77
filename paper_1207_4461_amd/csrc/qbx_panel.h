// Per-panel bodies shared by the per-contour and the batched kernels:
// the source grid and centers of one panel (upsample_panel) and the chain rule
// of the adjoint back to one panel's nodes and node densities (chain_panel).
//
//  * Section 4.1: a panel is the degree-15 polynomial through its 16 nodes at
//    the Gauss-Legendre abscissae of the panel parameter tau in [-1, 1].
//  * Section 3.4.2: the density is interpolated from the 16 nodes (target
//    grid) to the q_s = 16*oversample point Gauss-Legendre rule of the same
//    panel (source grid); source weights w = omega |dX/dtau|, outward normal
//    n = (y', -x') / |X'| for a counter-clockwise curve (Section 3.2).
//  * Section 3.3 step 4(a): c = x + s r h_m n with h_m the panel length,
//    radius R = r h_m, and theta = arg(x - c) = arg(-s n).
#pragma once

#include "qbx_internal.h"
#include "qbx_special.h"

namespace qbx {

// J_l(x) and J'_l(x), l = 0..nj-1, of one center into Jt[0..2nj): Miller's
// recurrence, then J'_l = (J_{l-1} - J_{l+1}) / 2 (DLMF 10.6.1) with J'_0 = -J_1
// and the last one from J_{l-1} - (l/x) J_l (DLMF 10.6.2)
__device__ __forceinline__ void center_bessel_table(double x, int nj, double* __restrict__ Jt) {
  bessel_j_miller(x, nj - 1, Jt);
  Jt[nj] = -Jt[1];
  for (int l = 1; l + 1 < nj; ++l) Jt[nj + l] = 0.5 * (Jt[l - 1] - Jt[l + 1]);
  Jt[2 * nj - 1] = (x > 0.0) ? Jt[nj - 2] - (nj - 1) / x * Jt[nj - 1] : 0.0;
}

// ---------------------------------------------------------------------------
// upsample: one block per panel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void upsample_panel(const Dims& d, int m, const double* __restrict__ nodes,
                                                  const double* __restrict__ density,
                                                  const double* __restrict__ tab,
                                                  double4* __restrict__ geo,
                                                  double2* __restrict__ dens,
                                                  double* __restrict__ wgt,
                                                  double* __restrict__ hpan,
                                                  CenterRec* __restrict__ ctr,
                                                  double* __restrict__ jtab) {
  const TableLayout L = table_layout(d.qs);
  const int t = threadIdx.x;
  __shared__ double X[kQ][2];
  __shared__ double2 S[2][kQ];
  __shared__ double red[128];
  if (t < 2 * kQ) X[t >> 1][t & 1] = nodes[(size_t)m * 2 * kQ + t];
  if (t < d.nk * kQ) {
    const int kk = t / kQ, a = t % kQ;
    const double* src = density + 2 * ((size_t)kk * d.T + (size_t)m * kQ + a);
    S[kk][a] = make_double2(src[0], src[1]);
  }
  __syncthreads();
  double wsum = 0.0;
  for (int b = t; b < d.qs; b += blockDim.x) {
    const double* Vr = tab + L.V + b * kQ;
    const double* Vdr = tab + L.Vd + b * kQ;
    double x = 0.0, y = 0.0, dx = 0.0, dy = 0.0;
    double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
      const double v = Vr[a], vd = Vdr[a];
      x = fma(v, X[a][0], x);
      y = fma(v, X[a][1], y);
      dx = fma(vd, X[a][0], dx);
      dy = fma(vd, X[a][1], dy);
      sr0 = fma(v, S[0][a].x, sr0);
      si0 = fma(v, S[0][a].y, si0);
      if (d.nk > 1) {
        sr1 = fma(v, S[1][a].x, sr1);
        si1 = fma(v, S[1][a].y, si1);
      }
    }
    const double speed = sqrt(dx * dx + dy * dy);
    const double w = tab[L.ws + b] * speed;
    const double inv = 1.0 / speed;
    const size_t j = (size_t)m * d.qs + b;
    // the direction of the D slot's source derivative: the outward normal, or
    // for the tangential dipole R the unit tangent (counter-clockwise)
    geo[j] = d.dipole ? make_double4(x, y, dx * inv, dy * inv)
                      : make_double4(x, y, dy * inv, -dx * inv);
    wgt[j] = w;
    dens[j] = make_double2(w * sr0, w * si0);
    if (d.nk > 1) dens[(size_t)d.N + j] = make_double2(w * sr1, w * si1);
    wsum += w;
  }
  red[t] = wsum;
  __syncthreads();
  for (int off = 64; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  const double hm = red[0];
  if (t == 0) hpan[m] = hm;
  if (t < kQ * d.n_sides) {
    const int a = t % kQ, si = t / kQ;
    const double sgn = side_sign(d.side, si);
    const double* Dr = tab + L.Dn + a * kQ;
    double tx = 0.0, ty = 0.0;
#pragma unroll
    for (int c = 0; c < kQ; ++c) {
      tx = fma(Dr[c], X[c][0], tx);
      ty = fma(Dr[c], X[c][1], ty);
    }
    const double inv = 1.0 / sqrt(tx * tx + ty * ty);
    const double nx = ty * inv, ny = -tx * inv;
    const double R = d.center_rule ? d.r * sqrt(hm) : d.r * hm;
    CenterRec c;
    c.x = X[a][0];
    c.y = X[a][1];
    c.cx = c.x + sgn * R * nx;
    c.cy = c.y + sgn * R * ny;
    c.R = R;
    c.ct = -sgn * nx;
    c.st = -sgn * ny;
    c.pad = 0.0;
    const size_t ci = (size_t)si * d.T + (size_t)m * kQ + a;
    ctr[ci] = c;
    center_bessel_table(d.k * R, d.NJ / 2, jtab + ci * d.NJ);
  }
}

// ---------------------------------------------------------------------------
// chain rule to the panel nodes and the node densities: one block per panel.
// Optional node terms (null when absent): gtw[t][2], a gradient with respect to
// the node tangent X'(tau_a) itself, and gde[kk][t] (complex), one added to the
// node density gradients (the split's far sources sit at the nodes).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chain_panel(const Dims& d, int m, const double* __restrict__ nodes,
                                               const double* __restrict__ density,
                                               const double* __restrict__ tab,
                                               const double* __restrict__ sg,
                                               const double* __restrict__ cg,
                                               const double* __restrict__ gtw,
                                               const double* __restrict__ gde,
                                               double* __restrict__ grad_density,
                                               double* __restrict__ grad_nodes) {
  const TableLayout L = table_layout(d.qs);
  const int t = threadIdx.x;
  __shared__ double X[kQ][2];
  __shared__ double2 S[2][kQ];
  __shared__ double red[128];
  __shared__ double gxs[128][2], gts[128][2];      // per source: grad x', grad tangent
  __shared__ double2 gsf[2][128];                   // per source: grad of the fine densities
  __shared__ double gtau[kQ][2], gxt[kQ][2];
  if (t < 2 * kQ) X[t >> 1][t & 1] = nodes[(size_t)m * 2 * kQ + t];
  if (t < d.nk * kQ) {
    const int kk = t / kQ, a = t % kQ;
    const double* src = density + 2 * ((size_t)kk * d.T + (size_t)m * kQ + a);
    S[kk][a] = make_double2(src[0], src[1]);
  }
  __syncthreads();
  // targets: sum the sides, push the normal gradient to the tangent
  double gR = 0.0;
  if (t < kQ) {
    const int a = t;
    double gx = 0.0, gy = 0.0, gnx = 0.0, gny = 0.0;
    for (int si = 0; si < d.n_sides; ++si) {
      const double* c = cg + ((size_t)si * d.T + (size_t)m * kQ + a) * 8;
      gx += c[0];
      gy += c[1];
      gR += c[2];
      gnx += c[3];
      gny += c[4];
    }
    const double* Dr = tab + L.Dn + a * kQ;
    double tx = 0.0, ty = 0.0;
#pragma unroll
    for (int c = 0; c < kQ; ++c) {
      tx = fma(Dr[c], X[c][0], tx);
      ty = fma(Dr[c], X[c][1], ty);
    }
    const double tn = sqrt(tx * tx + ty * ty);
    const double inv = 1.0 / tn;
    const double nx = ty * inv, ny = -tx * inv;
    // n = R90(tau)/|tau|, R90(a) = (a_y, -a_x): dL/dtau = R90^T(g_n)/|tau| - (g_n . n) tau/|tau|^2
    const double gn_n = gnx * nx + gny * ny;
    gtau[a][0] = (-gny - gn_n * tx * inv) * inv;
    gtau[a][1] = (gnx - gn_n * ty * inv) * inv;
    if (gtw) {
      const size_t o = (size_t)m * kQ + a;
      gtau[a][0] += gtw[2 * o];
      gtau[a][1] += gtw[2 * o + 1];
    }
    gxt[a][0] = gx;
    gxt[a][1] = gy;
  }
  red[t] = gR;
  __syncthreads();
  for (int off = 64; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  const double gh = d.r * red[0];   // R = r h_m for every center of the panel
  // sources
  for (int b = t; b < d.qs; b += blockDim.x) {
    const double* Vr = tab + L.V + b * kQ;
    const double* Vdr = tab + L.Vd + b * kQ;
    double dx = 0.0, dy = 0.0, sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
      dx = fma(Vdr[a], X[a][0], dx);
      dy = fma(Vdr[a], X[a][1], dy);
      sr0 = fma(Vr[a], S[0][a].x, sr0);
      si0 = fma(Vr[a], S[0][a].y, si0);
      if (d.nk > 1) {
        sr1 = fma(Vr[a], S[1][a].x, sr1);
        si1 = fma(Vr[a], S[1][a].y, si1);
      }
    }
    const double sp = sqrt(dx * dx + dy * dy);
    const double inv = 1.0 / sp;
    const double om = tab[L.ws + b];
    const double w = om * sp;
    const double* q = sg + ((size_t)m * d.qs + b) * 8;
    // the fine densities: sigma' (first kind) and mu' (second kind, if any)
    double gw = gh;
    const bool hasS = d.kind & 1;
    if (hasS) {
      gw += q[0] * sr0 + q[1] * si0;             // Re(conj(grad(w sigma)) sigma')
      gsf[0][b] = make_double2(w * q[0], w * q[1]);
    }
    if (d.kind & 2) {
      const double mr = hasS ? sr1 : sr0, mi = hasS ? si1 : si0;
      gw += q[2] * mr + q[3] * mi;
      gsf[hasS ? 1 : 0][b] = make_double2(w * q[2], w * q[3]);
    }
    const double nx = dy * inv, ny = -dx * inv;
    const double gn_n = q[6] * nx + q[7] * ny;
    // w = omega |t|,  n = R90(t)/|t|
    gts[b][0] = gw * om * dx * inv + (-q[7] - gn_n * dx * inv) * inv;
    gts[b][1] = gw * om * dy * inv + (q[6] - gn_n * dy * inv) * inv;
    gxs[b][0] = q[4];
    gxs[b][1] = q[5];
  }
  __syncthreads();
  // node gradients: thread (c, dim) sums over the sources and targets
  if (t < 2 * kQ) {
    const int c = t >> 1, dim = t & 1;
    double acc = gxt[c][dim];
    for (int b = 0; b < d.qs; ++b) {
      acc = fma(tab[L.V + b * kQ + c], gxs[b][dim], acc);
      acc = fma(tab[L.Vd + b * kQ + c], gts[b][dim], acc);
    }
    for (int a = 0; a < kQ; ++a) acc = fma(tab[L.Dn + a * kQ + c], gtau[a][dim], acc);
    if (grad_nodes) grad_nodes[(size_t)m * 2 * kQ + t] = acc;
  }
  if (grad_density && t < d.nk * kQ) {
    const int kk = t / kQ, c = t % kQ;
    double ar = 0.0, ai = 0.0;
    for (int b = 0; b < d.qs; ++b) {
      const double v = tab[L.V + b * kQ + c];
      ar = fma(v, gsf[kk][b].x, ar);
      ai = fma(v, gsf[kk][b].y, ai);
    }
    const size_t o = (size_t)kk * d.T + (size_t)m * kQ + c;
    if (gde) {
      ar += gde[2 * o];
      ai += gde[2 * o + 1];
    }
    grad_density[2 * o] = ar;
    grad_density[2 * o + 1] = ai;
  }
}

// ---------------------------------------------------------------------------
// per-element steps of the adjoint (also used by the batched kernels)
// ---------------------------------------------------------------------------
// G_i = conj(g_i) i/4 for element e = kind * Mc + center
__device__ __forceinline__ void make_G_elem(int e, int Mc, int T, int nk, const double* __restrict__ cot,
                                            double2* __restrict__ G) {
  const int kk = e / Mc, ci = e - kk * Mc;
  const int si = ci / T, t = ci - si * T;
  const size_t o = ((size_t)si * nk + kk) * T + t;
  const double gr = cot[2 * o], gi = cot[2 * o + 1];
  G[e] = make_double2(0.25 * gi, 0.25 * gr);   // (i/4)(gr - i gi)
}

// per-center gradients cg[ci] = {g_x, g_y, g_R, g_nx, g_ny} (target position,
// panel-scaled radius R, target normal), before the chain rule, from the
// center-side sums contracted with G: dR = Re G sum q K_R, dt = Re G sum q K_theta,
// (gvx, gvy) = Re G sum q grad_v K
__device__ __forceinline__ void center_grad_from_sums(int ci, int side, int T,
                                                      const CenterRec* __restrict__ ctr,
                                                      double dR, double dt, double gvx,
                                                      double gvy, double* __restrict__ cg) {
  const CenterRec c = ctr[ci];
  const double sgn = side_sign(side, ci / T);
  // target offset direction w^ = (ct, st), theta^_w = (-st, ct)
  const double gwx = dR * c.ct - dt / c.R * c.st;
  const double gwy = dR * c.st + dt / c.R * c.ct;
  const double gcx = -gvx - gwx, gcy = -gvy - gwy;
  const double nx = -sgn * c.ct, ny = -sgn * c.st;   // outward normal at the target
  double* o = cg + (size_t)ci * 8;
  o[0] = -gvx;                          // x moves c along: grad_x = g_w + g_c
  o[1] = -gvy;
  o[2] = sgn * (nx * gcx + ny * gcy);   // c = x + s R n
  o[3] = sgn * c.R * gcx;
  o[4] = sgn * c.R * gcy;
}

// the same from the tape (per center and kind: sum q K_R, K_theta, grad_v K)
__device__ __forceinline__ void center_grad_elem(int ci, int Mc, int nk, int side, int T,
                                                 const CenterRec* __restrict__ ctr,
                                                 const double2* __restrict__ tape,
                                                 const double2* __restrict__ G,
                                                 double* __restrict__ cg) {
  double dR = 0.0, dt = 0.0, gvx = 0.0, gvy = 0.0;
  for (int kk = 0; kk < nk; ++kk) {
    const double2 g = G[(size_t)kk * Mc + ci];
    const double2* tp = tape + ((size_t)ci * nk + kk) * 4;
    // Re(G * a)
    dR += g.x * tp[0].x - g.y * tp[0].y;
    dt += g.x * tp[1].x - g.y * tp[1].y;
    gvx += g.x * tp[2].x - g.y * tp[2].y;
    gvy += g.x * tp[3].x - g.y * tp[3].y;
  }
  center_grad_from_sums(ci, side, T, ctr, dR, dt, gvx, gvy, cg);
}

// per source: sg[j] = {grad(w sigma) re, im, grad(w mu) re, im, g_x', g_y', g_nx, g_ny}
__device__ __forceinline__ void source_finalize_elem(int j, int N, int kind, int n_csplit,
                                                     const double4* __restrict__ geo,
                                                     const double2* __restrict__ partial,
                                                     double* __restrict__ sg) {
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
  double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hasS) {
    o[0] = s[0][0];
    o[1] = s[0][1];
  }
  if (hasD) {
    o[2] = s[nk - 1][0];
    o[3] = s[nk - 1][1];
  }
  o[4] = s[nk][0];
  o[5] = s[nk][1];
  if (hasD) {
    const double rp = s[nk + 1][0];
    const double4 g = geo[j];
    o[6] = rp * g.w;    // Re(w mu Psi) (n_y, -n_x)
    o[7] = -rp * g.z;
  }
  double* q = sg + (size_t)j * 8;
#pragma unroll
  for (int b = 0; b < 8; ++b) q[b] = o[b];
}

}  // namespace qbx
