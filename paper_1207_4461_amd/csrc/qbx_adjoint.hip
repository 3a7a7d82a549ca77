// Adjoint of the QBX hot path: forward-with-tape, source-major gradient pass,
// per-center gradients and the chain rule back to the panel nodes.
//
// Notation (per pair): v = x'_j - c_i (rho, theta'), the target offset
// w = x_i - c_i = R e^{i theta}, Delta = theta - theta', psi = theta - arg(nu_j),
// and the pair kernels of the forward (see qbx_forward.hip)
//   K_S = sum_l' 2 H_l(k rho) J_l(k R) cos(l Delta),
//   K_D = k [H_0 J_1 cos psi + sum_{m<p} H_m J_{m+1} cos(m Delta + psi)
//            - sum_{m<=p+1} H_m J_{m-1} cos(m Delta - psi)].
// With G_i = conj(g_i) i/4 the loss is L = Re sum_ij G_i w_j sigma_j K_ij.
//
// Derivatives of the pair kernels (all from the same recurrences):
//   d/drho:    H -> k H',  H'_l = (H_{l-1} - H_{l+1})/2   (DLMF 10.6.1)
//   d/dR:      J -> k J'                                  (DLMF 10.6.1)
//   d/dtheta': cos(l Delta) -> l sin(l Delta), cos(m Delta +- psi) -> m sin(..)
//   d/dtheta:  Delta and psi both move: cos(m Delta +- psi) -> -(m +- 1) sin(..)
//   d/dpsi (D, through the source normal's angle).
// Source side (sum over centers, source-major pass):
//   grad(w sigma)_j = sum_i conj(G_i K_ij),
//   grad x'_j = Re w_j sigma_j sum_i G_i (K_rho v^ + K_theta' theta^ / rho),
//   grad nu_j = Re w_j mu_j sum_i G_i K_psi (n_y, -n_x).
// Center side (sum over sources, center-major tape pass): the forward also
// stores F_R = sum_j w sigma K_R, F_t = sum_j w sigma K_theta and
// GV = sum_j w sigma (K_rho v^ + K_theta' theta^/rho); then with c fixed the
// target gradient is dR w^ + dtheta/R theta^_w, and with x fixed the center
// gradient is -(Re G GV) - (that), which the chain rule through
// c = x + s R n (R = r h_m) carries to the nodes.
#include "qbx_internal.h"
#include "qbx_special.h"

namespace qbx {

struct Cplx {
  double r, i;
};

__device__ __forceinline__ void cmac(Cplx& acc, double f, double hr, double hi) {
  acc.r = fma(f, hr, acc.r);
  acc.i = fma(f, hi, acc.i);
}

// per-pair sums (complex): which ones are formed depends on MODE
//   MODE 0 (tape, center-major): K, K_R, K_theta, K_rho, K_theta'
//   MODE 1 (source-major):       K, K_rho, K_theta', K_psi (D)
struct PairOut {
  Cplx Ks, KRs, Kts, Krs, Ktps;          // single layer
  Cplx Kd, KRd, Ktd, Krd, Ktpd, Kpsid;   // double layer
};

template <int P, int KIND, int MODE>
__device__ __forceinline__ PairOut pair_sums(double z, double iz, double cd, double sd, double cps,
                                             double sps, double k, const double* __restrict__ J,
                                             const double* __restrict__ Jd,
                                             const double* __restrict__ cf) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr bool kTape = MODE == 0;
  constexpr int LMAX = kD ? P + 1 : P;
  const H01 h = hankel01(z, iz, cf);
  double hm_r = h.h0r, hm_i = h.h0i;  // H_{l-1}
  double hc_r = h.h1r, hc_i = h.h1i;  // H_l
  const double tz = 2.0 * iz;
  double tl = tz;
  const double two_cd = 2.0 * cd;
  Cplx sK = {0, 0}, sKR = {0, 0}, sKt = {0, 0}, sKr = {0, 0};
  Cplx dK = {0, 0}, dKR = {0, 0}, dKt = {0, 0}, dKr = {0, 0}, dKtp = {0, 0}, dKpsi = {0, 0};
  double c_m = 1.0, c_c = cd, s_m = 0.0, s_c = sd;           // cos, sin of l Delta
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);             // cos(l D + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);              // cos(l D - psi)
  double sa_m = sps, sa_c = fma(sd, cps, cd * sps);            // sin(l D + psi)
  double sb_m = -sps, sb_c = fma(sd, cps, -cd * sps);          // sin(l D - psi)
#pragma unroll
  for (int l = 1; l <= LMAX; ++l) {
    // H_{l+1} and d_l = H_{l-1} - H_{l+1} = 2 H_l'
    const double hn_r = fma(tl, hc_r, -hm_r);
    const double hn_i = fma(tl, hc_i, -hm_i);
    const double d_r = hm_r - hn_r, d_i = hm_i - hn_i;
    if (kS && l <= P) {
      const double f = J[l] * c_c;
      cmac(sK, f, hc_r, hc_i);
      cmac(sKr, f, d_r, d_i);
      const double g = (double)l * J[l] * s_c;
      cmac(sKt, g, hc_r, hc_i);
      if (kTape) cmac(sKR, Jd[l] * c_c, hc_r, hc_i);
    }
    if (kD) {
      const bool up = l <= P - 1;
      const double fb = J[l - 1] * b_c;
      const double f = up ? fma(J[l + 1], a_c, -fb) : -fb;
      cmac(dK, f, hc_r, hc_i);
      cmac(dKr, f, d_r, d_i);
      const double sA = up ? J[l + 1] * sa_c : 0.0;
      const double sB = J[l - 1] * sb_c;
      cmac(dKtp, (double)l * (sA - sB), hc_r, hc_i);
      if (kTape) {
        const double fbR = Jd[l - 1] * b_c;
        const double fR = up ? fma(Jd[l + 1], a_c, -fbR) : -fbR;
        cmac(dKR, fR, hc_r, hc_i);
        cmac(dKt, fma((double)(l - 1), sB, -(double)(l + 1) * sA), hc_r, hc_i);
      } else {
        cmac(dKpsi, -(sA + sB), hc_r, hc_i);
      }
    }
    hm_r = hc_r;
    hm_i = hc_i;
    hc_r = hn_r;
    hc_i = hn_i;
    tl += tz;
    if (kS) {
      const double cn = fma(two_cd, c_c, -c_m);
      c_m = c_c;
      c_c = cn;
      const double sn = fma(two_cd, s_c, -s_m);
      s_m = s_c;
      s_c = sn;
    }
    if (kD) {
      double t;
      t = fma(two_cd, a_c, -a_m); a_m = a_c; a_c = t;
      t = fma(two_cd, b_c, -b_m); b_m = b_c; b_c = t;
      t = fma(two_cd, sa_c, -sa_m); sa_m = sa_c; sa_c = t;
      t = fma(two_cd, sb_c, -sb_m); sb_m = sb_c; sb_c = t;
    }
  }
  PairOut o;
  const double H0r = h.h0r, H0i = h.h0i, H1r = h.h1r, H1i = h.h1i;
  if (kS) {
    o.Ks = {fma(2.0, sK.r, J[0] * H0r), fma(2.0, sK.i, J[0] * H0i)};
    o.Krs = {k * fma(-J[0], H1r, sKr.r), k * fma(-J[0], H1i, sKr.i)};
    o.Ktps = {2.0 * sKt.r, 2.0 * sKt.i};
    o.Kts = {-2.0 * sKt.r, -2.0 * sKt.i};
    if (kTape) o.KRs = {k * fma(2.0, sKR.r, Jd[0] * H0r), k * fma(2.0, sKR.i, Jd[0] * H0i)};
  }
  if (kD) {
    const double f0 = J[1] * cps, g0 = J[1] * sps;
    o.Kd = {k * fma(f0, H0r, dK.r), k * fma(f0, H0i, dK.i)};
    o.Krd = {k * k * fma(-f0, H1r, 0.5 * dKr.r), k * k * fma(-f0, H1i, 0.5 * dKr.i)};
    o.Ktpd = {k * dKtp.r, k * dKtp.i};
    if (kTape) {
      const double fR0 = Jd[1] * cps;
      o.KRd = {k * k * fma(fR0, H0r, dKR.r), k * k * fma(fR0, H0i, dKR.i)};
      o.Ktd = {k * fma(-g0, H0r, dKt.r), k * fma(-g0, H0i, dKt.i)};
    } else {
      o.Kpsid = {k * fma(-g0, H0r, dKpsi.r), k * fma(-g0, H0i, dKpsi.i)};
    }
  }
  return o;
}

__device__ __forceinline__ void cmul_acc(Cplx& acc, double wr, double wi, Cplx a) {
  // acc += w * a
  acc.r = fma(wr, a.r, fma(-wi, a.i, acc.r));
  acc.i = fma(wr, a.i, fma(wi, a.r, acc.i));
}

__device__ __forceinline__ void wave_sum(Cplx& a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.r += __shfl_xor(a.r, off);
    a.i += __shfl_xor(a.i, off);
  }
}

// ---------------------------------------------------------------------------
// forward with tape (center-major, one wave per center and source split)
// partial layout: [n_split][nk][Mc][5] complex = U, F_R, F_t, GV_x, GV_y
// ---------------------------------------------------------------------------
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_forward_tape(const double4* __restrict__ geo,
                                                      const double2* __restrict__ dens, int N,
                                                      const CenterRec* __restrict__ ctr,
                                                      const double* __restrict__ jtab, int NJ,
                                                      int Mc, int n_split, int chunks,
                                                      int chunks_per_split, double k,
                                                      double2* __restrict__ partial) {
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
  const int nj = NJ / 2;
  Cplx A[2][5];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) A[a][b] = {0.0, 0.0};
  const int c0 = sp * chunks_per_split;
  const int c1 = min(c0 + chunks_per_split, chunks);
  for (int c = c0; c < c1; ++c) {
    const int j = c * kWave + lane;
    if (j < N) {
      const int z0 = opaque_zero();
      const double* __restrict__ J = Jtab + z0;
      const double* __restrict__ cf = g_seed_table + z0;
      const double4 g = geo[j];
      const double vx = g.x - cx, vy = g.y - cy;
      const double rho = sqrt(fma(vx, vx, vy * vy));
      const double ir = 1.0 / rho;
      const double ux = vx * ir, uy = vy * ir;          // v^ ; theta^ = (-uy, ux)
      const double cd = ct * ux + st * uy;
      const double sd = st * ux - ct * uy;
      double cps = 0.0, sps = 0.0;
      if (kD) {
        cps = ct * g.z + st * g.w;
        sps = st * g.z - ct * g.w;
      }
      const PairOut o = pair_sums<P, KIND, 0>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J, J + nj, cf);
      int kk = 0;
      if (kS) {
        const double2 w = dens[j];
        const Cplx ex = {fma(o.Krs.r, ux, -o.Ktps.r * ir * uy), fma(o.Krs.i, ux, -o.Ktps.i * ir * uy)};
        const Cplx ey = {fma(o.Krs.r, uy, o.Ktps.r * ir * ux), fma(o.Krs.i, uy, o.Ktps.i * ir * ux)};
        cmul_acc(A[kk][0], w.x, w.y, o.Ks);
        cmul_acc(A[kk][1], w.x, w.y, o.KRs);
        cmul_acc(A[kk][2], w.x, w.y, o.Kts);
        cmul_acc(A[kk][3], w.x, w.y, ex);
        cmul_acc(A[kk][4], w.x, w.y, ey);
        ++kk;
      }
      if (kD) {
        const double2 w = dens[(kS ? (size_t)N : 0) + j];
        const Cplx ex = {fma(o.Krd.r, ux, -o.Ktpd.r * ir * uy), fma(o.Krd.i, ux, -o.Ktpd.i * ir * uy)};
        const Cplx ey = {fma(o.Krd.r, uy, o.Ktpd.r * ir * ux), fma(o.Krd.i, uy, o.Ktpd.i * ir * ux)};
        cmul_acc(A[kk][0], w.x, w.y, o.Kd);
        cmul_acc(A[kk][1], w.x, w.y, o.KRd);
        cmul_acc(A[kk][2], w.x, w.y, o.Ktd);
        cmul_acc(A[kk][3], w.x, w.y, ex);
        cmul_acc(A[kk][4], w.x, w.y, ey);
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int b = 0; b < 5; ++b) wave_sum(A[kk][b]);
  if (lane == 0) {
#pragma unroll
    for (int kk = 0; kk < NK; ++kk)
#pragma unroll
      for (int b = 0; b < 5; ++b)
        partial[(((size_t)sp * NK + kk) * Mc + ci) * 5 + b] = make_double2(A[kk][b].r, A[kk][b].i);
  }
}

// out = (i/4) sum_splits U;  tape[ci][kk][0..3] = F_R, F_t, GV_x, GV_y
__global__ __launch_bounds__(256) void k_finalize_tape(int Mc, int T, int nk, int n_split,
                                                       const double2* __restrict__ partial,
                                                       double* __restrict__ out,
                                                       double2* __restrict__ tape) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Mc * nk) return;
  const int kk = e / Mc, ci = e - kk * Mc;
  double s[5][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int sp = 0; sp < n_split; ++sp) {
    const double2* q = partial + (((size_t)sp * nk + kk) * Mc + ci) * 5;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      s[b][0] += q[b].x;
      s[b][1] += q[b].y;
    }
  }
  const int si = ci / T, t = ci - si * T;
  if (out) {
    const size_t o = ((size_t)si * nk + kk) * T + t;
    out[2 * o] = -0.25 * s[0][1];
    out[2 * o + 1] = 0.25 * s[0][0];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
    tape[((size_t)ci * nk + kk) * 4 + b] = make_double2(s[b + 1][0], s[b + 1][1]);
}

// ---------------------------------------------------------------------------
// G_i = conj(g_i) i/4 per center and kind: G[kk][ci]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_make_G(int Mc, int T, int nk, const double* __restrict__ cot,
                                                double2* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Mc * nk) return;
  const int kk = e / Mc, ci = e - kk * Mc;
  const int si = ci / T, t = ci - si * T;
  const size_t o = ((size_t)si * nk + kk) * T + t;
  const double gr = cot[2 * o], gi = cot[2 * o + 1];
  G[e] = make_double2(0.25 * gi, 0.25 * gr);   // (i/4)(gr - i gi)
}

// ---------------------------------------------------------------------------
// per-center gradients from the tape: cg[ci] = {g_x, g_y, g_R, g_nx, g_ny}
// (target position, panel-scaled radius R, target normal), before the chain rule
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_center_grads(int Mc, int nk, int side, int T,
                                                      const CenterRec* __restrict__ ctr,
                                                      const double2* __restrict__ tape,
                                                      const double2* __restrict__ G,
                                                      double* __restrict__ cg) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= Mc) return;
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

// ---------------------------------------------------------------------------
// source-major adjoint pass: one wave per (64 sources, center split), loop over
// centers; partial layout [n_csplit][NA][N] complex with
//   S: 0 = sum conj(G K), 1,2 = sum G (K_rho v^ + K_theta' theta^/rho)
//   D: +0 = sum conj(G K), +1,+2 = as above, +3 = sum G K_psi
// ---------------------------------------------------------------------------
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_adjoint_src(const double4* __restrict__ geo, int N,
                                                     const CenterRec* __restrict__ ctr,
                                                     const double* __restrict__ jtab, int NJ,
                                                     const double2* __restrict__ G, int Mc,
                                                     int n_csplit, int centers_per_split,
                                                     int chunks, double k,
                                                     double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NA = (kS ? 3 : 0) + (kD ? 4 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int sb = gw / n_csplit;
  const int cs = gw - sb * n_csplit;
  if (sb >= chunks) return;
  const int j = sb * kWave + lane;
  if (j >= N) return;   // no cross-lane communication below
  const double4 g = geo[j];
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
  Cplx A[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) A[a] = {0.0, 0.0};
  const int i0 = cs * centers_per_split;
  const int i1 = min(i0 + centers_per_split, Mc);
  for (int ci = i0; ci < i1; ++ci) {
    const int z0 = opaque_zero();
    const CenterRec* __restrict__ C = ctr + ci + z0;
    const double* __restrict__ J = jtab + (size_t)ci * NJ + z0;
    const double* __restrict__ cf = g_seed_table + z0;
    const double cx = C->cx, cy = C->cy, ct = C->ct, st = C->st;
    const double vx = g.x - cx, vy = g.y - cy;
    const double rho = sqrt(fma(vx, vx, vy * vy));
    const double ir = 1.0 / rho;
    const double ux = vx * ir, uy = vy * ir;
    const double cd = ct * ux + st * uy;
    const double sd = st * ux - ct * uy;
    double cps = 0.0, sps = 0.0;
    if (kD) {
      cps = ct * g.z + st * g.w;
      sps = st * g.z - ct * g.w;
    }
    const PairOut o = pair_sums<P, KIND, 1>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J, J + nj, cf);
    int a = 0;
    int kk = 0;
    if (kS) {
      const double2 Gs = G[(size_t)ci + z0];
      // conj(G K)
      A[0].r += Gs.x * o.Ks.r - Gs.y * o.Ks.i;
      A[0].i -= Gs.x * o.Ks.i + Gs.y * o.Ks.r;
      const Cplx ex = {fma(o.Krs.r, ux, -o.Ktps.r * ir * uy), fma(o.Krs.i, ux, -o.Ktps.i * ir * uy)};
      const Cplx ey = {fma(o.Krs.r, uy, o.Ktps.r * ir * ux), fma(o.Krs.i, uy, o.Ktps.i * ir * ux)};
      cmul_acc(A[1], Gs.x, Gs.y, ex);
      cmul_acc(A[2], Gs.x, Gs.y, ey);
      a = 3;
      kk = 1;
    }
    if (kD) {
      const double2 Gd = G[(size_t)kk * Mc + ci + z0];
      A[a].r += Gd.x * o.Kd.r - Gd.y * o.Kd.i;
      A[a].i -= Gd.x * o.Kd.i + Gd.y * o.Kd.r;
      const Cplx ex = {fma(o.Krd.r, ux, -o.Ktpd.r * ir * uy), fma(o.Krd.i, ux, -o.Ktpd.i * ir * uy)};
      const Cplx ey = {fma(o.Krd.r, uy, o.Ktpd.r * ir * ux), fma(o.Krd.i, uy, o.Ktpd.i * ir * ux)};
      cmul_acc(A[a + 1], Gd.x, Gd.y, ex);
      cmul_acc(A[a + 2], Gd.x, Gd.y, ey);
      cmul_acc(A[a + 3], Gd.x, Gd.y, o.Kpsid);
    }
  }
#pragma unroll
  for (int b = 0; b < NA; ++b)
    partial[((size_t)cs * NA + b) * N + j] = make_double2(A[b].r, A[b].i);
}

// per source: sg[j] = {grad(w sigma) re, im, grad(w mu) re, im, g_x', g_y', g_nx, g_ny}
__global__ __launch_bounds__(256) void k_source_finalize(int N, int nk, int kind, int n_csplit,
                                                         const double4* __restrict__ geo,
                                                         const double2* __restrict__ dens,
                                                         const double2* __restrict__ partial,
                                                         double* __restrict__ sg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const bool hasS = kind & 1, hasD = kind & 2;
  const int NA = (hasS ? 3 : 0) + (hasD ? 4 : 0);
  double s[7][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int cs = 0; cs < n_csplit; ++cs)
    for (int b = 0; b < NA; ++b) {
      const double2 v = partial[((size_t)cs * NA + b) * N + j];
      s[b][0] += v.x;
      s[b][1] += v.y;
    }
  double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int a = 0, kk = 0;
  if (hasS) {
    const double2 w = dens[j];
    o[0] = s[0][0];
    o[1] = s[0][1];
    o[4] += w.x * s[1][0] - w.y * s[1][1];
    o[5] += w.x * s[2][0] - w.y * s[2][1];
    a = 3;
    kk = 1;
  }
  if (hasD) {
    const double2 w = dens[(size_t)kk * N + j];
    o[2] = s[a][0];
    o[3] = s[a][1];
    o[4] += w.x * s[a + 1][0] - w.y * s[a + 1][1];
    o[5] += w.x * s[a + 2][0] - w.y * s[a + 2][1];
    const double rp = w.x * s[a + 3][0] - w.y * s[a + 3][1];
    const double4 g = geo[j];
    o[6] = rp * g.w;    // Re(w mu Psi) (n_y, -n_x)
    o[7] = -rp * g.z;
  }
  double* q = sg + (size_t)j * 8;
#pragma unroll
  for (int b = 0; b < 8; ++b) q[b] = o[b];
}

// ---------------------------------------------------------------------------
// chain rule to the panel nodes and the node densities: one block per panel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_chain(Dims d, const double* __restrict__ nodes,
                                               const double* __restrict__ density,
                                               const double* __restrict__ tab,
                                               const double* __restrict__ sg,
                                               const double* __restrict__ cg,
                                               double* __restrict__ grad_density,
                                               double* __restrict__ grad_nodes) {
  const TableLayout L = table_layout(d.qs);
  const int m = blockIdx.x;
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
    grad_density[2 * o] = ar;
    grad_density[2 * o + 1] = ai;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int P>
static hipError_t launch_forward_tape_p(const Dims& d, const double4* geo, const double2* dens,
                                        const CenterRec* ctr, const double* jtab,
                                        double2* partial, hipStream_t s) {
  const long waves = (long)d.Mc * d.n_split;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_LAUNCH(KD)                                                                          \
  hipLaunchKernelGGL((k_forward_tape<P, KD>), grid, block, 0, s, geo, dens, d.N, ctr, jtab, d.NJ, \
                     d.Mc, d.n_split, d.chunks, d.chunks_per_split, d.k, partial)
  if (d.kind == 1)
    QBX_LAUNCH(1);
  else if (d.kind == 2)
    QBX_LAUNCH(2);
  else
    QBX_LAUNCH(3);
#undef QBX_LAUNCH
  return hipGetLastError();
}

template <int P>
static hipError_t launch_adjoint_src_p(const Dims& d, const double4* geo, const CenterRec* ctr,
                                       const double* jtab, const double2* G, double2* partial,
                                       hipStream_t s) {
  const long waves = (long)d.chunks * d.n_csplit;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_LAUNCH(KD)                                                                             \
  hipLaunchKernelGGL((k_adjoint_src<P, KD>), grid, block, 0, s, geo, d.N, ctr, jtab, d.NJ, G, d.Mc, \
                     d.n_csplit, d.centers_per_split, d.chunks, d.k, partial)
  if (d.kind == 1)
    QBX_LAUNCH(1);
  else if (d.kind == 2)
    QBX_LAUNCH(2);
  else
    QBX_LAUNCH(3);
#undef QBX_LAUNCH
  return hipGetLastError();
}

#define QBX_P_SWITCH(FN, ...)                                                              \
  switch (d.p) {                                                                           \
    case 0: return FN<0>(__VA_ARGS__);   case 1: return FN<1>(__VA_ARGS__);                \
    case 2: return FN<2>(__VA_ARGS__);   case 3: return FN<3>(__VA_ARGS__);                \
    case 4: return FN<4>(__VA_ARGS__);   case 5: return FN<5>(__VA_ARGS__);                \
    case 6: return FN<6>(__VA_ARGS__);   case 7: return FN<7>(__VA_ARGS__);                \
    case 8: return FN<8>(__VA_ARGS__);   case 9: return FN<9>(__VA_ARGS__);                \
    case 10: return FN<10>(__VA_ARGS__); case 11: return FN<11>(__VA_ARGS__);              \
    case 12: return FN<12>(__VA_ARGS__); case 13: return FN<13>(__VA_ARGS__);              \
    case 14: return FN<14>(__VA_ARGS__); case 15: return FN<15>(__VA_ARGS__);              \
    case 16: return FN<16>(__VA_ARGS__); case 17: return FN<17>(__VA_ARGS__);              \
    case 18: return FN<18>(__VA_ARGS__); case 19: return FN<19>(__VA_ARGS__);              \
    case 20: return FN<20>(__VA_ARGS__); case 21: return FN<21>(__VA_ARGS__);              \
    case 22: return FN<22>(__VA_ARGS__); case 23: return FN<23>(__VA_ARGS__);              \
    case 24: return FN<24>(__VA_ARGS__);                                                   \
    default: return hipErrorInvalidValue;                                                  \
  }

hipError_t launch_forward_tape(const Dims& d, const double4* geo, const double2* dens,
                               const CenterRec* ctr, const double* jtab, double2* partial,
                               hipStream_t s) {
  QBX_P_SWITCH(launch_forward_tape_p, d, geo, dens, ctr, jtab, partial, s)
}

hipError_t launch_adjoint_src(const Dims& d, const double4* geo, const CenterRec* ctr,
                              const double* jtab, const double2* G, double2* partial,
                              hipStream_t s) {
  QBX_P_SWITCH(launch_adjoint_src_p, d, geo, ctr, jtab, G, partial, s)
}

hipError_t launch_finalize_tape(const Dims& d, const double2* partial, double* out, double2* tape,
                                hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_finalize_tape, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk,
                     d.n_split, partial, out, tape);
  return hipGetLastError();
}

hipError_t launch_adjoint_rest(const Dims& d, const double* nodes, const double* density,
                               const double* tables, const double4* geo, const double2* dens,
                               const CenterRec* ctr, const double* jtab, const double* cot,
                               const double2* tape, double2* G, double* cg, double2* spartial,
                               double* sg, double* grad_density, double* grad_nodes,
                               hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_make_G, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk, cot, G);
  hipLaunchKernelGGL(k_center_grads, dim3((d.Mc + 255) / 256), dim3(256), 0, s, d.Mc, d.nk, d.side,
                     d.T, ctr, tape, G, cg);
  timer_begin(1, s);
  hipError_t e = launch_adjoint_src(d, geo, ctr, jtab, G, spartial, s);
  timer_end(1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_source_finalize, dim3((d.N + 255) / 256), dim3(256), 0, s, d.N, d.nk, d.kind,
                     d.n_csplit, geo, dens, spartial, sg);
  hipLaunchKernelGGL(k_chain, dim3(d.P), dim3(128), 0, s, d, nodes, density, tables, sg, cg,
                     grad_density, grad_nodes);
  return hipGetLastError();
}

}  // namespace qbx
