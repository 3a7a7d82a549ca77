// Pair-loop bodies shared by the per-contour kernels (qbx_forward.hip,
// qbx_adjoint.hip) and the batched persistent kernels (qbx_batched.hip).
//
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
//   psi = theta_i - arg(nu)   (for p = 0 only the last sum, at m = 1, remains).
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
//
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
// Source side (sum over centers, source-major or fused pass):
//   grad(w sigma)_j = sum_i conj(G_i K_ij),
//   grad x'_j = sum_i Re G_i w_j sigma_j (K_rho v^ + K_theta' theta^ / rho),
//   grad nu_j = sum_i Re G_i w_j mu_j K_psi (n_y, -n_x),
// with the derivative sums projected on G_i w_j sigma_j per pair (pair_sums_proj).
// Center side (sum over sources, center-major tape pass): the forward also
// stores F_R = sum_j w sigma K_R, F_t = sum_j w sigma K_theta and
// GV = sum_j w sigma (K_rho v^ + K_theta' theta^/rho); then with c fixed the
// target gradient is dR w^ + dtheta/R theta^_w, and with x fixed the center
// gradient is -(Re G GV) - (that), which the chain rule through
// c = x + s R n (R = r h_m) carries to the nodes.
#pragma once

#include "qbx_internal.h"
#include "qbx_special.h"

// Unroll factors of the order loops (full unrolling by default).  Full
// unrolling keeps every recurrence in registers with compile-time indices but
// lets the scheduler interleave all orders, which raises the live register set.
#ifndef QBX_FWD_UNROLL
#define QBX_FWD_UNROLL 64
#endif
#ifndef QBX_SUMS_UNROLL
#define QBX_SUMS_UNROLL 64
#endif
#define QBX_PRAGMA(x) _Pragma(#x)
#define QBX_UNROLL_BY(n) QBX_PRAGMA(unroll n)

namespace qbx {

// Empty asm that takes the values as in/out operands: every order's recurrence
// state and running sums must be final at this point, so the compiler cannot
// run whole recurrence chains ahead and keep all orders live at once.
#define QBX_PIN1(a) asm volatile("" : "+v"(a))
#define QBX_PIN2(a, b) asm volatile("" : "+v"(a), "+v"(b))
#define QBX_PIN4(a, b, c, d) asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d))

struct Cplx {
  double r, i;
};

__device__ __forceinline__ void cmac(Cplx& acc, double f, double hr, double hi) {
  acc.r = fma(f, hr, acc.r);
  acc.i = fma(f, hi, acc.i);
}

// per-pair sums of the forward with tape (complex; the cotangent is not known
// yet): K, K_R, K_theta, K_rho, K_theta'
struct PairOut {
  Cplx Ks, KRs, Kts, Krs, Ktps;   // single layer
  Cplx Kd, KRd, Ktd, Krd, Ktpd;   // double layer
};

template <int P, int KIND>
__device__ __forceinline__ PairOut pair_sums(double z, double iz, double cd, double sd, double cps,
                                             double sps, double k, const double* __restrict__ J,
                                             const double* __restrict__ Jd,
                                             const double* __restrict__ cf) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr bool kTape = true;
  constexpr int LMAX = kD ? P + 1 : P;
  const H01 h = hankel01(z, iz, cf);
  double hm_r = h.h0r, hm_i = h.h0i;  // H_{l-1}
  double hc_r = h.h1r, hc_i = h.h1i;  // H_l
  const double tz = 2.0 * iz;
  double tl = tz;
  const double two_cd = 2.0 * cd;
  Cplx sK = {0, 0}, sKR = {0, 0}, sKt = {0, 0}, sKr = {0, 0};
  Cplx dK = {0, 0}, dKR = {0, 0}, dKt = {0, 0}, dKr = {0, 0}, dKtp = {0, 0};
  double c_m = 1.0, c_c = cd, s_m = 0.0, s_c = sd;           // cos, sin of l Delta
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);             // cos(l D + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);              // cos(l D - psi)
  double sa_m = sps, sa_c = fma(sd, cps, cd * sps);            // sin(l D + psi)
  double sb_m = -sps, sb_c = fma(sd, cps, -cd * sps);          // sin(l D - psi)
QBX_UNROLL_BY(QBX_SUMS_UNROLL)
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
      const double fbR = Jd[l - 1] * b_c;
      const double fR = up ? fma(Jd[l + 1], a_c, -fbR) : -fbR;
      cmac(dKR, fR, hc_r, hc_i);
      cmac(dKt, fma((double)(l - 1), sB, -(double)(l + 1) * sA), hc_r, hc_i);
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
    QBX_PIN4(hm_r, hm_i, hc_r, hc_i);
    if (kS) {
      QBX_PIN4(c_m, c_c, s_m, s_c);
      QBX_PIN4(sK.r, sK.i, sKt.r, sKt.i);
      QBX_PIN2(sKr.r, sKr.i);
      if (kTape) QBX_PIN2(sKR.r, sKR.i);
    }
    if (kD) {
      QBX_PIN4(a_m, a_c, b_m, b_c);
      QBX_PIN4(sa_m, sa_c, sb_m, sb_c);
      QBX_PIN4(dK.r, dK.i, dKr.r, dKr.i);
      QBX_PIN2(dKtp.r, dKtp.i);
      QBX_PIN4(dKR.r, dKR.i, dKt.r, dKt.i);
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
    // the m = 0 terms (H_0 J_1 cos psi and its derivatives) exist only when p >= 1
    const double f0 = P >= 1 ? J[1] * cps : 0.0, g0 = P >= 1 ? J[1] * sps : 0.0;
    o.Kd = {k * fma(f0, H0r, dK.r), k * fma(f0, H0i, dK.i)};
    o.Krd = {k * k * fma(-f0, H1r, 0.5 * dKr.r), k * k * fma(-f0, H1i, 0.5 * dKr.i)};
    o.Ktpd = {k * dKtp.r, k * dKtp.i};
    const double fR0 = P >= 1 ? Jd[1] * cps : 0.0;
    o.KRd = {k * k * fma(fR0, H0r, dKR.r), k * k * fma(fR0, H0i, dKR.i)};
    o.Ktd = {k * fma(-g0, H0r, dKt.r), k * fma(-g0, H0i, dKt.i)};
  }
  return o;
}

// ---------------------------------------------------------------------------
// per-pair sums of the target derivatives: K_R = dK/dR and K_theta = dK/dtheta
// at fixed source (the same terms as the tape's, without K, K_rho or grad_v K)
// ---------------------------------------------------------------------------
struct GradOut {
  Cplx KRs, Kts, KRd, Ktd;
};

template <int P, int KIND>
__device__ __forceinline__ GradOut grad_sums(double z, double iz, double cd, double sd, double cps,
                                             double sps, double k, const double* __restrict__ J,
                                             const double* __restrict__ Jd,
                                             const double* __restrict__ lJ,
                                             const double* __restrict__ cf) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int LMAX = kD ? P + 1 : P;
  const H01 h = hankel01(z, iz, cf);
  double hm_r = h.h0r, hm_i = h.h0i;  // H_{l-1}
  double hc_r = h.h1r, hc_i = h.h1i;  // H_l
  const double tz = 2.0 * iz;
  double tl = tz;
  const double two_cd = 2.0 * cd;
  Cplx sKR = {0, 0}, sKt = {0, 0}, dKR = {0, 0}, dKt = {0, 0};
  double c_m = 1.0, c_c = cd, s_m = 0.0, s_c = sd;           // cos, sin of l Delta
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);             // cos(l D + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);              // cos(l D - psi)
  double sa_m = sps, sa_c = fma(sd, cps, cd * sps);            // sin(l D + psi)
  double sb_m = -sps, sb_c = fma(sd, cps, -cd * sps);          // sin(l D - psi)
QBX_UNROLL_BY(QBX_SUMS_UNROLL)
  for (int l = 1; l <= LMAX; ++l) {
    if (kS && l <= P) {
      cmac(sKR, Jd[l] * c_c, hc_r, hc_i);
      cmac(sKt, lJ[l] * s_c, hc_r, hc_i);                     // lJ[l] = l J_l
    }
    if (kD) {
      const bool up = l <= P - 1;
      const double fbR = Jd[l - 1] * b_c;
      cmac(dKR, up ? fma(Jd[l + 1], a_c, -fbR) : -fbR, hc_r, hc_i);
      // (l - 1) J_{l-1} sin(l D - psi) - (l + 1) J_{l+1} sin(l D + psi), the
      // second term only up to l = p - 1
      const double mB = lJ[l - 1] * sb_c;
      cmac(dKt, up ? fma(-lJ[l + 1], sa_c, mB) : mB, hc_r, hc_i);
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
        double t;
        t = fma(two_cd, c_c, -c_m); c_m = c_c; c_c = t;
        t = fma(two_cd, s_c, -s_m); s_m = s_c; s_c = t;
      }
      if (kD) {
        double t;
        t = fma(two_cd, a_c, -a_m); a_m = a_c; a_c = t;
        t = fma(two_cd, b_c, -b_m); b_m = b_c; b_c = t;
        t = fma(two_cd, sa_c, -sa_m); sa_m = sa_c; sa_c = t;
        t = fma(two_cd, sb_c, -sb_m); sb_m = sb_c; sb_c = t;
      }
    }
    QBX_PIN4(hm_r, hm_i, hc_r, hc_i);
    if (kS) {
      QBX_PIN4(c_m, c_c, s_m, s_c);
      QBX_PIN4(sKR.r, sKR.i, sKt.r, sKt.i);
    }
    if (kD) {
      QBX_PIN4(a_m, a_c, b_m, b_c);
      QBX_PIN4(sa_m, sa_c, sb_m, sb_c);
      QBX_PIN4(dKR.r, dKR.i, dKt.r, dKt.i);
    }
  }
  GradOut o;
  const double H0r = h.h0r, H0i = h.h0i;
  if (kS) {
    o.KRs = {k * fma(2.0, sKR.r, Jd[0] * H0r), k * fma(2.0, sKR.i, Jd[0] * H0i)};
    o.Kts = {-2.0 * sKt.r, -2.0 * sKt.i};
  }
  if (kD) {
    // the m = 0 terms exist only when p >= 1
    const double g0 = P >= 1 ? J[1] * sps : 0.0, fR0 = P >= 1 ? Jd[1] * cps : 0.0;
    o.KRd = {k * k * fma(fR0, H0r, dKR.r), k * k * fma(fR0, H0i, dKR.i)};
    o.Ktd = {k * fma(-g0, H0r, dKt.r), k * fma(-g0, H0i, dKt.i)};
  }
  return o;
}

// ---------------------------------------------------------------------------
// per-pair sums of the adjoint once the cotangent is known.  Every gradient
// but the density's uses a derivative sum X only through Re(w X), w = G_i q_j
// (one weight per kind), and Re(w H_l) obeys the Hankel recurrence itself (its
// coefficients are real).  So the derivative sums run over the real sequences
// Re(w_S H_l), Re(w_D H_l) -- one multiply-add per order instead of two -- and
// only K, which the density gradient needs whole, uses the complex H_l.
//   kFused = false (source-major pass): K, Re w K_rho, Re w K_theta', Re w K_psi
//   kFused = true  (fused pass):        also Re w K_R; then K_theta = -K_theta'
//                                       (S) and K_psi - K_theta' (D)
// ---------------------------------------------------------------------------
struct ProjOut {
  Cplx Ks, Kd;
  double rs, ts, Rs;          // S: Re w K_rho, Re w K_theta', Re w K_R
  double rd, td, psid, Rd;    // D: Re w K_rho, Re w K_theta', Re w K_psi, Re w K_R
};

template <int P, int KIND, bool kFused>
__device__ __forceinline__ ProjOut pair_sums_proj(double z, double iz, double cd, double sd,
                                                  double cps, double sps, double k,
                                                  const double* __restrict__ J,
                                                  const double* __restrict__ Jd,
                                                  const double* __restrict__ cf, double2 wS,
                                                  double2 wD) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int LMAX = kD ? P + 1 : P;
  const H01 h = hankel01(z, iz, cf);
  double hm_r = h.h0r, hm_i = h.h0i;  // H_{l-1}
  double hc_r = h.h1r, hc_i = h.h1i;  // H_l
  // Re(w H_0), Re(w H_1) per kind
  const double ps0 = kS ? fma(wS.x, h.h0r, -wS.y * h.h0i) : 0.0;
  const double ps1 = kS ? fma(wS.x, h.h1r, -wS.y * h.h1i) : 0.0;
  const double pd0 = kD ? fma(wD.x, h.h0r, -wD.y * h.h0i) : 0.0;
  const double pd1 = kD ? fma(wD.x, h.h1r, -wD.y * h.h1i) : 0.0;
  double sm = ps0, sc = ps1;          // Re(w_S H_{l-1}), Re(w_S H_l)
  double dm = pd0, dc = pd1;          // Re(w_D H_{l-1}), Re(w_D H_l)
  const double tz = 2.0 * iz;
  double tl = tz;
  const double two_cd = 2.0 * cd;
  Cplx sK = {0, 0}, dK = {0, 0};
  double sKr = 0, sKt = 0, sKR = 0, dKr = 0, dKtp = 0, dKq = 0, dKR = 0;
  double c_m = 1.0, c_c = cd, s_m = 0.0, s_c = sd;           // cos, sin of l Delta
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);             // cos(l D + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);              // cos(l D - psi)
  double sa_m = sps, sa_c = fma(sd, cps, cd * sps);            // sin(l D + psi)
  double sb_m = -sps, sb_c = fma(sd, cps, -cd * sps);          // sin(l D - psi)
QBX_UNROLL_BY(QBX_SUMS_UNROLL)
  for (int l = 1; l <= LMAX; ++l) {
    const double hn_r = fma(tl, hc_r, -hm_r);
    const double hn_i = fma(tl, hc_i, -hm_i);
    const double sn = kS ? fma(tl, sc, -sm) : 0.0;
    const double dn = kD ? fma(tl, dc, -dm) : 0.0;
    if (kS && l <= P) {
      const double f = J[l] * c_c;
      cmac(sK, f, hc_r, hc_i);
      sKr = fma(f, sm - sn, sKr);                    // 2 H_l' = H_{l-1} - H_{l+1}
      sKt = fma((double)l * J[l] * s_c, sc, sKt);
      if (kFused) sKR = fma(Jd[l] * c_c, sc, sKR);
    }
    if (kD) {
      const bool up = l <= P - 1;
      const double fb = J[l - 1] * b_c;
      const double f = up ? fma(J[l + 1], a_c, -fb) : -fb;
      cmac(dK, f, hc_r, hc_i);
      dKr = fma(f, dm - dn, dKr);
      const double sA = up ? J[l + 1] * sa_c : 0.0;
      const double sB = J[l - 1] * sb_c;
      dKtp = fma((double)l * (sA - sB), dc, dKtp);
      dKq = fma(sA + sB, dc, dKq);
      if (kFused) {
        const double fbR = Jd[l - 1] * b_c;
        const double fR = up ? fma(Jd[l + 1], a_c, -fbR) : -fbR;
        dKR = fma(fR, dc, dKR);
      }
    }
    hm_r = hc_r;
    hm_i = hc_i;
    hc_r = hn_r;
    hc_i = hn_i;
    sm = sc;
    sc = sn;
    dm = dc;
    dc = dn;
    tl += tz;
    if (kS) {
      const double cn = fma(two_cd, c_c, -c_m);
      c_m = c_c;
      c_c = cn;
      const double snn = fma(two_cd, s_c, -s_m);
      s_m = s_c;
      s_c = snn;
    }
    if (kD) {
      double t;
      t = fma(two_cd, a_c, -a_m); a_m = a_c; a_c = t;
      t = fma(two_cd, b_c, -b_m); b_m = b_c; b_c = t;
      t = fma(two_cd, sa_c, -sa_m); sa_m = sa_c; sa_c = t;
      t = fma(two_cd, sb_c, -sb_m); sb_m = sb_c; sb_c = t;
    }
    QBX_PIN4(hm_r, hm_i, hc_r, hc_i);
    if (kS) {
      QBX_PIN4(c_m, c_c, s_m, s_c);
      QBX_PIN4(sm, sc, sK.r, sK.i);
      QBX_PIN2(sKr, sKt);
      if (kFused) QBX_PIN1(sKR);
    }
    if (kD) {
      QBX_PIN4(a_m, a_c, b_m, b_c);
      QBX_PIN4(sa_m, sa_c, sb_m, sb_c);
      QBX_PIN4(dm, dc, dK.r, dK.i);
      QBX_PIN2(dKr, dKtp);
      QBX_PIN1(dKq);
      if (kFused) QBX_PIN1(dKR);
    }
  }
  ProjOut o;
  const double H0r = h.h0r, H0i = h.h0i;
  if (kS) {
    o.Ks = {fma(2.0, sK.r, J[0] * H0r), fma(2.0, sK.i, J[0] * H0i)};
    o.rs = k * fma(-J[0], ps1, sKr);
    o.ts = 2.0 * sKt;
    o.Rs = kFused ? k * fma(2.0, sKR, Jd[0] * ps0) : 0.0;
  }
  if (kD) {
    // the m = 0 terms (H_0 J_1 cos psi and its derivatives) exist only when p >= 1
    const double f0 = P >= 1 ? J[1] * cps : 0.0, g0 = P >= 1 ? J[1] * sps : 0.0;
    o.Kd = {k * fma(f0, H0r, dK.r), k * fma(f0, H0i, dK.i)};
    o.rd = k * k * fma(-f0, pd1, 0.5 * dKr);
    o.td = k * dKtp;
    o.psid = k * fma(-g0, pd0, -dKq);
    const double fR0 = P >= 1 ? Jd[1] * cps : 0.0;
    o.Rd = kFused ? k * k * fma(fR0, pd0, dKR) : 0.0;
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
  if (kD && P >= 1) {   // the m = 0 term exists only when p >= 1
    const double f = J[1] * cps;
    dr = f * hm_r;
    di = f * hm_i;
  }
  double c_m = 1.0, c_c = cd;                            // cos((l-1)D), cos(lD)
  double a_m = cps, a_c = fma(cd, cps, -sd * sps);       // cos((l-1)D + psi), cos(lD + psi)
  double b_m = cps, b_c = fma(cd, cps, sd * sps);        // cos((l-1)D - psi), cos(lD - psi)
QBX_UNROLL_BY(QBX_FWD_UNROLL)
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
    QBX_PIN4(hm_r, hm_i, hc_r, hc_i);
    if (kS) {
      QBX_PIN2(c_m, c_c);
      QBX_PIN2(sr, si);
    }
    if (kD) {
      QBX_PIN4(a_m, a_c, b_m, b_c);
      QBX_PIN2(dr, di);
    }
  }
  s_r = fma(2.0, sr, a0r);
  s_i = fma(2.0, si, a0i);
  d_r = dr;
  d_i = di;
}


// ---------------------------------------------------------------------------
// forward, one pair: source j for the center (cx, cy) whose target lies in
// direction (ct, st); adds w sigma K_S and w mu K_D / k to the lane's sums
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void forward_source(const double4* __restrict__ geo,
                                               const double2* __restrict__ dens, int N, int j,
                                               double cx, double cy, double ct, double st,
                                               double k, double inv_k,
                                               const double* __restrict__ Jtab, double& accS_r,
                                               double& accS_i, double& accD_r, double& accD_i) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  // uniform tables re-read (scalar cache) every iteration, see opaque_zero()
  const int z0 = opaque_zero();
  const double* __restrict__ J = Jtab + z0;
  const double* __restrict__ cf = g_seed_table + z0;
  const double4 g = geo[j];
  const double vx = g.x - cx, vy = g.y - cy;
  const double rho2 = fma(vx, vx, vy * vy);
  const double ir = rsqrt_refined(rho2);
  const double rho = rho2 * ir;
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

// ---------------------------------------------------------------------------
// forward: one wave, one center, sources of chunks [c0, c1); returns the sums
// of w sigma K_S and w mu K_D / k reduced over the wave (in every lane)
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void forward_center(const double4* __restrict__ geo,
                                               const double2* __restrict__ dens, int N,
                                               const CenterRec* __restrict__ Crec,
                                               const double* __restrict__ Jtab, double k, int c0,
                                               int c1, int lane, Cplx& S, Cplx& Dd) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  const double cx = Crec->cx, cy = Crec->cy, ct = Crec->ct, st = Crec->st;
  const double inv_k = 1.0 / k;
  double accS_r = 0.0, accS_i = 0.0, accD_r = 0.0, accD_i = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int j = c * kWave + lane;
    if (j < N)
      forward_source<P, KIND>(geo, dens, N, j, cx, cy, ct, st, k, inv_k, Jtab, accS_r, accS_i,
                              accD_r, accD_i);
  }
  S = {accS_r, accS_i};
  Dd = {accD_r, accD_i};
  if (kS) wave_sum(S);
  if (kD) wave_sum(Dd);
}

// ---------------------------------------------------------------------------
// forward with tape, one pair: adds w*density times K, K_R, K_theta and the two
// components of grad_v K of source j for the center (cx, cy) with target
// direction (ct, st) to A[kind][0..4]
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void tape_source(const double4* __restrict__ geo,
                                            const double2* __restrict__ dens, int N, int j,
                                            double cx, double cy, double ct, double st, double k,
                                            double inv_k, const double* __restrict__ Jtab, int nj,
                                            Cplx (&A)[2][5]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  const int z0 = opaque_zero();
  const double* __restrict__ J = Jtab + z0;
  const double* __restrict__ cf = g_seed_table + z0;
  const double4 g = geo[j];
  const double vx = g.x - cx, vy = g.y - cy;
  const double rho2 = fma(vx, vx, vy * vy);
  const double ir = rsqrt_refined(rho2);
  const double rho = rho2 * ir;
  const double ux = vx * ir, uy = vy * ir;          // v^ ; theta^ = (-uy, ux)
  const double cd = ct * ux + st * uy;
  const double sd = st * ux - ct * uy;
  double cps = 0.0, sps = 0.0;
  if (kD) {
    cps = ct * g.z + st * g.w;
    sps = st * g.z - ct * g.w;
  }
  const PairOut o = pair_sums<P, KIND>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J, J + nj, cf);
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

// ---------------------------------------------------------------------------
// forward with tape: one wave, one center, chunks [c0, c1); A[kind][0..4] =
// sums of w*density times K, K_R, K_theta, and the two components of grad_v K,
// reduced over the wave
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void tape_center(const double4* __restrict__ geo,
                                            const double2* __restrict__ dens, int N,
                                            const CenterRec* __restrict__ Crec,
                                            const double* __restrict__ Jtab, int NJ, double k,
                                            int c0, int c1, int lane, Cplx (&A)[2][5]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const double cx = Crec->cx, cy = Crec->cy, ct = Crec->ct, st = Crec->st;
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) A[a][b] = {0.0, 0.0};
  for (int c = c0; c < c1; ++c) {
    const int j = c * kWave + lane;
    if (j < N) tape_source<P, KIND>(geo, dens, N, j, cx, cy, ct, st, k, inv_k, Jtab, nj, A);
  }
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int b = 0; b < 5; ++b) wave_sum(A[kk][b]);
}

// ---------------------------------------------------------------------------
// target derivatives: one wave, one center, chunks [c0, c1); A[kind][0..1] =
// sums of w*density times K_R and K_theta, reduced over the wave
// ---------------------------------------------------------------------------
// target derivatives, one pair: adds q K_R and q K_theta of source j for the
// center (cx, cy) with target direction (ct, st) to A[kind][0..1]
template <int P, int KIND>
__device__ __forceinline__ void grad_source(const double4* __restrict__ geo,
                                            const double2* __restrict__ dens, int N, int j,
                                            double cx, double cy, double ct, double st, double k,
                                            double inv_k, const double* __restrict__ Jtab, int nj,
                                            const double* __restrict__ Ltab, Cplx (&A)[2][2]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int z0 = opaque_zero();
  const double* __restrict__ J = Jtab + z0;
  const double* __restrict__ cf = g_seed_table + z0;
  const double4 g = geo[j];
  const double vx = g.x - cx, vy = g.y - cy;
  const double rho2 = fma(vx, vx, vy * vy);
  const double ir = rsqrt_refined(rho2);
  const double rho = rho2 * ir;
  const double cd = (ct * vx + st * vy) * ir;
  const double sd = (st * vx - ct * vy) * ir;
  double cps = 0.0, sps = 0.0;
  if (kD) {
    cps = ct * g.z + st * g.w;
    sps = st * g.z - ct * g.w;
  }
  const double* __restrict__ lJ = Ltab + z0;
  const GradOut o = grad_sums<P, KIND>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J, J + nj, lJ,
                                       cf);
  if (kS) {
    const double2 w = dens[j];
    cmul_acc(A[0][0], w.x, w.y, o.KRs);
    cmul_acc(A[0][1], w.x, w.y, o.Kts);
  }
  if (kD) {
    const double2 w = dens[(kS ? (size_t)N : 0) + j];
    cmul_acc(A[NK - 1][0], w.x, w.y, o.KRd);
    cmul_acc(A[NK - 1][1], w.x, w.y, o.Ktd);
  }
}

template <int P, int KIND>
__device__ __forceinline__ void grad_center(const double4* __restrict__ geo,
                                            const double2* __restrict__ dens, int N,
                                            const CenterRec* __restrict__ Crec,
                                            const double* __restrict__ Jtab, int NJ,
                                            const double* __restrict__ Ltab, double k,
                                            int c0, int c1, int lane, Cplx (&A)[2][2]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const double cx = Crec->cx, cy = Crec->cy, ct = Crec->ct, st = Crec->st;
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
#pragma unroll
  for (int a = 0; a < 2; ++a) A[a][0] = A[a][1] = {0.0, 0.0};
  for (int c = c0; c < c1; ++c) {
    const int j = c * kWave + lane;
    if (j < N)
      grad_source<P, KIND>(geo, dens, N, j, cx, cy, ct, st, k, inv_k, Jtab, nj, Ltab, A);
  }
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    wave_sum(A[kk][0]);
    wave_sum(A[kk][1]);
  }
}

// ---------------------------------------------------------------------------
// fused adjoint pair: one evaluation of the projected pair sums feeds both the
// source side (accumulated into A, the src_slots layout of the source-major
// pass; for D, K_theta = K_psi - K_theta': the target angle moves Delta and psi,
// the source angle only Delta) and the center side, four reals summed over
// kinds: cres = Re(G q) of K_R, K_theta and the two components of grad_v K.
// q: weighted densities of the source per kind; Gk: G of the center per kind.
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void fused_pair(const double4 g, const double2 (&q)[2], double cx,
                                           double cy, double ct, double st,
                                           const double* __restrict__ J, int nj,
                                           const double* __restrict__ cf, double k, double inv_k,
                                           const double2 (&Gk)[2], Cplx (&A)[src_slots(KIND)],
                                           double (&cres)[4]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = kS && kD ? 2 : 1;
  const double vx = g.x - cx, vy = g.y - cy;
  const double rho2 = fma(vx, vx, vy * vy);
  const double ir = rsqrt_refined(rho2);
  const double rho = rho2 * ir;
  const double ux = vx * ir, uy = vy * ir;
  const double cd = ct * ux + st * uy;
  const double sd = st * ux - ct * uy;
  double cps = 0.0, sps = 0.0;
  if (kD) {
    cps = ct * g.z + st * g.w;
    sps = st * g.z - ct * g.w;
  }
  // w = G q per kind
  const double2 GS = Gk[0], GD = Gk[NK - 1], qS = q[0], qD = q[NK - 1];
  const double2 wS = make_double2(GS.x * qS.x - GS.y * qS.y, GS.x * qS.y + GS.y * qS.x);
  const double2 wD = make_double2(GD.x * qD.x - GD.y * qD.y, GD.x * qD.y + GD.y * qD.x);
  const ProjOut o =
      pair_sums_proj<P, KIND, true>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J, J + nj, cf, wS, wD);
  // grad_v of Re(w K) over both kinds: K_rho v^ + K_theta' theta^ / rho
  double r = 0.0, t = 0.0, cR = 0.0, cT = 0.0;
  if (kS) {
    A[0].r += GS.x * o.Ks.r - GS.y * o.Ks.i;   // conj(G K)
    A[0].i -= GS.x * o.Ks.i + GS.y * o.Ks.r;
    r = o.rs;
    t = o.ts;
    cR = o.Rs;
    cT = -o.ts;                                 // K_theta = -K_theta'
  }
  if (kD) {
    A[NK - 1].r += GD.x * o.Kd.r - GD.y * o.Kd.i;
    A[NK - 1].i -= GD.x * o.Kd.i + GD.y * o.Kd.r;
    r += o.rd;
    t += o.td;
    cR += o.Rd;
    cT += o.psid - o.td;                        // K_theta = K_psi - K_theta'
    A[NK + 1].r += o.psid;
  }
  t *= ir;
  const double ex = fma(r, ux, -t * uy), ey = fma(r, uy, t * ux);
  A[NK].r += ex;
  A[NK].i += ey;
  cres[0] = cR;
  cres[1] = cT;
  cres[2] = ex;
  cres[3] = ey;
}

// ---------------------------------------------------------------------------
// fused adjoint tile: one workgroup of four waves, centers [i0, i0 + nc) x
// 64-source chunks [ch0, ch1) of one contour, taken in sub-blocks of
// fused_centers() centers.  For each sub-block, wave w takes the chunks
// ch0 + w, ch0 + w + 4, ... and runs through the sub-block's centers in the same
// order as the other three, so the center data one wave brings into the scalar
// cache serves the others.  Per pair one evaluation (fused_pair) feeds
//   * the source side (the src_slots layout), accumulated in the lane over the
//     sub-block's centers and added (in sub-block order, by the one wave that
//     owns the chunk) into spart_cb[slots][N], the tile's row;
//   * the center side, four reals summed over the wave (reduce-scatter) and
//     added into this wave's LDS sums of the center, acc[w][c][4]; at the end
//     of the sub-block the four waves' sums are added in wave order and written
//     to cpart_sb[ci][4] (the tile's source block).
// Every sum has a fixed order, so the result is reproducible bit for bit.
// Lanes past the last source take part with zero densities (the wave sums need
// every lane) and write nothing.  acc: LDS, 4 x 4 fused_centers() doubles.
// Starts and ends with a workgroup barrier.
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void fused_tile(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N,
    const CenterRec* __restrict__ ctr, const double* __restrict__ jtab, int NJ,
    const double2* __restrict__ G, int Mc, int i0, int nc, int ch0, int ch1, double k,
    double2* __restrict__ spart_cb, double* __restrict__ cpart_sb, double* acc) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NA = src_slots(KIND);
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  constexpr int kSub = fused_centers(KIND);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double* __restrict__ wacc = acc + (size_t)wave * kSub * 4;
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
  __syncthreads();
  for (int g0 = 0; g0 < nc; g0 += kSub) {
    const int ng = min(kSub, nc - g0);
    for (int t = lane; t < ng * 4; t += kWave) wacc[t] = 0.0;
    for (int ch = ch0 + wave; ch < ch1; ch += 4) {
      const int j = ch * kWave + lane;
      const bool valid = j < N;
      const int jj = valid ? j : N - 1;
      const double4 g = geo[jj];
      double2 q[2];
      q[0] = valid ? dens[jj] : make_double2(0.0, 0.0);
      q[1] = (NK == 2 && valid) ? dens[(size_t)N + jj] : make_double2(0.0, 0.0);
      Cplx A[NA];
#pragma unroll
      for (int b = 0; b < NA; ++b) A[b] = {0.0, 0.0};
      for (int c = 0; c < ng; ++c) {
        const int ci = i0 + g0 + c;
        const int z0 = opaque_zero();
        const CenterRec* __restrict__ C = ctr + ci + z0;
        const double* __restrict__ J = jtab + (size_t)ci * NJ + z0;
        const double* __restrict__ cf = g_seed_table + z0;
        double2 Gk[2];
        Gk[0] = G[(size_t)ci + z0];
        Gk[1] = NK == 2 ? G[(size_t)Mc + ci + z0] : Gk[0];
        double cres[4];
        fused_pair<P, KIND>(g, q, C->cx, C->cy, C->ct, C->st, J, nj, cf, k, inv_k, Gk, A, cres);
        // the four sums over the wave, reduce-scatter: the xor-32 and xor-16
        // exchanges leave in lane L a four-lane partial of sum (L >> 4) & 3, the
        // xor 8..1 butterfly completes it across each group of 16 lanes
        const bool h32 = (lane & 32) != 0, h16 = (lane & 16) != 0;
        const double k0 = h32 ? cres[2] : cres[0], k1 = h32 ? cres[3] : cres[1];
        const double e0 = h32 ? cres[0] : cres[2], e1 = h32 ? cres[1] : cres[3];
        const double p0 = k0 + __shfl_xor(e0, 32), p1 = k1 + __shfl_xor(e1, 32);
        double v = (h16 ? p1 : p0) + __shfl_xor(h16 ? p0 : p1, 16);
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off);
        // lanes 0, 16, 32, 48 add sums 0..3 to this wave's slots of the center
        if ((lane & 15) == 0) wacc[c * 4 + (lane >> 4)] += v;
      }
      // the chunk belongs to this wave: its row gathers the sub-blocks in order
      if (valid) {
#pragma unroll
        for (int b = 0; b < NA; ++b) {
          double2* o = spart_cb + (size_t)b * N + j;
          const double2 prev = g0 == 0 ? make_double2(0.0, 0.0) : *o;
          *o = make_double2(prev.x + A[b].r, prev.y + A[b].i);
        }
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ng * 4; t += blockDim.x) {
      const size_t w4 = (size_t)kSub * 4;
      cpart_sb[(size_t)(i0 + g0) * 4 + t] =
          ((acc[t] + acc[w4 + t]) + acc[2 * w4 + t]) + acc[3 * w4 + t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// adjoint, source side, one pair: source g with weighted densities q against the
// center C (J its Bessel table, GS, GD its cotangent weights per kind); adds to
// A in the src_slots layout
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void adjoint_pair(const double4 g, const double2 (&q)[2],
                                             const CenterRec* __restrict__ C,
                                             const double* __restrict__ J,
                                             const double* __restrict__ cf, double2 GS,
                                             double2 GD, double k, double inv_k, int nj,
                                             Cplx (&A)[src_slots(KIND)]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = kS && kD ? 2 : 1;
  const double cx = C->cx, cy = C->cy, ct = C->ct, st = C->st;
  const double vx = g.x - cx, vy = g.y - cy;
  const double rho2 = fma(vx, vx, vy * vy);
  const double ir = rsqrt_refined(rho2);
  const double rho = rho2 * ir;
  const double ux = vx * ir, uy = vy * ir;
  const double cd = ct * ux + st * uy;
  const double sd = st * ux - ct * uy;
  double cps = 0.0, sps = 0.0;
  if (kD) {
    cps = ct * g.z + st * g.w;
    sps = st * g.z - ct * g.w;
  }
  const double2 qS = q[0], qD = q[NK - 1];
  const double2 wS = make_double2(GS.x * qS.x - GS.y * qS.y, GS.x * qS.y + GS.y * qS.x);
  const double2 wD = make_double2(GD.x * qD.x - GD.y * qD.y, GD.x * qD.y + GD.y * qD.x);
  const ProjOut o = pair_sums_proj<P, KIND, false>(k * rho, ir * inv_k, cd, sd, cps, sps, k, J,
                                                   J + nj, cf, wS, wD);
  double r = 0.0, t = 0.0;
  if (kS) {
    A[0].r += GS.x * o.Ks.r - GS.y * o.Ks.i;   // conj(G K)
    A[0].i -= GS.x * o.Ks.i + GS.y * o.Ks.r;
    r = o.rs;
    t = o.ts;
  }
  if (kD) {
    A[NK - 1].r += GD.x * o.Kd.r - GD.y * o.Kd.i;
    A[NK - 1].i -= GD.x * o.Kd.i + GD.y * o.Kd.r;
    r += o.rd;
    t += o.td;
    A[NK + 1].r += o.psid;
  }
  t *= ir;
  A[NK].r += fma(r, ux, -t * uy);
  A[NK].i += fma(r, uy, t * ux);
}

// ---------------------------------------------------------------------------
// adjoint, source side: one lane, one source g with densities q, centers
// [i0, i1); A in the src_slots layout
// ---------------------------------------------------------------------------
template <int P, int KIND>
__device__ __forceinline__ void adjoint_source(const double4 g, const double2 (&q)[2],
                                               const CenterRec* __restrict__ ctr,
                                               const double* __restrict__ jtab, int NJ,
                                               const double2* __restrict__ G, int Mc, int i0,
                                               int i1, double k, Cplx (&A)[src_slots(KIND)]) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = kS && kD ? 2 : 1;
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
#pragma unroll
  for (int a = 0; a < src_slots(KIND); ++a) A[a] = {0.0, 0.0};
  for (int ci = i0; ci < i1; ++ci) {
    const int z0 = opaque_zero();
    const double2 GS = G[(size_t)ci + z0];
    const double2 GD = NK == 2 ? G[(size_t)Mc + ci + z0] : GS;
    adjoint_pair<P, KIND>(g, q, ctr + ci + z0, jtab + (size_t)ci * NJ + z0, g_seed_table + z0, GS,
                          GD, k, inv_k, nj, A);
  }
}

}  // namespace qbx
