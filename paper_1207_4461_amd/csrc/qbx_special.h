// Device special functions for the QBX pair kernels (gfx950, FP64).
//
//  * hankel01(z): H^(1)_0(z), H^(1)_1(z) for real z > 0, the two seeds of the
//    upward recurrence H_{l+1} = (2l/z) H_l - H_{l-1} (DLMF 10.6.1).
//  * bessel_j_miller(x, L, out): J_0..J_L(x) by Miller's downward recurrence
//    normalized with J_0 + 2 sum_{m>=1} J_{2m} = 1 (DLMF 10.12.4 at t = 0).
//  * gauss_legendre_node(n, i): i-th (ascending) root of P_n and its weight,
//    Newton's method on the three-term Legendre recurrence.
#pragma once

#include <hip/hip_runtime.h>

#include "qbx_seed_coeffs.h"

namespace qbx {

// ---------------------------------------------------------------------------
// Hankel seeds H_0(z), H_1(z), z > 0 (coefficients: qbx_seed_coeffs.h, made by
// gen_seed_coeffs.py from 40-digit reference values and exact rationals).
//  * z >= Z0 = 6: H_nu = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} (P_nu + i Q_nu)
//    with P_nu, Q_nu polynomial in s = (Z0/z)^2 (Q_nu carrying a factor Z0/z);
//    when every active lane of the wavefront has z >= ZM = 10 (a wave-uniform
//    vote, so no lane diverges) shorter fits in s = (ZM/z)^2 serve instead, past
//    ZF = 20 shorter still in s = (ZF/z)^2, past ZV = 60 in s = (ZV/z)^2, and
//    when every lane has z >= ZU = 80 the shortest, in s = (ZU/z)^2;
//    sqrt(2/pi) e^{i(z - pi/4)} = T_n e^{ir} with n = rint(z / delta),
//    delta = 2 pi / 1024, r = z - n delta by a two-part Cody-Waite reduction
//    (|r| <= delta / 2), T_n = sqrt(2/pi) e^{i(n delta - pi/4)} from a 1024-entry
//    table gathered per lane (the amplitude's constant rides in the table), and
//    the degree-2 Taylor polynomials in r^2 of sin r / r and cos r; the phase of
//    H_1 is that of H_0 turned by -pi/2.
//  * z < Z0: Y_nu = (2/pi)(ln(z/2) + gamma) J_nu - nu 2/(pi z) + R_nu with J_nu, R_nu
//    entire (DLMF 10.8.1, 10.8.2): for z < Z1 = 4 their ascending series in
//    w = z^2/4 (DLMF 10.2.2), for Z1 <= z < Z0 polynomial fits in (z - 5).
// Error <~ 2e-15 |H| for every z in (0, 4e5) (the reduction's first part is
// exact for n < 2^26).
// ---------------------------------------------------------------------------
struct H01 {
  double h0r, h0i, h1r, h1i;
};

// 1/sqrt(x) for a normal positive x: the hardware estimate y (relative error
// below 2^-23) refined by one third-order step of the series
// (1 - e)^{-1/2} = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2: y <- y + y e (1/2 + 3e/8);
// the first dropped term, 5e^3/16, is below 2^-66, so the result is within
// about one ulp.  The pair loops use it for 1/rho, rho = x (1/sqrt x) and the
// 1/sqrt(z) of the Hankel asymptotic form, where the correctly rounded sqrt and
// division sequences cost about three times as much.
__device__ __forceinline__ double rsqrt_refined(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

struct D4 {
  double a, b, c, d;
};

// Four interleaved polynomials c[4i + 0..3], i < LEN, at x, accumulated in the
// power basis (x^i shared by the four): each step is one multiply for x^i and one
// fused multiply-add per polynomial with the wave-uniform coefficient as a
// multiplicand, which the hardware takes straight from a scalar register.
// (Horner's rule would save the multiplies, but its coefficient is the addend,
// and the compiler then copies every coefficient into the accumulator
// register first: three instructions a step.)  The polynomials are well
// conditioned on their ranges (decaying coefficients), so the summation order
// costs no accuracy.
template <int LEN>
__host__ __device__ __forceinline__ D4 horner4(const double* __restrict__ c, double x) {
  D4 r = {c[0], c[1], c[2], c[3]};
  double pw = x;
#pragma unroll
  for (int i = 1; i < LEN; ++i) {
    r.a = fma(c[4 * i], pw, r.a);
    r.b = fma(c[4 * i + 1], pw, r.b);
    r.c = fma(c[4 * i + 2], pw, r.c);
    r.d = fma(c[4 * i + 3], pw, r.d);
    if (i + 1 < LEN) pw *= x;
  }
  return r;
}

// horner4 with the four constant terms given (c0), for callers that keep them in
// vector registers across a loop: each polynomial then starts with one fused
// multiply-add instead of two register copies and one
template <int LEN>
__host__ __device__ __forceinline__ D4 horner4_c0(const double* __restrict__ c, double x,
                                                  const D4& c0) {
  D4 r = c0;
  double pw = x;
#pragma unroll
  for (int i = 1; i < LEN; ++i) {
    r.a = fma(c[4 * i], pw, r.a);
    r.b = fma(c[4 * i + 1], pw, r.b);
    r.c = fma(c[4 * i + 2], pw, r.c);
    r.d = fma(c[4 * i + 3], pw, r.d);
    if (i + 1 < LEN) pw *= x;
  }
  return r;
}

// two interleaved polynomials c[2i + 0..1], i < LEN, same scheme, with the
// constant terms a0, b0; the first stops at degree LA - 1 (its higher slots are
// zero padding)
template <int LEN, int LA>
__host__ __device__ __forceinline__ void horner2(const double* __restrict__ c, double x, double a0,
                                                 double b0, double& a, double& b) {
  a = a0;
  b = b0;
  double pw = x;
#pragma unroll
  for (int i = 1; i < LEN; ++i) {
    if (i < LA) a = fma(c[2 * i], pw, a);
    b = fma(c[2 * i + 1], pw, b);
    if (i + 1 < LEN) pw *= x;
  }
}

// Device copies of the seed coefficient table and of the phase table (one per
// translation unit).  The phase table is read with a per-lane index.
static __constant__ double g_seed_table[seed::kTableLen] = {QBX_SEED_TABLE_VALUES};
static __constant__ __align__(16) double g_phase_table[2 * seed::kPhaseN] = {
    QBX_PHASE_TABLE_VALUES};

// H_0, H_1 from the amplitude functions P0, Q0, P1, Q1 of the asymptotic form:
// with E = sqrt(2/(pi z)) e^{i(z - pi/4)}, H_0 = E (P0 + i Q0), H_1 = E (Q1 - i P1).
// n = rint(z / delta) by adding and subtracting 1.5 * 2^52 (the sum's low word is n,
// the table index); r = z - n delta in two parts (the first exact); sin r / r and
// cos r to degree 2 in r^2, their constant terms and cos's -1/2 inline constants.
__device__ __forceinline__ H01 hankel01_asym(double z, double P0, double Q0, double P1, double Q1,
                                             const double* __restrict__ cf) {
  constexpr double kRound = 6755399441055744.0;   // 1.5 * 2^52
  H01 h;
  // e^{i(z - pi/4)} = T_n e^{ir}
  const double tq = fma(z, seed::kInvDelta, kRound);
  const double n = tq - kRound;
  double r = fma(-n, seed::kDeltaHi, z);
  r = fma(-n, seed::kDeltaLo, r);
  const double* __restrict__ T =
      g_phase_table + 2 * (__double2loint(tq) & (seed::kPhaseN - 1));
  const double tc = T[0], ts = T[1];
  const double u = r * r, u2 = u * u;
  double sn = fma(cf[seed::kTRIGOff + 2], u, 1.0);      // 1 - u/6 + u^2/120
  double cs = fma(u, -0.5, 1.0);                        // 1 - u/2 + u^2/24
  sn = fma(cf[seed::kTRIGOff + 4], u2, sn);
  cs = fma(cf[seed::kTRIGOff + 5], u2, cs);
  sn *= r;
  double er = fma(tc, cs, -ts * sn);
  double ei = fma(tc, sn, ts * cs);
  const double A = rsqrt_refined(z);   // sqrt(2/pi) is in T_n
  er *= A;
  ei *= A;
  h.h0r = fma(er, P0, -ei * Q0);     // E (P0 + i Q0)
  h.h0i = fma(er, Q0, ei * P0);
  h.h1r = fma(er, Q1, ei * P1);      // E (Q1 - i P1)
  h.h1i = fma(ei, Q1, -er * P1);
  return h;
}

// H_0(z), H_1(z) for z >= seed::kZV with the z >= kZV fits (degree 4 in
// (kZV/z)^2), no branches: the same values as hankel01's own z >= kZV tier,
// which the direct passes of the near/far split call straight when every lane
// of the wave is that far, without hankel01's per-lane range branches
__device__ __forceinline__ H01 hankel01_vfar(double z, double iz, const double* __restrict__ cf) {
  const double t = seed::kZV * iz;
  const D4 pq = horner4<seed::kVFARLen>(cf + seed::kVFAROff, t * t);
  return hankel01_asym(z, pq.a, t * pq.b, pq.c, t * pq.d, cf);
}

// A copy of a wave-uniform double in a vector register that the compiler cannot
// see through, so that it stays there across a loop: a loop-invariant addend of a
// fused multiply-add (the constant term of a polynomial) is then read in place
// instead of being copied in by two v_mov instructions at every use.
__device__ __forceinline__ double in_vgpr(double s) {
  double v;
  asm volatile("v_mov_b64 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// The constant terms of a fit block (its four interleaved polynomials), held in
// vector registers by loops over many pairs (8 VGPRs)
__device__ __forceinline__ D4 fit_c0(const double* __restrict__ fc) {
  return D4{in_vgpr(fc[0]), in_vgpr(fc[1]), in_vgpr(fc[2]), in_vgpr(fc[3])};
}

// H_0, H_1 from one fit block of LEN terms at fc (a seed::k*Off block of the table
// cf) with t = Zt / z for its threshold Zt, and its constant terms c0
template <int LEN>
__device__ __forceinline__ H01 hankel01_fit_c0(double z, double t, const double* __restrict__ fc,
                                               const D4& c0, const double* __restrict__ cf) {
  const D4 pq = horner4_c0<LEN>(fc, t * t, c0);
  return hankel01_asym(z, pq.a, t * pq.b, pq.c, t * pq.d, cf);
}

// iz = 1/z (callers already hold it); cf = the coefficient table seed::kTable
// (QBX_SEED_TABLE_VALUES), read with wave-uniform loads
__device__ __forceinline__ H01 hankel01(double z, double iz, const double* __restrict__ cf) {
  constexpr double kTwoOverPi = 0.63661977236758134308;
  constexpr double kEuler = 0.57721566490153286061;
  constexpr double kInvTwoPi = 0.15915494309189533577;
  H01 h;
  if (z >= seed::kZ0) {
    double P0, Q0, P1, Q1;
    if (__all(z >= seed::kZU)) {
      const double t = seed::kZU * iz;
      const D4 pq = horner4<seed::kUFARLen>(cf + seed::kUFAROff, t * t);
      P0 = pq.a;
      Q0 = t * pq.b;
      P1 = pq.c;
      Q1 = t * pq.d;
    } else if (__all(z >= seed::kZV)) {
      const double t = seed::kZV * iz;
      const D4 pq = horner4<seed::kVFARLen>(cf + seed::kVFAROff, t * t);
      P0 = pq.a;
      Q0 = t * pq.b;
      P1 = pq.c;
      Q1 = t * pq.d;
    } else if (__all(z >= seed::kZF)) {
      const double t = seed::kZF * iz;
      const D4 pq = horner4<seed::kFARLen>(cf + seed::kFAROff, t * t);
      P0 = pq.a;
      Q0 = t * pq.b;
      P1 = pq.c;
      Q1 = t * pq.d;
    } else if (__all(z >= seed::kZM)) {
      const double t = seed::kZM * iz;
      const D4 pq = horner4<seed::kMEDLen>(cf + seed::kMEDOff, t * t);
      P0 = pq.a;
      Q0 = t * pq.b;
      P1 = pq.c;
      Q1 = t * pq.d;
    } else {
      const double t = seed::kZ0 * iz;
      const D4 pq = horner4<seed::kLARGELen>(cf + seed::kLARGEOff, t * t);
      P0 = pq.a;
      Q0 = t * pq.b;
      P1 = pq.c;
      Q1 = t * pq.d;
    }
    h = hankel01_asym(z, P0, Q0, P1, Q1, cf);
  } else {
    const double L = log(0.5 * z) + kEuler;
    double J0, J1, R0, R1;   // Y0 = (2/pi) L J0 + R0,  Y1 = (2/pi)(L J1 - 1/z) + R1
    if (z >= seed::kZ1) {
      const D4 f = horner4<seed::kMIDLen>(cf + seed::kMIDOff, (z - seed::kZC) * seed::kInvZH);
      J0 = f.a;
      R0 = f.b;
      J1 = f.c;
      R1 = f.d;
    } else {
      const double w = 0.25 * z * z;
      const D4 f = horner4<seed::kSERLen>(cf + seed::kSEROff, w);
      J0 = f.a;
      J1 = 0.5 * z * f.b;
      R0 = kTwoOverPi * f.c;
      R1 = -kInvTwoPi * z * f.d;
    }
    h.h0r = J0;
    h.h0i = fma(kTwoOverPi * L, J0, R0);
    h.h1r = J1;
    h.h1i = fma(kTwoOverPi * L, J1, fma(-kTwoOverPi, iz, R1));
  }
  return h;
}


// An SGPR zero the compiler cannot see through: offsetting a table pointer by it
// inside a loop keeps the (uniform, scalar-cached) table loads in the loop instead
// of hoisting hundreds of constants into registers.
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// ---------------------------------------------------------------------------
// Miller's algorithm for J_0..J_L at x >= 0.
// Downward recurrence J_{l-1} = (2l/x) J_l - J_{l+1} from a start order N far
// above max(L, x), where the ratio J_{N+1}/J_N is negligible; the arbitrary
// scale is fixed by the identity 1 = J_0 + 2 (J_2 + J_4 + ...).
// ---------------------------------------------------------------------------
__host__ __device__ inline int miller_start(double x, int L) {
  double m = x > (double)L ? x : (double)L;
  if (m > 1.0e5) m = 1.0e5;  // bounded work for absurd arguments (k R is O(1..100) in QBX)
  int n = (int)m + 24 + (int)(sqrt(40.0 * (m + 1.0)));
  return n + (n & 1);  // even start order
}

// out[0..L]; L >= 0.  For x == 0: J_0 = 1, others 0.
__host__ __device__ inline void bessel_j_miller(double x, int L, double* out) {
  if (x == 0.0) {
    out[0] = 1.0;
    for (int l = 1; l <= L; ++l) out[l] = 0.0;
    return;
  }
  const int N = miller_start(x, L);
  const double inv2x = 2.0 / x;
  double jp = 0.0;       // J_{l+1} (scaled)
  double jc = 1e-290;    // J_l (scaled), l = N
  double norm = 0.0;     // J_0 + 2*sum even, scaled
  for (int l = N; l >= 1; --l) {
    // store J_l when l <= L
    if (l <= L) out[l] = jc;
    if ((l & 1) == 0) norm += 2.0 * jc;
    double jm = l * inv2x * jc - jp;   // J_{l-1}
    jp = jc;
    jc = jm;
    if (fabs(jc) > 1e250) {            // rescale everything computed so far
      jc *= 1e-250;
      jp *= 1e-250;
      norm *= 1e-250;
      for (int q = l; q <= L; ++q) out[q] *= 1e-250;
    }
  }
  out[0] = jc;
  norm += jc;
  const double s = 1.0 / norm;
  for (int l = 0; l <= L; ++l) out[l] *= s;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1]: node i (ascending) of n, and its weight.
// ---------------------------------------------------------------------------
__host__ __device__ inline void legendre_pair(int n, double x, double* pn, double* dpn) {
  // P_n(x) and P_n'(x) by (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *pn = 1.0;
    *dpn = 0.0;
    return;
  }
  for (int j = 1; j < n; ++j) {
    double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / ((x - 1.0) * (x + 1.0));
}

__host__ __device__ inline void gauss_legendre_node(int n, int i, double* node, double* weight) {
  // the i-th largest root is near cos(pi (i + 3/4) / (n + 1/2)); ascending
  // order reverses the index
  const double kPi = 3.14159265358979323846;
  int ii = n - 1 - i;
  double x = cos(kPi * (ii + 0.75) / (n + 0.5));
  double pn, dpn;
  for (int it = 0; it < 100; ++it) {
    legendre_pair(n, x, &pn, &dpn);
    double dx = pn / dpn;
    x -= dx;
    if (fabs(dx) < 1e-16) break;
  }
  legendre_pair(n, x, &pn, &dpn);
  x -= pn / dpn;
  // weight from 1/w = sum_{j<n} (j + 1/2) P_j(x)^2 (Christoffel-Darboux), a sum of
  // positive terms that keeps full relative accuracy up to the interval ends
  double p0 = 1.0, p1 = x, s = 0.5;
  if (n > 1) s += 1.5 * x * x;
  for (int j = 1; j + 1 < n; ++j) {
    double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
    s += (j + 1.5) * p2 * p2;
  }
  *node = x;
  *weight = 1.0 / s;
}

}  // namespace qbx
