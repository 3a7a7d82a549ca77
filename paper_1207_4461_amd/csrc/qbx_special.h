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

namespace qbx {

// ---------------------------------------------------------------------------
// Hankel seeds.  The ROCm device math library supplies j0, j1, y0, y1.
// ---------------------------------------------------------------------------
struct H01 {
  double h0r, h0i, h1r, h1i;
};

__device__ __forceinline__ H01 hankel01(double z) {
  H01 h;
  h.h0r = j0(z);
  h.h0i = y0(z);
  h.h1r = j1(z);
  h.h1i = y1(z);
  return h;
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
