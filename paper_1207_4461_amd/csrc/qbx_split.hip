// Near/far split of the forward (Section 5: QBX only for the panels near a
// target, direct evaluation by the smooth source rule for all others).
//
// Near relation.  Per panel, b_m is the mean of its 16 nodes (added in node
// order, then times 1/16) and rad2_m = max_a |X_{m,a} - b_m|^2.  Source panel m'
// is near target panel m when
//     |b_m - b_m'|^2 < gamma^2 max(rad2_m, rad2_m').
// Every product and sum of the test is rounded on its own (contraction off), so
// the near pass, the far pass and any IEEE double evaluation of the same formula
// take the same decisions.  A panel is always near itself (gamma > 0).
//
// Near pass (k_split_near): one wave per center, as the plain forward, but the
// wave first tests 64 source panels at a time against its target's panel and
// runs the QBX pair kernel (forward_source) over the sources of the near ones
// only.  Far pass (k_split_far): the 64 lanes are 64 consecutive targets and the
// sources of a run of panels are wave-uniform (scalar loads); a far pair adds
//     S: w sigma H_0(k rho),    D: w mu k H_1(k rho) (x - x').n' / rho,
// rho = |x - x'|, the normal derivative of H_0(k|x - x'|) at the source (the
// seeds from the shortest fits when every lane of the wave has k rho >= 60).  These
// sums do not depend on the side, so both sides share one far pass.  The
// finalize adds, per center, the near sum and the far sums of its target in a
// fixed order and applies i/4.
#include <type_traits>

#include "qbx_pair.h"
#include "qbx_panel.h"

namespace qbx {

__device__ __forceinline__ bool panels_near(double4 a, double4 b, double g2) {
#pragma clang fp contract(off)
  const double dx = a.x - b.x;
  const double dy = a.y - b.y;
  const double d2 = dx * dx + dy * dy;
  return d2 < g2 * fmax(a.z, b.z);
}

// Near lists: one wave per panel m scans all panels (64 per ballot) and writes
// the near ones in ascending order, at most kNearCap of them, and their count.
__global__ __launch_bounds__(256) void k_near_lists(int NP, const double4* __restrict__ bnd,
                                                    double g2, int* __restrict__ count,
                                                    int* __restrict__ list) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + wave;
  if (m >= NP) return;
  const double4 bm = bnd[m];
  int n = 0;
  for (int w0 = 0; w0 < NP; w0 += kWave) {
    const int mp = w0 + lane;
    const bool nr = mp < NP && panels_near(bm, bnd[mp], g2);
    const unsigned long long mask = __ballot(nr);
    const int pos = n + __popcll(mask & ((1ULL << lane) - 1ULL));
    if (nr && pos < kNearCap) list[(size_t)m * kNearCap + pos] = mp;
    n += __popcll(mask);
  }
  if (lane == 0) count[m] = n;
}

// f(pan) for every panel near panel m (wave-uniform), in ascending order: from
// m's list when it fits, else by the wave's scan of all NP panels
template <typename F>
__device__ __forceinline__ void for_near_panels(int m, const double4* __restrict__ bnd, int NP,
                                                double g2, NearLists nl, int lane, F&& f) {
  const int cnt = nl.count[m];
  if (cnt <= kNearCap) {
    const int* __restrict__ L = nl.list + (size_t)m * kNearCap;
    for (int i = 0; i < cnt; ++i) f(L[i]);
    return;
  }
  const double4 bm = bnd[m];
  for (int w0 = 0; w0 < NP; w0 += kWave) {
    const int mp = w0 + lane;
    const bool nr = mp < NP && panels_near(bm, bnd[mp], g2);
    unsigned long long mask = __ballot(nr);
    while (mask) {
      const int pan = w0 + __builtin_ctzll(mask);
      mask &= mask - 1;
      f(pan);
    }
  }
}

// f(m) once for every panel m near any of the panels pa..pb (a 64-source chunk's
// panels; the relation is symmetric): from their lists, each m at the first list
// that holds it, when every list fits; else by the wave's scan (ascending)
template <typename F>
__device__ __forceinline__ void for_near_any(int pa, int pb, const double4* __restrict__ bnd,
                                             int NP, double g2, NearLists nl, int lane, F&& f) {
  bool fits = true;
  for (int ps = pa; ps <= pb; ++ps) fits = fits && nl.count[ps] <= kNearCap;
  if (fits) {
    for (int ps = pa; ps <= pb; ++ps) {
      const int* __restrict__ L = nl.list + (size_t)ps * kNearCap;
      const int cnt = nl.count[ps];
      for (int i = 0; i < cnt; ++i) {
        const int m = L[i];
        bool seen = false;
        for (int pq = pa; pq < ps; ++pq) seen = seen || panels_near(bnd[m], bnd[pq], g2);
        if (!seen) f(m);
      }
    }
    return;
  }
  for (int w0 = 0; w0 < NP; w0 += kWave) {
    const int mt = w0 + lane;
    bool any = false;
    if (mt < NP) {
      const double4 bt = bnd[mt];
      for (int ps = pa; ps <= pb; ++ps) any = any || panels_near(bt, bnd[ps], g2);
    }
    unsigned long long mask = __ballot(any);
    while (mask) {
      const int m = w0 + __builtin_ctzll(mask);
      mask &= mask - 1;
      f(m);
    }
  }
}

// bnd[m] = {b_x, b_y, rad2, 0}
__global__ __launch_bounds__(256) void k_panel_bounds(int NP, const double* __restrict__ nodes,
                                                      double4* __restrict__ bnd) {
#pragma clang fp contract(off)
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= NP) return;
  const double* X = nodes + (size_t)m * 2 * kQ;
  double sx = X[0], sy = X[1];
  for (int a = 1; a < kQ; ++a) {
    sx = sx + X[2 * a];
    sy = sy + X[2 * a + 1];
  }
  const double bx = sx * 0.0625, by = sy * 0.0625;
  double r2 = 0.0;
  for (int a = 0; a < kQ; ++a) {
    const double dx = X[2 * a] - bx;
    const double dy = X[2 * a + 1] - by;
    r2 = fmax(r2, dx * dx + dy * dy);
  }
  // .w: the node radius, which bounds |x - x'| from below for a whole panel of
  // the far sources (the panel's nodes) at once
  bnd[m] = make_double4(bx, by, r2, sqrt(r2));
}

// The Nystrom grid as the far sources (one thread per node t = 16 m + a): the node
// itself, the outward normal n = (y', -x')/|X'| from the 16-node derivative (the
// table's Dn rows, as for the centers), the 16-point Gauss-Legendre weight
// w = omega_a |X'(tau_a)| (the table's w16) and the weighted node densities w sigma.
__global__ __launch_bounds__(256) void k_nystrom_sources(int T, int nk,
                                                         const double* __restrict__ nodes,
                                                         const double* __restrict__ density,
                                                         const double* __restrict__ Dn,
                                                         const double* __restrict__ w16,
                                                         double4* __restrict__ ngeo,
                                                         double2* __restrict__ ndens,
                                                         double* __restrict__ nw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int m = t / kQ, a = t - m * kQ;
  const double* X = nodes + (size_t)m * 2 * kQ;
  const double* Dr = Dn + a * kQ;
  double tx = 0.0, ty = 0.0;
  for (int c = 0; c < kQ; ++c) {
    tx = fma(Dr[c], X[2 * c], tx);
    ty = fma(Dr[c], X[2 * c + 1], ty);
  }
  const double sp = sqrt(tx * tx + ty * ty);
  const double inv = 1.0 / sp;
  const double w = w16[a] * sp;
  ngeo[t] = make_double4(X[2 * a], X[2 * a + 1], ty * inv, -tx * inv);
  nw[t] = w;
  for (int kk = 0; kk < nk; ++kk) {
    const double* sg = density + 2 * ((size_t)kk * T + t);
    ndens[(size_t)kk * T + t] = make_double2(w * sg[0], w * sg[1]);
  }
}

// partial[kk][ci]: QBX sums of center ci over the sources of near panels
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_split_near(const double4* __restrict__ geo,
                                                    const double2* __restrict__ dens, int N,
                                                    int qs, const CenterRec* __restrict__ ctr,
                                                    const double* __restrict__ jtab, int NJ,
                                                    int Mc, int T, const double4* __restrict__ bnd,
                                                    int NP, double g2, NearLists nl, double k,
                                                    double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ci = blockIdx.x * 4 + wave;
  if (ci >= Mc) return;
  const int m = (ci % T) / kQ;                 // the target's panel
  const CenterRec* C = ctr + ci;
  const double cx = C->cx, cy = C->cy, ct = C->ct, st = C->st;
  const double inv_k = 1.0 / k;
  const double* Jtab = jtab + (size_t)ci * NJ;
  double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
  for_near_panels(m, bnd, NP, g2, nl, lane, [&](int pan) {
    for (int s0 = 0; s0 < qs; s0 += kWave) {
      if (s0 + lane < qs)
        forward_source<P, KIND>(geo, dens, N, pan * qs + s0 + lane, cx, cy, ct, st, k, inv_k,
                                Jtab, sr, si, dr, di);
    }
  });
  Cplx S = {sr, si}, Dd = {dr, di};
  if (kS) wave_sum(S);
  if (kD) wave_sum(Dd);
  if (lane == 0) {
    int kk = 0;
    if (kS) partial[(size_t)(kk++) * Mc + ci] = make_double2(S.r, S.i);
    if (kD) partial[(size_t)kk * Mc + ci] = make_double2(k * Dd.r, k * Dd.i);
  }
}

// one far pair: w sigma H_0 (S) and w mu H_1 (x - x').n' / rho (D; the factor k is
// applied once per sum), with the pair's weighted densities wS (S) and wD (D)
template <bool kS, bool kD>
__device__ __forceinline__ void far_accumulate_q(const double2& wS, const double2& wD,
                                                 const double4& g, double dx, double dy,
                                                 double ir, const H01& h, double& sr, double& si,
                                                 double& dr, double& di) {
  if (kS) {
    sr = fma(wS.x, h.h0r, fma(-wS.y, h.h0i, sr));
    si = fma(wS.x, h.h0i, fma(wS.y, h.h0r, si));
  }
  if (kD) {
    const double f = fma(dx, g.z, dy * g.w) * ir;   // (x - x').n' / rho
    const double wr = wD.x * f, wi = wD.y * f;
    dr = fma(wr, h.h1r, fma(-wi, h.h1i, dr));
    di = fma(wr, h.h1i, fma(wi, h.h1r, di));
  }
}

// partial[sp][kk][t]: direct sums of target t over the far sources of panels
// sp, sp + n_fsplit, sp + 2 n_fsplit, ... (interleaved, so that the costly
// panels next to each target's near zone spread over all splits); wave
// gw = sp * n_tb + tb covers targets tb*64 ..
// Per (wave, far panel) a vote: is every active lane at least zt / k from every
// far source of the panel, its nodes (the distance to the panel's mean less its
// node radius bnd.w, with a relative margin for rounding), for the seed fits' thresholds
// zt = 80, 60, 20 in turn?  The first that holds (75%, 9% and 11% of the pairs at
// 4096 panels) gives the panel's pairs that fit with no per-pair vote: the
// coefficient block is addressed once per panel, so its loads stay in scalar
// registers through the panel's loop, and its constant terms are copied into
// vector registers once per panel.  Otherwise (5%) each pair votes as in
// hankel01.  (Panel votes for the z >= 10 and z >= 6 fits as well cost 20 more
// vector registers, one wave a SIMD fewer and 3% of the time; staging the source
// panels in LDS instead of reading them by scalar loads was measured 4% slower.)
template <int KIND>
__global__ __launch_bounds__(256) void k_split_far(const double4* __restrict__ geo,
                                                   const double2* __restrict__ dens, int N,
                                                   const double* __restrict__ nodes, int T,
                                                   const double4* __restrict__ bnd, int NP,
                                                   double g2, double k, int n_tb, int n_fsplit,
                                                   double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int sp = gw / n_tb;
  const int tb = gw - sp * n_tb;
  if (sp >= n_fsplit) return;
  const int t = tb * kWave + lane;
  const bool valid = t < T;
  const int tt = valid ? t : T - 1;
  const double tx = nodes[2 * (size_t)tt], ty = nodes[2 * (size_t)tt + 1];
  const double4 bt = bnd[tt / kQ];
  const double inv_k = 1.0 / k;
  const double zv = seed::kZV * (1.0 + 1e-12), zu = seed::kZU * (1.0 + 1e-12);
  const double zf = seed::kZF * (1.0 + 1e-12);
  const double2* __restrict__ densD = dens + (kS ? (size_t)N : 0);
  double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
  // the pairs of one far panel with one fit block: LEN terms at offset OFF, for z
  // past zt (t = zt / z = (zt / k) / rho)
  auto panel_fit = [&](auto len, auto off, double zt, int j0) {
    constexpr int LEN = decltype(len)::value;
    const double* __restrict__ cf = g_seed_table + opaque_zero();
    const double* __restrict__ fc = cf + decltype(off)::value;
    const D4 c0 = fit_c0(fc);
    const double kt = zt * inv_k;
    for (int b = 0; b < kQ; ++b) {
      const int j = j0 + b;
      const double4 g = geo[j];
      const double dx = tx - g.x, dy = ty - g.y;
      const double rho2 = fma(dx, dx, dy * dy);
      const double ir = rsqrt_refined(rho2);
      const double z = k * (rho2 * ir);
      const H01 h = hankel01_fit_c0<LEN>(z, kt * ir, fc, c0, cf);
      far_accumulate_q<kS, kD>(dens[j], densD[j], g, dx, dy, ir, h, sr, si, dr, di);
    }
  };
  for (int pm = sp; pm < NP; pm += n_fsplit) {
    const double4 bp = bnd[pm];
    const bool far = valid && !panels_near(bt, bp, g2);
    if (far) {
      const int j0 = pm * kQ;
      const double ex = tx - bp.x, ey = ty - bp.y;
      const double e2 = fma(ex, ex, ey * ey);
      const double lo = e2 * rsqrt_refined(e2) - bp.w;
      if (__all(k * lo >= zu)) {
        panel_fit(std::integral_constant<int, seed::kUFARLen>{},
                  std::integral_constant<int, seed::kUFAROff>{}, seed::kZU, j0);
      } else if (__all(k * lo >= zv)) {
        panel_fit(std::integral_constant<int, seed::kVFARLen>{},
                  std::integral_constant<int, seed::kVFAROff>{}, seed::kZV, j0);
      } else if (__all(k * lo >= zf)) {
        panel_fit(std::integral_constant<int, seed::kFARLen>{},
                  std::integral_constant<int, seed::kFAROff>{}, seed::kZF, j0);
      } else {
        for (int b = 0; b < kQ; ++b) {
          const int z0 = opaque_zero();
          const double* __restrict__ cf = g_seed_table + z0;
          const int j = j0 + b;
          const double4 g = geo[j];
          const double dx = tx - g.x, dy = ty - g.y;
          const double rho2 = fma(dx, dx, dy * dy);
          const double ir = rsqrt_refined(rho2);
          const double z = k * (rho2 * ir), iz = ir * inv_k;
          const H01 h = __all(z >= seed::kZV) ? hankel01_vfar(z, iz, cf) : hankel01(z, iz, cf);
          far_accumulate_q<kS, kD>(dens[j], densD[j], g, dx, dy, ir, h, sr, si, dr, di);
        }
      }
    }
  }
  if (valid) {
    int kk = 0;
    if (kS) partial[((size_t)sp * NK + kk++) * T + t] = make_double2(sr, si);
    if (kD) partial[((size_t)sp * NK + kk) * T + t] = make_double2(k * dr, k * di);
  }
}

// out[si][kk][t] = (i/4) (near[kk][ci] + sum over far splits of far[sp][kk][t])
__global__ __launch_bounds__(256) void k_split_finalize(int Mc, int T, int nk, int n_fsplit,
                                                        const double2* __restrict__ nearp,
                                                        const double2* __restrict__ farp,
                                                        double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Mc * nk) return;
  const int kk = e / Mc, ci = e - kk * Mc;
  const int si = ci / T, t = ci - si * T;
  const double2 v0 = nearp[(size_t)kk * Mc + ci];
  double r = v0.x, im = v0.y;
  for (int sp = 0; sp < n_fsplit; ++sp) {
    const double2 v = farp[((size_t)sp * nk + kk) * T + t];
    r += v.x;
    im += v.y;
  }
  const size_t o = ((size_t)si * nk + kk) * T + t;
  out[2 * o] = -0.25 * im;
  out[2 * o + 1] = 0.25 * r;
}

// ---------------------------------------------------------------------------
// Adjoint of the split with respect to the density.  With G_i = conj(g_i) i/4
// (per kind and center) the gradient of L = Re <g, u> with respect to q_j =
// w_j sigma_j is conj(sum_i G_i K_ij), K the pair kernel of whichever rule
// (QBX or direct) the pair takes; the density gradient is then the transposed
// interpolation of w_j conj(...) (PyTorch's convention, A^H g).
// ---------------------------------------------------------------------------

// acc[kk][j] = sum over the centers i of target panels near j's panel of G_i K_ij
// (QBX pairs).  One wave per 64-source chunk: the wave scans the target panels
// near any of its chunk's source panels, and each lane adds the centers of a
// scanned panel only when that panel is near its own source panel.
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_split_near_adj(
    const double4* __restrict__ geo, int N, int qs, const CenterRec* __restrict__ ctr,
    const double* __restrict__ jtab, int NJ, int Mc, int T, int n_sides,
    const double4* __restrict__ bnd, int NP, double g2, NearLists nl, double k,
    const double2* __restrict__ G, double2* __restrict__ acc) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave;
  if (c * kWave >= N) return;
  const int j = c * kWave + lane;
  const bool valid = j < N;
  const int jj = valid ? j : N - 1;
  const double4 bj = bnd[jj / qs];
  const int pa = (c * kWave) / qs;
  const int pb = min(c * kWave + kWave - 1, N - 1) / qs;
  const double4 g = geo[jj];
  const double inv_k = 1.0 / k;
  double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
  for_near_any(pa, pb, bnd, NP, g2, nl, lane, [&](int m) {
    if (valid && panels_near(bnd[m], bj, g2)) {
      for (int si_ = 0; si_ < n_sides; ++si_) {
        for (int a = 0; a < kQ; ++a) {
          const int ci = si_ * T + m * kQ + a;
          const int z0 = opaque_zero();
          const double* __restrict__ J = jtab + (size_t)ci * NJ + z0;
          const double* __restrict__ cf = g_seed_table + z0;
          const CenterRec* C = ctr + ci;
          const double vx = g.x - C->cx, vy = g.y - C->cy;
          const double rho2 = fma(vx, vx, vy * vy);
          const double ir = rsqrt_refined(rho2);
          const double rho = rho2 * ir;
          const double cd = (C->ct * vx + C->st * vy) * ir;
          const double sd = (C->st * vx - C->ct * vy) * ir;
          double cps = 0.0, sps = 0.0;
          if (kD) {
            cps = C->ct * g.z + C->st * g.w;
            sps = C->st * g.z - C->ct * g.w;
          }
          double ks_r, ks_i, kd_r, kd_i;
          pair_kernel<P, KIND>(k * rho, ir * inv_k, cd, sd, cps, sps, J, cf, ks_r, ks_i, kd_r,
                               kd_i);
          int kk = 0;
          if (kS) {
            const double2 Gi = G[(size_t)(kk++) * Mc + ci];
            sr = fma(Gi.x, ks_r, fma(-Gi.y, ks_i, sr));
            si = fma(Gi.x, ks_i, fma(Gi.y, ks_r, si));
          }
          if (kD) {
            const double2 Gi = G[(size_t)kk * Mc + ci];
            dr = fma(Gi.x, kd_r, fma(-Gi.y, kd_i, dr));
            di = fma(Gi.x, kd_i, fma(Gi.y, kd_r, di));
          }
        }
      }
    }
  });
  if (valid) {
    int kk = 0;
    if (kS) acc[(size_t)(kk++) * N + j] = make_double2(sr, si);
    if (kD) acc[(size_t)kk * N + j] = make_double2(k * dr, k * di);
  }
}

// Gf[kk][t] = sum over the sides of G[kk][si T + t]: the far sums do not depend on
// the side, so their transpose takes the two sides' cotangents together
__global__ __launch_bounds__(256) void k_split_gfar(int T, int nk, int n_sides,
                                                   const double2* __restrict__ G,
                                                   double2* __restrict__ Gf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * nk) return;
  const int kk = e / T, t = e - kk * T;
  const size_t Mc = (size_t)n_sides * T;
  double2 v = G[kk * Mc + t];
  if (n_sides == 2) {
    const double2 w = G[kk * Mc + T + t];
    v = make_double2(v.x + w.x, v.y + w.y);
  }
  Gf[e] = v;
}

// partial[sp][kk][j]: sum over the targets t of far panels in split sp (panels
// sp, sp + n_asplit, ...) of Gf_t K_far(t, j); lanes are 64 consecutive sources,
// targets wave-uniform
// The vote of k_split_far per (wave, target panel); here the targets are the
// panel's nodes, so its node radius bounds them.
// GEO adds the far pairs' gradients for the source's position and normal,
// contracted with its weighted densities q (slots NK and NK + 1 of the split's
// NK + 2): with u = (x - x')/rho, f = u.n' and H_0' = -H_1 (DLMF 10.6.2),
//   d/dx' H_0(k rho) = k H_1 u,
//   d/dx' [k H_1 f] = -k [k H_0 f u + (H_1/rho)(n' - 2 f u)],   d/dn' [k H_1 f] = k H_1 u,
// each summed as Re(q G_t .) over the split's targets.
template <int KIND, bool GEO>
__global__ __launch_bounds__(256) void k_split_far_adj(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N,
    const double* __restrict__ nodes, int T, const double4* __restrict__ bnd, int NP, double g2,
    double k, const double2* __restrict__ Gf, int n_sb, int n_asplit,
    double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  constexpr int NS = NK + (GEO ? 2 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int sp = gw / n_sb;
  const int sb = gw - sp * n_sb;
  if (sp >= n_asplit) return;
  const int j = sb * kWave + lane;
  const bool valid = j < N;
  const int jj = valid ? j : N - 1;
  const double4 g = geo[jj];
  const double4 bj = bnd[jj / kQ];
  const double inv_k = 1.0 / k;
  const double zv = seed::kZV * (1.0 + 1e-12), zu = seed::kZU * (1.0 + 1e-12);
  const double zf = seed::kZF * (1.0 + 1e-12);
  double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
  double2 qS = make_double2(0.0, 0.0), qD = qS;
  if (GEO) {
    qS = dens[jj];
    qD = dens[(size_t)(NK - 1) * N + jj];
  }
  double gxp = 0.0, gyp = 0.0, gnx = 0.0, gny = 0.0;   // GEO: without the factor k
  // one far pair: the cotangent weights of target t times H_0 (S) and
  // H_1 (x - x').n' / rho (D)
  auto add = [&](int t, double dx, double dy, double ir, const H01& h) {
    int kk = 0;
    if (kS) {
      const double2 Gt = Gf[(size_t)(kk++) * T + t];
      sr = fma(Gt.x, h.h0r, fma(-Gt.y, h.h0i, sr));
      si = fma(Gt.x, h.h0i, fma(Gt.y, h.h0r, si));
      if (GEO) {
        const double cr = qS.x * Gt.x - qS.y * Gt.y, cim = qS.x * Gt.y + qS.y * Gt.x;
        const double a1 = cr * h.h1r - cim * h.h1i;   // Re(q G H_1)
        gxp = fma(a1 * ir, dx, gxp);
        gyp = fma(a1 * ir, dy, gyp);
      }
    }
    if (kD) {
      const double2 Gt = Gf[(size_t)kk * T + t];
      const double f = fma(dx, g.z, dy * g.w) * ir;   // (x - x').n' / rho
      const double wr = Gt.x * f, wi = Gt.y * f;
      dr = fma(wr, h.h1r, fma(-wi, h.h1i, dr));
      di = fma(wr, h.h1i, fma(wi, h.h1r, di));
      if (GEO) {
        const double cr = qD.x * Gt.x - qD.y * Gt.y, cim = qD.x * Gt.y + qD.y * Gt.x;
        const double a0 = cr * h.h0r - cim * h.h0i;   // Re(q G H_0)
        const double a1 = cr * h.h1r - cim * h.h1i;   // Re(q G H_1)
        const double ux = dx * ir, uy = dy * ir;
        const double b = (k * a0 - 2.0 * a1 * ir) * f;
        gxp -= fma(b, ux, a1 * ir * g.z);
        gyp -= fma(b, uy, a1 * ir * g.w);
        gnx = fma(a1, ux, gnx);
        gny = fma(a1, uy, gny);
      }
    }
  };
  for (int mt = sp; mt < NP; mt += n_asplit) {
    const double4 bt = bnd[mt];
    const bool far = valid && !panels_near(bt, bj, g2);
    if (far) {
      // every pair of the active lanes with this target panel at z >= kZV: the
      // distance to the panel's mean less its node radius (the targets are the
      // nodes) bounds |x - x'| from below
      const double ex = g.x - bt.x, ey = g.y - bt.y;
      const double e2 = fma(ex, ex, ey * ey);
      const double lo = e2 * rsqrt_refined(e2) - bt.w;
      // the pairs of this target panel with one fit block (as in k_split_far)
      auto panel_fit = [&](auto len, auto off, double zt) {
        constexpr int LEN = decltype(len)::value;
        const double* __restrict__ cf = g_seed_table + opaque_zero();
        const double* __restrict__ fc = cf + decltype(off)::value;
        const D4 c0 = fit_c0(fc);
        const double kt = zt * inv_k;
        for (int a = 0; a < kQ; ++a) {
          const int t = mt * kQ + a;
          const double dx = nodes[2 * (size_t)t] - g.x, dy = nodes[2 * (size_t)t + 1] - g.y;
          const double rho2 = fma(dx, dx, dy * dy);
          const double ir = rsqrt_refined(rho2);
          const double z = k * (rho2 * ir);
          add(t, dx, dy, ir, hankel01_fit_c0<LEN>(z, kt * ir, fc, c0, cf));
        }
      };
      if (__all(k * lo >= zu)) {
        panel_fit(std::integral_constant<int, seed::kUFARLen>{},
                  std::integral_constant<int, seed::kUFAROff>{}, seed::kZU);
      } else if (__all(k * lo >= zv)) {
        panel_fit(std::integral_constant<int, seed::kVFARLen>{},
                  std::integral_constant<int, seed::kVFAROff>{}, seed::kZV);
      } else if (__all(k * lo >= zf)) {
        panel_fit(std::integral_constant<int, seed::kFARLen>{},
                  std::integral_constant<int, seed::kFAROff>{}, seed::kZF);
      } else {
        for (int a = 0; a < kQ; ++a) {
          const int t = mt * kQ + a;
          const int z0 = opaque_zero();
          const double* __restrict__ cf = g_seed_table + z0;
          const double dx = nodes[2 * (size_t)t] - g.x, dy = nodes[2 * (size_t)t + 1] - g.y;
          const double rho2 = fma(dx, dx, dy * dy);
          const double ir = rsqrt_refined(rho2);
          const double z = k * (rho2 * ir), iz = ir * inv_k;
          add(t, dx, dy, ir,
              __all(z >= seed::kZV) ? hankel01_vfar(z, iz, cf) : hankel01(z, iz, cf));
        }
      }
    }
  }
  if (valid) {
    int kk = 0;
    if (kS) partial[((size_t)sp * NS + kk++) * N + j] = make_double2(sr, si);
    if (kD) partial[((size_t)sp * NS + kk) * N + j] = make_double2(k * dr, k * di);
    if (GEO) {
      partial[((size_t)sp * NS + NK) * N + j] = make_double2(k * gxp, k * gyp);
      partial[((size_t)sp * NS + NK + 1) * N + j] = make_double2(k * gnx, k * gny);
    }
  }
}

// grad_density[kk][t] = sum_b V[b][a] w_j conj(acc[kk][j]) (j = m qs + b, the
// near sources of panel m) + w_t conj(sum_sp partial[sp][kk][t]) (the far source
// at node t = 16 m + a, weight w_t): one thread per node and kind
__global__ __launch_bounds__(256) void k_split_density_grad(
    int T, int N, int qs, int nk, int n_asplit, const double* __restrict__ tab,
    const double* __restrict__ wgt, const double* __restrict__ nw,
    const double2* __restrict__ acc, const double2* __restrict__ partial,
    double* __restrict__ grad_density) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * nk) return;
  const TableLayout L = table_layout(qs);
  const int kk = e / T, t = e - kk * T;
  const int m = t / kQ, a = t - m * kQ;
  double gr = 0.0, gi = 0.0;
  for (int b = 0; b < qs; ++b) {
    const size_t j = (size_t)m * qs + b;
    const double2 v = acc[(size_t)kk * N + j];
    const double c = tab[L.V + b * kQ + a] * wgt[j];
    gr = fma(c, v.x, gr);
    gi = fma(-c, v.y, gi);      // conj
  }
  double fr = 0.0, fi = 0.0;
  for (int sp = 0; sp < n_asplit; ++sp) {
    const double2 q = partial[((size_t)sp * nk + kk) * T + t];
    fr += q.x;
    fi += q.y;
  }
  const double w = nw[t];
  grad_density[2 * (size_t)e] = fma(w, fr, gr);
  grad_density[2 * (size_t)e + 1] = fma(-w, fi, gi);
}

template <int P>
static hipError_t launch_split_near_adj_p(const Dims& d, const double4* geo, const CenterRec* ctr,
                                          const double* jtab, const double4* bnd, double g2,
                                          NearLists nl, const double2* G, double2* acc,
                                          hipStream_t s) {
  const int chunks = (d.N + kWave - 1) / kWave;
  const dim3 grid((unsigned)((chunks + 3) / 4)), block(256);
#define QBX_NADJ_ARGS \
  geo, d.N, d.qs, ctr, jtab, d.NJ, d.Mc, d.T, d.n_sides, bnd, d.P, g2, nl, d.k, G, acc
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_near_adj<P, 1>), grid, block, 0, s, QBX_NADJ_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_near_adj<P, 2>), grid, block, 0, s, QBX_NADJ_ARGS); break;
    default: hipLaunchKernelGGL((k_split_near_adj<P, 3>), grid, block, 0, s, QBX_NADJ_ARGS); break;
  }
#undef QBX_NADJ_ARGS
  return hipGetLastError();
}

hipError_t launch_split_adjoint_density(const Dims& d, const double* nodes, const double* tables,
                                        const double4* geo, const double* wgt, NystromSources ns,
                                        const CenterRec* ctr, const double* jtab,
                                        const double4* bnd, double g2, NearLists nl,
                                        const double2* G, double2* Gf, double2* acc,
                                        double2* partial, double* grad_density, hipStream_t s) {
  hipError_t e;
  {
    auto launch = [&]() -> hipError_t {
      QBX_P_SWITCH(d.p, launch_split_near_adj_p, d, geo, ctr, jtab, bnd, g2, nl, G, acc, s)
    };
    e = launch();
    if (e != hipSuccess) return e;
  }
  const int nt = d.T * d.nk;
  hipLaunchKernelGGL(k_split_gfar, dim3((nt + 255) / 256), dim3(256), 0, s, d.T, d.nk, d.n_sides,
                     G, Gf);
  const int n_sb = (d.T + kWave - 1) / kWave;
  const long waves = (long)n_sb * d.n_asplit;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_FADJ_ARGS                                                                       \
  ns.geo, nullptr, d.T, nodes, d.T, bnd, d.P, g2, d.k, Gf, n_sb, d.n_asplit,             \
      partial
  timer_begin(8, s);
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_far_adj<1, false>), grid, block, 0, s, QBX_FADJ_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_far_adj<2, false>), grid, block, 0, s, QBX_FADJ_ARGS); break;
    default: hipLaunchKernelGGL((k_split_far_adj<3, false>), grid, block, 0, s, QBX_FADJ_ARGS); break;
  }
  timer_end(8, s);
#undef QBX_FADJ_ARGS
  hipLaunchKernelGGL(k_split_density_grad, dim3((nt + 255) / 256), dim3(256), 0, s, d.T, d.N, d.qs,
                     d.nk, d.n_asplit, tables, wgt, ns.w, acc, partial, grad_density);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Node gradient of the split.  The loss L = Re sum_i conj(g_i) u_i is a sum over
// pairs, each taken by one rule, so its gradient is the plain adjoint's per-pair
// terms over the near pairs plus the direct rule's over the far ones:
//  * center side, near pairs (k_split_near_cg): the tape sums of the near sources
//    (K_R, K_theta, grad_v K; tape_source) contracted with G_i, then the per-center
//    gradients of center_grad_from_sums (target, radius, normal);
//  * source side, near pairs (k_split_near_adj_nodes): the plain adjoint's pair
//    body (adjoint_pair) over the centers of near target panels;
//  * far pairs, source side: k_split_far_adj<KIND, true> over the far sources
//    (the nodes); target side: the far target gradients of the split's
//    derivative pass (k_split_far_grad); k_split_nystrom_grad puts both on the
//    nodes (position, normal, the weight's tangent term, the density);
//  * k_split_source_finalize puts the near source terms into the per-source
//    layout of the plain adjoint, and the plain chain rule (chain_panel) maps
//    everything to the nodes and node densities.
// ---------------------------------------------------------------------------

// cg[ci]: center_grad_from_sums of the near sources' tape sums, contracted with G
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_split_near_cg(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N, int qs,
    const CenterRec* __restrict__ ctr, const double* __restrict__ jtab, int NJ, int Mc, int T,
    int side, const double4* __restrict__ bnd, int NP, double g2, NearLists nl, double k,
    const double2* __restrict__ G, double* __restrict__ cg) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ci = blockIdx.x * 4 + wave;
  if (ci >= Mc) return;
  const int m = (ci % T) / kQ;
  const CenterRec* C = ctr + ci;
  const double cx = C->cx, cy = C->cy, ct = C->ct, st = C->st;
  const double inv_k = 1.0 / k;
  const double* Jtab = jtab + (size_t)ci * NJ;
  Cplx A[2][5];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) A[a][b] = {0.0, 0.0};
  for_near_panels(m, bnd, NP, g2, nl, lane, [&](int pan) {
    for (int s0 = 0; s0 < qs; s0 += kWave) {
      if (s0 + lane < qs)
        tape_source<P, KIND>(geo, dens, N, pan * qs + s0 + lane, cx, cy, ct, st, k, inv_k, Jtab,
                             NJ / 2, A);
    }
  });
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int b = 1; b < 5; ++b) wave_sum(A[kk][b]);
  if (lane == 0) {
    double dR = 0.0, dt = 0.0, gvx = 0.0, gvy = 0.0;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      const double2 g = G[(size_t)kk * Mc + ci];
      dR += g.x * A[kk][1].r - g.y * A[kk][1].i;   // Re(G a)
      dt += g.x * A[kk][2].r - g.y * A[kk][2].i;
      gvx += g.x * A[kk][3].r - g.y * A[kk][3].i;
      gvy += g.x * A[kk][4].r - g.y * A[kk][4].i;
    }
    center_grad_from_sums(ci, side, T, ctr, dR, dt, gvx, gvy, cg);
  }
}

// The far pairs' terms of the node gradient, per node t = 16 m + a (added to
// the first side's center slot t, which the chain rule sums with the other's):
//  * target side: Re(Gf_t . far target gradient) over kinds and far splits, into
//    cg[t][0..1];
//  * source side (the far source at node t), from the far splits' sums of
//    k_split_far_adj<KIND, true>: F_kk (density), the position gradient into
//    cg[t][0..1] and the normal gradient into cg[t][3..4] (the far source's normal
//    is the node's own, as the center's); its weight w = omega_a |X'| enters through
//    g_w = sum_kk Re(F_kk sigma_kk), gtw[t] = g_w omega_a X'/|X'| with X'/|X'| =
//    (-n_y, n_x); gde[kk][t] = w conj(F_kk) joins the node density gradient.
__global__ __launch_bounds__(256) void k_split_nystrom_grad(
    int T, int nk, int n_fsplit, int n_asplit, const double* __restrict__ density,
    const double4* __restrict__ ngeo, const double* __restrict__ nw,
    const double* __restrict__ w16, const double2* __restrict__ Gf,
    const double2* __restrict__ fpart, const double2* __restrict__ apart,
    double* __restrict__ cg, double* __restrict__ gtw, double2* __restrict__ gde) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int ns = nk + 2;
  const double w = nw[t];
  double gx = 0.0, gy = 0.0, gnx = 0.0, gny = 0.0, gw = 0.0;
  for (int kk = 0; kk < nk; ++kk) {
    double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
    for (int sp = 0; sp < n_fsplit; ++sp) {
      const double2* q = fpart + (((size_t)sp * nk + kk) * T + t) * 2;
      xr += q[0].x;
      xi += q[0].y;
      yr += q[1].x;
      yi += q[1].y;
    }
    const double2 g = Gf[(size_t)kk * T + t];
    gx += g.x * xr - g.y * xi;
    gy += g.x * yr - g.y * yi;
    double fr = 0.0, fi = 0.0;
    for (int sp = 0; sp < n_asplit; ++sp) {
      const double2 v = apart[((size_t)sp * ns + kk) * T + t];
      fr += v.x;
      fi += v.y;
    }
    const double* sg = density + 2 * ((size_t)kk * T + t);
    gw += fr * sg[0] - fi * sg[1];   // Re(F sigma)
    gde[(size_t)kk * T + t] = make_double2(w * fr, -w * fi);
  }
  for (int sp = 0; sp < n_asplit; ++sp) {
    const double2 x = apart[((size_t)sp * ns + nk) * T + t];
    const double2 n = apart[((size_t)sp * ns + nk + 1) * T + t];
    gx += x.x;
    gy += x.y;
    gnx += n.x;
    gny += n.y;
  }
  double* c = cg + (size_t)t * 8;
  c[0] += gx;
  c[1] += gy;
  c[3] += gnx;
  c[4] += gny;
  const double4 g = ngeo[t];
  const double om = w16[t % kQ];
  gtw[2 * (size_t)t] = -gw * om * g.w;
  gtw[2 * (size_t)t + 1] = gw * om * g.z;
}

// part[b][j], b < src_slots(KIND): the plain adjoint's source-side sums over the
// centers of the target panels near j's panel (the scan of k_split_near_adj)
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_split_near_adj_nodes(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N, int qs,
    const CenterRec* __restrict__ ctr, const double* __restrict__ jtab, int NJ, int Mc, int T,
    int n_sides, const double4* __restrict__ bnd, int NP, double g2, NearLists nl, double k,
    const double2* __restrict__ G, double2* __restrict__ part) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = kS && kD ? 2 : 1;
  constexpr int NA = src_slots(KIND);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave;
  if (c * kWave >= N) return;
  const int j = c * kWave + lane;
  const bool valid = j < N;
  const int jj = valid ? j : N - 1;
  const double4 bj = bnd[jj / qs];
  const int pa = (c * kWave) / qs;
  const int pb = min(c * kWave + kWave - 1, N - 1) / qs;
  const double4 g = geo[jj];
  double2 q[2];
  q[0] = dens[jj];
  q[1] = dens[(size_t)(NK - 1) * N + jj];
  const double inv_k = 1.0 / k;
  const int nj = NJ / 2;
  Cplx A[NA];
#pragma unroll
  for (int b = 0; b < NA; ++b) A[b] = {0.0, 0.0};
  for_near_any(pa, pb, bnd, NP, g2, nl, lane, [&](int m) {
    if (valid && panels_near(bnd[m], bj, g2)) {
      for (int si_ = 0; si_ < n_sides; ++si_) {
        for (int a = 0; a < kQ; ++a) {
          const int ci = si_ * T + m * kQ + a;
          const int z0 = opaque_zero();
          const double2 GS = G[(size_t)ci + z0];
          const double2 GD = NK == 2 ? G[(size_t)Mc + ci + z0] : GS;
          adjoint_pair<P, KIND>(g, q, ctr + ci + z0, jtab + (size_t)ci * NJ + z0,
                                g_seed_table + z0, GS, GD, k, inv_k, nj, A);
        }
      }
    }
  });
  if (valid) {
#pragma unroll
    for (int b = 0; b < NA; ++b) part[(size_t)b * N + j] = make_double2(A[b].r, A[b].i);
  }
}

// sg[j] (the per-source layout of source_finalize_elem) from the near slots:
// density gradients conj(near), source position, normal psi-projection (the far
// pairs' source terms sit on the far sources, the nodes: k_split_nystrom_grad)
__global__ __launch_bounds__(256) void k_split_source_finalize(int N, int kind,
                                                               const double4* __restrict__ geo,
                                                               const double2* __restrict__ nearp,
                                                               double* __restrict__ sg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const bool hasS = kind & 1, hasD = kind & 2;
  const int nk = hasS && hasD ? 2 : 1;
  double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hasS) {
    const double2 a = nearp[j];
    o[0] = a.x;
    o[1] = a.y;
  }
  if (hasD) {
    const double2 a = nearp[(size_t)(nk - 1) * N + j];
    o[2] = a.x;
    o[3] = a.y;
  }
  const double2 x = nearp[(size_t)nk * N + j];
  o[4] = x.x;
  o[5] = x.y;
  if (hasD) {
    const double rp = nearp[(size_t)(nk + 1) * N + j].x;
    const double4 g = geo[j];
    o[6] = rp * g.w;   // Re(w mu Psi) (n_y, -n_x)
    o[7] = -rp * g.z;
  }
  double* q = sg + (size_t)j * 8;
#pragma unroll
  for (int b = 0; b < 8; ++b) q[b] = o[b];
}

// ---------------------------------------------------------------------------
// Target derivatives with the split (Section 3.2 for the near sources' local
// expansion, the chain rule for the direct ones).  Near: per center the sums
// F_R = sum q dK/dR and F_theta = sum q dK/dtheta over the near sources
// (grad_source); far: per target
//   S: grad H_0(k rho) = -k H_1 u,   D: grad [k H_1 f] = k [k H_0 f u + (H_1/rho)(n' - 2 f u)],
// u = (x - x')/rho, f = u . n'; the finalize combines them as grad u = (i/4)
// (F_R w^ + (F_theta/R) theta^ + far) and n . grad u with n = -s w^.
// ---------------------------------------------------------------------------

// partial[kk][ci][0..1] = F_R, F_theta over the near sources of center ci
template <int P, int KIND>
__global__ __launch_bounds__(256) void k_split_near_grad(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N, int qs,
    const CenterRec* __restrict__ ctr, const double* __restrict__ jtab, int NJ, int Mc, int T,
    const double4* __restrict__ bnd, int NP, double g2, NearLists nl, double k,
    double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ci = blockIdx.x * 4 + wave;
  if (ci >= Mc) return;
  const int m = (ci % T) / kQ;
  const CenterRec* C = ctr + ci;
  const double cx = C->cx, cy = C->cy, ct = C->ct, st = C->st;
  const double inv_k = 1.0 / k;
  const double* Jtab = jtab + (size_t)ci * NJ;
  const double* Ltab = jtab + (size_t)Mc * NJ + (size_t)ci * (NJ / 2);   // l J_l
  Cplx A[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) A[a][0] = A[a][1] = {0.0, 0.0};
  for_near_panels(m, bnd, NP, g2, nl, lane, [&](int pan) {
    for (int s0 = 0; s0 < qs; s0 += kWave) {
      if (s0 + lane < qs)
        grad_source<P, KIND>(geo, dens, N, pan * qs + s0 + lane, cx, cy, ct, st, k, inv_k, Jtab,
                             NJ / 2, Ltab, A);
    }
  });
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    wave_sum(A[kk][0]);
    wave_sum(A[kk][1]);
  }
  if (lane == 0) {
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      double2* q = partial + ((size_t)kk * Mc + ci) * 2;
      q[0] = make_double2(A[kk][0].r, A[kk][0].i);
      q[1] = make_double2(A[kk][1].r, A[kk][1].i);
    }
  }
}

// partial[sp][kk][t][0..1]: the direct gradient (x, y) of target t over the far
// sources of panels sp, sp + n_fsplit, ..., without the factors -k (S), k (D)
template <int KIND>
__global__ __launch_bounds__(256) void k_split_far_grad(
    const double4* __restrict__ geo, const double2* __restrict__ dens, int N,
    const double* __restrict__ nodes, int T, const double4* __restrict__ bnd, int NP, double g2,
    double k, int n_tb, int n_fsplit, double2* __restrict__ partial) {
  constexpr bool kS = (KIND & 1) != 0;
  constexpr bool kD = (KIND & 2) != 0;
  constexpr int NK = (kS ? 1 : 0) + (kD ? 1 : 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + wave;
  const int sp = gw / n_tb;
  const int tb = gw - sp * n_tb;
  if (sp >= n_fsplit) return;
  const int t = tb * kWave + lane;
  const bool valid = t < T;
  const int tt = valid ? t : T - 1;
  const double tx = nodes[2 * (size_t)tt], ty = nodes[2 * (size_t)tt + 1];
  const double4 bt = bnd[tt / kQ];
  const double inv_k = 1.0 / k;
  double sxr = 0.0, sxi = 0.0, syr = 0.0, syi = 0.0;
  double dxr = 0.0, dxi = 0.0, dyr = 0.0, dyi = 0.0;
  for (int pm = sp; pm < NP; pm += n_fsplit) {
    const bool far = valid && !panels_near(bt, bnd[pm], g2);
    if (far) {
      const int j0 = pm * kQ;
      for (int b = 0; b < kQ; ++b) {
        const int z0 = opaque_zero();
        const double* __restrict__ cf = g_seed_table + z0;
        const int j = j0 + b;
        const double4 g = geo[j];
        const double dx = tx - g.x, dy = ty - g.y;
        const double rho2 = fma(dx, dx, dy * dy);
        const double ir = rsqrt_refined(rho2);
        const double z = k * (rho2 * ir), iz = ir * inv_k;
        const H01 h = __all(z >= seed::kZV) ? hankel01_vfar(z, iz, cf) : hankel01(z, iz, cf);
        const double ux = dx * ir, uy = dy * ir;
        if (kS) {
          const double2 w = dens[j];
          const double hr = fma(w.x, h.h1r, -w.y * h.h1i), hi = fma(w.x, h.h1i, w.y * h.h1r);
          sxr = fma(hr, ux, sxr);
          sxi = fma(hi, ux, sxi);
          syr = fma(hr, uy, syr);
          syi = fma(hi, uy, syi);
        }
        if (kD) {
          const double2 w = dens[(kS ? (size_t)N : 0) + j];
          const double f = fma(ux, g.z, uy * g.w);
          // k H_0 f u + (H_1 / rho)(n' - 2 f u), times w mu
          const double a_r = k * f * h.h0r, a_i = k * f * h.h0i;
          const double b_r = h.h1r * ir, b_i = h.h1i * ir;
          const double vx = fma(-2.0 * f, ux, g.z), vy = fma(-2.0 * f, uy, g.w);
          const double cxr = fma(a_r, ux, b_r * vx), cxi = fma(a_i, ux, b_i * vx);
          const double cyr = fma(a_r, uy, b_r * vy), cyi = fma(a_i, uy, b_i * vy);
          dxr = fma(w.x, cxr, fma(-w.y, cxi, dxr));
          dxi = fma(w.x, cxi, fma(w.y, cxr, dxi));
          dyr = fma(w.x, cyr, fma(-w.y, cyi, dyr));
          dyi = fma(w.x, cyi, fma(w.y, cyr, dyi));
        }
      }
    }
  }
  if (valid) {
    int kk = 0;
    if (kS) {
      double2* q = partial + (((size_t)sp * NK + kk++) * T + t) * 2;
      q[0] = make_double2(-k * sxr, -k * sxi);
      q[1] = make_double2(-k * syr, -k * syi);
    }
    if (kD) {
      double2* q = partial + (((size_t)sp * NK + kk) * T + t) * 2;
      q[0] = make_double2(k * dxr, k * dxi);
      q[1] = make_double2(k * dyr, k * dyi);
    }
  }
}

// grad[si][kk][t][0..1] and dn[si][kk][t] from the near sums of center ci and the
// far sums of its target
__global__ __launch_bounds__(256) void k_split_finalize_gradient(
    int Mc, int T, int nk, int n_fsplit, int side, const CenterRec* __restrict__ ctr,
    const double2* __restrict__ nearp, const double2* __restrict__ farp, double* __restrict__ grad,
    double* __restrict__ dn) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Mc * nk) return;
  const int kk = e / Mc, ci = e - kk * Mc;
  const int si = ci / T, t = ci - si * T;
  const double2 F = nearp[((size_t)kk * Mc + ci) * 2], Ft = nearp[((size_t)kk * Mc + ci) * 2 + 1];
  const CenterRec c = ctr[ci];
  const double ir = 1.0 / c.R;
  // F_R w^ + (F_theta / R) theta^, theta^ = (-sin, cos)
  double gxr = fma(F.x, c.ct, -Ft.x * ir * c.st), gxi = fma(F.y, c.ct, -Ft.y * ir * c.st);
  double gyr = fma(F.x, c.st, Ft.x * ir * c.ct), gyi = fma(F.y, c.st, Ft.y * ir * c.ct);
  for (int sp = 0; sp < n_fsplit; ++sp) {
    const double2* q = farp + (((size_t)sp * nk + kk) * T + t) * 2;
    gxr += q[0].x;
    gxi += q[0].y;
    gyr += q[1].x;
    gyi += q[1].y;
  }
  const double s = side != 0 ? (double)side : (si == 0 ? 1.0 : -1.0);
  const size_t o = ((size_t)si * nk + kk) * T + t;
  if (grad) {   // (i/4) z = (-Im z / 4, Re z / 4)
    double* q = grad + 4 * o;
    q[0] = -0.25 * gxi;
    q[1] = 0.25 * gxr;
    q[2] = -0.25 * gyi;
    q[3] = 0.25 * gyr;
  }
  if (dn) {     // n = -s w^
    const double nr = -s * fma(c.ct, gxr, c.st * gyr), ni = -s * fma(c.ct, gxi, c.st * gyi);
    dn[2 * o] = -0.25 * ni;
    dn[2 * o + 1] = 0.25 * nr;
  }
}

template <int P>
static hipError_t launch_split_near_grad_p(const Dims& d, const double4* geo, const double2* dens,
                                           const CenterRec* ctr, const double* jtab,
                                           const double4* bnd, double g2, NearLists nl,
                                           double2* partial, hipStream_t s) {
  const dim3 grid((unsigned)((d.Mc + 3) / 4)), block(256);
#define QBX_NGRAD_ARGS \
  geo, dens, d.N, d.qs, ctr, jtab, d.NJ, d.Mc, d.T, bnd, d.P, g2, nl, d.k, partial
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_near_grad<P, 1>), grid, block, 0, s, QBX_NGRAD_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_near_grad<P, 2>), grid, block, 0, s, QBX_NGRAD_ARGS); break;
    default: hipLaunchKernelGGL((k_split_near_grad<P, 3>), grid, block, 0, s, QBX_NGRAD_ARGS); break;
  }
#undef QBX_NGRAD_ARGS
  return hipGetLastError();
}

hipError_t launch_split_gradient(const Dims& d, const double* nodes, const double4* geo,
                                 const double2* dens, NystromSources ns, const CenterRec* ctr,
                                 const double* jtab, const double4* bnd, double g2, NearLists nl,
                                 double2* nearp, double2* farp, double* grad, double* dn,
                                 hipStream_t s) {
  hipError_t e;
  {
    auto launch = [&]() -> hipError_t {
      QBX_P_SWITCH(d.p, launch_split_near_grad_p, d, geo, dens, ctr, jtab, bnd, g2, nl, nearp, s)
    };
    e = launch();
    if (e != hipSuccess) return e;
  }
  const int n_tb = (d.T + kWave - 1) / kWave;
  const long waves = (long)n_tb * d.n_fsplit;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_FGRAD_ARGS \
  ns.geo, ns.dens, d.T, nodes, d.T, bnd, d.P, g2, d.k, n_tb, d.n_fsplit, \
      farp
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_far_grad<1>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_far_grad<2>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
    default: hipLaunchKernelGGL((k_split_far_grad<3>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
  }
#undef QBX_FGRAD_ARGS
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_split_finalize_gradient, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T,
                     d.nk, d.n_fsplit, d.side, ctr, nearp, farp, grad, dn);
  return hipGetLastError();
}

hipError_t launch_panel_bounds(const Dims& d, const double* nodes, double4* bnd, hipStream_t s) {
  hipLaunchKernelGGL(k_panel_bounds, dim3((d.P + 255) / 256), dim3(256), 0, s, d.P, nodes, bnd);
  return hipGetLastError();
}

hipError_t launch_nystrom_sources(const Dims& d, const double* nodes, const double* density,
                                  const double* tables, NystromSources ns, hipStream_t s) {
  const TableLayout L = table_layout(d.qs);
  hipLaunchKernelGGL(k_nystrom_sources, dim3((d.T + 255) / 256), dim3(256), 0, s, d.T, d.nk,
                     nodes, density, tables + L.Dn, tables + L.w16, ns.geo, ns.dens, ns.w);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_split_near_p(const Dims& d, const double4* geo, const double2* dens,
                                      const CenterRec* ctr, const double* jtab,
                                      const double4* bnd, double g2, NearLists nl,
                                      double2* partial, hipStream_t s) {
  const dim3 grid((unsigned)((d.Mc + 3) / 4)), block(256);
#define QBX_NEAR_ARGS \
  geo, dens, d.N, d.qs, ctr, jtab, d.NJ, d.Mc, d.T, bnd, d.P, g2, nl, d.k, partial
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_near<P, 1>), grid, block, 0, s, QBX_NEAR_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_near<P, 2>), grid, block, 0, s, QBX_NEAR_ARGS); break;
    default: hipLaunchKernelGGL((k_split_near<P, 3>), grid, block, 0, s, QBX_NEAR_ARGS); break;
  }
#undef QBX_NEAR_ARGS
  return hipGetLastError();
}

hipError_t launch_split_near(const Dims& d, const double4* geo, const double2* dens,
                             const CenterRec* ctr, const double* jtab, const double4* bnd,
                             double g2, NearLists nl, double2* partial, hipStream_t s) {
  QBX_P_SWITCH(d.p, launch_split_near_p, d, geo, dens, ctr, jtab, bnd, g2, nl, partial, s)
}

hipError_t launch_near_lists(const Dims& d, const double4* bnd, double g2, int* count, int* list,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_near_lists, dim3((unsigned)((d.P + 3) / 4)), dim3(256), 0, s, d.P, bnd,
                     g2, count, list);
  return hipGetLastError();
}

hipError_t launch_split_far(const Dims& d, NystromSources ns, const double* nodes,
                            const double4* bnd, double g2, double2* partial, hipStream_t s) {
  const int n_tb = (d.T + kWave - 1) / kWave;
  const long waves = (long)n_tb * d.n_fsplit;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_FAR_ARGS \
  ns.geo, ns.dens, d.T, nodes, d.T, bnd, d.P, g2, d.k, n_tb, d.n_fsplit, \
      partial
  switch (d.kind) {
    case 1: hipLaunchKernelGGL((k_split_far<1>), grid, block, 0, s, QBX_FAR_ARGS); break;
    case 2: hipLaunchKernelGGL((k_split_far<2>), grid, block, 0, s, QBX_FAR_ARGS); break;
    default: hipLaunchKernelGGL((k_split_far<3>), grid, block, 0, s, QBX_FAR_ARGS); break;
  }
#undef QBX_FAR_ARGS
  return hipGetLastError();
}

hipError_t launch_split_finalize(const Dims& d, const double2* nearp, const double2* farp,
                                 double* out, hipStream_t s) {
  const int n = d.Mc * d.nk;
  hipLaunchKernelGGL(k_split_finalize, dim3((n + 255) / 256), dim3(256), 0, s, d.Mc, d.T, d.nk,
                     d.n_fsplit, nearp, farp, out);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_split_nodes_near_p(const Dims& d, const double4* geo,
                                            const double2* dens, const CenterRec* ctr,
                                            const double* jtab, const double4* bnd, double g2,
                                            NearLists nl, const double2* G, double* cg,
                                            double2* spart, hipStream_t s) {
  const dim3 gc((unsigned)((d.Mc + 3) / 4)), block(256);
  const int chunks = (d.N + kWave - 1) / kWave;
  const dim3 gs((unsigned)((chunks + 3) / 4));
#define QBX_NCG_ARGS \
  geo, dens, d.N, d.qs, ctr, jtab, d.NJ, d.Mc, d.T, d.side, bnd, d.P, g2, nl, d.k, G, cg
#define QBX_NSRC_ARGS \
  geo, dens, d.N, d.qs, ctr, jtab, d.NJ, d.Mc, d.T, d.n_sides, bnd, d.P, g2, nl, d.k, G, spart
  switch (d.kind) {
    case 1:
      hipLaunchKernelGGL((k_split_near_cg<P, 1>), gc, block, 0, s, QBX_NCG_ARGS);
      hipLaunchKernelGGL((k_split_near_adj_nodes<P, 1>), gs, block, 0, s, QBX_NSRC_ARGS);
      break;
    case 2:
      hipLaunchKernelGGL((k_split_near_cg<P, 2>), gc, block, 0, s, QBX_NCG_ARGS);
      hipLaunchKernelGGL((k_split_near_adj_nodes<P, 2>), gs, block, 0, s, QBX_NSRC_ARGS);
      break;
    default:
      hipLaunchKernelGGL((k_split_near_cg<P, 3>), gc, block, 0, s, QBX_NCG_ARGS);
      hipLaunchKernelGGL((k_split_near_adj_nodes<P, 3>), gs, block, 0, s, QBX_NSRC_ARGS);
      break;
  }
#undef QBX_NCG_ARGS
#undef QBX_NSRC_ARGS
  return hipGetLastError();
}

hipError_t launch_split_adjoint_nodes(const Dims& d, const double* nodes, const double* density,
                                      const double* tables, const double4* geo,
                                      const double2* dens, NystromSources ns,
                                      const CenterRec* ctr, const double* jtab,
                                      const double4* bnd, double g2, NearLists nl,
                                      const double2* G, SplitNodeScratch w,
                                      double* grad_density, double* grad_nodes, hipStream_t s) {
  hipError_t e;
  {
    auto launch = [&]() -> hipError_t {
      QBX_P_SWITCH(d.p, launch_split_nodes_near_p, d, geo, dens, ctr, jtab, bnd, g2, nl, G, w.cg,
                   w.spart, s)
    };
    e = launch();
    if (e != hipSuccess) return e;
  }
  const int nt = d.T * d.nk;
  hipLaunchKernelGGL(k_split_gfar, dim3((nt + 255) / 256), dim3(256), 0, s, d.T, d.nk, d.n_sides,
                     G, w.Gf);
  // far, target side: the split's far target gradients
  {
    const int n_tb = (d.T + kWave - 1) / kWave;
    const long waves = (long)n_tb * d.n_fsplit;
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_FGRAD_ARGS                                                                          \
  ns.geo, ns.dens, d.T, nodes, d.T, bnd, d.P, g2, d.k, n_tb, d.n_fsplit, \
      w.fpart
    switch (d.kind) {
      case 1: hipLaunchKernelGGL((k_split_far_grad<1>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
      case 2: hipLaunchKernelGGL((k_split_far_grad<2>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
      default: hipLaunchKernelGGL((k_split_far_grad<3>), grid, block, 0, s, QBX_FGRAD_ARGS); break;
    }
#undef QBX_FGRAD_ARGS
  }
  // far, source side (the far sources at the nodes)
  {
    const int n_sb = (d.T + kWave - 1) / kWave;
    const long waves = (long)n_sb * d.n_asplit;
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define QBX_FADJ_ARGS                                                                       \
  ns.geo, ns.dens, d.T, nodes, d.T, bnd, d.P, g2, d.k, w.Gf, n_sb, d.n_asplit,          \
      w.apart
    switch (d.kind) {
      case 1: hipLaunchKernelGGL((k_split_far_adj<1, true>), grid, block, 0, s, QBX_FADJ_ARGS); break;
      case 2: hipLaunchKernelGGL((k_split_far_adj<2, true>), grid, block, 0, s, QBX_FADJ_ARGS); break;
      default: hipLaunchKernelGGL((k_split_far_adj<3, true>), grid, block, 0, s, QBX_FADJ_ARGS); break;
    }
#undef QBX_FADJ_ARGS
  }
  const TableLayout L = table_layout(d.qs);
  hipLaunchKernelGGL(k_split_nystrom_grad, dim3((d.T + 255) / 256), dim3(256), 0, s, d.T, d.nk,
                     d.n_fsplit, d.n_asplit, density, ns.geo, ns.w, tables + L.w16, w.Gf, w.fpart,
                     w.apart, w.cg, w.gtw, w.gde);
  hipLaunchKernelGGL(k_split_source_finalize, dim3((d.N + 255) / 256), dim3(256), 0, s, d.N,
                     d.kind, geo, w.spart, w.sg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_chain(d, nodes, density, tables, w.sg, w.cg, w.gtw,
                      reinterpret_cast<const double*>(w.gde), grad_density, grad_nodes, s);
}

}  // namespace qbx
