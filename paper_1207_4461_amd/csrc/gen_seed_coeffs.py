"""Generate qbx_seed_coeffs.h: coefficients of the device Hankel seeds H_0, H_1.

Two regimes (z = k*rho > 0):

* z >= Z0: H_nu(z) = sqrt(2/(pi z)) exp(i(z - nu pi/2 - pi/4)) (P_nu(z) + i Q_nu(z))
  defines the smooth, non-oscillatory auxiliary functions P_nu, Q_nu (their large-z
  behaviour is the Hankel expansion, DLMF 10.17.3).  They are interpolated here
  at Chebyshev points in s = (Z0/z)^2 in (0, 1] from 40-digit mpmath values of
  J_nu + i Y_nu and stored as monomial coefficients in s:
      P_nu = sum_j p_j s^j,   Q_nu = (Z0/z) sum_j q_j s^j.
  Shorter fits of the same functions serve the wavefronts whose every lane is
  farther: in s = (ZM/z)^2 for z >= ZM, in s = (ZF/z)^2 for z >= ZF, in
  s = (ZV/z)^2 for z >= ZV and, shortest, in s = (ZU/z)^2 for z >= ZU.
* the phase with the amplitude's constant, sqrt(2/pi) e^{i(z - pi/4)} = T_n e^{ir}:
  n = rint(z N / 2 pi), r = z - 2 pi n / N by a two-part Cody-Waite reduction (the
  first part's 29 bits make n times it exact; the second enters through one fused
  multiply-add), T_n = sqrt(2/pi) e^{i(2 pi n/N - pi/4)} from a table of N = 1024
  entries (40-digit values rounded once; the factor sqrt(2/pi) of the amplitude
  sqrt(2/(pi z)) rides in the table, so the kernels multiply by 1/sqrt(z) only), and
  sin r / r, cos r by their Taylor polynomials of degree 2 in r^2 (|r| <= pi/N, so
  the first dropped terms are below 2e-18).
* Z1 <= z < Z0: the entire functions J_0, J_1, R_0 = Y_0 - (2/pi) L J_0 and
  R_1 = Y_1 + 2/(pi z) - (2/pi) L J_1, L = ln(z/2) + gamma (the log terms of
  DLMF 10.8.1/10.8.2 split off), each interpolated at Chebyshev points of [Z1, Z0]
  (40-digit values) and stored as monomials in x = (z - ZC)/ZH.
* z < Z1: the ascending series (DLMF 10.2.2 for J, 10.8.1 / 10.8.2 for Y) in
  w = z^2/4:
      J0 = sum (-w)^k/(k!)^2,   J1 = (z/2) sum (-w)^k/(k!(k+1)!),
      Y0 = (2/pi)(ln(z/2) + gamma) J0 + (2/pi) sum_{k>=1} (-1)^{k+1} H_k w^k/(k!)^2,
      Y1 = -2/(pi z) + (2/pi) ln(z/2) J1
           - (z/(2 pi)) sum (psi(k+1) + psi(k+2)) (-w)^k/(k!(k+1)!).
  Coefficients are exact rationals (harmonic numbers) rounded once to double.

Run:  python gen_seed_coeffs.py   (writes qbx_seed_coeffs.h next to this file and
prints the double-precision evaluation error of every approximation).
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import mpmath
import numpy as np

Z0 = 6.0
DEG = 12          # degree in s of the P, Q fits
ZM = 10.0
DEG_MED = 9       # degree in s = (ZM/z)^2 of the fits for z >= ZM
ZF = 20.0
DEG_FAR = 6       # degree in s = (ZF/z)^2 of the far fits
ZV = 60.0
DEG_VFAR = 4      # degree in s = (ZV/z)^2 of the fits for z >= ZV
ZU = 80.0
DEG_UFAR = 3      # degree in s = (ZU/z)^2 of the fits for z >= ZU
PHASE_N = 1024    # phase table entries sqrt(2/pi) e^{i(2 pi n/N - pi/4)}
R_TRIG = 0.00307  # reduced argument bound (pi/N plus the reduction's rounding)
Z1 = 4.0          # below: ascending series; [Z1, Z0): interpolated entire parts
NSER = 17         # series terms for z < Z1
DEG_MID = 15      # degree of the mid-range fits in x = (z - ZC)/ZH in [-1, 1]
ZC = 0.5 * (Z0 + Z1)
ZH = 0.5 * (Z0 - Z1)
mpmath.mp.dps = 40


def pq(nu: int, z) -> tuple:
    z = mpmath.mpf(z)
    H = mpmath.besselj(nu, z) + 1j * mpmath.bessely(nu, z)
    v = H * mpmath.sqrt(mpmath.pi * z / 2) * mpmath.exp(-1j * (z - nu * mpmath.pi / 2 - mpmath.pi / 4))
    return mpmath.re(v), mpmath.im(v)


def cheb_fit_monomial(f, deg: int, M: int = 64):
    """Chebyshev interpolation of f on s in [0,1] (M points), truncated to `deg`,
    returned as monomial coefficients in s (mp floats)."""
    xs = [mpmath.cos(mpmath.pi * (j + mpmath.mpf(1) / 2) / M) for j in range(M)]   # in (-1,1)
    fs = [f((x + 1) / 2) for x in xs]
    c = []
    for kk in range(deg + 1):
        acc = mpmath.mpf(0)
        for j in range(M):
            acc += fs[j] * mpmath.cos(kk * mpmath.pi * (j + mpmath.mpf(1) / 2) / M)
        c.append(acc * (1 if kk == 0 else 2) / M)
    # T_k(2s-1) -> monomials in s
    mono = [mpmath.mpf(0)] * (deg + 1)
    Tm1 = [mpmath.mpf(1)]                      # T_0
    T0 = [mpmath.mpf(-1), mpmath.mpf(2)]       # T_1(2s-1) = 2s - 1
    for kk in range(deg + 1):
        Tk = Tm1 if kk == 0 else T0
        if kk >= 2:
            # T_k = 2(2s-1)T_{k-1} - T_{k-2}
            prev = T0
            new = [mpmath.mpf(0)] * (kk + 1)
            for i, a in enumerate(prev):
                new[i] += -2 * a
                new[i + 1] += 4 * a
            for i, a in enumerate(Tm1):
                new[i] -= a
            Tm1, T0 = T0, new
            Tk = new
        for i, a in enumerate(Tk):
            mono[i] += c[kk] * a
    return mono


def cheb_fit_monomial_pm1(f, deg: int, M: int = 64):
    """Chebyshev interpolation of f on x in [-1, 1], as monomial coefficients in x."""
    xs = [mpmath.cos(mpmath.pi * (j + mpmath.mpf(1) / 2) / M) for j in range(M)]
    fs = [f(x) for x in xs]
    c = []
    for kk in range(deg + 1):
        acc = mpmath.mpf(0)
        for j in range(M):
            acc += fs[j] * mpmath.cos(kk * mpmath.pi * (j + mpmath.mpf(1) / 2) / M)
        c.append(acc * (1 if kk == 0 else 2) / M)
    mono = [mpmath.mpf(0)] * (deg + 1)
    Tm1, T0 = [mpmath.mpf(1)], [mpmath.mpf(0), mpmath.mpf(1)]
    for kk in range(deg + 1):
        if kk == 0:
            Tk = Tm1
        elif kk == 1:
            Tk = T0
        else:
            new = [mpmath.mpf(0)] * (kk + 1)
            for i, a in enumerate(T0):
                new[i + 1] += 2 * a
            for i, a in enumerate(Tm1):
                new[i] -= a
            Tm1, T0 = T0, new
            Tk = new
        for i, a in enumerate(Tk):
            mono[i] += c[kk] * a
    return mono


def horner(coefs, x):
    acc = 0.0
    for a in reversed(coefs):
        acc = acc * x + a
    return acc


def main():
    fits = {}
    for nu in (0, 1):
        fits[f"P{nu}"] = cheb_fit_monomial(lambda s, nu=nu: pq(nu, Z0 / mpmath.sqrt(s))[0], DEG)
        fits[f"Q{nu}"] = cheb_fit_monomial(
            lambda s, nu=nu: pq(nu, Z0 / mpmath.sqrt(s))[1] * (Z0 / mpmath.sqrt(s)) / Z0, DEG)
        fits[f"FP{nu}"] = cheb_fit_monomial(lambda s, nu=nu: pq(nu, ZF / mpmath.sqrt(s))[0],
                                            DEG_FAR)
        fits[f"FQ{nu}"] = cheb_fit_monomial(
            lambda s, nu=nu: pq(nu, ZF / mpmath.sqrt(s))[1] * (ZF / mpmath.sqrt(s)) / ZF, DEG_FAR)
        fits[f"MP{nu}"] = cheb_fit_monomial(lambda s, nu=nu: pq(nu, ZM / mpmath.sqrt(s))[0],
                                            DEG_MED)
        fits[f"MQ{nu}"] = cheb_fit_monomial(
            lambda s, nu=nu: pq(nu, ZM / mpmath.sqrt(s))[1] * (ZM / mpmath.sqrt(s)) / ZM, DEG_MED)
        fits[f"UP{nu}"] = cheb_fit_monomial(lambda s, nu=nu: pq(nu, ZU / mpmath.sqrt(s))[0],
                                            DEG_UFAR)
        fits[f"UQ{nu}"] = cheb_fit_monomial(
            lambda s, nu=nu: pq(nu, ZU / mpmath.sqrt(s))[1] * (ZU / mpmath.sqrt(s)) / ZU, DEG_UFAR)
        fits[f"VP{nu}"] = cheb_fit_monomial(lambda s, nu=nu: pq(nu, ZV / mpmath.sqrt(s))[0],
                                            DEG_VFAR)
        fits[f"VQ{nu}"] = cheb_fit_monomial(
            lambda s, nu=nu: pq(nu, ZV / mpmath.sqrt(s))[1] * (ZV / mpmath.sqrt(s)) / ZV, DEG_VFAR)
    zc, zh = mpmath.mpf(ZC), mpmath.mpf(ZH)
    fits["MJ0"] = cheb_fit_monomial_pm1(lambda x: mpmath.besselj(0, zc + zh * x), DEG_MID)
    def Lg(z):
        return mpmath.log(z / 2) + mpmath.euler

    fits["MY0"] = cheb_fit_monomial_pm1(
        lambda x: mpmath.bessely(0, zc + zh * x) - 2 / mpmath.pi * Lg(zc + zh * x) * mpmath.besselj(0, zc + zh * x),
        DEG_MID)
    fits["MJ1"] = cheb_fit_monomial_pm1(lambda x: mpmath.besselj(1, zc + zh * x), DEG_MID)
    fits["MY1"] = cheb_fit_monomial_pm1(
        lambda x: (mpmath.bessely(1, zc + zh * x) + 2 / (mpmath.pi * (zc + zh * x))
                   - 2 / mpmath.pi * Lg(zc + zh * x) * mpmath.besselj(1, zc + zh * x)), DEG_MID)
    dbl = {k: [float(a) for a in v] for k, v in fits.items()}

    # series coefficients (exact rationals)
    fact = [math.factorial(k) for k in range(NSER + 2)]
    Hk = [Fraction(0)]
    for k in range(1, NSER + 2):
        Hk.append(Hk[-1] + Fraction(1, k))
    # J0 = sum a_k w^k, a_k = (-1)^k/(k!)^2
    aJ0 = [Fraction((-1) ** k, fact[k] ** 2) for k in range(NSER)]
    # J1 = (z/2) sum b_k w^k, b_k = (-1)^k/(k!(k+1)!)
    bJ1 = [Fraction((-1) ** k, fact[k] * fact[k + 1]) for k in range(NSER)]
    # Y0 remainder: sum_{k>=1} c_k w^k, c_k = (-1)^{k+1} H_k/(k!)^2  (times 2/pi)
    cY0 = [Fraction(0)] + [Fraction((-1) ** (k + 1)) * Hk[k] / fact[k] ** 2 for k in range(1, NSER)]
    # Y1 remainder: -(z/(2pi)) sum (psi(k+1)+psi(k+2)) (-w)^k/(k!(k+1)!)
    # psi(k+1) + psi(k+2) = -2 gamma + H_k + H_{k+1}; the gamma part sums to (2 gamma/pi) J1,
    # so Y1 = -2/(pi z) + (2/pi)(ln(z/2) + gamma) J1 - (z/(2 pi)) sum d_k w^k with
    # d_k = (-1)^k (H_k + H_{k+1})/(k!(k+1)!)
    dY1 = [Fraction((-1) ** k) * (Hk[k] + Hk[k + 1]) / (fact[k] * fact[k + 1]) for k in range(NSER)]

    # ---- verification in double -------------------------------------------------
    rng = np.random.default_rng(0)
    zs_big = np.concatenate([np.geomspace(Z0, 2e4, 1500), rng.uniform(Z0, 40, 500)])
    zs_small = np.concatenate([np.geomspace(1e-4, Z1, 1500), rng.uniform(0.5, Z1, 500)])
    zs_mid = np.concatenate([np.linspace(Z1, Z0, 1500), rng.uniform(Z1, Z0, 500)])
    worst_mid = 0.0
    for z in zs_mid:
        x = (z - ZC) / ZH
        L = math.log(z / 2) + float(mpmath.euler)
        for nu in (0, 1):
            Jv = horner(dbl[f"MJ{nu}"], x)
            Yv = horner(dbl[f"MY{nu}"], x) + 2 / math.pi * L * Jv - (2 / (math.pi * z) if nu else 0.0)
            ref = complex(mpmath.besselj(nu, z) + 1j * mpmath.bessely(nu, z))
            worst_mid = max(worst_mid, abs(complex(Jv, Yv) - ref) / abs(ref))
    g = float(mpmath.euler)
    worst_far = 0.0
    for z in np.concatenate([np.geomspace(ZF, 2e4, 1500), rng.uniform(ZF, 80, 500)]):
        s = (ZF / z) ** 2
        for nu in (0, 1):
            P = horner(dbl[f"FP{nu}"], s)
            Qv = (ZF / z) * horner(dbl[f"FQ{nu}"], s)
            pr, qr = pq(nu, z)
            worst_far = max(worst_far, abs(complex(P - float(pr), Qv - float(qr))))
    worst_med = 0.0
    for z in np.concatenate([np.geomspace(ZM, 2e4, 1500), rng.uniform(ZM, 30, 500)]):
        s = (ZM / z) ** 2
        for nu in (0, 1):
            P = horner(dbl[f"MP{nu}"], s)
            Qv = (ZM / z) * horner(dbl[f"MQ{nu}"], s)
            pr, qr = pq(nu, z)
            worst_med = max(worst_med, abs(complex(P - float(pr), Qv - float(qr))))
    worst_ufar = 0.0
    for z in np.concatenate([np.geomspace(ZU, 2e4, 1500), rng.uniform(ZU, 250, 500)]):
        s = (ZU / z) ** 2
        for nu in (0, 1):
            P = horner(dbl[f"UP{nu}"], s)
            Qv = (ZU / z) * horner(dbl[f"UQ{nu}"], s)
            pr, qr = pq(nu, z)
            worst_ufar = max(worst_ufar, abs(complex(P - float(pr), Qv - float(qr))))
    worst_vfar = 0.0
    for z in np.concatenate([np.geomspace(ZV, 2e4, 1500), rng.uniform(ZV, 200, 500)]):
        s = (ZV / z) ** 2
        for nu in (0, 1):
            P = horner(dbl[f"VP{nu}"], s)
            Qv = (ZV / z) * horner(dbl[f"VQ{nu}"], s)
            pr, qr = pq(nu, z)
            worst_vfar = max(worst_vfar, abs(complex(P - float(pr), Qv - float(qr))))
    worst_big = worst_small = 0.0
    for z in zs_big:
        s = (Z0 / z) ** 2
        for nu in (0, 1):
            P = horner(dbl[f"P{nu}"], s)
            Qv = (Z0 / z) * horner(dbl[f"Q{nu}"], s)
            pr, qr = pq(nu, z)
            err = abs(complex(P - float(pr), Qv - float(qr)))   # error of the fitted factor
            worst_big = max(worst_big, err)
    for z in zs_small:
        w = z * z / 4
        J0 = horner([float(a) for a in aJ0], w)
        ln = math.log(z / 2)
        J1 = (z / 2) * horner([float(b) for b in bJ1], w)
        Y0 = (2 / math.pi) * ((ln + g) * J0 + horner([float(c) for c in cY0], w))
        Y1 = (-2 / (math.pi * z) + (2 / math.pi) * (ln + g) * J1
              - (z / (2 * math.pi)) * horner([float(dd) for dd in dY1], w))
        for nu, (Jv, Yv) in enumerate(((J0, Y0), (J1, Y1))):
            ref = complex(mpmath.besselj(nu, z) + 1j * mpmath.bessely(nu, z))
            worst_small = max(worst_small, abs(complex(Jv, Yv) - ref) / abs(ref))
    print(f"fit error of P,Q (absolute, |P+iQ| ~ 1) for z >= {Z0}: {worst_big:.3e}")
    print(f"medium fit error of P,Q for z >= {ZM} (degree {DEG_MED}): {worst_med:.3e}")
    print(f"far fit error of P,Q for z >= {ZF} (degree {DEG_FAR}): {worst_far:.3e}")
    print(f"very-far fit error of P,Q for z >= {ZV} (degree {DEG_VFAR}): {worst_vfar:.3e}")
    print(f"ultra-far fit error of P,Q for z >= {ZU} (degree {DEG_UFAR}): {worst_ufar:.3e}")
    print(f"mid-range relative error of H for {Z1} <= z < {Z0}: {worst_mid:.3e}")
    print(f"series relative error of H for z < {Z1}: {worst_small:.3e}")

    # ---- write the header ------------------------------------------------------------
    def arr(name, vals):
        body = ",\n    ".join(f"{v:.17e}" for v in vals)
        return f"constexpr double {name}[{len(vals)}] = {{\n    {body}}};\n"

    # delta = 2 pi / N split for the Cody-Waite reduction z - n delta (n < 2^26, so
    # z < 4e5): the first part carries 27 significant bits, so n*part is exact and z
    # minus it is exact (Sterbenz); the second is the rest, rounded to double, and
    # enters through one fused multiply-add
    delta = 2 * mpmath.pi / PHASE_N
    e = mpmath.floor(mpmath.log(abs(delta), 2))
    scale = mpmath.mpf(2) ** (26 - e)
    hi = mpmath.floor(delta * scale) / scale
    parts = [float(hi), float(delta - hi)]
    phase = []
    amp = mpmath.sqrt(2 / mpmath.pi)
    for n in range(PHASE_N):
        a = n * delta - mpmath.pi / 4
        phase += [float(amp * mpmath.cos(a)), float(amp * mpmath.sin(a))]
    # sin(r)/r and cos(r): Taylor polynomials of degree 2 in u = r^2 (constant terms
    # exactly 1, which the kernels take as inline constants)
    sin_c = [1.0, float(mpmath.mpf(-1) / 6), float(mpmath.mpf(1) / 120)]
    cos_c = [1.0, -0.5, float(mpmath.mpf(1) / 24)]
    worst_trig = 0.0
    for r in np.linspace(-R_TRIG, R_TRIG, 4001):
        u = r * r
        sv, cv = r * horner(sin_c, u), horner(cos_c, u)
        worst_trig = max(worst_trig, abs(sv - float(mpmath.sin(r))), abs(cv - float(mpmath.cos(r))))
    print(f"sin/cos error for |r| <= {R_TRIG} (degree 2 in r^2): {worst_trig:.3e}")
    # the whole phase in double against 40 digits, z up to 2^24 delta
    worst_phase = 0.0
    for z in np.concatenate([rng.uniform(6, 60, 3000), np.geomspace(6, 4e5, 3000)]):
        n = float(np.rint(z * float(PHASE_N / (2 * mpmath.pi))))
        r = z - n * parts[0]        # n * parts[0] is exact, and so is the difference
        r = float(mpmath.mpf(r) - mpmath.mpf(n) * mpmath.mpf(parts[1]))   # one fma
        i = int(n) & (PHASE_N - 1)
        u = r * r
        sv, cv = r * horner(sin_c, u), horner(cos_c, u)
        er = phase[2 * i] * cv - phase[2 * i + 1] * sv
        ei = phase[2 * i] * sv + phase[2 * i + 1] * cv
        ref = amp * mpmath.exp(1j * (mpmath.mpf(z) - mpmath.pi / 4))
        worst_phase = max(worst_phase, abs(complex(er, ei) - complex(ref)) / float(amp))
    print(f"phase sqrt(2/pi) e^(i(z - pi/4)) relative error for 6 <= z <= 4e5 (double "
          f"evaluation): {worst_phase:.3e}")

    out = []
    out.append("// Generated by gen_seed_coeffs.py -- do not edit.\n")
    out.append("// Coefficients of the Hankel seeds H_0, H_1 (see qbx_special.h).\n#pragma once\n\n")
    out.append("namespace qbx {\nnamespace seed {\n\n")
    out.append(f"constexpr double kZ0 = {Z0:.17e};\nconstexpr double kZ1 = {Z1:.17e};\n")
    out.append(f"constexpr double kZM = {ZM:.17e};\n")
    out.append(f"constexpr double kZF = {ZF:.17e};\n")
    out.append(f"constexpr double kZV = {ZV:.17e};\n")
    out.append(f"constexpr double kZU = {ZU:.17e};\n")
    out.append(f"constexpr double kZC = {ZC:.17e};\nconstexpr double kInvZH = {1.0 / ZH:.17e};\n")
    out.append(f"constexpr int kPhaseN = {PHASE_N};\n")
    out.append(f"constexpr double kInvDelta = {float(PHASE_N / (2 * mpmath.pi)):.17e};\n")
    out.append(f"constexpr double kDeltaHi = {parts[0]:.17e};\n")
    out.append(f"constexpr double kDeltaLo = {parts[1]:.17e};\n")
    # one packed table; four polynomials of a regime interleaved so that a wave reads
    # the coefficients of one Horner step with a single scalar load
    table, offs = [], {}

    def block(name, polys):
        n = max(len(p_) for p_ in polys)
        offs[name] = (len(table), n)
        for i in range(n):
            for p_ in polys:
                table.append(p_[i] if i < len(p_) else 0.0)

    block("LARGE", [dbl["P0"], dbl["Q0"], dbl["P1"], dbl["Q1"]])
    block("MID", [dbl["MJ0"], dbl["MY0"], dbl["MJ1"], dbl["MY1"]])
    block("SER", [[float(a) for a in aJ0], [float(a) for a in bJ1], [float(a) for a in cY0],
                  [float(a) for a in dY1]])
    block("TRIG", [sin_c, cos_c])
    block("FAR", [dbl["FP0"], dbl["FQ0"], dbl["FP1"], dbl["FQ1"]])
    block("VFAR", [dbl["VP0"], dbl["VQ0"], dbl["VP1"], dbl["VQ1"]])
    block("MED", [dbl["MP0"], dbl["MQ0"], dbl["MP1"], dbl["MQ1"]])
    block("UFAR", [dbl["UP0"], dbl["UQ0"], dbl["UP1"], dbl["UQ1"]])
    for name, (o, n) in offs.items():
        out.append(f"constexpr int k{name}Off = {o};\nconstexpr int k{name}Len = {n};\n")
    out.append(f"constexpr int kTableLen = {len(table)};\n")
    body = ", \\\n    ".join(f"{v:.17e}" for v in table)
    out.append(f"#define QBX_SEED_TABLE_VALUES \\\n    {body}\n")
    body = ", \\\n    ".join(f"{v:.17e}" for v in phase)
    out.append(f"// e^(i(2 pi n/N - pi/4)), n = 0..N-1, as (cos, sin) pairs\n")
    out.append(f"#define QBX_PHASE_TABLE_VALUES \\\n    {body}\n")
    out.append("\n}  // namespace seed\n}  // namespace qbx\n")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qbx_seed_coeffs.h")
    with open(path, "w") as f:
        f.write("".join(out))
    print("wrote", path)


if __name__ == "__main__":
    main()
