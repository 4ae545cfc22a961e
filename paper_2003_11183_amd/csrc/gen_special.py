"""Generate special_tables.hpp: polynomial coefficients of the device Phi, Phi^-1.

Two functions are approximated, each by polynomials whose coefficients are
computed here in 60-digit arithmetic (mpmath) by Chebyshev interpolation,
converted to the monomial basis in high precision and rounded to double:

* erfcx(z) = exp(z^2) erfc(z) on z >= 0, as a polynomial in
  t = (z - K) / (z + K) in [-1, 1) (the rational map of Schonfelder 1978,
  which makes erfcx analytic in t up to z = infinity).  Phi follows as
  Phi(x) = erfcx(|x|/sqrt2) exp(-x^2/2) / 2 for x <= 0.
* erfinv, after Giles ("Approximating the erfinv function", GPU Computing
  Gems, 2011): erfinv(x) = x p(w) with w = -log((1 - x)(1 + x)), p a
  polynomial in w on [0, 6.25] and in sqrt(w) on four intervals up to
  sqrt(w) = 27.5 (u down to about 1e-330).
  Phi^-1(u) = sqrt2 erfinv(2u - 1) with w = -log(4 u (1 - u)).
* exp(r) on |r| <= ln2/2 (after x = k ln2 + r) and, for log, the odd part
  of log((1+s)/(1-s)) = 2s + s^3 Q(s^2) on |s| <= (sqrt2-1)/(sqrt2+1), the
  range of s = f/(2+f) for a mantissa 1 + f in [sqrt(1/2), sqrt 2).

The script prints the worst relative error of the double-precision Horner
evaluation over a dense grid.  Run:  python gen_special.py > special_tables.hpp
"""

from __future__ import annotations

import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 60
K_ERFCX = 3.75
Z_MAX = 12.0                      # erfcx polynomial range; continued fraction above
T_MAX = (Z_MAX - K_ERFCX) / (Z_MAX + K_ERFCX)
DEG_ERFCX = 22
ASYM_TERMS = 12                   # terms of the asymptotic series of erfcx above Z_MAX
# Phi^-1 regions: (variable, lower, upper, degree); variable "w" or "s" = sqrt(w)
INV_REGIONS = [("w", 0.0, 6.25, 26), ("s", 2.5, 4.0, 22), ("s", 4.0, 8.0, 22),
               ("s", 8.0, 14.0, 18), ("s", 14.0, 27.5, 18)]


def cheb_fit(f, a, b, deg):
    """Monomial coefficients (in s = (x - c) / h, c, h centre/half-width) of the
    degree-deg Chebyshev interpolant of f on [a, b], in high precision."""
    N = deg + 1
    c, h = (mp.mpf(a) + mp.mpf(b)) / 2, (mp.mpf(b) - mp.mpf(a)) / 2
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / N) for k in range(N)]
    vals = [f(c + h * s) for s in nodes]
    cheb = []
    for j in range(N):
        sm = mp.fsum(vals[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / N) for k in range(N))
        cheb.append(sm * (1 if j == 0 else 2) / N)
    # Chebyshev -> monomial in s
    T = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for j in range(2, N):
        prev, prev2 = T[-1], T[-2]
        nxt = [mp.mpf(0)] + [2 * x for x in prev]
        for i, x in enumerate(prev2):
            nxt[i] -= x
        T.append(nxt)
    mono = [mp.mpf(0)] * N
    for j in range(N):
        for i, x in enumerate(T[j]):
            mono[i] += cheb[j] * x
    return [float(x) for x in mono], float(c), float(h)


def horner(coef, s):
    acc = np.zeros_like(s) + coef[-1]
    for cf in reversed(coef[:-1]):
        acc = acc * s + cf
    return acc


def erfcx_t(t):
    z = K_ERFCX * (1 + t) / (1 - t)
    return mp.exp(z * z) * mp.erfc(z)


def erfcx_scaled_t(t):
    """g(t) = erfcx(z) (z + K) / K; erfcx(z) = g(t) (1 - t) / 2."""
    z = K_ERFCX * (1 + t) / (1 - t)
    return erfcx_t(t) * (z + K_ERFCX) / K_ERFCX


def erfinv_p_of_w(w):
    # x with -log((1-x)(1+x)) = w, x in [0, 1): x = sqrt(1 - exp(-w)).
    if w == 0:
        return mp.sqrt(mp.pi) / 2
    x = mp.sqrt(-mp.expm1(-w))
    if w < 20:
        return mp.erfinv(x) / x
    # Far tail: erfinv(x) = y with erfc(y) = 1 - x = exp(-w) / (1 + x),
    # solved by Newton on log erfc (exact to the working precision).
    lq = -w - mp.log(1 + x)
    y = mp.sqrt(w)
    for _ in range(200):
        f = mp.log(mp.erfc(y)) - lq
        d = -2 / mp.sqrt(mp.pi) * mp.exp(-y * y) / mp.erfc(y)
        dy = f / d
        y -= dy
        if abs(dy) < mp.mpf(10) ** (-50):
            break
    return y / x


def erfinv_p_of_sqrtw(s):
    return erfinv_p_of_w(s * s)


def check(name, coef, c, h, f, lo, hi, n=2001):
    xs = np.linspace(lo, hi, n)
    got = horner(coef, (xs - c) / h)
    ref = np.array([float(f(mp.mpf(x))) for x in xs])
    err = float(np.max(np.abs(got - ref) / np.abs(ref)))
    print(f"// {name}: degree {len(coef) - 1}, max relative error {err:.2e}", file=sys.stderr)
    return err


def emit(name, coef):
    body = ",\n    ".join(f"{x:.17e}" for x in coef)
    return f"constexpr double {name}[{len(coef)}] = {{\n    {body}}};\n"


LN2 = mp.log(2)
EXP_DEG = 13
LOG_DEG = 9
LOG_SMAX = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)   # s = f / (2 + f), f = m - 1, m in [sqrt(1/2), sqrt 2)


def exp_r(r):
    return mp.exp(r)


def log_q(v):
    """Q(v) with log((1+s)/(1-s)) = 2s + s^3 Q(s^2), v = s^2."""
    if v == 0:
        return mp.mpf(2) / 3
    sq = mp.sqrt(v)
    return (mp.log((1 + sq) / (1 - sq)) - 2 * sq) / (sq ** 3)


# FP32 centre-region forms of the precision variant (coefficients rounded to
# float32; checked by float32 Horner evaluation).
Z_MAX32 = 8.0
K32 = 2.5
T_MAX32 = (Z_MAX32 - K32) / (Z_MAX32 + K32)
DEG32_ERFCX = 11
DEG32_INV = 10
W_MAX32 = 6.25
# float32 tail of erfinv in sqrt(w), out to w = 90 (u down to about 3e-40,
# below the float32 normal range): two intervals split at sqrt(w) = 4.5
INV32_TAIL = [(2.5, 4.5, 8), (4.5, 9.5, 8)]


def erfcx_scaled_t32(t):
    z = K32 * (1 + t) / (1 - t)
    return mp.exp(z * z) * mp.erfc(z) * (z + K32) / K32


def fit32(f, a, b, deg, name):
    cf, c, h = cheb_fit(f, a, b, deg)
    c32 = [float(np.float32(x)) for x in cf]
    xs = np.linspace(a, b, 3001)
    s = ((xs - c) / h).astype(np.float32)
    acc = np.float32(c32[-1]) + np.zeros_like(s)
    for cc in reversed(c32[:-1]):
        acc = (acc * s + np.float32(cc)).astype(np.float32)
    ref = np.array([float(f(mp.mpf(x))) for x in xs])
    err = float(np.max(np.abs(acc.astype(np.float64) - ref) / np.abs(ref)))
    print(f"// {name} (float32): degree {deg}, max relative error {err:.2e}", file=sys.stderr)
    return c32, c, h


def asym_check():
    """Worst relative error of the truncated asymptotic series at z >= Z_MAX."""
    worst = 0.0
    for z in np.linspace(Z_MAX, 200.0, 400):
        v = 1.0 / (2.0 * z * z)
        acc, term = 0.0, 1.0
        for k in range(ASYM_TERMS):
            acc += term
            term *= -(2 * k + 1) * v
        got = acc / (z * float(mp.sqrt(mp.pi)))
        ref = float(mp.exp(mp.mpf(z) ** 2) * mp.erfc(mp.mpf(z)))
        worst = max(worst, abs(got - ref) / ref)
    print(f"// erfcx asymptotic series, {ASYM_TERMS} terms, z >= {Z_MAX}: max relative error {worst:.2e}",
          file=sys.stderr)


def main():
    out = ["// Generated by gen_special.py; do not edit.",
           "// Polynomial coefficients (monomial basis, constant term first), all in",
           "// one table so that device code can fetch them with scalar loads; the",
           "// kOff* / kN* constants give each polynomial's offset and length.",
           "#pragma once", "", "#ifndef TLRQMC_SPECIAL_TABLE", "#define TLRQMC_SPECIAL_TABLE constexpr",
           "#endif", "", "namespace tlrqmc {", "namespace dev {", "",
           f"constexpr double kErfcxK = {K_ERFCX!r};",
           f"constexpr double kErfcxZmax = {Z_MAX!r};",
           f"constexpr int kErfcxAsymTerms = {ASYM_TERMS};"]
    table = []
    ce, c0, h0 = cheb_fit(erfcx_scaled_t, -1, T_MAX, DEG_ERFCX)
    check("erfcx g(t), z in [0, 12]", ce, c0, h0, erfcx_scaled_t, -1, T_MAX)
    asym_check()
    out.append(f"constexpr double kErfcxC = {c0!r}, kErfcxH = {1.0 / h0!r};  // s = (t - C) * H")
    out.append(f"constexpr int kOffErfcx = {len(table)}, kNErfcx = {len(ce)};")
    table += ce
    for idx, (var, lo, hi, deg) in enumerate(INV_REGIONS, start=1):
        f = erfinv_p_of_w if var == "w" else erfinv_p_of_sqrtw
        cf, mc, hh = cheb_fit(f, lo, hi, deg)
        check(f"erfinv p({var}) on [{lo}, {hi}]", cf, mc, hh, f, lo, hi)
        out.append(f"constexpr double kInvC{idx} = {mc!r}, kInvH{idx} = {1.0 / hh!r};  // region {var} in [{lo}, {hi}]")
        out.append(f"constexpr int kOffInv{idx} = {len(table)}, kNInv{idx} = {len(cf)};")
        table += cf
    # exp(r) on |r| <= ln2 / 2 (range reduction x = k ln2 + r)
    half = float(LN2 / 2)
    cx, mx_, hx = cheb_fit(exp_r, -half, half, EXP_DEG)
    check("exp(r), |r| <= ln2/2", cx, mx_, hx, exp_r, -half, half)
    out.append(f"constexpr double kExpH = {1.0 / hx!r};  // polynomial variable r * H")
    out.append(f"constexpr int kOffExp = {len(table)}, kNExp = {len(cx)};")
    table += cx
    vmax = float(LOG_SMAX ** 2)
    cl, ml, hl = cheb_fit(log_q, 0.0, vmax, LOG_DEG)
    check("log Q(s^2)", cl, ml, hl, log_q, 0.0, vmax)
    out.append(f"constexpr double kLogC = {ml!r}, kLogH = {1.0 / hl!r};  // (s^2 - C) * H")
    out.append(f"constexpr int kOffLog = {len(table)}, kNLog = {len(cl)};")
    table += cl
    # float32 polynomials (compile-time constants: 32-bit literals in the code)
    c32e, m32e, h32e = fit32(erfcx_scaled_t32, -1, T_MAX32, DEG32_ERFCX, "erfcx g(t), z in [0, 8]")
    c32i, m32i, h32i = fit32(erfinv_p_of_w, 0.0, W_MAX32, DEG32_INV, "erfinv p(w), w in [0, 6.25]")
    tails32 = [fit32(erfinv_p_of_sqrtw, lo, hi, deg, f"erfinv p(sqrt w), sqrt w in [{lo}, {hi}]")
               for lo, hi, deg in INV32_TAIL]
    out.append(f"constexpr float kErfcx32K = {K32!r}f, kErfcx32Zmax = {Z_MAX32!r}f;")
    out.append(f"constexpr float kErfcx32C = {float(np.float32(m32e))!r}f, kErfcx32H = {float(np.float32(1.0 / h32e))!r}f;")
    out.append(f"constexpr float kErfcx32[{len(c32e)}] = {{" + ", ".join(f"{x!r}f" for x in c32e) + "};")
    out.append(f"constexpr float kInv32C = {float(np.float32(m32i))!r}f, kInv32H = {float(np.float32(1.0 / h32i))!r}f;")
    out.append(f"constexpr float kInv32[{len(c32i)}] = {{" + ", ".join(f"{x!r}f" for x in c32i) + "};")
    for k, (cf, mc, hh) in enumerate(tails32):
        lo, hi, _ = INV32_TAIL[k]
        out.append(f"// float32 erfinv tail {k}: sqrt(w) in [{lo}, {hi}]")
        out.append(f"constexpr float kInv32T{k}C = {float(np.float32(mc))!r}f, kInv32T{k}H = {float(np.float32(1.0 / hh))!r}f;")
        out.append(f"constexpr float kInv32T{k}[{len(cf)}] = {{" + ", ".join(f"{x!r}f" for x in cf) + "};")
    out.append(f"constexpr float kInv32Split = {INV32_TAIL[0][1]!r}f;")
    body = ",\n    ".join(f"{x:.17e}" for x in table)
    out.append(f"constexpr int kSpecialTableSize = {len(table)};")
    out.append(f"TLRQMC_SPECIAL_TABLE double kSpecialTable[{len(table)}] = {{\n    {body}}};")
    out += ["", "}  // namespace dev", "}  // namespace tlrqmc", ""]
    print("\n".join(out))


if __name__ == "__main__":
    main()
