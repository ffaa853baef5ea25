"""Write csrc/vmc_mass_start.hpp: start polynomials for the mass step of
RAMBO on diet (Plaetzer, arXiv:1308.2922), used by the phase-space map.

The mass fraction t in [0, 1] has CDF F(t) = (k+1) t^k - k t^(k+1).  The
kernels invert F(t) = r for v = t when r < 1/2 and for v = u = 1 - t
otherwise.  Their start inverts the leading term: s = (r / (k+1))^(1/k) on
the low side, s = sqrt(2 (1 - r) / (k (k+1))) on the high side, both as
exp2(e log2(a)).  It then multiplies s by rho(s), a degree-DEG polynomial fitted here to v / s.  The
fit is least squares, reweighted towards the smallest maximum relative
error.

Run `python -m paper_1010_2107_amd.gen_mass_start` to regenerate the header.
The script also reports the start error, and the error after the FP32
Newton step, emulated in numpy float32 arithmetic against a bisection
solution in float64.
"""
from __future__ import annotations

import os
from math import comb

import numpy as np

DEG = 5
KS = (2, 3, 4)
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "csrc", "vmc_mass_start.hpp")


def comp_coefs(k: int) -> np.ndarray:
    """Coefficients (index = power of u) of 1 - F(1 - u)."""
    c = np.zeros(k + 2)
    c[0] = 1.0
    for j in range(k + 1):
        c[j] -= (k + 1) * comb(k, j) * (-1) ** j
    for j in range(k + 2):
        c[j] += k * comb(k + 1, j) * (-1) ** j
    return c


def fit(k: int, deg: int = DEG):
    t = 0.5 - 0.5 * np.cos(np.linspace(0.0, np.pi, 800_001))
    t = t[(t > 1e-7) & (t < 1 - 1e-7)]
    u = 1.0 - t
    F = (k + 1) * t**k - k * t ** (k + 1)
    G = np.polynomial.polynomial.polyval(u, comp_coefs(k))  # 1 - F without cancellation
    lo = F < 0.5
    sides = []
    s_lo = (F[lo] / (k + 1)) ** (1.0 / k)
    sides.append((s_lo, t[lo] / s_lo))
    s_hi = np.sqrt(2.0 * G[~lo] / (k * (k + 1)))
    sides.append((s_hi, u[~lo] / s_hi))
    coefs = []
    for s, rho in sides:
        w = np.ones_like(s)
        for _ in range(30):
            c = np.polynomial.polynomial.polyfit(s, rho, deg, w=np.sqrt(w))
            e = np.abs(np.polynomial.polynomial.polyval(s, c) / rho - 1.0)
            w = w * (1.0 + 50.0 * e / e.max())
            w /= w.mean()
        coefs.append(c)
    return coefs[0], coefs[1]


def bisect(k: int, r: np.ndarray) -> np.ndarray:
    a, b = np.zeros_like(r), np.ones_like(r)
    for _ in range(64):
        m = 0.5 * (a + b)
        F = (k + 1) * m**k - k * m ** (k + 1)
        a, b = np.where(F < r, m, a), np.where(F < r, b, m)
    return 0.5 * (a + b)


def emulate_f32(k: int, a: np.ndarray, b: np.ndarray, r: np.ndarray, iters: int):
    """The kernels' FP32 steps, in numpy float32 arithmetic."""
    T = np.float32
    r = r.astype(T)
    lo = r < T(0.5)
    q = (T(1) - r).astype(T)
    arg = np.where(lo, r * T(1.0 / (k + 1)), q * T(2.0 / (k * (k + 1)))).astype(T)
    with np.errstate(all="ignore"):
        s = np.where(arg > 0, np.exp2(np.log2(arg) * np.where(lo, T(1.0 / k), T(0.5))), T(0)).astype(T)
    rl, rh = np.full_like(r, T(a[DEG])), np.full_like(r, T(b[DEG]))
    for j in range(DEG - 1, -1, -1):
        rl = (rl * s + T(a[j])).astype(T)
        rh = (rh * s + T(b[j])).astype(T)
    v = np.clip(s * np.where(lo, rl, rh), 0, 1).astype(T)
    v0 = v.copy()
    c = comp_coefs(k)
    h = [np.where(lo, T(k + 1.0 if j == k - 2 else (-k if j == k - 1 else 0.0)), T(c[j + 2])).astype(T)
         for j in range(k)]
    target = np.where(lo, r, q).astype(T)
    for _ in range(iters):
        H, Hd = h[k - 1], np.zeros_like(v)
        for j in range(k - 2, -1, -1):
            Hd = (Hd * v + H).astype(T)
            H = (H * v + h[j]).astype(T)
        res = ((v * v).astype(T) * H - target).astype(T)
        dP = (v * (v * Hd + T(2) * H)).astype(T)
        with np.errstate(all="ignore"):
            step = (res * (T(1) / np.maximum(dP, T(1e-30)))).astype(T)
        v = np.clip(v - step, 0, 1).astype(T)
    t = np.where(lo, v, T(1) - v).astype(T)
    u = np.where(lo, T(1) - v, v).astype(T)
    return v0, t, u


def report(k: int, a: np.ndarray, b: np.ndarray) -> str:
    rng = np.random.default_rng(0)
    r = np.concatenate([rng.random(200_000), np.logspace(-7, 0, 3000, endpoint=False),
                        1 - np.logspace(-7, -0.3, 3000)]).astype(np.float32).astype(np.float64)
    ex = bisect(k, r)
    v0, t, u = emulate_f32(k, a, b, r, 1)
    lo = r < 0.5
    vex = np.where(lo, ex, 1 - ex)
    e0 = np.abs(v0 - vex) / np.maximum(vex, 1e-300)
    et = np.abs(t - ex) / np.maximum(ex, 1e-300)
    eu = np.abs(u - (1 - ex)) / np.maximum(1 - ex, 1e-300)
    return (f"k={k}: start max rel err {e0[vex > 0].max():.2e}; after one FP32 Newton step "
            f"t {et[ex > 0].max():.2e}, u {eu[ex < 1].max():.2e}")


def main() -> None:
    rows_lo, rows_hi, notes = [], [], []
    for k in KS:
        a, b = fit(k)
        rows_lo.append(a)
        rows_hi.append(b)
        notes.append(report(k, a, b))
    def table(name, rows):
        lines = [f"constexpr double {name}[{len(KS)}][{DEG + 1}] = {{"]
        for k, row in zip(KS, rows):
            lines.append("    {" + ", ".join(f"{x:.17e}" for x in row) + f"}},  // k = {k}")
        lines.append("};")
        return "\n".join(lines)
    text = f"""// vmc_mass_start.hpp -- written by paper_1010_2107_amd/gen_mass_start.py; do not edit.
//
// Start of the Newton inversion of the RAMBO-on-diet mass fraction CDF
// F(t) = (k+1) t^k - k t^(k+1): v ~ s rho(s), with v = t, s = (r/(k+1))^(1/k)
// for r < 1/2 and v = 1 - t, s = sqrt(2 (1 - r) / (k (k+1))) otherwise;
// rho is a degree-{DEG} polynomial fitted to v / s (coefficients by ascending
// power, rows k = {KS[0]}..{KS[-1]}).
""" + "".join(f"//   {n}\n" for n in notes) + f"""#pragma once

namespace vmc {{

constexpr int kMassStartDeg = {DEG};
constexpr int kMassStartMinK = {KS[0]};
constexpr int kMassStartMaxK = {KS[-1]};
{table("kMassStartLo", rows_lo)}
{table("kMassStartHi", rows_hi)}

}}  // namespace vmc
"""
    with open(OUT, "w") as f:
        f.write(text)
    print("\n".join(notes))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
