// vmc_phys.hpp -- physics-shaped integrand: pp -> W(-> e nu) + NP partons.
//
// The paper integrates u dbar -> W+(-> mu+ nu) + n gluons over a
// 3(n+2)-4 dimensional phase space plus 2 parton momentum fractions
// (Sec. 5, eq. 1).  Its amplitudes (HELAS/HEGET) and PDFs (CTEQ6L1) are
// replaced by a toy with the same shape:
//   x0, x1      -> parton fractions: ln xa = L (1 - x0), ln xb = L x0 (1 - x1),
//                  L = ln tau0, tau0 = ((1 + NP) pTmin)^2 / S, covering
//                  xa xb >= tau0 once with Jacobian L^2 x0 xa xb;
//   flux        -> F(xa) F(xb), F(x) = x^-1.5 (1 - x)^3;
//   x2..x_{D-1} -> n = NP + 2 massless momenta in the partonic rest frame
//                  with the "RAMBO on diet" construction (Plaetzer,
//                  arXiv:1308.2922): n-2 mass fractions, then one direction
//                  (cos theta, phi) per two-body step;
//   cuts        -> pT > pTmin, |eta_lab| < etamax for partons and e, and
//                  Delta R > dRmin for every pair of them (nu unconstrained);
//   |M|^2       -> g^(2 NP) BW(m_enu^2) 2 s^4 sum_sigma 1/prod s_{sigma_i
//                  sigma_i+1} over the distinct cyclic orders of the coloured
//                  set {a, b, partons} (Parke-Taylor denominators);
//   f           -> flux x Jacobian x |M|^2 x V_n(s) / (2 s), with V_n the
//                  massless n-body phase-space volume.
// Per-sample arithmetic is in T; constants are prepared in double in setup().
#pragma once

#include "vmc_device.hpp"
#include "vmc_mass_start.hpp"

namespace vmc {

// ---------------------------------------------------------------------------
// Colour-ordered denominators: the sum over the (M-1)!/2 distinct cyclic
// orders (up to rotation and reflection) of M objects.
// ---------------------------------------------------------------------------
constexpr int factorial(int n) { return n <= 1 ? 1 : n * factorial(n - 1); }

// Sum over the distinct cyclic orders of prod y along the cycle, by dynamic
// programming over subsets: P[S][v] is the sum of the products along all
// paths that start at object 0, visit exactly the objects in S and end at v.
// Closing every full path back to 0 counts each undirected cycle twice (once
// per direction), hence the factor 1/2.  For six objects this is 165
// multiply-adds instead of ~290 operations for the 60 explicit products.
template <int M, typename T>
__device__ __forceinline__ T cycle_sum(const T (&y)[M][M]) {
  constexpr int K = M - 1;  // objects 1..M-1, bit b <-> object b+1
  constexpr int FULL = (1 << K) - 1;
  T P[1 << K][K];
#pragma unroll
  for (int mask = 1; mask <= FULL; ++mask) {
#pragma unroll
    for (int v = 0; v < K; ++v) {
      if (!((mask >> v) & 1)) continue;
      const int prev = mask ^ (1 << v);
      if (prev == 0) {
        P[mask][v] = y[0][v + 1];
      } else {
        T acc = T(0);
        bool first = true;
#pragma unroll
        for (int u = 0; u < K; ++u) {
          if (!((prev >> u) & 1)) continue;
          acc = first ? P[prev][u] * y[u + 1][v + 1] : fma(P[prev][u], y[u + 1][v + 1], acc);
          first = false;
        }
        P[mask][v] = acc;
      }
    }
  }
  T total = P[FULL][0] * y[1][0];
#pragma unroll
  for (int v = 1; v < K; ++v) total = fma(P[FULL][v], y[v + 1][0], total);
  return T(0.5) * total;
}

// Six objects, meet in the middle.  Every cycle through object 0 has one
// object z opposite 0, and its two arcs are paths 0 -> z through two objects
// each.  With A(z, {x, w}) = y_xw (y_0x y_wz + y_0w y_xz), the sum over both
// such paths, the cycle sum is the sum over z and over the three ways to
// split the other four objects into two pairs {T, T'} of A(z, T) A(z, T').
// Each undirected cycle appears once (the split is unordered): 105
// operations instead of the 165 of the subset recursion.
template <typename T>
__device__ __forceinline__ T cycle_sum6(const T (&y)[6][6]) {
  T total = T(0);
#pragma unroll
  for (int z = 1; z <= 5; ++z) {
    int o[4];
    int n = 0;
#pragma unroll
    for (int v = 1; v <= 5; ++v)
      if (v != z) o[n++] = v;
    auto arc = [&](int x, int w) { return y[x][w] * fma(y[0][x], y[w][z], y[0][w] * y[x][z]); };
    total = fma(arc(o[0], o[1]), arc(o[2], o[3]), total);
    total = fma(arc(o[0], o[2]), arc(o[1], o[3]), total);
    total = fma(arc(o[0], o[3]), arc(o[1], o[2]), total);
  }
  return total;
}

// ---------------------------------------------------------------------------
// Mass step of RAMBO on diet: the fraction t = M_i^2 / M_{i-1}^2 has CDF
// F(t) = (k+1) t^k - k t^(k+1), k = n - i.  The inversion F(t) = r works on
// v = t for r < 1/2 and on v = u = 1 - t otherwise.  On the high side the
// residual is (1 - F(1-u)) - (1 - r), with 1 - F(1-u) written as a
// polynomial in u that starts at u^2, so that no low-order terms cancel.
// On both sides the residual is v^2 H(v) - target, H of degree k-1, and each
// lane picks its coefficients once (the FP64 build's steps; the FP32 build's
// one step has an FP64 residual, which needs no such care, and takes it in
// t on both sides).  The start inverts the leading term and
// corrects it with a fitted polynomial (vmc_mass_start.hpp); its relative
// error is below 1.5e-4, so one Newton step reaches FP32 round-off and
// three reach FP64 round-off.  Returns t and u = 1 - t.
// ---------------------------------------------------------------------------
template <int K>
constexpr double binom(int n, int j) {
  double r = 1;
  for (int i = 1; i <= j; ++i) r = r * (n - j + i) / i;
  return r;
}

// coefficient of u^j in 1 - F(1-u)
template <int K>
constexpr double comp_coef(int j) {
  double c = (j == 0) ? 1.0 : 0.0;
  c -= (K + 1) * binom<K>(K, j) * ((j & 1) ? -1.0 : 1.0) * (j <= K ? 1.0 : 0.0);
  c += K * binom<K>(K + 1, j) * ((j & 1) ? -1.0 : 1.0);
  return c;
}

// coefficient of t^(j+2) in F(t)
template <int K>
constexpr double low_coef(int j) {
  return j == K - 2 ? K + 1.0 : (j == K - 1 ? -static_cast<double>(K) : 0.0);
}

// t, u = 1 - t, and t in FP64 (the resonance variable is formed from it)
template <typename T>
struct TU {
  T t, u;
  double t64;
};

// In the FP32 build the Newton step evaluates the residual in FP64: the FP32
// residual is limited by its own rounding (final error 1-3 ulps), while the
// FP64 one leaves the step's quadratic error, (K-1)/2 times the square of
// the start's 1.5e-4, i.e. 3e-8 relative.  The derivative and its
// reciprocal stay FP32 (their error enters the step multiplied by the
// start's error).  The FP64 build takes three all-FP64 steps.
template <int K, typename T>
__device__ __forceinline__ TU<T> mass_fraction(T r) {
  constexpr bool F32 = sizeof(T) == 4;
  if constexpr (K == 1) {
    const T s = vsqrt(T(1) - r);
    const T t = r * vrcp(T(1) + s);
    if constexpr (!F32) {
      return TU<T>{t, s, t};
    } else {
      // one step on F(t) = 2t - t^2 = r (low side) or on u^2 = 1 - r (high side, u = 1 - t)
      const double rd = static_cast<double>(r);
      const double inv = static_cast<double>(vrcp(T(2) * s));
      double t64;
      if (r < T(0.5)) {
        const double tt = static_cast<double>(t);
        t64 = tt - fma(tt, 2.0 - tt, -rd) * inv;
      } else {
        const double uu = static_cast<double>(s);
        t64 = 1.0 - (uu - fma(uu, uu, rd - 1.0) * inv);
      }
      return TU<T>{static_cast<T>(t64), static_cast<T>(1.0 - t64), t64};
    }
  } else {
    static_assert(K >= kMassStartMinK && K <= kMassStartMaxK, "no start polynomial for this k");
    constexpr int ITERS = F32 ? 1 : 3;
    constexpr int row = K - kMassStartMinK;
    const bool lo = r < T(0.5);
    const T q = T(1) - r;  // exact for r >= 1/2
    // s = (r / (K+1))^(1/K) or (2 q / (K (K+1)))^(1/2): square roots where
    // both sides' powers are roots of two, else one log2 and one exp2
    // (a = 0 gives log2 = -inf and s = 0)
    const T a = lo ? r * T(1.0 / (K + 1)) : q * T(2.0 / (K * (K + 1)));
    T s;
    if constexpr (K == 2) {
      s = vsqrt(a);
    } else if constexpr (K == 4) {
      const T sa = vsqrt(a);
      s = lo ? vsqrt(sa) : sa;
    } else {
      s = vexp2_fast(vlog2_fast(a) * (lo ? T(1.0 / K) : T(0.5)));
    }
    T rl = T(kMassStartLo[row][kMassStartDeg]), rh = T(kMassStartHi[row][kMassStartDeg]);
#pragma unroll
    for (int j = kMassStartDeg - 1; j >= 0; --j) {
      rl = fma(rl, s, T(kMassStartLo[row][j]));
      rh = fma(rh, s, T(kMassStartHi[row][j]));
    }
    T v = fmin(s * (lo ? rl : rh), T(1));
    const T target = lo ? r : q;
    if constexpr (F32) {
      // The step in t on both sides: t = v or 1 - v (exact in FP64), the
      // residual F(t) - r = t^K ((K+1) - K t) - r in FP64, the derivative
      // F'(t) = K (K+1) t^(K-1) (1 - t) in FP32.  Near t = 1, F(t) rounds to
      // an absolute 6e-16, which is 5e-9 of the smallest 1 - r of an FP32 r
      // (2^-24); the step's own error dominates.
      const double vd = static_cast<double>(v);
      const double td = lo ? vd : 1.0 - vd;
      double tk = td;
#pragma unroll
      for (int j = 1; j < K; ++j) tk *= td;
      const double res = fma(tk, fma(-static_cast<double>(K), td, K + 1.0), -static_cast<double>(r));
      const T om = T(1) - v;
      const T tt = lo ? v : om, uu = lo ? om : v;
      T tp = T(K * (K + 1));
#pragma unroll
      for (int j = 0; j < K - 1; ++j) tp *= tt;
      const T dP = tp * uu;  // > 0 inside (0, 1); 0 at t = 0 or 1, where res = 0
      double t64 = td - res * static_cast<double>(vrcp(fmax(dP, T(1e-30))));
      t64 = fmin(fmax(t64, 0.0), 1.0);
      return TU<T>{static_cast<T>(t64), static_cast<T>(1.0 - t64), t64};
    } else {
      T h[K];
#pragma unroll
      for (int j = 0; j < K; ++j) h[j] = lo ? T(low_coef<K>(j)) : T(comp_coef<K>(j + 2));
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        T H = h[K - 1], Hd = T(0);
#pragma unroll
        for (int j = K - 2; j >= 0; --j) {
          Hd = fma(Hd, v, H);
          H = fma(H, v, h[j]);
        }
        const T res = fma(v * v, H, -target);
        const T dP = v * fma(v, Hd, T(2) * H);  // > 0 inside (0, 1]; 0 at v = 0 where res = 0
        v = fmin(fmax(v - res * vrcp(fmax(dP, T(1e-30))), T(0)), T(1));
      }
      return lo ? TU<T>{v, T(1) - v, v} : TU<T>{T(1) - v, v, T(1) - v};
    }
  }
}

// Boost v, given in the rest frame of a system of mass M, to the frame
// where that system has four-momentum (E, P).
template <typename T>
__device__ __forceinline__ void boost(const T (&Q)[4], T invM, T invEM, const T (&v)[4], T (&out)[4]) {
  const T pdot = Q[1] * v[1] + Q[2] * v[2] + Q[3] * v[3];
  const T e = (Q[0] * v[0] + pdot) * invM;
  const T f = fma(pdot, invEM, v[0]) * invM;
  out[0] = e;
  out[1] = fma(f, Q[1], v[1]);
  out[2] = fma(f, Q[2], v[2]);
  out[3] = fma(f, Q[3], v[3]);
}


__device__ __forceinline__ int ilogb_(float x) { return __builtin_amdgcn_frexp_expf(x) - 1; }
__device__ __forceinline__ int ilogb_(double x) { return __builtin_amdgcn_frexp_exp(x) - 1; }
__device__ __forceinline__ float ldexp_(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
__device__ __forceinline__ double ldexp_(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }

// The resonance variable in FP64.  The Breit-Wigner factor depends on
// m^2 - M^2, and its logarithmic slope in m^2 reaches m^2 / (M Gamma), about
// 38 for the W: a relative error of m^2 reaches the weight 38 times larger.
// In FP32 the partonic energy s = S exp(L (1 - x0 x1)) alone carries up to
// 2e-6 (the exponent's argument, up to |ln tau0| ~ 11, is rounded) and each
// mass fraction 1e-7 to 2e-7, which would put errors of up to 1e-4 into the
// heaviest weights.  The FP32 build therefore forms m^2 = s t_2 ... t_{n-1}
// in FP64 from the same FP32 point: s with an FP64 exponential, each t_i
// from the Newton step with the FP64 residual (mass_fraction), the product
// in FP64, and dm = m^2 - M^2 rounded once to FP32.  Everything else (the
// momenta, cuts and matrix element) stays FP32.
struct Resonance64 {
  double m2;   // in: s; then s t_2 ... t_i
  double Mv2;  // M^2
  float dm;    // out: m^2 - M^2 of the last pair
};

template <int NOUT, int X0, int I, bool RES64, typename T, int D>
__device__ __forceinline__ void mass_chain(const T (&x)[D], T (&Mi)[NOUT + 1], T (&Ui)[NOUT + 1],
                                           Resonance64& res) {
  if constexpr (I <= NOUT - 1) {
    const TU<T> tu = mass_fraction<NOUT - I, T>(x[X0 + I - 2]);
    Mi[I] = Mi[I - 1] * vsqrt(tu.t);
    Ui[I] = tu.u;
    if constexpr (RES64 && I < NOUT - 1) res.m2 *= tu.t64;
    if constexpr (RES64 && I == NOUT - 1) {  // the last pair: m^2 - M^2, its product fused
      float dm = static_cast<float>(fma(res.m2, tu.t64, -res.Mv2));
      asm volatile("" : "+v"(dm));  // formed here, where its inputs are live anyway
      res.dm = dm;
    }
    mass_chain<NOUT, X0, I + 1, RES64>(x, Mi, Ui, res);
  } else if constexpr (RES64 && NOUT == 2) {  // no mass step: m^2 = s
    float dm = static_cast<float>(res.m2 - res.Mv2);
    asm volatile("" : "+v"(dm));
    res.dm = dm;
  }
}

// RAMBO on diet (Plaetzer, arXiv:1308.2922): NOUT massless momenta in the
// rest frame of a system of mass rs from x[X0 .. X0 + 3 NOUT - 5]: first
// the masses M_2 > ... > M_{NOUT-1} (x[X0 + i - 2] fixes M_i), then one
// direction (cos theta, phi) per two-body step i = 1..NOUT-1: the massless
// momentum of step i is boosted by the current Q_i, and the recoiling
// system is what remains of Q_i (the boost is linear and takes Q_i's rest
// momentum to Q_i itself, so boosting the recoil gives Q_i - p_i).
// Mi[1..NOUT] and Ui[i] = 1 - M_i^2 / M_{i-1}^2 are returned with the
// momenta p[0..NOUT-1].
// RES64: also form the resonance variable in FP64 (res.m2 = s on entry).
template <int NOUT, int X0, bool RES64, typename T, int D>
__device__ __forceinline__ void rambo_diet(const T (&x)[D], T rs, T (&Mi)[NOUT + 1], T (&Ui)[NOUT + 1],
                                           T (&p)[NOUT][4], Resonance64& res) {
  Mi[1] = rs;
  Ui[1] = T(0);
  mass_chain<NOUT, X0, 2, RES64>(x, Mi, Ui, res);
  Mi[NOUT] = T(0);
  Ui[NOUT] = T(1);
  T Q[4] = {rs, T(0), T(0), T(0)};
#pragma unroll
  for (int i = 1; i <= NOUT - 1; ++i) {
    const T q = T(0.5) * Mi[i] * Ui[i + 1];  // (M_i^2 - M_{i+1}^2) / (2 M_i)
    const T rc = x[X0 + NOUT - 2 + 2 * i - 2];
    const T rp = x[X0 + NOUT - 2 + 2 * i - 1];
    const T cth = fma(T(2), rc, T(-1));
    const T sth = vsqrt(rc * fma(T(-4), rc, T(4)));  // 2 sqrt(rc (1 - rc))
    T sp, cp;
    vsincos2pi(rp, sp, cp);
    const T nx = sth * cp, ny = sth * sp, nz = cth;
    const T pr[4] = {q, q * nx, q * ny, q * nz};
    if (i == 1) {
      p[0][0] = q;
      Q[0] = Mi[1] - q;
#pragma unroll
      for (int c = 1; c < 4; ++c) {
        p[0][c] = pr[c];
        Q[c] = -pr[c];
      }
    } else {
      const T iM = vrcp(Mi[i]);
      const T iEM = vrcp(Q[0] + Mi[i]);
      boost(Q, iM, iEM, pr, p[i - 1]);
#pragma unroll
      for (int c = 0; c < 4; ++c) Q[c] -= p[i - 1][c];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) p[NOUT - 1][c] = Q[c];
}

// e^a for a <= 0 of moderate size (here a >= ln tau0 > -30), with the
// argument reduction in FP64 and the reduced exponential in FP32: with
// z = a log2 e = n + f, n = rint(z), |f| <= 1/2, e^a = 2^n 2^f, where 2^f
// comes from the hardware exp2 (about 1 ulp, 6e-8) of f rounded to FP32
// (absolute error below 3e-8, i.e. 2e-8 relative in 2^f).  The FP32 path
// rounded the whole argument instead, up to |ln tau0| ~ 11 in size, which
// alone made 7e-7 relative error in the partonic energy.
__device__ __forceinline__ double exp_neg_fp64(double a) {
  const double z = a * 1.4426950408889634;
  const double n = rint(z);
  const float e = __builtin_amdgcn_exp2f(static_cast<float>(z - n));
  return __builtin_amdgcn_ldexp(static_cast<double>(e), static_cast<int>(n));
}

// The partonic energy s = S exp(L (1 - x0 x1)) in FP64 from the FP32 point
// (x0 x1 and 1 - x0 x1 are exact in FP64); L = ln tau0 and S the collider
// energy squared, each given as an FP32 (high, low) pair.
__device__ __forceinline__ double shat_fp64(float x0, float x1, float Lh, float Ll, float Sh, float Sl) {
  const double L = static_cast<double>(Lh) + static_cast<double>(Ll);
  const double S = static_cast<double>(Sh) + static_cast<double>(Sl);
  return S * exp_neg_fp64(L * (1.0 - static_cast<double>(x0) * static_cast<double>(x1)));
}

// Massless light-cone components E +- pz, rapidity and pT of a momentum:
// the larger component directly, the smaller as pT^2 / larger; rapidity =
// +-ln(larger / pT).
template <typename T>
struct LightCone {
  T pt2, pt, rpt, rpt2, big, lp, lm, eta;
};
template <typename T>
__device__ __forceinline__ LightCone<T> light_cone(const T (&v)[4]) {
  LightCone<T> r;
  r.pt2 = v[1] * v[1] + v[2] * v[2];
  const T e = v[0], z = v[3];
  const T big = e + fabs(z);
  const T small = r.pt2 * vrcp(big);
  const T rpt = vrsqrt(r.pt2);
  const T ya = vlog_fast(big * rpt);
  r.big = big;
  r.lp = z > T(0) ? big : small;
  r.lm = z > T(0) ? small : big;
  r.eta = copysign(ya, z);
  r.pt = r.pt2 * rpt;
  r.rpt = rpt;
  r.rpt2 = rpt * rpt;
  return r;
}

template <typename TT, int NP, bool FULL>
struct WJetsF {
  using T = TT;
  static constexpr int NOUT = NP + 2;  // final-state particles
  static constexpr int D = 3 * NP + 4;
  static constexpr int NGRAD = FULL ? 3 : 0;
  static constexpr int NTHETA = FULL ? 7 : 2;
  static constexpr int MC = NP + 2;  // coloured: a, b and the partons

  T L, LL, sqrtS, pre;
  T M, Mv2, MG, MGpi, M2G2, invM, invG, two_np_over_g, twoMG2;
  T ptmin2, etamax, dr2;
  // FP64 constants of the resonance variable as (high, low) FP32 pairs (a
  // double member makes the compiler keep the whole functor in registers)
  T L_lo, S_hi, S_lo, Mv2_lo;

  __device__ void setup(const double* th) {
    const double pi = 3.14159265358979323846;
    const double sS = FULL ? th[3] : th[0];
    const double ptm = FULL ? th[4] : th[1];
    const double S = sS * sS;
    const double tau0 = ((1.0 + NP) * ptm) * ((1.0 + NP) * ptm) / S;
    const double Ld = log(tau0);
    // V_n(s) = cV s^(n-2), cV = (2pi)^(4-3n) (pi/2)^(n-1) / ((n-1)! (n-2)!)
    const double cV = pow(2.0 * pi, 4.0 - 3.0 * NOUT) * pow(pi / 2.0, NOUT - 1) /
                      (static_cast<double>(factorial(NOUT - 1)) * factorial(NOUT - 2));
    L = static_cast<T>(Ld);
    LL = static_cast<T>(Ld * Ld);
    sqrtS = static_cast<T>(sS);
    ptmin2 = static_cast<T>(ptm * ptm);
    L_lo = static_cast<T>(Ld - static_cast<double>(L));
    S_hi = static_cast<T>(S);
    S_lo = static_cast<T>(S - static_cast<double>(S_hi));
    Mv2_lo = FULL ? static_cast<T>(th[0] * th[0] - static_cast<double>(static_cast<T>(th[0] * th[0]))) : T(0);
    if (FULL) {
      const double Md = th[0], Gd = th[1], gd = th[2];
      // f = flux Jx g^(2NP) BW [2 s^4 sum 1/prod s] cV s^(n-2) / (2 s)
      pre = static_cast<T>(cV * pow(gd, 2.0 * NP));
      M = static_cast<T>(Md);
      Mv2 = static_cast<T>(Md * Md);
      MG = static_cast<T>(Md * Gd);
      MGpi = static_cast<T>(Md * Gd / pi);
      M2G2 = static_cast<T>(Md * Md * Gd * Gd);
      invM = static_cast<T>(1.0 / Md);
      invG = static_cast<T>(1.0 / Gd);
      two_np_over_g = static_cast<T>(2.0 * NP / gd);
      twoMG2 = static_cast<T>(2.0 * Md * Gd * Gd);
      etamax = static_cast<T>(th[5]);
      dr2 = static_cast<T>(th[6] * th[6]);
    } else {
      pre = static_cast<T>(cV / 2.0);
    }
  }

  // The evaluation in two stages so that a kernel can queue the samples
  // that pass the cuts and run everything else on full waves: stage 1 maps
  // x to momenta and applies the cuts, keeping what the rest needs (per
  // parton E + |pz| signed as pz, 1 / pT^2 and the transverse momentum;
  // x0, m_enu^2 - M^2 and ln xa, ln xb, from which stage 2 forms sqrt(s)
  // again, bit for bit, as well as the flux factor);
  // stage 2 forms the invariants of the coloured set, the prefactor, the
  // flux, |M|^2 and f.  Most samples fail the cuts (about 60 % for four
  // partons), so work moved from stage 1 to stage 2 is done on fewer lanes.
  struct State {
    T bp[NP];    // E + |pz|, with the sign of pz (the larger light-cone component)
    T rpt2[NP];  // 1 / pT^2
    T px[NP], py[NP];
    T x0;
    T dm;        // m_enu^2 - M^2
    T la, lb;    // ln xa, ln xb: the flux factor is ((1 - xa)(1 - xb))^3
  };
  static constexpr int kStateWords = 4 * NP + 4;
  static constexpr bool kStaged = FULL && sizeof(T) == 4;  // the queue holds FP32

  __device__ __forceinline__ static void store_state(const State& st, float* q, int stride, int e) {
    int k = 0;
    auto put = [&](T v) { q[(k++) * stride + e] = static_cast<float>(v); };
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      put(st.bp[j]);
      put(st.rpt2[j]);
      put(st.px[j]);
      put(st.py[j]);
    }
    put(st.x0);
    put(st.dm);
    put(st.la);
    put(st.lb);
  }
  __device__ __forceinline__ static State load_state(const float* q, int stride, int e) {
    State st;
    int k = 0;
    auto get = [&]() { return static_cast<T>(q[(k++) * stride + e]); };
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      st.bp[j] = get();
      st.rpt2[j] = get();
      st.px[j] = get();
      st.py[j] = get();
    }
    st.x0 = get();
    st.dm = get();
    st.la = get();
    st.lb = get();
    return st;
  }

  // PDF map, phase space and cuts; false when the sample fails the cuts
  __device__ __forceinline__ bool stage1(const T (&x)[D], State& st) const {
    // parton fractions and flux x Jacobian = L^2 x0 tau^-1/2 ((1-xa)(1-xb))^3;
    // the last factor is formed in stage 2
    const T la = L * (T(1) - x[0]);
    const T lb = L * x[0] * (T(1) - x[1]);
    const T ltau = la + lb;
    const T h = vexp2_fast(ltau * T(0.5 * 1.4426950408889634));  // sqrt(tau)
    const T rs = sqrtS * h;           // sqrt(s)
    const T dl = la - lb;  // twice the boost rapidity y_b
    // ---- RAMBO on diet: masses M_1 = sqrt(s) > M_2 > ... > M_{n-1} > M_n = 0
    T Mi[NOUT + 1], Ui[NOUT + 1];
    T p[NOUT][4];
    constexpr bool RES64 = sizeof(T) == 4;
    Resonance64 res{};
    if constexpr (RES64) {
      res.m2 = shat_fp64(x[0], x[1], L, L_lo, S_hi, S_lo);
      res.Mv2 = static_cast<double>(Mv2) + static_cast<double>(Mv2_lo);
    }
    rambo_diet<NOUT, 2, RES64>(x, rs, Mi, Ui, p, res);
    if constexpr (RES64) st.dm = res.dm;

    // ---- visible particles: partons 0..NP-1 and the electron NP
    constexpr int NV = NP + 1;
    T pt2[NV], eta[NV], ux[NV], uy[NV];
    // the pT and rapidity cuts on the smallest pT^2 and the largest |eta|;
    // fmin and fmax skip a NaN (degenerate momenta), which then fails the
    // Delta R test below (every visible particle is in a pair there)
    T pt2_min = T(0), yabs_max = T(0);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const LightCone<T> lc = light_cone(p[j]);
      pt2[j] = lc.pt2;
      eta[j] = lc.eta;
      if (j < NP) {
        st.bp[j] = p[j][3] > T(0) ? lc.big : -lc.big;
        st.rpt2[j] = lc.rpt2;
        st.px[j] = p[j][1];
        st.py[j] = p[j][2];
      }
      ux[j] = p[j][1] * lc.rpt;  // transverse direction
      uy[j] = p[j][2] * lc.rpt;
      const T ya = fabs(fma(T(0.5), dl, eta[j]));  // |eta + y_b|
      pt2_min = j == 0 ? pt2[0] : fmin(pt2_min, pt2[j]);
      yabs_max = j == 0 ? ya : fmax(yabs_max, ya);
    }
    bool pass = (pt2_min > ptmin2) & (yabs_max < etamax);
    // Delta R > R: either Delta eta^2 >= R^2, or cos(Delta phi) < cos(phi0)
    // with phi0 = sqrt(R^2 - Delta eta^2) <= R.  For Delta eta^2 >= R^2 the
    // series below is at least 1 and cos(Delta phi) never exceeds 1, so one
    // comparison covers both cases.  cos(phi0) from its Taylor series in
    // z = phi0^2: in FP64 terms to z^6 (remainder below 1e-16 for R <= 0.4),
    // in FP32 to z^3 (for R <= 0.4 the z^4 term is below 1.6e-8, a third of
    // an ulp of the cosine).
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = i + 1; j < NV; ++j) {
        const T de = eta[i] - eta[j];
        const T z = dr2 - de * de;
        T c;
        if constexpr (sizeof(T) == 8) {
          c = T(1.0 / 479001600.0);
          c = fma(c, -z, T(1.0 / 3628800.0));
          c = fma(c, -z, T(1.0 / 40320.0));
          c = fma(c, -z, T(1.0 / 720.0));
        } else {
          c = T(1.0 / 720.0);
        }
        c = fma(c, -z, T(1.0 / 24.0));
        c = fma(c, -z, T(1.0 / 2.0));
        c = fma(c, -z, T(1));
        pass = pass & (fma(ux[i], ux[j], uy[i] * uy[j]) < c);
      }
    if constexpr (sizeof(T) == 8) st.dm = fma(Mi[NOUT - 1], Mi[NOUT - 1], -Mv2);
    st.x0 = x[0];
    st.la = la;
    st.lb = lb;
    return pass;
  }

  // |M|^2 and f of a sample that passed the cuts
  template <bool GRAD>
  __device__ __forceinline__ T stage2(const State& st, T (&g)[NGRAD + 1]) const {
    // ---- light-cone components E +- pz of the partons: the larger one is
    // kept, the smaller is pT^2 over it
    T lp[NP], lm[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const T big = fabs(st.bp[j]);
      const T small = vrcp(st.rpt2[j] * big);
      lp[j] = st.bp[j] > T(0) ? big : small;
      lm[j] = st.bp[j] > T(0) ? small : big;
    }
    // ---- invariants of the coloured set, scaled: y = c / s_kl with c a power
    // of two near s^(4/m), so s^4 / prod s = (s^4 / c^m) prod y exactly
    // sqrt(s) as stage 1 formed it (the same operations on the same values)
    const T rs = sqrtS * vexp2_fast((st.la + st.lb) * T(0.5 * 1.4426950408889634));
    const T shat = rs * rs, rrs = vrcp(rs);
    const int ce = (4 * ilogb_(shat)) / MC;
    const T c = ldexp_(T(1), ce);
    const T crs = c * rrs;
    T y[MC][MC];
    y[0][1] = y[1][0] = crs * rrs;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      y[0][2 + j] = y[2 + j][0] = crs * lp[j] * st.rpt2[j];  // c / s_aj, s_aj = sqrt(s)(E - pz)
      y[1][2 + j] = y[2 + j][1] = crs * lm[j] * st.rpt2[j];  // c / s_bj
    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = i + 1; j < NP; ++j) {
        const T sij = fma(lp[i], lm[j], lm[i] * lp[j]) - T(2) * (st.px[i] * st.px[j] + st.py[i] * st.py[j]);
        y[2 + i][2 + j] = y[2 + j][2 + i] = c * vrcp(sij);
      }
#pragma unroll
    for (int i = 0; i < MC; ++i) y[i][i] = T(0);
    // prefactor pre s^(n-3) L^2 x0 / sqrt(tau) s^4 / c^m (1 / sqrt(tau) =
    // sqrt(S) / sqrt(s))
    T spow = T(1);
#pragma unroll
    for (int i = 0; i < NOUT - 3; ++i) spow *= shat;
    const T s2 = shat * shat;
    const T pref = ((pre * spow) * (LL * st.x0 * (sqrtS * rrs))) * ldexp_(s2 * s2, -ce * MC);
    T ptsum;
    if constexpr (MC == 6) {
      ptsum = cycle_sum6<T>(y);
    } else {
      ptsum = cycle_sum<MC, T>(y);
    }
    // ---- Breit-Wigner in m_enu^2 = M_{n-1}^2 (e nu are the last pair)
    const T dm = st.dm;
    const T invD = vrcp(fma(dm, dm, M2G2));
    const T om = vexpm1_fast(st.la) * vexpm1_fast(st.lb);  // (1 - xa)(1 - xb) without cancellation
    const T f = (pref * (om * om * om)) * (MGpi * invD) * ptsum;
    if (GRAD) {
      g[0] = f * (invM - fma(T(-4) * M, dm, twoMG2) * invD);
      g[1] = f * (invG - T(2) * M * MG * invD);
      g[2] = f * two_np_over_g;
    }
    return f;
  }

  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&g)[NGRAD + 1]) const {
    if constexpr (!FULL) {
      const T la = L * (T(1) - x[0]);
      const T lb = L * x[0] * (T(1) - x[1]);
      const T h = vexp2_fast((la + lb) * T(0.5 * 1.4426950408889634));
      const T shat = sqrtS * h * (sqrtS * h);
      const T om = vexpm1_fast(la) * vexpm1_fast(lb);
      const T fluxjac = LL * x[0] * (om * om * om) * vrcp(h);
      T spow = T(1);
#pragma unroll
      for (int i = 0; i < NOUT - 3; ++i) spow *= shat;
      return pre * fluxjac * spow;
    } else {
      State st;
      if (!stage1(x, st)) {
        if (GRAD) g[0] = g[1] = g[2] = T(0);
        return T(0);
      }
      return stage2<GRAD>(st, g);
    }
  }
};

template <typename T, int D>
using WJets = WJetsF<T, (D - 4) / 3, true>;
template <typename T, int D>
using PsVol = WJetsF<T, (D - 4) / 3, false>;

}  // namespace vmc
