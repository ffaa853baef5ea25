// vmc_whel.hpp -- the paper's process, u dbar -> W+(-> mu+ nu) + NG gluons
// (Kanzaki, arXiv:1010.2107, Sec. 5, eq. 1; Table 4: 1, 2 and 8 Feynman
// diagrams for NG = 0, 1, 2), from tree-level helicity amplitudes.
//
//   x0, x1          -> parton fractions and flux as for the W + partons toy
//                      (toy PDF F(x) = x^-1.5 (1-x)^3 for u and dbar);
//   x2..x_{3NG+3}   -> RAMBO on diet for g_1..g_NG, mu+, nu (so m_munu is
//                      the last mass of the chain);
//   x_{3NG+4}       -> the gluon helicities: one of the 2^NG configurations,
//                      weight 2^NG (quark and lepton helicities are fixed by
//                      the left-handed W coupling; the others vanish);
//   cuts            -> gluons pT > pTmin, |eta| < eta_g, Durham
//                      min(pT_i, pT_j) Delta R_ij > pTij between gluons; the
//                      muon pT > pTmin, |eta| < eta_mu; eta in the pp frame;
//   |M|^2           -> massless left-handed quark and lepton lines as chains
//                      of 2x2 blocks on Weyl spinors (vertex V: V.sigmabar,
//                      propagator P: P.sigma / P^2), colour-ordered
//                      amplitudes summed with the colour matrix; Feynman
//                      gauge, fixed g_W^2 = 4 sqrt2 G_F (80.4 GeV)^2;
//   f               -> flux x Jacobian x V_n(s) / (2 s) x (1/36) x 2^NG x |M|^2.
// theta = (M_W, Gamma_W, g_s, sqrtS, pTmin, eta_mu, eta_g, pTij); gradients
// with respect to the first three.
#pragma once

#include "vmc_phys.hpp"

namespace vmc {

template <typename T>
struct Cx {
  T r, i;
};
template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) {
  return {a.r + b.r, a.i + b.i};
}
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) {
  return {a.r - b.r, a.i - b.i};
}
template <typename T>
__device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}
template <typename T>
__device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) {
  return {s * a.r, s * a.i};
}
template <typename T>
__device__ __forceinline__ T norm2(Cx<T> a) {
  return fma(a.r, a.r, a.i * a.i);
}
// a b + c and s a + c with every product fused into its sum (the library is
// built so that only fusions written out like these happen, which keeps
// every kernel's rounding of this code the same)
template <typename T>
__device__ __forceinline__ Cx<T> cfma(Cx<T> a, Cx<T> b, Cx<T> c) {
  return {fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i))};
}
template <typename T>
__device__ __forceinline__ Cx<T> cfma(T s, Cx<T> a, Cx<T> c) {
  return {fma(s, a.r, c.r), fma(s, a.i, c.i)};
}

template <typename T>
struct Sp {  // a 2-component spinor
  Cx<T> a, b;
};
template <typename T>
__device__ __forceinline__ Sp<T> operator+(const Sp<T>& x, const Sp<T>& y) {
  return {x.a + y.a, x.b + y.b};
}
template <typename T>
__device__ __forceinline__ Sp<T> operator-(const Sp<T>& x, const Sp<T>& y) {
  return {x.a - y.a, x.b - y.b};
}
// A complex four-vector V held as its 2x2 block V.sigmabar =
// [[p, lo], [hi, m]] with p = V0 + V3, m = V0 - V3, lo = V1 - i V2,
// hi = V1 + i V2: the light-cone components are formed directly from
// their sources, never as differences of nearly equal V0 and V3 (which for
// momenta close to a beam lose up to (E / pT)^2 of their precision).
template <typename T>
struct SB {
  Cx<T> p, m, lo, hi;
};

// (V . sigmabar) x, and (V . sigmabar) x + y
template <typename T>
__device__ __forceinline__ Sp<T> sbar(const SB<T>& V, const Sp<T>& x) {
  return {cfma(V.lo, x.b, V.p * x.a), cfma(V.m, x.b, V.hi * x.a)};
}
template <typename T>
__device__ __forceinline__ Sp<T> sbar_add(const SB<T>& V, const Sp<T>& x, const Sp<T>& y) {
  return {cfma(V.lo, x.b, cfma(V.p, x.a, y.a)), cfma(V.m, x.b, cfma(V.hi, x.a, y.b))};
}
// first component only (the last vertex before v_L(p_dbar) = (r, 0)), and
// that plus c
template <typename T>
__device__ __forceinline__ Cx<T> sbar_top(const SB<T>& V, const Sp<T>& x) {
  return cfma(V.lo, x.b, V.p * x.a);
}
template <typename T>
__device__ __forceinline__ Cx<T> sbar_top_add(const SB<T>& V, const Sp<T>& x, Cx<T> c) {
  return cfma(V.lo, x.b, cfma(V.p, x.a, c));
}
// (V . sigmabar) (0, 1): the first vertex on u_L(p_u) = (0, r)
template <typename T>
__device__ __forceinline__ Sp<T> sbar_u(const SB<T>& V) {
  return {V.lo, V.m};
}
// A real momentum by its light-cone components P+ = P0 + P3, P- = P0 - P3
// and its transverse part.
template <typename T>
struct LC {
  T p, m, x, y;
};
// the propagator (P . sigma) x / P^2; every propagator here is space-like
// with P+ >= 0 >= P-, so P^2 = P+ P- - Px^2 - Py^2 adds terms of one sign
template <typename T>
__device__ __forceinline__ Sp<T> prop(const LC<T>& P, const Sp<T>& x) {
  const T inv = vrcp(fma(P.p, P.m, -fma(P.x, P.x, P.y * P.y)));
  const T m = P.m * inv, p = P.p * inv;
  const Cx<T> lo = {-P.x * inv, P.y * inv};   // -(P1 - i P2) / P^2
  const Cx<T> hi = {-P.x * inv, -P.y * inv};  // -(P1 + i P2) / P^2
  return {cfma(lo, x.b, m * x.a), cfma(p, x.b, hi * x.a)};
}
// light-cone components of a massless momentum: the larger of E +- pz
// directly, the smaller as pT^2 over it
template <typename T>
__device__ __forceinline__ LC<T> massless_lc(const T (&k)[4]) {
  const T big = k[0] + fabs(k[3]);
  const T small = fma(k[1], k[1], k[2] * k[2]) * vrcp(big);
  return k[3] > T(0) ? LC<T>{big, small, k[1], k[2]} : LC<T>{small, big, k[1], k[2]};
}

// left-chirality spinor of a massless momentum (p.sigmabar u = 0, |u|^2 = 2E)
template <typename T>
__device__ __forceinline__ Sp<T> weyl(const T (&p)[4]) {
  const T pp = p[0] + p[3], pm = p[0] - p[3];
  if (pp >= pm) {
    const T r = vrsqrt(pp);
    return {{-p[1] * r, p[2] * r}, {pp * r, T(0)}};
  }
  const T r = vrsqrt(pm);
  return {{pm * r, T(0)}, {-p[1] * r, -p[2] * r}};
}

template <typename TT, int NG>
struct WHelF {
  using T = TT;
  static constexpr int NOUT = NG + 2;  // g_1..g_NG, mu+, nu
  static constexpr int D = 3 * NG + 5;
  static constexpr int NGRAD = 3;
  static constexpr int NTHETA = 8;

  T L, LL, sqrtS, pre, ptmin2, eta_mu, eta_g, ptij2;
  T M, Mv2, M2G2, twoMG2, m2M2G, two_ng_over_g;
  T L_lo, S_hi, S_lo, Mv2_lo;  // FP64 constants of the resonance variable as FP32 (high, low) pairs

  __device__ void setup(const double* th) {
    const double pi = 3.14159265358979323846;
    const double Md = th[0], Gd = th[1], gs = th[2], sS = th[3], ptm = th[4];
    const double S = sS * sS;
    const double tau0 = ((1.0 + NG) * ptm) * ((1.0 + NG) * ptm) / S;
    const double Ld = log(tau0);
    const double cV = pow(2.0 * pi, 4.0 - 3.0 * NOUT) * pow(pi / 2.0, NOUT - 1) /
                      (static_cast<double>(factorial(NOUT - 1)) * factorial(NOUT - 2));
    const double gw2 = 4.0 * sqrt(2.0) * 1.1663787e-5 * 80.4 * 80.4;
    // f = flux Jx cV s^(n-2) / (2 s) (2^NG / 36) g_s^(2NG) (g_W^2/2)^2 |A|^2 / |D|^2,
    // |A|^2 = s |chain|^2 (the spinors of p_u and p_dbar contribute sqrt(s) each)
    pre = static_cast<T>(cV * 0.5 * (1 << NG) / 36.0 * pow(gs, 2.0 * NG) * gw2 * gw2 / 4.0);
    L = static_cast<T>(Ld);
    LL = static_cast<T>(Ld * Ld);
    sqrtS = static_cast<T>(sS);
    L_lo = static_cast<T>(Ld - static_cast<double>(L));
    S_hi = static_cast<T>(S);
    S_lo = static_cast<T>(S - static_cast<double>(S_hi));
    Mv2_lo = static_cast<T>(Md * Md - static_cast<double>(static_cast<T>(Md * Md)));
    ptmin2 = static_cast<T>(ptm * ptm);
    eta_mu = static_cast<T>(th[5]);
    eta_g = static_cast<T>(th[6]);
    ptij2 = static_cast<T>(th[7] * th[7]);
    M = static_cast<T>(Md);
    Mv2 = static_cast<T>(Md * Md);
    M2G2 = static_cast<T>(Md * Md * Gd * Gd);
    twoMG2 = static_cast<T>(2.0 * Md * Gd * Gd);
    m2M2G = static_cast<T>(-2.0 * Md * Md * Gd);
    two_ng_over_g = static_cast<T>(2.0 * NG / gs);
  }

  // outgoing gluon k, helicity lam: conj of (0, (-lam e1 - i e2) / sqrt2),
  // e1, e2 the polar and azimuthal unit vectors of k; returned as its
  // sigmabar block (eps^0 = 0) and its spatial components (for the dot
  // products of the three-gluon vertex)
  struct Eps {
    SB<T> b;
    Cx<T> v[3];
  };
  __device__ __forceinline__ static Eps eps_out(const T (&k)[4], T pt, T lam) {
    const T s = T(0.70710678118654752440);
    const T ik = vrcp(k[0]), ip = vrcp(pt);
    const T e1x = k[3] * k[1] * ik * ip, e1y = k[3] * k[2] * ik * ip, e1z = -pt * ik;
    const T e2x = -k[2] * ip, e2y = k[1] * ip;
    const T a = -lam * s;
    Eps e;
    e.v[0] = {a * e1x, s * e2x};
    e.v[1] = {a * e1y, s * e2y};
    e.v[2] = {a * e1z, T(0)};
    e.b.p = e.v[2];
    e.b.m = {-e.v[2].r, -e.v[2].i};
    e.b.lo = {e.v[0].r + e.v[1].i, e.v[0].i - e.v[1].r};  // V1 - i V2
    e.b.hi = {e.v[0].r - e.v[1].i, e.v[0].i + e.v[1].r};  // V1 + i V2
    return e;
  }

  // The evaluation in two stages so that a kernel can queue the samples
  // that pass the cuts and evaluate the amplitudes on full waves: stage 1
  // maps x to momenta and applies the cuts; stage 2 forms sqrt(s) again
  // from ln xa + ln xb (the same operations as stage 1, bit for bit), the
  // prefactor, |M|^2 and f.
  struct State {
    T p[NOUT][3];  // g_1..g_NG, mu+, nu in the partonic frame: momenta (E = |p| is formed in stage 2)
    T x0, dm, hel;  // x0, m_munu^2 - M^2, helicity configuration
    T la, lb;       // ln xa, ln xb: sqrt(s) and the flux factor ((1 - xa)(1 - xb))^3 are formed in stage 2
  };
  static constexpr int kStateWords = 3 * NOUT + 5;
  static constexpr bool kStaged = sizeof(T) == 4;  // the queue holds FP32

  __device__ __forceinline__ static void store_state(const State& st, float* q, int stride, int e) {
#pragma unroll
    for (int i = 0; i < NOUT; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) q[(3 * i + c) * stride + e] = static_cast<float>(st.p[i][c]);
    q[(3 * NOUT + 0) * stride + e] = static_cast<float>(st.x0);
    q[(3 * NOUT + 1) * stride + e] = static_cast<float>(st.dm);
    q[(3 * NOUT + 2) * stride + e] = static_cast<float>(st.hel);
    q[(3 * NOUT + 3) * stride + e] = static_cast<float>(st.la);
    q[(3 * NOUT + 4) * stride + e] = static_cast<float>(st.lb);
  }
  __device__ __forceinline__ static State load_state(const float* q, int stride, int e) {
    State st;
#pragma unroll
    for (int i = 0; i < NOUT; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) st.p[i][c] = static_cast<T>(q[(3 * i + c) * stride + e]);
    st.x0 = static_cast<T>(q[(3 * NOUT + 0) * stride + e]);
    st.dm = static_cast<T>(q[(3 * NOUT + 1) * stride + e]);
    st.hel = static_cast<T>(q[(3 * NOUT + 2) * stride + e]);
    st.la = static_cast<T>(q[(3 * NOUT + 3) * stride + e]);
    st.lb = static_cast<T>(q[(3 * NOUT + 4) * stride + e]);
    return st;
  }

  __device__ __forceinline__ bool stage1(const T (&x)[D], State& st) const {
    const T la = L * (T(1) - x[0]);
    const T lb = L * x[0] * (T(1) - x[1]);
    const T h = vexp2_fast((la + lb) * T(0.5 * 1.4426950408889634));  // sqrt(tau)
    const T rs = sqrtS * h;
    const T dl = la - lb;  // twice the boost rapidity y_b
    T Mi[NOUT + 1], Ui[NOUT + 1];
    constexpr bool RES64 = sizeof(T) == 4;
    Resonance64 res{};
    if constexpr (RES64) {
      res.m2 = shat_fp64(x[0], x[1], L, L_lo, S_hi, S_lo);
      res.Mv2 = static_cast<double>(Mv2) + static_cast<double>(Mv2_lo);
    }
    T p[NOUT][4];
    rambo_diet<NOUT, 2, RES64>(x, rs, Mi, Ui, p, res);
    if constexpr (RES64) st.dm = res.dm;
#pragma unroll
    for (int i = 0; i < NOUT; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) st.p[i][c] = p[i][c + 1];

    // ---- cuts: gluons 0..NG-1, the muon NG
    bool pass = true;
    T pt[NG + 1], pt2[NG + 1], eta[NG + 1];
#pragma unroll
    for (int j = 0; j <= NG; ++j) {
      const LightCone<T> lc = light_cone(p[j]);
      pt[j] = lc.pt;
      pt2[j] = lc.pt2;
      eta[j] = lc.eta;
      pass = pass & (lc.pt2 > ptmin2) & (fabs(fma(T(0.5), dl, lc.eta)) < (j < NG ? eta_g : eta_mu));
    }
    if constexpr (NG == 2) {
      // min(pT_i, pT_j)^2 (Delta eta^2 + Delta phi^2) > pTij^2: with
      // z = pTij^2 / min pT^2 - Delta eta^2, pass when z <= 0, else when
      // Delta phi > sqrt z, i.e. cos Delta phi < cos sqrt z (z < pi^2)
      const T de = eta[0] - eta[1];
      const T z = ptij2 * vrcp(fmin(pt2[0], pt2[1])) - de * de;
      const T dot = p[0][1] * p[1][1] + p[0][2] * p[1][2];
      T cz;
      if constexpr (sizeof(T) == 8) {
        cz = cos(sqrt(fmax(z, T(0))));
      } else {
        T sz;
        vsincos2pi(vsqrt(fmax(z, T(0))) * T(0.15915494309189535), sz, cz);
      }
      pass = pass & ((z <= T(0)) | ((z < T(9.869604401089358)) & (dot < cz * pt[0] * pt[1])));
    }
    if (!pass) return false;
    if constexpr (sizeof(T) == 8) st.dm = fma(Mi[NOUT - 1], Mi[NOUT - 1], -Mv2);
    st.x0 = x[0];
    st.la = la;
    st.lb = lb;
    // the gluon helicity configuration, floor(x 2^NG)
    const int hel = static_cast<int>(x[D - 1] * T(1 << NG));
    st.hel = static_cast<T>(hel < (1 << NG) - 1 ? hel : (1 << NG) - 1);
    return true;
  }

  template <bool GRAD>
  __device__ __forceinline__ T stage2(const State& st, T (&g)[NGRAD + 1]) const {
    // the massless momenta, E = |p| (the same in every kernel, whether the
    // state came through the queue or not)
    T p[NOUT][4];
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
      p[i][1] = st.p[i][0];
      p[i][2] = st.p[i][1];
      p[i][3] = st.p[i][2];
      p[i][0] = vsqrt(fma(p[i][1], p[i][1], fma(p[i][2], p[i][2], p[i][3] * p[i][3])));
    }
    const int hel = static_cast<int>(st.hel);
    const T h = vexp2_fast((st.la + st.lb) * T(0.5 * 1.4426950408889634));  // sqrt(tau), as in stage 1
    const T rs = sqrtS * h;
    const T shat = rs * rs;
    T spow = T(1);
#pragma unroll
    for (int i = 0; i < NG; ++i) spow *= shat;  // s^(n-3) from V_n / (2 s), s from |A|^2
    const T pref = (pre * spow) * (LL * st.x0 * vrcp(h));

    // ---- lepton current L = u_L(nu)^dagger sigmabar v_L(mu), sigmabar = (1, -sigma),
    // as its block: L0 + L3 = 2 a1* b1, L0 - L3 = 2 a0* b0, L1 - i L2 = -2 a1* b0,
    // L1 + i L2 = -2 a0* b1 (a = u(nu), b = v(mu))
    const Sp<T> a = weyl(p[NOUT - 1]);
    const Sp<T> b = weyl(p[NOUT - 2]);
    const Cx<T> ac0 = {a.a.r, -a.a.i}, ac1 = {a.b.r, -a.b.i};
    SB<T> Lc;
    Lc.p = T(2) * (ac1 * b.b);
    Lc.m = T(2) * (ac0 * b.a);
    Lc.lo = T(-2) * (ac1 * b.a);
    Lc.hi = T(-2) * (ac0 * b.b);

    T cs;  // colour sum of |chain|^2
    if constexpr (NG == 0) {
      const Cx<T> A = sbar_top(Lc, Sp<T>{{T(0), T(0)}, {T(1), T(0)}});
      cs = T(3) * norm2(A);
    } else {
      // light-cone components of the gluons and of q = p_mu + p_nu; each
      // propagator momentum p_u - (...) = (...)' - p_dbar takes its + part
      // from the particles it leaves out and its - part from those it
      // contains, both sums of non-negative terms (p_u = (2Eh, 0) and
      // p_dbar = (0, 2Eh) in (+, -))
      const LC<T> lm = massless_lc(p[NOUT - 2]), ln = massless_lc(p[NOUT - 1]);
      const LC<T> q = {lm.p + ln.p, lm.m + ln.m, lm.x + ln.x, lm.y + ln.y};
      const Sp<T> uL = sbar_u(Lc);  // W first from the u end
      if constexpr (NG == 1) {
        const LC<T> k = massless_lc(p[0]);
        const T ptg = vsqrt(fma(p[0][1], p[0][1], p[0][2] * p[0][2]));
        const Eps e = eps_out(p[0], ptg, (hel & 1) ? T(1) : T(-1));
        const LC<T> Pk = {q.p, -k.m, -k.x, -k.y};  // p_u - k
        const LC<T> Pq = {k.p, -q.m, k.x, k.y};    // p_u - q
        const Cx<T> A = sbar_top_add(Lc, prop(Pk, sbar_u(e.b)), sbar_top(e.b, prop(Pq, uL)));
        cs = T(4) * norm2(A);
      } else {
        const T(&k1)[4] = p[0];
        const T(&k2)[4] = p[1];
        const LC<T> c1 = massless_lc(k1), c2 = massless_lc(k2);
        const T pt1 = vsqrt(fma(k1[1], k1[1], k1[2] * k1[2])), pt2v = vsqrt(fma(k2[1], k2[1], k2[2] * k2[2]));
        const Eps e1 = eps_out(k1, pt1, (hel & 1) ? T(1) : T(-1));
        const Eps e2 = eps_out(k2, pt2v, (hel & 2) ? T(1) : T(-1));
        // off-shell gluon of the three-gluon vertex, V / K^2 with
        // V = (e1.e2)(k2 - k1) - 2 (k2.e1) e2 + 2 (k1.e2) e1 (e^0 = 0), and
        // K^2 = 2 k1.k2 = E1 E2 |k1/E1 - k2/E2|^2 (no cancellation for
        // nearly collinear gluons)
        const T i1 = vrcp(k1[0]), i2 = vrcp(k2[0]);
        const T dx = fma(k1[1], i1, -k2[1] * i2), dy = fma(k1[2], i1, -k2[2] * i2), dz = fma(k1[3], i1, -k2[3] * i2);
        const T iK2 = vrcp(k1[0] * k2[0] * fma(dx, dx, fma(dy, dy, dz * dz)));
        Cx<T> e12 = {T(0), T(0)}, k2e1 = {T(0), T(0)}, k1e2 = {T(0), T(0)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          e12 = cfma(Cx<T>{-e1.v[c].r, -e1.v[c].i}, e2.v[c], e12);
          k2e1 = cfma(-k2[c + 1], e1.v[c], k2e1);
          k1e2 = cfma(-k1[c + 1], e2.v[c], k1e2);
        }
        const Cx<T> t2 = T(-2) * iK2 * k2e1, t1 = T(2) * iK2 * k1e2, tk = iK2 * e12;
        const LC<T> dk = {c2.p - c1.p, c2.m - c1.m, c2.x - c1.x, c2.y - c1.y};  // k2 - k1
        SB<T> J;
        J.p = cfma(t1, e1.b.p, cfma(t2, e2.b.p, dk.p * tk));
        J.m = cfma(t1, e1.b.m, cfma(t2, e2.b.m, dk.m * tk));
        J.lo = cfma(t1, e1.b.lo, cfma(t2, e2.b.lo, Cx<T>{dk.x, -dk.y} * tk));
        J.hi = cfma(t1, e1.b.hi, cfma(t2, e2.b.hi, Cx<T>{dk.x, dk.y} * tk));
        const LC<T> Pk1 = {c2.p + q.p, -c1.m, -c1.x, -c1.y};                // p_u - k1
        const LC<T> Pk2 = {c1.p + q.p, -c2.m, -c2.x, -c2.y};                // p_u - k2
        const LC<T> PK = {q.p, -(c1.m + c2.m), -(c1.x + c2.x), -(c1.y + c2.y)};  // p_u - k1 - k2
        const LC<T> Pk1q = {c2.p, -(c1.m + q.m), c2.x, c2.y};               // p_u - k1 - q
        const LC<T> Pk2q = {c1.p, -(c2.m + q.m), c1.x, c1.y};               // p_u - k2 - q
        const LC<T> Pq = {c1.p + c2.p, -q.m, c1.x + c2.x, c1.y + c2.y};     // p_u - q
        const Sp<T> ya = prop(Pk2, sbar_u(e2.b));  // gluon 2 first
        const Sp<T> yw = prop(Pk1, sbar_u(e1.b));  // gluon 1 first
        const Sp<T> yc = prop(Pq, uL);             // W first
        // colour T^a1 T^a2 (gluon 1 nearer the dbar end) and T^a2 T^a1; the
        // three-gluon diagrams enter the two with opposite signs.  Chains
        // that end in the same vertex and propagator are summed before them
        // (both are linear maps of the spinor they act on).
        const Sp<T> uJ = sbar_u(J);
        const Cx<T> tJ = sbar_top(J, yc);
        const Cx<T> A12 = sbar_top_add(Lc, prop(PK, sbar_add(e1.b, ya, uJ)),
                                       sbar_top_add(e1.b, prop(Pk2q, sbar_add(Lc, ya, sbar(e2.b, yc))), tJ));
        const Sp<T> muJ = {{-uJ.a.r, -uJ.a.i}, {-uJ.b.r, -uJ.b.i}};
        const Cx<T> A21 = sbar_top_add(Lc, prop(PK, sbar_add(e2.b, yw, muJ)),
                                       sbar_top_add(e2.b, prop(Pk1q, sbar_add(Lc, yw, sbar(e1.b, yc))), Cx<T>{-tJ.r, -tJ.i}));
        cs = T(16.0 / 3.0) * (norm2(A12) + norm2(A21)) - T(4.0 / 3.0) * fma(A12.r, A21.r, A12.i * A21.i);
      }
    }
    // ---- W propagator in m_munu^2 = M_{n-1}^2 (mu nu are the last pair)
    const T dm = st.dm;
    const T invD = vrcp(fma(dm, dm, M2G2));
    const T om = vexpm1_fast(st.la) * vexpm1_fast(st.lb);  // (1 - xa)(1 - xb) without cancellation
    const T f = (pref * (om * om * om)) * (cs * invD);
    if (GRAD) {
      g[0] = f * fma(T(4) * M, dm, -twoMG2) * invD;
      g[1] = f * m2M2G * invD;
      g[2] = f * two_ng_over_g;
    }
    return f;
  }

  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&g)[NGRAD + 1]) const {
    State st;
    if (!stage1(x, st)) {
      if (GRAD) g[0] = g[1] = g[2] = T(0);
      return T(0);
    }
    return stage2<GRAD>(st, g);
  }
};

template <typename T, int D>
using WHel = WHelF<T, (D - 5) / 3>;

}  // namespace vmc
