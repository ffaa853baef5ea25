// vmc_gauss.hpp -- compiled-in test integrands: constants, a linear
// function and the Gaussian families of the d=4, d=8 and batched
// configurations, each with its parameter gradient.
//
// Functor contract (used by every sample kernel):
//   using T; static constexpr int D, NGRAD, NTHETA (NTHETA < 0: D + 1)
//   __device__ void setup(const double* theta)   // once per thread, FP64
//   template <bool GRAD> __device__ T eval(const T (&x)[D], T (&g)[NGRAD+1])
// setup() does the per-parameter work (normalisations, erf) in double
// precision; eval() is the per-sample arithmetic in T.
#pragma once

#include "vmc_device.hpp"

namespace vmc {

template <typename TT, int DD>
struct ConstF {
  using T = TT;
  static constexpr int D = DD, NGRAD = 1, NTHETA = 1, ID = 0;
  T c;
  __device__ void setup(const double* th) { c = static_cast<T>(th[0]); }
  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&)[D], T (&g)[NGRAD + 1]) const {
    if (GRAD) g[0] = T(1);
    return c;
  }
};

template <typename TT, int DD>
struct LinearF {
  using T = TT;
  static constexpr int D = DD, NGRAD = 0, NTHETA = 0, ID = 1;
  __device__ void setup(const double*) {}
  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&)[NGRAD + 1]) const {
    return x[0];
  }
};

// One cube-normalised Gaussian peak exp(-sum_a (x_a-c)^2/s^2) / G^D with
// G = int_0^1 exp(-(x-c)^2/s^2) dx = (s sqrt(pi)/2)(erf((1-c)/s) + erf(c/s)).
// The normalisation and the constant parts of the gradient of its
// logarithm are precomputed in double precision.
template <typename T>
struct Peak {
  T c, inv_s2, log_norm, two_inv_s2, two_inv_s3, kc, ks;
  __device__ void setup(double cd, double sd, int D) {
    const double rpi = 1.7724538509055160273;
    const double G = 0.5 * sd * rpi * (erf((1.0 - cd) / sd) + erf(cd / sd));
    const double ea = exp(-(cd * cd) / (sd * sd));
    const double eb = exp(-((1.0 - cd) * (1.0 - cd)) / (sd * sd));
    const double Gc = ea - eb;
    const double Gs = G / sd - ((1.0 - cd) * eb + cd * ea) / sd;
    c = static_cast<T>(cd);
    inv_s2 = static_cast<T>(1.0 / (sd * sd));
    log_norm = static_cast<T>(-D * log(G));
    two_inv_s2 = static_cast<T>(2.0 / (sd * sd));
    two_inv_s3 = static_cast<T>(2.0 / (sd * sd * sd));
    kc = static_cast<T>(D * Gc / G);
    ks = static_cast<T>(D * Gs / G);
  }
  // value; with GRAD also d ln f / dc and d ln f / ds
  template <bool GRAD, int D>
  __device__ __forceinline__ T eval(const T (&x)[D], T& dlc, T& dls) const {
    T q = T(0), l = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T t = x[a] - c;
      q = fma(t, t, q);
      if (GRAD) l += t;
    }
    const T f = vexp_fast(fma(-q, inv_s2, log_norm));
    if (GRAD) {
      dlc = fma(two_inv_s2, l, -kc);
      dls = fma(two_inv_s3, q, -ks);
    }
    return f;
  }
};

template <typename TT, int DD>
struct GaussF {
  using T = TT;
  static constexpr int D = DD, NGRAD = 2, NTHETA = 2, ID = 2;
  Peak<T> p;
  __device__ void setup(const double* th) { p.setup(th[0], th[1], D); }
  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&g)[NGRAD + 1]) const {
    T dc, ds;
    const T f = p.template eval<GRAD, D>(x, dc, ds);
    if (GRAD) {
      g[0] = f * dc;
      g[1] = f * ds;
    }
    return f;
  }
};

template <typename TT, int DD>
struct DGaussF {
  using T = TT;
  static constexpr int D = DD, NGRAD = 3, NTHETA = 3, ID = 3;
  Peak<T> p1, p2;
  __device__ void setup(const double* th) {
    p1.setup(th[0], th[2], D);
    p2.setup(th[1], th[2], D);
  }
  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&g)[NGRAD + 1]) const {
    T dc1, ds1, dc2, ds2;
    const T a = p1.template eval<GRAD, D>(x, dc1, ds1);
    const T b = p2.template eval<GRAD, D>(x, dc2, ds2);
    if (GRAD) {
      g[0] = T(0.5) * a * dc1;
      g[1] = T(0.5) * b * dc2;
      g[2] = T(0.5) * fma(a, ds1, b * ds2);
    }
    return T(0.5) * (a + b);
  }
};

// Per-axis centres, common width, each axis normalised on the real line:
// prod_a exp(-(x_a-c_a)^2/s^2)/(s sqrt(pi)).
template <typename TT, int DD>
struct GaussAxesF {
  using T = TT;
  static constexpr int D = DD, NGRAD = DD + 1, NTHETA = DD + 1, ID = 4;
  T c[D];
  T inv_s2, log_norm, two_inv_s2, two_inv_s3, d_over_s;
  __device__ void setup(const double* th) {
    const double sd = th[D];
#pragma unroll
    for (int a = 0; a < D; ++a) c[a] = static_cast<T>(th[a]);
    inv_s2 = static_cast<T>(1.0 / (sd * sd));
    log_norm = static_cast<T>(-D * log(sd * 1.7724538509055160273));
    two_inv_s2 = static_cast<T>(2.0 / (sd * sd));
    two_inv_s3 = static_cast<T>(2.0 / (sd * sd * sd));
    d_over_s = static_cast<T>(D / sd);
  }
  template <bool GRAD>
  __device__ __forceinline__ T eval(const T (&x)[D], T (&g)[NGRAD + 1]) const {
    T q = T(0);
    T t[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      t[a] = x[a] - c[a];
      q = fma(t[a], t[a], q);
    }
    const T f = vexp_fast(fma(-q, inv_s2, log_norm));
    if (GRAD) {
      const T f2 = f * two_inv_s2;
#pragma unroll
      for (int a = 0; a < D; ++a) g[a] = f2 * t[a];
      g[D] = f * fma(two_inv_s3, q, -d_over_s);
    }
    return f;
  }
};

}  // namespace vmc
