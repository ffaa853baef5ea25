/*
 * vmc_oracle.c -- plain FP64 CPU oracle for the VEGAS/BASES iteration of
 * Kanzaki, "Monte Carlo integration on GPU" (arXiv:1010.2107).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the GPU
 * library.  Written for clarity, not speed: one sample at a time, in the
 * order the method defines, every quantity in double precision.
 *
 * The paper (Sec. 3.1) splits each iteration into: generate a point from k
 * random numbers (step 2), evaluate the integrand (step 3), accumulate
 * (step 4), re-optimise the grid after N calls (step 5), and repeat
 * (step 6).  The functions below follow that order.
 *
 * Parity status of each function is stated in the test suite; every
 * function here is pinned by at least one test that does not re-use its
 * own arithmetic (closed forms, invariants, a library Philox, brute-force
 * quadrature, an independent RAMBO generator).
 */
#include "vmc_oracle.h"

#include <complex.h>
#undef I /* the imaginary unit is written _Complex_I; I is a result field */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_MAXD 64
#define TWO24 16777216.0

/* ===================================================================== */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4.1 of that paper).          */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to                      */
/*   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));    */
/* the key is advanced by the Weyl constants between rounds.              */
/* ===================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void orc_sample_words(uint64_t seed, uint32_t s, uint32_t it, uint32_t kid, int d, uint32_t *out)
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    for (int a = 0; a < d; a += 4) {
        uint32_t ctr[4] = {s, (uint32_t)(a / 4), it, kid};
        uint32_t blk[4];
        orc_philox4x32_10(ctr, key, blk);
        for (int q = 0; q < 4 && a + q < d; ++q)
            out[a + q] = blk[q];
    }
}

/* ===================================================================== */
/* Step 2: a point from random words.                                     */
/* The top 23 bits m of a word give the uniform u = (2m+1) 2^-24, the     */
/* centre of one of 2^23 equal cells of (0,1); it is never 0 or 1.        */
/* ===================================================================== */
double orc_uniform(uint32_t word)
{
    uint32_t m = word >> 9;
    return (2.0 * (double)m + 1.0) / TWO24;
}

/* Plain mode: y = u, bin j = floor(y N), delta = y N - j, in exact
 * integer arithmetic: y N = (2m+1) N / 2^24. */
void orc_bin_plain(uint32_t word, int nbins, int *j, double *delta)
{
    uint64_t m = word >> 9;
    uint64_t P = (2 * m + 1) * (uint64_t)nbins;
    *j = (int)(P >> 24);
    *delta = (double)(P & 0xFFFFFFu) / TWO24;
}

/* Stratified mode (BASES): the cube coordinate c_a in [0, ng) places the
 * point at y = (c_a + u)/ng, so y N = (c_a 2^24 + 2m+1) N / (ng 2^24). */
void orc_bin_strat(uint32_t word, int cube_coord, int ng, int nbins, int *j, double *delta)
{
    uint64_t m = word >> 9;
    uint64_t Q = ((uint64_t)cube_coord * (uint64_t)(1u << 24) + 2 * m + 1) * (uint64_t)nbins;
    uint64_t D = (uint64_t)ng << 24;
    *j = (int)(Q / D);
    *delta = (double)(Q % D) / (double)D;
}

void orc_bin_batch(int64_t n, const uint32_t *words, const int32_t *cube_coord, int ng,
                   int nbins, int32_t *j, double *delta)
{
    for (int64_t i = 0; i < n; ++i) {
        int jj;
        if (ng <= 1)
            orc_bin_plain(words[i], nbins, &jj, &delta[i]);
        else
            orc_bin_strat(words[i], cube_coord[i], ng, nbins, &jj, &delta[i]);
        j[i] = jj;
    }
}

/* ===================================================================== */
/* Grid map (Sec. 2: each axis divided into bins).  Within bin j of axis  */
/* a the map is linear: x = e_j + delta (e_{j+1} - e_j), and the Jacobian  */
/* of y -> x is N (e_{j+1} - e_j) per axis.                                */
/* ===================================================================== */
double orc_map(int d, int nbins, const double *edges, const int32_t *j, const double *delta, double *x)
{
    double jac = 1.0;
    for (int a = 0; a < d; ++a) {
        const double *e = edges + (size_t)a * (size_t)(nbins + 1);
        double lo = e[j[a]];
        double width = e[j[a] + 1] - e[j[a]];
        x[a] = lo + delta[a] * width;
        jac *= (double)nbins * width;
    }
    return jac;
}

/* ===================================================================== */
/* Step 3: integrands.                                                    */
/* ===================================================================== */

/* Gaussian with the "sigma" of the configurations: phi = exp(-(x-c)^2/s^2). */
static double gauss_phi(double x, double c, double s)
{
    double t = (x - c) / s;
    return exp(-t * t);
}

/* G(c,s) = int_0^1 phi(x;c,s) dx = (s sqrt(pi)/2) [erf((1-c)/s) + erf(c/s)] */
static double gauss_G(double c, double s)
{
    return 0.5 * s * sqrt(M_PI) * (erf((1.0 - c) / s) + erf(c / s));
}

/* dG/dc and dG/ds */
static void gauss_G_grad(double c, double s, double *dGdc, double *dGds)
{
    double ea = exp(-(c * c) / (s * s));
    double eb = exp(-((1.0 - c) * (1.0 - c)) / (s * s));
    *dGdc = ea - eb;
    *dGds = gauss_G(c, s) / s - ((1.0 - c) * eb + c * ea) / s;
}

/* One cube-normalised Gaussian product over d axes and the gradient of its
 * logarithm in (c, s). */
static double gauss_cube(int d, const double *x, double c, double s, double *dlog_dc, double *dlog_ds)
{
    double G = gauss_G(c, s);
    double prod = 1.0, sum_dc = 0.0, sum_ds = 0.0;
    for (int a = 0; a < d; ++a) {
        prod *= gauss_phi(x[a], c, s) / G;
        sum_dc += 2.0 * (x[a] - c) / (s * s);
        sum_ds += 2.0 * (x[a] - c) * (x[a] - c) / (s * s * s);
    }
    if (dlog_dc) {
        double Gc, Gs;
        gauss_G_grad(c, s, &Gc, &Gs);
        *dlog_dc = sum_dc - d * Gc / G;
        *dlog_ds = sum_ds - d * Gs / G;
    }
    return prod;
}

int orc_integrand_nparams(int id, int d)
{
    switch (id) {
    case ORC_CONST: return 1;
    case ORC_LINEAR: return 0;
    case ORC_GAUSS: return 2;
    case ORC_DGAUSS: return 3;
    case ORC_GAUSS_AXES: return d + 1;
    case ORC_WJETS: return 7;
    case ORC_PSVOL: return 2;
    case ORC_WHEL: return 8;
    default: return ORC_E_INTEGRAND;
    }
}

int orc_integrand_ngrad(int id, int d)
{
    switch (id) {
    case ORC_CONST: return 1;
    case ORC_LINEAR: return 0;
    case ORC_GAUSS: return 2;
    case ORC_DGAUSS: return 3;
    case ORC_GAUSS_AXES: return d + 1;
    case ORC_WJETS: return 3;
    case ORC_PSVOL: return 0;
    case ORC_WHEL: return 3;
    default: return ORC_E_INTEGRAND;
    }
}

/* ---------------------------------------------------------------------- */
/* Physics toy: pp -> W(-> e nu) + n_p partons.  The paper's process       */
/* (Sec. 5, eq. 1) with HELAS amplitudes and CTEQ6L1 is replaced by a toy  */
/* of the same shape: n_p + 2 massless final-state particles, 3n-4 phase-  */
/* space variables plus 2 for the parton momentum fractions.               */
/* ---------------------------------------------------------------------- */

/* Massless n-body phase-space volume (Kleiss-Stirling-Ellis normalisation,
 * prod d^3p/((2pi)^3 2E) (2pi)^4 delta^4):
 *   V_n(s) = (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!). */
double orc_massless_ps_volume(int n, double shat)
{
    double fact1 = 1.0, fact2 = 1.0;
    for (int i = 2; i <= n - 1; ++i) fact1 *= i;
    for (int i = 2; i <= n - 2; ++i) fact2 *= i;
    return pow(2.0 * M_PI, 4.0 - 3.0 * n) * pow(M_PI / 2.0, n - 1) * pow(shat, n - 2) / (fact1 * fact2);
}

/* RAMBO on diet, mass step: the fraction t = M_i^2/M_{i-1}^2 has density
 * proportional to (1-t) t^(k-1), k = n-i, i.e. CDF (k+1) t^k - k t^(k+1).
 * Solved by bisection to the last bit. */
int orc_solve_mass_fraction(int n, int i, double r, double *t)
{
    int k = n - i;
    if (k < 1 || r < 0.0 || r > 1.0) return ORC_E_INVALID;
    double lo = 0.0, hi = 1.0;
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double F = (k + 1) * pow(mid, k) - k * pow(mid, k + 1);
        if (F < r)
            lo = mid;
        else
            hi = mid;
    }
    *t = hi;
    return ORC_OK;
}

/* Boost p, given in the rest frame of Q (mass M), to the frame where Q has
 * four-momentum (E, P). */
static void boost_from_rest(const double Q[4], double M, const double p[4], double out[4])
{
    double pdotP = Q[1] * p[1] + Q[2] * p[2] + Q[3] * p[3];
    double e = (Q[0] * p[0] + pdotP) / M;
    double f = (p[0] + pdotP / (Q[0] + M)) / M;
    out[0] = e;
    out[1] = p[1] + f * Q[1];
    out[2] = p[2] + f * Q[2];
    out[3] = p[3] + f * Q[3];
}

/* RAMBO on diet (Plaetzer): n massless momenta in the rest frame of a
 * system of mass sqrt_shat from 3n-4 uniforms r.  r[0..n-3] fix the
 * intermediate masses M_2..M_{n-1}; then for each stage i = 1..n-1 the
 * pair (r_cos, r_phi) fixes the direction of p_i in the rest frame of
 * Q_i = p_i + ... + p_n.  Returns the (constant) weight V_n(shat). */
double orc_rambo_diet(int n, double sqrt_shat, const double *r, double *p)
{
    double M[ORC_MAXD];
    M[1] = sqrt_shat;
    for (int i = 2; i <= n - 1; ++i) {
        double t;
        orc_solve_mass_fraction(n, i, r[i - 2], &t);
        M[i] = M[i - 1] * sqrt(t);
    }
    M[n] = 0.0;
    double Q[4] = {sqrt_shat, 0.0, 0.0, 0.0};
    for (int i = 1; i <= n - 1; ++i) {
        double q = (M[i] * M[i] - M[i + 1] * M[i + 1]) / (2.0 * M[i]);
        double cth = 2.0 * r[n - 2 + 2 * (i - 1)] - 1.0;
        double phi = 2.0 * M_PI * r[n - 2 + 2 * (i - 1) + 1];
        double sth = sqrt(1.0 - cth * cth);
        double nx = sth * cos(phi), ny = sth * sin(phi), nz = cth;
        double pr[4] = {q, q * nx, q * ny, q * nz};
        double qr[4] = {M[i] - q, -q * nx, -q * ny, -q * nz};
        double Qnext[4];
        boost_from_rest(Q, M[i], pr, p + 4 * (i - 1));
        boost_from_rest(Q, M[i], qr, Qnext);
        memcpy(Q, Qnext, sizeof Q);
    }
    memcpy(p + 4 * (n - 1), Q, sizeof Q);
    return orc_massless_ps_volume(n, sqrt_shat * sqrt_shat);
}

static double pt_of(const double *p) { return sqrt(p[1] * p[1] + p[2] * p[2]); }
static double eta_of(const double *p) { return asinh(p[3] / pt_of(p)); }
static double phi_of(const double *p) { return atan2(p[2], p[1]); }
static double mdot(const double *a, const double *b)
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* Acceptance: the n_p partons and the charged lepton (indices 0..n_p)
 * need pT > ptmin and |eta_lab| < etamax, and every pair of them needs
 * Delta R > drmin; the neutrino (index n_p+1) is not constrained.  eta_lab
 * is the CM pseudorapidity shifted by the rapidity of the CM frame. */
int orc_pass_cuts(int n_p, const double *p, double y_boost, double ptmin, double etamax, double drmin)
{
    int nvis = n_p + 1;
    for (int i = 0; i < nvis; ++i) {
        const double *pi = p + 4 * i;
        if (!(pt_of(pi) > ptmin)) return 0;
        if (!(fabs(eta_of(pi) + y_boost) < etamax)) return 0;
    }
    for (int i = 0; i < nvis; ++i)
        for (int k = i + 1; k < nvis; ++k) {
            double deta = eta_of(p + 4 * i) - eta_of(p + 4 * k);
            double dphi = fabs(phi_of(p + 4 * i) - phi_of(p + 4 * k));
            if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
            if (!(sqrt(deta * deta + dphi * dphi) > drmin)) return 0;
        }
    return 1;
}

/* Distinct cyclic orders of m objects, up to rotation and reflection:
 * object 0 first, the rest permuted, reflection removed by keeping only
 * orders whose second entry is smaller than their last.  (m-1)!/2 orders. */
#define ORC_MAXM 7
static int cyc_count[ORC_MAXM + 1];
static unsigned char cyc_table[ORC_MAXM + 1][720][ORC_MAXM];
static int cyc_built[ORC_MAXM + 1];

static int next_permutation(unsigned char *a, int n)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    unsigned char t = a[i];
    a[i] = a[j];
    a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) {
        t = a[l];
        a[l] = a[r];
        a[r] = t;
    }
    return 1;
}

static void build_cycles(int m)
{
    if (cyc_built[m]) return;
    unsigned char rest[ORC_MAXM];
    for (int i = 0; i < m - 1; ++i) rest[i] = (unsigned char)(i + 1);
    int cnt = 0;
    do {
        if (m < 3 || rest[0] < rest[m - 2]) {
            cyc_table[m][cnt][0] = 0;
            for (int i = 0; i < m - 1; ++i) cyc_table[m][cnt][i + 1] = rest[i];
            ++cnt;
        }
    } while (next_permutation(rest, m - 1));
    cyc_count[m] = cnt;
    cyc_built[m] = 1;
}

int orc_num_cycles(int m)
{
    if (m < 3 || m > ORC_MAXM) return ORC_E_INVALID;
    build_cycles(m);
    return cyc_count[m];
}

/* sum over distinct cyclic orders sigma of 1 / prod_i s[sigma_i][sigma_{i+1}] */
double orc_cyclic_sum(int m, const double *s)
{
    if (m < 3 || m > ORC_MAXM) return NAN;
    build_cycles(m);
    double total = 0.0;
    for (int c = 0; c < cyc_count[m]; ++c) {
        const unsigned char *o = cyc_table[m][c];
        double prod = 1.0;
        for (int i = 0; i < m; ++i) prod *= s[o[i] * m + o[(i + 1) % m]];
        total += 1.0 / prod;
    }
    return total;
}

/* Toy parton flux F(x) = x^-1.5 (1-x)^3 */
static double toy_pdf(double x) { return pow(x, -1.5) * pow(1.0 - x, 3.0); }

double orc_wjets_event(int d, const double *x, const double *theta, int ntheta,
                       double *p, double *aux, double *grad)
{
    int n_p = (d - 4) / 3;
    int n = n_p + 2;
    int full = (ntheta == 7);
    double sqrtS = full ? theta[3] : theta[0];
    double ptmin = full ? theta[4] : theta[1];
    double S = sqrtS * sqrtS;

    /* parton momentum fractions: ln x1 = L (1-x0), ln x2 = L x0 (1-x1),
     * covering x1 x2 >= tau0 once; dx1 dx2 = L^2 x0 x1 x2 dx0 dx1 */
    double tau0 = ((1.0 + n_p) * ptmin) * ((1.0 + n_p) * ptmin) / S;
    double L = log(tau0);
    double x1 = exp(L * (1.0 - x[0]));
    double x2 = exp(L * x[0] * (1.0 - x[1]));
    double Jx = L * L * x[0] * x1 * x2;
    double shat = x1 * x2 * S;
    double lum = toy_pdf(x1) * toy_pdf(x2);
    double Vn = orc_rambo_diet(n, sqrt(shat), x + 2, p);
    double y_boost = 0.5 * log(x1 / x2);
    double m2 = 2.0 * mdot(p + 4 * n_p, p + 4 * (n_p + 1));

    double ps_part = lum * Jx * Vn / (2.0 * shat);
    if (aux) {
        aux[0] = x1; aux[1] = x2; aux[2] = shat; aux[3] = Jx;
        aux[4] = lum; aux[5] = Vn; aux[6] = m2; aux[7] = 1.0;
    }
    if (!full) return ps_part;

    double M = theta[0], Gam = theta[1], g = theta[2];
    double etamax = theta[5], drmin = theta[6];
    if (grad) grad[0] = grad[1] = grad[2] = 0.0;
    if (!orc_pass_cuts(n_p, p, y_boost, ptmin, etamax, drmin)) {
        if (aux) aux[7] = 0.0;
        return 0.0;
    }
    /* Breit-Wigner in m_{e nu}^2, unit normalised over m^2 */
    double D = (m2 - M * M) * (m2 - M * M) + M * M * Gam * Gam;
    double bw = (M * Gam / M_PI) / D;

    /* coloured set: a (incoming along +z), b (along -z), partons */
    int m = n_p + 2;
    double rs = sqrt(shat);
    double mom[ORC_MAXM][4];
    double pa[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs};
    double pb[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};
    memcpy(mom[0], pa, sizeof pa);
    memcpy(mom[1], pb, sizeof pb);
    for (int i = 0; i < n_p; ++i) memcpy(mom[2 + i], p + 4 * i, 4 * sizeof(double));
    double smat[ORC_MAXM * ORC_MAXM];
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k) smat[i * m + k] = (i == k) ? 0.0 : 2.0 * mdot(mom[i], mom[k]);
    double pt_sum = 2.0 * shat * shat * shat * shat * orc_cyclic_sum(m, smat);

    double me2 = pow(g, 2.0 * n_p) * bw * pt_sum;
    double f = ps_part * me2;
    if (grad) {
        grad[0] = f * (1.0 / M - (-4.0 * M * (m2 - M * M) + 2.0 * M * Gam * Gam) / D);
        grad[1] = f * (1.0 / Gam - 2.0 * M * M * Gam / D);
        grad[2] = f * (2.0 * n_p / g);
    }
    return f;
}

/* ===================================================================== */
/* The paper's process, u dbar -> W+(-> mu+ nu) + n gluons (Sec. 5, eq. 1; */
/* Table 4: 1, 2 and 8 diagrams for n = 0, 1, 2), from tree-level          */
/* helicity amplitudes.  All fermions are massless and the W couples only */
/* to left-handed fermions, so the quark line and the lepton line are     */
/* chains of 2x2 blocks acting on left-chirality Weyl spinors:            */
/*   vertex with vector V:  V_mu sigmabar^mu;  propagator P: P_mu sigma^mu */
/*   / P^2;  line = v_L(p_dbar)^dagger [...] u_L(p_u).                    */
/* Feynman rules (Feynman gauge): quark-gluon  i g_s gamma^mu T^a; three- */
/* gluon  g_s f^abc [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu +            */
/* g^{rho mu}(q-k)^nu] (momenta incoming); quark propagator i pslash/p^2; */
/* gluon propagator -i g/k^2; W: i g_W/sqrt2 gamma^mu P_L at each line,   */
/* propagator -i g/(q^2 - M^2 + i M Gamma) (the q q term vanishes on the   */
/* massless lepton current).  Colour: M = sum over orderings sigma of      */
/* (T^{a_sigma1} .. T^{a_sigman})_{ji} A_sigma with f^abc T^c =            */
/* -i [T^a, T^b]; the colour sum of |M|^2 is A^dagger C A with C = 3       */
/* (n=0), 4 (n=1), [[16/3, -2/3], [-2/3, 16/3]] (n=2).                     */
/* ===================================================================== */
typedef double complex cplx;

#define WHEL_GF 1.1663787e-5 /* Fermi constant, GeV^-2                    */
#define WHEL_MWREF 80.4      /* g_W^2 = 4 sqrt2 G_F MWREF^2 (fixed coupling) */

static double whel_gw2(void) { return 4.0 * sqrt(2.0) * WHEL_GF * WHEL_MWREF * WHEL_MWREF; }

/* left-chirality spinor of a massless momentum: p.sigmabar u = 0, u^dagger u = 2 E */
static void weyl_spinor(const double p[4], cplx u[2])
{
    double pp = p[0] + p[3], pm = p[0] - p[3];
    if (pp >= pm) {
        double r = sqrt(pp);
        u[0] = -(p[1] - _Complex_I * p[2]) / r;
        u[1] = r;
    } else {
        double r = sqrt(pm);
        u[0] = r;
        u[1] = -(p[1] + _Complex_I * p[2]) / r;
    }
}

/* x <- (a_mu sigmabar^mu) x, a contravariant */
static void apply_sbar(const cplx a[4], cplx x[2])
{
    cplx y0 = (a[0] + a[3]) * x[0] + (a[1] - _Complex_I * a[2]) * x[1];
    cplx y1 = (a[1] + _Complex_I * a[2]) * x[0] + (a[0] - a[3]) * x[1];
    x[0] = y0;
    x[1] = y1;
}

/* x <- (a_mu sigma^mu) x */
static void apply_sig(const cplx a[4], cplx x[2])
{
    cplx y0 = (a[0] - a[3]) * x[0] - (a[1] - _Complex_I * a[2]) * x[1];
    cplx y1 = -(a[1] + _Complex_I * a[2]) * x[0] + (a[0] + a[3]) * x[1];
    x[0] = y0;
    x[1] = y1;
}

static double rdot(const double a[4], const double b[4]) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
static cplx cdot(const cplx a[4], const cplx b[4]) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
static cplx cdot_r(const double a[4], const cplx b[4]) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }

/* One quark line: vertices V[0..k-1] from the u end, V[i] carrying away
 * momentum out[i]; propagators between them. */
static cplx quark_line(int k, const cplx *const *V, const double *const *out, const cplx uL[2],
                       const cplx vL[2], const double pu[4])
{
    cplx x[2] = {uL[0], uL[1]};
    double P[4] = {pu[0], pu[1], pu[2], pu[3]};
    for (int i = 0; i < k; ++i) {
        if (i > 0) {
            cplx Pc[4] = {P[0], P[1], P[2], P[3]};
            apply_sig(Pc, x);
            double P2 = rdot(P, P);
            x[0] /= P2;
            x[1] /= P2;
        }
        apply_sbar(V[i], x);
        for (int c = 0; c < 4; ++c) P[c] -= out[i][c];
    }
    return conj(vL[0]) * x[0] + conj(vL[1]) * x[1];
}

int orc_whel_partials(int n, const double *mom, const double *eps, double *A)
{
    /* mom: pu, pd, k_1..k_n, p_mu, p_nu (4 each); eps: per gluon the
     * polarisation vector used at the vertex (re[4], im[4]); A: the
     * colour-ordered amplitudes (re, im) without couplings and W
     * propagator: n <= 1 one of them, n = 2 A_12 (colour T^a1 T^a2) and
     * A_21. */
    if (n < 0 || n > 2) return ORC_E_INVALID;
    const double *pu = mom, *pd = mom + 4, *pmu = mom + 4 * (n + 2), *pnu = mom + 4 * (n + 3);
    cplx uL[2], vL[2], a[2], b[2];
    weyl_spinor(pu, uL);
    weyl_spinor(pd, vL);
    weyl_spinor(pnu, a);
    weyl_spinor(pmu, b);
    /* lepton current L^mu = u_L(nu)^dagger sigmabar^mu v_L(mu), sigmabar = (1, -sigma) */
    cplx L[4];
    L[0] = conj(a[0]) * b[0] + conj(a[1]) * b[1];
    L[1] = -(conj(a[0]) * b[1] + conj(a[1]) * b[0]);
    L[2] = -(conj(a[0]) * (-_Complex_I * b[1]) + conj(a[1]) * (_Complex_I * b[0]));
    L[3] = -(conj(a[0]) * b[0] - conj(a[1]) * b[1]);
    double q[4];
    for (int c = 0; c < 4; ++c) q[c] = pmu[c] + pnu[c];
    cplx e[2][4];
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c) e[i][c] = eps[8 * i + c] + _Complex_I * eps[8 * i + 4 + c];
    const double *k1 = mom + 8, *k2 = mom + 12;
    if (n == 0) {
        const cplx *V[1] = {L};
        const double *o[1] = {q};
        cplx r = quark_line(1, V, o, uL, vL, pu);
        A[0] = creal(r);
        A[1] = cimag(r);
    } else if (n == 1) {
        const cplx *V1[2] = {e[0], L}, *V2[2] = {L, e[0]};
        const double *o1[2] = {k1, q}, *o2[2] = {q, k1};
        cplx r = quark_line(2, V1, o1, uL, vL, pu) + quark_line(2, V2, o2, uL, vL, pu);
        A[0] = creal(r);
        A[1] = cimag(r);
    } else {
        /* the off-shell gluon of the three-gluon vertex: V^rho / K^2 with
         * V = (e1.e2)(k2-k1) - 2 (k2.e1) e2 + 2 (k1.e2) e1 */
        double K[4];
        for (int c = 0; c < 4; ++c) K[c] = k1[c] + k2[c];
        cplx e12 = cdot(e[0], e[1]), k2e1 = cdot_r(k2, e[0]), k1e2 = cdot_r(k1, e[1]);
        double K2 = rdot(K, K);
        cplx J[4];
        for (int c = 0; c < 4; ++c) J[c] = (e12 * (k2[c] - k1[c]) - 2.0 * k2e1 * e[1][c] + 2.0 * k1e2 * e[0][c]) / K2;
        /* colour T^a1 T^a2: gluon 1 nearer the dbar end, i.e. gluon 2 first from the u end */
        const cplx *Va[3] = {e[1], e[0], L}, *Vb[3] = {e[1], L, e[0]}, *Vc[3] = {L, e[1], e[0]};
        const double *oa[3] = {k2, k1, q}, *ob[3] = {k2, q, k1}, *oc[3] = {q, k2, k1};
        cplx A12 = quark_line(3, Va, oa, uL, vL, pu) + quark_line(3, Vb, ob, uL, vL, pu) +
                   quark_line(3, Vc, oc, uL, vL, pu);
        const cplx *Wa[3] = {e[0], e[1], L}, *Wb[3] = {e[0], L, e[1]}, *Wc[3] = {L, e[0], e[1]};
        const double *pa_[3] = {k1, k2, q}, *pb_[3] = {k1, q, k2}, *pc_[3] = {q, k1, k2};
        cplx A21 = quark_line(3, Wa, pa_, uL, vL, pu) + quark_line(3, Wb, pb_, uL, vL, pu) +
                   quark_line(3, Wc, pc_, uL, vL, pu);
        const cplx *T1[2] = {J, L}, *T2[2] = {L, J};
        const double *t1[2] = {K, q}, *t2[2] = {q, K};
        cplx T = quark_line(2, T1, t1, uL, vL, pu) + quark_line(2, T2, t2, uL, vL, pu);
        A12 += T;
        A21 -= T;
        A[0] = creal(A12);
        A[1] = cimag(A12);
        A[2] = creal(A21);
        A[3] = cimag(A21);
    }
    return ORC_OK;
}

/* Polarisation vector of gluon momentum k, helicity lam = +-1:
 * (0, (-lam e1 - i e2)/sqrt2) with e1, e2 the polar and azimuthal unit
 * vectors of k; returned conjugated (outgoing gluon) as re[4], im[4]. */
static void gluon_eps_out(const double k[4], int lam, double *re, double *im)
{
    double pt = sqrt(k[1] * k[1] + k[2] * k[2]);
    double kk = sqrt(pt * pt + k[3] * k[3]);
    double e1[3], e2[3];
    if (pt > 0.0) {
        e1[0] = k[3] * k[1] / (kk * pt);
        e1[1] = k[3] * k[2] / (kk * pt);
        e1[2] = -pt / kk;
        e2[0] = -k[2] / pt;
        e2[1] = k[1] / pt;
        e2[2] = 0.0;
    } else {
        e1[0] = k[3] >= 0.0 ? 1.0 : -1.0;
        e1[1] = 0.0;
        e1[2] = 0.0;
        e2[0] = 0.0;
        e2[1] = 1.0;
        e2[2] = 0.0;
    }
    double r = 1.0 / sqrt(2.0);
    re[0] = im[0] = 0.0;
    for (int c = 0; c < 3; ++c) {
        re[1 + c] = -lam * e1[c] * r;
        im[1 + c] = +e2[c] * r; /* conjugate of -i e2 / sqrt2 */
    }
}

double orc_whel_me2(int n, const double *mom, int hel, const double *theta)
{
    /* colour-summed |M|^2 of gluon helicities hel (bit i set: gluon i has
     * helicity +1), quark and lepton helicities fixed by the W coupling */
    double eps[16] = {0};
    for (int i = 0; i < n; ++i)
        gluon_eps_out(mom + 4 * (2 + i), ((hel >> i) & 1) ? 1 : -1, eps + 8 * i, eps + 8 * i + 4);
    double A[4];
    if (orc_whel_partials(n, mom, eps, A)) return NAN;
    double cs;
    if (n == 0)
        cs = 3.0 * (A[0] * A[0] + A[1] * A[1]);
    else if (n == 1)
        cs = 4.0 * (A[0] * A[0] + A[1] * A[1]);
    else {
        double a2 = A[0] * A[0] + A[1] * A[1], b2 = A[2] * A[2] + A[3] * A[3];
        double re_ab = A[0] * A[2] + A[1] * A[3];
        cs = (16.0 / 3.0) * (a2 + b2) - (4.0 / 3.0) * re_ab;
    }
    double M = theta[0], Gam = theta[1], gs = theta[2];
    const double *pmu = mom + 4 * (n + 2), *pnu = mom + 4 * (n + 3);
    double q[4];
    for (int c = 0; c < 4; ++c) q[c] = pmu[c] + pnu[c];
    double q2 = rdot(q, q);
    double D = (q2 - M * M) * (q2 - M * M) + M * M * Gam * Gam;
    double gw2 = whel_gw2();
    return pow(gs, 2.0 * n) * (gw2 * gw2 / 4.0) * cs / D;
}

int orc_whel_pass_cuts(int n, const double *p, double y_boost, double ptmin, double eta_mu, double eta_g,
                       double ptij_min)
{
    /* p: final state in the partonic frame, order g_1..g_n, mu+, nu */
    for (int i = 0; i <= n; ++i) {
        const double *v = p + 4 * i;
        double pt = pt_of(v);
        double eta = eta_of(v) + y_boost;
        if (!(pt > ptmin)) return 0;
        if (!(fabs(eta) < (i < n ? eta_g : eta_mu))) return 0;
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double *a = p + 4 * i, *b = p + 4 * j;
            double deta = eta_of(a) - eta_of(b);
            double dphi = fabs(phi_of(a) - phi_of(b));
            if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
            double dr = sqrt(deta * deta + dphi * dphi);
            double ptij = fmin(pt_of(a), pt_of(b)) * dr;
            if (!(ptij > ptij_min)) return 0;
        }
    return 1;
}

double orc_whel_event(int d, const double *x, const double *theta, int ntheta, double *p, double *aux,
                      double *grad)
{
    int n = (d - 5) / 3; /* gluons */
    int nf = n + 2;      /* final state: g_1..g_n, mu+, nu */
    (void)ntheta;
    double M = theta[0], Gam = theta[1], gs = theta[2], sqrtS = theta[3], ptmin = theta[4];
    double eta_mu = theta[5], eta_g = theta[6], ptij_min = theta[7];
    double S = sqrtS * sqrtS;
    double tau0 = ((1.0 + n) * ptmin) * ((1.0 + n) * ptmin) / S;
    double L = log(tau0);
    double x1 = exp(L * (1.0 - x[0]));
    double x2 = exp(L * x[0] * (1.0 - x[1]));
    double Jx = L * L * x[0] * x1 * x2;
    double shat = x1 * x2 * S;
    double lum = toy_pdf(x1) * toy_pdf(x2);
    double Vn = orc_rambo_diet(nf, sqrt(shat), x + 2, p);
    double y_boost = 0.5 * log(x1 / x2);
    /* helicity sampling: the last variable picks one of the 2^n gluon
     * helicity configurations, weight 2^n */
    int nh = 1 << n;
    int hel = (int)(x[d - 1] * nh);
    if (hel >= nh) hel = nh - 1;
    if (grad) grad[0] = grad[1] = grad[2] = 0.0;
    if (aux) {
        aux[0] = x1; aux[1] = x2; aux[2] = shat; aux[3] = Jx;
        aux[4] = lum; aux[5] = Vn; aux[6] = 2.0 * mdot(p + 4 * n, p + 4 * (n + 1)); aux[7] = 0.0;
    }
    if (!orc_whel_pass_cuts(n, p, y_boost, ptmin, eta_mu, eta_g, ptij_min)) return 0.0;
    if (aux) aux[7] = 1.0;
    double rs = sqrt(shat);
    double mom[4 * 6];
    double pu[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs}, pd[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};
    memcpy(mom, pu, sizeof pu);
    memcpy(mom + 4, pd, sizeof pd);
    memcpy(mom + 8, p, 4 * (size_t)nf * sizeof(double));
    double me2 = orc_whel_me2(n, mom, hel, theta);
    /* spin (1/4) and colour (1/9) average of the initial state */
    double f = lum * Jx * Vn / (2.0 * shat) * (nh / 36.0) * me2;
    if (grad) {
        double q2 = aux ? aux[6] : 2.0 * mdot(p + 4 * n, p + 4 * (n + 1));
        double D = (q2 - M * M) * (q2 - M * M) + M * M * Gam * Gam;
        grad[0] = f * (4.0 * M * (q2 - M * M) - 2.0 * M * Gam * Gam) / D;
        grad[1] = f * (-2.0 * M * M * Gam / D);
        grad[2] = f * (2.0 * n / gs);
    }
    return f;
}

double orc_integrand(int id, int d, const double *x, const double *theta, int ntheta, double *grad)
{
    switch (id) {
    case ORC_CONST:
        if (grad) grad[0] = 1.0;
        return theta[0];
    case ORC_LINEAR:
        return x[0];
    case ORC_GAUSS: {
        double dc, ds;
        double f = gauss_cube(d, x, theta[0], theta[1], &dc, &ds);
        if (grad) {
            grad[0] = f * dc;
            grad[1] = f * ds;
        }
        return f;
    }
    case ORC_DGAUSS: {
        double dc1, ds1, dc2, ds2;
        double A = gauss_cube(d, x, theta[0], theta[2], &dc1, &ds1);
        double B = gauss_cube(d, x, theta[1], theta[2], &dc2, &ds2);
        if (grad) {
            grad[0] = 0.5 * A * dc1;
            grad[1] = 0.5 * B * dc2;
            grad[2] = 0.5 * (A * ds1 + B * ds2);
        }
        return 0.5 * (A + B);
    }
    case ORC_GAUSS_AXES: {
        double s = theta[d];
        double f = 1.0, dsum = 0.0;
        for (int a = 0; a < d; ++a) {
            f *= gauss_phi(x[a], theta[a], s) / (s * sqrt(M_PI));
            dsum += 2.0 * (x[a] - theta[a]) * (x[a] - theta[a]) / (s * s * s) - 1.0 / s;
        }
        if (grad) {
            for (int a = 0; a < d; ++a) grad[a] = f * 2.0 * (x[a] - theta[a]) / (s * s);
            grad[d] = f * dsum;
        }
        return f;
    }
    case ORC_WJETS:
    case ORC_PSVOL: {
        double p[4 * ORC_MAXM];
        return orc_wjets_event(d, x, theta, ntheta, p, NULL, grad);
    }
    case ORC_WHEL: {
        double p[4 * ORC_MAXM];
        return orc_whel_event(d, x, theta, ntheta, p, NULL, grad);
    }
    default:
        return NAN;
    }
}

static int check_integrand(int id, int d, int ntheta)
{
    int np = orc_integrand_nparams(id, d);
    if (np < 0) return ORC_E_INTEGRAND;
    if (np != ntheta) return ORC_E_PARAMS;
    if (id == ORC_WJETS || id == ORC_PSVOL) {
        if (d < 7 || (d - 4) % 3 != 0 || (d - 4) / 3 > ORC_MAXM - 2) return ORC_E_DIM;
    }
    if (id == ORC_WHEL && d != 5 && d != 8 && d != 11) return ORC_E_DIM;
    return ORC_OK;
}

/* ===================================================================== */
/* The point as a single-precision map forms it (the paper evaluates the   */
/* integrand in single precision, Sec. 3.2).  The grid is held per bin as  */
/* the lower edge and the width times 2^-24, each rounded once to FP32     */
/* from the FP64 edges; the in-bin offset is the integer 2^24 delta (plain */
/* sampling, or stratification with ng dividing N), otherwise the FP32     */
/* value of (r_hi 2^24 + r_lo) / ng formed as one fused multiply-add of    */
/* r_hi with (1/ng) 2^24 and the FP32 product r_lo (1/ng), where r_hi =    */
/* floor(Q / 2^24) mod ng and r_lo = Q mod 2^24 for the position           */
/* Q = (c 2^24 + 2m + 1) N; the point is one fused multiply-add of the     */
/* offset and the scaled width onto the lower edge.  This mode changes     */
/* only the point handed to the integrand (the Jacobian and all arithmetic */
/* stay FP64); it lets a single-precision integrand be compared with this  */
/* one on identical inputs.                                                */
/* ===================================================================== */
static int g_point32 = 0;

void orc_set_point32(int on) { g_point32 = on ? 1 : 0; }

static double point32_offset(uint32_t word, int cube_coord, int ng, int nbins)
{
    uint64_t m = word >> 9;
    if (ng <= 1) return (double)(((2 * m + 1) * (uint64_t)nbins) & 0xFFFFFFu);
    uint64_t Q = ((uint64_t)cube_coord * (uint64_t)(1u << 24) + 2 * m + 1) * (uint64_t)nbins;
    if (nbins % ng == 0) return (double)(Q % ((uint64_t)ng << 24)) / (double)ng; /* an integer */
    uint64_t hi = Q >> 24;
    float r_hi = (float)(hi % (uint64_t)ng);
    float r_lo = (float)(Q & 0xFFFFFFu);
    float inv = (float)(1.0 / (double)ng);
    float lo_part = r_lo * inv;
    return (double)fmaf(r_hi, inv * 16777216.0f, lo_part);
}

static void point32_map(int d, int nbins, const double *edges, const int32_t *j, const uint32_t *words,
                        const int *cc, int ng, double *x)
{
    for (int a = 0; a < d; ++a) {
        const double *e = edges + (size_t)a * (size_t)(nbins + 1);
        float lo = (float)e[j[a]];
        float w = (float)((e[j[a] + 1] - e[j[a]]) / TWO24);
        float off = (float)point32_offset(words[a], cc ? cc[a] : 0, ng, nbins);
        x[a] = (double)fmaf(off, w, lo);
    }
}

/* ===================================================================== */
/* Steps 2-4 for one iteration.                                           */
/* ===================================================================== */
typedef struct {
    int id, d, nbins, ng, ntheta, ngrad;
    const double *edges, *theta;
    uint64_t seed;
    uint32_t it, kid;
    int64_t ncubes; /* ng^d in stratified mode */
} problem;

/* Evaluate sample s: its words, bins, point, Jacobian, f and grad. */
static double eval_sample(const problem *pb, uint32_t s, uint32_t *words, int32_t *j, double *x,
                          double *jac, double *f, double *grad)
{
    uint32_t wloc[ORC_MAXD];
    double delta[ORC_MAXD];
    int cc[ORC_MAXD];
    if (!words) words = wloc;
    orc_sample_words(pb->seed, s, pb->it, pb->kid, pb->d, words);
    if (pb->ng <= 1) {
        for (int a = 0; a < pb->d; ++a) {
            int jj;
            orc_bin_plain(words[a], pb->nbins, &jj, &delta[a]);
            j[a] = jj;
        }
    } else {
        int64_t c = (int64_t)s % pb->ncubes;
        for (int a = 0; a < pb->d; ++a) {
            int jj;
            cc[a] = (int)(c % pb->ng);
            orc_bin_strat(words[a], cc[a], pb->ng, pb->nbins, &jj, &delta[a]);
            j[a] = jj;
            c /= pb->ng;
        }
    }
    double J = orc_map(pb->d, pb->nbins, pb->edges, j, delta, x);
    if (g_point32) point32_map(pb->d, pb->nbins, pb->edges, j, words, pb->ng > 1 ? cc : NULL, pb->ng, x);
    double fv = orc_integrand(pb->id, pb->d, x, pb->theta, pb->ntheta, grad);
    if (jac) *jac = J;
    if (f) *f = fv;
    return fv * J;
}

/* The grid, integrand and stream of a problem, without a call count. */
static int setup_grid_problem(problem *pb, int id, int d, int nbins, const double *edges, int ng,
                              const double *theta, int ntheta, uint64_t seed, uint32_t it, uint32_t kid)
{
    if (d < 1 || d > ORC_MAXD) return ORC_E_DIM;
    if (nbins < 2 || nbins > 256) return ORC_E_NBINS;
    int rc = check_integrand(id, d, ntheta);
    if (rc) return rc;
    pb->id = id;
    pb->d = d;
    pb->nbins = nbins;
    pb->ng = ng;
    pb->ntheta = ntheta;
    pb->ngrad = orc_integrand_ngrad(id, d);
    pb->edges = edges;
    pb->theta = theta;
    pb->seed = seed;
    pb->it = it;
    pb->kid = kid;
    pb->ncubes = 1;
    if (ng > 1) {
        for (int a = 0; a < d; ++a) {
            pb->ncubes *= ng;
            if (pb->ncubes > (1LL << 40)) return ORC_E_STRAT;
        }
    }
    return ORC_OK;
}

static int setup_problem(problem *pb, int id, int d, int nbins, const double *edges, int ng,
                         const double *theta, int ntheta, int64_t ncall, uint64_t seed,
                         uint32_t it, uint32_t kid)
{
    int rc = setup_grid_problem(pb, id, d, nbins, edges, ng, theta, ntheta, seed, it, kid);
    if (rc) return rc;
    if (ncall < 2 || ncall > 4294967296LL) return ORC_E_NCALLS;
    if (ng > 1 && ncall / pb->ncubes < 2) return ORC_E_NCALLS;
    return ORC_OK;
}

int orc_iterate(int id, int d, int nbins, const double *edges, int ng,
                const double *theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t kid, double *bins, orc_iter_result *res,
                double *gsum, const float *w_in)
{
    problem pb;
    int rc = setup_problem(&pb, id, d, nbins, edges, ng, theta, ntheta, ncall, seed, it, kid);
    if (rc) return rc;
    int P = gsum ? pb.ngrad : 0;
    size_t nb = (size_t)d * (size_t)nbins;
    memset(bins, 0, 2 * nb * sizeof(double));
    memset(res, 0, sizeof *res);
    if (gsum) memset(gsum, 0, 5 * (size_t)pb.ngrad * sizeof(double));

    int32_t j[ORC_MAXD];
    double x[ORC_MAXD], jac, grad[ORC_MAXD + 8];

    /* one sample: accumulate w into the totals and the per-axis bins */
#define ACCUMULATE_SAMPLE(sidx, S1c, S2c, G1c, G2c)                                   \
    do {                                                                               \
        double w = eval_sample(&pb, (uint32_t)(sidx), NULL, j, x, &jac, NULL,          \
                               P ? grad : NULL);                                        \
        if (w_in) w = (double)w_in[(sidx)];                                            \
        if (!isfinite(w)) res->nonfinite++;                                            \
        res->S1 += w;                                                                  \
        res->S2 += w * w;                                                              \
        S1c += w;                                                                      \
        S2c += w * w;                                                                  \
        for (int a = 0; a < d; ++a) {                                                  \
            bins[(size_t)a * nbins + j[a]] += w;                                       \
            bins[nb + (size_t)a * nbins + j[a]] += w * w;                              \
        }                                                                              \
        for (int q = 0; q < P; ++q) {                                                  \
            double wg = jac * grad[q];                                                 \
            gsum[5 * q + 0] += wg;                                                     \
            gsum[5 * q + 1] += wg * wg;                                                \
            G1c[q] += wg;                                                              \
            G2c[q] += wg * wg;                                                         \
        }                                                                              \
    } while (0)

    double G1c[ORC_MAXD + 8], G2c[ORC_MAXD + 8];
    if (ng <= 1) {
        double S1c = 0.0, S2c = 0.0;
        for (int q = 0; q < P; ++q) G1c[q] = G2c[q] = 0.0;
        for (int64_t s = 0; s < ncall; ++s) ACCUMULATE_SAMPLE(s, S1c, S2c, G1c, G2c);
        double N = (double)ncall;
        res->n_eff = ncall;
        res->I = res->S1 / N;
        res->var = (res->S2 / N - res->I * res->I) / (N - 1.0);
        for (int q = 0; q < P; ++q) {
            double Gq = gsum[5 * q] / N;
            gsum[5 * q + 3] = Gq;
            gsum[5 * q + 4] = (gsum[5 * q + 1] / N - Gq * Gq) / (N - 1.0);
        }
    } else {
        int64_t M = pb.ncubes;
        int64_t k = ncall / M;
        for (int64_t c = 0; c < M; ++c) {
            double S1c = 0.0, S2c = 0.0;
            for (int q = 0; q < P; ++q) G1c[q] = G2c[q] = 0.0;
            for (int64_t t = 0; t < k; ++t) ACCUMULATE_SAMPLE(c + t * M, S1c, S2c, G1c, G2c);
            res->V += (double)k * S2c - S1c * S1c;
            for (int q = 0; q < P; ++q) gsum[5 * q + 2] += (double)k * G2c[q] - G1c[q] * G1c[q];
        }
        double N = (double)(k * M), kd = (double)k, Md = (double)M;
        double denom = kd * kd * (kd - 1.0) * Md * Md;
        res->n_eff = k * M;
        res->I = res->S1 / N;
        res->var = res->V / denom;
        for (int q = 0; q < P; ++q) {
            gsum[5 * q + 3] = gsum[5 * q] / N;
            gsum[5 * q + 4] = gsum[5 * q + 2] / denom;
        }
    }
#undef ACCUMULATE_SAMPLE
    return ORC_OK;
}

int orc_accumulate_range(int id, int d, int nbins, const double *edges, const double *theta, int ntheta,
                         int64_t ncall, uint64_t seed, uint32_t it, uint32_t kid, int64_t s0, int64_t s1,
                         double *bins, orc_iter_result *res)
{
    problem pb;
    int rc = setup_problem(&pb, id, d, nbins, edges, 1, theta, ntheta, ncall, seed, it, kid);
    if (rc) return rc;
    if (s0 < 0 || s1 < s0 || s1 > ncall) return ORC_E_INVALID;
    size_t nb = (size_t)d * (size_t)nbins;
    memset(bins, 0, 2 * nb * sizeof(double));
    memset(res, 0, sizeof *res);
    int32_t j[ORC_MAXD];
    double x[ORC_MAXD], jac;
    for (int64_t s = s0; s < s1; ++s) {
        double w = eval_sample(&pb, (uint32_t)s, NULL, j, x, &jac, NULL, NULL);
        if (!isfinite(w)) res->nonfinite++;
        res->S1 += w;
        res->S2 += w * w;
        for (int a = 0; a < d; ++a) {
            bins[(size_t)a * nbins + j[a]] += w;
            bins[nb + (size_t)a * nbins + j[a]] += w * w;
        }
    }
    res->n_eff = s1 - s0;
    return ORC_OK;
}

void orc_estimate_plain(orc_iter_result *res, int64_t ncall)
{
    double N = (double)ncall;
    res->n_eff = ncall;
    res->I = res->S1 / N;
    res->var = (res->S2 / N - res->I * res->I) / (N - 1.0);
}

int orc_eval_samples(int id, int d, int nbins, const double *edges, int ng,
                     const double *theta, int ntheta, int64_t ncall, uint64_t seed,
                     uint32_t it, uint32_t kid, int64_t s0, int64_t count,
                     uint32_t *words, int32_t *j, double *x, double *jac, double *f, double *w,
                     double *grad)
{
    problem pb;
    int rc = setup_problem(&pb, id, d, nbins, edges, ng, theta, ntheta, ncall, seed, it, kid);
    if (rc) return rc;
    if (s0 < 0 || count < 0 || s0 + count > 4294967296LL) return ORC_E_INVALID;
    int32_t jl[ORC_MAXD];
    double xl[ORC_MAXD], gl[ORC_MAXD + 8];
    for (int64_t i = 0; i < count; ++i) {
        double J, fv;
        double wv = eval_sample(&pb, (uint32_t)(s0 + i), words ? words + i * d : NULL, jl, xl, &J, &fv,
                                gl);
        if (j) memcpy(j + i * d, jl, d * sizeof(int32_t));
        if (x) memcpy(x + i * d, xl, d * sizeof(double));
        if (jac) jac[i] = J;
        if (f) f[i] = fv;
        if (w) w[i] = wv;
        if (grad && pb.ngrad > 0) memcpy(grad + i * pb.ngrad, gl, pb.ngrad * sizeof(double));
    }
    return ORC_OK;
}

/* ===================================================================== */
/* SPRING: unweighted events from the result of the BASES integration     */
/* phase (Sec. 3.1; Kawabata, CPC 41 (1986) 127).  Reading used here: the  */
/* integration phase records the largest weight w = f J seen in each      */
/* cube; the envelope g_c >= that maximum is constant on cube c.  A trial */
/* picks a cube with probability proportional to g_c, a point uniform in */
/* the cube's y-range (mapped through the frozen grid), and keeps it when */
/* u g_c < w.  Kept points are distributed as w(y) dy, i.e. as f(x) dx,    */
/* wherever w <= g_c (a trial with w > g_c is kept and counted as an      */
/* overflow).  The envelope is held as integers, q_c quanta of            */
/* gmax / 2^20 each, so that the running sums and the cube choice are     */
/* exact integer arithmetic.                                              */
/* ===================================================================== */
#define ORC_SPRING_QSCALE 1048576.0 /* 2^20 quanta at the largest cube maximum */
#define ORC_SPRING_TAG 2u           /* counter word 1 = group | tag << 8       */

int orc_cube_max(int id, int d, int nbins, const double *edges, int ng, const double *theta, int ntheta,
                 int64_t ncall, uint64_t seed, uint32_t it, double *wmax)
{
    problem pb;
    if (ng <= 1) return ORC_E_STRAT;
    int rc = setup_problem(&pb, id, d, nbins, edges, ng, theta, ntheta, ncall, seed, it, 0);
    if (rc) return rc;
    int64_t M = pb.ncubes, k = ncall / pb.ncubes;
    int32_t j[ORC_MAXD];
    double x[ORC_MAXD], jac;
    for (int64_t c = 0; c < M; ++c)
        for (int64_t t = 0; t < k; ++t) {
            double w = eval_sample(&pb, (uint32_t)(c + t * M), NULL, j, x, &jac, NULL, NULL);
            if (w > wmax[c]) wmax[c] = w; /* NaN never replaces the maximum */
        }
    return ORC_OK;
}

int orc_spring_envelope(int64_t M, const double *wmax, uint64_t *q, double *unit)
{
    if (M < 1) return ORC_E_INVALID;
    double gmax = 0.0;
    for (int64_t c = 0; c < M; ++c) {
        if (wmax[c] > gmax) gmax = wmax[c];
    }
    if (!(gmax > 0.0) || isinf(gmax)) return ORC_E_INVALID;
    for (int64_t c = 0; c < M; ++c)
        q[c] = wmax[c] > 0.0 ? (uint64_t)ceil((wmax[c] / gmax) * ORC_SPRING_QSCALE) : 0u;
    *unit = gmax / ORC_SPRING_QSCALE;
    return ORC_OK;
}

int64_t orc_spring_pick(int64_t M, const uint64_t *P, uint64_t r64)
{
    /* P[0..M] running sums of q; r = floor(r64 T / 2^64) is uniform over
     * [0, T); the cube is the last c with P[c] <= r */
    uint64_t T = P[M];
    uint64_t r = (uint64_t)(((unsigned __int128)r64 * T) >> 64);
    int64_t lo = 0, hi = M - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (P[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

int orc_spring_trials(int id, int d, int nbins, const double *edges, int ng, const double *theta, int ntheta,
                      const uint64_t *q, double unit, uint64_t seed, uint32_t pass, uint64_t trial0,
                      int64_t ntrials, int64_t *cube, double *x, double *w, double *env, double *u,
                      int32_t *kept)
{
    problem pb;
    if (ng <= 1) return ORC_E_STRAT;
    int rc = setup_grid_problem(&pb, id, d, nbins, edges, ng, theta, ntheta, seed, pass, 0);
    if (rc) return rc;
    int64_t M = pb.ncubes;
    if (M > (1LL << 28) || ntrials < 0) return ORC_E_INVALID;
    uint64_t *P = (uint64_t *)malloc((size_t)(M + 1) * sizeof(uint64_t));
    if (!P) return ORC_E_INVALID;
    P[0] = 0;
    for (int64_t c = 0; c < M; ++c) P[c + 1] = P[c] + q[c];
    if (P[M] == 0) {
        free(P);
        return ORC_E_INVALID;
    }
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    int nw = d + 3;
    for (int64_t i = 0; i < ntrials; ++i) {
        uint64_t t = trial0 + (uint64_t)i;
        /* words 0..d-1: the point in the cube; d, d+1: the cube choice (low,
         * high half of a 64-bit integer); d+2: the acceptance uniform */
        uint32_t words[ORC_MAXD + 4];
        for (int a = 0; a < nw; a += 4) {
            uint32_t ctr[4] = {(uint32_t)t, (uint32_t)(a / 4) | (ORC_SPRING_TAG << 8), pass, (uint32_t)(t >> 32)};
            uint32_t out[4];
            orc_philox4x32_10(ctr, key, out);
            for (int b = 0; b < 4 && a + b < nw; ++b) words[a + b] = out[b];
        }
        uint64_t r64 = ((uint64_t)words[d + 1] << 32) | words[d];
        int64_t c = orc_spring_pick(M, P, r64);
        int32_t j[ORC_MAXD];
        double delta[ORC_MAXD], xl[ORC_MAXD];
        int64_t cc = c;
        for (int a = 0; a < d; ++a) {
            int jj;
            orc_bin_strat(words[a], (int)(cc % ng), ng, nbins, &jj, &delta[a]);
            j[a] = jj;
            cc /= ng;
        }
        double J = orc_map(d, nbins, edges, j, delta, xl);
        double wv = orc_integrand(id, d, xl, theta, ntheta, NULL) * J;
        double g = (double)(P[c + 1] - P[c]) * unit;
        double ua = orc_uniform(words[d + 2]);
        if (cube) cube[i] = c;
        if (x) memcpy(x + i * d, xl, (size_t)d * sizeof(double));
        if (w) w[i] = wv;
        if (env) env[i] = g;
        if (u) u[i] = ua;
        if (kept) kept[i] = (ua * g < wv) ? 1 : 0;
    }
    free(P);
    return ORC_OK;
}

/* ===================================================================== */
/* Step 5: grid refinement, classic VEGAS, axis by axis.                   */
/*  1. d_j = sum of w^2 of the samples that fell in bin j;                 */
/*  2. smooth with the neighbours (3-point average, 2-point at the ends);  */
/*  3. normalise, rho_j = dbar_j / sum dbar (axis left alone if the sum is */
/*     zero);                                                             */
/*  4. damp: r_j = ((1 - rho_j)/(-ln rho_j))^alpha (r = 0 at rho = 0 and   */
/*     r = 1 at rho = 1, the limits);                                      */
/*  5. place the new edges so that every new bin holds the same share of   */
/*     sum r, with r_j spread uniformly over old bin j.                    */
/* ===================================================================== */
int orc_refine(int d, int nbins, const double *edges_in, const double *b2, double alpha, double *edges_out)
{
    if (d < 1 || d > ORC_MAXD) return ORC_E_DIM;
    if (nbins < 2 || nbins > 256) return ORC_E_NBINS;
    if (!(alpha >= 0.0)) return ORC_E_INVALID;
    int N = nbins;
    double dbar[256], r[256], C[257];
    for (int a = 0; a < d; ++a) {
        const double *e = edges_in + (size_t)a * (N + 1);
        double *eo = edges_out + (size_t)a * (N + 1);
        const double *dv = b2 + (size_t)a * N;
        dbar[0] = (dv[0] + dv[1]) / 2.0;
        dbar[N - 1] = (dv[N - 2] + dv[N - 1]) / 2.0;
        for (int i = 1; i < N - 1; ++i) dbar[i] = (dv[i - 1] + dv[i] + dv[i + 1]) / 3.0;
        double D = 0.0;
        for (int i = 0; i < N; ++i) D += dbar[i];
        if (!(D > 0.0) || !isfinite(D)) {
            memmove(eo, e, (N + 1) * sizeof(double));
            continue;
        }
        for (int i = 0; i < N; ++i) {
            double rho = dbar[i] / D;
            double base;
            if (rho <= 0.0)
                base = 0.0;
            else if (rho >= 1.0)
                base = 1.0;
            else
                base = (1.0 - rho) / (-log(rho));
            r[i] = pow(base, alpha);
        }
        C[0] = 0.0;
        for (int i = 0; i < N; ++i) C[i + 1] = C[i] + r[i];
        double T = C[N] / N;
        double enew[257];
        enew[0] = e[0];
        enew[N] = e[N];
        int jj = 0;
        for (int kk = 1; kk < N; ++kk) {
            double target = kk * T;
            while (jj < N - 1 && C[jj + 1] <= target) ++jj;
            enew[kk] = e[jj] + ((target - C[jj]) / r[jj]) * (e[jj + 1] - e[jj]);
        }
        memcpy(eo, enew, (N + 1) * sizeof(double));
    }
    return ORC_OK;
}

/* ===================================================================== */
/* Step 6: combination of iterations, weights 1/var_k:                     */
/*   Ibar = sum(I_k/var_k)/sum(1/var_k), sigbar = sum(1/var_k)^-1/2,       */
/*   chi2/dof = sum (I_k - Ibar)^2/var_k / (m-1).                          */
/* Iterations with var_k = 0 are exact: if any, Ibar is their mean and    */
/* sigbar = 0 (chi2/dof then reported as 0).                               */
/* ===================================================================== */
void orc_combine(int m, const double *I, const double *var, double *Ibar, double *sigbar, double *chi2dof)
{
    int nexact = 0;
    double sum_exact = 0.0;
    for (int k = 0; k < m; ++k)
        if (var[k] == 0.0) {
            nexact++;
            sum_exact += I[k];
        }
    if (nexact > 0) {
        *Ibar = sum_exact / nexact;
        *sigbar = 0.0;
        *chi2dof = 0.0;
        return;
    }
    double W = 0.0, WI = 0.0;
    for (int k = 0; k < m; ++k) {
        W += 1.0 / var[k];
        WI += I[k] / var[k];
    }
    double mean = WI / W;
    double chi2 = 0.0;
    for (int k = 0; k < m; ++k) chi2 += (I[k] - mean) * (I[k] - mean) / var[k];
    *Ibar = mean;
    *sigbar = 1.0 / sqrt(W);
    *chi2dof = (m > 1) ? chi2 / (m - 1) : NAN;
}
