/*
 * vmc_oracle.h -- plain FP64 CPU oracle for the VEGAS/BASES iteration of
 * Kanzaki, "Monte Carlo integration on GPU" (arXiv:1010.2107).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the CPU-baseline leg of the benchmark can check the GPU
 * library against an independent, slow, obviously-correct implementation.
 * No product code links, loads or calls it, and it shares no code, header,
 * table or constant with the GPU library.
 *
 * The paper states the method in prose only (Sec. 2 and the six-step
 * program structure of Sec. 3.1).  The steps are taken from the published
 * methods it builds on:
 *   - Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *     as easy as 1, 2, 3", SC'11.
 *   - VEGAS grid, bin statistic, smoothing, damping, rebinning and the
 *     combination of iterations: Lepage, J. Comput. Phys. 27 (1978) 192.
 *   - BASES stratification: Kawabata, Comput. Phys. Commun. 41 (1986) 127.
 *   - Massless n-body phase space with 3n-4 variables: Plaetzer, "RAMBO on
 *     diet", arXiv:1308.2922; flat weight as in Kleiss, Stirling, Ellis,
 *     Comput. Phys. Commun. 40 (1986) 359.
 *   - Colour-ordered MHV denominators: Parke, Taylor, PRL 56 (1986) 2459.
 *
 * Everything is double precision.  All functions are re-entrant except the
 * lazily built cyclic-order table (built once, guarded by a flag; call
 * orc_init() from one thread first if that matters).
 */
#ifndef VMC_ORACLE_H
#define VMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Integrand identifiers (the same numbering is used by the GPU library's
 * public header; the numbering is an interface, not shared code). */
enum {
    ORC_CONST = 0,      /* f = theta[0]                                  */
    ORC_LINEAR = 1,     /* f = x_0                                       */
    ORC_GAUSS = 2,      /* prod_a phi(x_a;c,s) / G(c,s)^d, theta=(c,s)   */
    ORC_DGAUSS = 3,     /* double Gaussian, theta=(c1,c2,s)              */
    ORC_GAUSS_AXES = 4, /* prod_a phi(x_a;c_a,s)/(s sqrt(pi)), theta=(c_0..c_{d-1},s) */
    ORC_WJETS = 5,      /* W(->e nu) + n_p partons toy cross section     */
    ORC_PSVOL = 6,      /* PDF x phase-space weight only (no cuts, |M|^2=1) */
    ORC_WHEL = 7        /* u dbar -> W+(-> mu+ nu) + n gluons, helicity amplitudes, d = 3n+5 */
};

/* Error codes returned by the int-valued functions. */
enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_DIM = -2,
    ORC_E_NBINS = -3,
    ORC_E_NCALLS = -4,
    ORC_E_INTEGRAND = -5,
    ORC_E_PARAMS = -6,
    ORC_E_STRAT = -7
};

/* ---------------------------------------------------------------- Philox */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The d random words of sample s of iteration `it` of integral `kid`:
 * word a is word (a mod 4) of the Philox block with counter
 * (s, a div 4, it, kid) and key (seed lo 32 bits, seed hi 32 bits). */
void orc_sample_words(uint64_t seed, uint32_t s, uint32_t it, uint32_t kid, int d, uint32_t *out);

/* ------------------------------------------------- uniforms and bin index */
double orc_uniform(uint32_t word);
void orc_bin_plain(uint32_t word, int nbins, int *j, double *delta);
void orc_bin_strat(uint32_t word, int cube_coord, int ng, int nbins, int *j, double *delta);
/* batch forms for exhaustive tests; ng <= 1 selects the plain form */
void orc_bin_batch(int64_t n, const uint32_t *words, const int32_t *cube_coord, int ng,
                   int nbins, int32_t *j, double *delta);

/* ------------------------------------------------------------ grid map */
/* x_a = e[a][j_a] + delta_a * (e[a][j_a+1]-e[a][j_a]);  returns J = prod N*width */
double orc_map(int d, int nbins, const double *edges, const int32_t *j, const double *delta, double *x);
/* Hand the integrand the point as a single-precision grid map forms it
 * (on != 0) or the FP64 point (0, the default).  Process-wide setting. */
void orc_set_point32(int on);

/* ----------------------------------------------------------- integrands */
int orc_integrand_nparams(int id, int d);   /* theta length, <0 on error   */
int orc_integrand_ngrad(int id, int d);     /* number of differentiable params */
/* f(x; theta); if grad != NULL also writes df/dtheta_p for p < ngrad. */
double orc_integrand(int id, int d, const double *x, const double *theta, int ntheta, double *grad);

/* physics pieces, exposed for the tests */
double orc_rambo_diet(int n, double sqrt_shat, const double *r, double *p /* [n][4] */);
double orc_massless_ps_volume(int n, double shat);
int orc_solve_mass_fraction(int n, int i, double r, double *t);
int orc_pass_cuts(int n_p, const double *p /* [n_p+2][4], CM frame */, double y_boost,
                  double ptmin, double etamax, double drmin);
double orc_cyclic_sum(int m, const double *s /* [m][m] symmetric */);
int orc_num_cycles(int m);
/* W + n_p partons event: fills momenta p[n][4] (CM frame, order j_1..j_np, e, nu)
 * and aux = {x1, x2, shat, Jx, lum, Vn, m_enu^2, pass}; returns f (0 when cut). */
double orc_wjets_event(int d, const double *x, const double *theta, int ntheta,
                       double *p, double *aux, double *grad);

/* u dbar -> W+(-> mu+ nu) + n gluons (n = (d-5)/3 <= 2), see the .c file.
 * theta = (M_W, Gamma_W, g_s, sqrtS, pTmin, etamax_mu, etamax_g, pTij_min).
 *  orc_whel_partials: colour-ordered amplitudes for given momenta (pu, pd,
 *    k_1..k_n, p_mu, p_nu) and gluon polarisation vectors (re[4], im[4] each)
 *  orc_whel_me2: colour-summed |M|^2 for gluon helicity bits hel
 *  orc_whel_event: f at x[d], momenta p[(n+2)][4] (g.., mu, nu; partonic
 *    frame), aux as orc_wjets_event; grad w.r.t. (M_W, Gamma_W, g_s) */
int orc_whel_partials(int n, const double *mom, const double *eps, double *A);
double orc_whel_me2(int n, const double *mom, int hel, const double *theta);
int orc_whel_pass_cuts(int n, const double *p, double y_boost, double ptmin, double eta_mu, double eta_g,
                       double ptij_min);
double orc_whel_event(int d, const double *x, const double *theta, int ntheta, double *p, double *aux,
                      double *grad);

/* ------------------------------------------------------------ iteration */
typedef struct {
    double S1, S2;      /* sum w, sum w^2 over all samples                     */
    double V;           /* stratified: sum_c (k S2_c - S1_c^2); 0 in plain mode */
    double I, var;      /* this iteration's estimate and its variance          */
    int64_t n_eff;      /* samples used                                        */
    int64_t nonfinite;  /* samples whose w was NaN or Inf                      */
} orc_iter_result;

/* One iteration of sample -> map -> f -> accumulate.
 *  edges  [d][nbins+1]; bins out [2][d][nbins] (plane 0: sum w, plane 1: sum w^2)
 *  ng <= 1 plain mode, else stratified with ng^d cubes, k = ncall div ng^d >= 2.
 *  gsum (may be NULL) receives per differentiable parameter p the triple
 *  {sum J df/dp, sum (J df/dp)^2, V_p} followed by {G_p, var G_p} (5 per p).
 *  w_in (may be NULL): replay mode -- use (double)w_in[s] instead of f*J.
 */
int orc_iterate(int id, int d, int nbins, const double *edges, int ng,
                const double *theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t kid, double *bins, orc_iter_result *res,
                double *gsum, const float *w_in);

/* Plain-mode sums over the sample range [s0, s1) only (I and var are left
 * 0): disjoint ranges added together give exactly the sums of orc_iterate
 * up to summation order; orc_estimate_plain then forms I and var from the
 * merged sums of all ncall samples. */
int orc_accumulate_range(int id, int d, int nbins, const double *edges, const double *theta, int ntheta,
                         int64_t ncall, uint64_t seed, uint32_t it, uint32_t kid, int64_t s0, int64_t s1,
                         double *bins, orc_iter_result *res);
void orc_estimate_plain(orc_iter_result *res, int64_t ncall);

/* Per-sample dump for samples s0 .. s0+count-1 (stratified when ng > 1).
 * Any output pointer may be NULL. */
int orc_eval_samples(int id, int d, int nbins, const double *edges, int ng,
                     const double *theta, int ntheta, int64_t ncall, uint64_t seed,
                     uint32_t it, uint32_t kid, int64_t s0, int64_t count,
                     uint32_t *words, int32_t *j, double *x, double *jac, double *f, double *w,
                     double *grad /* [count][ngrad] */);

/* SPRING (unweighted events from the BASES integration phase), see the .c
 * file for the reading.  Stratified mode only (ng >= 2).
 *  orc_cube_max: fold the largest w of each cube of one iteration into
 *    wmax[ng^d] (the caller zeroes it before the first iteration).
 *  orc_spring_envelope: q[c] = ceil(wmax[c]/gmax 2^20) (0 where wmax <= 0),
 *    *unit = gmax / 2^20; ORC_E_INVALID when no cube has a positive finite max.
 *  orc_spring_pick: the cube of a 64-bit random integer, P = running sums of q.
 *  orc_spring_trials: trials trial0 .. trial0+ntrials-1 of pass `pass`; per
 *    trial its cube, point x[d], weight w, envelope value g_c, acceptance
 *    uniform u and whether it is kept (u g_c < w).  Any output may be NULL. */
int orc_cube_max(int id, int d, int nbins, const double *edges, int ng, const double *theta, int ntheta,
                 int64_t ncall, uint64_t seed, uint32_t it, double *wmax);
int orc_spring_envelope(int64_t M, const double *wmax, uint64_t *q, double *unit);
int64_t orc_spring_pick(int64_t M, const uint64_t *P, uint64_t r64);
int orc_spring_trials(int id, int d, int nbins, const double *edges, int ng, const double *theta, int ntheta,
                      const uint64_t *q, double unit, uint64_t seed, uint32_t pass, uint64_t trial0,
                      int64_t ntrials, int64_t *cube, double *x, double *w, double *env, double *u,
                      int32_t *kept);

/* Grid refinement of every axis (classic VEGAS), see the .c file. */
int orc_refine(int d, int nbins, const double *edges_in, const double *b2 /* [d][nbins] */,
               double alpha, double *edges_out);

/* Weighted combination of m iteration results. */
void orc_combine(int m, const double *I, const double *var, double *Ibar, double *sigbar,
                 double *chi2dof);

#ifdef __cplusplus
}
#endif
#endif
