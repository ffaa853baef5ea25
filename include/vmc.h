/*
 * vmc.h -- C ABI of libvmc.so, an MI355X (gfx950) implementation of the
 * per-iteration sample-and-accumulate pass and grid refinement of the
 * VEGAS and BASES adaptive Monte Carlo integrators as parallelised on a
 * GPU in Kanzaki, "Monte Carlo integration on GPU" (arXiv:1010.2107).
 *
 * The paper's user-facing parameters are the dimension (ndim), calls per
 * iteration (NCALL), iteration count (ITMX) and accuracy (ACC), plus
 * BASES's grid-optimisation / integration phase split (ITMX1, ITMX2)
 * (Sec. 6.1 and Appendix A.1.1).  One iteration is steps 2-5 of the
 * six-step program structure of Sec. 3.1: make points from random numbers,
 * evaluate the integrand, accumulate, and re-optimise the grid.  In this
 * library all four run on the GPU; only the driver loop (step 6) is on the
 * host, and it never needs a device-to-host copy inside the loop.
 *
 * Conventions
 *  - Every call returns 0 (VMC_OK) or a negative VMC_E_* code and never
 *    throws; vmc_last_error() gives a message for the calling thread.
 *  - Device memory is owned by the caller and bound to a grid handle with
 *    vmc_bind(); the library never allocates device memory.  Sizes come
 *    from vmc_workspace_sizes().
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *    enqueued on it in call order; no call synchronises the host, except
 *    vmc_get_edges / vmc_set_edges, which copy synchronously.
 *  - A handle is not thread-safe: do not use one handle from two host
 *    threads at once.
 *  - Integrands are compiled in and chosen by their VMC_* id (the paper's
 *    gVEGAS likewise compiles the user function into the kernel).
 */
#ifndef VMC_H
#define VMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- errors */
#define VMC_OK 0
#define VMC_E_INVALID (-1)   /* bad argument not covered below                */
#define VMC_E_DIM (-2)       /* dimension outside [1,16] or not compiled in     */
#define VMC_E_NBINS (-3)     /* bins per axis outside [2,256]                   */
#define VMC_E_NCALLS (-4)    /* ncall < 2, ncall > 2^32, or < 2 per cube        */
#define VMC_E_INTEGRAND (-5) /* unknown integrand id                            */
#define VMC_E_PARAMS (-6)    /* wrong ntheta                                    */
#define VMC_E_STRAT (-7)     /* ng^dim > 2^40                                   */
#define VMC_E_GRID (-8)      /* edges not strictly increasing from 0 to 1, or an */
                             /* adjoint pass on a grid that moved since its     */
                             /* forward pass                                    */
#define VMC_E_HIP (-9)       /* a HIP runtime call or launch failed             */
#define VMC_E_UNBOUND (-10)  /* device buffers not bound with vmc_bind()        */
#define VMC_E_SCHEDULE (-11) /* schedule values outside their documented range  */
#define VMC_E_SPRING (-12)   /* SPRING set-up missing or impossible             */

/* --------------------------------------------------------- integrands */
/* theta is a device array of doubles of the stated length.               */
#define VMC_CONST 0      /* f = theta[0]; ntheta 1, 1 gradient               */
#define VMC_LINEAR 1     /* f = x_0; ntheta 0                                */
#define VMC_GAUSS 2      /* prod_a exp(-(x_a-c)^2/s^2) / G(c,s)^d with        */
                         /* G = int_0^1 exp(-(x-c)^2/s^2) dx; theta (c, s)    */
#define VMC_DGAUSS 3     /* [prod_a phi(x_a;c1,s)/G(c1,s) + same with c2]/2; */
                         /* theta (c1, c2, s)                                 */
#define VMC_GAUSS_AXES 4 /* prod_a exp(-(x_a-c_a)^2/s^2)/(s sqrt(pi));       */
                         /* theta (c_0..c_{d-1}, s), d+1 gradients            */
#define VMC_WJETS 5      /* pp -> W(-> e nu) + n_p partons toy, d = 3 n_p + 4 */
                         /* (n_p = 1..4); theta (M, Gamma, g, sqrtS, pTmin,   */
                         /* etamax, dRmin); gradients w.r.t. (M, Gamma, g)    */
#define VMC_PSVOL 6      /* PDF x massless phase-space weight of VMC_WJETS    */
                         /* without cuts or |M|^2; theta (sqrtS, pTmin)       */
#define VMC_WHEL 7       /* u dbar -> W+(-> mu+ nu) + n gluons (Sec. 5, eq. 1)*/
                         /* from helicity amplitudes, n = 0..2, d = 3n + 5   */
                         /* (last variable: gluon helicities); theta (M,     */
                         /* Gamma, g_s, sqrtS, pTmin, etamax_mu, etamax_g,    */
                         /* pTij_min); gradients w.r.t. (M, Gamma, g_s)       */

/* iterate flags */
#define VMC_FLAG_FP64 1u /* evaluate map and integrand in double precision   */
                         /* (test instantiation; sums are FP64 either way)    */

/* ------------------------------------------------ scalar block layout */
/* vmc_bind's `scal` array (VMC_SCAL_LEN doubles) holds, after an        */
/* iteration has completed on the stream:                                 */
#define VMC_S_S1 0        /* sum w, w = f J                                   */
#define VMC_S_S2 1        /* sum w^2                                          */
#define VMC_S_V 2         /* stratified: sum_c (k S2_c - S1_c^2)              */
#define VMC_S_NONFINITE 3 /* samples with non-finite w                        */
#define VMC_S_I 4         /* this iteration's estimate I_k                    */
#define VMC_S_VAR 5       /* its variance                                     */
#define VMC_S_NEFF 6      /* samples used this iteration                      */
#define VMC_S_NZERO 7     /* samples with w = 0 (e.g. outside the cuts)       */
#define VMC_S_IBAR 14     /* combined estimate over the iterations folded in  */
#define VMC_S_SIGBAR 15   /* its standard deviation                           */
#define VMC_S_CHI2 16     /* chi^2 per degree of freedom (NaN for one)        */
#define VMC_S_NITER 11    /* number of iterations folded in                   */
#define VMC_S_GRAD 32     /* adjoint: 5 doubles per gradient p:               */
                          /* {sum J df/dp, sum (J df/dp)^2, V_p, G_p, var G_p}*/
#define VMC_SCAL_LEN 128
#define VMC_MAX_GRAD 17

typedef struct vmc_grid_s *vmc_grid_t;

/* Last error message of the calling thread ("" if none). */
const char *vmc_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int vmc_version(void);

/* Bytes of the four device buffers a (dim, nbins) grid needs:
 *   out[0] edges  double[dim][nbins+1]   FP64 bin edges, row per axis
 *   out[1] table  float [dim][nbins][2]  FP32 (lower edge, width x 2^-32) per bin
 *   out[2] bins   double[2][dim][nbins]  plane 0: sum w per bin,
 *                                        plane 1: sum w^2 per bin,
 *                 followed by a library-private tail (the blocks' partial
 *                 sums in 32 copies, about 64 x the two planes; zero
 *                 between calls; not used by vmc_iterate_static)
 *   out[3] scal   double[VMC_SCAL_LEN]   scalar block (layout above)
 * Errors: VMC_E_DIM, VMC_E_NBINS. */
int vmc_workspace_sizes(int dim, int nbins, size_t out[4]);

/* Create a grid handle for `dim` axes of `nbins` bins each (Sec. 2: each
 * axis is divided into bins, the volume into hypercubes).  Plain (VEGAS)
 * sampling until bases_stratify() is called.  Errors: VMC_E_DIM (dim
 * outside [1,16]), VMC_E_NBINS (outside [2,256]), VMC_E_INVALID (out NULL). */
int vmc_create(int dim, int nbins, vmc_grid_t *out);

/* Release a handle (not the caller's device buffers). NULL is accepted. */
int vmc_destroy(vmc_grid_t g);

/* Bind caller-owned device buffers of at least the sizes given by
 * vmc_workspace_sizes().  They must stay allocated while the handle uses
 * them.  The library-private tail of the bins buffer is taken as unknown
 * and cleared before the next sample pass (vmc_reset clears everything and
 * sets the uniform grid).  Errors: VMC_E_INVALID (NULL handle or pointer). */
int vmc_bind(vmc_grid_t g, double *edges, float *table, double *bins, double *scal);

/* Reset to the uniform grid, clear the bin sums, the scalar block and the
 * running combination (stream-ordered); the private tail of the bins
 * buffer is cleared before the next pass that uses it.
 * Errors: VMC_E_UNBOUND, VMC_E_HIP. */
int vmc_reset(vmc_grid_t g, void *stream);

/* BASES-style stratification: split [0,1]^dim into ng^dim equal cubes and
 * draw k = ncall div ng^dim points in each (the samples of cube c are
 * s = c + t ng^dim, t < k).  ng <= 1 returns to plain sampling.  Any ng is
 * accepted (ng need not divide nbins).  Errors: VMC_E_STRAT (ng^dim > 2^40). */
int bases_stratify(vmc_grid_t g, int ng);

/* One iteration, steps 2-4 of Sec. 3.1 plus the estimate: draw ncall
 * points with Philox4x32-10 (seed, counter = (sample, word group, it, 0)),
 * map them through the grid, evaluate the integrand with parameters theta
 * (device doubles, ntheta of them), accumulate sum w, sum w^2 and the
 * per-axis per-bin sums (bins buffer), then write I_k and its variance and
 * fold them into the running combination (weights 1/var).  Stream-ordered:
 * the sample kernel (one tile of samples per block) and a small
 * publish kernel that adds up the blocks' partial sums and writes the bin
 * sums, the scalar block and the combination.  Calls on one handle must be
 * ordered on one stream: they share the bound buffers.
 * Errors: VMC_E_UNBOUND, VMC_E_INTEGRAND, VMC_E_PARAMS, VMC_E_NCALLS,
 * VMC_E_DIM (integrand not compiled for this dim), VMC_E_HIP. */
int vmc_iterate(vmc_grid_t g, int integrand, const double *theta, int ntheta, int64_t ncall,
                uint64_t seed, uint32_t it, uint32_t flags, void *stream);

/* vmc_iterate for callers that cannot allocate device memory or use a
 * workspace of their own (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same iteration, arguments
 * and results, with the blocks' partial sums kept in a static device array
 * of the library (32 copies of the 2 dim nbins bin sums and 64 scalar
 * slots, room for dim 16 x 256 bins: 2.02 MiB per GPU, held until the
 * process ends) instead of the private tail of the bound bins buffer, which
 * then needs only double[2][dim][nbins].  No call allocates; the first on a
 * device looks up the array's address and clears it with a kernel on
 * `stream`, and every pass leaves it at zero.  All calls on one GPU share
 * the array: calls that overlap in time on one GPU (on different streams or
 * from different host threads) race and must be ordered by the caller.
 * Errors: as vmc_iterate. */
int vmc_iterate_static(vmc_grid_t g, int integrand, const double *theta, int ntheta, int64_t ncall,
                       uint64_t seed, uint32_t it, uint32_t flags, void *stream);

/* Per-cube maxima for SPRING (Sec. 3.1: the results of the BASES
 * integration phase feed event generation).  While a buffer is bound,
 * every stratified vmc_iterate also folds the largest weight w = f J of
 * each cube c into cube_max[c] (max with the present value; NaN weights
 * never win).  The buffer is caller-owned device memory of ncubes >= ng^dim
 * doubles, zeroed by the caller at the start of the integration phase;
 * NULL unbinds.  Plain-mode iterations, vmc_iterate_adjoint and
 * vmc_iterate_fused leave it alone.  Errors: VMC_E_INVALID (also at
 * iterate time when ncubes < ng^dim). */
int bases_cube_max(vmc_grid_t g, double *cube_max, int64_t ncubes);

/* Step 5 of Sec. 3.1: re-optimise every axis from the plane-1 bin sums of
 * the last iteration: 3-point smoothing, normalisation, damping
 * ((1-rho)/(-ln rho))^alpha, and rebinning to equal damped weight; writes
 * new FP64 edges and the FP32 table.  An axis whose smoothed sum is zero
 * is left unchanged; alpha = 0 leaves every axis unchanged.
 * Errors: VMC_E_INVALID (alpha < 0 or NaN), VMC_E_UNBOUND, VMC_E_HIP. */
int vmc_refine(vmc_grid_t g, double alpha, void *stream);

/* Clear the running combination (BASES: start of the integration phase). */
int vmc_combine_reset(vmc_grid_t g, void *stream);

/* Gradient of the integral with respect to the integrand parameters on
 * the same samples as vmc_iterate with the same (seed, it) and the grid
 * unchanged since: accumulates sum J df/dtheta_p and its square (and the
 * per-cube form when stratified), then writes G_p and var G_p into the
 * scalar block at VMC_S_GRAD (the first ngrad of the 5-double groups, see
 * vmc_integrand_info; the groups beyond are left as they were).  It does
 * not touch the bin sums, S1/S2/V, the estimate or the running
 * combination.  The grid has not moved since the forward pass it
 * differentiates: the handle's grid-state version (vmc_grid_version) must
 * equal the one recorded by the last vmc_iterate or vmc_iterate_fused.
 * Errors: as vmc_iterate; VMC_E_INTEGRAND for an integrand without
 * parameters; VMC_E_GRID when no forward pass ran on the present grid
 * state (refine, set_edges, reset, stratify or bind since). */
int vmc_iterate_adjoint(vmc_grid_t g, int integrand, const double *theta, int ntheta, int64_t ncall,
                        uint64_t seed, uint32_t it, uint32_t flags, void *stream);

/* Forward and adjoint in one pass over the samples: the results of
 * vmc_iterate (bin sums, estimate, running combination) and of
 * vmc_iterate_adjoint (gradient block) at the cost of one sample pass.
 * Records the grid-state version as vmc_iterate does.  Errors: as
 * vmc_iterate, and VMC_E_INTEGRAND for an integrand without parameters. */
int vmc_iterate_fused(vmc_grid_t g, int integrand, const double *theta, int ntheta, int64_t ncall,
                      uint64_t seed, uint32_t it, uint32_t flags, void *stream);

/* Grid-state version of the handle: a counter advanced by vmc_bind,
 * vmc_reset, bases_stratify, vmc_refine and vmc_set_edges, i.e. by every
 * call that can move the samples of an iteration (paper Sec. 2: the grid is
 * re-optimised between iterations).  A caller that pairs a forward pass
 * with a later adjoint pass can record it and compare.
 * Errors: VMC_E_INVALID (NULL argument). */
int vmc_grid_version(vmc_grid_t g, uint64_t *version);

/* Parameters of a compiled integrand: *ntheta values in theta, of which
 * the first *ngrad are differentiated by the adjoint pass (either pointer
 * may be NULL).  Errors: VMC_E_INTEGRAND, VMC_E_DIM (not compiled for
 * this dimension and precision). */
int vmc_integrand_info(int integrand, int dim, uint32_t flags, int *ntheta, int *ngrad);

/* Copy the FP64 edges to / from host memory (synchronous on `stream`).
 * vmc_set_edges validates e[a][0] = 0, e[a][nbins] = 1 and strict increase
 * (VMC_E_GRID) and rebuilds the FP32 table. */
int vmc_get_edges(vmc_grid_t g, double *host_edges, void *stream);
int vmc_set_edges(vmc_grid_t g, const double *host_edges, void *stream);

/* Per-sample dump of samples s0 .. s0+count-1 of an iteration (same points
 * as vmc_iterate): the Philox words [count][dim] u32, the bin index of
 * every axis [count][dim] u8 (what the accumulation adds the sample into),
 * w = f J [count], f [count], J [count], and df/dtheta_p [count][ngrad].
 * Device arrays; w, f, jac and grad are float, or double with
 * VMC_FLAG_FP64; any may be NULL.  Used by the tests and by the paper's
 * split of the work (Sec. 3.2: the GPU evaluates, the host accumulates),
 * which needs the weights and the bin indices on the host.
 * Errors: as vmc_iterate; VMC_E_INVALID for a range beyond ncall (or
 * k ng^dim when stratified); VMC_E_INTEGRAND for grad with an integrand
 * without parameters. */
int vmc_dump_samples(vmc_grid_t g, int integrand, const double *theta, int ntheta, int64_t ncall,
                     uint64_t seed, uint32_t it, uint32_t flags, int64_t s0, int64_t count,
                     uint32_t *words, uint8_t *bins, void *w, void *f, void *jac, void *grad,
                     void *stream);

/* Launch shape of the sample kernels: one tile per thread block.
 * block_samples: samples (plain) or cube units (stratified) per tile, a
 * multiple of 256 in [256, 2^24], or 0 for the built-in choice (plain: at
 * least 1024 tiles of at most 8192 samples, and for the W + partons and
 * helicity integrands at least two tiles per block the device holds at
 * once unless that takes tiles below 1024 samples; stratified: 256 units, one
 * per thread, or up to 1024 when a unit holds few samples, toward 4096
 * samples per tile (8192 for the W + partons and helicity integrands), but
 * at least about 512 tiles);
 * chunks_per_cube: lanes that share one cube in stratified mode, a power of
 * two in [1, 256] (up to 64 share a wave, more span the waves of a block),
 * or 0 for the built-in choice (the smallest power of two with ng^dim x
 * lanes >= 2^18, at most 256 and at most k; then, for the W + partons and
 * helicity integrands, doubled toward 2^19 while each lane keeps at least
 * 8 samples).  Errors: VMC_E_SCHEDULE. */
int vmc_set_schedule(vmc_grid_t g, int block_samples, int chunks_per_cube);

/* Kernel timing with HIP events recorded on the launch stream around every
 * sample-kernel launch of this handle while enabled.  Each call waits for
 * the recorded launches, returns their summed duration (ms) and count
 * (either pointer may be NULL), forgets them, and then enables (enable != 0)
 * or disables recording.  Errors: VMC_E_INVALID, VMC_E_HIP. */
int vmc_timing(vmc_grid_t g, int enable, double *total_ms, int64_t *launches);

/* Calibration: the chip's LDS FP64 atomic-add rate (adds per second) with
 * one LDS double per lane and 8 independent adds per loop trip, `blocks`
 * blocks of 256 threads, `iters` trips.  Waits for the stream.  It bounds
 * the per-bin histogram step of the sample pass (Sec. 3.1 step 4: 2 dim LDS
 * atomics per sample).  Errors: VMC_E_INVALID, VMC_E_HIP. */
int vmc_probe_lds_atomics(int blocks, int iters, double *rate, void *stream);

/* Calibration: the chip's sustained FP32 fused multiply-add rate (flops per
 * second, 2 per FMA) with 8 independent FMA chains per lane, `blocks`
 * blocks of 256 threads, `iters` trips, at the clock the chip holds under
 * that load.  Waits for the stream.  It bounds the integrand arithmetic of
 * the sample pass (Sec. 3.1 step 3).  Errors: VMC_E_INVALID, VMC_E_HIP. */
int vmc_probe_fp32_fma(int blocks, int iters, double *flops, void *stream);

/* ------------------------------------------------------------ batches */
/* Many independent integrals of uneven dimension and call count advanced
 * together by one persistent launch per iteration.  Integral k has its own
 * grid (nbins per axis), parameters and accumulators; its samples use the
 * Philox counter (s, word group, it, k), so its results equal those of a
 * single-integral run with integral id k, whatever the schedule. */
typedef struct vmc_batch_s *vmc_batch_t;

/* n integrals; dims[k] in [1,12]; ncall[k] in [2, 2^32); integrand must be
 * VMC_GAUSS_AXES (theta_k = (c_0..c_{d_k-1}, s), d_k + 1 values).
 * Errors: VMC_E_INVALID, VMC_E_DIM, VMC_E_NCALLS, VMC_E_NBINS,
 * VMC_E_INTEGRAND. */
int vmc_batch_create(int n, const int *dims, int nbins, int integrand, const int64_t *ncall,
                     vmc_batch_t *out);
int vmc_batch_destroy(vmc_batch_t b);

/* Bytes of the six caller-owned device buffers, concatenated over k in
 * order: out[0] edges (d_k (nbins+1) doubles each), out[1] table (d_k nbins
 * float pairs), out[2] bins (2 d_k nbins doubles), out[3] scal
 * (VMC_SCAL_LEN doubles per integral, layout as for one grid), out[4] theta
 * (d_k + 1 doubles each, written by the caller), out[5] meta (work list for
 * the current schedule). */
int vmc_batch_workspace_sizes(vmc_batch_t b, size_t out[6]);

/* Bind the device buffers; meta_bytes is the size of `meta`.  Errors:
 * VMC_E_INVALID. */
int vmc_batch_bind(vmc_batch_t b, double *edges, float *table, double *bins, double *scal,
                   const double *theta, void *meta, size_t meta_bytes);

/* Schedule of the persistent launch: samples_per_thread sets the tile
 * size (256 x samples_per_thread samples of one integral), blocks the
 * persistent grid; 0 selects the built-in value.  Changes the work list
 * (re-query out[5] of vmc_batch_workspace_sizes).  Errors: VMC_E_SCHEDULE. */
int vmc_batch_set_schedule(vmc_batch_t b, int samples_per_thread, int blocks);

/* Uniform grids and cleared accumulators for every integral; uploads the
 * work list and waits for that copy.  Errors: VMC_E_UNBOUND,
 * VMC_E_SCHEDULE (meta too small), VMC_E_HIP. */
int vmc_batch_reset(vmc_batch_t b, void *stream);

/* One iteration of every integral in one persistent launch: kind 1
 * forward (bin sums, estimate, running combination), 2 adjoint (gradient
 * block only), 3 both in one pass.  Kind 2 needs a forward pass (kind 1 or
 * 3) since the last vmc_batch_bind, vmc_batch_reset or vmc_refine_batched.
 * Errors: VMC_E_UNBOUND, VMC_E_INVALID, VMC_E_SCHEDULE, VMC_E_GRID (kind 2
 * without that forward pass), VMC_E_HIP. */
int vmc_iterate_batched(vmc_batch_t b, uint64_t seed, uint32_t it, int kind, uint32_t flags, void *stream);

/* Refine every axis of every integral (one block per axis), as
 * vmc_refine.  Errors: VMC_E_INVALID, VMC_E_UNBOUND, VMC_E_HIP. */
int vmc_refine_batched(vmc_batch_t b, double alpha, void *stream);

/* Set the grid of integral k from host memory (d_k axes of nbins + 1
 * edges, each from 0 to 1 and strictly increasing, in the layout of that
 * integral's part of out[0]) and rebuild its FP32 table, as vmc_set_edges
 * does for one grid (Sec. 2: the grid the next iteration samples).  Copies
 * synchronously; advances the grid-state version.  Errors: VMC_E_UNBOUND,
 * VMC_E_INVALID (k out of range, NULL), VMC_E_GRID (edges not a grid),
 * VMC_E_HIP. */
int vmc_batch_set_edges(vmc_batch_t b, int k, const double *host_edges, void *stream);

/* Clear every integral's running combination (BASES integration phase). */
int vmc_batch_combine_reset(vmc_batch_t b, void *stream);

/* As vmc_timing, for the batched launches of this handle. */
int vmc_batch_timing(vmc_batch_t b, int enable, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- SPRING */
/* Unweighted event generation from the BASES integration phase (Sec. 3.1;
 * Kawabata's SPRING).  A trial picks cube c with probability proportional
 * to its envelope g_c >= the cube's recorded maximum weight, a point
 * uniform in the cube's y-range mapped through the (frozen) grid, and keeps
 * the point when u g_c < w = f J.  Kept points are distributed as f(x) dx
 * where w <= g_c; trials with w > g_c are kept and counted as overflows.
 * The envelope is integer: g_c = q_c h gmax/2^20 with q_c = ceil(wmax_c /
 * gmax 2^20) and a headroom h >= 1 over the recorded maxima (which, being
 * maxima of a finite sample, underestimate a cube's largest weight), so the
 * cube choice is exact integer arithmetic.  Trial t of
 * pass p draws Philox words with counter (t mod 2^32, group | 2 << 8, p,
 * t div 2^32): words 0..dim-1 place the point, words dim and dim+1 form
 * the 64-bit cube choice r64 (low, high), word dim+2 the acceptance
 * uniform.  The grid must be stratified (ng >= 2, ng^dim <= 2^28).
 *
 * State buffer (8-byte slots): 0 one quantum h gmax / 2^20 (double),
 * 1 gmax (double),
 * 2 T = sum q_c, 3 envelope integral T quantum / ng^dim (double; the
 * keep rate is about I / this), 4 log2 of the guide size, 5 ng^dim,
 * 8 trials run, 9 trials kept, 10 overflows, 11 next event slot. */
#define VMC_SP_UNIT 0
#define VMC_SP_GMAX 1
#define VMC_SP_TOTAL 2
#define VMC_SP_ENV 3
#define VMC_SP_TRIALS 8
#define VMC_SP_KEPT 9
#define VMC_SP_OVER 10
#define VMC_SP_SLOT 11

/* Bytes of the SPRING buffers of a stratified grid: out[0] running sums
 * uint64[ng^dim + 1], out[1] guide table uint32[K+1] (K the smallest power
 * of two >= ng^dim), out[2] state.  Errors: VMC_E_STRAT. */
int spring_workspace_sizes(vmc_grid_t g, size_t out[3]);

/* Build the envelope from cube_max (ng^dim doubles, e.g. filled through
 * bases_cube_max) with headroom h (g_c = h x the cube's quantised maximum;
 * 1 keeps the recorded maxima, more trades keep rate for fewer overflows):
 * zeroes the state's counters.  Synchronous on `stream`.
 * Errors: VMC_E_STRAT, VMC_E_INVALID (also h < 1 or not finite),
 * VMC_E_SPRING (a +Inf maximum, or no positive one), VMC_E_HIP. */
int spring_setup(vmc_grid_t g, const double *cube_max, double headroom, uint64_t *prefix, uint32_t *guide,
                 uint64_t *state, void *stream);

/* Zero the trial, keep, overflow and slot counters (stream-ordered). */
int spring_clear_counts(uint64_t *state, void *stream);

/* Run trials trial0 .. trial0+ntrials-1 of pass `pass` with the buffers of
 * the last spring_setup on this handle (same stratification).  Kept points
 * are appended at the state's slot counter: events[slot][dim] (float, or
 * double with VMC_FLAG_FP64) and event_trial[slot] (may be NULL) for slots
 * below max_events; the order of slots within a call is not specified,
 * event_trial identifies each event.  Stream-ordered.  Errors: as
 * vmc_iterate, VMC_E_SPRING (buffers not set up), VMC_E_INVALID. */
int spring_generate(vmc_grid_t g, int integrand, const double *theta, int ntheta, const uint64_t *prefix,
                    const uint32_t *guide, uint64_t *state, uint64_t seed, uint32_t pass, int64_t trial0,
                    int64_t ntrials, int64_t max_events, void *events, uint64_t *event_trial, uint32_t flags,
                    void *stream);

#ifdef __cplusplus
}
#endif
#endif
