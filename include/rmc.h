/*
 * rmc.h -- C ABI of librmc: Monte Carlo resonant-line radiative transfer on
 * an adaptive octree, on AMD MI355X (gfx950).
 *
 * Method: Michel-Dansac et al. 2020, "RASCAS: RAdiation SCattering in
 * Astrophysical Simulations" (A&A 635, A154).  The library runs the
 * per-photon-packet propagation loop of the paper on one GPU: leaf location
 * and ray-cell traversal (Sect. 4.3), optical depth to the next event
 * (Sect. 3), line opacity with the Voigt profile (Sect. 3.1.1, 3.3.2) and
 * dust opacity (Sect. 3.1.2), the choice of interaction (Sect. 3.2),
 * resonant scattering with the parallel-velocity sampler, core/wing or
 * isotropic phase functions and recoil (Sect. 3.2.1, 3.3.1, 3.3.3), dust
 * absorption or Henyey-Greenstein scattering (Sect. 3.2.2) and peel-off of
 * each emission and scattering toward observers (Sect. 5.1).
 *
 * Conventions (all calls):
 *  - Every call returns an rmc_status; nothing throws across the ABI.  On
 *    failure rmc_last_error() gives a message owned by the context, valid
 *    until the next call on it.
 *  - The caller owns every buffer it passes.  Setters copy what they are
 *    given (host -> device) and keep no pointer.  Buffers flagged
 *    RMC_DEVICE are device pointers on the context's device; work on them
 *    is ordered on the context's stream (rmc_set_stream), and calls return
 *    once that work is complete.
 *  - Positions are in box units: the octree spans [0,1)^3 and the box has
 *    physical side box_cm.  Densities cm^-3, temperatures K, velocities
 *    cm/s, dust opacity cm^-1.
 *  - Packet frequencies are x_ext: external-frame offset from the rest
 *    frequency of the first line, in Doppler widths of that line at the
 *    reference temperature T_ref given to rmc_set_lines.
 *  - A context is thread-compatible, not thread-safe.
 */
#ifndef RMC_H
#define RMC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmc_ctx rmc_ctx;

typedef enum {
  RMC_OK = 0,
  RMC_EINVAL = -1,       /* bad argument, NaN or negative physical input   */
  RMC_ENOMEM = -2,       /* device or host allocation failed               */
  RMC_EDEVICE = -3,      /* HIP runtime or kernel launch error             */
  RMC_EMESH = -4,        /* leaves overlap, leave a gap, or are not 2:1    */
  RMC_ESTATE = -5,       /* call made before the inputs it needs           */
  RMC_EUNSUPPORTED = -6  /* valid request the library does not handle      */
} rmc_status;

enum { RMC_FP64 = 0, RMC_FP32_BULK = 1 };          /* context precision        */
enum { RMC_HOST = 0, RMC_DEVICE = 1 };             /* where a buffer lives     */
enum { RMC_F32 = 0, RMC_F64 = 1 };                 /* element type of outputs  */
enum { RMC_DOM_BOX = 0, RMC_DOM_SLAB_Z = 1, RMC_DOM_SPHERE = 2 };
enum { RMC_PHASE_LYA_DIPOLE = 0, RMC_PHASE_ISOTROPIC = 1 };
enum { RMC_ST_NONE = 0, RMC_ST_ESCAPED = 1, RMC_ST_ABSORBED = 2, RMC_ST_STUCK = 3 };
enum {
  RMC_OPT_FORWARD_ONLY = 1,  /* 1: scatterings keep direction and frequency
                                (the precision test of Sect. 4.5)            */
  RMC_OPT_MAX_EVENTS = 2,    /* >0: a packet stops, status STUCK, at its
                                max_events-th interaction (0: no limit)     */
  RMC_OPT_BLOCK = 3,         /* threads per block of the transport kernel    */
  RMC_OPT_WAVES_PER_CU = 4,  /* resident waves per CU the grid is sized for  */
  RMC_OPT_REFILL = 5,        /* idle lanes a wave gathers before it takes new
                                packets (1..64)                              */
  RMC_OPT_PEEL_DEFER = 6,    /* 1 (default): a peel-off ray whose optical
                                depth does not reach the cut inside the leaf
                                of its scattering is queued (device memory
                                that grows on demand, at most 32 GiB) and
                                walked by a ray-cast pass after each
                                transport launch; 0: walked inline by the
                                transport kernel.  Results agree up to the
                                order of the cube additions.                 */
  RMC_OPT_SLICE_ITERS = 7,   /* loop iterations (events or cell crossings)
                                per lane in one transport launch            */
  RMC_OPT_REGROUP = 9,       /* 1: the transport loop runs one rejection
                                round of a line scattering's atom-velocity
                                draw per pass; a rejected round leaves the
                                event pending (the packet stays at its event
                                point) and its next round runs at the next
                                pass, in step with the other lanes' events,
                                instead of the wave looping until its last
                                lane accepts (the same draws, so the same
                                packets); 0: the looping draw.  Default 1
                                for RMC_FP64 contexts, 0 for RMC_FP32_BULK
                                (the faster of the two on each path).
                                Applies with RMC_OPT_PEEL_DEFER = 1.         */
  RMC_OPT_COMPACT = 10,      /* 1 (default): once every packet of a run has
                                started, the packets still walking are
                                gathered into the first lanes after each
                                launch that leaves at most three quarters of
                                its lanes busy, and the next launches use
                                only the waves they fill (the last, longest
                                walks then run faster per wave); 0: every
                                launch keeps the full grid.  The same packets
                                either way.                                  */
  RMC_OPT_VOIGT = 8          /* Voigt function H(a,x) of the opacity:
                                0 (default) the Tasitsiomi form the paper
                                uses (Sect. 3.3.2; within ~1% for Lya at
                                1e4 K, 2.5% at a = 0.022); 1 H to ~1e-14
                                relative, for RMC_FP64 contexts only
                                (RMC_EUNSUPPORTED on RMC_FP32_BULK; the
                                float kernels are built without it) (Sect.
                                3.1.1 definition): the
                                trapezoidal rule for the Faddeeva integral
                                with its pole term, an asymptotic series
                                for |x| >= 30.  With 1 the image gradient
                                (rmc_raycast_image_backward*) returns
                                RMC_EUNSUPPORTED: it uses dH/dx of the
                                Tasitsiomi form.                            */
};

/* One transition (Table 1 of the paper). */
typedef struct {
  double lambda0_A;   /* vacuum rest wavelength, Angstrom                   */
  double A_ul;        /* Einstein coefficient, s^-1                         */
  double f_lu;        /* oscillator strength                                */
  double mass_amu;    /* mass of the scatterer                              */
  double abundance;   /* scatterer density / n_HI                           */
  int phase;          /* RMC_PHASE_LYA_DIPOLE (core/wing) or ISOTROPIC      */
  int recoil;         /* 1: recoil term of the outgoing-frequency relation  */
  /* Fluorescent decay channels of the upper level (Sect. 3.2.1, Table 1):
   * after an absorption the atom decays through channel i with probability
   * A_i / (A_ul + sum A_i), else resonantly; a fluorescent photon leaves
   * isotropically at the channel's rest frequency in the scatterer's frame
   * (no recoil) and is not absorbed by any line again.  n_fluor in [0, 2];
   * wavelengths (Angstrom) and A (s^-1) positive and finite.  Lines with
   * channels run in the multi-line transport kernel.                       */
  int n_fluor;
  double fluor_lambda_A[2];
  double fluor_A_ul[2];
} rmc_line;

typedef struct {
  uint64_t emitted, escaped, absorbed, stuck;
  uint64_t scatterings;       /* line scatterings                            */
  uint64_t dust_scatterings;
  uint64_t crossings;         /* transport ray-cell segments run to their end */
  uint64_t peel_rays;         /* peel-off rays (one per emission or event and
                                 observer)                                    */
  uint64_t peel_crossings;    /* ray-cell segments of peel-off rays           */
  uint64_t peel_dropped;      /* peel-off deposits outside a cube (rays whose
                                 optical depth reaches the exp(-tau) = 0 cut
                                 in the leaf they start in are not binned)   */
  uint64_t peel_deferred;     /* peel-off rays handed from the transport
                                 launch to the ray-cast pass (whole launch;
                                 0 in per-problem reports)                    */
  double kernel_ms;           /* device time of the transport launch(es)      */
  double peel_pass_ms;        /* device time of the ray-cast passes over the
                                 deferred peel-off rays                       */
  uint64_t slices_cut;        /* transport launches in which some wave ended
                                 its slice early because its region of the
                                 peel-off queue was nearly full (the queue
                                 grows after such a launch; results do not
                                 change, only the work per launch)           */
} rmc_run_stats;

/* ------------------------------------------------------------- lifetime */
/* Create a context on HIP device `device`; precision RMC_FP64 (all
 * physics in double, correctly rounded operations) or RMC_FP32_BULK
 * (frequency, direction and cross-section work in float with the hardware
 * transcendental and reciprocal instructions, a few ulp each; position,
 * path length, optical depths and leaf traversal in double). */
rmc_status rmc_create(rmc_ctx **out, int device, int precision);
void rmc_destroy(rmc_ctx *ctx);
const char *rmc_last_error(const rmc_ctx *ctx);
/* Stream for all device work of this context (a hipStream_t; NULL = the
 * null stream).  The stream must outlive its use by the context. */
rmc_status rmc_set_stream(rmc_ctx *ctx, void *hip_stream);
rmc_status rmc_set_option(rmc_ctx *ctx, int option, int64_t value);
/* Core-skipping (Sect. 3.2.1, the acceleration of Ahn et al. 2002 and
 * Laursen et al. 2009 the paper uses in its galaxy example): in a resonant
 * scattering at cell-frame |x| < x_crit the atom's perpendicular velocity
 * is drawn from the Gaussian restricted to |u_perp| >= x_crit, so that a
 * packet deep in the core of a thick cell moves to the wing at once.  The
 * paper takes x_crit from Smith et al. 2015; here it comes from the cell:
 * with tau_c = n_X sigma0(T) h the line-centre optical depth across the
 * cell's edge and a its damping parameter,
 *   x_crit = min(sqrt(ln(tau_c / tau_skip)), frac (a tau_c)^(1/3)),
 * and 0 (no bias) where tau_c <= tau_skip.  tau_skip = 1, frac = 0.2 keep
 * the escape spectra of dust-free media (the tests check them against the
 * slab and sphere solutions and against unbiased runs); with dust, skipped
 * core scatterings take no path length, so extinction comes out slightly
 * low, as the paper notes.  tau_skip <= 0 turns it off (the default); a
 * non-finite tau_skip or a negative or non-finite frac gives RMC_EINVAL.
 * Takes effect at the next run or stream_begin. */
rmc_status rmc_set_core_skip(rmc_ctx *ctx, double tau_skip, double frac);
/* Source spectrum (Sect. 2.1), drawn on the device at each packet's
 * emission from its own counter-based stream and added to the x_ext the
 * source was given (rmc_set_sources):
 *   RMC_SPEC_MONO (default): no change (monochromatic; params unused);
 *   RMC_SPEC_GAUSS: Gaussian line, params[0] = standard deviation in
 *     Doppler widths of line 0 at T_ref (the paper's relative width
 *     sigma_nu is sigma x Doppler width / nu_0), Box-Muller draw;
 *   RMC_SPEC_POWER_LAW: continuum F_lambda ~ lambda^beta, params = {
 *     lambda_min, lambda_max (Angstrom), beta}: the photon-number
 *     distribution lambda F_lambda is sampled by its inverse CDF (the
 *     beta = -2 branch logarithmic) and lambda becomes
 *     x_ext += (lambda_0 - lambda) / (lambda b), b = v_th(T_ref) / c of
 *     line 0 (nu = c / lambda).
 * params is a host array of 3 doubles (copied).  Errors: RMC_EINVAL for an
 * unknown kind, a null params (other than MONO), sigma < 0 or not finite,
 * lambda_min <= 0, lambda_max <= lambda_min or a non-finite value.  Takes
 * effect at the next run or stream_begin. */
enum { RMC_SPEC_MONO = 0, RMC_SPEC_GAUSS = 1, RMC_SPEC_POWER_LAW = 2, RMC_SPEC_TABLE = 3 };
rmc_status rmc_set_source_spectrum(rmc_ctx *ctx, int kind, const double *params);
/* Tabulated continuum (Sect. 2.1): n >= 2 points (host arrays, copied),
 * wavelengths lambda_A increasing (Angstrom) and F_lambda > 0.  Between
 * neighbouring points F_lambda is the power law through them; a packet
 * takes a bin with probability proportional to the integral of
 * lambda F_lambda over it (bisection on the cumulative counts), then
 * lambda inside it by that power law's inverse CDF, and x_ext as for
 * RMC_SPEC_POWER_LAW.  Selects RMC_SPEC_TABLE (rmc_set_source_spectrum with
 * another kind switches it off again).  Errors: RMC_EINVAL for n < 2, null
 * arrays, non-increasing or non-positive wavelengths, non-positive or
 * non-finite F_lambda, or a bin whose photon count overflows. */
rmc_status rmc_set_source_table(rmc_ctx *ctx, int n, const double *lambda_A, const double *f_lambda);

/* ---------------------------------------------------------------- inputs */
/* Leaves of a graded octree (Sect. 4.3): level[n] in [0,16], ijk[3n] the
 * integer coordinates of each leaf at its own level.  Host arrays.  The
 * leaves must tile the unit cube without overlap and face neighbours may
 * differ by at most one level, else RMC_EMESH.  Builds the breadth-first
 * node array on the host and uploads it. */
rmc_status rmc_set_mesh(rmc_ctx *ctx, int64_t n_leaves, const int8_t *level,
                        const int32_t *ijk, double box_cm);
/* Per-leaf gas (Sect. 4.1 cells: n_HI, T, bulk velocity; Sect. 3.1.2
 * dust, tau_dust = int kappa_d dl): arrays of n_leaves elements (v_cms is
 * [3n], x,y,z per leaf) of type dtype (RMC_F32 or RMC_F64), in host memory
 * (mem = RMC_HOST) or device memory of the context's device (RMC_DEVICE:
 * read in place on the context's stream, no copy through the host).  The
 * values are checked and converted to double on the device and kept there;
 * the leaf records the kernels read are built from them (again whenever the
 * lines or the domain change).  Needs the mesh and the lines.  A
 * non-finite or negative value, T <= 0 or a velocity component of 0.1 c or
 * more gives RMC_EINVAL (the message names the first such leaf) and leaves
 * the previous gas in place; an unknown dtype or mem gives RMC_EINVAL.
 * Only a 16-byte status word returns to the host. */
rmc_status rmc_set_gas(rmc_ctx *ctx, const void *n_hi, const void *T_K, const void *v_cms,
                       const void *kappa_d, int dtype, int mem);
/* Up to 4 lines; line 0 and T_ref define the x_ext unit. */
rmc_status rmc_set_lines(rmc_ctx *ctx, int n_lines, const rmc_line *lines, double T_ref);
/* Dust albedo (probability of scattering at a dust interaction) and HG
 * asymmetry g (Sect. 3.2.2; defaults 0.32 and 0.73). */
rmc_status rmc_set_dust(rmc_ctx *ctx, double albedo, double g_hg);
/* Computational domain (Sect. 4): BOX = the unit cube; SLAB_Z: params
 * (zc, half_z), periodic in x and y; SPHERE: (cx, cy, cz, R) inside the
 * unit cube.  A shell is a SPHERE domain whose gas is zero inside the inner
 * radius: the inner radius bounds no packet (sources sit inside it), it is
 * a density edge in the mesh. */
rmc_status rmc_set_domain(rmc_ctx *ctx, int kind, const double params[4]);
/* Packet initial conditions (the paper's PPIC lists, Sect. 2): pos[3n],
 * dir[3n] unit vectors or NULL for isotropic emission, x_ext[n], doubles in
 * host (RMC_HOST) or device (RMC_DEVICE) memory.  Packet i is identified by
 * its index i, which keys its random numbers.  A position outside the unit
 * cube, a non-finite x or a direction with |k|^2 more than 1e-6 from 1 is
 * rejected with RMC_EINVAL (device arrays are checked by a kernel). */
rmc_status rmc_set_sources(rmc_ctx *ctx, int64_t n, const double *pos, const double *dir,
                           const double *x_ext, int mem);
/* Peel-off observer (Sect. 5.1): direction k_obs (unit), image nx by ny
 * over fov = (u0,u1,v0,v1) in box units relative to the box centre along
 * e1 = normalize(z x k) (x if k is along z) and e2 = k x e1, and nbins
 * spectral bins over [x_min, x_max).  The cube is [ny][nx][nbins], per
 * steradian per emitted packet, accumulated over runs until reset. */
rmc_status rmc_add_observer(rmc_ctx *ctx, const double k_obs[3], int nx, int ny, int nbins,
                            const double fov[4], double x_min, double x_max, int *id);
rmc_status rmc_reset_cubes(rmc_ctx *ctx);

/* ------------------------------------------------------------- transport */
/* Propagate packets [first, first+n) of the sources until each escapes,
 * is absorbed or stops at the event limit.  `seed` keys the counter-based
 * generator, so any split of a packet range gives the same packets. */
rmc_status rmc_run(rmc_ctx *ctx, uint64_t seed, int64_t first, int64_t n,
                   rmc_run_stats *stats);
/* Streaming form of rmc_run.  begin queues packets [first, first+n) and
 * parks nothing; each step is one bounded launch (RMC_OPT_SLICE_ITERS loop
 * iterations per lane) in which every lane advances the packet it holds,
 * parks it in device memory if it is still alive, and idle lanes take new
 * packets from the queue.  step reports the work of that launch (emitted =
 * packets finished in it = escaped + absorbed + stuck in it; peel_dropped
 * counts the dropped deposits of those packets, except in FP32 contexts
 * with deferred peel-off, where the launch's ray-cast pass bins the rays
 * and peel_dropped counts those it found outside the cube) and the packets
 * not finished yet; end runs the
 * remaining launches and reports the totals of the range.  rmc_run is
 * begin + steps + end.  Results do not depend on how a run is sliced.
 * begin on a context whose stream is still open abandons that stream (its
 * packets keep no results; cubes keep what it deposited). */
rmc_status rmc_stream_begin(rmc_ctx *ctx, uint64_t seed, int64_t first, int64_t n);
rmc_status rmc_stream_step(rmc_ctx *ctx, rmc_run_stats *slice, int64_t *remaining);
rmc_status rmc_stream_end(rmc_ctx *ctx, rmc_run_stats *total);
/* Per-packet results of the last run (any pointer may be NULL): status,
 * escaped x_ext, final direction k[3n], final position pos[3n], line
 * scattering count, path length in box units.  While a stream is open,
 * packets not finished yet have status RMC_ST_NONE (their other fields are
 * undefined). */
rmc_status rmc_get_packets(rmc_ctx *ctx, int32_t *status, double *x_out, double *k_out,
                           double *pos_out, int32_t *n_scat, double *path_out, int mem);
/* Histogram (counts) of x_ext of the escaped packets of the last run. */
rmc_status rmc_get_spectrum(rmc_ctx *ctx, int nbins, double x_min, double x_max, double *hist,
                            int mem);
/* rmc_get_spectrum for callers that cannot allocate device memory (code
 * that runs between graph replays, tight serving loops, harnesses that
 * forbid hipMalloc): the same counts, written as doubles to hist, a device
 * pointer to nbins doubles on the context's device, on the context's
 * stream.  The counting goes through a fixed array of 65536 64-bit counters
 * that each device holds for the life of the process, so nbins is at most
 * 65536 (RMC_EINVAL beyond); the call allocates and frees nothing.  Every
 * call on one device shares that array and clears it first: calls that
 * overlap on one GPU (other threads, or contexts on other streams) race,
 * and the caller must order them.  Returns once hist is written. */
rmc_status rmc_get_spectrum_noalloc(rmc_ctx *ctx, int nbins, double x_min, double x_max, double *hist);
/* Peel-off cube of observer `id`, [ny][nx][nbins], as RMC_F32 or RMC_F64. */
rmc_status rmc_get_cube(rmc_ctx *ctx, int id, void *out, int dtype, int mem);

/* --------------------------------------------------- deterministic probes */
/* Leaves crossed by rays from orig[3n] along dir[3n] (unit) up to the
 * domain border: leaf_out[n*max_cells], seg_out[n*max_cells] (box units),
 * n_out[n].  Traversal rule: a point on a face belongs to the leaf the ray
 * enters; the exit axes are snapped onto the face. */
rmc_status rmc_trace_cells(rmc_ctx *ctx, int64_t n, const double *orig, const double *dir,
                           int32_t max_cells, int32_t *leaf_out, double *seg_out, int32_t *n_out,
                           int mem);
/* Optical depth from orig along dir to the domain border at external
 * frequency x_ext (no events). */
rmc_status rmc_tau(rmc_ctx *ctx, int64_t n, const double *orig, const double *dir,
                   const double *x_ext, double *tau_out, int mem);

/* ---------------------------------------- peel-off image and its adjoint */
/* Image (ny*nx) of fixed rays toward observer `id`, each ray at its own
 * x_ext (no spectral binning): image[p] = sum_r w_r exp(-tau_r) over the
 * rays whose origin projects onto pixel p. */
rmc_status rmc_raycast_image(rmc_ctx *ctx, int id, int64_t n_rays, const double *orig,
                             const double *x_ext, const double *w, double *image, int mem);
/* Gradient of L = sum_p grad_image[p] image[p] with respect to per-leaf
 * n_HI, kappa_d and v_los = k_obs . v (cm/s), by replaying each ray:
 * outputs g_nhi, g_kd, g_vlos [n_leaves], overwritten, and, if g_v is not
 * NULL, the gradient with respect to the leaf velocity vector, g_v[3n] =
 * g_vlos k_obs (the chain rule through v_los; only v_los enters the image). */
rmc_status rmc_raycast_image_backward(rmc_ctx *ctx, int id, int64_t n_rays, const double *orig,
                                      const double *x_ext, const double *w,
                                      const double *grad_image, double *g_nhi, double *g_kd,
                                      double *g_vlos, double *g_v, int mem);
/* rmc_raycast_image that also keeps each ray's crossing list (leaf and
 * segment of every ray-cell crossing, in walk order; the tape) in device
 * memory of the context, for rmc_raycast_image_backward_tape.  The tape
 * takes 8 B (float path) or 12 B (double path) per crossing plus 24 B per
 * ray, grows on demand (a pass that runs out is repeated with the size it
 * needed) up to 32 GiB (RMC_ENOMEM beyond: use the replaying backward), and
 * is kept until the next call of this function or a change of the mesh,
 * lines, gas or domain.  The image equals rmc_raycast_image's up to the
 * order of the additions. */
rmc_status rmc_raycast_image_tape(rmc_ctx *ctx, int id, int64_t n_rays, const double *orig,
                                  const double *x_ext, const double *w, double *image, int mem);
/* Gradient of L = sum_p grad_image[p] image[p] (grad_image for the
 * observer of the tape) for the rays of the last rmc_raycast_image_tape
 * call, read from its tape instead of walking the rays again: the outputs
 * of rmc_raycast_image_backward for the same rays, up to the order of the
 * additions (and the float path's segments, kept as float).  RMC_ESTATE if
 * there is no tape for the current model. */
rmc_status rmc_raycast_image_backward_tape(rmc_ctx *ctx, const double *grad_image, double *g_nhi,
                                           double *g_kd, double *g_vlos, double *g_v, int mem);
/* Ray-cell crossings and device time (ms) of the last image or image
 * adjoint call of this context (RMC_ESTATE if none since the last
 * transport run). */
rmc_status rmc_image_stats(rmc_ctx *ctx, uint64_t *crossings, double *kernel_ms);

/* ---------------------------------------------------------------- batches */
/* Run many independent problems (contexts on one device with the same
 * precision) in one persistent launch: problem i propagates packets
 * [0, n_packets_i) with seed seeds[i].  per_problem[i] (may be NULL)
 * receives the per-problem counts; total the sums and the kernel time. */
rmc_status rmc_batch_run(rmc_ctx *const *problems, int n_problems, const uint64_t *seeds,
                         const int64_t *n_packets, rmc_run_stats *per_problem,
                         rmc_run_stats *total);
/* Streaming form of rmc_batch_run: opens the batch's stream on
 * problems[0]; rmc_stream_step(problems[0]) advances every problem of the
 * batch by one launch and rmc_stream_end(problems[0]) runs the rest and
 * reports the totals.  Per-packet results land in each problem's context
 * as with rmc_batch_run. */
rmc_status rmc_batch_begin(rmc_ctx *const *problems, int n_problems, const uint64_t *seeds,
                           const int64_t *n_packets);

/* Pick the transport launch shape for a batch by measurement: every
 * candidate (threads per block x idle lanes a wave gathers before refilling
 * x loop iterations per launch) runs the same stretch of this batch: 8192
 * loop iterations per lane untimed, then `trial_slices` windows of 8192
 * timed (their results are discarded; each launch timed whole,
 * synchronisation included), and the one with the most scatterings plus
 * ray-cell crossings per second is kept as the options of problems[0] for
 * later rmc_batch_run calls.  best[3] (may be NULL) receives the chosen
 * {block, refill, slice_iters}. */
rmc_status rmc_batch_autotune(rmc_ctx *const *problems, int n_problems, const uint64_t *seeds,
                              const int64_t *n_packets, int trial_slices, int best[3]);

/* ------------------------------------------------ host-only helpers */
/* Mesh check without a device: RMC_OK or RMC_EMESH/RMC_EINVAL with a
 * message in msg (may be NULL). */
rmc_status rmc_mesh_check(int64_t n_leaves, const int8_t *level, const int32_t *ijk, char *msg,
                          int msg_len);
/* Line quantities at T (Sect. 3.1.1): out = {nu0 [Hz], v_th [cm/s],
 * dnu_D [Hz], a, sigma0 [cm^2]}. */
rmc_status rmc_line_quantities(const rmc_line *line, double T_K, double out[5]);
/* Version of this interface; it changes whenever a declaration or a struct
 * layout here changes (8: rmc_set_source_table; 9: rmc_set_gas with dtype
 * and mem, velocity-vector gradients, per-slice end counts). */
int rmc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
