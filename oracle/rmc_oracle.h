/*
 * rmc_oracle.h -- plain FP64 CPU oracle for Monte Carlo resonant-line
 * transfer on an adaptive octree (Michel-Dansac et al. 2020, "RASCAS").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the GPU library; the two are written separately from the paper.
 *
 * Everything is double precision and deliberately slow: frequencies are
 * carried in Hz, every per-cell line quantity is recomputed from T at each
 * use, the leaf holding a point is found by probing a (level,i,j,k) hash map
 * coarse to fine, and every peel-off ray is integrated to the domain edge
 * (unless peel_tau_cut asks to stop where exp(-tau) has become zero).
 *
 * Units: positions in box units (the octree spans [0,1)^3, physical side
 * box_cm), densities in cm^-3, T in K, velocities in cm/s, dust opacity
 * kappa_d in cm^-1.  Packet frequencies at the interface are x_ext: the
 * external-frame offset from the first line's rest frequency in units of
 * that line's Doppler width at T_ref.
 */
#ifndef RMC_ORACLE_H
#define RMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DOM_BOX = 0, ORC_DOM_SLAB_Z = 1, ORC_DOM_SPHERE = 2 };
enum { ORC_PHASE_LYA = 0, ORC_PHASE_ISO = 1 };
enum { ORC_ST_NONE = 0, ORC_ST_ESCAPED = 1, ORC_ST_ABSORBED = 2, ORC_ST_STUCK = 3 };

typedef struct {
  double lambda0_A;  /* rest wavelength, Angstrom (Table 1)            */
  double A_ul;       /* Einstein A, s^-1                               */
  double f_lu;       /* oscillator strength                            */
  double mass_amu;   /* scatterer mass                                 */
  double abundance;  /* n_X / n_HI                                     */
  int phase;         /* ORC_PHASE_LYA (core/wing dipole) or ISO        */
  int recoil;        /* 1: recoil term of the nu_out relation on       */
  int n_fluor;       /* fluorescent decay channels (0..2)              */
  double fluor_lambda_A[2], fluor_A_ul[2];
} orc_line;

typedef struct {
  int64_t n_leaves;
  const int8_t *level;     /* [n]                                      */
  const int32_t *ijk;      /* [3n] integer coords at the leaf's level  */
  double box_cm;
  const double *n_hi;      /* [n] cm^-3                                */
  const double *T;         /* [n] K                                    */
  const double *v;         /* [3n] cm/s                                */
  const double *kappa_d;   /* [n] cm^-1                                */
  int domain_kind;
  double domain[4];        /* sphere: cx,cy,cz,R ; slab: zc,half_z     */
  int n_lines;
  orc_line lines[4];
  double T_ref;            /* defines the x_ext unit                   */
  double albedo, g_hg;
  int forward_only;        /* scatterings keep direction and frequency */
  int64_t max_events;      /* >0: the packet stops, status stuck, at its
                              max_events-th interaction (0: no limit)  */
  double core_skip_tau;    /* >0: core-skipping, x_crit from the cell:  */
  double core_skip_frac;   /* min(sqrt(ln(tau_cell/core_skip_tau)),
                              core_skip_frac (a tau_cell)^(1/3)); 0: off */
  int voigt_exact;         /* 1: H from its defining integral (quadrature)
                              instead of the Tasitsiomi form             */
  int spec_kind;           /* source spectrum: 0 monochromatic (src x),
                              1 Gaussian (spec_p[0] = sigma in Doppler
                              widths of the reference line), 2 power-law
                              continuum (spec_p = lambda_min, lambda_max
                              in Angstrom, beta of F_lambda)             */
  double spec_p[3];
  int spec_n;              /* spec_kind 3, tabulated continuum: spec_n
                              wavelengths (A, increasing) and F_lambda > 0 */
  const double *spec_lambda, *spec_flux;
  double peel_tau_cut;     /* >0: a peel-off ray stops integrating once its
                              optical depth reaches this value (0: walked
                              to the domain border).  From 746 on exp(-tau)
                              is exactly 0 in double: deposits unchanged */
} orc_problem;

typedef struct {
  double k[3];             /* unit vector toward the observer          */
  int nx, ny, nbins;
  double fov[4];           /* u0,u1,v0,v1 relative to the box centre   */
  double x_min, x_max;     /* x_ext range of the spectral axis         */
} orc_observer;

typedef struct {
  int64_t emitted, escaped, absorbed, stuck;
  int64_t scatterings, dust_scatterings, crossings, peel_rays, peel_crossings;
  int64_t peel_dropped;
} orc_stats;

/* Philox4x32-10 block (Salmon et al. 2011) */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* uniform number j of event `event` of packet `pid` (stream layout in the
 * method notes); returns a value in (0,1) */
double orc_uniform(uint64_t seed, uint64_t pid, uint32_t event, uint32_t j);

/* line quantities at temperature T: out = {nu0, v_th, dnu_D, a, sigma0} */
void orc_line_quantities(const orc_line *ln, double T, double out[5]);
double orc_voigt_h(double a, double x);
double orc_voigt_dhdx(double a, double x);
/* H(a,x) from its defining integral by adaptive quadrature (~1e-14) */
double orc_voigt_h_exact(double a, double x);

/* sampler batches for distribution tests (counter-keyed by index) */
void orc_sample_upar(int64_t n, double x, double a, uint64_t seed, double *out);
/* kind: 0 core, 1 wing, 2 Henyey-Greenstein(g), 3 isotropic */
void orc_sample_mu(int64_t n, int kind, double g, uint64_t seed, double *out);
/* core-skipping perpendicular atom velocities: n pairs (u1, u2) drawn
 * from the two-dimensional Gaussian exp(-u^2)/pi restricted to
 * |u| >= x_crit (counter-keyed by index) */
void orc_sample_uperp(int64_t n, double x_crit, uint64_t seed, double *out);
/* one scattering of a packet at x_in in a static cell at T, in the cell
 * frame; returns x_out per packet */
void orc_single_scatter(int64_t n, const orc_line *ln, double T, double x_in,
                        uint64_t seed, double *x_out);

/* mesh checks; returns 0 if valid, else a negative code:
 * -1 leaf out of range, -2 overlap/duplicate, -3 gap, -4 not 2:1 graded */
int orc_mesh_validate(int64_t n, const int8_t *level, const int32_t *ijk);
/* leaf holding point p for direction k (ties broken by the sign of k) */
int64_t orc_locate(const orc_problem *pb, const double p[3], const double k[3]);

/* deterministic probes */
int orc_trace(const orc_problem *pb, int64_t n, const double *orig, const double *dir,
              int32_t max_cells, int32_t *leaf_out, double *seg_out, int32_t *n_out);
int orc_tau(const orc_problem *pb, int64_t n, const double *orig, const double *dir,
            const double *x_ext, double *tau_out);

/* forward Monte Carlo transport of packets [first, first+n) */
int orc_run(const orc_problem *pb, int64_t n_src, const double *src_pos,
            const double *src_dir /* NULL: isotropic */, const double *src_x,
            uint64_t seed, int64_t first, int64_t n,
            int n_obs, const orc_observer *obs, double *const *cubes,
            int32_t *status, double *x_out, double *k_out, double *pos_out,
            int32_t *n_scat, double *path_out, int n_threads, orc_stats *stats);

/* peel-off image of fixed rays and its exact gradient.
 * image: [ny*nx] (each ray at its own x_ext); grad_image may be NULL, else
 * the gradients of L = sum_p grad_image[p] * image[p] with respect to
 * per-leaf n_HI, kappa_d and v_los = k_obs . v are written to g_nhi, g_kd,
 * g_vlos.  n_crossings (may be NULL) receives the ray-cell segments walked. */
int orc_raycast_image(const orc_problem *pb, const orc_observer *ob, int64_t n_rays,
                      const double *orig, const double *x_ext, const double *w,
                      double *image, const double *grad_image,
                      double *g_nhi, double *g_kd, double *g_vlos, int n_threads,
                      int64_t *n_crossings);

#ifdef __cplusplus
}
#endif
#endif
