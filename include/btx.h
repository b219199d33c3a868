/*
 * btx.h -- C ABI of libbtx: one time step of the locally implicit
 * Lax-Wendroff discrete-ordinate Boltzmann neutrino transport scheme of
 * C. Chan and B. Mueller, "A Novel Multi-Dimensional Boltzmann Neutrino
 * Transport Scheme for Core-Collapse Supernovae" (MNRAS 2020,
 * arXiv:2003.02845), on an AMD Instinct MI355X (gfx950).
 *
 * Scheme (paper Sec. 3): the phase space is a spherical-polar grid in space
 * (flat-faced cells, Sec. 3.1) times a comoving momentum grid of logarithmic
 * energy groups, mu cells with Gauss quadrature widths and uniform Phi cells.
 * One step computes, for every cell face, a Lax-Wendroff interface value with
 * an implicit interface collision (Eq. halfstep) and a donor-cell upwind flux
 * (Sec. 3.3.2), blends them with w = exp(-(ka+ks) dx) (Sec. 3.3.3), moves the
 * resulting number content between cells through the momentum-space remap of
 * Sec. 3.2 (Lorentz boost, conformally flat frame change, Hamiltonian kick,
 * geometric rotation), and ends with the zone-local closed-form solve of
 * absorption, emission and isotropic elastic scattering (Sec. 3.4-3.5).
 *
 * Conventions
 *   Units: c = 1; lengths km; time km/c; energies MeV; opacities 1/km.  The
 *   1/h^3 normalisation of moments is omitted.
 *   State layout: f[zone][species][group][direction], zone = b*n_r + a
 *   (theta index b, radius index a), direction = j*n_phi + k (mu index j,
 *   Phi index k); occupations, FP64 in BTX_PREC_FP64 mode, FP32 in
 *   BTX_PREC_MIXED mode.
 *   Ownership: the library owns all device memory it allocates.  Host arrays
 *   passed in are copied before the call returns.  A device pointer passed
 *   with is_device_ptr = 1 is borrowed for the duration of the call only.
 *   Streams: work is enqueued on the hipStream_t given at create time
 *   (NULL = default stream).  btx_step is asynchronous; btx_get_state,
 *   btx_moments and the timing query synchronise that stream.
 *   Errors: every call returns a btx_status; nothing aborts or throws across
 *   the ABI.  btx_last_error() returns a thread-local message for the last
 *   failing call on that thread.
 *   Threads: one context must not be used by two threads at once.
 *   Limits: at most 1024 directions (n_mu n_phi), 61 energy groups (29
 *   beyond 256 directions) and 2048 (species x groups) rows.  A face
 *   workgroup keeps three stencil blocks of one species in the 160 KB of LDS
 *   of a compute unit, and its remap tables too where they fit (else it reads
 *   them through the caches), which bounds directions x groups: FP64 takes up
 *   to 61 groups with 80 directions, 29 with 160, 13 with 256, 5 with 544 and
 *   1 with 768; mixed precision 61 with 160 directions, 29 with 256, 13 with
 *   544 and 5 with 1024.  btx_create reports BTX_E_UNSUPPORTED beyond.
 */
#ifndef BTX_H
#define BTX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BTX_OK = 0,
  BTX_E_INVAL = 1,        /* invalid argument, size or layout                 */
  BTX_E_NOMEM = 2,        /* device or host allocation failed                 */
  BTX_E_DEVICE = 3,       /* HIP runtime error                                */
  BTX_E_CFL = 4,          /* dt above the Courant limit (btx_max_dt, cfl = 1) */
  BTX_E_STATE = 5,        /* background or state not set                      */
  BTX_E_UNSUPPORTED = 6   /* valid input the library does not handle          */
} btx_status;

typedef enum { BTX_PREC_FP64 = 0, BTX_PREC_MIXED = 1 } btx_precision;
/* 1D spherically symmetric column (one zone per radius at the equator, theta
 * and phi periodic); 2D axisymmetric (r, theta) wedge periodic in phi; slab
 * (planar, no momentum rotation) */
typedef enum { BTX_GEOM_COLUMN = 0, BTX_GEOM_AXISYM2D = 1, BTX_GEOM_PLANAR = 2 } btx_geometry;
typedef enum { BTX_MU_GAUSS_LEGENDRE = 0, BTX_MU_GAUSS_LOBATTO = 1 } btx_mu_rule;
/* Phi split of the remap: keep the direction of the transverse momentum
 * (weights ~ sin of the angular distances; needs n_phi >= 3) or linear in Phi */
typedef enum { BTX_PHI_DIRECTION = 0, BTX_PHI_LINEAR = 1 } btx_phi_rule;
/* radial boundary ghosts: specular mirror (mu -> -mu), outflow (empty, zero
 * opacity at the face), equilibrium (the zone's own equilibrium occupation) */
typedef enum { BTX_BC_REFLECT = 0, BTX_BC_OUTFLOW = 1, BTX_BC_EQUIL = 2 } btx_bc;
/* theta range of the 2D grid (Sec. 4.5.2): [0, pi] with the polar axis at both
 * ends, or [0, pi/2] with the equatorial plane a boundary that is an
 * optically thick disk inside disk_radius (ghost: the isotropic equilibrium
 * occupation of the adjacent zone) and empty outside it (outflow ghost).  The
 * ghost sits at the mirror position pi - theta with the zone's background in
 * its own basis. */
typedef enum { BTX_THETA_AXIS = 0, BTX_THETA_DISK = 1 } btx_theta_bc;

typedef struct {
  int32_t n_r, n_theta, n_eps, n_mu, n_phi, n_species;
  int32_t geometry;          /* btx_geometry                                        */
  int32_t mu_rule;           /* btx_mu_rule                                         */
  int32_t phi_rule;          /* btx_phi_rule                                        */
  int32_t inner_bc, outer_bc;/* btx_bc (outer: OUTFLOW or EQUIL)                     */
  int32_t precision;         /* btx_precision                                       */
  const double *r_edges;     /* n_r+1 ascending, >= 0 (z edges in slab geometry)    */
  const double *theta_edges; /* 2D: n_theta+1 ascending from 0 to pi (pi/2 for a
                                disk boundary); else ignored                        */
  double dphi;               /* 2D: wedge width in phi (> 0).  Column: its theta and
                                phi width, free by Sec. 3.3.4 (0: the width at which
                                the outermost zone's lateral and radial faces have
                                equal area, (r_N - r_{N-1}) / r_N; at most pi/2).
                                Slab: ignored                                       */
  const double *eps_edges;   /* n_eps+1 ascending, logarithmically spaced (> 0)     */
  double fp64_threshold;     /* mixed mode: the collision solve of a (zone, species,
                                group) runs in FP64 where dt_c (ka + ks) exceeds it;
                                <= 0 selects the default 1.0                        */
  int32_t theta_bc;          /* 2D: btx_theta_bc; else ignored                       */
  double disk_radius;        /* BTX_THETA_DISK: the disk's radius (> 0)              */
  int32_t n_phi_zones;       /* BTX_GEOM_AXISYM2D: phi zones of width dphi, periodic
                                over n_phi_zones * dphi (<= 2 pi); 0 or 1: the
                                axisymmetric wedge, > 1: a 3D grid.  Zone index
                                (c n_theta + b) n_r + a for phi zone c          */
} btx_grid_desc;

typedef struct {             /* host arrays, copied during the call                  */
  const double *v_r;         /* [zone] radial fluid velocity (units of c, |v| < 1)   */
  const double *v_theta;     /* [zone] polar fluid velocity                          */
  const double *alpha;       /* [zone] lapse (> 0)                                   */
  const double *psi;         /* [zone] conformal factor (> 0)                        */
  const double *kappa_a;     /* [zone][species][group] absorption opacity (>= 0)     */
  const double *kappa_s;     /* [zone][species][group] scattering opacity (>= 0)     */
  const double *f_eq;        /* [zone][species][group] equilibrium occupation        */
  const double *v_phi;       /* [zone] azimuthal fluid velocity, or NULL for none    */
} btx_background;

typedef struct btx_ctx btx_ctx;

/* Validate the grid, compute geometry and quadrature (paper Sec. 3.1) in FP64
 * on the host, allocate the device state.  hip_stream: a hipStream_t or NULL. */
btx_status btx_create(const btx_grid_desc *desc, int hip_device, void *hip_stream,
                      btx_ctx **out);
/* Fluid velocity, metric (conformally flat, zero shift, Sec. 3.1) and
 * opacities (Eq. sourceterms).  Static until the next call. */
btx_status btx_set_background(btx_ctx *ctx, const btx_background *bg);
/* Evolving background (Sec. 3.2, the remap applied as time advances; the
 * closing T_{n->n+1} of a step, Sec. 3.3): the current state of every zone is
 * remapped from its comoving frame under the current background to its
 * comoving frame under bg (same place, no rotation; the covariant spatial
 * momentum is kept and the energy follows from the new metric), then bg
 * replaces the background.  Without a state or background it acts as
 * btx_set_background.  Synchronises the stream. */
btx_status btx_update_background(btx_ctx *ctx, const btx_background *bg);
/* btx_update_background with every array of bg (FP64, same layouts) in device
 * memory of the context's device (hipMalloc'd or managed; else BTX_E_INVAL):
 * nothing crosses the host link.  The values are checked on the device
 * (BTX_E_INVAL, background unchanged, if any is out of range); the copies,
 * the time remap and the table rebuild are ordered on the context's stream,
 * which the call synchronises before returning.  The arrays stay the
 * caller's. */
btx_status btx_update_background_device(btx_ctx *ctx, const btx_background *bg);
/* Largest stable global step (Sec. 3.3): cfl times the smallest Courant
 * length (zone volume over its largest face on an axis) of the grid. */
btx_status btx_max_dt(const btx_ctx *ctx, double cfl, double *dt_out);
/* State in the H-layout above, FP64 (FP64 mode) or FP32 (mixed mode);
 * resets the cumulative boundary outflow. */
btx_status btx_set_state(btx_ctx *ctx, const void *f, int is_device_ptr);
btx_status btx_get_state(btx_ctx *ctx, void *f, int is_device_ptr);
/* n_steps steps of size dt (Eq. fullstep + Sec. 3.5); BTX_E_CFL if dt exceeds
 * btx_max_dt(cfl = 1). */
btx_status btx_step(btx_ctx *ctx, double dt, int32_t n_steps);
/* zone_moments[zone][species][5] = N (number), J, H, K, number flux (Sec. 4.1,
 * 4.2); totals[species][3] = total number, cumulative boundary outflow, total
 * energy.  Either pointer may be NULL.  Zone moments are computed on the
 * device as compensated FP64 sums over the bins, the totals on the host as
 * compensated sums over the zones and boundary faces. */
btx_status btx_moments(btx_ctx *ctx, double *zone_moments, double *totals);
/* For callers that cannot allocate device or host memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): btx_moments with DEVICE outputs on the context's device,
 * enqueued on the context's stream without synchronising.  zone_moments
 * [zone][species][5] and totals [species][3] are as for btx_moments (either
 * may be NULL) and must stay valid until the stream reaches the call's work.
 * The per-zone partial results live in a library array of 24 MiB per GPU
 * (allocated with the library's code on each GPU it runs on, kept until the
 * process ends), so the grid may have at most 524288 (zone, species) pairs
 * (BTX_E_UNSUPPORTED beyond).  Calls on one GPU share that array: calls that
 * overlap in time on one GPU (different streams, or threads) race.  The zone
 * moments equal btx_moments's; the totals are compensated sums in another
 * fixed order. */
btx_status btx_moments_device(btx_ctx *ctx, double *zone_moments, double *totals);
/* Hydro source terms of the last step (coupling to matter, Sec. 3.4,
 * Eq. hydrosource1-3): q[zone][5] = Q_Ye, Q_E, Q_M,r, Q_M,theta, Q_M,phi, what
 * the fluid gains per unit comoving volume and comoving time.  They integrate
 * the collision term of Eq. sourceterms_discrete at the new state (backward
 * Euler puts the step's whole collision change there) over each bin's
 * momentum cell G_i dOmega_d (group i, direction d): weight +1 for
 * species 0 (electron neutrinos), -1 for species 1 (antineutrinos), 0
 * otherwise (Q_Ye); eps (Q_E); eps n in the zone's comoving (r, theta,
 * phi) directions (Q_M).  No 1/h^3.  Zero before the first step.  Computed
 * in FP64 by the zone update; synchronises the stream. */
btx_status btx_source_terms(btx_ctx *ctx, double *q);
/* Local time stepping (the saving Sec. 5 proposes over the global step set
 * by the smallest zones; the paper gives no scheme, this is the library's).
 * btx_time_levels proposes a level per zone: zone z may take 2^l global
 * steps at once when 2^l times the smallest Courant length is within its own
 * (l <= max_level <= 16), and zones sharing a face are at most one level
 * apart.  btx_set_time_levels adopts levels[zone] (0..16; NULL returns to the
 * global step).  With levels, one btx_step step of size dt is 2^L substeps of
 * dt (L the highest level): at substep k every face whose finer zone starts a
 * step (k mod 2^m = 0) is evaluated with dt 2^m, and every zone whose step
 * ends (k + 1 mod 2^l = 0) is updated with the content changes it gathered
 * since its last update and dt 2^l; so every zone advances 2^L dt per step
 * and the number crossing a face leaves one zone and enters the other.
 * btx_step rejects dt when a zone's 2^l dt exceeds its own Courant length.
 * Source terms are those of each zone's last update.  btx_timing records
 * global steps only.  Synchronises the stream. */
btx_status btx_time_levels(const btx_ctx *ctx, int32_t max_level, int32_t *levels);
btx_status btx_set_time_levels(btx_ctx *ctx, const int32_t *levels);
/* Per-kernel GPU time: enable = 1 records HIP events around the kernels of
 * each btx_step step on the context's stream (no synchronisation; up to 256
 * steps between two queries).  The query synchronises the recorded events and
 * returns in ms[k] / launches[k] (k = 0 face kernel, 1 zone-update kernel) the
 * accumulated time and count since the last reset (reset = 1 clears them). */
btx_status btx_timing(btx_ctx *ctx, int enable, double *ms, int64_t *launches, int reset);
btx_status btx_destroy(btx_ctx *ctx);
const char *btx_last_error(void);

/* ---- Batches: many independent models (grids of uneven sizes, one shared
 * precision) stepped together.  Each step is one face-kernel launch per face
 * shape class plus one zone-update launch over every zone of every model,
 * replayed from a HIP graph captured at the first step (the same kernels and
 * arithmetic as btx_step; per-model results equal those of btx_step up to the
 * summation order of the angle sums when the face shapes differ).  The face
 * shape of each model class (precision, directions, groups) is chosen by a
 * built-in autotuner at the first step, timed on the batch's own faces;
 * choices persist as a JSON object in tune_cache_path (NULL: no cache).
 * Models are indexed 0 .. n_models-1 in the order of descs.  Streams,
 * ownership and errors as for the single-model calls above. */
typedef struct btx_batch btx_batch;
btx_status btx_batch_create(const btx_grid_desc *descs, int32_t n_models, int hip_device, void *hip_stream,
                            const char *tune_cache_path, btx_batch **out);
btx_status btx_batch_set_background(btx_batch *b, int32_t model, const btx_background *bg);
btx_status btx_batch_update_background(btx_batch *b, int32_t model, const btx_background *bg);
btx_status btx_batch_update_background_device(btx_batch *b, int32_t model, const btx_background *bg);
btx_status btx_batch_max_dt(const btx_batch *b, int32_t model, double cfl, double *dt_out);
btx_status btx_batch_set_state(btx_batch *b, int32_t model, const void *f, int is_device_ptr);
btx_status btx_batch_get_state(btx_batch *b, int32_t model, void *f, int is_device_ptr);
/* n_steps steps; dt_per_model[n_models] (each within its model's Courant
 * limit).  The first call tunes and captures (synchronising the stream). */
btx_status btx_batch_step(btx_batch *b, const double *dt_per_model, int32_t n_steps);
/* enable = 0: launch the kernels of each step directly instead of replaying
 * the captured graph (same work, same results) */
btx_status btx_batch_use_graph(btx_batch *b, int enable);
/* the face shape the autotuner chose for a model: work items per direction
 * and energy groups per work item (valid after the first step) */
btx_status btx_batch_shape(const btx_batch *b, int32_t model, int32_t *items_per_direction,
                           int32_t *groups_per_item);
btx_status btx_batch_moments(btx_batch *b, int32_t model, double *zone_moments, double *totals);
btx_status btx_batch_source_terms(btx_batch *b, int32_t model, double *q);
/* Local time stepping in a batch (as btx_time_levels and btx_set_time_levels
 * for one model).  Once any model has been given levels (NULL: all zones at
 * level 0), every model updates its state in place and one btx_batch_step
 * step is 2^L substeps of each model's dt, L the highest level of any model;
 * a model whose highest level is below L thus takes several of its own
 * level-stepped steps.  The faces of every model at a substep share one
 * launch per face-shape class and the zones one launch; no graph is used.
 * Synchronises the stream. */
btx_status btx_batch_time_levels(const btx_batch *b, int32_t model, int32_t max_level, int32_t *levels);
btx_status btx_batch_set_time_levels(btx_batch *b, int32_t model, const int32_t *levels);
btx_status btx_batch_destroy(btx_batch *b);

#ifdef __cplusplus
}
#endif
#endif
