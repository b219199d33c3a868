/*
 * btx_oracle.h -- plain FP64 CPU reference of one time step of the locally
 * implicit Lax-Wendroff discrete-ordinate Boltzmann transport scheme of
 * Chan & Mueller, "A Novel Multi-Dimensional Boltzmann Neutrino Transport
 * Scheme for Core-Collapse Supernovae" (arXiv:2003.02845).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check
 * and the CPU-baseline leg of the benchmark may load or call this code.  The
 * GPU library never links, loads or calls it, and it shares no code with the
 * GPU library.
 *
 * State layout: f[zone][species][energy][direction], zone = b*n_r + a
 * (theta index b, radius index a), direction d = j*n_phi + k (mu index j,
 * Phi index k).  Units: c = 1, lengths km, time km/c, energy MeV.
 */
#ifndef BTX_ORACLE_H
#define BTX_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GEOM_COLUMN = 0, ORC_GEOM_AXISYM2D = 1, ORC_GEOM_PLANAR = 2 };
enum { ORC_PHI_SIN = 0, ORC_PHI_LINEAR = 1 };
enum { ORC_BC_REFLECT = 0, ORC_BC_OUTFLOW = 1, ORC_BC_EQUIL = 2 };
/* theta range of the 2D grid: [0, pi] with the polar axis at both ends, or
 * [0, pi/2] with the equatorial plane a boundary: an optically thick disk
 * (equilibrium ghost) inside disk_radius, vacuum (outflow ghost) outside */
enum { ORC_THETA_AXIS = 0, ORC_THETA_DISK = 1 };

typedef struct {
  int n_r, n_theta, n_eps, n_mu, n_phi, n_species;
  int geometry, phi_rule, inner_bc, outer_bc;
  const double *r_edges;     /* n_r+1 ascending (z edges in planar geometry)   */
  const double *theta_edges; /* n_theta+1 in 2D, spanning [0, pi]; unused else  */
  double dphi;               /* 2D wedge width in phi; column: its theta and phi
                                width (0: (r_N - r_{N-1}) / r_N); unused else    */
  const double *eps_edges;   /* n_eps+1 ascending                              */
  const double *mu_nodes;    /* n_mu ascending quadrature nodes                */
  const double *mu_weights;  /* n_mu weights, summing to 2                     */
  int theta_bc;              /* ORC_THETA_* (2D only)                          */
  double disk_radius;        /* ORC_THETA_DISK: radius of the disk             */
  int n_phi_zones;           /* 2D geometry: phi zones of width dphi, periodic
                                (<= 1: the axisymmetric wedge; > 1: 3D)        */
} orc_desc;

typedef struct orc_ctx orc_ctx;

orc_ctx *orc_create(const orc_desc *d);
void orc_destroy(orc_ctx *c);
/* v_phi may be NULL (no azimuthal motion) */
int orc_set_background(orc_ctx *c, const double *v_r, const double *v_theta,
                       const double *v_phi, const double *alpha, const double *psi,
                       const double *kappa_a, const double *kappa_s,
                       const double *f_eq);
/* new background: remaps the state from the old to the new comoving frames
 * (forward in time, no rotation), then adopts it; 5 if no background/state */
int orc_update_background(orc_ctx *c, const double *v_r, const double *v_theta,
                          const double *v_phi, const double *alpha, const double *psi,
                          const double *ka, const double *ks, const double *feq);
/* hydro source terms of the last full step (Eq. hydrosource1-3):
 * q[zone][5] = Q_Ye, Q_E, Q_M,r, Q_M,theta, Q_M,phi */
int orc_source_terms(const orc_ctx *c, double *q);
/* local time stepping: time levels from the zones' Courant lengths (at most
 * max_level, neighbours at most one apart), and the levels to step with
 * (NULL: the global step).  With levels, one orc_step step is 2^L substeps of
 * dt, L the highest level. */
int orc_time_levels(const orc_ctx *c, int max_level, int *levels);
int orc_set_levels(orc_ctx *c, const int *levels);
int orc_set_state(orc_ctx *c, const double *f);
int orc_get_state(const orc_ctx *c, double *f);
double orc_max_dt(const orc_ctx *c, double cfl);
int orc_step(orc_ctx *c, double dt, int n_steps);
/* f^{n+1} of the listed zones only, from the current state; the state is not
 * modified.  fout holds n_list blocks of n_species*n_eps*n_dir values. */
int orc_step_sample(orc_ctx *c, double dt, int n_list, const int *zones, double *fout);
/* zone_moments[zone][species][5] = N, J, H, K, number flux;
 * totals[species][3] = total number, cumulative boundary outflow, total energy */
int orc_moments(const orc_ctx *c, double *zone_moments, double *totals);
/* -1: smooth switching; 0: pure Lax-Wendroff; 1: pure upwind (tests) */
void orc_set_blend_mode(orc_ctx *c, int mode);
int orc_n_faces(const orc_ctx *c);
/* geometry: vol[nz], r/theta centres[nz] */
int orc_geometry(const orc_ctx *c, double *vol, double *r_c, double *theta_c);
/* one face from the current state: interface LW value and LW flux (interface
 * frame), and the content changes of the L and R sides (dN: 2 blocks), each
 * block n_species*n_eps*n_dir; info[8] = axis, area, h, dL, dR, active,
 * L kind, R kind */
int orc_face_debug(orc_ctx *c, int fid, double dt, double *f_lw, double *flux_lw,
                   double *dN, double *info);

/* geometry of face fid: zones[2] on its L and R sides (-1: ghost or
 * inactive), info[3] = axis, area, active (1) */
int orc_face_geom(const orc_ctx *c, int fid, int *zones, double *info);

/* building blocks, exposed for the pins.  A frame is packed as
 * {v_r, v_theta, v_phi, alpha, psi, theta, phi}. */
void orc_chain(const double *S, const double *D, int axis, int rotate,
               const double *u_in, double *u_out);
/* remap of one species block X[n_eps][n_dir] from frame S to frame D; density=1
 * remaps an occupation (point density), 0 remaps number content; general=1
 * disables the exact identity short-cut for identical frames */
int orc_remap_block(const orc_ctx *c, const double *S, const double *D, int axis,
                    int rotate, int density, int general, const double *X, double *Y);
void orc_collide(int n_dir, const double *f, const double *dJ, double tau,
                 double ka, double ks, double feq, const double *dOmega, double *out);

#ifdef __cplusplus
}
#endif
#endif
