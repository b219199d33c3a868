/*
 * btx_oracle.c -- plain FP64 CPU reference of one time step of the locally
 * implicit Lax-Wendroff discrete-ordinate Boltzmann transport scheme of
 * Chan & Mueller (arXiv:2003.02845).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the package smoke check
 * and the CPU-baseline leg of the benchmark; never by the GPU library, with
 * which it shares no code.  Written for clarity, not speed: every remap is the
 * literal scatter of each source bin into the eight bracketing destination
 * bins (the column view of the remap operator, Sec. 3.2), the chain of frame
 * transformations is evaluated once per source direction, and the step is
 * assembled face by face in the order of Sec. 3.3.
 *
 * Readings of the paper that this file fixes (where the text is silent,
 * garbled or inconsistent) are marked "Reading:".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "btx_oracle.h"

#define PI 3.14159265358979323846
#define FOUR_PI (4.0 * PI)

enum { SIDE_ZONE = 0, SIDE_MIRROR = 1, SIDE_ZERO = 2, SIDE_EQ = 3 };

typedef struct {
  double v[3];      /* fluid 3-velocity, local orthonormal (r, theta, phi) components */
  double alpha, psi;/* lapse and conformal factor                                     */
  double th, ph;    /* angles of the local basis                                      */
} frame_t;

typedef struct {
  int kind;         /* SIDE_* : where the data comes from                            */
  int z;            /* underlying zone                                               */
  int has_slope;    /* real zone (or a periodic copy of one): reconstructed          */
  frame_t fr;
} side_t;

typedef struct {
  int axis;         /* 0: r (z in planar geometry), 1: theta, 2: phi                 */
  int active;
  side_t L, R;      /* normal points from L to R                                    */
  frame_t s;        /* interface frame                                              */
  int zero_opacity; /* interface opacities forced to zero (outflow boundary)        */
  double area, h, dL, dR;
} face_t;

struct orc_ctx {
  int nr, nth, nph, ne, nmu, nphi, ns, geom, phi_rule, inner_bc, outer_bc, theta_bc;
  double disk_r;
  int ndir, nz, blk, eblk;
  int nfr, nft, nfp, nf;
  double *r_e, *th_e, dphi, delta, *e_e;
  double *eps, *G, *mu, *wmu, *Phi, *dOm, *nvec;
  double *rc, *thc, *vol;
  double *vr, *vth, *vph, *alp, *psi, *ka, *ks, *feq;
  int have_bg, have_state;
  double *f, *fn, *outflow;
  double *q;        /* hydro source terms of the last full step, [zone][5] */
  int *lev;         /* time level of every zone (local time stepping), or NULL */
  int lmax;
  int blend_mode;
};

/* ------------------------------------------------------------------ helpers */

static double sq(double x) { return x * x; }
static int zone_faces(const orc_ctx *c, int z, int *fids, int *sgn);

static void vertex(double r, double th, double ph, double out[3])
{
  out[0] = r * sin(th) * cos(ph);
  out[1] = r * sin(th) * sin(ph);
  out[2] = r * cos(th);
}

/* Area of the flat quadrilateral V1 V2 V3 V4 (Sec. 3.1): half the norm of the
 * cross product of its diagonals.  nrm receives the unnormalised normal. */
static double quad_area(const double V1[3], const double V2[3], const double V3[3],
                        const double V4[3], double nrm[3])
{
  double a[3], b[3];
  for (int i = 0; i < 3; ++i) { a[i] = V3[i] - V1[i]; b[i] = V4[i] - V2[i]; }
  nrm[0] = a[1] * b[2] - a[2] * b[1];
  nrm[1] = a[2] * b[0] - a[0] * b[2];
  nrm[2] = a[0] * b[1] - a[1] * b[0];
  return 0.5 * sqrt(sq(nrm[0]) + sq(nrm[1]) + sq(nrm[2]));
}

/* local orthonormal basis at angles (th, ph); columns e_r, e_theta, e_phi */
static void basis(double th, double ph, double R[3][3])
{
  double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
  R[0][0] = st * cp; R[1][0] = st * sp; R[2][0] = ct;
  R[0][1] = ct * cp; R[1][1] = ct * sp; R[2][1] = -st;
  R[0][2] = -sp;     R[1][2] = cp;      R[2][2] = 0.0;
}

/* components in the D basis of a vector given in the S basis: R_D^T R_S x.
 * Reading: the geometric rotation G of Sec. 3.2.1 is taken as this exact basis
 * change, which fixes the axis of the phi-move rotation. */
static void rotate_vec(double thS, double phS, double thD, double phD,
                       const double x[3], double y[3])
{
  if (thS == thD && phS == phD) { y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; return; }
  double RS[3][3], RD[3][3], c[3];
  basis(thS, phS, RS);
  basis(thD, phD, RD);
  for (int k = 0; k < 3; ++k) c[k] = RS[k][0] * x[0] + RS[k][1] * x[1] + RS[k][2] * x[2];
  for (int i = 0; i < 3; ++i) y[i] = RD[0][i] * c[0] + RD[1][i] * c[1] + RD[2][i] * c[2];
}

/* Lorentz boost of Sec. 3.2.2: u_out = Lambda(v) u_in. */
static void boost(const double v[3], const double u[4], double o[4])
{
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double g = 1.0 / sqrt(1.0 - v2);
  double k = g * g / (g + 1.0);           /* (gamma - 1)/v^2 without cancellation */
  double vu = v[0] * u[1] + v[1] * u[2] + v[2] * u[3];
  o[0] = g * (u[0] + vu);
  for (int i = 0; i < 3; ++i) o[i + 1] = u[i + 1] + (k * vu + g * u[0]) * v[i];
}

static double gamma_of(const double v[3])
{
  return 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
}

/* Full chain of Eq. (transformchain): comoving(S) -> Eulerian(S) -> coordinate
 * (S) -> Hamiltonian kick and geometric rotation -> coordinate(D) ->
 * Eulerian(D) -> comoving(D).  Conformally flat metric with zero shift
 * (Sec. 3.2.3).  The kick (Sec. 3.2.4) changes only the covariant component
 * along the axis of motion so that the null condition holds with the
 * destination metric; the root keeps the sign of the source component
 * (Reading: sign(0) = +); without a real root the component is set to zero and
 * the others are scaled to keep the four-velocity null.  The kick is skipped
 * when the two metrics are identical (it is then the identity).
 * axis < 0 is the remap forward in time at a fixed place (Sec. 3.2, the same
 * procedure applied as time advances).  Reading: with no motion across the
 * grid the covariant spatial momentum is kept and the covariant energy is set
 * by the null condition of the new metric. */
static void chain_frames(const frame_t *S, const frame_t *D, int axis, int rotate,
                         const double uS[4], double uD[4])
{
  double uh[4];
  boost(S->v, uS, uh);
  double low0 = -S->alpha * uh[0];              /* u_0 = -alpha^2 u^0, u^0 = uh^0/alpha */
  double low[3];
  for (int i = 0; i < 3; ++i) low[i] = S->psi * S->psi * uh[i + 1]; /* psi^4 * uh^i/psi^2 */
  if (axis < 0 && (S->alpha != D->alpha || S->psi != D->psi)) {
    double p2 = 0.0;
    for (int i = 0; i < 3; ++i) p2 += low[i] * low[i];
    low0 = -D->alpha * sqrt(p2) / (D->psi * D->psi);
  } else if (S->alpha != D->alpha || S->psi != D->psi) {
    double perp2 = 0.0;
    for (int i = 0; i < 3; ++i) if (i != axis) perp2 += low[i] * low[i];
    double p4 = sq(D->psi * D->psi);
    double rad = p4 * low0 * low0 / (D->alpha * D->alpha) - perp2;
    if (rad >= 0.0) {
      low[axis] = (low[axis] >= 0.0 ? 1.0 : -1.0) * sqrt(rad);
    } else {
      double scale = (D->psi * D->psi * fabs(low0) / D->alpha) / sqrt(perp2);
      low[axis] = 0.0;
      for (int i = 0; i < 3; ++i) if (i != axis) low[i] *= scale;
    }
  }
  double lowD[3];
  if (rotate) rotate_vec(S->th, S->ph, D->th, D->ph, low, lowD);
  else { lowD[0] = low[0]; lowD[1] = low[1]; lowD[2] = low[2]; }
  double ue[4];
  ue[0] = -low0 / D->alpha;                       /* alpha_D * u^0, u^0 = -u_0/alpha_D^2 */
  for (int i = 0; i < 3; ++i) ue[i + 1] = lowD[i] / (D->psi * D->psi);
  double mv[3] = { -D->v[0], -D->v[1], -D->v[2] };
  boost(mv, ue, uD);
}

static void unpack_frame(const double *p, frame_t *f)
{
  f->v[0] = p[0]; f->v[1] = p[1]; f->v[2] = p[2];
  f->alpha = p[3]; f->psi = p[4]; f->th = p[5]; f->ph = p[6];
}

static int frames_equal(const frame_t *a, const frame_t *b)
{
  return a->v[0] == b->v[0] && a->v[1] == b->v[1] && a->v[2] == b->v[2] &&
         a->alpha == b->alpha && a->psi == b->psi && a->th == b->th && a->ph == b->ph;
}

/* Bracketing nodes of x among ascending nodes xs[0..n-1] with linear weights
 * (Sec. 3.2, Eq. interpolation).  Reading: values outside the node range are
 * given entirely to the edge node. */
static void bracket(const double *xs, int n, double x, int *L, int *R, double *wR)
{
  if (n == 1 || x <= xs[0]) { *L = *R = 0; *wR = 0.0; return; }
  if (x >= xs[n - 1]) { *L = *R = n - 1; *wR = 0.0; return; }
  int l = 0;
  while (xs[l + 1] <= x) ++l;
  *L = l; *R = l + 1;
  *wR = (x - xs[l]) / (xs[l + 1] - xs[l]);
}

/* Periodic bracket in Phi.  Reading: the garbled cos/sin conditions of
 * Sec. 3.2 are taken as "preserve the direction of the transverse momentum":
 * w_L ~ sin(Phi_R - Phi*), w_R ~ sin(Phi* - Phi_L), normalised to one. */
static void bracket_phi(const orc_ctx *c, double P, int *L, int *R, double *wR)
{
  int n = c->nphi;
  if (n == 1) { *L = *R = 0; *wR = 0.0; return; }
  double dP = 2.0 * PI / n;
  int kl = (int)floor(P / dP - 0.5);
  double PL = (kl + 0.5) * dP, PR = PL + dP;
  if (c->phi_rule == ORC_PHI_SIN) {
    double a = sin(PR - P), b = sin(P - PL);
    *wR = b / (a + b);
  } else {
    *wR = (P - PL) / dP;
  }
  *L = ((kl % n) + n) % n;
  *R = (((kl + 1) % n) + n) % n;
}

/* ---------------------------------------------------------- remap operator */

/* Eulerian energy component of the comoving unit direction d in frame fr */
static double u0_of(const orc_ctx *c, const frame_t *fr, int d)
{
  const double *n = c->nvec + 3 * d;
  double g = gamma_of(fr->v);
  return g * (1.0 + fr->v[0] * n[0] + fr->v[1] * n[1] + fr->v[2] * n[2]);
}

/* Y = T_{S->D}[X] for one species block X[ne][ndir] (Eq. transformation).
 * Reading: T moves number content n = W f, W = psi^6 u0_d dGamma_{i,d}
 * (Sec. 3.1, number integral); density=1 converts occupations to content
 * before and back after, density=0 moves content as is.  Each source bin is
 * split over the 2x2x2 bracketing destination bins with the product of the
 * energy, mu and Phi weights. */
static void remap(const orc_ctx *c, const frame_t *S, const frame_t *D, int axis,
                  int rotate, int density, int general, const double *X, double *Y)
{
  int ne = c->ne, nd = c->ndir;
  if (!general && frames_equal(S, D)) {
    memcpy(Y, X, sizeof(double) * ne * nd);
    return;
  }
  double *acc = (double *)calloc((size_t)ne * nd, sizeof(double));
  double pS6 = pow(S->psi, 6.0), pD6 = pow(D->psi, 6.0);
  for (int d = 0; d < nd; ++d) {
    int k = d % c->nphi;
    double u[4] = { 1.0, c->nvec[3 * d], c->nvec[3 * d + 1], c->nvec[3 * d + 2] };
    double o[4];
    chain_frames(S, D, axis, rotate, u, o);
    double rho = o[0];
    double mus = o[1] / o[0];
    if (mus > 1.0) mus = 1.0;
    if (mus < -1.0) mus = -1.0;
    double Ps;
    /* Reading: Phi is undefined on the mu = +-1 axis; a direction within 1e-6
     * rad of it keeps the Phi label of its source bin */
    if (o[2] * o[2] + o[3] * o[3] <= 1e-12 * o[0] * o[0]) Ps = c->Phi[k];
    else { Ps = atan2(o[3], o[2]); if (Ps < 0.0) Ps += 2.0 * PI; }
    int jL, jR, kL, kR; double wj, wk;
    bracket(c->mu, c->nmu, mus, &jL, &jR, &wj);
    bracket_phi(c, Ps, &kL, &kR, &wk);
    double Wsd = density ? pS6 * u0_of(c, S, d) * c->dOm[d] : 1.0;
    for (int i = 0; i < ne; ++i) {
      double n = X[i * nd + d] * (density ? Wsd * c->G[i] : 1.0);
      if (n == 0.0) continue;
      int iL, iR; double wi;
      bracket(c->eps, ne, rho * c->eps[i], &iL, &iR, &wi);
      int ii[2] = { iL, iR }, jj[2] = { jL, jR }, kk[2] = { kL, kR };
      double wI[2] = { 1.0 - wi, wi }, wJ[2] = { 1.0 - wj, wj }, wK[2] = { 1.0 - wk, wk };
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int e = 0; e < 2; ++e)
            acc[ii[a] * nd + jj[b] * c->nphi + kk[e]] += n * wI[a] * wJ[b] * wK[e];
    }
  }
  for (int i = 0; i < ne; ++i)
    for (int d = 0; d < nd; ++d) {
      double W = density ? pD6 * u0_of(c, D, d) * c->G[i] * c->dOm[d] : 1.0;
      Y[i * nd + d] = acc[i * nd + d] / W;
    }
  free(acc);
}

/* ------------------------------------------------ implicit collision solve */

/* Backward-Euler solve of f' = S + tau*[ka (feq - f') + ks (<f'> - f')] with
 * S = f + tau ka feq + dJ and <x> = (1/4pi) sum_d x_d dOmega_d (Eq.
 * sourceterms_discrete).  Reading: the closed form printed in Sec. 3.5 divides
 * the scattering sum by 1 + (ka+ks) tau; the exact solution of the linear
 * system divides it by 1 + ka tau, which is what is used here. */
void orc_collide(int nd, const double *f, const double *dJ, double tau, double ka,
                 double ks, double feq, const double *dOm, double *out)
{
  double sum = 0.0;
  for (int d = 0; d < nd; ++d) {
    double S = f[d] + tau * ka * feq + (dJ ? dJ[d] : 0.0);
    out[d] = S;
    sum += S * dOm[d];
  }
  double avg = sum / FOUR_PI;
  double fav = avg / (1.0 + tau * ka);
  for (int d = 0; d < nd; ++d)
    out[d] = (out[d] + tau * ks * fav) / (1.0 + tau * (ka + ks));
}

/* ------------------------------------------------------------- grid set-up */

/* zone z = (c n_theta + b) n_r + a: radius a, theta row b, phi zone c */
static int zone_b(const orc_ctx *c, int z) { return (z / c->nr) % c->nth; }
static int zone_c(const orc_ctx *c, int z) { return z / (c->nr * c->nth); }
static int zone_at(const orc_ctx *c, int a, int b, int cz) { return (cz * c->nth + b) * c->nr + a; }
/* theta faces of one phi zone: between rows, plus the equatorial boundary */
static int theta_slab(const orc_ctx *c)
{
  return c->nr * (c->theta_bc == ORC_THETA_DISK ? c->nth : c->nth - 1);
}

static void column_angles(const orc_ctx *c, int b, double *tlo, double *thi,
                          double *plo, double *phi_)
{
  if (c->geom == ORC_GEOM_AXISYM2D) {
    *tlo = c->th_e[b]; *thi = c->th_e[b + 1];
    *plo = -0.5 * c->dphi; *phi_ = 0.5 * c->dphi;
  } else {
    *tlo = 0.5 * PI - 0.5 * c->delta; *thi = 0.5 * PI + 0.5 * c->delta;
    *plo = -0.5 * c->delta; *phi_ = 0.5 * c->delta;
  }
}

/* unit-radius r-face area of angular row b */
static double unit_rface(const orc_ctx *c, int b, double *h1)
{
  double tlo, thi, plo, phi_;
  column_angles(c, b, &tlo, &thi, &plo, &phi_);
  double V1[3], V2[3], V3[3], V4[3], n[3];
  vertex(1.0, tlo, plo, V1); vertex(1.0, thi, plo, V2);
  vertex(1.0, thi, phi_, V3); vertex(1.0, tlo, phi_, V4);
  double A = quad_area(V1, V2, V3, V4, n);
  double nn = sqrt(sq(n[0]) + sq(n[1]) + sq(n[2]));
  *h1 = fabs(n[0] * V1[0] + n[1] * V1[1] + n[2] * V1[2]) / nn;
  return A;
}

static void free_all(orc_ctx *c)
{
  free(c->r_e); free(c->th_e); free(c->e_e); free(c->eps); free(c->G); free(c->mu);
  free(c->wmu); free(c->Phi); free(c->dOm); free(c->nvec); free(c->rc); free(c->thc);
  free(c->vol); free(c->vr); free(c->vth); free(c->vph); free(c->alp); free(c->psi); free(c->ka);
  free(c->ks); free(c->feq); free(c->f); free(c->fn); free(c->outflow); free(c->q); free(c->lev);
}

orc_ctx *orc_create(const orc_desc *d)
{
  if (!d || d->n_r < 1 || d->n_eps < 1 || d->n_mu < 2 || d->n_phi < 1 || d->n_species < 1)
    return NULL;
  if (d->geometry < 0 || d->geometry > 2) return NULL;
  if (d->phi_rule == ORC_PHI_SIN && d->n_phi > 1 && d->n_phi < 3) return NULL;
  int nth = d->geometry == ORC_GEOM_AXISYM2D ? d->n_theta : 1;
  if (nth < 1) return NULL;
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->nr = d->n_r; c->nth = nth; c->ne = d->n_eps; c->nmu = d->n_mu; c->nphi = d->n_phi;
  c->ns = d->n_species; c->geom = d->geometry; c->phi_rule = d->phi_rule;
  c->inner_bc = d->inner_bc; c->outer_bc = d->outer_bc;
  c->theta_bc = c->geom == ORC_GEOM_AXISYM2D ? d->theta_bc : ORC_THETA_AXIS;
  c->disk_r = d->disk_radius;
  /* 3D: n_phi_zones phi zones of width dphi, periodic in phi (Sec. 3.1);
   * one zone is the axisymmetric wedge */
  c->nph = (c->geom == ORC_GEOM_AXISYM2D && d->n_phi_zones > 1) ? d->n_phi_zones : 1;
  c->ndir = c->nmu * c->nphi; c->nz = c->nr * c->nth * c->nph;
  c->eblk = c->ne * c->ndir; c->blk = c->ns * c->eblk;
  c->blend_mode = -1;
  c->r_e = (double *)malloc(sizeof(double) * (c->nr + 1));
  memcpy(c->r_e, d->r_edges, sizeof(double) * (c->nr + 1));
  c->th_e = (double *)malloc(sizeof(double) * (nth + 1));
  if (c->geom == ORC_GEOM_AXISYM2D) memcpy(c->th_e, d->theta_edges, sizeof(double) * (nth + 1));
  else { c->th_e[0] = 0.0; c->th_e[1] = PI; }
  c->dphi = d->dphi;
  /* Reading: the 1D column is one zone at the equator with equal theta and
   * phi widths delta.  Sec. 3.3.4 leaves the width free and recommends
   * faces of similar area; a column grid takes delta = dphi when given
   * (> 0), else the width that makes the lateral area of the outermost zone
   * match its radial area: delta = (r_N - r_{N-1}) / r_N. */
  c->delta = (c->geom == ORC_GEOM_COLUMN && d->dphi > 0.0) ? d->dphi
                                                           : (c->r_e[c->nr] - c->r_e[c->nr - 1]) / c->r_e[c->nr];
  c->e_e = (double *)malloc(sizeof(double) * (c->ne + 1));
  memcpy(c->e_e, d->eps_edges, sizeof(double) * (c->ne + 1));
  /* momentum grid (Sec. 3.1).  Reading: group centres are geometric means of
   * the edges; dGamma_i = (eps_hi^3 - eps_lo^3)/3 per unit solid angle. */
  c->eps = (double *)malloc(sizeof(double) * c->ne);
  c->G = (double *)malloc(sizeof(double) * c->ne);
  for (int i = 0; i < c->ne; ++i) {
    c->eps[i] = sqrt(c->e_e[i] * c->e_e[i + 1]);
    c->G[i] = (pow(c->e_e[i + 1], 3.0) - pow(c->e_e[i], 3.0)) / 3.0;
  }
  c->mu = (double *)malloc(sizeof(double) * c->nmu);
  c->wmu = (double *)malloc(sizeof(double) * c->nmu);
  memcpy(c->mu, d->mu_nodes, sizeof(double) * c->nmu);
  memcpy(c->wmu, d->mu_weights, sizeof(double) * c->nmu);
  c->Phi = (double *)malloc(sizeof(double) * c->nphi);
  /* Reading: Phi bins are uniform on [0, 2pi) with centres (k + 1/2) 2pi/n_Phi */
  for (int k = 0; k < c->nphi; ++k) c->Phi[k] = (k + 0.5) * 2.0 * PI / c->nphi;
  c->dOm = (double *)malloc(sizeof(double) * c->ndir);
  c->nvec = (double *)malloc(sizeof(double) * 3 * c->ndir);
  for (int j = 0; j < c->nmu; ++j)
    for (int k = 0; k < c->nphi; ++k) {
      int dd = j * c->nphi + k;
      c->dOm[dd] = c->wmu[j] * 2.0 * PI / c->nphi;
      double st = sqrt(1.0 - c->mu[j] * c->mu[j]);
      /* Reading: local components ordered (r, theta, phi) with mu along r */
      c->nvec[3 * dd] = c->mu[j];
      c->nvec[3 * dd + 1] = st * cos(c->Phi[k]);
      c->nvec[3 * dd + 2] = st * sin(c->Phi[k]);
    }
  /* zones */
  c->rc = (double *)malloc(sizeof(double) * c->nz);
  c->thc = (double *)malloc(sizeof(double) * c->nz);
  c->vol = (double *)malloc(sizeof(double) * c->nz);
  for (int cz = 0; cz < c->nph; ++cz)
  for (int b = 0; b < nth; ++b) {
    double h1 = 0.0, A1 = 0.0;
    if (c->geom != ORC_GEOM_PLANAR) A1 = unit_rface(c, b, &h1);
    for (int a = 0; a < c->nr; ++a) {
      int z = (cz * nth + b) * c->nr + a;
      double rlo = c->r_e[a], rhi = c->r_e[a + 1];
      c->rc[z] = 0.5 * (rlo + rhi);
      if (c->geom == ORC_GEOM_AXISYM2D) c->thc[z] = 0.5 * (c->th_e[b] + c->th_e[b + 1]);
      else if (c->geom == ORC_GEOM_COLUMN) c->thc[z] = 0.5 * PI;
      else c->thc[z] = 0.0;
      /* flat-faced cell: difference of two pyramids with apex at the origin */
      if (c->geom == ORC_GEOM_PLANAR) c->vol[z] = rhi - rlo;
      else c->vol[z] = (rhi * rhi * rhi - rlo * rlo * rlo) * A1 * h1 / 3.0;
    }
  }
  c->nfr = c->nph * nth * (c->nr + 1);
  if (c->geom == ORC_GEOM_AXISYM2D) c->nft = c->nph * theta_slab(c);
  else if (c->geom == ORC_GEOM_COLUMN) c->nft = c->nr;
  else c->nft = 0;
  c->nfp = c->geom == ORC_GEOM_PLANAR ? 0 : c->nz;
  c->nf = c->nfr + c->nft + c->nfp;
  c->f = (double *)calloc((size_t)c->nz * c->blk, sizeof(double));
  c->fn = (double *)calloc((size_t)c->nz * c->blk, sizeof(double));
  c->outflow = (double *)calloc(c->ns, sizeof(double));
  c->q = (double *)calloc((size_t)c->nz * 5, sizeof(double));
  return c;
}

void orc_destroy(orc_ctx *c)
{
  if (!c) return;
  free_all(c);
  free(c);
}

int orc_set_background(orc_ctx *c, const double *v_r, const double *v_theta,
                       const double *v_phi, const double *alpha, const double *psi,
                       const double *ka, const double *ks, const double *feq)
{
  if (!c) return 1;
  size_t nz = c->nz, nk = (size_t)c->nz * c->ns * c->ne;
#define CP(dst, src, n) do { free(dst); dst = (double *)malloc(sizeof(double) * (n)); \
    memcpy(dst, src, sizeof(double) * (n)); } while (0)
  CP(c->vr, v_r, nz); CP(c->vth, v_theta, nz); CP(c->alp, alpha, nz); CP(c->psi, psi, nz);
  free(c->vph);
  c->vph = (double *)calloc(nz, sizeof(double));
  if (v_phi) memcpy(c->vph, v_phi, sizeof(double) * nz);
  CP(c->ka, ka, nk); CP(c->ks, ks, nk); CP(c->feq, feq, nk);
#undef CP
  c->have_bg = 1;
  return 0;
}

int orc_set_state(orc_ctx *c, const double *f)
{
  if (!c) return 1;
  memcpy(c->f, f, sizeof(double) * (size_t)c->nz * c->blk);
  memset(c->outflow, 0, sizeof(double) * c->ns);
  c->have_state = 1;
  return 0;
}

int orc_get_state(const orc_ctx *c, double *f)
{
  if (!c) return 1;
  memcpy(f, c->f, sizeof(double) * (size_t)c->nz * c->blk);
  return 0;
}

void orc_set_blend_mode(orc_ctx *c, int mode) { if (c) c->blend_mode = mode; }
int orc_n_faces(const orc_ctx *c) { return c ? c->nf : 0; }

int orc_geometry(const orc_ctx *c, double *vol, double *r_c, double *theta_c)
{
  if (!c) return 1;
  memcpy(vol, c->vol, sizeof(double) * c->nz);
  memcpy(r_c, c->rc, sizeof(double) * c->nz);
  memcpy(theta_c, c->thc, sizeof(double) * c->nz);
  return 0;
}

static void get_face_geom(const orc_ctx *c, int fid, double *area);

/* Global time step (Sec. 3.3): the Courant number in the smallest cell.
 * Reading: the Courant length of a zone along an axis is its volume over the
 * larger of its two faces on that axis (the cell width for a box), taken over
 * every axis with non-zero faces, periodic self-faces included; the step is
 * cfl times the smallest such length on the grid. */
double orc_max_dt(const orc_ctx *c, double cfl)
{
  double m = 1e300;
  int fids[8], sg[8];
  for (int z = 0; z < c->nz; ++z) {
    double amax[3] = { 0.0, 0.0, 0.0 };
    int nfz = zone_faces(c, z, fids, sg);
    for (int q = 0; q < nfz; ++q) {
      double A;
      int ax = fids[q] < c->nfr ? 0 : (fids[q] < c->nfr + c->nft ? 1 : 2);
      get_face_geom(c, fids[q], &A);
      if (A > amax[ax]) amax[ax] = A;
    }
    for (int ax = 0; ax < 3; ++ax)
      if (amax[ax] > 0.0 && c->vol[z] / amax[ax] < m) m = c->vol[z] / amax[ax];
  }
  return cfl * m;
}

/* ------------------------------------------------------ frames and faces */

static frame_t zone_frame(const orc_ctx *c, int z, double th, double ph)
{
  frame_t f;
  int bg = c->have_bg;
  f.v[0] = bg ? c->vr[z] : 0.0; f.v[1] = bg ? c->vth[z] : 0.0; f.v[2] = bg ? c->vph[z] : 0.0;
  f.alpha = bg ? c->alp[z] : 1.0; f.psi = bg ? c->psi[z] : 1.0;
  f.th = th; f.ph = ph;
  return f;
}

static double zone_th(const orc_ctx *c, int z)
{
  return c->geom == ORC_GEOM_PLANAR ? 0.0 : c->thc[z];
}

static int rotating(const orc_ctx *c) { return c->geom != ORC_GEOM_PLANAR; }

/* Euclidean distance between the points r1 n(t1,p1) and r2 n(t2,p2) */
static double centre_dist(double r1, double t1, double p1, double r2, double t2, double p2)
{
  double A[3], B[3];
  vertex(r1, t1, p1, A); vertex(r2, t2, p2, B);
  return sqrt(sq(A[0] - B[0]) + sq(A[1] - B[1]) + sq(A[2] - B[2]));
}

/* Boundary ghost next to real zone z on the radial axis (Sec. 3.3.4).
 * Reading: the inner boundary is a specular mirror (mu -> -mu, radial fluid
 * velocity reversed); the outer boundary is outflow (f = 0, zero opacity at the
 * face); "equilibrium" ghosts (tests only) hold the zone's own equilibrium. */
static side_t ghost_side(const orc_ctx *c, int z, int bc)
{
  side_t s;
  s.z = z; s.has_slope = 0;
  s.fr = zone_frame(c, z, zone_th(c, z), 0.0);
  if (bc == ORC_BC_REFLECT) { s.kind = SIDE_MIRROR; s.fr.v[0] = -s.fr.v[0]; }
  else if (bc == ORC_BC_OUTFLOW) s.kind = SIDE_ZERO;
  else s.kind = SIDE_EQ;
  return s;
}

/* Ghost beyond the equatorial boundary of a theta-disk grid, next to zone z
 * of the last theta row (Sec. 4.5.2, radiating disk).  Reading: it sits at the
 * mirror position pi - theta_z and carries the zone's background expressed
 * in its own basis; inside the disk radius it holds the isotropic
 * equilibrium of the zone (an optically thick disk), outside it is empty
 * (nothing enters from the vacuum below the plane). */
static side_t theta_ghost_side(const orc_ctx *c, int z)
{
  side_t s;
  s.z = z; s.has_slope = 0;
  s.fr = zone_frame(c, z, PI - c->thc[z], 0.0);
  s.kind = c->rc[z] < c->disk_r ? SIDE_EQ : SIDE_ZERO;
  return s;
}

static side_t zone_side(const orc_ctx *c, int z, double th, double ph)
{
  side_t s;
  s.kind = SIDE_ZONE; s.z = z; s.has_slope = 1;
  s.fr = zone_frame(c, z, th, ph);
  return s;
}

/* interface frame: mean of the two side frames, velocities first rotated into
 * the interface basis (Reading: Sec. 3.3 leaves interface values unspecified) */
static frame_t mean_frame(const frame_t *L, const frame_t *R, double th, double ph)
{
  frame_t s;
  double vl[3], vr[3];
  rotate_vec(L->th, L->ph, th, ph, L->v, vl);
  rotate_vec(R->th, R->ph, th, ph, R->v, vr);
  for (int i = 0; i < 3; ++i) s.v[i] = 0.5 * (vl[i] + vr[i]);
  s.alpha = 0.5 * (L->alpha + R->alpha);
  s.psi = 0.5 * (L->psi + R->psi);
  s.th = th; s.ph = ph;
  return s;
}

static void get_face(const orc_ctx *c, int fid, face_t *F)
{
  memset(F, 0, sizeof(*F));
  F->active = 1;
  if (fid < c->nfr) {                            /* radial (planar: z) faces */
    int col = fid / (c->nr + 1), b = col % c->nth, a = fid % (c->nr + 1) - 1; /* between a and a+1 */
    double R = c->r_e[a + 1];
    F->axis = 0;
    double th = c->geom == ORC_GEOM_PLANAR ? 0.0 : (c->geom == ORC_GEOM_AXISYM2D ?
                0.5 * (c->th_e[b] + c->th_e[b + 1]) : 0.5 * PI);
    if (c->geom == ORC_GEOM_PLANAR) F->area = 1.0;
    else { double h1; F->area = R * R * unit_rface(c, b, &h1); }
    if (c->geom != ORC_GEOM_PLANAR && R == 0.0) { F->active = 0; return; }
    int zL = col * c->nr + a, zR = col * c->nr + a + 1;
    if (a >= 0) F->L = zone_side(c, zL, th, 0.0);
    else F->L = ghost_side(c, zR, c->inner_bc);
    if (a + 1 < c->nr) F->R = zone_side(c, zR, th, 0.0);
    else F->R = ghost_side(c, zL, c->outer_bc);
    if (a >= 0 && a + 1 < c->nr) F->h = c->rc[zR] - c->rc[zL];
    else if (a < 0) F->h = 2.0 * (c->rc[zR] - R);
    else F->h = 2.0 * (R - c->rc[zL]);
    F->dL = a >= 0 ? R - c->rc[zL] : 0.5 * F->h;
    F->dR = a + 1 < c->nr ? -(c->rc[zR] - R) : -0.5 * F->h;
    F->s = mean_frame(&F->L.fr, &F->R.fr, th, 0.0);
    F->zero_opacity = (F->L.kind == SIDE_ZERO || F->R.kind == SIDE_ZERO);
    return;
  }
  fid -= c->nfr;
  if (fid < c->nft) {                            /* theta faces */
    F->axis = 1;
    if (c->geom == ORC_GEOM_AXISYM2D) {
      int cz = fid / theta_slab(c), b = fid % theta_slab(c) / c->nr, a = fid % c->nr;
      int zL = zone_at(c, a, b, cz), zR = zL + c->nr;
      double tf = c->th_e[b + 1], rlo = c->r_e[a], rhi = c->r_e[a + 1];
      double p0 = -0.5 * c->dphi, p1 = 0.5 * c->dphi, V1[3], V2[3], V3[3], V4[3], n[3];
      vertex(rlo, tf, p0, V1); vertex(rhi, tf, p0, V2); vertex(rhi, tf, p1, V3); vertex(rlo, tf, p1, V4);
      F->area = quad_area(V1, V2, V3, V4, n);
      F->L = zone_side(c, zL, c->thc[zL], 0.0);
      if (b + 1 < c->nth) {
        F->R = zone_side(c, zR, c->thc[zR], 0.0);
        F->h = centre_dist(c->rc[zL], c->thc[zL], 0.0, c->rc[zR], c->thc[zR], 0.0);
      } else {                                   /* equatorial boundary of a disk grid */
        F->R = theta_ghost_side(c, zL);
        F->h = centre_dist(c->rc[zL], c->thc[zL], 0.0, c->rc[zL], PI - c->thc[zL], 0.0);
        F->zero_opacity = F->R.kind == SIDE_ZERO;
      }
      F->s = mean_frame(&F->L.fr, &F->R.fr, tf, 0.0);
    } else {                                     /* column: periodic self-face */
      int a = fid, z = a;
      double t0 = 0.5 * PI, tf = t0 + 0.5 * c->delta, t1 = t0 + c->delta;
      double rlo = c->r_e[a], rhi = c->r_e[a + 1];
      double p0 = -0.5 * c->delta, p1 = 0.5 * c->delta, V1[3], V2[3], V3[3], V4[3], n[3];
      vertex(rlo, tf, p0, V1); vertex(rhi, tf, p0, V2); vertex(rhi, tf, p1, V3); vertex(rlo, tf, p1, V4);
      F->area = quad_area(V1, V2, V3, V4, n);
      F->L = zone_side(c, z, t0, 0.0);
      F->R = zone_side(c, z, t1, 0.0);
      F->h = centre_dist(c->rc[z], t0, 0.0, c->rc[z], t1, 0.0);
      F->s = mean_frame(&F->L.fr, &F->R.fr, tf, 0.0);
    }
    F->dL = 0.5 * F->h; F->dR = -0.5 * F->h;
    return;
  }
  fid -= c->nft;                  /* phi faces: to the next phi zone, periodic (itself in 2D) */
  {
    int z = fid, a = z % c->nr, b = zone_b(c, z);
    int zR = c->geom == ORC_GEOM_AXISYM2D ? zone_at(c, a, b, (zone_c(c, z) + 1) % c->nph) : z;
    double tlo, thi, plo, phi_;
    column_angles(c, b, &tlo, &thi, &plo, &phi_);
    double w = phi_ - plo;
    double pf = 0.5 * w, th = c->thc[z];
    double rlo = c->r_e[a], rhi = c->r_e[a + 1], V1[3], V2[3], V3[3], V4[3], n[3];
    vertex(rlo, tlo, pf, V1); vertex(rhi, tlo, pf, V2); vertex(rhi, thi, pf, V3); vertex(rlo, thi, pf, V4);
    F->axis = 2;
    F->area = quad_area(V1, V2, V3, V4, n);
    F->L = zone_side(c, z, th, 0.0);
    F->R = zone_side(c, zR, th, w);
    F->h = centre_dist(c->rc[z], th, 0.0, c->rc[z], th, w);
    F->dL = 0.5 * F->h; F->dR = -0.5 * F->h;
    F->s = mean_frame(&F->L.fr, &F->R.fr, th, pf);
  }
}

static void get_face_geom(const orc_ctx *c, int fid, double *area)
{
  face_t F;
  get_face(c, fid, &F);
  *area = F.active ? F.area : 0.0;
}

/* faces touching zone z, with the side the zone is on (+1: R, -1: L) */
static int zone_faces(const orc_ctx *c, int z, int *fids, int *sgn)
{
  int a = z % c->nr, b = zone_b(c, z), cz = zone_c(c, z), n = 0;
  int base = (z / c->nr) * (c->nr + 1);
  fids[n] = base + a;     sgn[n++] = +1;         /* face a-1/2: zone is R */
  fids[n] = base + a + 1; sgn[n++] = -1;         /* face a+1/2: zone is L */
  if (c->geom == ORC_GEOM_AXISYM2D) {
    int tb = c->nfr + cz * theta_slab(c);
    if (b > 0) { fids[n] = tb + (b - 1) * c->nr + a; sgn[n++] = +1; }
    if (b < c->nth - 1 || c->theta_bc == ORC_THETA_DISK) { fids[n] = tb + b * c->nr + a; sgn[n++] = -1; }
  } else if (c->geom == ORC_GEOM_COLUMN) {
    fids[n] = c->nfr + a; sgn[n++] = -1;
    fids[n] = c->nfr + a; sgn[n++] = +1;
  }
  if (c->geom != ORC_GEOM_PLANAR) {
    int zprev = c->geom == ORC_GEOM_AXISYM2D ? zone_at(c, a, b, (cz + c->nph - 1) % c->nph) : z;
    fids[n] = c->nfr + c->nft + z; sgn[n++] = -1;
    fids[n] = c->nfr + c->nft + zprev; sgn[n++] = +1;
  }
  return n;
}

/* the species-s data of a side, in the side's own frame */
static void side_data(const orc_ctx *c, const side_t *sd, const double *f, int s, double *X)
{
  int ne = c->ne, nd = c->ndir;
  const double *src = f + (size_t)sd->z * c->blk + (size_t)s * c->eblk;
  if (sd->kind == SIDE_ZONE) { memcpy(X, src, sizeof(double) * ne * nd); return; }
  for (int i = 0; i < ne; ++i)
    for (int j = 0; j < c->nmu; ++j)
      for (int k = 0; k < c->nphi; ++k) {
        int d = j * c->nphi + k;
        double v = 0.0;
        if (sd->kind == SIDE_MIRROR) v = src[i * nd + (c->nmu - 1 - j) * c->nphi + k];
        else if (sd->kind == SIDE_EQ) v = c->feq[((size_t)sd->z * c->ns + s) * ne + i];
        X[i * nd + d] = v;
      }
}

/* neighbours of zone z along an axis, for the limited slope */
static void axis_neighbours(const orc_ctx *c, int z, int axis, side_t *m, side_t *p,
                            double *hm, double *hp)
{
  int a = z % c->nr, b = zone_b(c, z);
  double th = zone_th(c, z);
  if (axis == 0) {
    if (a > 0) { *m = zone_side(c, z - 1, th, 0.0); *hm = c->rc[z] - c->rc[z - 1]; }
    else { *m = ghost_side(c, z, c->inner_bc); *hm = 2.0 * (c->rc[z] - c->r_e[0]); }
    if (a < c->nr - 1) { *p = zone_side(c, z + 1, th, 0.0); *hp = c->rc[z + 1] - c->rc[z]; }
    else { *p = ghost_side(c, z, c->outer_bc); *hp = 2.0 * (c->r_e[c->nr] - c->rc[z]); }
  } else if (axis == 1) {
    if (c->geom == ORC_GEOM_AXISYM2D) {
      /* Reading: beyond the axis the ghost is the zone itself (zero gradient) */
      int zm = b > 0 ? z - c->nr : z, zp = b < c->nth - 1 ? z + c->nr : z;
      *m = zone_side(c, zm, c->thc[zm], 0.0);
      *p = zone_side(c, zp, c->thc[zp], 0.0);
      *hm = zm == z ? 1.0 : centre_dist(c->rc[zm], c->thc[zm], 0.0, c->rc[z], c->thc[z], 0.0);
      *hp = zp == z ? 1.0 : centre_dist(c->rc[zp], c->thc[zp], 0.0, c->rc[z], c->thc[z], 0.0);
      if (zp == z && c->theta_bc == ORC_THETA_DISK) {   /* the equatorial ghost */
        *p = theta_ghost_side(c, z);
        *hp = centre_dist(c->rc[z], c->thc[z], 0.0, c->rc[z], PI - c->thc[z], 0.0);
      }
    } else {
      *m = zone_side(c, z, th - c->delta, 0.0);
      *p = zone_side(c, z, th + c->delta, 0.0);
      *hm = *hp = centre_dist(c->rc[z], th, 0.0, c->rc[z], th + c->delta, 0.0);
    }
  } else {
    double w = c->geom == ORC_GEOM_AXISYM2D ? c->dphi : c->delta;
    int zm = z, zp = z;
    if (c->geom == ORC_GEOM_AXISYM2D) {
      zm = zone_at(c, a, b, (zone_c(c, z) + c->nph - 1) % c->nph);
      zp = zone_at(c, a, b, (zone_c(c, z) + 1) % c->nph);
    }
    *m = zone_side(c, zm, th, -w);
    *p = zone_side(c, zp, th, w);
    *hm = *hp = centre_dist(c->rc[z], th, 0.0, c->rc[z], th, w);
  }
}

/* MC limiter (Sec. 3.3.2).  Reading: minmod(2 D-, 2 D+, (D- + D+)/2), zero
 * unless all three arguments have the same strict sign. */
static double mc_limit(double dm, double dp)
{
  double a = 2.0 * dm, b = 2.0 * dp, m = 0.5 * (dm + dp);
  if (a > 0.0 && b > 0.0 && m > 0.0) return fmin(a, fmin(b, m));
  if (a < 0.0 && b < 0.0 && m < 0.0) return fmax(a, fmax(b, m));
  return 0.0;
}

/* limited slope of zone z along axis (per unit length), all species.
 * Reading: neighbours are first remapped into the zone's frame (the
 * reconstruction "along characteristics"), differences are divided by the
 * centre distances. */
static void zone_slope(const orc_ctx *c, const double *f, int z, int axis, double *sig)
{
  side_t m, p;
  double hm, hp;
  axis_neighbours(c, z, axis, &m, &p, &hm, &hp);
  frame_t self = zone_frame(c, z, zone_th(c, z), 0.0);
  int n = c->eblk, rot = rotating(c);
  double *Xm = (double *)malloc(sizeof(double) * n), *Xp = (double *)malloc(sizeof(double) * n);
  double *Ym = (double *)malloc(sizeof(double) * n), *Yp = (double *)malloc(sizeof(double) * n);
  for (int s = 0; s < c->ns; ++s) {
    side_data(c, &m, f, s, Xm);
    side_data(c, &p, f, s, Xp);
    remap(c, &m.fr, &self, axis, rot, 1, 0, Xm, Ym);
    remap(c, &p.fr, &self, axis, rot, 1, 0, Xp, Yp);
    const double *fz = f + (size_t)z * c->blk + (size_t)s * n;
    for (int q = 0; q < n; ++q)
      sig[(size_t)s * n + q] = mc_limit((fz[q] - Ym[q]) / hm, (Yp[q] - fz[q]) / hp);
  }
  free(Xm); free(Xp); free(Ym); free(Yp);
}

/* interface opacity / equilibrium (Reading: arithmetic means of the two
 * zones; zero at an outflow face) */
static void face_opacity(const orc_ctx *c, const face_t *F, int s, int i,
                         double *ka, double *ks, double *feq)
{
  if (F->zero_opacity) { *ka = *ks = *feq = 0.0; return; }
  size_t l = ((size_t)F->L.z * c->ns + s) * c->ne + i, r = ((size_t)F->R.z * c->ns + s) * c->ne + i;
  *ka = 0.5 * (c->ka[l] + c->ka[r]);
  *ks = 0.5 * (c->ks[l] + c->ks[r]);
  *feq = 0.5 * (c->feq[l] + c->feq[r]);
}

/* Eulerian direction of comoving bin d of frame X, expressed in the basis of
 * frame s, and the corresponding number speed through a face of axis ax:
 * alpha_s psi_s^4 uhat^n (flux integral of Sec. 3.1 with zero shift). */
static double donor_speed(const orc_ctx *c, const frame_t *X, const frame_t *s, int ax,
                          int rot, int d)
{
  double u[4] = { 1.0, c->nvec[3 * d], c->nvec[3 * d + 1], c->nvec[3 * d + 2] }, uh[4], y[3];
  boost(X->v, u, uh);
  if (rot) rotate_vec(X->th, X->ph, s->th, s->ph, uh + 1, y);
  else { y[0] = uh[1]; y[1] = uh[2]; y[2] = uh[3]; }
  return s->alpha * sq(s->psi * s->psi) * y[ax];
}

/* Contribution of face F to the number content of its two sides, all
 * species (Eq. fullstep).  dNL / dNR are in the bins of the L / R side frames.
 *
 * Lax-Wendroff part (Eq. halfstep): both neighbours are remapped into the
 * interface frame, advanced half a step with the implicit interface collision,
 * and the resulting flux U_rad f_LW is taken out of L and put into R through
 * the interface-to-cell remaps.
 * Upwind part (Sec. 3.3.2 and the upwind flow of Fig. 3).  Reading: each side
 * is a donor cell: every bin of a side whose velocity, taken at the cell centre
 * and expressed in the interface basis, points through the face, carries
 * U f~ of its linearly reconstructed value out of that bin, and the carried
 * number is deposited into the other side through the full source-to-
 * destination chain.
 * Blend (Sec. 3.3.3): the radiative flux is (1-w) LW + w upwind with
 * w = exp(-(ka+ks) dx); the fluid-advection part alpha psi^4 gamma v^n of the
 * speed is always upwinded (Sec. 3.2.2), i.e. its (1-w) share is carried by the
 * donor cell picked by the sign of the interface fluid velocity.
 * Optional outputs: the LW interface value and the blended interface flux
 * (interface frame, LW part only) for the diffusion-limit pin. */
static void face_contrib(const orc_ctx *c, const face_t *F, const double *f, const double *sigL,
                         const double *sigR, double dt, double *dNL, double *dNR,
                         double *flw_out, double *flux_out)
{
  int ne = c->ne, nd = c->ndir, n = c->eblk, rot = rotating(c), ax = F->axis;
  double *X = (double *)malloc(sizeof(double) * n), *A = (double *)malloc(sizeof(double) * n);
  double *B = (double *)malloc(sizeof(double) * n), *FL = (double *)malloc(sizeof(double) * n);
  double *EL = (double *)malloc(sizeof(double) * n), *ER = (double *)malloc(sizeof(double) * n);
  double *Y = (double *)malloc(sizeof(double) * n), *Sv = (double *)malloc(sizeof(double) * nd);
  double *flw = (double *)malloc(sizeof(double) * nd);
  double *Ur = (double *)malloc(sizeof(double) * nd), *Vn = (double *)malloc(sizeof(double) * nd);
  double *UL = (double *)malloc(sizeof(double) * nd), *UR = (double *)malloc(sizeof(double) * nd);
  const frame_t *s = &F->s;
  double g = gamma_of(s->v), kk = g * g / (g + 1.0);
  double ap4 = s->alpha * sq(s->psi * s->psi);
  double vn = s->v[ax];
  double Uadv = ap4 * g * vn;
  for (int d = 0; d < nd; ++d) {
    const double *nv = c->nvec + 3 * d;
    double vdn = s->v[0] * nv[0] + s->v[1] * nv[1] + s->v[2] * nv[2];
    double u0 = g * (1.0 + vdn);
    double un = nv[ax] + (kk * vdn + g) * vn;
    Ur[d] = ap4 * (nv[ax] + kk * vdn * vn);
    /* Reading: the half step uses the coordinate speed u^n/u^0 */
    Vn[d] = s->alpha * un / (s->psi * s->psi * u0);
    UL[d] = donor_speed(c, &F->L.fr, s, ax, rot, d);
    UR[d] = donor_speed(c, &F->R.fr, s, ax, rot, d);
  }
  double tau = 0.5 * s->alpha * dt / g;          /* half of dt_c = alpha dt/gamma */
  double cA = dt * F->area;
  for (int sp = 0; sp < c->ns; ++sp) {
    double *dl = dNL + (size_t)sp * n, *dr = dNR + (size_t)sp * n;
    side_data(c, &F->L, f, sp, X);
    remap(c, &F->L.fr, s, ax, rot, 1, 0, X, A);
    for (int q = 0; q < n; ++q) {                /* reconstructed donor values */
      double t = X[q] + (F->L.has_slope ? F->dL * sigL[(size_t)sp * n + q] : 0.0);
      EL[q] = t;
    }
    side_data(c, &F->R, f, sp, X);
    remap(c, &F->R.fr, s, ax, rot, 1, 0, X, B);
    for (int q = 0; q < n; ++q) {
      double t = X[q] + (F->R.has_slope ? F->dR * sigR[(size_t)sp * n + q] : 0.0);
      ER[q] = t;
    }
    for (int i = 0; i < ne; ++i) {
      double ka, ks, feq;
      face_opacity(c, F, sp, i, &ka, &ks, &feq);
      for (int d = 0; d < nd; ++d) {
        int q = i * nd + d;
        double fbar = 0.5 * (A[q] + B[q]);
        double dJ = -0.5 * dt * Vn[d] * (B[q] - A[q]) / F->h;
        Sv[d] = fbar + dJ;
      }
      orc_collide(nd, Sv, NULL, tau, ka, ks, feq, c->dOm, flw);
      double w = exp(-(ka + ks) * F->h);
      if (c->blend_mode == 0) w = 0.0;
      if (c->blend_mode == 1) w = 1.0;
      for (int d = 0; d < nd; ++d) {
        int q = i * nd + d;
        double dG = c->G[i] * c->dOm[d];
        FL[q] = cA * (1.0 - w) * Ur[d] * flw[d] * dG;
        double eL = w * (UL[d] > 0.0 ? UL[d] : 0.0) + (1.0 - w) * (Uadv > 0.0 ? Uadv : 0.0);
        double eR = w * (UR[d] < 0.0 ? -UR[d] : 0.0) + (1.0 - w) * (Uadv < 0.0 ? -Uadv : 0.0);
        EL[q] = cA * eL * EL[q] * dG;
        ER[q] = cA * eR * ER[q] * dG;
        if (flw_out) flw_out[(size_t)sp * n + q] = flw[d];
        if (flux_out) flux_out[(size_t)sp * n + q] = FL[q];
      }
    }
    /* L: - T_{s->L} F_LW - E_L + T_{R->L} E_R ; R: + T_{s->R} F_LW - E_R + T_{L->R} E_L */
    remap(c, s, &F->L.fr, ax, rot, 0, 0, FL, Y);
    for (int q = 0; q < n; ++q) dl[q] = -Y[q] - EL[q];
    remap(c, s, &F->R.fr, ax, rot, 0, 0, FL, Y);
    for (int q = 0; q < n; ++q) dr[q] = Y[q] - ER[q];
    remap(c, &F->R.fr, &F->L.fr, ax, rot, 0, 0, ER, Y);
    for (int q = 0; q < n; ++q) dl[q] += Y[q];
    remap(c, &F->L.fr, &F->R.fr, ax, rot, 0, 0, EL, Y);
    for (int q = 0; q < n; ++q) dr[q] += Y[q];
  }
  free(X); free(A); free(B); free(FL); free(EL); free(ER); free(Y); free(Sv); free(flw);
  free(Ur); free(Vn); free(UL); free(UR);
}

/* ------------------------------------------------------------------ step */

typedef struct {
  int *slot_face, *slot_slope;   /* -1: not needed */
  int *face_list, nfl, *slope_list, nsl;
  double *fbuf, *sbuf;           /* per face: dN_L then dN_R */
} work_t;

static void mark_slope(const orc_ctx *c, work_t *w, int axis, int z)
{
  int key = axis * c->nz + z;
  if (w->slot_slope[key] < 0) { w->slot_slope[key] = w->nsl; w->slope_list[w->nsl++] = key; }
}

static const double *slope_ptr(const orc_ctx *c, const work_t *w, int axis, int z)
{
  int slot = w->slot_slope[axis * c->nz + z];
  return slot < 0 ? NULL : w->sbuf + (size_t)slot * c->blk;
}

/* Conservative update and zone-local implicit collision of zone z (Eq.
 * fullstep, Sec. 3.5) over a step dt: the zone's summed face content changes
 * dN are divided by its bin content weights W = psi^6 dV u0 dGamma and the
 * collisions are solved; writes f^{n+1} of the zone to out and its hydro
 * source terms to qz[5]. */
static void zone_update(const orc_ctx *c, int z, const double *dN, double dt, double *out, double qz[5])
{
  int n = c->eblk, ne = c->ne, nd = c->ndir;
  double *dJ = (double *)malloc(sizeof(double) * nd), *tmp = (double *)malloc(sizeof(double) * nd);
  frame_t self = zone_frame(c, z, zone_th(c, z), 0.0);
  double g = gamma_of(self.v), p6 = pow(self.psi, 6.0);
  double tau = self.alpha * dt / g;             /* Reading: dt_c = alpha dt / gamma */
  for (int k = 0; k < 5; ++k) qz[k] = 0.0;
  for (int s = 0; s < c->ns; ++s)
    for (int i = 0; i < ne; ++i) {
      const double *fz0 = c->f + (size_t)z * c->blk + (size_t)s * n + (size_t)i * nd;
      for (int d = 0; d < nd; ++d) {
        double W = p6 * c->vol[z] * u0_of(c, &self, d) * c->G[i] * c->dOm[d];
        dJ[d] = dN[(size_t)s * n + i * nd + d] / W;
      }
      size_t kidx = ((size_t)z * c->ns + s) * ne + i;
      orc_collide(nd, fz0, dJ, tau, c->ka[kidx], c->ks[kidx], c->feq[kidx], c->dOm, tmp);
      memcpy(out + (size_t)s * n + (size_t)i * nd, tmp, sizeof(double) * nd);
      /* hydro source terms (Eq. hydrosource1-3): the collision term of
       * Eq. sourceterms_discrete at the new distribution f' (backward Euler
       * puts the whole collision change of the step there), integrated over
       * each bin's momentum-space cell G_i dOmega_d with weight 1 (lepton
       * number: + for the first species, - for the second), eps_i (energy)
       * and eps_i n_d (momentum, r, theta and phi components); the fluid gains
       * what the radiation loses.  Readings: d^3p = eps^2 deps dOmega, so
       * the bin integrals are G_i dOmega_d; the 1/h^3 normalisation is
       * omitted; comoving frame, per unit comoving volume and time. */
      double ka = c->ka[kidx], ks = c->ks[kidx], fe = c->feq[kidx], avg = 0.0;
      for (int d = 0; d < nd; ++d) avg += tmp[d] * c->dOm[d];
      avg /= 4.0 * PI;
      double lep = s == 0 ? 1.0 : (s == 1 ? -1.0 : 0.0);
      for (int d = 0; d < nd; ++d) {
        double C = ka * (fe - tmp[d]) + ks * avg - ks * tmp[d];
        double wgt = C * c->G[i] * c->dOm[d];
        qz[0] -= lep * wgt;
        qz[1] -= wgt * c->eps[i];
        qz[2] -= wgt * c->eps[i] * c->nvec[3 * d];
        qz[3] -= wgt * c->eps[i] * c->nvec[3 * d + 1];
        qz[4] -= wgt * c->eps[i] * c->nvec[3 * d + 2];
      }
    }
  free(dJ); free(tmp);
}

/* one step for the listed zones; writes f^{n+1} blocks to fout (list order) */
static int do_step(orc_ctx *c, double dt, int nlist, const int *zones, double *fout,
                   double *out_tally)
{
  work_t w;
  memset(&w, 0, sizeof(w));
  w.slot_face = (int *)malloc(sizeof(int) * c->nf);
  w.slot_slope = (int *)malloc(sizeof(int) * 3 * c->nz);
  w.face_list = (int *)malloc(sizeof(int) * c->nf);
  w.slope_list = (int *)malloc(sizeof(int) * 3 * c->nz);
  for (int q = 0; q < c->nf; ++q) w.slot_face[q] = -1;
  for (int q = 0; q < 3 * c->nz; ++q) w.slot_slope[q] = -1;
  int fids[8], sg[8];
  for (int l = 0; l < nlist; ++l) {
    int nfz = zone_faces(c, zones[l], fids, sg);
    for (int q = 0; q < nfz; ++q)
      if (w.slot_face[fids[q]] < 0) { w.slot_face[fids[q]] = w.nfl; w.face_list[w.nfl++] = fids[q]; }
  }
  for (int q = 0; q < w.nfl; ++q) {
    face_t F;
    get_face(c, w.face_list[q], &F);
    if (!F.active) continue;
    if (F.L.has_slope) mark_slope(c, &w, F.axis, F.L.z);
    if (F.R.has_slope) mark_slope(c, &w, F.axis, F.R.z);
  }
  w.fbuf = (double *)malloc(sizeof(double) * 2 * ((size_t)w.nfl + 1) * c->blk);
  w.sbuf = (double *)malloc(sizeof(double) * ((size_t)w.nsl + 1) * c->blk);
  if (!w.fbuf || !w.sbuf) return 2;
  const double *f = c->f;
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < w.nsl; ++q) {
    int key = w.slope_list[q];
    zone_slope(c, f, key % c->nz, key / c->nz, w.sbuf + (size_t)q * c->blk);
  }
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < w.nfl; ++q) {
    face_t F;
    get_face(c, w.face_list[q], &F);
    double *dl = w.fbuf + 2 * (size_t)q * c->blk, *dr = dl + c->blk;
    if (!F.active) { memset(dl, 0, sizeof(double) * 2 * c->blk); continue; }
    face_contrib(c, &F, f, slope_ptr(c, &w, F.axis, F.L.z), slope_ptr(c, &w, F.axis, F.R.z),
                 dt, dl, dr, NULL, NULL);
  }
  /* conservative update and zone-local implicit collision (Eq. fullstep,
   * Sec. 3.5): the zone sums the content changes of its faces, divides by
   * its bin content weights W = psi^6 dV u0 dGamma and solves the collisions. */
#pragma omp parallel for schedule(dynamic)
  for (int l = 0; l < nlist; ++l) {
    int z = zones[l];
    int fz[8], sz[8];
    int nfz = zone_faces(c, z, fz, sz);
    double *dN = (double *)calloc((size_t)c->blk, sizeof(double));
    for (int q = 0; q < nfz; ++q) {
      const double *src = w.fbuf + 2 * (size_t)w.slot_face[fz[q]] * c->blk + (sz[q] > 0 ? c->blk : 0);
      for (int p = 0; p < c->blk; ++p) dN[p] += src[p];
    }
    double qz[5];
    zone_update(c, z, dN, dt, fout + (size_t)l * c->blk, qz);
    if (out_tally) memcpy(c->q + 5 * (size_t)z, qz, sizeof(qz));
    free(dN);
  }
  /* number leaving the domain: what the boundary ghosts would receive */
  if (out_tally) {
    for (int q = 0; q < w.nfl; ++q) {
      face_t F;
      get_face(c, w.face_list[q], &F);
      if (!F.active) continue;
      for (int side = 0; side < 2; ++side) {
        const side_t *sd = side ? &F.R : &F.L;
        if (sd->kind == SIDE_ZONE) continue;
        const double *src = w.fbuf + 2 * (size_t)q * c->blk + (side ? c->blk : 0);
        for (int s = 0; s < c->ns; ++s) {
          double t = 0.0;
          for (int p = 0; p < c->eblk; ++p) t += src[(size_t)s * c->eblk + p];
          out_tally[s] += t;
        }
      }
    }
  }
  free(w.slot_face); free(w.slot_slope); free(w.face_list); free(w.slope_list);
  free(w.fbuf); free(w.sbuf);
  return 0;
}

static int lts_step(orc_ctx *c, double dt0);

int orc_step(orc_ctx *c, double dt, int n_steps)
{
  if (!c || !c->have_bg || !c->have_state) return 5;
  if (c->lev) {
    for (int t = 0; t < n_steps; ++t) {
      int rc = lts_step(c, dt);
      if (rc) return rc;
    }
    return 0;
  }
  int *all = (int *)malloc(sizeof(int) * c->nz);
  for (int z = 0; z < c->nz; ++z) all[z] = z;
  for (int t = 0; t < n_steps; ++t) {
    int rc = do_step(c, dt, c->nz, all, c->fn, c->outflow);
    if (rc) { free(all); return rc; }
    double *tmp = c->f; c->f = c->fn; c->fn = tmp;
  }
  free(all);
  return 0;
}

int orc_step_sample(orc_ctx *c, double dt, int n_list, const int *zones, double *fout)
{
  if (!c || !c->have_bg || !c->have_state) return 5;
  for (int l = 0; l < n_list; ++l) if (zones[l] < 0 || zones[l] >= c->nz) return 1;
  return do_step(c, dt, n_list, zones, fout, NULL);
}

int orc_face_debug(orc_ctx *c, int fid, double dt, double *f_lw, double *flux_lw,
                   double *dN, double *info)
{
  if (!c || fid < 0 || fid >= c->nf || !c->have_bg || !c->have_state) return 1;
  face_t F;
  get_face(c, fid, &F);
  info[0] = F.axis; info[1] = F.area; info[2] = F.h; info[3] = F.dL; info[4] = F.dR;
  info[5] = F.active; info[6] = F.L.kind; info[7] = F.R.kind;
  if (!F.active) return 0;
  double *sL = (double *)calloc(c->blk, sizeof(double)), *sR = (double *)calloc(c->blk, sizeof(double));
  if (F.L.has_slope) zone_slope(c, c->f, F.L.z, F.axis, sL);
  if (F.R.has_slope) zone_slope(c, c->f, F.R.z, F.axis, sR);
  face_contrib(c, &F, c->f, sL, sR, dt, dN, dN + c->blk, f_lw, flux_lw);
  free(sL); free(sR);
  return 0;
}


/* Geometry of one face, for the pins: zones[2] = the zones on its L and R
 * sides (-1 for a ghost side), info[3] = axis, area, active. */
int orc_face_geom(const orc_ctx *c, int fid, int *zones, double *info)
{
  if (!c || fid < 0 || fid >= c->nf) return 1;
  face_t F;
  get_face(c, fid, &F);
  zones[0] = F.active && F.L.kind == SIDE_ZONE ? F.L.z : -1;
  zones[1] = F.active && F.R.kind == SIDE_ZONE ? F.R.z : -1;
  info[0] = F.axis;
  info[1] = F.active ? F.area : 0.0;
  info[2] = F.active;
  return 0;
}

/* ------------------------------------------------------------- moments */

/* Moments of Sec. 4.1/4.2 per zone and species (the 1/h^3 normalisation is
 * omitted): N = psi^6 dV sum f u0 dGamma, J, H, K = (1/4pi) sum f eps mu^{0,1,2}
 * dGamma, number flux = (1/4pi) sum f mu dGamma (Reading: the quantity the
 * text calls the number density is defined with mu, i.e. a number flux). */
int orc_moments(const orc_ctx *c, double *zm, double *tot)
{
  if (!c || !c->have_bg) return 5;
  for (int s = 0; s < c->ns; ++s) { tot[3 * s] = 0.0; tot[3 * s + 1] = c->outflow[s]; tot[3 * s + 2] = 0.0; }
  for (int z = 0; z < c->nz; ++z) {
    frame_t self = zone_frame(c, z, zone_th(c, z), 0.0);
    double p6v = pow(self.psi, 6.0) * c->vol[z];
    for (int s = 0; s < c->ns; ++s) {
      double N = 0, J = 0, H = 0, K = 0, Hn = 0, E = 0;
      for (int i = 0; i < c->ne; ++i)
        for (int d = 0; d < c->ndir; ++d) {
          double fv = c->f[(size_t)z * c->blk + (size_t)s * c->eblk + i * c->ndir + d];
          double dG = c->G[i] * c->dOm[d], mu = c->mu[d / c->nphi];
          double nn = p6v * u0_of(c, &self, d) * dG * fv;
          N += nn;
          E += nn * c->eps[i];
          J += fv * c->eps[i] * dG;
          H += fv * mu * c->eps[i] * dG;
          K += fv * mu * mu * c->eps[i] * dG;
          Hn += fv * mu * dG;
        }
      double *m = zm + ((size_t)z * c->ns + s) * 5;
      m[0] = N; m[1] = J / FOUR_PI; m[2] = H / FOUR_PI; m[3] = K / FOUR_PI; m[4] = Hn / FOUR_PI;
      tot[3 * s] += N;
      tot[3 * s + 2] += E;
    }
  }
  return 0;
}

/* ------------------------------------------------------- pin entry points */

void orc_chain(const double *S, const double *D, int axis, int rotate, const double *u_in,
               double *u_out)
{
  frame_t a, b;
  unpack_frame(S, &a);
  unpack_frame(D, &b);
  chain_frames(&a, &b, axis, rotate, u_in, u_out);
}

int orc_remap_block(const orc_ctx *c, const double *S, const double *D, int axis,
                    int rotate, int density, int general, const double *X, double *Y)
{
  if (!c) return 1;
  frame_t a, b;
  unpack_frame(S, &a);
  unpack_frame(D, &b);
  remap(c, &a, &b, axis, rotate, density, general, X, Y);
  return 0;
}

/* Time-dependent background (Sec. 3.2, the remap applied as particles travel
 * forward in time; the closing T_{n->n+1} of a step, Sec. 3.3): every zone's
 * distribution is remapped from its comoving frame under the current
 * background to its comoving frame under the new one (same place and basis,
 * no rotation, time kick of chain_frames), then the new background is
 * adopted.  The outflow tally is kept. */
int orc_update_background(orc_ctx *c, const double *v_r, const double *v_theta,
                          const double *v_phi, const double *alpha, const double *psi,
                          const double *ka, const double *ks, const double *feq)
{
  if (!c) return 1;
  if (!c->have_bg || !c->have_state) return 5;
  int n = c->eblk;
  double *tmp = (double *)malloc(sizeof(double) * n);
  for (int z = 0; z < c->nz; ++z) {
    frame_t S = zone_frame(c, z, zone_th(c, z), 0.0), D = S;
    D.v[0] = v_r[z]; D.v[1] = v_theta[z]; D.v[2] = v_phi ? v_phi[z] : 0.0;
    D.alpha = alpha[z]; D.psi = psi[z];
    for (int s = 0; s < c->ns; ++s) {
      double *blk = c->f + (size_t)z * c->blk + (size_t)s * n;
      remap(c, &S, &D, -1, 0, 1, 0, blk, tmp);
      memcpy(blk, tmp, sizeof(double) * n);
    }
  }
  free(tmp);
  return orc_set_background(c, v_r, v_theta, v_phi, alpha, psi, ka, ks, feq);
}

/* hydro source terms of the last full step: q[zone][5] = Q_Ye, Q_E, Q_M,r,
 * Q_M,theta, Q_M,phi (comoving frame, per unit volume and time, without 1/h^3) */
int orc_source_terms(const orc_ctx *c, double *q)
{
  if (!c) return 1;
  memcpy(q, c->q, sizeof(double) * 5 * (size_t)c->nz);
  return 0;
}

/* ------------------------------------------------- local time stepping */

/* Courant length of zone z: its volume over its largest face on an axis,
 * the smallest over the axes (the global step is cfl times its minimum) */
static double courant_length(const orc_ctx *c, int z)
{
  int fids[8], sg[8];
  double amax[3] = { 0.0, 0.0, 0.0 }, m = 1e300;
  int nfz = zone_faces(c, z, fids, sg);
  for (int q = 0; q < nfz; ++q) {
    double A;
    int ax = fids[q] < c->nfr ? 0 : (fids[q] < c->nfr + c->nft ? 1 : 2);
    get_face_geom(c, fids[q], &A);
    if (A > amax[ax]) amax[ax] = A;
  }
  for (int ax = 0; ax < 3; ++ax)
    if (amax[ax] > 0.0 && c->vol[z] / amax[ax] < m) m = c->vol[z] / amax[ax];
  return m;
}

/* Time levels for local time stepping (Sec. 5 names it as the way to stop
 * the small central zones from setting every zone's step; the paper gives no
 * scheme).  Reading: zone z steps with 2^l dt0, l = floor(log2(L_z / L_min))
 * of its Courant length L_z, capped at max_level, then lowered until zones
 * that share a face differ by at most one level. */
int orc_time_levels(const orc_ctx *c, int max_level, int *lev)
{
  if (!c || max_level < 0 || max_level > 16) return 1;
  double lmin = 1e300;
  double *L = (double *)malloc(sizeof(double) * c->nz);
  for (int z = 0; z < c->nz; ++z) { L[z] = courant_length(c, z); if (L[z] < lmin) lmin = L[z]; }
  for (int z = 0; z < c->nz; ++z) {
    int l = 0;
    while (l < max_level && L[z] >= lmin * (double)(2 << l) * (1.0 - 1e-12)) ++l;
    lev[z] = l;
  }
  free(L);
  for (int changed = 1; changed;) {
    changed = 0;
    for (int f = 0; f < c->nf; ++f) {
      face_t F;
      get_face(c, f, &F);
      if (!F.active || F.L.kind != SIDE_ZONE || F.R.kind != SIDE_ZONE) continue;
      int a = F.L.z, b = F.R.z;
      if (lev[a] > lev[b] + 1) { lev[a] = lev[b] + 1; changed = 1; }
      if (lev[b] > lev[a] + 1) { lev[b] = lev[a] + 1; changed = 1; }
    }
  }
  return 0;
}

/* levels: per zone, 0..16, neighbours at most one apart; NULL: global step */
int orc_set_levels(orc_ctx *c, const int *levels)
{
  if (!c) return 1;
  free(c->lev);
  c->lev = NULL;
  c->lmax = 0;
  if (!levels) return 0;
  c->lev = (int *)malloc(sizeof(int) * c->nz);
  for (int z = 0; z < c->nz; ++z) {
    if (levels[z] < 0 || levels[z] > 16) { free(c->lev); c->lev = NULL; return 1; }
    c->lev[z] = levels[z];
    if (levels[z] > c->lmax) c->lmax = levels[z];
  }
  return 0;
}

/* One step with time levels: 2^L substeps of dt0, L the highest level.  At
 * substep k every face whose finer zone starts a step (k mod 2^m = 0, m the
 * smaller level of the zones on its sides) is evaluated from the current
 * state with dt = 2^m dt0, and its content changes are added to the zones on
 * both sides; then every zone whose step ends (k + 1 mod 2^l = 0) is updated
 * with the changes it gathered and dt = 2^l dt0.  A zone at a coarser level
 * thus receives the fluxes of each of its finer neighbour's steps, and what
 * leaves one zone enters the other.  With every level 0 this is the global
 * step. */
static int lts_step(orc_ctx *c, double dt0)
{
  const size_t blk = c->blk;
  double *acc = (double *)calloc((size_t)c->nz * blk, sizeof(double));
  double *fbuf = (double *)malloc(sizeof(double) * 2 * blk * (size_t)c->nf);
  int *on = (int *)malloc(sizeof(int) * c->nf);
  if (!acc || !fbuf || !on) { free(acc); free(fbuf); free(on); return 2; }
  const int nsub = 1 << c->lmax;
  for (int k = 0; k < nsub; ++k) {
    const double *f = c->f;
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < c->nf; ++q) {
      face_t F;
      get_face(c, q, &F);
      int m = c->lev[F.L.z] < c->lev[F.R.z] ? c->lev[F.L.z] : c->lev[F.R.z];
      on[q] = F.active && k % (1 << m) == 0;
      if (!on[q]) continue;
      double *sL = (double *)calloc(blk, sizeof(double)), *sR = (double *)calloc(blk, sizeof(double));
      if (F.L.has_slope) zone_slope(c, f, F.L.z, F.axis, sL);
      if (F.R.has_slope) zone_slope(c, f, F.R.z, F.axis, sR);
      double *dl = fbuf + 2 * (size_t)q * blk;
      face_contrib(c, &F, f, sL, sR, dt0 * (double)(1 << m), dl, dl + blk, NULL, NULL);
      free(sL); free(sR);
    }
#pragma omp parallel for schedule(dynamic)
    for (int z = 0; z < c->nz; ++z) {
      int fz[8], sz[8], nfz = zone_faces(c, z, fz, sz);
      for (int q = 0; q < nfz; ++q) {
        if (!on[fz[q]]) continue;
        const double *src = fbuf + 2 * (size_t)fz[q] * blk + (sz[q] > 0 ? blk : 0);
        double *dst = acc + (size_t)z * blk;
        for (size_t p = 0; p < blk; ++p) dst[p] += src[p];
      }
    }
    for (int q = 0; q < c->nf; ++q) {             /* number leaving the domain */
      if (!on[q]) continue;
      face_t F;
      get_face(c, q, &F);
      for (int side = 0; side < 2; ++side) {
        const side_t *sd = side ? &F.R : &F.L;
        if (sd->kind == SIDE_ZONE) continue;
        const double *src = fbuf + 2 * (size_t)q * blk + (side ? blk : 0);
        for (int s = 0; s < c->ns; ++s) {
          double t = 0.0;
          for (int p = 0; p < c->eblk; ++p) t += src[(size_t)s * c->eblk + p];
          c->outflow[s] += t;
        }
      }
    }
#pragma omp parallel for schedule(dynamic)
    for (int z = 0; z < c->nz; ++z) {
      if ((k + 1) % (1 << c->lev[z])) continue;
      zone_update(c, z, acc + (size_t)z * blk, dt0 * (double)(1 << c->lev[z]),
                  c->fn + (size_t)z * blk, c->q + 5 * (size_t)z);
    }
    for (int z = 0; z < c->nz; ++z) {            /* the updated zones take their new state */
      if ((k + 1) % (1 << c->lev[z])) continue;
      memcpy(c->f + (size_t)z * blk, c->fn + (size_t)z * blk, sizeof(double) * blk);
      memset(acc + (size_t)z * blk, 0, sizeof(double) * blk);
    }
  }
  free(acc); free(fbuf); free(on);
  return 0;
}
