// Host-side grid set-up for libbtx (see btx_grid.h).
#include "btx_grid.h"

#include <algorithm>
#include <cmath>

namespace btx {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Legendre P_n and P_{n-1} at x by the three-term recurrence
void legendre(int n, double x, double &pn, double &pn1)
{
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

struct P3 { double x, y, z; };

P3 point(double r, double th, double ph)
{
  return { r * std::sin(th) * std::cos(ph), r * std::sin(th) * std::sin(ph), r * std::cos(th) };
}

P3 sub(P3 a, P3 b) { return { a.x - b.x, a.y - b.y, a.z - b.z }; }
P3 cross(P3 a, P3 b) { return { a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x }; }
double norm(P3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

// planar quadrilateral a-b-c-d (in order around the face): half the cross
// product of the diagonals
double quad(P3 a, P3 b, P3 c, P3 d) { return 0.5 * norm(cross(sub(c, a), sub(d, b))); }

double dist(double r1, double t1, double p1, double r2, double t2, double p2)
{
  return norm(sub(point(r1, t1, p1), point(r2, t2, p2)));
}

}  // namespace

bool gauss_rule(int rule, int n, std::vector<double> &x, std::vector<double> &w)
{
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  if (rule == 0) {                       // Gauss-Legendre: roots of P_n
    if (n < 1) return false;
    for (int k = 0; k < n; ++k) {
      double t = std::cos(kPi * (k + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p, pm;
        legendre(n, t, p, pm);
        double dp = n * (t * p - pm) / (t * t - 1.0);
        double dt = p / dp;
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
      double p, pm;
      legendre(n, t, p, pm);
      double dp = n * (t * p - pm) / (t * t - 1.0);
      x[k] = t;
      w[k] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
  } else {                               // Gauss-Lobatto: +-1 and roots of P'_{n-1}
    if (n < 2) return false;
    int m = n - 1;
    x[0] = -1.0;
    x[n - 1] = 1.0;
    for (int k = 1; k < n - 1; ++k) {
      double t = -std::cos(kPi * k / m);
      // (1 - t^2) P'_m(t) = m (P_{m-1}(t) - t P_m(t)); Newton on g = P_{m-1} - t P_m
      for (int it = 0; it < 100; ++it) {
        double p, pm;
        legendre(m, t, p, pm);
        double g = pm - t * p;
        // g' = -(m+1) P_m(t) ... from d/dt[(1-t^2) P'_m] = -m(m+1) P_m
        double dg = -(m + 1.0) * p;
        double dt = g / dg;
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
      x[k] = t;
    }
    std::sort(x.begin(), x.end());
    for (int k = 0; k < n; ++k) {
      double p, pm;
      legendre(m, x[k], p, pm);
      w[k] = 2.0 / (n * (n - 1.0) * p * p);
    }
  }
  if (rule == 0) std::sort(x.begin(), x.end());
  if (rule == 0) {                       // re-pair weights with the sorted nodes
    for (int k = 0; k < n; ++k) {
      double p, pm;
      legendre(n, x[k], p, pm);
      double dp = n * (x[k] * p - pm) / (x[k] * x[k] - 1.0);
      w[k] = 2.0 / ((1.0 - x[k] * x[k]) * dp * dp);
    }
  }
  return true;
}

std::string build_grid(Grid &g)
{
  g.ndir = g.nmu * g.nphi;
  g.nz = g.nr * g.nth * g.nph;        // zone (c n_theta + b) n_r + a
  // momentum grid: geometric group centres, shell volumes per unit solid angle
  g.eps.resize(g.ne);
  g.G.resize(g.ne);
  for (int i = 0; i < g.ne; ++i) {
    g.eps[i] = std::sqrt(g.eps_e[i] * g.eps_e[i + 1]);
    g.G[i] = (std::pow(g.eps_e[i + 1], 3.0) - std::pow(g.eps_e[i], 3.0)) / 3.0;
  }
  // the remap shifts all groups of a direction by the same log-energy step
  g.lnq = std::log(g.eps_e[g.ne] / g.eps_e[0]) / g.ne;
  g.q = std::exp(g.lnq);
  for (int i = 0; i < g.ne; ++i) {
    double r = std::log(g.eps_e[i + 1] / g.eps_e[i]);
    if (std::fabs(r - g.lnq) > 1e-9 * g.lnq) return "energy edges must be logarithmically spaced";
  }
  if (!gauss_rule(g.mu_rule == 0 ? 0 : 1, g.nmu, g.mu, g.wmu)) return "bad mu quadrature size";
  g.Phi.resize(g.nphi);
  for (int k = 0; k < g.nphi; ++k) g.Phi[k] = (k + 0.5) * 2.0 * kPi / g.nphi;
  g.dOm.resize(g.ndir);
  g.nvec.resize(3 * g.ndir);
  for (int j = 0; j < g.nmu; ++j) {
    double st = std::sqrt(1.0 - g.mu[j] * g.mu[j]);
    for (int k = 0; k < g.nphi; ++k) {
      int d = j * g.nphi + k;
      g.dOm[d] = g.wmu[j] * 2.0 * kPi / g.nphi;
      g.nvec[3 * d + 0] = g.mu[j];
      g.nvec[3 * d + 1] = st * std::cos(g.Phi[k]);
      g.nvec[3 * d + 2] = st * std::sin(g.Phi[k]);
    }
  }
  // column width: free (Sec. 3.3.4 recommends faces of similar area); the
  // grid's dphi when given, else the width at which the outermost zone's
  // lateral faces match its radial face
  g.delta = g.geom == 0 && g.dphi > 0.0 ? g.dphi : (g.r_e[g.nr] - g.r_e[g.nr - 1]) / g.r_e[g.nr];
  const bool planar = g.geom == 2, twod = g.geom == 1;
  auto row_angles = [&](int b, double &t0, double &t1, double &p0, double &p1) {
    if (twod) { t0 = g.th_e[b]; t1 = g.th_e[b + 1]; p0 = -0.5 * g.dphi; p1 = 0.5 * g.dphi; }
    else { t0 = 0.5 * kPi - 0.5 * g.delta; t1 = 0.5 * kPi + 0.5 * g.delta; p0 = -0.5 * g.delta; p1 = 0.5 * g.delta; }
  };
  auto row_th = [&](int b) { return planar ? 0.0 : (twod ? 0.5 * (g.th_e[b] + g.th_e[b + 1]) : 0.5 * kPi); };
  g.rc.resize(g.nz);
  g.thc.resize(g.nz);
  g.vol.resize(g.nz);
  std::vector<double> A1(g.nth, 1.0);
  for (int b = 0; b < g.nth; ++b) {
    double h1 = 1.0;
    if (!planar) {
      double t0, t1, p0, p1;
      row_angles(b, t0, t1, p0, p1);
      P3 a = point(1, t0, p0), bb = point(1, t1, p0), c = point(1, t1, p1), d = point(1, t0, p1);
      P3 n = cross(sub(c, a), sub(d, bb));
      A1[b] = 0.5 * norm(n);
      h1 = std::fabs(n.x * a.x + n.y * a.y + n.z * a.z) / norm(n);
    }
    for (int c = 0; c < g.nph; ++c)
      for (int a = 0; a < g.nr; ++a) {
        int z = (c * g.nth + b) * g.nr + a;
        double r0 = g.r_e[a], r1 = g.r_e[a + 1];
        g.rc[z] = 0.5 * (r0 + r1);
        g.thc[z] = row_th(b);
        // flat-faced cell = difference of two pyramids with apex at the origin
        g.vol[z] = planar ? (r1 - r0) : (r1 * r1 * r1 - r0 * r0 * r0) * A1[b] * h1 / 3.0;
      }
  }
  auto zone_side = [&](int z, double th, double ph) {
    SideDesc s{ SIDE_ZONE, z, 1, 0, th, ph };
    return s;
  };
  auto ghost = [&](int z, int bc) {
    SideDesc s{ bc == 0 ? SIDE_MIRROR : (bc == 1 ? SIDE_ZERO : SIDE_EQ), z, 0, 0, g.thc[z], 0.0 };
    return s;
  };
  // beyond the equatorial plane of a disk grid: the mirror position of zone z,
  // a thick disk (equilibrium) inside the disk radius, empty outside
  const bool disk = twod && g.theta_bc == 1;
  auto theta_ghost = [&](int z) {
    SideDesc s{ g.rc[z] < g.disk_r ? SIDE_EQ : SIDE_ZERO, z, 0, 0, kPi - g.thc[z], 0.0 };
    return s;
  };
  auto mirror_dist = [&](int z) { return dist(g.rc[z], g.thc[z], 0.0, g.rc[z], kPi - g.thc[z], 0.0); };
  g.faces.clear();
  g.zfaces.assign(g.nz, ZoneFaces{});
  auto add_zone_face = [&](int z, int fid, int side) {
    ZoneFaces &zf = g.zfaces[z];
    zf.fid[zf.n] = fid;
    zf.side[zf.n] = side;
    ++zf.n;
  };
  // radial (slab: z) faces, per (phi zone, theta row) column
  for (int col = 0; col < g.nph * g.nth; ++col) {
    const int b = col % g.nth;
    double th = row_th(b);
    for (int a = -1; a < g.nr; ++a) {
      FaceDesc F{};
      double R = g.r_e[a + 1];
      int zL = col * g.nr + a, zR = zL + 1;
      F.axis = 0;
      F.active = planar || R > 0.0;
      F.area = planar ? 1.0 : R * R * A1[b];
      F.L = a >= 0 ? zone_side(zL, th, 0.0) : ghost(zR, g.inner_bc);
      F.R = a + 1 < g.nr ? zone_side(zR, th, 0.0) : ghost(zL, g.outer_bc);
      if (a >= 0 && a + 1 < g.nr) F.h = g.rc[zR] - g.rc[zL];
      else if (a < 0) F.h = 2.0 * (g.rc[zR] - R);
      else F.h = 2.0 * (R - g.rc[zL]);
      F.dL = a >= 0 ? R - g.rc[zL] : 0.5 * F.h;
      F.dR = a + 1 < g.nr ? -(g.rc[zR] - R) : -0.5 * F.h;
      F.ths = th;
      F.phs = 0.0;
      F.zero_opacity = (F.L.kind == SIDE_ZERO || F.R.kind == SIDE_ZERO);
      if (a >= 0) {                       // L's inner neighbour
        if (a >= 1) { F.Lm = zone_side(zL - 1, th, 0.0); F.hLm = g.rc[zL] - g.rc[zL - 1]; }
        else { F.Lm = ghost(zL, g.inner_bc); F.hLm = 2.0 * (g.rc[zL] - g.r_e[0]); }
      }
      if (a + 1 < g.nr) {                 // R's outer neighbour
        if (a + 2 < g.nr) { F.Rp = zone_side(zR + 1, th, 0.0); F.hRp = g.rc[zR + 1] - g.rc[zR]; }
        else { F.Rp = ghost(zR, g.outer_bc); F.hRp = 2.0 * (g.r_e[g.nr] - g.rc[zR]); }
      }
      int fid = (int)g.faces.size();
      g.faces.push_back(F);
      if (F.L.kind != SIDE_ZONE || F.R.kind != SIDE_ZONE) g.bface.push_back(fid);
      if (a + 1 < g.nr) add_zone_face(zR, fid, 1);
      if (a >= 0) add_zone_face(zL, fid, 0);
    }
  }
  // theta faces
  if (twod) {
    for (int c = 0; c < g.nph; ++c) {
    for (int b = 0; b + 1 < g.nth; ++b)
      for (int a = 0; a < g.nr; ++a) {
        FaceDesc F{};
        int zL = (c * g.nth + b) * g.nr + a, zR = zL + g.nr;
        double tf = g.th_e[b + 1], p0 = -0.5 * g.dphi, p1 = 0.5 * g.dphi;
        F.axis = 1;
        F.active = 1;
        F.area = quad(point(g.r_e[a], tf, p0), point(g.r_e[a + 1], tf, p0),
                      point(g.r_e[a + 1], tf, p1), point(g.r_e[a], tf, p1));
        F.L = zone_side(zL, g.thc[zL], 0.0);
        F.R = zone_side(zR, g.thc[zR], 0.0);
        F.h = dist(g.rc[zL], g.thc[zL], 0.0, g.rc[zR], g.thc[zR], 0.0);
        F.dL = 0.5 * F.h;
        F.dR = -0.5 * F.h;
        F.ths = tf;
        F.phs = 0.0;
        if (b >= 1) { F.Lm = zone_side(zL - g.nr, g.thc[zL - g.nr], 0.0);
                      F.hLm = dist(g.rc[zL - g.nr], g.thc[zL - g.nr], 0.0, g.rc[zL], g.thc[zL], 0.0); }
        else { F.Lm = zone_side(zL, g.thc[zL], 0.0); F.hLm = 1.0; }   // zero-gradient axis ghost
        if (b + 2 < g.nth) { F.Rp = zone_side(zR + g.nr, g.thc[zR + g.nr], 0.0);
                             F.hRp = dist(g.rc[zR], g.thc[zR], 0.0, g.rc[zR + g.nr], g.thc[zR + g.nr], 0.0); }
        else if (disk) { F.Rp = theta_ghost(zR); F.hRp = mirror_dist(zR); }
        else { F.Rp = zone_side(zR, g.thc[zR], 0.0); F.hRp = 1.0; }
        int fid = (int)g.faces.size();
        g.faces.push_back(F);
        add_zone_face(zR, fid, 1);
        add_zone_face(zL, fid, 0);
      }
    if (disk)                             // the equatorial boundary faces
      for (int a = 0; a < g.nr; ++a) {
        FaceDesc F{};
        const int b = g.nth - 1, zL = (c * g.nth + b) * g.nr + a;
        double tf = g.th_e[g.nth], p0 = -0.5 * g.dphi, p1 = 0.5 * g.dphi;
        F.axis = 1;
        F.active = 1;
        F.area = quad(point(g.r_e[a], tf, p0), point(g.r_e[a + 1], tf, p0),
                      point(g.r_e[a + 1], tf, p1), point(g.r_e[a], tf, p1));
        F.L = zone_side(zL, g.thc[zL], 0.0);
        F.R = theta_ghost(zL);
        F.h = mirror_dist(zL);
        F.dL = 0.5 * F.h;
        F.dR = -0.5 * F.h;
        F.ths = tf;
        F.phs = 0.0;
        F.zero_opacity = F.R.kind == SIDE_ZERO;
        if (b >= 1) { F.Lm = zone_side(zL - g.nr, g.thc[zL - g.nr], 0.0);
                      F.hLm = dist(g.rc[zL - g.nr], g.thc[zL - g.nr], 0.0, g.rc[zL], g.thc[zL], 0.0); }
        else { F.Lm = zone_side(zL, g.thc[zL], 0.0); F.hLm = 1.0; }
        int fid = (int)g.faces.size();
        g.faces.push_back(F);
        g.bface.push_back(fid);
        add_zone_face(zL, fid, 0);
      }
    }
  } else if (!planar) {                   // column: periodic self-face in theta
    for (int a = 0; a < g.nr; ++a) {
      FaceDesc F{};
      int z = a;
      double t0 = 0.5 * kPi, tf = t0 + 0.5 * g.delta, t1 = t0 + g.delta;
      double p0 = -0.5 * g.delta, p1 = 0.5 * g.delta;
      F.axis = 1;
      F.active = 1;
      F.self = 1;
      F.area = quad(point(g.r_e[a], tf, p0), point(g.r_e[a + 1], tf, p0),
                    point(g.r_e[a + 1], tf, p1), point(g.r_e[a], tf, p1));
      F.L = zone_side(z, t0, 0.0);
      F.R = zone_side(z, t1, 0.0);
      F.Lm = zone_side(z, t0 - g.delta, 0.0);
      F.Rp = zone_side(z, t1 + g.delta, 0.0);
      F.h = dist(g.rc[z], t0, 0.0, g.rc[z], t1, 0.0);
      F.hLm = F.hRp = F.h;
      F.dL = 0.5 * F.h;
      F.dR = -0.5 * F.h;
      F.ths = tf;
      F.phs = 0.0;
      int fid = (int)g.faces.size();
      g.faces.push_back(F);
      add_zone_face(z, fid, 0);
      add_zone_face(z, fid, 1);
    }
  }
  // phi faces: between phi zone c and c+1 (periodic); the zone's own image
  // one wedge over in the axisymmetric wedge and the column
  if (!planar) {
    const int base = (int)g.faces.size();   // the phi face of zone z is base + z
    for (int z = 0; z < g.nz; ++z) {
      FaceDesc F{};
      int a = z % g.nr, b = (z / g.nr) % g.nth, c = z / (g.nr * g.nth);
      auto at = [&](int cc) { return (((cc % g.nph) + g.nph) % g.nph * g.nth + b) * g.nr + a; };
      double t0, t1, p0, p1;
      row_angles(b, t0, t1, p0, p1);
      double w = p1 - p0, pf = 0.5 * w, th = g.thc[z];
      F.axis = 2;
      F.active = 1;
      F.self = g.nph == 1;
      F.area = quad(point(g.r_e[a], t0, pf), point(g.r_e[a + 1], t0, pf),
                    point(g.r_e[a + 1], t1, pf), point(g.r_e[a], t1, pf));
      F.L = zone_side(z, th, 0.0);
      F.R = zone_side(at(c + 1), th, w);
      F.Lm = zone_side(at(c - 1), th, -w);
      F.Rp = zone_side(at(c + 2), th, 2.0 * w);
      F.h = dist(g.rc[z], th, 0.0, g.rc[z], th, w);
      F.hLm = F.hRp = F.h;
      F.dL = 0.5 * F.h;
      F.dR = -0.5 * F.h;
      F.ths = th;
      F.phs = pf;
      g.faces.push_back(F);
      // each zone lists its own phi face (zone is L), then its predecessor's
      // (zone is R), the order of the axisymmetric wedge's self-face
      add_zone_face(z, base + z, 0);
      add_zone_face(z, base + at(c - 1), 1);
    }
  }
  // the sines and cosines of every basis angle, once per grid: the remap
  // tables are built again for every background, the angles stay
  auto trig = [](SideDesc &s) {
    s.sth = std::sin(s.th); s.cth = std::cos(s.th);
    s.sph = std::sin(s.ph); s.cph = std::cos(s.ph);
  };
  for (FaceDesc &F : g.faces) {
    trig(F.L); trig(F.R); trig(F.Lm); trig(F.Rp);
    F.sts = std::sin(F.ths); F.cts = std::cos(F.ths);
    F.sps = std::sin(F.phs); F.cps = std::cos(F.phs);
  }
  return "";
}

double max_dt(const Grid &g, double cfl)
{
  double m = 1e300;
  for (int z = 0; z < g.nz; ++z) {
    double amax[3] = { 0.0, 0.0, 0.0 };
    const ZoneFaces &zf = g.zfaces[z];
    for (int q = 0; q < zf.n; ++q) {
      const FaceDesc &F = g.faces[zf.fid[q]];
      if (F.active && F.area > amax[F.axis]) amax[F.axis] = F.area;
    }
    for (int ax = 0; ax < 3; ++ax)
      if (amax[ax] > 0.0) m = std::min(m, g.vol[z] / amax[ax]);
  }
  return cfl * m;
}

}  // namespace btx
