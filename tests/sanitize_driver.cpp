// Host-only driver for the address and undefined-behaviour sanitizer build of
// the reference stepper (oracle/btx_oracle.c) and of libbtx's host-side grid
// set-up (csrc/btx_grid.cpp).  Built and run by tests/test_sanitizers.py with
// gcc's -fsanitize=address,undefined; any invalid access, overflow or
// undefined operation aborts the run.
//
// Each case builds one small grid of every kind the library accepts (the
// column from r = 0 and on logarithmic radii, the axisymmetric wedge with the
// axis at both ends, the equatorial disk boundary, a 3D grid of phi zones,
// the slab) through both codes, then drives every entry point of the
// reference: background, state, steps, sampled steps, moments, source terms,
// time levels, background update, per-face debug output, face geometry, the
// frame chain, the block remap and the collision solve.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../oracle/btx_oracle.h"
#include "../paper_2003_02845_amd/csrc/btx_grid.h"

namespace {

const double kPi = 3.14159265358979323846;

struct Case {
  const char *name;
  int n_r, n_theta, n_eps, n_mu, n_phi, n_species;
  int geometry, phi_rule, inner_bc, outer_bc, lobatto;
  double r0, r1;
  bool log_r;
  double dphi;
  int theta_bc;
  double disk_radius;
  int n_phi_zones;
};

// quadrature nodes of the two rules at the sizes used here (closed forms)
void quadrature(bool lobatto, int n, std::vector<double> &x, std::vector<double> &w)
{
  if (!lobatto && n == 4) {
    const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
    x = { -b, -a, a, b };
    w = { wb, wa, wa, wb };
  } else if (lobatto && n == 5) {
    const double a = std::sqrt(3.0 / 7.0);
    x = { -1.0, -a, 0.0, a, 1.0 };
    w = { 0.1, 49.0 / 90.0, 32.0 / 45.0, 49.0 / 90.0, 0.1 };
  } else {
    std::fprintf(stderr, "no quadrature for n=%d\n", n);
    std::exit(2);
  }
}

double urand(unsigned long long &s)
{
  s = s * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(s >> 11) * (1.0 / 9007199254740992.0);
}

int run_case(const Case &k)
{
  const int nth = k.geometry == ORC_GEOM_AXISYM2D ? k.n_theta : 1;
  const int nph = k.geometry == ORC_GEOM_AXISYM2D && k.n_phi_zones > 1 ? k.n_phi_zones : 1;
  const int nz = k.n_r * nth * nph, ndir = k.n_mu * k.n_phi, blk = k.n_species * k.n_eps * ndir;
  std::vector<double> re(k.n_r + 1), te(nth + 1), ee(k.n_eps + 1), mu, wmu;
  for (int a = 0; a <= k.n_r; ++a)
    re[a] = k.log_r ? k.r0 * std::pow(k.r1 / k.r0, (double)a / k.n_r) : k.r0 + (k.r1 - k.r0) * a / k.n_r;
  const double tmax = k.theta_bc == ORC_THETA_DISK ? 0.5 * kPi : kPi;
  for (int b = 0; b <= nth; ++b) te[b] = tmax * b / nth;
  for (int i = 0; i <= k.n_eps; ++i) ee[i] = 2.0 * std::pow(100.0, (double)i / k.n_eps);
  quadrature(k.lobatto, k.n_mu, mu, wmu);

  // the library's host-side grid
  btx::Grid g;
  g.nr = k.n_r; g.nth = nth; g.ne = k.n_eps; g.nmu = k.n_mu; g.nphi = k.n_phi; g.ns = k.n_species;
  g.geom = k.geometry; g.mu_rule = k.lobatto; g.phi_rule = k.phi_rule;
  g.inner_bc = k.inner_bc; g.outer_bc = k.outer_bc; g.prec = 0;
  g.theta_bc = k.geometry == ORC_GEOM_AXISYM2D ? k.theta_bc : ORC_THETA_AXIS;
  g.nph = nph; g.disk_r = k.disk_radius; g.dphi = k.dphi;
  g.r_e = re; g.eps_e = ee;
  g.th_e = k.geometry == ORC_GEOM_AXISYM2D ? te : std::vector<double>{ 0.0, kPi };
  const std::string why = btx::build_grid(g);
  if (!why.empty()) { std::fprintf(stderr, "%s: build_grid: %s\n", k.name, why.c_str()); return 1; }
  const double dt_lib = btx::max_dt(g, 0.4);
  if (g.nz != nz || g.ndir != ndir || !(dt_lib > 0.0)) { std::fprintf(stderr, "%s: grid sizes\n", k.name); return 1; }
  std::vector<double> qx, qw;
  for (int rule = 0; rule < 2; ++rule)
    for (int n = 2; n <= 24; ++n)
      if (!btx::gauss_rule(rule, n, qx, qw)) { std::fprintf(stderr, "gauss_rule %d %d\n", rule, n); return 1; }

  // the reference
  orc_desc d = {};
  d.n_r = k.n_r; d.n_theta = nth; d.n_eps = k.n_eps; d.n_mu = k.n_mu; d.n_phi = k.n_phi;
  d.n_species = k.n_species; d.geometry = k.geometry; d.phi_rule = k.phi_rule;
  d.inner_bc = k.inner_bc; d.outer_bc = k.outer_bc;
  d.r_edges = re.data(); d.theta_edges = te.data(); d.dphi = k.dphi; d.eps_edges = ee.data();
  d.mu_nodes = mu.data(); d.mu_weights = wmu.data();
  d.theta_bc = k.theta_bc; d.disk_radius = k.disk_radius; d.n_phi_zones = k.n_phi_zones;
  orc_ctx *c = orc_create(&d);
  if (!c) { std::fprintf(stderr, "%s: orc_create\n", k.name); return 1; }

  unsigned long long seed = 0x2003028450ULL + (unsigned long long)nz;
  const size_t nk = (size_t)nz * k.n_species * k.n_eps;
  std::vector<double> vr(nz), vt(nz), vp(nz), al(nz), ps(nz), ka(nk), ks(nk), fe(nk), f((size_t)nz * blk);
  auto background = [&](double amp) {
    for (int z = 0; z < nz; ++z) {
      vr[z] = amp * (urand(seed) - 0.5);
      vt[z] = k.geometry == ORC_GEOM_AXISYM2D ? 0.5 * amp * (urand(seed) - 0.5) : 0.0;
      vp[z] = nph > 1 ? 0.3 * amp * (urand(seed) - 0.5) : 0.0;
      al[z] = 0.8 + 0.2 * urand(seed);
      ps[z] = 1.0 / std::sqrt(al[z]);
    }
    for (size_t i = 0; i < nk; ++i) {
      ka[i] = std::pow(10.0, 4.0 * urand(seed) - 2.0);
      ks[i] = std::pow(10.0, 4.0 * urand(seed) - 2.0);
      fe[i] = urand(seed);
    }
  };
  background(0.2);
  int rc = orc_set_background(c, vr.data(), vt.data(), vp.data(), al.data(), ps.data(), ka.data(), ks.data(), fe.data());
  for (double &x : f) x = urand(seed);
  rc |= orc_set_state(c, f.data());
  const double dt = orc_max_dt(c, 0.4);
  if (rc || !(dt > 0.0)) { std::fprintf(stderr, "%s: set-up\n", k.name); orc_destroy(c); return 1; }

  for (int mode : { 0, 1, -1 }) {
    orc_set_blend_mode(c, mode);
    rc |= orc_step(c, dt, 1);
  }
  std::vector<int> zl = { 0, nz - 1, nz / 2 };
  std::vector<double> fs(zl.size() * (size_t)blk);
  rc |= orc_step_sample(c, dt, (int)zl.size(), zl.data(), fs.data());

  std::vector<double> zm((size_t)nz * k.n_species * 5), tot(k.n_species * 3), q((size_t)nz * 5);
  rc |= orc_moments(c, zm.data(), tot.data());
  rc |= orc_source_terms(c, q.data());

  std::vector<int> lev(nz);
  rc |= orc_time_levels(c, 3, lev.data());
  rc |= orc_set_levels(c, lev.data());
  rc |= orc_step(c, dt, 1);
  rc |= orc_set_levels(c, nullptr);

  background(0.25);
  rc |= orc_update_background(c, vr.data(), vt.data(), vp.data(), al.data(), ps.data(), ka.data(), ks.data(), fe.data());
  rc |= orc_step(c, dt, 1);

  const int nf = orc_n_faces(c);
  std::vector<double> flw(blk), flux(blk), dN(2 * (size_t)blk), info(8);
  for (int fid = 0; fid < nf; fid += 1 + nf / 7) {
    rc |= orc_face_debug(c, fid, dt, flw.data(), flux.data(), dN.data(), info.data());
    int zones[2];
    double ginfo[3];
    rc |= orc_face_geom(c, fid, zones, ginfo);
  }
  std::vector<double> vol(nz), rcen(nz), tcen(nz);
  rc |= orc_geometry(c, vol.data(), rcen.data(), tcen.data());
  rc |= orc_get_state(c, f.data());

  const double S[7] = { 0.2, 0.05, 0.0, 0.9, 1.05, 0.6, 0.0 };
  const double D[7] = { -0.1, 0.02, 0.0, 0.85, 1.08, 0.7, 0.1 };
  const double u_in[4] = { 1.0, 0.6, 0.0, 0.8 };
  double u_out[4];
  for (int axis = 0; axis < 3; ++axis) orc_chain(S, D, axis, 1, u_in, u_out);
  std::vector<double> X((size_t)k.n_eps * ndir), Y((size_t)k.n_eps * ndir);
  for (double &x : X) x = urand(seed);
  for (int density = 0; density < 2; ++density)
    rc |= orc_remap_block(c, S, D, 0, 1, density, 1, X.data(), Y.data());
  std::vector<double> dOm(ndir, 4.0 * kPi / ndir), fc(ndir), out(ndir);
  for (double &x : fc) x = urand(seed);
  orc_collide(ndir, fc.data(), nullptr, dt, 1.0, 10.0, 0.5, dOm.data(), out.data());
  orc_destroy(c);

  double s = 0.0;
  for (double x : f) s += x;
  if (rc || !std::isfinite(s)) { std::fprintf(stderr, "%s: rc %d, sum %g\n", k.name, rc, s); return 1; }
  std::printf("%s: %d zones, %d faces, dt %.3e (library %.3e)\n", k.name, nz, nf, dt, dt_lib);
  return 0;
}

}  // namespace

int main()
{
  const Case cases[] = {
    // name        n_r th eps mu phi s  geometry          phi rule        inner bc        outer bc        lob r0    r1      log    dphi  theta bc        disk  phi zones
    { "column",    6,  1, 3,  4, 4,  2, ORC_GEOM_COLUMN,   ORC_PHI_SIN,    ORC_BC_REFLECT, ORC_BC_OUTFLOW, 0, 0.0,  2.0,    false, 0.0,  ORC_THETA_AXIS, 0.0, 0 },
    { "log_column", 5, 1, 4,  5, 4,  1, ORC_GEOM_COLUMN,   ORC_PHI_LINEAR, ORC_BC_REFLECT, ORC_BC_EQUIL,   1, 10.0, 1000.0, true,  0.3,  ORC_THETA_AXIS, 0.0, 0 },
    { "axisym",    4,  5, 3,  4, 4,  2, ORC_GEOM_AXISYM2D, ORC_PHI_SIN,    ORC_BC_REFLECT, ORC_BC_OUTFLOW, 0, 1.0,  3.0,    false, 0.4,  ORC_THETA_AXIS, 0.0, 0 },
    { "disk",      4,  3, 2,  5, 4,  1, ORC_GEOM_AXISYM2D, ORC_PHI_LINEAR, ORC_BC_REFLECT, ORC_BC_OUTFLOW, 1, 0.0,  4.0,    false, 0.5,  ORC_THETA_DISK, 2.0, 0 },
    { "3d",        3,  4, 2,  4, 4,  1, ORC_GEOM_AXISYM2D, ORC_PHI_SIN,    ORC_BC_REFLECT, ORC_BC_OUTFLOW, 0, 1.0,  2.0,    false, 0.5,  ORC_THETA_AXIS, 0.0, 3 },
    { "slab",      7,  1, 2,  4, 1,  1, ORC_GEOM_PLANAR,   ORC_PHI_SIN,    ORC_BC_OUTFLOW, ORC_BC_OUTFLOW, 0, -1.0, 1.0,    false, 0.0,  ORC_THETA_AXIS, 0.0, 0 },
  };
  int bad = 0;
  for (const Case &k : cases) bad += run_case(k);
  std::printf(bad ? "FAILED\n" : "all cases done\n");
  return bad ? 1 : 0;
}
