// Host-side grid set-up for libbtx: quadrature, flat-faced cell geometry,
// face descriptors and time-step limit (paper Sec. 3.1 and Sec. 3.3).
// Everything here runs once per grid in FP64 on the host; the per-step work
// lives in btx.hip.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace btx {

enum SideKind : int32_t { SIDE_ZONE = 0, SIDE_MIRROR = 1, SIDE_ZERO = 2, SIDE_EQ = 3 };

// One side of a face, or a slope neighbour: where its data comes from and the
// basis angles of the frame in which that data is expressed.
struct SideDesc {
  int32_t kind;      // SideKind
  int32_t z;         // zone supplying data and background
  int32_t slope;     // 1: a real zone (or its periodic image) that is reconstructed
  int32_t pad;
  double th, ph;     // basis angles of the side's frame
  double sth, cth, sph, cph;  // their sines and cosines (set once per grid)
};

// Everything a face kernel needs about one face.  Normal from L to R.
struct FaceDesc {
  SideDesc L, R;     // the two sides
  SideDesc Lm, Rp;   // L's neighbour away from the face, R's neighbour away from it
  double ths, phs;   // interface basis angles
  double sts, cts, sps, cps;  // their sines and cosines (set once per grid)
  double area;       // flat quadrilateral area
  double h;          // L-R centre distance (Lax-Wendroff dx and blend optical depth)
  double dL, dR;     // signed reconstruction distances L -> face, R -> face
  double hLm, hRp;   // centre distances L-Lm and R-Rp
  int32_t axis;      // 0 r (z), 1 theta, 2 phi
  int32_t active;    // 0: zero-area face (apex), contributes nothing
  int32_t zero_opacity;  // outflow ghost on one side: interface opacity 0
  int32_t self;      // periodic self-face: R is the zone's own image, sigma_R = sigma_L
};

struct ZoneFaces {   // faces touching a zone, and the side the zone is on
  int32_t n;
  int32_t fid[8];
  int32_t side[8];   // 0: zone is L, 1: zone is R
};

struct Grid {
  int nr = 0, nth = 0, nph = 1, ne = 0, nmu = 0, nphi = 0, ns = 0, ndir = 0, nz = 0;
  int geom = 0, mu_rule = 0, phi_rule = 0, inner_bc = 0, outer_bc = 0, prec = 0;
  int theta_bc = 0;                                     // 1: equatorial disk boundary at pi/2
  double disk_r = 0;
  double dphi = 0, delta = 0, q = 0, lnq = 0, fp64_thr = 1.0;
  std::vector<double> r_e, th_e, eps_e;
  std::vector<double> eps, G, mu, wmu, Phi, dOm, nvec;  // momentum grid
  std::vector<double> rc, thc, vol;                     // zones
  std::vector<FaceDesc> faces;
  std::vector<ZoneFaces> zfaces;
  std::vector<int32_t> bface;                           // faces with a ghost side
};

// Fills quadrature nodes (ascending) and weights; false if n is out of range.
bool gauss_rule(int rule, int n, std::vector<double> &x, std::vector<double> &w);
// Builds the whole grid; returns an empty string on success, else the reason.
std::string build_grid(Grid &g);
// Courant limit: cfl times the smallest zone volume / largest face on an axis.
double max_dt(const Grid &g, double cfl);

}  // namespace btx
