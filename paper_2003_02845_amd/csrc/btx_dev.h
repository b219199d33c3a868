// Device side of libbtx: data descriptors, device helpers and kernel
// templates, shared by the translation units that instantiate them (btx.hip
// for the table, time-remap, zone and moment kernels; btx_face32.hip and
// btx_face64.hip for the face kernels, compiled in parallel).
// Everything device-side has internal linkage in each unit; units exchange
// kernels as function pointers only.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../include/btx.h"
#include "btx_grid.h"

namespace btx {

// Face work-item shape: nch items per direction (a power of two), CE groups
// per item, the workgroup size bound and whether group -1 ends an item.
// FP32 takes 8 items per direction by default (up to 96 directions in
// workgroups of up to 768 threads, up to 128 in 1024) or 4.  FP64 takes 8 up
// to 96 directions where its buffers fit in LDS, else 4 (up to 128
// directions, 512 threads).  CE is the smallest instantiated value with
// nch CE >= ne + 3.
struct FaceShape {
  int nch = 0, ce = 0, maxt = 0;
  bool split = false;
  bool gtab = false;                 // tables read from global memory
  bool operator==(const FaceShape &o) const
  {
    return nch == o.nch && ce == o.ce && maxt == o.maxt && split == o.split && gtab == o.gtab;
  }
};

// the face-kernel instances of a shape (nullptr: none)
const void *face_fn_f32(const FaceShape &f);
const void *face_fn_f64(const FaceShape &f);

}  // namespace btx

namespace {

using btx::FaceDesc;
using btx::SideDesc;

constexpr int kTables = 8;    // remap tables per face
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------ device data

constexpr int kQpow = 257;          // the powers q^k, k = -128 .. 128

struct DevGrid {
  int nr, nth, ne, nmu, nphi, ns, ndir, nz, geom, phi_rule;
  int eblk, blk, nfaces, nch, ce;   // face work items per direction, groups per item
  double lnq, q, fp64_thr;
  double om[4];                     // sum over directions of dOmega and dOmega n (r, theta, phi)
  const double *mu, *Phi, *dOm, *nvec, *G, *eps, *vol;
  const double *vr, *vth, *vph, *alp, *psi;
  const double *qpow;               // q^k for k = -128 .. 128 (index k + 128)
  double iq1;                       // 1/(q - 1)
  const double *cphi, *sphi;        // cos and sin of the Phi nodes
};

struct Frame {
  double v[3];
  double alpha, psi, th, ph;
  double st, ct, sp, cp;       // sin and cos of th and ph
};

// Per-face frame data computed once per background by the table build: the five
// frames (0 Lm, 1 L, 2 R, 3 Rp, 4 interface) with their Lorentz factor and
// psi^6, and the basis changes L -> interface and R -> interface.
struct FaceAux {
  double v[5][3];
  double alpha[5], psi[5], gam[5], p6[5];
  double M[2][9];
};

// Everything the kernels need about one model (a grid with its background,
// state and per-face data), in device memory.  A batch holds one per model; a
// single context holds one.  Work items name (model, face) or (model, zone).
struct ModelDev {
  DevGrid g;
  const FaceDesc *faces;
  const btx::ZoneFaces *zf;
  char *tabs;                  // remap tables of every face
  FaceAux *aux;                // frame data of every face
  void *f[2];                  // state double buffer (storage precision)
  const void *ka, *ks, *feq;   // [zone][species][group] (storage precision)
  void *dN;                    // [face][side][species][group][direction]
  double *tally;               // [face][species] cumulative content through ghost faces
  double *q;                   // [zone][5] hydro source terms of the last step
  const unsigned char *zlev;   // [zone] time level (local time stepping), or null
  double dt;                   // step of the current launch
};

__device__ inline double dsq(double x) { return x * x; }

// Pointers read from a descriptor in memory are generic; these all point to
// device global memory, and saying so lets the compiler use global (not flat)
// loads and stores, which do not hold up the LDS wait counter.
template <typename P>
__device__ __forceinline__ P *as_global(P *p)
{
  return (P *)((__attribute__((address_space(1))) P *)(uintptr_t)p);
}

// a descriptor's grid with its pointers marked global
__device__ __forceinline__ DevGrid global_grid(const DevGrid &src)
{
  DevGrid g = src;
  g.mu = as_global(g.mu); g.Phi = as_global(g.Phi); g.dOm = as_global(g.dOm);
  g.nvec = as_global(g.nvec); g.G = as_global(g.G); g.eps = as_global(g.eps);
  g.vol = as_global(g.vol); g.vr = as_global(g.vr); g.vth = as_global(g.vth);
  g.vph = as_global(g.vph);
  g.alp = as_global(g.alp); g.psi = as_global(g.psi);
  g.qpow = as_global(g.qpow); g.cphi = as_global(g.cphi); g.sphi = as_global(g.sphi);
  return g;
}

__device__ Frame side_frame(const DevGrid &g, const SideDesc &s)
{
  Frame f;
  int z = s.z;
  f.v[0] = g.vr[z];
  f.v[1] = g.vth[z];
  f.v[2] = g.vph[z];
  if (s.kind == btx::SIDE_MIRROR) f.v[0] = -f.v[0];
  f.alpha = g.alp[z];
  f.psi = g.psi[z];
  f.th = s.th;
  f.ph = s.ph;
  f.st = s.sth; f.ct = s.cth; f.sp = s.sph; f.cp = s.cph;
  return f;
}

__device__ inline bool same_frame(const Frame &a, const Frame &b)
{
  return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2] && a.alpha == b.alpha &&
         a.psi == b.psi && a.th == b.th && a.ph == b.ph;
}

// orthonormal basis (e_r, e_theta, e_phi) at (theta, phi) as columns, from
// the sines and cosines of the two angles
__device__ void basis_cols(double st, double ct, double sp, double cp, double B[3][3])
{
  B[0][0] = st * cp; B[1][0] = st * sp; B[2][0] = ct;
  B[0][1] = ct * cp; B[1][1] = ct * sp; B[2][1] = -st;
  B[0][2] = -sp;     B[1][2] = cp;      B[2][2] = 0.0;
}

// x given in frame a's basis -> components in the basis at the angles
// (tb, pb), whose sines and cosines are given
__device__ void change_basis(const Frame &a, double tb, double pb, double stb, double ctb, double spb,
                             double cpb, const double x[3], double y[3])
{
  if (a.th == tb && a.ph == pb) { y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; return; }
  double A[3][3], B[3][3], c[3];
  basis_cols(a.st, a.ct, a.sp, a.cp, A);
  basis_cols(stb, ctb, spb, cpb, B);
  for (int r = 0; r < 3; ++r) c[r] = A[r][0] * x[0] + A[r][1] * x[1] + A[r][2] * x[2];
  for (int r = 0; r < 3; ++r) y[r] = B[0][r] * c[0] + B[1][r] * c[1] + B[2][r] * c[2];
}

// psi^6 by products (the remap kernels' frame weights)
__device__ inline double pow6(double x)
{
  const double x2 = x * x;
  return x2 * x2 * x2;
}

// A frame with what the chain needs of it evaluated once per frame rather
// than once per direction: the Lorentz-factor terms of its velocity and its
// orthonormal basis.
struct FrameP {
  Frame f;
  double gam, kv;              // 1/sqrt(1 - v^2), gam^2/(gam + 1)
  double ia, ip2;              // 1/alpha, 1/psi^2
  double B[3][3];              // basis_cols at (th, ph)
};

__device__ inline FrameP prep_frame(const Frame &f)
{
  FrameP p;
  p.f = f;
  const double v2 = f.v[0] * f.v[0] + f.v[1] * f.v[1] + f.v[2] * f.v[2];
  p.gam = 1.0 / sqrt(1.0 - v2);
  p.kv = p.gam * p.gam / (p.gam + 1.0);
  p.ia = 1.0 / f.alpha;
  p.ip2 = 1.0 / (f.psi * f.psi);
  basis_cols(f.st, f.ct, f.sp, f.cp, p.B);
  return p;
}

// Lorentz boost by the frame's fluid velocity v (sgn -1: by -v) (paper
// Sec. 3.2.2), with gam and kv of the frame
__device__ inline void lorentz_p(const FrameP &F, double sgn, const double u[4], double o[4])
{
  const double v[3] = { sgn * F.f.v[0], sgn * F.f.v[1], sgn * F.f.v[2] };
  const double vu = v[0] * u[1] + v[1] * u[2] + v[2] * u[3];
  const double a = F.kv * vu + F.gam * u[0];
  o[0] = F.gam * (u[0] + vu);
  o[1] = u[1] + a * v[0];
  o[2] = u[2] + a * v[1];
  o[3] = u[3] + a * v[2];
}

// comoving(S) -> comoving(D) through Eulerian and coordinate frames, the
// Hamiltonian kick on the axis of motion and the geometric rotation
// (Eq. transformchain, Sec. 3.2.1-3.2.4; conformally flat, zero shift).
// axis < 0: the remap forward in time at a fixed place, where the covariant
// spatial momentum is kept and the covariant energy follows from the null
// condition of the new metric.
__device__ void frame_chain_p(const FrameP &SP, const FrameP &DP, int axis, bool rot, const double u[4], double o[4])
{
  const Frame &S = SP.f, &D = DP.f;
  double e[4];
  lorentz_p(SP, 1.0, u, e);
  double u0 = -S.alpha * e[0];                       // covariant time component
  double p2 = S.psi * S.psi;
  double uc[3] = { p2 * e[1], p2 * e[2], p2 * e[3] };  // covariant spatial components
  if (axis < 0 && (S.alpha != D.alpha || S.psi != D.psi)) {
    u0 = -D.alpha * sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]) * DP.ip2;
  } else if (S.alpha != D.alpha || S.psi != D.psi) {
    double tr = 0.0;
    for (int i = 0; i < 3; ++i) if (i != axis) tr += uc[i] * uc[i];
    double dp2 = D.psi * D.psi;
    double rad = dp2 * dp2 * u0 * u0 * (DP.ia * DP.ia) - tr;
    if (rad >= 0.0) {
      uc[axis] = copysign(sqrt(rad), uc[axis] >= 0.0 ? 1.0 : -1.0);
    } else {                                          // no real root: reflect along the axis
      double sc = dp2 * fabs(u0) / D.alpha / sqrt(tr);
      uc[axis] = 0.0;
      for (int i = 0; i < 3; ++i) if (i != axis) uc[i] *= sc;
    }
  }
  double ud[3];
  if (rot && !(S.th == D.th && S.ph == D.ph)) {        // change of basis, as change_basis
    double c[3];
    for (int r = 0; r < 3; ++r) c[r] = SP.B[r][0] * uc[0] + SP.B[r][1] * uc[1] + SP.B[r][2] * uc[2];
    for (int r = 0; r < 3; ++r) ud[r] = DP.B[0][r] * c[0] + DP.B[1][r] * c[1] + DP.B[2][r] * c[2];
  } else {
    ud[0] = uc[0]; ud[1] = uc[1]; ud[2] = uc[2];
  }
  double eD[4] = { -u0 * DP.ia, ud[0] * DP.ip2, ud[1] * DP.ip2, ud[2] * DP.ip2 };
  lorentz_p(DP, -1.0, eD, o);
}

__device__ inline double u0_dir(const Frame &f, const double *n)
{
  double v2 = f.v[0] * f.v[0] + f.v[1] * f.v[1] + f.v[2] * f.v[2];
  double gam = 1.0 / sqrt(1.0 - v2);
  return gam * (1.0 + f.v[0] * n[0] + f.v[1] * n[1] + f.v[2] * n[2]);
}

// ------------------------------------------------------------ LDS tables

// A remap T_{S->D} of one face in gather form.  For every target direction d'
// the entries [start[d'], start[d'+1]) hold the two energy-tap weights
// (cl, cr) and a 16-bit key: on a logarithmic energy grid one shift di serves
// every group, and source group i of direction src sends cl to group i + di and
// cr to group i + di + 1.  Keys are first built as src | (di + 128) << 8 and
// sorted; when every shift of the table is within one group (flag bit 0 of
// start[nd + 1] clear) they are then replaced by the source window offset
// src * cs - di + 2 in the direction-major data buffers.  Tables act on number
// content; occupations are turned into content before (x G_i a(d)) and back
// after (/ (G_i a(d'))) by the caller.
template <typename T>
struct Tab {
  const T *cw;                   // 2 x 4 nd tap weights (cl, cr)
  const unsigned short *key;     // 4 nd
  const unsigned short *start;   // nd + 2
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t tab_stride(int nd, size_t szT)
{
  return align16(8 * (size_t)nd * szT + (5 * (size_t)nd + 2) * 2);
}

template <typename T>
__device__ inline Tab<T> tab_at(const char *base, int nd)
{
  Tab<T> t;
  t.cw = (const T *)base;
  t.key = (const unsigned short *)(t.cw + 8 * nd);
  t.start = t.key + 4 * nd;
  return t;
}

// Work items of the face kernel: nch (a power of two) per target direction,
// each owning CE consecutive rows (energy groups).  The nch * CE rows of a
// direction end at group ne + 1, so that the rows ne and ne + 1, which collect
// the content an upward shift pushes past the top group, share a work item
// with group ne - 1, and they start at or below group -1.

// Data buffers in LDS are direction-major: column d holds the rows
// ne - nch CE .. ne + 2 contiguously; rows outside 0 .. ne-1 are zero.  The
// stride nch CE + 3 is odd, so neighbouring lanes reading different columns
// hit distinct banks.
__host__ __device__ inline int col_rows(int nch, int ce) { return nch * ce + 3; }

__host__ __device__ inline size_t buf_bytes(int nd, int nch, int ce, size_t szT)
{
  return align16((size_t)nd * col_rows(nch, ce) * szT);
}

// scratch of table_kernel_g for tpr tables at a time: counts and cursors per
// target, four records per source (target and shift; tap weights), the
// records' indexes in target order and their keys
__host__ __device__ inline size_t scratch_bytes(int nd, size_t szT, int tpr)
{
  return (size_t)tpr * nd * 4 * 2 + (size_t)4 * tpr * nd * 4 + (size_t)8 * tpr * nd * szT +
         (size_t)4 * tpr * nd * 4 + (size_t)4 * tpr * nd * 2;
}

// 16-bit gather keys before their conversion to window offsets: the source
// direction and the energy shift.  Up to 256 directions they take 8 bits
// each; up to 1024 directions the source takes 10 bits and the shift 6, which
// is exact there: such grids have at most 29 groups, and a shift that takes
// every group past the edge of the grid folds like one just past it.
__host__ __device__ inline unsigned short pack_key(int src, int di, int nd)
{
  if (nd > 256) {
    di = di < -31 ? -31 : (di > 31 ? 31 : di);
    return (unsigned short)(src | ((di + 32) << 10));
  }
  return (unsigned short)(src | ((di + 128) << 8));
}

__host__ __device__ inline void unpack_key(unsigned key, int nd, int &src, int &di)
{
  if (nd > 256) { src = key & 0x3ff; di = (int)(key >> 10) - 32; }
  else { src = key & 0xff; di = (int)(key >> 8) - 128; }
}

// LDS of one face workgroup: 8 tables, 3 data buffers (Lm, then Rp; L; R), per-row
// constants (G, 1/G as T; per species: source and blend weight as T, two
// collision coefficients as FP64, a precision flag), the wave partials and
// totals of the angle sums, and the tally partials
__host__ __device__ inline size_t face_lds_bytes(int nd, int ns, int nch, int ce, size_t szT, bool gtab = false)
{
  const size_t nrow = col_rows(nch, ce), nsr = (size_t)ns * nrow;
  return (gtab ? 0 : kTables * tab_stride(nd, szT)) + 3 * buf_bytes(nd, nch, ce, szT) + 2 * align16(nrow * szT) +
         2 * align16(nsr * szT) + 2 * align16(nsr * 8) + align16(nsr * 4) + align16(16 * nrow * 8) +
         align16(nrow * 8) + align16(16 * 8);
}

// ascending node bracket with edge clamping (all weight to the edge node)
__device__ inline void node_bracket(const double *x, int n, double v, int &L, int &R, double &wR)
{
  if (n == 1 || v <= x[0]) { L = R = 0; wR = 0.0; return; }
  if (v >= x[n - 1]) { L = R = n - 1; wR = 0.0; return; }
  int l = 0;
  while (x[l + 1] <= v) ++l;
  L = l;
  R = l + 1;
  wR = (v - x[l]) / (x[l + 1] - x[l]);
}

// One source direction of one remap: frame chain, energy shift and taps,
// (mu, Phi) corners.  rt[4] receive the targets (-1 unused), rl/rr the tap
// weights times the corner weight.
// mu: the mu nodes (the grid's, or a copy of them in LDS)
__device__ __forceinline__ void remap_source(const DevGrid &g, const double *mu, const FrameP &S, const FrameP &D, int axis,
                             bool rot, bool ident, int d, int rt[4], double rl[4], double rr[4], int &di_out)
{
  const double *n = g.nvec + 3 * d;
  rt[1] = rt[2] = rt[3] = -1;
  rl[1] = rl[2] = rl[3] = rr[1] = rr[2] = rr[3] = 0.0;
  if (ident) {
    di_out = 0;
    rt[0] = d; rl[0] = 1.0; rr[0] = 0.0;
    return;
  }
  double u[4] = { 1.0, n[0], n[1], n[2] }, o[4];
  frame_chain_p(S, D, axis, rot, u, o);
  // energy: eps* = rho eps_i; on logarithmic groups one shift di serves every
  // i: q^di <= rho < q^(di+1), estimated in FP32 and settled on the table of
  // powers of q
  const double rho = o[0];
  int di = (int)floorf(__logf((float)rho) / (float)g.lnq);
  di = max(-127, min(127, di));
  while (di > -127 && rho < g.qpow[di + 128]) --di;
  while (di < 127 && rho >= g.qpow[di + 129]) ++di;
  double we = (rho * g.qpow[128 - di] - 1.0) * g.iq1;
  we = fmin(1.0, fmax(0.0, we));
  di_out = di;
  // direction
  double mus = fmin(1.0, fmax(-1.0, o[1] / rho));
  int jL, jR;
  double wj;
  node_bracket(mu, g.nmu, mus, jL, jR, wj);
  int kL, kR;
  double wk;
  if (g.nphi == 1) { kL = kR = 0; wk = 0.0; }
  else {
    const double dP = 2.0 * kPi / g.nphi;
    int kl;
    if (o[2] * o[2] + o[3] * o[3] <= 1e-12 * o[0] * o[0]) {
      kl = d % g.nphi;                              // on the mu = +-1 axis: keep the Phi label
      wk = 0.0;
    } else if (g.phi_rule == 0) {
      // direction-preserving split between the nodes P_L <= P < P_R (Phi
      // nodes (k + 1/2) dP): sin(P - P_L) / (sin(P_R - P) + sin(P - P_L)),
      // from the unit vector (cos P, sin P) and the nodes' cos and sin.  The
      // bracket is estimated in FP32 and settled by the signs of the sines; a
      // sine within rounding of zero (a direction on a node, where the split
      // is 0 or 1 either way) settles it too, so that it cannot flip between
      // the two brackets that share the node.
      const double irp = 1.0 / sqrt(o[2] * o[2] + o[3] * o[3]);
      const double c = o[2] * irp, sn = o[3] * irp;
      float Pf = atan2f((float)o[3], (float)o[2]);
      if (Pf < 0.0f) Pf += 2.0f * (float)kPi;
      kl = (int)floorf(Pf / (float)dP - 0.5f);
      double a = 0.0, b = 0.0;
      for (int it = 0; it < 4; ++it) {
        const int l = ((kl % g.nphi) + g.nphi) % g.nphi, r = (((kl + 1) % g.nphi) + g.nphi) % g.nphi;
        b = sn * g.cphi[l] - c * g.sphi[l];          // sin(P - P_L)
        a = g.sphi[r] * c - g.cphi[r] * sn;          // sin(P_R - P)
        if (it == 3) break;                          // (unreachable: the estimate is off by < 1 bin)
        if (b < -1e-12) --kl;
        else if (a < -1e-12) ++kl;
        else break;
      }
      wk = fmin(1.0, fmax(0.0, b / (a + b)));
    } else {
      double P = atan2(o[3], o[2]);
      if (P < 0.0) P += 2.0 * kPi;
      kl = (int)floor(P / dP - 0.5);
      wk = (P - (kl + 0.5) * dP) / dP;
    }
    kL = ((kl % g.nphi) + g.nphi) % g.nphi;
    kR = (((kl + 1) % g.nphi) + g.nphi) % g.nphi;
  }
  // coinciding brackets (clamped or a single Phi bin) are merged so that the
  // four records of a source have distinct targets
  const bool oneJ = jL == jR, oneK = kL == kR;
  const double wj0 = oneJ ? 1.0 : 1.0 - wj, wj1 = oneJ ? 0.0 : wj;
  const double wk0 = oneK ? 1.0 : 1.0 - wk, wk1 = oneK ? 0.0 : wk;
  const double c[4] = { wj0 * wk0, wj0 * wk1, wj1 * wk0, wj1 * wk1 };
  const int tg[4] = { jL * g.nphi + kL, jL * g.nphi + kR, jR * g.nphi + kL, jR * g.nphi + kR };
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    // corner weights at rounding level (a direction that lands on a node up
    // to the last bit) are dropped: they move less than 1e-15 of a bin
    rt[r] = c[r] > 1e-15 ? tg[r] : -1;
    rl[r] = c[r] * (1.0 - we);
    rr[r] = c[r] * we;
  }
}

// Gather of one remap for target direction dp over the rows r0 .. r0+CE-1 of
// a work item.  X points at group 0 of column 0 of a direction-major buffer
// (column stride cs, zero outside groups 0 .. ne-1).  Content that the energy
// shift pushes below group 0 or above group ne-1 stays in that group: for
// shifts of at most one group it lands on row -1 (kb: its position in this
// item, folded into group 0; with SPLIT, row -1 ends the previous item,
// the neighbouring lane, and is carried over) or on rows ne, ne+1 (the last
// two rows of the top item, folded into group ne-1); tables with larger
// shifts take the explicit path.  Called by all lanes of a wave together.
template <typename T, int CE, bool SPLIT>
__device__ __forceinline__ void gather(const Tab<T> &tb, int nd, const T *__restrict__ X, int cs, int ne,
                                       int dp, int r0, bool top, int kb, T acc[CE])
{
#pragma unroll
  for (int k = 0; k < CE; ++k) acc[k] = (T)0;
  const int e0 = tb.start[dp], e1 = tb.start[dp + 1];
  if ((tb.start[nd + 1] & 1) == 0) {
    const T *base = X + (r0 - 3);
#pragma unroll 2
    for (int e = e0; e < e1; ++e) {
      const T *w = base + tb.key[e];                 // window of rows r0-di-1 .. r0-di+CE-1
      const T cl = tb.cw[2 * e], cr = tb.cw[2 * e + 1];
      T x[CE + 1];
#pragma unroll
      for (int k = 0; k <= CE; ++k) x[k] = w[k];
#pragma unroll
      for (int k = 0; k < CE; ++k) acc[k] = fma(cl, x[k + 1], fma(cr, x[k], acc[k]));
    }
    if (top) acc[CE - 3] += acc[CE - 2] + acc[CE - 1];
#pragma unroll
    for (int k = 0; k + 1 < CE; ++k) acc[k + 1] += k == kb ? acc[k] : (T)0;
  } else {
    for (int e = e0; e < e1; ++e) {
      int d, di;
      unpack_key(tb.key[e], nd, d, di);
      const T cl = tb.cw[2 * e], cr = tb.cw[2 * e + 1];
      const T *col = X + d * cs;
#pragma unroll
      for (int k = 0; k < CE; ++k) {
        const int i = r0 + k;
        if (i < 0 || i >= ne) continue;
        const int iL = i - di, iR = iL - 1;
        T v = (T)0;
        if (iL >= 0 && iL < ne) v += cl * col[iL];
        if (iR >= 0 && iR < ne) v += cr * col[iR];
        if (i == 0) {                                   // sent below group 0
          for (int j = 0; j < ne && j + di < 0; ++j) v += cl * col[j];
          for (int j = 0; j < ne && j + di + 1 < 0; ++j) v += cr * col[j];
        }
        if (i == ne - 1) {                              // sent above group ne-1
          for (int j = max(0, ne - di); j < ne; ++j) v += cl * col[j];
          for (int j = max(0, ne - 1 - di); j < ne; ++j) v += cr * col[j];
        }
        acc[k] += v;
      }
    }
  }
  if constexpr (SPLIT) {
    const T carry = __shfl_up(acc[CE - 1], 1, 64);
    if (r0 == 0) acc[0] += carry;
  }
}

// MC limiter minmod(2 dm, 2 dp, (dm + dp)/2): the argument closest to zero
// when all three have the same strict sign, else zero (branch-free form)
template <typename T>
__device__ inline T mc_limiter(T dm, T dp)
{
  const T a = (T)2 * dm, b = (T)2 * dp, m = (T)0.5 * (dm + dp);
  const T lo = fmin(a, fmin(b, m)), hi = fmax(a, fmax(b, m));
  return lo > (T)0 ? lo : (hi < (T)0 ? hi : (T)0);
}

__device__ inline double wave_sum(double v)
{
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// three wave sums with their shuffles interleaved
__device__ inline void wave_sum3(double &a, double &b, double &c)
{
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(a, o, 64), y = __shfl_xor(b, o, 64), w = __shfl_xor(c, o, 64);
    a += x;
    b += y;
    c += w;
  }
}

// frame weight psi^6 u0 dOmega of direction d in frame k of a face
__device__ inline double frame_weight(const DevGrid &g, const FaceAux &A, int k, int d)
{
  const double *nv = g.nvec + 3 * d;
  double vdn = A.v[k][0] * nv[0] + A.v[k][1] * nv[1] + A.v[k][2] * nv[2];
  return A.p6[k] * A.gam[k] * (1.0 + vdn) * g.dOm[d];
}

// ------------------------------------------------------------ table kernel

// frames of table t (0 Lm->L, 1 R->L, 2 L->R, 3 Rp->R, 4 L->s, 5 R->s, 6 s->L,
// 7 s->R) among 0 Lm, 1 L, 2 R, 3 Rp, 4 the interface s
__device__ inline int tab_src(int t) { return t == 0 ? 0 : (t == 1 || t == 5) ? 2 : (t == 2 || t == 4) ? 1 : t == 3 ? 3 : 4; }
__device__ inline int tab_dst(int t) { return (t == 0 || t == 1 || t == 6) ? 1 : (t == 2 || t == 3 || t == 7) ? 2 : 4; }

// The five frames of a face (0 Lm, 1 L, 2 R, 3 Rp, 4 the interface), one per
// lane k < 5, with what the chain needs of each evaluated once.
__device__ __forceinline__ void face_frames(const DevGrid &g, const FaceDesc &F, FrameP *frm, int k)
{
  if (k >= 5) return;
  const Frame a = side_frame(g, F.L), b = side_frame(g, F.R);
  Frame fr;
  if (k == 0) fr = side_frame(g, F.Lm);
  else if (k == 1) fr = a;
  else if (k == 2) fr = b;
  else if (k == 3) fr = side_frame(g, F.Rp);
  else {
    double vl[3], vr[3];
    change_basis(a, F.ths, F.phs, F.sts, F.cts, F.sps, F.cps, a.v, vl);
    change_basis(b, F.ths, F.phs, F.sts, F.cts, F.sps, F.cps, b.v, vr);
    for (int i = 0; i < 3; ++i) fr.v[i] = 0.5 * (vl[i] + vr[i]);
    fr.alpha = 0.5 * (a.alpha + b.alpha);
    fr.psi = 0.5 * (a.psi + b.psi);
    fr.th = F.ths;
    fr.ph = F.phs;
    fr.st = F.sts; fr.ct = F.cts; fr.sp = F.sps; fr.cp = F.cps;
  }
  frm[k] = prep_frame(fr);
}

// The face's frame data from its five frames: lane k < 5 writes frame k,
// lanes 5 .. 10 one column each of the basis changes L -> interface and
// R -> interface.
__device__ __forceinline__ void face_aux(const FrameP *frm, bool rot, FaceAux &A, int k)
{
  if (k < 5) {
    const FrameP &fr = frm[k];
    for (int i = 0; i < 3; ++i) A.v[k][i] = fr.f.v[i];
    A.alpha[k] = fr.f.alpha;
    A.psi[k] = fr.f.psi;
    A.gam[k] = fr.gam;
    A.p6[k] = pow6(fr.f.psi);
  } else if (k < 11) {
    const int side = (k - 5) / 3, c = (k - 5) % 3;
    const FrameP &fr = frm[1 + side], &fs = frm[4];
    const bool same = !rot || (fr.f.th == fs.f.th && fr.f.ph == fs.f.ph);
    for (int r = 0; r < 3; ++r)
      A.M[side][3 * r + c] = same ? (r == c ? 1.0 : 0.0)
                                  : fs.B[0][r] * fr.B[0][c] + fs.B[1][r] * fr.B[1][c] + fs.B[2][r] * fr.B[2][c];
  }
}

// Builds the eight remap tables of one face (frame chain once per direction,
// inverted into sorted per-target gather lists) in place in global memory,
// one table at a time with the whole workgroup: the build for grids whose
// face kernels read their tables through the caches (large momentum grids,
// where one wave's scratch per table would not fit).  Run once per
// background; table_kernel_w (below) builds the same tables elsewhere.
// table t: 0 Lm->L, 1 R->L, 2 L->R, 3 Rp->R, 4 L->s, 5 R->s, 6 s->L, 7 s->R
template <typename T>
__global__ void __launch_bounds__(512)
table_kernel_g(const ModelDev *__restrict__ models, const int2 *__restrict__ items)
{
  constexpr int TPR = 1;                            // tables per round
  extern __shared__ __align__(16) char lds[];
  __shared__ int flg[kTables];
  const int2 it = items[blockIdx.x];
  const ModelDev &M = models[it.x];
  const DevGrid g = global_grid(M.g);
  char *__restrict__ tabs_g = as_global(M.tabs);
  FaceAux *__restrict__ aux = as_global(M.aux);
  const int fid = it.y;
  const FaceDesc &F = as_global(M.faces)[fid];
  const int nd = g.ndir, tid = threadIdx.x, nthr = blockDim.x;
  const size_t tstride = tab_stride(nd, sizeof(T));
  char *p = lds;
  char *tabs = tabs_g + (size_t)fid * kTables * tstride;
  FrameP *frm = (FrameP *)p;   p += align16(5 * sizeof(FrameP));
  char *data = p;
  int *cnt = (int *)data;                      // TPR nd
  int *cur = cnt + TPR * nd;                   // TPR nd
  int *rtg = cur + TPR * nd;                   // 4 TPR nd
  T *rcf = (T *)(rtg + 4 * TPR * nd);          // 8 TPR nd
  int *idx = (int *)(rcf + 8 * TPR * nd);      // 4 TPR nd
  unsigned short *skey = (unsigned short *)(idx + 4 * TPR * nd);  // 4 TPR nd: key of each placed record
  // the mu nodes, the powers of q and the cos and sin of the Phi nodes,
  // looked up (each lookup depending on the last) for every direction of
  // every table: copies in LDS
  double *smu = (double *)(data + align16(scratch_bytes(nd, sizeof(T), TPR)));
  double *sqp = (double *)((char *)smu + align16((size_t)g.nmu * 8));
  double *scp = (double *)((char *)sqp + align16((size_t)kQpow * 8)), *ssp = scp + g.nphi;
  for (int q = tid; q < g.nmu; q += nthr) smu[q] = g.mu[q];
  for (int q = tid; q < kQpow; q += nthr) sqp[q] = g.qpow[q];
  for (int q = tid; q < g.nphi; q += nthr) { scp[q] = g.cphi[q]; ssp[q] = g.sphi[q]; }
  DevGrid gs = g;
  gs.qpow = sqp; gs.cphi = scp; gs.sphi = ssp;
  const int cs = col_rows(g.nch, g.ce);
  auto tw = [&](int t, T *&cw, unsigned short *&key, unsigned short *&start) {
    char *b = tabs + t * tstride;
    cw = (T *)b;
    key = (unsigned short *)(cw + 8 * nd);
    start = key + 4 * nd;
  };
  if (tid < kTables) flg[tid] = 0;
  face_frames(g, F, frm, tid);
  const bool rot = g.geom != 2;
  const int ax = F.axis;
  for (int round = 0; round < kTables / TPR; ++round) {
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) cnt[q] = 0;
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) {
      int tl = q / nd, d = q - tl * nd, t = TPR * round + tl;
      const FrameP &S = frm[tab_src(t)], &D = frm[tab_dst(t)];
      int rt[4], di;
      double rl[4], rr[4];
      remap_source(gs, smu, S, D, ax, rot, same_frame(S.f, D.f), d, rt, rl, rr, di);
      if (di < -1 || di > 1) atomicOr(&flg[t], 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rtg[q * 4 + r] = rt[r] >= 0 ? (rt[r] | ((di + 128) << 16)) : -1;
        rcf[(q * 4 + r) * 2] = (T)rl[r];
        rcf[(q * 4 + r) * 2 + 1] = (T)rr[r];
        if (rt[r] >= 0) atomicAdd(&cnt[tl * nd + rt[r]], 1);
      }
    }
    __syncthreads();
    if ((tid >> 6) < TPR) {                            // exclusive scan per table, one wave each
      // lane l takes the K consecutive targets from l K: its own sum, one
      // wave scan of the lane sums, then its targets' starts in turn
      const int tl = tid >> 6, ln = tid & 63, K = (nd + 63) >> 6, d0 = ln * K;
      T *cw;
      unsigned short *key, *start;
      tw(TPR * round + tl, cw, key, start);
      const int *ct = cnt + tl * nd;
      int loc = 0;
      for (int j = 0; j < K; ++j)
        if (d0 + j < nd) loc += ct[d0 + j];
      int incl = loc;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (ln >= o) incl += y;
      }
      int run = incl - loc;
      for (int j = 0; j < K; ++j) {
        const int d = d0 + j;
        if (d < nd) {
          start[d] = (unsigned short)run;
          cur[tl * nd + d] = run;
          run += ct[d];
        }
      }
      const int total = __shfl(incl, 63, 64);
      if (ln == 0) {
        start[nd] = (unsigned short)total;
        start[nd + 1] = (unsigned short)flg[TPR * round + tl];
      }
    }
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) {       // record indexes into their target lists
      const int tl = q / nd;
      for (int r = 0; r < 4; ++r) {
        const int v = rtg[q * 4 + r];
        if (v < 0) continue;
        const int sl = tl * 4 * nd + atomicAdd(&cur[tl * nd + (v & 0xffff)], 1);
        idx[sl] = q * 4 + r;
        skey[sl] = pack_key(q - tl * nd, (v >> 16) - 128, nd);
      }
    }
    __syncthreads();
    // Each record takes the place of its rank by key within its target's list
    // (keys are distinct there: a source sends at most one record to a
    // target), which fixes the summation order whatever order the lists were
    // filled in; with shifts within one group the key becomes the source
    // window offset.
    for (int x = tid; x < TPR * 4 * nd; x += nthr) {
      const int tl = x / (4 * nd), sl = x - tl * 4 * nd;
      T *cw;
      unsigned short *key, *start;
      tw(TPR * round + tl, cw, key, start);
      if (sl >= start[nd]) continue;
      const int rec = idx[x], v = rtg[rec];
      const int tg = v & 0xffff, a = start[tg], b = start[tg + 1];
      const unsigned kx = skey[x];
      const unsigned short *lk = skey + tl * 4 * nd;
      int rank = 0;
      for (int y = a; y < b; ++y) rank += lk[y] < kx;
      const int slot = a + rank;
      key[slot] = (start[nd + 1] & 1) ? (unsigned short)kx
                                      : (unsigned short)((rec / 4 - tl * nd) * cs - ((v >> 16) - 128) + 2);
      cw[2 * slot] = rcf[rec * 2];
      cw[2 * slot + 1] = rcf[rec * 2 + 1];
    }
  }
  __syncthreads();

  // the face's frame data, one lane per frame and one per basis column
  face_aux(frm, rot, aux[fid], tid);
}

// LDS of one wave of table_kernel_w: the counts (then cursors) per target,
// four records per source (target and shift; tap weights) and the records'
// keys in target order
__host__ __device__ inline size_t wave_scratch_bytes(int nd, size_t szT)
{
  return align16((size_t)nd * 4) + align16((size_t)16 * nd) + align16((size_t)8 * nd * szT) +
         align16((size_t)8 * nd);
}

// LDS of a table_kernel_w workgroup: the five frames, the mu nodes, the
// powers of q, the cos and sin of the Phi nodes and one scratch per table
__host__ __device__ inline size_t table_w_lds_bytes(int nd, int nmu, int nphi, size_t szT, size_t frames)
{
  return align16(frames) + align16((size_t)nmu * 8) + align16((size_t)kQpow * 8) + align16((size_t)2 * nphi * 8) +
         kTables * wave_scratch_bytes(nd, szT);
}

__device__ __forceinline__ void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same tables as table_kernel_g (the same records, keys and order within
// each target's list), built by one wave per table: after the frames, the
// eight waves of the workgroup go through the chains, the scan, the list
// placement and the ranking of their own table with no workgroup barrier,
// and write the table in place in global memory.  (Barrier-separated rounds
// of four tables kept every wave of the face waiting for the slowest at each
// of a dozen phases, most of them short and bound by latency.)
// FP32: held to 80 registers, so that three workgroups share a CU (their LDS
// allows three at 96 directions): 17.4 -> 15.2 ms at 600 x 256 zones with 14
// registers spilled.  FP64 scratch allows two, which 4 waves per SIMD give.
template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 4)))
table_kernel_w(const ModelDev *__restrict__ models, const int2 *__restrict__ items)
{
  extern __shared__ __align__(16) char lds[];
  const int2 it = items[blockIdx.x];
  const ModelDev &M = models[it.x];
  const DevGrid g = global_grid(M.g);
  const int fid = it.y;
  const FaceDesc &F = as_global(M.faces)[fid];
  const int nd = g.ndir, tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, t = tid >> 6;
  const size_t tstride = tab_stride(nd, sizeof(T));
  char *p = lds;
  FrameP *frm = (FrameP *)p;        p += align16(5 * sizeof(FrameP));
  double *smu = (double *)p;        p += align16((size_t)g.nmu * 8);
  double *sqp = (double *)p;        p += align16((size_t)kQpow * 8);
  double *scp = (double *)p, *ssp = scp + g.nphi;  p += align16((size_t)2 * g.nphi * 8);
  char *ws = p + (size_t)t * wave_scratch_bytes(nd, sizeof(T));
  int *cur = (int *)ws;                                                      // nd
  int *rtg = (int *)(ws + align16((size_t)nd * 4));                          // 4 nd
  T *rcf = (T *)((char *)rtg + align16((size_t)16 * nd));                    // 8 nd
  unsigned short *skey = (unsigned short *)((char *)rcf + align16((size_t)8 * nd * sizeof(T)));  // 4 nd
  for (int q = tid; q < g.nmu; q += nthr) smu[q] = g.mu[q];
  for (int q = tid; q < kQpow; q += nthr) sqp[q] = g.qpow[q];
  for (int q = tid; q < g.nphi; q += nthr) { scp[q] = g.cphi[q]; ssp[q] = g.sphi[q]; }
  DevGrid gs = g;
  gs.qpow = sqp; gs.cphi = scp; gs.sphi = ssp;
  face_frames(g, F, frm, tid);
  for (int q = lane; q < nd; q += 64) cur[q] = 0;
  __syncthreads();                                   // frames and lookup copies ready
  if (t >= kTables) return;
  const bool rot = g.geom != 2;
  const FrameP &S = frm[tab_src(t)], &D = frm[tab_dst(t)];
  const bool ident = same_frame(S.f, D.f);
  // chains: four records per source, counted per target
  int big = 0;
  for (int q = lane; q < nd; q += 64) {
    int rt[4], di;
    double rl[4], rr[4];
    remap_source(gs, smu, S, D, F.axis, rot, ident, q, rt, rl, rr, di);
    big |= di < -1 || di > 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rtg[q * 4 + r] = rt[r] >= 0 ? (rt[r] | ((di + 128) << 16)) : -1;
      rcf[(q * 4 + r) * 2] = (T)rl[r];
      rcf[(q * 4 + r) * 2 + 1] = (T)rr[r];
      if (rt[r] >= 0) atomicAdd(&cur[rt[r]], 1);
    }
  }
  const bool large = __any(big) != 0;                // some shift beyond one group
  wave_sync();
  char *tab = as_global(M.tabs) + ((size_t)fid * kTables + t) * tstride;
  T *cw = (T *)tab;
  unsigned short *key = (unsigned short *)(cw + 8 * nd);
  unsigned short *start = key + 4 * nd;
  {
    // exclusive scan of the counts: lane l takes the K consecutive targets
    // from l K; the starts go out, the cursors take the counts' place
    const int K = (nd + 63) >> 6, d0 = lane * K;
    int loc = 0;
    for (int j = 0; j < K; ++j)
      if (d0 + j < nd) loc += cur[d0 + j];
    int incl = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    int run = incl - loc;
    for (int j = 0; j < K; ++j) {
      const int d = d0 + j;
      if (d < nd) {
        const int c = cur[d];
        start[d] = (unsigned short)run;
        cur[d] = run;
        run += c;
      }
    }
    const int total = __shfl(incl, 63, 64);
    if (lane == 0) {
      start[nd] = (unsigned short)total;
      start[nd + 1] = (unsigned short)(large ? 1 : 0);
    }
  }
  wave_sync();
  for (int q = lane; q < nd; q += 64)                // keys into their target lists, in any order
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = rtg[q * 4 + r];
      if (v < 0) continue;
      skey[atomicAdd(&cur[v & 0xffff], 1)] = pack_key(q, (v >> 16) - 128, nd);
    }
  wave_sync();
  // Each record at the place of its rank by key within its target's list,
  // as in table_kernel_g.  Target tg's cursor now marks the end of its list
  // and tg - 1's its start.
  const int cs = col_rows(g.nch, g.ce);
  for (int q = lane; q < nd; q += 64)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = rtg[q * 4 + r];
      if (v < 0) continue;
      const int tg = v & 0xffff, di = (v >> 16) - 128;
      const int a = tg > 0 ? cur[tg - 1] : 0, b = cur[tg];
      const unsigned kx = pack_key(q, di, nd);
      int rank = 0;
      for (int y = a; y < b; ++y) rank += skey[y] < kx;
      const int slot = a + rank;
      key[slot] = large ? (unsigned short)kx : (unsigned short)(q * cs - di + 2);
      cw[2 * slot] = rcf[(q * 4 + r) * 2];
      cw[2 * slot + 1] = rcf[(q * 4 + r) * 2 + 1];
    }
  if (t == 0) face_aux(frm, rot, as_global(M.aux)[fid], lane);
}

// ------------------------------------------------------------ time remap

// LDS of the time-remap workgroup: one remap table under construction and in
// gather form, the frame weights of both frames and one species block
__host__ __device__ inline size_t time_lds_bytes(int nd, int ne, size_t szT)
{
  return align16((size_t)nd * 4) * 2 + align16((size_t)16 * nd) + align16((size_t)8 * nd * szT) * 2 +
         align16((size_t)4 * nd * 2) + align16((size_t)(nd + 1) * 2) + align16((size_t)nd * 8) * 2 +
         align16((size_t)nd * ne * szT) + align16((size_t)16 * nd);
}

// Remaps every species block of one zone from its comoving frame under the
// current background to its comoving frame under a new one: the remap forward
// in time of Sec. 3.2 (the closing T_{n->n+1} of a step, Sec. 3.3), at a fixed
// place, so without rotation and with the time kick of frame_chain_p.  The
// zone's gather table is built in LDS and applied in place to the number
// content (W = psi^6 u0 G dOmega; the cell volume is unchanged).
// nbg: the new background of the model, [5][zone] = v_r, v_theta, v_phi, alpha, psi.
// Held to 64 registers in FP32 (8 waves per SIMD, 32 spilled) and 80 in
// FP64 (6, what its LDS allows): the build is latency-bound, and at 600 x 256
// zones, 96 directions, the FP32 kernel takes 5.5 ms against 7.4 ms at its
// natural 109 registers (4 waves per SIMD).
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 6)))
time_remap_kernel(const ModelDev *__restrict__ models, const int2 *__restrict__ items, int parity,
                  const double *__restrict__ nbg)
{
  extern __shared__ __align__(16) char lds[];
  const int2 it = items[blockIdx.x];
  const ModelDev &M = models[it.x];
  const DevGrid g = global_grid(M.g);
  T *__restrict__ f = as_global((T *)M.f[parity]);
  const int z = it.y, nd = g.ndir, ne = g.ne, tid = threadIdx.x, nthr = blockDim.x;
  Frame S;
  S.v[0] = g.vr[z]; S.v[1] = g.vth[z]; S.v[2] = g.vph[z];
  S.alpha = g.alp[z]; S.psi = g.psi[z];
  S.th = 0.0; S.ph = 0.0;
  S.st = 0.0; S.ct = 1.0; S.sp = 0.0; S.cp = 1.0;
  Frame D = S;
  const double *nb = as_global(nbg);
  D.v[0] = nb[z]; D.v[1] = nb[g.nz + z]; D.v[2] = nb[2 * g.nz + z];
  D.alpha = nb[3 * g.nz + z]; D.psi = nb[4 * g.nz + z];
  if (same_frame(S, D)) return;                          // the whole workgroup leaves
  const FrameP SP = prep_frame(S), DP = prep_frame(D);
  char *p = lds;
  int *cnt = (int *)p;                 p += align16((size_t)nd * 4);
  int *cur = (int *)p;                 p += align16((size_t)nd * 4);
  int *rtg = (int *)p;                 p += align16((size_t)16 * nd);
  T *rcf = (T *)p;                     p += align16((size_t)8 * nd * sizeof(T));
  T *cw = (T *)p;                      p += align16((size_t)8 * nd * sizeof(T));
  unsigned short *key = (unsigned short *)p;  p += align16((size_t)4 * nd * 2);
  unsigned short *start = (unsigned short *)p; p += align16((size_t)(nd + 1) * 2);
  double *aS = (double *)p;            p += align16((size_t)nd * 8);
  double *aD = (double *)p;            p += align16((size_t)nd * 8);
  T *cont = (T *)p;                    p += align16((size_t)nd * ne * sizeof(T));
  int *idx = (int *)p;                 // record indexes in target order
  const double gS = 1.0 / sqrt(1.0 - (S.v[0] * S.v[0] + S.v[1] * S.v[1] + S.v[2] * S.v[2]));
  const double gD = 1.0 / sqrt(1.0 - (D.v[0] * D.v[0] + D.v[1] * D.v[1] + D.v[2] * D.v[2]));
  const double p6S = pow6(S.psi), p6D = pow6(D.psi);
  for (int q = tid; q < nd; q += nthr) {
    cnt[q] = 0;
    const double *nv = g.nvec + 3 * q;
    aS[q] = p6S * gS * (1.0 + S.v[0] * nv[0] + S.v[1] * nv[1] + S.v[2] * nv[2]) * g.dOm[q];
    aD[q] = p6D * gD * (1.0 + D.v[0] * nv[0] + D.v[1] * nv[1] + D.v[2] * nv[2]) * g.dOm[q];
  }
  __syncthreads();
  for (int q = tid; q < nd; q += nthr) {               // each source direction
    int rt[4], di;
    double rl[4], rr[4];
    remap_source(g, g.mu, SP, DP, -1, false, false, q, rt, rl, rr, di);
    for (int r = 0; r < 4; ++r) {
      rtg[q * 4 + r] = rt[r] >= 0 ? (rt[r] | ((di + 128) << 16)) : -1;
      rcf[(q * 4 + r) * 2] = (T)rl[r];
      rcf[(q * 4 + r) * 2 + 1] = (T)rr[r];
      if (rt[r] >= 0) atomicAdd(&cnt[rt[r]], 1);
    }
  }
  __syncthreads();
  if (tid < 64) {                                      // list starts per target: wave scan
    int base = 0;
    for (int d0 = 0; d0 < nd; d0 += 64) {
      const int d = d0 + tid;
      const int c = d < nd ? cnt[d] : 0;
      int incl = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (tid >= o) incl += y;
      }
      if (d < nd) {
        start[d] = (unsigned short)(base + incl - c);
        cur[d] = base + incl - c;
      }
      base += __shfl(incl, 63, 64);
    }
    if (tid == 0) start[nd] = (unsigned short)base;
  }
  __syncthreads();
  for (int q = tid; q < nd; q += nthr)
    for (int r = 0; r < 4; ++r) {
      const int v = rtg[q * 4 + r];
      if (v >= 0) idx[atomicAdd(&cur[v & 0xffff], 1)] = q * 4 + r;
    }
  __syncthreads();
  // each record at the place of its rank by key in its target's list (a
  // fixed summation order, whatever order the lists were filled in)
  for (int x = tid; x < start[nd]; x += nthr) {
    const int rec = idx[x], v = rtg[rec];
    const int tg = v & 0xffff, a = start[tg], b = start[tg + 1];
    const unsigned kx = pack_key(rec / 4, (v >> 16) - 128, nd);
    int rank = 0;
    for (int y = a; y < b; ++y) rank += pack_key(idx[y] / 4, (rtg[idx[y]] >> 16) - 128, nd) < kx;
    key[a + rank] = (unsigned short)kx;
    cw[2 * (a + rank)] = rcf[rec * 2];
    cw[2 * (a + rank) + 1] = rcf[rec * 2 + 1];
  }
  __syncthreads();
  for (int s = 0; s < g.ns; ++s) {
    T *blk = f + (size_t)z * g.blk + (size_t)s * g.eblk;
    for (int q = tid; q < ne * nd; q += nthr) {          // content, direction-major
      const int i = q / nd, d = q - i * nd;
      cont[d * ne + i] = (T)((double)blk[q] * g.G[i] * aS[d]);
    }
    __syncthreads();
    for (int q = tid; q < ne * nd; q += nthr) {
      const int i = q / nd, dp = q - i * nd;
      T acc = (T)0;
      for (int e = start[dp]; e < start[dp + 1]; ++e) {
        int src, di;
        unpack_key(key[e], nd, src, di);
        const T cl = cw[2 * e], cr = cw[2 * e + 1];
        const T *col = cont + src * ne;
        const int iL = i - di, iR = iL - 1;
        if (iL >= 0 && iL < ne) acc += cl * col[iL];
        if (iR >= 0 && iR < ne) acc += cr * col[iR];
        if (i == 0) {                                     // sent below group 0
          for (int j = 0; j < ne && j + di < 0; ++j) acc += cl * col[j];
          for (int j = 0; j < ne && j + di + 1 < 0; ++j) acc += cr * col[j];
        }
        if (i == ne - 1) {                                // sent above group ne-1
          for (int j = max(0, ne - di); j < ne; ++j) acc += cl * col[j];
          for (int j = max(0, ne - 1 - di); j < ne; ++j) acc += cr * col[j];
        }
      }
      blk[q] = (T)((double)acc / (g.G[i] * aD[dp]));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ face kernel

// one side's species-s values of a work item's load rows (li, li + NCH, ...)
template <typename T, int NCH, int CE>
__device__ __forceinline__ void fetch_side(const DevGrid &g, const SideDesc &sd, const T *__restrict__ f,
                                           const T *__restrict__ feq, int s, int li, int ld, T v[CE])
{
  const int nd = g.ndir, ne = g.ne;
  // one load site per row (a zone's block, or the equilibrium of a ghost), so
  // that the loads of all rows and sides are in flight together
  const bool data = sd.kind == btx::SIDE_ZONE || sd.kind == btx::SIDE_MIRROR;
  const bool any = data || sd.kind == btx::SIDE_EQ;
  const T *base = data ? f + (size_t)sd.z * g.blk + (size_t)s * g.eblk + ld : feq + ((size_t)sd.z * g.ns + s) * ne;
  const size_t stride = data ? (size_t)nd : 1;
#pragma unroll
  for (int m = 0; m < CE; ++m) {
    const int i = li + NCH * m;
    T x = (T)0;
    if (any && i < ne) x = base[(size_t)i * stride];
    v[m] = x;
  }
}

template <typename T, int NCH, int CE>
__device__ __forceinline__ void store_side(const T v[CE], const T gl[CE], T a, int col, int li, int ne, int cs,
                                           T *X)
{
#pragma unroll
  for (int m = 0; m < CE; ++m) {
    const int i = li + NCH * m;
    if (i < ne) X[col * cs + i] = v[m] * gl[m] * a;
  }
}

// One workgroup per face, NCH work items per direction.  Per species:
//   load    the four stencil zones' blocks (coalesced rows, transposed into
//           direction-major LDS columns as number content; three buffers,
//           Rp taking Lm's after the slopes of L)
//   phase 1 MC-limited slopes of both sides in their own frames (Sec. 3.3.2)
//           and the reconstructed donor values
//   phase 2 Lax-Wendroff half-step source in the interface frame; angle sums
//           by wave shuffles; implicit interface collision (Eq. halfstep);
//           blend (Sec. 3.3.3) into flux and donor contents
//   phase 3 remapped content change of both sides (Eq. fullstep)
// GTAB: the face's tables are read from global memory (through the caches)
// instead of LDS, for momentum grids whose tables do not fit beside the
// stencil blocks.
template <typename T, int NCH, int CE, int MAXT, bool SPLIT, bool GTAB = false>
__global__ void __launch_bounds__(MAXT)
face_kernel(const ModelDev *__restrict__ models, const int2 *__restrict__ items, int parity, int sub)
{
  extern __shared__ __align__(16) char lds[];
  const int2 it = items[blockIdx.x];
  const ModelDev &M = models[it.x];
  const DevGrid g = global_grid(M.g);
  const char *__restrict__ tabs_g = as_global((const char *)M.tabs);
  const FaceAux *__restrict__ aux = as_global((const FaceAux *)M.aux);
  const T *__restrict__ f = as_global((const T *)M.f[parity]);
  const T *__restrict__ ka = as_global((const T *)M.ka);
  const T *__restrict__ ks = as_global((const T *)M.ks);
  const T *__restrict__ feq = as_global((const T *)M.feq);
  T *__restrict__ dN = as_global((T *)M.dN);
  double *__restrict__ tally = as_global(M.tally);
  const int fid = it.y;
  const FaceDesc &F = as_global(M.faces)[fid];
  // Time levels: the face steps with its finer zone, dt0 2^m; a side whose
  // zone is at a coarser level adds this step's changes to those it already
  // holds, unless its own step starts at this substep.
  int lvL = 0, lvR = 0;
  if (M.zlev) { lvL = as_global(M.zlev)[F.L.z]; lvR = as_global(M.zlev)[F.R.z]; }
  const double dt = M.dt * (double)(1 << min(lvL, lvR));
  const bool accL = (sub & ((1 << lvL) - 1)) != 0, accR = (sub & ((1 << lvR) - 1)) != 0;
  const int nd = g.ndir, ne = g.ne, tid = threadIdx.x, nthr = blockDim.x;
  T *outL = dN + (size_t)fid * 2 * g.blk, *outR = outL + g.blk;
  if (!F.active) {
    for (size_t q = tid; q < (size_t)g.blk; q += nthr) {
      if (!accL) outL[q] = (T)0;
      if (!accR) outR[q] = (T)0;
    }
    return;
  }
  const int nrow = col_rows(NCH, CE), cs = nrow, gb = NCH * CE - ne;
  // ---- LDS carve-up
  const size_t tstride = tab_stride(nd, sizeof(T));
  const size_t bb = buf_bytes(nd, NCH, CE, sizeof(T));
  char *p = lds;
  const char *tabs = GTAB ? tabs_g + (size_t)fid * kTables * tstride : p;
  if (!GTAB) p += kTables * tstride;
  char *bufs = p;               p += 3 * bb;
  T *XLm = (T *)(bufs) + gb, *XL = (T *)(bufs + bb) + gb, *XR = (T *)(bufs + 2 * bb) + gb,
    *XRp = XLm;                   // Rp takes Lm's buffer once the slopes of L are done
  const int nsr = g.ns * nrow;
  T *rG = (T *)p + gb;          p += align16(nrow * sizeof(T));
  T *riG = (T *)p + gb;         p += align16(nrow * sizeof(T));
  T *rsrc0 = (T *)p + gb;       p += align16(nsr * sizeof(T));
  T *rw0 = (T *)p + gb;         p += align16(nsr * sizeof(T));
  double *rc00 = (double *)p + gb;  p += align16(nsr * 8);
  double *rc10 = (double *)p + gb;  p += align16(nsr * 8);
  int *rthick0 = (int *)p + gb; p += align16(nsr * 4);
  double *spart = (double *)p;  p += align16(16 * nrow * 8);
  double *savr = (double *)p + gb;  p += align16(nrow * 8);
  double *tpart = (double *)p;

#define TB(t) tab_at<T>(tabs + (t) * tstride, nd)

  // ---- remap tables of this face (built once per background)
  if (!GTAB) {
    const uint4 *src = (const uint4 *)(tabs_g + (size_t)fid * kTables * tstride);
    uint4 *dst = (uint4 *)lds;
    const int n16 = (int)(kTables * tstride / 16);
    // four loads in flight per thread: indexes past the end are clamped to
    // the last entry (loaded and stored again), so that no load is guarded
    for (int q0 = tid; q0 < n16; q0 += 4 * nthr) {
      uint4 t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] = src[min(q0 + u * nthr, n16 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[min(q0 + u * nthr, n16 - 1)] = t[u];
    }
  }
  // ---- zero rows of the data buffers, per-row constants outside 0 .. ne-1
  {
    const int ng = nrow - ne;
    for (int q = tid; q < 3 * nd * ng; q += nthr) {
      int b = q / (nd * ng), rem = q - b * nd * ng, d = rem / ng, r = rem - d * ng;
      ((T *)(bufs + b * bb))[d * cs + (r < gb ? r : r + ne)] = (T)0;
    }
    for (int q = tid; q < nrow; q += nthr) {
      const int r = q - gb;
      const bool in = r >= 0 && r < ne;
      rG[r] = in ? (T)g.G[r] : (T)0;
      riG[r] = in ? (T)(1.0 / g.G[r]) : (T)0;
    }
  }
  const FaceAux &A = aux[fid];
  const int ax = F.axis;
  const bool slopeL = F.L.slope, slopeR = F.R.slope && !F.self;
  const bool ghost = F.L.kind != btx::SIDE_ZONE || F.R.kind != btx::SIDE_ZONE;
  const double gs = A.gam[4];
  const double ap4 = A.alpha[4] * dsq(A.psi[4] * A.psi[4]);
  const double vn = A.v[4][ax];
  const double Uadv = ap4 * gs * vn;
  const double tau = 0.5 * A.alpha[4] * dt / gs;
  // ---- per (species, group) interface opacities and collision coefficients
  for (int q = tid; q < nsr; q += nthr) {
    const int sp = q / nrow, i = q - sp * nrow - gb;
    double a_ = 0.0, b_ = 0.0, e_ = 0.0;
    const bool in = i >= 0 && i < ne;
    if (in && !F.zero_opacity) {
      size_t l = ((size_t)F.L.z * g.ns + sp) * ne + i, r = ((size_t)F.R.z * g.ns + sp) * ne + i;
      a_ = 0.5 * ((double)ka[l] + (double)ka[r]);
      b_ = 0.5 * ((double)ks[l] + (double)ks[r]);
      e_ = 0.5 * ((double)feq[l] + (double)feq[r]);
    }
    const double den = 1.0 + tau * (a_ + b_);
    const int o = sp * nrow + i;
    rc00[o] = in ? 1.0 / den : 0.0;
    rc10[o] = in ? tau * b_ / (1.0 + tau * a_) / den : 0.0;
    rsrc0[o] = (T)(tau * a_ * e_);
    rw0[o] = in ? (T)exp(-(a_ + b_) * F.h) : (T)0;
    rthick0[o] = sizeof(T) == 8 || tau * (a_ + b_) > g.fp64_thr;
  }

  // ---- load mapping: direction ld, rows li, li + NCH, ...
  const bool ldown = tid < NCH * nd;
  const int ld = ldown ? tid % nd : 0, li = ldown ? tid / nd : ne;
  T gl[CE];
#pragma unroll
  for (int m = 0; m < CE; ++m) {
    const int i = li + NCH * m;
    const double Gi = g.G[min(i, ne - 1)];           // unguarded, so the loads overlap
    gl[m] = i < ne ? (T)Gi : (T)0;
  }
  const SideDesc *sides[4] = { &F.Lm, &F.L, &F.R, &F.Rp };
  int colS[4];
  T aS_[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int col = ld;
    if (sides[k]->kind == btx::SIDE_MIRROR) {
      int j = ld / g.nphi, kk = ld - j * g.nphi;
      col = (g.nmu - 1 - j) * g.nphi + kk;
    }
    colS[k] = col;
    aS_[k] = (T)frame_weight(g, A, k, col);
  }

  // ---- compute mapping: target direction dp, rows r0 .. r0 + CE - 1
  const bool own = tid < NCH * nd;
  const int dp = own ? tid / NCH : 0, ch = tid % NCH;
  const int r0 = ne + 2 - (NCH - ch) * CE;
  const bool top = ch == NCH - 1;
  const int kb = -1 - r0;
  T iaL, iaR, iaS, cv, kF, uLp, uap, uRn, uan;
  double dOd;
  {
    const double *nv = g.nvec + 3 * dp;
    const double dO = g.dOm[dp];
    iaL = (T)(1.0 / frame_weight(g, A, 1, dp));
    iaR = (T)(1.0 / frame_weight(g, A, 2, dp));
    iaS = (T)(1.0 / frame_weight(g, A, 4, dp));
    // interface speeds (flux integral with zero shift) and the donor speeds of
    // both sides (cell-centre direction expressed in the interface basis)
    const double kvs = gs * gs / (gs + 1.0);
    double vdn = A.v[4][0] * nv[0] + A.v[4][1] * nv[1] + A.v[4][2] * nv[2];
    double u0 = gs * (1.0 + vdn);
    double un = nv[ax] + (kvs * vdn + gs) * vn;
    const double Urad = ap4 * (nv[ax] + kvs * vdn * vn);
    const double Vn = A.alpha[4] * un / (A.psi[4] * A.psi[4] * u0);
    double Us[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double *v = A.v[1 + side];
      double gm = A.gam[1 + side], kv = gm * gm / (gm + 1.0);
      double vu = v[0] * nv[0] + v[1] * nv[1] + v[2] * nv[2];
      double a_ = kv * vu + gm;
      double e0 = nv[0] + a_ * v[0], e1 = nv[1] + a_ * v[1], e2 = nv[2] + a_ * v[2];
      const double *M = A.M[side];
      Us[side] = ap4 * (M[3 * ax] * e0 + M[3 * ax + 1] * e1 + M[3 * ax + 2] * e2);
    }
    const double gwd = dO * dt * F.area;
    cv = (T)(-0.5 * dt * Vn / F.h);
    kF = (T)(Urad * gwd);
    uLp = (T)(fmax(Us[0], 0.0) * gwd);
    uRn = (T)(fmax(-Us[1], 0.0) * gwd);
    uap = (T)(fmax(Uadv, 0.0) * gwd);
    uan = (T)(fmax(-Uadv, 0.0) * gwd);
    dOd = own ? dO : 0.0;
  }
  const T dL = (T)F.dL, dR = (T)F.dR, ih = (T)(1.0 / F.h);
  const T ihLm = (T)(1.0 / F.hLm), ihRp = (T)(1.0 / F.hRp);
  const int lane = tid & 63, wave = tid >> 6, nw = (nthr + 63) >> 6;
  // a launch with one workgroup row per species (gridDim.y = ns, for launches
  // with few faces) takes the species of its row; else every species in turn
  const int s_lo = gridDim.y > 1 ? (int)blockIdx.y : 0, s_hi = gridDim.y > 1 ? s_lo + 1 : g.ns;

#pragma unroll 1
  for (int s = s_lo; s < s_hi; ++s) {
    // ---- load the stencil blocks as content densities
    // Rp goes into Lm's buffer after stage 0.  FP32 loads it with the other
    // sides and holds it in registers; FP64, short of registers, loads it then.
    constexpr bool kHoldRp = sizeof(T) == 4;
    T v3[CE];
    {
      T v0[CE], v1[CE], v2[CE];
      if (slopeL) fetch_side<T, NCH, CE>(g, F.Lm, f, feq, s, li, ld, v0);
      fetch_side<T, NCH, CE>(g, F.L, f, feq, s, li, ld, v1);
      fetch_side<T, NCH, CE>(g, F.R, f, feq, s, li, ld, v2);
      if (kHoldRp && slopeR) fetch_side<T, NCH, CE>(g, F.Rp, f, feq, s, li, ld, v3);
      if (slopeL) store_side<T, NCH, CE>(v0, gl, aS_[0], colS[0], li, ne, cs, XLm);
      store_side<T, NCH, CE>(v1, gl, aS_[1], colS[1], li, ne, cs, XL);
      store_side<T, NCH, CE>(v2, gl, aS_[2], colS[2], li, ne, cs, XR);
    }
    const T *rsrc = rsrc0 + s * nrow, *rw = rw0 + s * nrow;
    const double *rc0 = rc00 + s * nrow, *rc1 = rc10 + s * nrow;
    const int *rthick = rthick0 + s * nrow;
    __syncthreads();
    // ---- five remap stages, each the sum of two gathers a = Ta . Xa, b = Tb . Xb
    //   0 slopes of L      T0 . Lm,  T1 . R
    //   1 slopes of R      T2 . L,   T3 . Rp
    //   2 interface        T4 . L,   T5 . R    -> S, <S>, collision, blend
    //   3 content to L     T6 . FL,  T1 . ER
    //   4 content to R     T7 . FL,  T2 . EL
    // (buffers: 0 Lm, Rp after stage 0, FL after stage 2; 1 L (EL content
    // after stage 2); 2 R (ER content after stage 2))
    T EL[CE], ER[CE];
    double sumL = 0.0, sumR = 0.0;
#pragma unroll 1
    for (int st = 0; st < 5; ++st) {
      T a[CE], b[CE];
#pragma unroll
      for (int k = 0; k < CE; ++k) a[k] = b[k] = (T)0;
      const int nj = (st == 0 && !slopeL) || (st == 1 && !slopeR) ? 0 : 2;
#pragma unroll 1
      for (int j = 0; j < nj; ++j) {
        const int t = (int)((0x2716543210ull >> (4 * (2 * st + j))) & 0xf);
        const int x = (int)((0x1020210120ull >> (4 * (2 * st + j))) & 0xf);
        T c[CE];
        gather<T, CE, SPLIT>(TB(t), nd, (const T *)(bufs + x * bb) + gb, cs, ne, dp, r0, top, kb, c);
#pragma unroll
        for (int k = 0; k < CE; ++k) {
          a[k] = j == 0 ? c[k] : a[k];
          b[k] = j == 0 ? b[k] : c[k];
        }
      }
      if (st == 0) {                                   // MC-limited slope of L (Sec. 3.3.2)
#pragma unroll
        for (int k = 0; k < CE; ++k) {
          const int r = r0 + k;
          const T sc = riG[r] * iaL, fl = XL[dp * cs + r] * sc;
          const T sl = slopeL ? mc_limiter<T>((fl - a[k] * sc) * ihLm, (b[k] * sc - fl) * ih) : (T)0;
          EL[k] = fl + dL * sl;
          if (F.self) ER[k] = XR[dp * cs + r] * riG[r] * iaR + dR * sl;
        }
        if (slopeR) {                                  // Rp into Lm's buffer
          if (!kHoldRp) fetch_side<T, NCH, CE>(g, F.Rp, f, feq, s, li, ld, v3);
          __syncthreads();
          store_side<T, NCH, CE>(v3, gl, aS_[3], colS[3], li, ne, cs, XRp);
          __syncthreads();
        }
      } else if (st == 1) {                            // MC-limited slope of R
        if (!F.self) {
#pragma unroll
          for (int k = 0; k < CE; ++k) {
            const int r = r0 + k;
            const T sc = riG[r] * iaR, fr = XR[dp * cs + r] * sc;
            ER[k] = slopeR ? fr + dR * mc_limiter<T>((fr - a[k] * sc) * ih, (b[k] * sc - fr) * ihRp) : fr;
          }
        }
      } else if (st == 2) {
        // Lax-Wendroff half-step source S in the interface frame
        T Sv[CE];
#pragma unroll
        for (int k = 0; k < CE; ++k) {
          const int r = r0 + k;
          const T sc = riG[r] * iaS;
          const T x = a[k] * sc, y = b[k] * sc;
          Sv[k] = (T)0.5 * (x + y) + cv * (y - x) + rsrc[r];
        }
        // angle sums of S per group (FP64): lanes NCH apart share rows
#pragma unroll
        for (int k = 0; k < CE; ++k) {
          double v = (double)Sv[k] * dOd;
#pragma unroll
          for (int o = NCH; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
          if (lane < NCH) spart[wave * nrow + r0 + k + gb] = v;
        }
        __syncthreads();                               // partial sums visible, buffers free
        if (tid < nrow) {                              // totals over the waves, fixed order
          double t = 0.0;
#pragma unroll 4
          for (int w = 0; w < nw; ++w) t += spart[w * nrow + tid];
          savr[tid - gb] = t * (1.0 / (4.0 * kPi));
        }
        __syncthreads();
        // implicit interface collision, blend weights and content fluxes
        if (own) {
#pragma unroll
          for (int k = 0; k < CE; ++k) {
            const int r = r0 + k;
            if (r < 0 || r >= ne) continue;
            const double sav = savr[r];
            T flw;
            if (rthick[r]) flw = (T)((double)Sv[k] * rc0[r] + rc1[r] * sav);
            else flw = (T)((float)Sv[k] * (float)rc0[r] + (float)rc1[r] * (float)sav);
            const T w = rw[r], G = rG[r];
            XLm[dp * cs + r] = ((T)1 - w) * kF * G * flw;
            XL[dp * cs + r] = (w * (uLp - uap) + uap) * G * EL[k];
            XR[dp * cs + r] = (w * (uRn - uan) + uan) * G * ER[k];
          }
        }
        __syncthreads();
      } else {                                         // remapped content changes
        T *o = (st == 3 ? outL : outR) + (size_t)s * g.eblk;
        const T *own_c = st == 3 ? XL : XR;
        const T sg = st == 3 ? (T)-1 : (T)1;
        const bool acc = st == 3 ? accL : accR;
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < CE; ++k) {
          const int r = r0 + k;
          if (!own || r < 0 || r >= ne) continue;
          const T v = sg * a[k] - own_c[dp * cs + r] + b[k];
          o[r * nd + dp] = acc ? o[r * nd + dp] + v : v;
          sum += (double)v;
        }
        if (st == 3) sumL = sum;
        else sumR = sum;
      }
    }
    if (ghost) {
      double v = wave_sum(F.L.kind != btx::SIDE_ZONE ? sumL : sumR);
      if (lane == 0) tpart[wave] = v;
    }
    __syncthreads();                                   // buffers and partials free for the next species
    if (ghost && tid == 0) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += tpart[w];
      tally[(size_t)fid * g.ns + s] += t;
    }
  }
#undef TB
}

// ------------------------------------------------------------ zone kernel

// segmented wave sum over aligned groups of W lanes (W a power of two)
__device__ inline double seg_sum(double v, int W)
{
  for (int o = W >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline void seg_sum3(double &a, double &b, double &c, int W)
{
  for (int o = W >> 1; o > 0; o >>= 1) {
    const double x = __shfl_xor(a, o, 64), y = __shfl_xor(b, o, 64), w = __shfl_xor(c, o, 64);
    a += x;
    b += y;
    c += w;
  }
}

// Lanes per (species, group) row in the zone kernel: the power of two W
// (4 .. 64) with at most R directions per lane that leaves the fewest lanes
// idle (the widest among equals); 64 / W rows then share a wave.
__host__ __device__ inline int zone_row_lanes(int nd, int R)
{
  int W = 64, best = 64 * ((nd + 63) / 64);
  for (int w = 32; w >= 4; w >>= 1) {
    const int k = (nd + w - 1) / w;
    if (k > R) break;
    if (w * k < best) { best = w * k; W = w; }
  }
  return W;
}

// R: directions per lane (64 R directions at most).  W lanes take a row
// (zone_row_lanes), lane j of them the directions j, j + W, ...  A direction's
// loads (the state and the changes from every face side of the zone) all go
// out before the first is used; at 4 waves per SIMD (not 8) the compiler
// keeps them in registers, and the kernel is faster for it.  With 16
// directions per lane (above 256 directions) the register bound is that of 2
// waves per SIMD: at 4 the kernel spilled; it takes about 120 registers.
template <typename T, int R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R > 4 ? 2 : 4)))
zone_kernel(const ModelDev *__restrict__ models, const int2 *__restrict__ items, int parity)
{
  const int2 it = items[blockIdx.x];
  const ModelDev &M = models[it.x];
  const DevGrid g = global_grid(M.g);
  const btx::ZoneFaces *__restrict__ zf = as_global(M.zf);
  const T *__restrict__ f = as_global((const T *)M.f[parity]);
  T *__restrict__ fout = as_global((T *)M.f[parity ^ 1]);
  const T *__restrict__ dN = as_global((const T *)M.dN);
  const T *__restrict__ ka = as_global((const T *)M.ka);
  const T *__restrict__ ks = as_global((const T *)M.ks);
  const T *__restrict__ feq = as_global((const T *)M.feq);
  const int z = it.y;
  const double dt = M.zlev ? M.dt * (double)(1 << as_global(M.zlev)[z]) : M.dt;   // dt0 2^level
  const int nd = g.ndir, ne = g.ne, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int W = zone_row_lanes(nd, R), sh_w = __builtin_ctz(W);
  const int dl = lane & (W - 1);                      // lane within the row's segment
  const int rpw = 64 >> sh_w;                         // rows per wave at once
  const int nwaves = blockDim.x >> 6;
  const int nslots = nwaves * rpw;                    // rows per pass of the workgroup
  const int slot = wave * rpw + (lane >> sh_w);
  const btx::ZoneFaces &L = zf[z];        // uniform: read through the scalar cache
  const int nq = L.n;                     // at most 8 face sides
  const double vr = g.vr[z], vt = g.vth[z], vp = g.vph[z];
  const double gam = 1.0 / sqrt(1.0 - (vr * vr + vt * vt + vp * vp));
  const double p6v = pow(g.psi[z], 6.0) * g.vol[z];
  const double tau = g.alp[z] * dt / gam;
  // per (species, group) row: the sums of S dOmega and S dOmega n (r, theta,
  // phi), for the source terms after the update; then per direction
  // 1 / ((1 + v.n) dOmega), the direction's part of the content weight
  extern __shared__ __align__(16) char lds[];
  // (with dOmega and n of each direction, read for every row)
  double *rs = (double *)lds;
  double *iwd = rs + 5 * (size_t)g.ns * ne;
  double *sdo = iwd + nd;                  // dOmega_d
  double *snv = sdo + nd;                  // n_d, 3 per direction
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    const double *nv = g.nvec + 3 * d;
    const double n0 = nv[0], n1 = nv[1], n2 = nv[2], dO = g.dOm[d];
    iwd[d] = 1.0 / ((1.0 + vr * n0 + vt * n1 + vp * n2) * dO);
    sdo[d] = dO;
    snv[3 * d] = n0; snv[3 * d + 1] = n1; snv[3 * d + 2] = n2;
  }
  __syncthreads();
  // the zone's blocks (its state, its next state and the change of each
  // face side) from uniform bases: a value's place in every one of them is
  // the same 32-bit offset
  const T *__restrict__ fz0 = f + (size_t)z * g.blk;
  T *__restrict__ fo0 = fout + (size_t)z * g.blk;
  const T *__restrict__ dq[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) dq[q] = dN + ((size_t)L.fid[q] * 2 + L.side[q]) * g.blk;
  // a row's opacities are loaded one row ahead, with the previous row's data
  const int nrows = g.ns * ne;
  const size_t kz = (size_t)z * nrows;
  T kan = (T)0, ksn = (T)0, fen = (T)0;
  {
    const int r0 = min(slot, nrows - 1);
    kan = ka[kz + r0]; ksn = ks[kz + r0]; fen = feq[kz + r0];
  }
  // every wave runs the same number of passes (a segment past the last row
  // idles), so that the shuffles of a pass see all the wave's lanes
  const int npass = (nrows + nslots - 1) / nslots;
  for (int pass = 0; pass < npass; ++pass) {
    const int row = pass * nslots + slot;
    const bool live = row < nrows;
    const int rr = live ? row : nrows - 1;
    int s = rr / ne, i = rr - s * ne;
    const double ka_ = (double)kan, ks_ = (double)ksn, fe_ = (double)fen;
    {
      const int nx = min(row + nslots, nrows - 1);
      kan = ka[kz + nx];
      ksn = ks[kz + nx];
      fen = feq[kz + nx];
    }
    bool wide = (sizeof(T) == 8) || tau * (ka_ + ks_) > g.fp64_thr;
    const double ci = 1.0 / (p6v * gam * g.G[i]);      // the row's part of 1/W
    const double src = tau * ka_ * fe_;
    double Sd[R];
    double part = 0.0;
    for (int r = 0; r < R; ++r) {
      int d = dl + W * r;
      Sd[r] = 0.0;
      if (!live || d >= nd) continue;
      const unsigned bo = (unsigned)(s * g.eblk + i * nd + d) * (unsigned)sizeof(T);   // byte offset
      const T fz = *(const T *)((const char *)fz0 + bo);
      T dv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) dv[q] = *(const T *)((const char *)dq[q] + bo);
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) acc += (double)dv[q];
      // content -> occupation: / W, W = psi^6 dV gamma (1 + v.n) G_i dOmega_d
      double S = (double)fz + src + acc * (ci * iwd[d]);
      if (!wide) S = (double)(float)S;
      Sd[r] = S;
      part += S * sdo[d];
    }
    const double ssum = seg_sum(part, W);
    double avg = ssum / (4.0 * kPi);
    // the implicit solve f' = (S + tau ks avg / (1 + tau ka)) / (1 + tau (ka + ks)),
    // its row constants once per row (in FP32 for an optically thin row)
    const double sh = tau * ks_ * avg / (1.0 + tau * ka_), rden = 1.0 / (1.0 + tau * (ka_ + ks_));
    const float tf = (float)tau, af = (float)ka_, bf = (float)ks_;
    const float shf = tf * bf * (float)avg / (1.0f + tf * af), rdenf = 1.0f / (1.0f + tf * (af + bf));
    double pr = 0.0, pt = 0.0, pp = 0.0;
    for (int r = 0; r < R; ++r) {
      int d = dl + W * r;
      if (!live || d >= nd) continue;
      const unsigned bo = (unsigned)(s * g.eblk + i * nd + d) * (unsigned)sizeof(T);
      const double sw = Sd[r] * sdo[d];
      pr += sw * snv[3 * d];
      pt += sw * snv[3 * d + 1];
      pp += sw * snv[3 * d + 2];
      const double out = wide ? (Sd[r] + sh) * rden : (double)(((float)Sd[r] + shf) * rdenf);
      *(T *)((char *)fo0 + bo) = (T)out;
    }
    seg_sum3(pr, pt, pp, W);
    if (live && dl == 0) { rs[5 * row] = ssum; rs[5 * row + 1] = pr; rs[5 * row + 2] = pt; rs[5 * row + 3] = pp; }
  }
  // Hydro source terms (Eq. hydrosource1-3), in FP64, one row per thread:
  // the collision term at the new state (backward Euler) is
  // C_d = ka feq + ks avg' - (ka + ks) f'_d with the new angle average
  // avg' = avg / (1 + tau ka) and f'_d = (S_d + tau ks avg') / (1 + tau (ka + ks)),
  // i.e. C_d = B - K S_d, so its dOmega- and dOmega n-weighted sums need only
  // the row sums of S.  Kept out of the update loop, which is latency bound.
  __syncthreads();
  const int nrow = g.ns * ne;
  for (int row = threadIdx.x; row < nrow; row += blockDim.x) {
    const int s = row / ne, i = row - s * ne;
    const size_t kidx = ((size_t)z * g.ns + s) * ne + i;
    const double ka_ = (double)ka[kidx], ks_ = (double)ks[kidx], fe_ = (double)feq[kidx];
    const double ssum = rs[5 * row], avg1 = ssum / (4.0 * kPi) / (1.0 + tau * ka_);
    const double K = (ka_ + ks_) / (1.0 + tau * (ka_ + ks_));
    const double B = ka_ * fe_ + ks_ * avg1 - K * tau * ks_ * avg1;
    const double cw = B * g.om[0] - K * ssum, cr = B * g.om[1] - K * rs[5 * row + 1];
    const double ct = B * g.om[2] - K * rs[5 * row + 2], cp = B * g.om[3] - K * rs[5 * row + 3];
    const double ge = g.G[i] * g.eps[i], lep = s == 0 ? 1.0 : (s == 1 ? -1.0 : 0.0);
    rs[5 * row] = -lep * g.G[i] * cw;
    rs[5 * row + 1] = -ge * cw;
    rs[5 * row + 2] = -ge * cr;
    rs[5 * row + 3] = -ge * ct;
    rs[5 * row + 4] = -ge * cp;
  }
  __syncthreads();
  // component k is summed over the rows by wave k mod 4 (fixed order:
  // lane-strided, then a wave sum), so the result does not depend on timing
  for (int k = wave; k < 5; k += nwaves) {
    double v = 0.0;
    for (int row = lane; row < nrow; row += 64) v += rs[5 * row + k];
    v = wave_sum(v);
    if (lane == 0) as_global(M.q)[(size_t)z * 5 + k] = v;
  }
}

// Compensated summation (Neumaier's variant of Kahan's): s + c carries the
// sum of the added values with the rounding error of every addition kept in c.
__device__ inline void comp_add(double &s, double &c, double x)
{
  const double t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// per-zone moments in FP64 (paper Sec. 4.1-4.2, without 1/h^3), each a
// compensated sum over the zone's bins (per thread, over the lanes of a wave
// and over the waves in a fixed order):
// zm[z][s][0..4] = N, J, H, K, number flux; ze[z][s] = energy content
template <typename T>
__global__ void __launch_bounds__(256)
moments_kernel(const ModelDev *__restrict__ models, int m, int parity, double *__restrict__ zm,
               double *__restrict__ ze)
{
  const ModelDev &M = models[m];
  const DevGrid g = global_grid(M.g);
  const T *__restrict__ f = as_global((const T *)M.f[parity]);
  const int z = blockIdx.x;
  __shared__ double red[6][16], redc[6][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const double vr = g.vr[z], vt = g.vth[z], vp = g.vph[z];
  const double gam = 1.0 / sqrt(1.0 - (vr * vr + vt * vt + vp * vp));
  const double p6v = pow(g.psi[z], 6.0) * g.vol[z];
  for (int s = 0; s < g.ns; ++s) {
    double m[6] = { 0, 0, 0, 0, 0, 0 }, mc[6] = { 0, 0, 0, 0, 0, 0 };
    for (int q = threadIdx.x; q < g.eblk; q += blockDim.x) {
      int i = q / g.ndir, d = q - i * g.ndir;
      double fv = (double)f[(size_t)z * g.blk + (size_t)s * g.eblk + q];
      const double *nv = g.nvec + 3 * d;
      double dG = g.G[i] * g.dOm[d], mu = nv[0], e = g.eps[i];
      double nn = p6v * gam * (1.0 + vr * nv[0] + vt * nv[1] + vp * nv[2]) * dG * fv;
      comp_add(m[0], mc[0], nn);
      comp_add(m[1], mc[1], fv * e * dG);
      comp_add(m[2], mc[2], fv * mu * e * dG);
      comp_add(m[3], mc[3], fv * mu * mu * e * dG);
      comp_add(m[4], mc[4], fv * mu * dG);
      comp_add(m[5], mc[5], nn * e);
    }
    for (int k = 0; k < 6; ++k) {
      double v = m[k], c = mc[k];
      for (int o = 32; o > 0; o >>= 1) {
        const double vo = __shfl_xor(v, o, 64), co = __shfl_xor(c, o, 64);
        comp_add(v, c, vo);
        c += co;
      }
      if (lane == 0) { red[k][wave] = v; redc[k][wave] = c; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t[6];
      for (int k = 0; k < 6; ++k) {
        double v = 0.0, c = 0.0;
        for (int w = 0; w < nwaves; ++w) {
          comp_add(v, c, red[k][w]);
          c += redc[k][w];
        }
        t[k] = v + c;
      }
      double *o = zm + ((size_t)z * g.ns + s) * 5;
      o[0] = t[0];
      for (int k = 1; k < 5; ++k) o[k] = t[k] / (4.0 * kPi);
      ze[(size_t)z * g.ns + s] = t[5];
    }
    __syncthreads();
  }
}

// Totals of btx_moments_device: block (s, k) sums, for species s, the zone
// numbers (k = 0), the boundary tallies (k = 1) or the zone energies (k = 2)
// as compensated sums in a fixed order (per thread over a stride, over the
// lanes of a wave, over the waves), and writes totals[3 s + k].
__global__ void __launch_bounds__(256)
totals_kernel(const double *__restrict__ zm, const double *__restrict__ ze, const double *__restrict__ tally,
              const int32_t *__restrict__ bface, int nz, int ns, int nb, double *__restrict__ totals)
{
  const int s = blockIdx.x / 3, k = blockIdx.x % 3;
  const int n = k == 1 ? nb : nz;
  __shared__ double red[2][4];
  double v = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = k == 0 ? zm[((size_t)i * ns + s) * 5]
                            : (k == 1 ? tally[(size_t)bface[i] * ns + s] : ze[(size_t)i * ns + s]);
    comp_add(v, c, x);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double vo = __shfl_xor(v, o, 64), co = __shfl_xor(c, o, 64);
    comp_add(v, c, vo);
    c += co;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[0][wave] = v; red[1][wave] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, tc = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      comp_add(t, tc, red[0][w]);
      tc += red[1][w];
    }
    totals[3 * s + k] = t + tc;
  }
}

template <typename T>
__global__ void cast_kernel(const double *__restrict__ src, T *__restrict__ dst, size_t n)
{
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

// Checks a background held in device memory (grid-stride): bit 0 of *err for
// a zone whose |v| >= 1 or whose alpha or psi is not positive and finite, bit
// 1 for an opacity that is negative or not finite or an equilibrium
// occupation that is not finite.  v_phi may be null.
__global__ void __launch_bounds__(256)
bg_check_kernel(const double *__restrict__ vr, const double *__restrict__ vth, const double *__restrict__ vph,
                const double *__restrict__ alp, const double *__restrict__ psi, size_t nz,
                const double *__restrict__ ka, const double *__restrict__ ks, const double *__restrict__ feq,
                size_t nk, int *__restrict__ err)
{
  int bad = 0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t z = (size_t)blockIdx.x * blockDim.x + threadIdx.x; z < nz; z += stride) {
    const double vp = vph ? vph[z] : 0.0;
    const double v2 = vr[z] * vr[z] + vth[z] * vth[z] + vp * vp;
    if (!(v2 < 1.0) || !(alp[z] > 0.0) || !(psi[z] > 0.0) || !isfinite(alp[z]) || !isfinite(psi[z])) bad |= 1;
  }
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += stride)
    if (!(ka[k] >= 0.0) || !(ks[k] >= 0.0) || !isfinite(ka[k]) || !isfinite(ks[k]) || !isfinite(feq[k])) bad |= 2;
  if (bad) atomicOr(err, bad);
}

}  // namespace
