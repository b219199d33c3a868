// libbtx: HIP (gfx950) implementation of one time step of the locally implicit
// Lax-Wendroff discrete-ordinate neutrino transport scheme of Chan & Mueller
// (arXiv:2003.02845), behind the C ABI of include/btx.h.
//
// One step = two kernels:
//   face_kernel   one workgroup per cell face.  Builds the momentum-space remap
//                 tables of the face in LDS (frame chain of Sec. 3.2 evaluated
//                 once per direction, then inverted into per-target gather
//                 lists), then per species: limited slopes of both sides,
//                 Lax-Wendroff interface value with the implicit interface
//                 collision (Eq. halfstep), donor-cell upwind content
//                 (Sec. 3.3.2), smooth flux switching (Sec. 3.3.3) and the
//                 remapped number-content change of both sides (Eq. fullstep).
//   zone_kernel   one workgroup per zone: sums the content changes of its
//                 faces, converts them to occupation and applies the
//                 zone-local closed-form implicit collision solve (Sec. 3.5).
// Precision: T = double (FP64 mode) or float (mixed mode: storage, remap and
// fluxes in FP32; angle sums in FP64; the collision solve of a (zone, species,
// group) in FP64 where dt_c (ka + ks) exceeds the threshold).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/btx.h"
#include "btx_grid.h"

using btx::FaceDesc;
using btx::SideDesc;

namespace {

constexpr int kTables = 8;    // remap tables per face
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_err;

btx_status fail(btx_status s, const std::string &msg)
{
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(BTX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------------ device data

struct DevGrid {
  int nr, nth, ne, nmu, nphi, ns, ndir, nz, geom, phi_rule;
  int eblk, blk, nfaces, nch, ce;   // face work items per direction, groups per item
  double lnq, q, fp64_thr;
  double om[4];                     // sum over directions of dOmega and dOmega n (r, theta, phi)
  const double *mu, *Phi, *dOm, *nvec, *G, *eps, *vol;
  const double *vr, *vth, *vph, *alp, *psi;
};

struct Frame {
  double v[3];
  double alpha, psi, th, ph;
};

// Per-face frame data computed once per background by table_kernel: the five
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
  return f;
}

__device__ inline bool same_frame(const Frame &a, const Frame &b)
{
  return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2] && a.alpha == b.alpha &&
         a.psi == b.psi && a.th == b.th && a.ph == b.ph;
}

// orthonormal basis (e_r, e_theta, e_phi) as columns
__device__ void basis_cols(double th, double ph, double B[3][3])
{
  double st, ct, sp, cp;
  sincos(th, &st, &ct);
  sincos(ph, &sp, &cp);
  B[0][0] = st * cp; B[1][0] = st * sp; B[2][0] = ct;
  B[0][1] = ct * cp; B[1][1] = ct * sp; B[2][1] = -st;
  B[0][2] = -sp;     B[1][2] = cp;      B[2][2] = 0.0;
}

// x given in the basis at (ta, pa) -> components in the basis at (tb, pb)
__device__ void change_basis(double ta, double pa, double tb, double pb, const double x[3], double y[3])
{
  if (ta == tb && pa == pb) { y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; return; }
  double A[3][3], B[3][3], c[3];
  basis_cols(ta, pa, A);
  basis_cols(tb, pb, B);
  for (int r = 0; r < 3; ++r) c[r] = A[r][0] * x[0] + A[r][1] * x[1] + A[r][2] * x[2];
  for (int r = 0; r < 3; ++r) y[r] = B[0][r] * c[0] + B[1][r] * c[1] + B[2][r] * c[2];
}

// Lorentz boost by fluid velocity v (paper Sec. 3.2.2)
__device__ void lorentz(const double v[3], const double u[4], double o[4])
{
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double gam = 1.0 / sqrt(1.0 - v2);
  double kv = gam * gam / (gam + 1.0);
  double vu = v[0] * u[1] + v[1] * u[2] + v[2] * u[3];
  double a = kv * vu + gam * u[0];
  o[0] = gam * (u[0] + vu);
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
__device__ void frame_chain(const Frame &S, const Frame &D, int axis, bool rot, const double u[4], double o[4])
{
  double e[4];
  lorentz(S.v, u, e);
  double u0 = -S.alpha * e[0];                       // covariant time component
  double p2 = S.psi * S.psi;
  double uc[3] = { p2 * e[1], p2 * e[2], p2 * e[3] };  // covariant spatial components
  if (axis < 0 && (S.alpha != D.alpha || S.psi != D.psi)) {
    u0 = -D.alpha * sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]) / (D.psi * D.psi);
  } else if (S.alpha != D.alpha || S.psi != D.psi) {
    double tr = 0.0;
    for (int i = 0; i < 3; ++i) if (i != axis) tr += uc[i] * uc[i];
    double dp2 = D.psi * D.psi;
    double rad = dp2 * dp2 * u0 * u0 / (D.alpha * D.alpha) - tr;
    if (rad >= 0.0) {
      uc[axis] = copysign(sqrt(rad), uc[axis] >= 0.0 ? 1.0 : -1.0);
    } else {                                          // no real root: reflect along the axis
      double sc = dp2 * fabs(u0) / D.alpha / sqrt(tr);
      uc[axis] = 0.0;
      for (int i = 0; i < 3; ++i) if (i != axis) uc[i] *= sc;
    }
  }
  double ud[3];
  if (rot) change_basis(S.th, S.ph, D.th, D.ph, uc, ud);
  else { ud[0] = uc[0]; ud[1] = uc[1]; ud[2] = uc[2]; }
  double dp2 = D.psi * D.psi;
  double eD[4] = { -u0 / D.alpha, ud[0] / dp2, ud[1] / dp2, ud[2] / dp2 };
  double mv[3] = { -D.v[0], -D.v[1], -D.v[2] };
  lorentz(mv, eD, o);
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

// table-build scratch for one round of 4 tables
// table build scratch for tpr tables at a time
__host__ __device__ inline size_t scratch_bytes(int nd, size_t szT, int tpr = 4)
{
  return (size_t)tpr * nd * 4 * 2 + (size_t)4 * tpr * nd * 4 + (size_t)8 * tpr * nd * szT;
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
__device__ void remap_source(const DevGrid &g, const double *mu, const Frame &S, const Frame &D, int axis,
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
  frame_chain(S, D, axis, rot, u, o);
  // energy: eps* = rho eps_i; logarithmic groups -> one shift for every i
  double rho = o[0];
  int di = (int)floor(log(rho) / g.lnq);
  double we = (rho * exp(-di * g.lnq) - 1.0) / (g.q - 1.0);
  we = fmin(1.0, fmax(0.0, we));
  di = max(-127, min(127, di));
  di_out = di;
  // direction
  double mus = fmin(1.0, fmax(-1.0, o[1] / o[0]));
  int jL, jR;
  double wj;
  node_bracket(mu, g.nmu, mus, jL, jR, wj);
  int k0 = d % g.nphi;
  double P;
  if (o[2] * o[2] + o[3] * o[3] <= 1e-12 * o[0] * o[0]) {
    P = g.Phi[k0];                                  // on the mu = +-1 axis: keep the Phi label
  } else {
    P = atan2(o[3], o[2]);
    if (P < 0.0) P += 2.0 * kPi;
  }
  int kL, kR;
  double wk;
  if (g.nphi == 1) { kL = kR = 0; wk = 0.0; }
  else {
    double dP = 2.0 * kPi / g.nphi;
    int kl = (int)floor(P / dP - 0.5);
    double PL = (kl + 0.5) * dP, PR = PL + dP;
    if (g.phi_rule == 0) {
      double a = sin(PR - P), b = sin(P - PL);
      wk = b / (a + b);
    } else {
      wk = (P - PL) / dP;
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

// Builds the eight remap tables of one face (frame chain once per direction,
// inverted into sorted per-target gather lists) and stores them in global
// memory; run once per background.
// table t: 0 Lm->L, 1 R->L, 2 L->R, 3 Rp->R, 4 L->s, 5 R->s, 6 s->L, 7 s->R
// GTAB: the tables are built in place in global memory (grids whose tables do
// not fit in LDS), one table at a time.
template <typename T, bool GTAB>
__global__ void __launch_bounds__(256)
table_kernel(const ModelDev *__restrict__ models, const int2 *__restrict__ items)
{
  constexpr int TPR = GTAB ? 1 : 4;                 // tables per round
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
  char *tabs = GTAB ? tabs_g + (size_t)fid * kTables * tstride : p;
  if (!GTAB) p += kTables * tstride;
  Frame *frm = (Frame *)p;     p += align16(5 * sizeof(Frame));
  char *data = p;
  int *cnt = (int *)data;                      // TPR nd
  int *cur = cnt + TPR * nd;                   // TPR nd
  int *rtg = cur + TPR * nd;                   // 4 TPR nd
  T *rcf = (T *)(rtg + 4 * TPR * nd);          // 8 TPR nd
  // the mu nodes, searched for every direction of every table
  double *smu = (double *)(data + align16(scratch_bytes(nd, sizeof(T), TPR)));
  for (int q = tid; q < g.nmu; q += nthr) smu[q] = g.mu[q];
  const int cs = col_rows(g.nch, g.ce);
  auto tw = [&](int t, T *&cw, unsigned short *&key, unsigned short *&start) {
    char *b = tabs + t * tstride;
    cw = (T *)b;
    key = (unsigned short *)(cw + 8 * nd);
    start = key + 4 * nd;
  };
  if (tid < kTables) flg[tid] = 0;
  if (tid == 0) {
    Frame a = side_frame(g, F.L), b = side_frame(g, F.R);
    frm[0] = side_frame(g, F.Lm);
    frm[1] = a;
    frm[2] = b;
    frm[3] = side_frame(g, F.Rp);
    Frame fs_;
    double vl[3], vr[3];
    change_basis(a.th, a.ph, F.ths, F.phs, a.v, vl);
    change_basis(b.th, b.ph, F.ths, F.phs, b.v, vr);
    for (int i = 0; i < 3; ++i) fs_.v[i] = 0.5 * (vl[i] + vr[i]);
    fs_.alpha = 0.5 * (a.alpha + b.alpha);
    fs_.psi = 0.5 * (a.psi + b.psi);
    fs_.th = F.ths;
    fs_.ph = F.phs;
    frm[4] = fs_;
  }
  const bool rot = g.geom != 2;
  const int ax = F.axis;
  for (int round = 0; round < kTables / TPR; ++round) {
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) cnt[q] = 0;
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) {
      int tl = q / nd, d = q - tl * nd, t = TPR * round + tl;
      const Frame S = frm[tab_src(t)], D = frm[tab_dst(t)];
      int rt[4], di;
      double rl[4], rr[4];
      remap_source(g, smu, S, D, ax, rot, same_frame(S, D), d, rt, rl, rr, di);
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
      const int tl = tid >> 6, ln = tid & 63;
      T *cw;
      unsigned short *key, *start;
      tw(TPR * round + tl, cw, key, start);
      int base = 0;
      for (int d0 = 0; d0 < nd; d0 += 64) {
        const int d = d0 + ln;
        const int c = d < nd ? cnt[tl * nd + d] : 0;
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o, 64);
          if (ln >= o) incl += y;
        }
        if (d < nd) {
          start[d] = (unsigned short)(base + incl - c);
          cur[tl * nd + d] = base + incl - c;
        }
        base += __shfl(incl, 63, 64);
      }
      if (ln == 0) {
        start[nd] = (unsigned short)base;
        start[nd + 1] = (unsigned short)flg[TPR * round + tl];
      }
    }
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) {       // records into their target lists
      int tl = q / nd, d = q - tl * nd;
      T *cw;
      unsigned short *key, *start;
      tw(TPR * round + tl, cw, key, start);
      for (int r = 0; r < 4; ++r) {
        int v = rtg[q * 4 + r];
        if (v < 0) continue;
        int tg = v & 0xffff, dib = v >> 16;
        int slot = atomicAdd(&cur[tl * nd + tg], 1);
        key[slot] = pack_key(d, dib - 128, nd);
        cw[2 * slot] = rcf[(q * 4 + r) * 2];
        cw[2 * slot + 1] = rcf[(q * 4 + r) * 2 + 1];
      }
    }
    __syncthreads();
    for (int q = tid; q < TPR * nd; q += nthr) {       // fixed summation order: sort by key
      int tl = q / nd, d = q - tl * nd;
      T *cw;
      unsigned short *key, *start;
      tw(TPR * round + tl, cw, key, start);
      int a = start[d], b = start[d + 1];
      for (int x = a + 1; x < b; ++x) {
        unsigned short kx = key[x];
        T c0 = cw[2 * x], c1 = cw[2 * x + 1];
        int y = x - 1;
        while (y >= a && key[y] > kx) {
          key[y + 1] = key[y];
          cw[2 * y + 2] = cw[2 * y];
          cw[2 * y + 3] = cw[2 * y + 1];
          --y;
        }
        key[y + 1] = kx;
        cw[2 * y + 2] = c0;
        cw[2 * y + 3] = c1;
      }
      // shifts within one group: keys become source window offsets
      if (!(start[nd + 1] & 1))
        for (int x = a; x < b; ++x) {
          int src, di;
          unpack_key(key[x], nd, src, di);
          key[x] = (unsigned short)(src * cs - di + 2);
        }
    }
  }
  __syncthreads();

  if (tid == 0) {
    FaceAux A;
    for (int k = 0; k < 5; ++k) {
      const Frame &fr = frm[k];
      for (int i = 0; i < 3; ++i) A.v[k][i] = fr.v[i];
      A.alpha[k] = fr.alpha;
      A.psi[k] = fr.psi;
      A.gam[k] = 1.0 / sqrt(1.0 - (fr.v[0] * fr.v[0] + fr.v[1] * fr.v[1] + fr.v[2] * fr.v[2]));
      A.p6[k] = pow(fr.psi, 6.0);
    }
    for (int side = 0; side < 2; ++side) {
      const Frame &fr = frm[1 + side];
      for (int c = 0; c < 3; ++c) {
        double e[3] = { c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0 }, y[3];
        if (rot) change_basis(fr.th, fr.ph, F.ths, F.phs, e, y);
        else { y[0] = e[0]; y[1] = e[1]; y[2] = e[2]; }
        for (int r = 0; r < 3; ++r) A.M[side][3 * r + c] = y[r];
      }
    }
    aux[fid] = A;
  }
  __syncthreads();
  if (!GTAB) {
    uint4 *dst = (uint4 *)(tabs_g + (size_t)fid * kTables * tstride);
    const uint4 *src = (const uint4 *)tabs;
    const int n16 = (int)(kTables * tstride / 16);
    for (int q = tid; q < n16; q += nthr) dst[q] = src[q];
  }
}

// ------------------------------------------------------------ time remap

// LDS of the time-remap workgroup: one remap table under construction and in
// gather form, the frame weights of both frames and one species block
__host__ __device__ inline size_t time_lds_bytes(int nd, int ne, size_t szT)
{
  return align16((size_t)nd * 4) * 2 + align16((size_t)16 * nd) + align16((size_t)8 * nd * szT) * 2 +
         align16((size_t)4 * nd * 2) + align16((size_t)(nd + 1) * 2) + align16((size_t)nd * 8) * 2 +
         align16((size_t)nd * ne * szT);
}

// Remaps every species block of one zone from its comoving frame under the
// current background to its comoving frame under a new one: the remap forward
// in time of Sec. 3.2 (the closing T_{n->n+1} of a step, Sec. 3.3), at a fixed
// place, so without rotation and with the time kick of frame_chain.  The
// zone's gather table is built in LDS and applied in place to the number
// content (W = psi^6 u0 G dOmega; the cell volume is unchanged).
// nbg: the new background of the model, [5][zone] = v_r, v_theta, v_phi, alpha, psi.
template <typename T>
__global__ void __launch_bounds__(256)
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
  Frame D = S;
  const double *nb = as_global(nbg);
  D.v[0] = nb[z]; D.v[1] = nb[g.nz + z]; D.v[2] = nb[2 * g.nz + z];
  D.alpha = nb[3 * g.nz + z]; D.psi = nb[4 * g.nz + z];
  if (same_frame(S, D)) return;                          // the whole workgroup leaves
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
  T *cont = (T *)p;
  const double gS = 1.0 / sqrt(1.0 - (S.v[0] * S.v[0] + S.v[1] * S.v[1] + S.v[2] * S.v[2]));
  const double gD = 1.0 / sqrt(1.0 - (D.v[0] * D.v[0] + D.v[1] * D.v[1] + D.v[2] * D.v[2]));
  const double p6S = pow(S.psi, 6.0), p6D = pow(D.psi, 6.0);
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
    remap_source(g, g.mu, S, D, -1, false, false, q, rt, rl, rr, di);
    for (int r = 0; r < 4; ++r) {
      rtg[q * 4 + r] = rt[r] >= 0 ? (rt[r] | ((di + 128) << 16)) : -1;
      rcf[(q * 4 + r) * 2] = (T)rl[r];
      rcf[(q * 4 + r) * 2 + 1] = (T)rr[r];
      if (rt[r] >= 0) atomicAdd(&cnt[rt[r]], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {                                       // list starts per target
    int acc = 0;
    for (int d = 0; d < nd; ++d) { start[d] = (unsigned short)acc; cur[d] = acc; acc += cnt[d]; }
    start[nd] = (unsigned short)acc;
  }
  __syncthreads();
  for (int q = tid; q < nd; q += nthr)
    for (int r = 0; r < 4; ++r) {
      const int v = rtg[q * 4 + r];
      if (v < 0) continue;
      const int slot = atomicAdd(&cur[v & 0xffff], 1);
      key[slot] = pack_key(q, (v >> 16) - 128, nd);
      cw[2 * slot] = rcf[(q * 4 + r) * 2];
      cw[2 * slot + 1] = rcf[(q * 4 + r) * 2 + 1];
    }
  __syncthreads();
  for (int q = tid; q < nd; q += nthr) {               // fixed summation order: sort by key
    const int a = start[q], b = start[q + 1];
    for (int x = a + 1; x < b; ++x) {
      const unsigned short kx = key[x];
      const T c0 = cw[2 * x], c1 = cw[2 * x + 1];
      int y = x - 1;
      while (y >= a && key[y] > kx) {
        key[y + 1] = key[y];
        cw[2 * y + 2] = cw[2 * y];
        cw[2 * y + 3] = cw[2 * y + 1];
        --y;
      }
      key[y + 1] = kx;
      cw[2 * y + 2] = c0;
      cw[2 * y + 3] = c1;
    }
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

  // ---- remap tables of this face (built once per background by table_kernel)
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

// R: directions per lane (64 R directions at most).  A direction's loads (the
// state and the changes from every face side of the zone) all go out before
// the first is used; at 4 waves per SIMD (not 8) the compiler keeps them in
// registers, and the kernel is faster for it.  With 16 directions per lane
// (above 256 directions) the register bound is that of 2 waves per SIMD: at
// 4 the kernel spilled; it takes about 120 registers.
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
  const int nwaves = blockDim.x >> 6;
  const btx::ZoneFaces &L = zf[z];        // uniform: read through the scalar cache
  const int nq = L.n;                     // at most 8 face sides
  const double vr = g.vr[z], vt = g.vth[z], vp = g.vph[z];
  const double gam = 1.0 / sqrt(1.0 - (vr * vr + vt * vt + vp * vp));
  const double p6v = pow(g.psi[z], 6.0) * g.vol[z];
  const double tau = g.alp[z] * dt / gam;
  // per (species, group) row: the sums of S dOmega and S dOmega n (r, theta,
  // phi), for the source terms after the update
  extern __shared__ __align__(16) char lds[];
  double *rs = (double *)lds;
  // a row's opacities are loaded one row ahead, with the previous row's data
  const int nrows = g.ns * ne;
  const size_t kz = (size_t)z * nrows;
  T kan = (T)0, ksn = (T)0, fen = (T)0;
  if (wave < nrows) { kan = ka[kz + wave]; ksn = ks[kz + wave]; fen = feq[kz + wave]; }
  for (int row = wave; row < nrows; row += nwaves) {
    int s = row / ne, i = row - s * ne;
    const double ka_ = (double)kan, ks_ = (double)ksn, fe_ = (double)fen;
    {
      const int nx = min(row + nwaves, nrows - 1);
      kan = ka[kz + nx];
      ksn = ks[kz + nx];
      fen = feq[kz + nx];
    }
    bool wide = (sizeof(T) == 8) || tau * (ka_ + ks_) > g.fp64_thr;
    double Sd[R];
    double part = 0.0;
    for (int r = 0; r < R; ++r) {
      int d = lane + 64 * r;
      Sd[r] = 0.0;
      if (d >= nd) continue;
      size_t off = (size_t)s * g.eblk + (size_t)i * nd + d;
      const T fz = f[(size_t)z * g.blk + off];
      T dv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) dv[q] = dN[((size_t)L.fid[q] * 2 + L.side[q]) * g.blk + off];
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) acc += (double)dv[q];
      const double *nv = g.nvec + 3 * d;
      double W = p6v * gam * (1.0 + vr * nv[0] + vt * nv[1] + vp * nv[2]) * g.G[i] * g.dOm[d];
      double S = (double)fz + tau * ka_ * fe_ + acc / W;
      if (!wide) S = (double)(float)S;
      Sd[r] = S;
      part += S * g.dOm[d];
    }
    const double ssum = wave_sum(part);
    double avg = ssum / (4.0 * kPi);
    double pr = 0.0, pt = 0.0, pp = 0.0;
    for (int r = 0; r < R; ++r) {
      int d = lane + 64 * r;
      if (d >= nd) continue;
      size_t off = (size_t)s * g.eblk + (size_t)i * nd + d;
      const double sw = Sd[r] * g.dOm[d];
      pr += sw * g.nvec[3 * d];
      pt += sw * g.nvec[3 * d + 1];
      pp += sw * g.nvec[3 * d + 2];
      double out;
      if (wide) out = (Sd[r] + tau * ks_ * avg / (1.0 + tau * ka_)) / (1.0 + tau * (ka_ + ks_));
      else {
        float t = (float)tau, a = (float)ka_, b = (float)ks_;
        out = ((float)Sd[r] + t * b * (float)avg / (1.0f + t * a)) / (1.0f + t * (a + b));
      }
      fout[(size_t)z * g.blk + off] = (T)out;
    }
    wave_sum3(pr, pt, pp);
    if (lane == 0) { rs[5 * row] = ssum; rs[5 * row + 1] = pr; rs[5 * row + 2] = pt; rs[5 * row + 3] = pp; }
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

// Scratch of btx_moments_device (the entry point for callers that cannot
// allocate): the energy content of every (zone, species) pair, followed by
// room for the zone moments when the caller passes no buffer for them.  It is
// one array per GPU, alive until the process ends, and shared by every call on
// that GPU; every value a call reads is written earlier in the same call, so
// nothing needs clearing, and calls that overlap on one GPU race.  Host code
// never passes the array's name to a kernel: it passes the device address
// that scratch_base() resolves once per device.
constexpr size_t kScratchPairs = (size_t)1 << 19;   // (zone, species) pairs
static __device__ __align__(256) double scratch[kScratchPairs * 6];   // 24 MiB

template <typename T>
__global__ void cast_kernel(const double *__restrict__ src, T *__restrict__ dst, size_t n)
{
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

}  // namespace

// ---------------------------------------------------------------- host side

namespace {

// face workgroups that fill the device, one per CU (256 compute units)
constexpr int kFillFaces = 256;

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

constexpr int kCE8[] = { 3, 4, 5, 6, 8 };
constexpr int kCE4[] = { 4, 5, 6, 7, 8, 12, 16 };

FaceShape make_shape(int prec, int nd, int ne, int nch)
{
  FaceShape f;
  if (nd > 128 || (nch != 4 && nch != 8) || (prec == BTX_PREC_FP64 && nch == 8 && nd > 96)) return f;
  f.nch = nch;
  f.maxt = nch == 4 ? 512 : (nd <= 96 ? 768 : 1024);
  const int *c = nch == 8 ? kCE8 : kCE4;
  const int n = nch == 8 ? 5 : 7;
  for (int k = 0; k < n && !f.ce; ++k)
    if (nch * c[k] >= ne + 3) f.ce = c[k];
  f.split = f.ce && (ne + 2) % f.ce == 0;
  return f;
}

// Shapes for momentum grids whose tables do not fit in LDS beside the stencil
// blocks (or with more than 128 directions): tables read from global memory,
// nch = 4, 2 or 1 work items per direction (nch nd <= 1024) and 4, 8 or 16
// groups per item, chosen so that group -1 never ends an item.
FaceShape make_gtab_shape(int nd, int ne, int nch)
{
  FaceShape f;
  if (nch * nd > 1024) return f;
  f.nch = nch;
  f.maxt = 1024;
  f.gtab = true;
  for (int c : { 4, 8, 16 })
    if (!f.ce && f.nch * c >= ne + 3 && (ne + 2) % c != 0) f.ce = c;
  return f;
}

FaceShape default_shape(const btx::Grid &g, size_t lds_cap)
{
  if (g.prec == BTX_PREC_FP64) {
    const FaceShape f8 = make_shape(g.prec, g.ndir, g.ne, 8);
    if (f8.ce && face_lds_bytes(g.ndir, g.ns, 8, f8.ce, 8) <= lds_cap) return f8;
    return make_shape(g.prec, g.ndir, g.ne, 4);
  }
  return make_shape(g.prec, g.ndir, g.ne, 8);
}

template <typename T, int NCH, int MAXT, bool SPLIT>
const void *face_fn_t(int ce)
{
  if constexpr (NCH == 8) {
    switch (ce) {
    case 3: return (const void *)face_kernel<T, 8, 3, MAXT, SPLIT>;
    case 4: return (const void *)face_kernel<T, 8, 4, MAXT, SPLIT>;
    case 5: return (const void *)face_kernel<T, 8, 5, MAXT, SPLIT>;
    case 6: return (const void *)face_kernel<T, 8, 6, MAXT, SPLIT>;
    case 8: return (const void *)face_kernel<T, 8, 8, MAXT, SPLIT>;
    default: return nullptr;
    }
  } else {
    switch (ce) {
    case 4: return (const void *)face_kernel<T, 4, 4, MAXT, SPLIT>;
    case 5: return (const void *)face_kernel<T, 4, 5, MAXT, SPLIT>;
    case 6: return (const void *)face_kernel<T, 4, 6, MAXT, SPLIT>;
    case 7: return (const void *)face_kernel<T, 4, 7, MAXT, SPLIT>;
    case 8: return (const void *)face_kernel<T, 4, 8, MAXT, SPLIT>;
    case 12: return (const void *)face_kernel<T, 4, 12, MAXT, SPLIT>;
    case 16: return (const void *)face_kernel<T, 4, 16, MAXT, SPLIT>;
    default: return nullptr;
    }
  }
}

template <typename T, int NCH>
const void *face_fn_g(int ce)
{
  switch (ce) {
  case 4: return (const void *)face_kernel<T, NCH, 4, 1024, false, true>;
  case 8: return (const void *)face_kernel<T, NCH, 8, 1024, false, true>;
  case 16: return (const void *)face_kernel<T, NCH, 16, 1024, false, true>;
  default: return nullptr;
  }
}

// the face-kernel instance of a shape
template <typename T>
const void *face_fn(const FaceShape &f)
{
  if (f.ce == 0) return nullptr;
  if (f.gtab) {
    if (f.split) return nullptr;
    return f.nch == 4 ? face_fn_g<T, 4>(f.ce) : f.nch == 2 ? face_fn_g<T, 2>(f.ce)
                      : f.nch == 1 ? face_fn_g<T, 1>(f.ce) : nullptr;
  }
  if (f.nch == 4) return f.split ? face_fn_t<T, 4, 512, true>(f.ce) : face_fn_t<T, 4, 512, false>(f.ce);
  if (f.maxt == 768) return f.split ? face_fn_t<T, 8, 768, true>(f.ce) : face_fn_t<T, 8, 768, false>(f.ce);
  if constexpr (sizeof(T) == 4)
    return f.split ? face_fn_t<T, 8, 1024, true>(f.ce) : face_fn_t<T, 8, 1024, false>(f.ce);
  return nullptr;
}

const void *face_fn(size_t tsize, const FaceShape &f)
{
  return tsize == 8 ? face_fn<double>(f) : face_fn<float>(f);
}

template <typename X>
btx_status upload(X **dst, const X *src, size_t n)
{
  HIP_TRY(hipMalloc((void **)dst, sizeof(X) * std::max<size_t>(n, 1)));
  if (n) HIP_TRY(hipMemcpy(*dst, src, sizeof(X) * n, hipMemcpyHostToDevice));
  return BTX_OK;
}

btx_status device_lds_cap(int device, size_t *cap)
{
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  *cap = std::max<size_t>((size_t)prop.sharedMemPerBlock, (size_t)prop.maxSharedMemoryPerMultiProcessor);
  return BTX_OK;
}

// Raises the dynamic-LDS limit of a kernel to at least lds bytes.  The
// attribute belongs to the function and is shared by every context and batch
// of the process, so it is only ever raised (each launch still allocates just
// what it asks for).
btx_status raise_lds_limit(const void *fn, size_t lds)
{
  static std::mutex mu;
  static std::map<const void *, size_t> limit;
  std::lock_guard<std::mutex> lock(mu);
  size_t &cur = limit[fn];
  if (lds <= cur) return BTX_OK;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess)
    return fail(BTX_E_UNSUPPORTED, "a workgroup needs " + std::to_string(lds) + " B of LDS: " + hipGetErrorString(e));
  cur = lds;
  return BTX_OK;
}

// Device address of the scratch array on the current device (its name in
// host code is only a stand-in).  Resolved once per device, at context or
// batch creation with that device current, and kept for later calls.
btx_status scratch_base(int device, double **out)
{
  static std::mutex mu;
  static std::map<int, double *> base;
  std::lock_guard<std::mutex> lock(mu);
  auto it = base.find(device);
  if (it == base.end()) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BTX_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = base.emplace(device, (double *)p).first;
  }
  *out = it->second;
  return BTX_OK;
}

// ------------------------------------------------------------ one model

// Host-side owner of one model's device memory.
struct Model {
  btx::Grid g;
  int index = 0;                     // position in the device descriptor array
  size_t tsize = 8;                  // bytes per stored value
  FaceShape shape;
  double *d_mu = nullptr, *d_Phi = nullptr, *d_dOm = nullptr, *d_nvec = nullptr, *d_G = nullptr,
         *d_eps = nullptr, *d_vol = nullptr;
  double *d_vr = nullptr, *d_vth = nullptr, *d_vph = nullptr, *d_alp = nullptr, *d_psi = nullptr;
  void *d_ka = nullptr, *d_ks = nullptr, *d_feq = nullptr, *d_f[2] = { nullptr, nullptr }, *d_dN = nullptr;
  char *d_tabs = nullptr;
  FaceAux *d_aux = nullptr;
  double *d_tally = nullptr, *d_zm = nullptr, *d_ze = nullptr, *d_stage = nullptr, *d_q = nullptr;
  double *d_nbg = nullptr;           // new v_r, v_theta, v_phi, alpha, psi of a background update
  FaceDesc *d_faces = nullptr;
  int32_t *d_bface = nullptr;        // faces with a ghost side (boundary tallies)
  btx::ZoneFaces *d_zf = nullptr;
  int2 *d_fitems = nullptr, *d_zitems = nullptr;   // (index, face), (index, zone)
  // local time stepping: zone levels, and the face (zone) items sorted by
  // level so that the work of a substep is a prefix of each list
  std::vector<int> lev;              // empty: the global step
  int lmax = 0;
  std::vector<int> nf_lev, nz_lev;   // items with level <= l
  unsigned char *d_zlev = nullptr;
  int2 *d_fitems_lts = nullptr, *d_zitems_lts = nullptr;
  bool have_bg = false, have_state = false;
  double dt_max1 = 0.0;
  size_t tab_lds = 0;
};

// Checks a grid description; the message names the first problem.
btx_status validate_desc(const btx_grid_desc *d)
{
  if (!d) return fail(BTX_E_INVAL, "null grid description");
  if (d->n_r < 1 || d->n_eps < 1 || d->n_mu < 2 || d->n_phi < 1 || d->n_species < 1)
    return fail(BTX_E_INVAL, "sizes must be positive (n_mu >= 2)");
  if (d->geometry < 0 || d->geometry > 2) return fail(BTX_E_INVAL, "unknown geometry");
  if (d->mu_rule < 0 || d->mu_rule > 1) return fail(BTX_E_INVAL, "unknown mu rule");
  if (d->phi_rule < 0 || d->phi_rule > 1) return fail(BTX_E_INVAL, "unknown phi rule");
  if (d->phi_rule == BTX_PHI_DIRECTION && d->n_phi > 1 && d->n_phi < 3)
    return fail(BTX_E_INVAL, "direction-preserving Phi split needs n_phi >= 3");
  if (d->inner_bc < 0 || d->inner_bc > 2 || d->outer_bc < 1 || d->outer_bc > 2)
    return fail(BTX_E_INVAL, "bad boundary condition");
  if (d->precision != BTX_PREC_FP64 && d->precision != BTX_PREC_MIXED)
    return fail(BTX_E_INVAL, "unknown precision");
  if (!d->r_edges || !d->eps_edges) return fail(BTX_E_INVAL, "null edge array");
  const int nth = d->geometry == BTX_GEOM_AXISYM2D ? d->n_theta : 1;
  if (nth < 1) return fail(BTX_E_INVAL, "n_theta must be positive");
  if (d->n_mu * d->n_phi > 1024) return fail(BTX_E_UNSUPPORTED, "at most 1024 directions");
  if (d->n_mu * d->n_phi > 256 && d->n_eps > 29)
    return fail(BTX_E_UNSUPPORTED, "more than 256 directions take at most 29 groups");
  if (d->n_eps > 61) return fail(BTX_E_UNSUPPORTED, "at most 61 energy groups");
  if (d->n_species * d->n_eps > 2048) return fail(BTX_E_UNSUPPORTED, "at most 2048 species x groups");
  for (int a = 0; a < d->n_r; ++a)
    if (!(d->r_edges[a + 1] > d->r_edges[a])) return fail(BTX_E_INVAL, "r edges must ascend");
  if (d->geometry != BTX_GEOM_PLANAR && !(d->r_edges[0] >= 0.0)) return fail(BTX_E_INVAL, "r edges must be >= 0");
  for (int i = 0; i < d->n_eps; ++i)
    if (!(d->eps_edges[i + 1] > d->eps_edges[i]) || !(d->eps_edges[i] > 0.0))
      return fail(BTX_E_INVAL, "energy edges must be positive and ascend");
  if (d->geometry == BTX_GEOM_AXISYM2D) {
    if (!d->theta_edges) return fail(BTX_E_INVAL, "null theta edges");
    if (d->theta_bc < 0 || d->theta_bc > 1) return fail(BTX_E_INVAL, "unknown theta boundary");
    const double tmax = d->theta_bc == BTX_THETA_DISK ? 0.5 * kPi : kPi;
    if (d->theta_edges[0] != 0.0 || std::fabs(d->theta_edges[nth] - tmax) > 1e-12)
      return fail(BTX_E_UNSUPPORTED, "2D theta edges must span [0, pi] ([0, pi/2] with a disk boundary)");
    if (d->theta_bc == BTX_THETA_DISK && !(d->disk_radius > 0.0)) return fail(BTX_E_INVAL, "disk radius must be positive");
    if (d->n_phi_zones < 0) return fail(BTX_E_INVAL, "n_phi_zones must be >= 0");
    if (d->n_phi_zones > 1 && d->n_phi_zones * d->dphi > 2.0 * kPi * (1.0 + 1e-12))
      return fail(BTX_E_INVAL, "the phi zones must fit in 2 pi");
    for (int b = 0; b < nth; ++b)
      if (!(d->theta_edges[b + 1] > d->theta_edges[b])) return fail(BTX_E_INVAL, "theta edges must ascend");
    if (!(d->dphi > 0.0) || d->dphi > kPi) return fail(BTX_E_INVAL, "dphi must be in (0, pi]");
  }
  return BTX_OK;
}

void model_free(Model &m)
{
  void *ptrs[] = { m.d_mu, m.d_Phi, m.d_dOm, m.d_nvec, m.d_G, m.d_eps, m.d_vol, m.d_vr, m.d_vth, m.d_vph,
                   m.d_alp, m.d_psi, m.d_ka, m.d_ks, m.d_feq, m.d_f[0], m.d_f[1], m.d_dN, m.d_tally,
                   m.d_zm, m.d_ze, m.d_stage, m.d_faces, m.d_zf, m.d_tabs, m.d_aux, m.d_fitems, m.d_zitems,
                   m.d_nbg, m.d_q, m.d_zlev, m.d_fitems_lts, m.d_zitems_lts, m.d_bface };
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  m = Model();
}

// Grid, quadrature and faces (paper Sec. 3.1) on the host, device buffers.
// The current device must be set.  On failure nothing stays allocated.
btx_status model_init(Model &m, const btx_grid_desc *d, int index, size_t lds_cap)
{
  btx_status st = validate_desc(d);
  if (st != BTX_OK) return st;
  btx::Grid &g = m.g;
  const int nth = d->geometry == BTX_GEOM_AXISYM2D ? d->n_theta : 1;
  g.nr = d->n_r; g.nth = nth; g.ne = d->n_eps; g.nmu = d->n_mu; g.nphi = d->n_phi; g.ns = d->n_species;
  g.geom = d->geometry; g.mu_rule = d->mu_rule; g.phi_rule = d->phi_rule;
  g.inner_bc = d->inner_bc; g.outer_bc = d->outer_bc; g.prec = d->precision;
  g.theta_bc = d->geometry == BTX_GEOM_AXISYM2D ? d->theta_bc : BTX_THETA_AXIS;
  g.nph = d->geometry == BTX_GEOM_AXISYM2D ? std::max(1, (int)d->n_phi_zones) : 1;
  g.disk_r = d->disk_radius;
  g.dphi = d->dphi;
  g.fp64_thr = d->fp64_threshold > 0.0 ? d->fp64_threshold : 1.0;
  g.r_e.assign(d->r_edges, d->r_edges + g.nr + 1);
  g.eps_e.assign(d->eps_edges, d->eps_edges + g.ne + 1);
  if (g.geom == BTX_GEOM_AXISYM2D) g.th_e.assign(d->theta_edges, d->theta_edges + nth + 1);
  else g.th_e = { 0.0, kPi };
  std::string why = btx::build_grid(g);
  if (!why.empty()) return fail(BTX_E_UNSUPPORTED, why);
  m.index = index;
  m.tsize = g.prec == BTX_PREC_FP64 ? 8 : 4;
  m.dt_max1 = btx::max_dt(g, 1.0);
  m.shape = default_shape(g, lds_cap);
  if (m.shape.ce == 0 || face_lds_bytes(g.ndir, g.ns, m.shape.nch, m.shape.ce, m.tsize) > lds_cap) {
    FaceShape fit, first;                          // tables through the caches instead of LDS
    for (int nch : { 4, 2, 1 }) {
      const FaceShape f = make_gtab_shape(g.ndir, g.ne, nch);
      if (!f.ce) continue;
      if (!first.ce) first = f;
      if (face_lds_bytes(g.ndir, g.ns, nch, f.ce, m.tsize, true) <= lds_cap) { fit = f; break; }
    }
    m.shape = fit.ce ? fit : first;                // the first that fits, else report the LDS
  }
  if (m.shape.ce == 0) return fail(BTX_E_UNSUPPORTED, "no face work-item shape for this grid");
  const size_t flds = face_lds_bytes(g.ndir, g.ns, m.shape.nch, m.shape.ce, m.tsize, m.shape.gtab);
  if (flds > lds_cap)
    return fail(BTX_E_UNSUPPORTED, "face workgroup needs " + std::to_string(flds) + " B of LDS");
  m.tab_lds = (m.shape.gtab ? 0 : kTables * tab_stride(g.ndir, m.tsize)) + align16(5 * sizeof(Frame)) +
              align16(scratch_bytes(g.ndir, m.tsize, m.shape.gtab ? 1 : 4)) + align16((size_t)g.nmu * 8);
  if (m.tab_lds > lds_cap) return fail(BTX_E_UNSUPPORTED, "table build needs too much LDS");
  const size_t nz = g.nz, blk = (size_t)g.ns * g.ne * g.ndir, nk = nz * g.ns * g.ne, nf = g.faces.size();
  std::vector<int2> fit(nf), zit(nz);
  for (size_t k = 0; k < nf; ++k) fit[k] = make_int2(index, (int)k);
  for (size_t k = 0; k < nz; ++k) zit[k] = make_int2(index, (int)k);
  std::vector<double> zero(nz, 0.0), one(nz, 1.0);
#define TRY(x) do { st = (x); if (st != BTX_OK) { model_free(m); return st; } } while (0)
  TRY(upload(&m.d_mu, g.mu.data(), g.mu.size()));
  TRY(upload(&m.d_Phi, g.Phi.data(), g.Phi.size()));
  TRY(upload(&m.d_dOm, g.dOm.data(), g.dOm.size()));
  TRY(upload(&m.d_nvec, g.nvec.data(), g.nvec.size()));
  TRY(upload(&m.d_G, g.G.data(), g.G.size()));
  TRY(upload(&m.d_eps, g.eps.data(), g.eps.size()));
  TRY(upload(&m.d_vol, g.vol.data(), g.vol.size()));
  TRY(upload(&m.d_faces, g.faces.data(), nf));
  TRY(upload(&m.d_zf, g.zfaces.data(), g.zfaces.size()));
  TRY(upload(&m.d_fitems, fit.data(), nf));
  TRY(upload(&m.d_zitems, zit.data(), nz));
  if (!g.bface.empty()) TRY(upload(&m.d_bface, g.bface.data(), g.bface.size()));
  TRY(upload(&m.d_vr, zero.data(), nz));
  TRY(upload(&m.d_vth, zero.data(), nz));
  TRY(upload(&m.d_vph, zero.data(), nz));
  TRY(upload(&m.d_alp, one.data(), nz));
  TRY(upload(&m.d_psi, one.data(), nz));
#undef TRY
  auto dmalloc = [&](void **p, size_t bytes) -> bool {
    if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
    return hipMemset(*p, 0, std::max<size_t>(bytes, 16)) == hipSuccess;
  };
  if (!dmalloc(&m.d_ka, nk * m.tsize) || !dmalloc(&m.d_ks, nk * m.tsize) || !dmalloc(&m.d_feq, nk * m.tsize) ||
      !dmalloc(&m.d_f[0], nz * blk * m.tsize) || !dmalloc(&m.d_f[1], nz * blk * m.tsize) ||
      !dmalloc(&m.d_dN, nf * 2 * blk * m.tsize) || !dmalloc((void **)&m.d_tally, nf * g.ns * 8) ||
      !dmalloc((void **)&m.d_zm, nz * g.ns * 5 * 8) || !dmalloc((void **)&m.d_ze, nz * g.ns * 8) ||
      !dmalloc((void **)&m.d_stage, nk * 8) || !dmalloc((void **)&m.d_nbg, nz * 5 * 8) ||
      !dmalloc((void **)&m.d_q, nz * 5 * 8) ||
      !dmalloc((void **)&m.d_tabs, nf * kTables * tab_stride(g.ndir, m.tsize)) ||
      !dmalloc((void **)&m.d_aux, nf * sizeof(FaceAux))) {
    model_free(m);
    return fail(BTX_E_NOMEM, "device allocation failed");
  }
  return BTX_OK;
}

// the device descriptor of a model (its current face shape and step)
ModelDev model_dev(const Model &m, double dt)
{
  const btx::Grid &g = m.g;
  ModelDev M;
  DevGrid &d = M.g;
  d.nr = g.nr; d.nth = g.nth; d.ne = g.ne; d.nmu = g.nmu; d.nphi = g.nphi; d.ns = g.ns;
  d.ndir = g.ndir; d.nz = g.nz; d.geom = g.geom; d.phi_rule = g.phi_rule;
  d.eblk = g.ne * g.ndir; d.blk = g.ns * d.eblk;
  d.nfaces = (int)g.faces.size();
  d.nch = m.shape.nch;
  d.ce = m.shape.ce;
  d.lnq = g.lnq; d.q = g.q; d.fp64_thr = g.fp64_thr;
  d.om[0] = d.om[1] = d.om[2] = d.om[3] = 0.0;
  for (int k = 0; k < g.ndir; ++k) {
    d.om[0] += g.dOm[k];
    d.om[1] += g.dOm[k] * g.nvec[3 * k];
    d.om[2] += g.dOm[k] * g.nvec[3 * k + 1];
    d.om[3] += g.dOm[k] * g.nvec[3 * k + 2];
  }
  d.mu = m.d_mu; d.Phi = m.d_Phi; d.dOm = m.d_dOm; d.nvec = m.d_nvec; d.G = m.d_G;
  d.eps = m.d_eps; d.vol = m.d_vol;
  d.vr = m.d_vr; d.vth = m.d_vth; d.vph = m.d_vph; d.alp = m.d_alp; d.psi = m.d_psi;
  M.faces = m.d_faces;
  M.zf = m.d_zf;
  M.tabs = m.d_tabs;
  M.aux = m.d_aux;
  M.f[0] = m.d_f[0];
  M.f[1] = m.lev.empty() ? m.d_f[1] : m.d_f[0];    // time levels: updated in place
  M.zlev = m.lev.empty() ? nullptr : m.d_zlev;
  M.ka = m.d_ka; M.ks = m.d_ks; M.feq = m.d_feq;
  M.dN = m.d_dN;
  M.tally = m.d_tally;
  M.q = m.d_q;
  M.dt = dt;
  return M;
}

btx_status check_background(const Model &m, const btx_background *bg)
{
  if (!bg) return fail(BTX_E_INVAL, "null argument");
  if (!bg->v_r || !bg->v_theta || !bg->alpha || !bg->psi || !bg->kappa_a || !bg->kappa_s || !bg->f_eq)
    return fail(BTX_E_INVAL, "null background array");
  const btx::Grid &g = m.g;
  const size_t nz = g.nz, nk = nz * g.ns * g.ne;
  for (size_t z = 0; z < nz; ++z) {
    const double vp = bg->v_phi ? bg->v_phi[z] : 0.0;
    double v2 = bg->v_r[z] * bg->v_r[z] + bg->v_theta[z] * bg->v_theta[z] + vp * vp;
    if (!(v2 < 1.0) || !(bg->alpha[z] > 0.0) || !(bg->psi[z] > 0.0) || !std::isfinite(bg->alpha[z]) ||
        !std::isfinite(bg->psi[z]))
      return fail(BTX_E_INVAL, "background velocity/metric out of range at zone " + std::to_string(z));
  }
  for (size_t k = 0; k < nk; ++k)
    if (!(bg->kappa_a[k] >= 0.0) || !(bg->kappa_s[k] >= 0.0) || !std::isfinite(bg->kappa_a[k]) ||
        !std::isfinite(bg->kappa_s[k]) || !std::isfinite(bg->f_eq[k]))
      return fail(BTX_E_INVAL, "opacities must be finite and >= 0 (entry " + std::to_string(k) + ")");
  return BTX_OK;
}

// copies the background into the model's buffers (storage precision)
btx_status upload_background(Model &m, const btx_background *bg, hipStream_t s)
{
  const btx::Grid &g = m.g;
  const size_t nz = g.nz, nk = nz * g.ns * g.ne;
  HIP_TRY(hipMemcpy(m.d_vr, bg->v_r, nz * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m.d_vth, bg->v_theta, nz * 8, hipMemcpyHostToDevice));
  if (bg->v_phi) HIP_TRY(hipMemcpy(m.d_vph, bg->v_phi, nz * 8, hipMemcpyHostToDevice));
  else HIP_TRY(hipMemset(m.d_vph, 0, nz * 8));
  HIP_TRY(hipMemcpy(m.d_alp, bg->alpha, nz * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m.d_psi, bg->psi, nz * 8, hipMemcpyHostToDevice));
  const double *src[3] = { bg->kappa_a, bg->kappa_s, bg->f_eq };
  void *dst[3] = { m.d_ka, m.d_ks, m.d_feq };
  for (int k = 0; k < 3; ++k) {
    if (m.tsize == 8) {
      HIP_TRY(hipMemcpy(dst[k], src[k], nk * 8, hipMemcpyHostToDevice));
    } else {
      HIP_TRY(hipMemcpy(m.d_stage, src[k], nk * 8, hipMemcpyHostToDevice));
      hipLaunchKernelGGL((cast_kernel<float>), dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s,
                         m.d_stage, (float *)dst[k], nk);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipStreamSynchronize(s));
    }
  }
  return BTX_OK;
}

// remap tables and frame data of every face of a model (its descriptor must
// be current on the device: the window offsets depend on the face shape)
btx_status build_tables(const Model &m, const ModelDev *d_models, hipStream_t s)
{
  const int nf = (int)m.g.faces.size();
  if (nf == 0) return BTX_OK;
  const void *tk = m.shape.gtab
                       ? (m.tsize == 8 ? (const void *)table_kernel<double, true> : (const void *)table_kernel<float, true>)
                       : (m.tsize == 8 ? (const void *)table_kernel<double, false> : (const void *)table_kernel<float, false>);
  btx_status st = raise_lds_limit(tk, m.tab_lds);
  if (st != BTX_OK) return st;
  const int2 *items = m.d_fitems;
  void *args[] = { &d_models, &items };
  HIP_TRY(hipLaunchKernel(tk, dim3(nf), dim3(256), args, m.tab_lds, s));
  return BTX_OK;
}

// species_rows: one workgroup per (face, species) instead of per face (all
// models of the launch must then have that many species)
btx_status launch_faces(const FaceShape &shape, size_t tsize, const ModelDev *d_models, const int2 *items,
                        int n, int threads, size_t lds, int parity, hipStream_t s, int sub = 0,
                        int species_rows = 1)
{
  if (n == 0) return BTX_OK;
  const void *fn = face_fn(tsize, shape);
  if (!fn) return fail(BTX_E_UNSUPPORTED, "no face kernel for this shape");
  void *args[] = { &d_models, &items, &parity, &sub };
  HIP_TRY(hipLaunchKernel(fn, dim3(n, std::max(species_rows, 1)), dim3(threads), args, lds, s));
  return BTX_OK;
}

// zone kernel LDS: five FP64 row values per (species, group) row
size_t zone_lds_bytes(int rows) { return (size_t)std::max(rows, 1) * 5 * sizeof(double); }

btx_status launch_zones(size_t tsize, const ModelDev *d_models, const int2 *items, int n, int max_rows,
                        int parity, hipStream_t s, int max_dirs = 0)
{
  if (n == 0) return BTX_OK;
  const void *zk = max_dirs > 256 ? (tsize == 8 ? (const void *)zone_kernel<double, 16> : (const void *)zone_kernel<float, 16>)
                                  : (tsize == 8 ? (const void *)zone_kernel<double, 4> : (const void *)zone_kernel<float, 4>);
  void *args[] = { &d_models, &items, &parity };
  HIP_TRY(hipLaunchKernel(zk, dim3(n), dim3(256), args, zone_lds_bytes(max_rows), s));
  return BTX_OK;
}

int face_threads(const Model &m) { return ((m.shape.nch * m.g.ndir + 63) / 64) * 64; }

size_t face_lds(const Model &m)
{
  return face_lds_bytes(m.g.ndir, m.g.ns, m.shape.nch, m.shape.ce, m.tsize, m.shape.gtab);
}

btx_status set_face_lds(size_t tsize, const FaceShape &f, size_t lds)
{
  const void *fn = face_fn(tsize, f);
  if (!fn) return fail(BTX_E_UNSUPPORTED, "no face kernel for this shape");
  return raise_lds_limit(fn, lds);
}

// A new background for a model (set_background), or, once a state exists, a
// background that evolves: the state is first remapped from the comoving
// frames of the current background to those of the new one (forward in time,
// time_remap_kernel), then the new background and its face tables are adopted.
btx_status model_update_background(Model &m, const btx_background *bg, const ModelDev *d_models, int parity,
                                   hipStream_t s)
{
  btx_status st = check_background(m, bg);
  if (st != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  if (m.have_bg && m.have_state) {
    const size_t nz = m.g.nz;
    HIP_TRY(hipMemcpy(m.d_nbg, bg->v_r, nz * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m.d_nbg + nz, bg->v_theta, nz * 8, hipMemcpyHostToDevice));
    if (bg->v_phi) HIP_TRY(hipMemcpy(m.d_nbg + 2 * nz, bg->v_phi, nz * 8, hipMemcpyHostToDevice));
    else HIP_TRY(hipMemset(m.d_nbg + 2 * nz, 0, nz * 8));
    HIP_TRY(hipMemcpy(m.d_nbg + 3 * nz, bg->alpha, nz * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m.d_nbg + 4 * nz, bg->psi, nz * 8, hipMemcpyHostToDevice));
    const void *tk = m.tsize == 8 ? (const void *)time_remap_kernel<double> : (const void *)time_remap_kernel<float>;
    const size_t lds = time_lds_bytes(m.g.ndir, m.g.ne, m.tsize);
    if ((st = raise_lds_limit(tk, lds)) != BTX_OK) return st;
    const int2 *items = m.d_zitems;
    const double *nbg = m.d_nbg;
    void *args[] = { &d_models, &items, &parity, &nbg };
    HIP_TRY(hipLaunchKernel(tk, dim3((unsigned)nz), dim3(256), args, lds, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if ((st = upload_background(m, bg, s)) != BTX_OK) return st;
  if ((st = build_tables(m, d_models, s)) != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  m.have_bg = true;
  return BTX_OK;
}

btx_status model_set_state(Model &m, int parity, const void *f, int is_device_ptr, hipStream_t s)
{
  if (!f) return fail(BTX_E_INVAL, "null state");
  const btx::Grid &g = m.g;
  const size_t bytes = (size_t)g.nz * g.ns * g.ne * g.ndir * m.tsize;
  HIP_TRY(hipMemcpyAsync(m.d_f[parity], f, bytes, is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(m.d_tally, 0, std::max<size_t>(g.faces.size(), 1) * g.ns * 8, s));
  HIP_TRY(hipStreamSynchronize(s));
  m.have_state = true;
  return BTX_OK;
}

btx_status model_get_state(const Model &m, int parity, void *f, int is_device_ptr, hipStream_t s)
{
  if (!f) return fail(BTX_E_INVAL, "null state");
  if (!m.have_state) return fail(BTX_E_STATE, "no state set");
  const btx::Grid &g = m.g;
  const size_t bytes = (size_t)g.nz * g.ns * g.ne * g.ndir * m.tsize;
  HIP_TRY(hipMemcpyAsync(f, m.d_f[parity], bytes, is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return BTX_OK;
}

btx_status model_moments(const Model &m, const ModelDev *d_models, int parity, double *zone_moments,
                         double *totals, hipStream_t s)
{
  if (!m.have_bg || !m.have_state) return fail(BTX_E_STATE, "background and state must be set");
  const btx::Grid &g = m.g;
  int idx = m.index;
  double *zm = m.d_zm, *ze = m.d_ze;
  void *args[] = { &d_models, &idx, &parity, &zm, &ze };
  const void *mk = m.tsize == 8 ? (const void *)moments_kernel<double> : (const void *)moments_kernel<float>;
  HIP_TRY(hipLaunchKernel(mk, dim3(g.nz), dim3(256), args, 0, s));
  std::vector<double> hzm((size_t)g.nz * g.ns * 5), hze((size_t)g.nz * g.ns), tally(g.faces.size() * g.ns);
  HIP_TRY(hipMemcpyAsync(hzm.data(), m.d_zm, hzm.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hze.data(), m.d_ze, hze.size() * 8, hipMemcpyDeviceToHost, s));
  if (!tally.empty()) HIP_TRY(hipMemcpyAsync(tally.data(), m.d_tally, tally.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (zone_moments) std::memcpy(zone_moments, hzm.data(), hzm.size() * 8);
  if (totals) {
    // compensated sums over the zones and the boundary faces
    auto add = [](double &s, double &c, double x) {
      const double t = s + x;
      c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
    };
    for (int sp = 0; sp < g.ns; ++sp) {
      double N = 0.0, Nc = 0.0, E = 0.0, Ec = 0.0, out = 0.0, outc = 0.0;
      for (int z = 0; z < g.nz; ++z) {
        add(N, Nc, hzm[((size_t)z * g.ns + sp) * 5]);
        add(E, Ec, hze[(size_t)z * g.ns + sp]);
      }
      for (int f : g.bface) add(out, outc, tally[(size_t)f * g.ns + sp]);
      totals[3 * sp] = N + Nc;
      totals[3 * sp + 1] = out + outc;
      totals[3 * sp + 2] = E + Ec;
    }
  }
  return BTX_OK;
}

// btx_moments with device outputs and the scratch array for its partial
// results: no allocation, no synchronisation.  zm (may be null) and totals
// (may be null) are device pointers.
btx_status model_moments_device(const Model &m, const ModelDev *d_models, int parity, double *zm,
                                double *totals, double *scr, hipStream_t s)
{
  const btx::Grid &g = m.g;
  const size_t pairs = (size_t)g.nz * g.ns;
  if (pairs > kScratchPairs)
    return fail(BTX_E_UNSUPPORTED, "btx_moments_device takes at most " + std::to_string(kScratchPairs) +
                                       " (zone, species) pairs; this grid has " + std::to_string(pairs));
  if (!m.have_bg || !m.have_state) return fail(BTX_E_STATE, "background and state must be set");
  if (!zm && !totals) return BTX_OK;
  int idx = m.index;
  double *ze = scr, *zmo = zm ? zm : scr + kScratchPairs;
  void *args[] = { &d_models, &idx, &parity, &zmo, &ze };
  const void *mk = m.tsize == 8 ? (const void *)moments_kernel<double> : (const void *)moments_kernel<float>;
  HIP_TRY(hipLaunchKernel(mk, dim3(g.nz), dim3(256), args, 0, s));
  if (totals) {
    const double *tally = m.d_tally;
    const int32_t *bface = m.d_bface;
    int nz = g.nz, ns = g.ns, nb = (int)g.bface.size();
    const double *zmc = zmo, *zec = ze;
    void *targs[] = { &zmc, &zec, &tally, &bface, &nz, &ns, &nb, &totals };
    HIP_TRY(hipLaunchKernel((const void *)totals_kernel, dim3(3 * g.ns), dim3(256), targs, 0, s));
  }
  return BTX_OK;
}

btx_status model_source_terms(const Model &m, double *q, hipStream_t s)
{
  if (!q) return fail(BTX_E_INVAL, "null argument");
  if (!m.have_bg || !m.have_state) return fail(BTX_E_STATE, "background and state must be set");
  HIP_TRY(hipMemcpyAsync(q, m.d_q, (size_t)m.g.nz * 5 * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return BTX_OK;
}

// Courant length of every zone: its volume over its largest face on an
// axis, the smallest over the axes (btx::max_dt is cfl times the minimum)
std::vector<double> courant_lengths(const btx::Grid &g)
{
  std::vector<double> len(g.nz);
  for (int z = 0; z < g.nz; ++z) {
    double amax[3] = { 0.0, 0.0, 0.0 }, m = 1e300;
    const btx::ZoneFaces &zf = g.zfaces[z];
    for (int q = 0; q < zf.n; ++q) {
      const FaceDesc &F = g.faces[zf.fid[q]];
      if (F.active && F.area > amax[F.axis]) amax[F.axis] = F.area;
    }
    for (int ax = 0; ax < 3; ++ax)
      if (amax[ax] > 0.0) m = std::min(m, g.vol[z] / amax[ax]);
    len[z] = m;
  }
  return len;
}

// Time levels (local time stepping, Sec. 6): zone z takes 2^l global steps
// at once, l the largest with 2^l times the smallest Courant length within
// its own (at most max_level); then zones that share a face are brought to
// at most one level apart by lowering the coarser.
void assign_levels(const btx::Grid &g, int max_level, std::vector<int> &lev)
{
  const std::vector<double> len = courant_lengths(g);
  const double lmin = *std::min_element(len.begin(), len.end());
  lev.assign(g.nz, 0);
  for (int z = 0; z < g.nz; ++z) {
    int l = 0;
    while (l < max_level && len[z] >= lmin * (double)(2 << l) * (1.0 - 1e-12)) ++l;
    lev[z] = l;
  }
  bool changed = true;
  while (changed) {
    changed = false;
    for (const FaceDesc &F : g.faces) {
      if (!F.active || F.L.kind != btx::SIDE_ZONE || F.R.kind != btx::SIDE_ZONE) continue;
      int &a = lev[F.L.z], &b = lev[F.R.z];
      if (a > b + 1) { a = b + 1; changed = true; }
      if (b > a + 1) { b = a + 1; changed = true; }
    }
  }
}

// Adopts per-zone time levels (null: back to the global step).  The state is
// then updated in place (the descriptor points both buffers at the current
// one); face and zone items are sorted by level for the substep prefixes.
btx_status model_set_levels(Model &m, const int32_t *levels, int &parity, hipStream_t s)
{
  HIP_TRY(hipStreamSynchronize(s));
  if (m.d_zlev) { (void)hipFree(m.d_zlev); m.d_zlev = nullptr; }
  if (m.d_fitems_lts) { (void)hipFree(m.d_fitems_lts); m.d_fitems_lts = nullptr; }
  if (m.d_zitems_lts) { (void)hipFree(m.d_zitems_lts); m.d_zitems_lts = nullptr; }
  if (parity == 1)
    HIP_TRY(hipMemcpy(m.d_f[0], m.d_f[1], (size_t)m.g.nz * m.g.ns * m.g.ne * m.g.ndir * m.tsize,
                      hipMemcpyDeviceToDevice));
  parity = 0;
  m.lev.clear();
  m.lmax = 0;
  if (!levels) return BTX_OK;
  const btx::Grid &g = m.g;
  std::vector<int> lev(levels, levels + g.nz);
  for (int l : lev)
    if (l < 0 || l > 16) return fail(BTX_E_INVAL, "time levels must be in 0..16");
  const int lmax = *std::max_element(lev.begin(), lev.end());
  std::vector<unsigned char> l8(lev.begin(), lev.end());
  std::vector<std::pair<int, int>> fs, zs;
  for (int f = 0; f < (int)g.faces.size(); ++f)
    fs.emplace_back(std::min(lev[g.faces[f].L.z], lev[g.faces[f].R.z]), f);
  for (int z = 0; z < g.nz; ++z) zs.emplace_back(lev[z], z);
  std::stable_sort(fs.begin(), fs.end());
  std::stable_sort(zs.begin(), zs.end());
  std::vector<int2> fit, zit;
  m.nf_lev.assign(lmax + 1, 0);
  m.nz_lev.assign(lmax + 1, 0);
  for (auto &p : fs) { fit.push_back(make_int2(m.index, p.second)); for (int l = p.first; l <= lmax; ++l) ++m.nf_lev[l]; }
  for (auto &p : zs) { zit.push_back(make_int2(m.index, p.second)); for (int l = p.first; l <= lmax; ++l) ++m.nz_lev[l]; }
  btx_status st;
  if ((st = upload(&m.d_zlev, l8.data(), l8.size())) != BTX_OK) return st;
  if ((st = upload(&m.d_fitems_lts, fit.data(), fit.size())) != BTX_OK) return st;
  if ((st = upload(&m.d_zitems_lts, zit.data(), zit.size())) != BTX_OK) return st;
  m.lev = lev;
  m.lmax = lmax;
  return BTX_OK;
}

btx_status check_dt(const Model &m, double dt)
{
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BTX_E_INVAL, "dt must be positive and finite");
  if (dt > m.dt_max1 * (1.0 + 1e-12)) return fail(BTX_E_CFL, "dt exceeds the Courant limit");
  if (!m.lev.empty()) {                  // every zone within its own limit at its level
    const std::vector<double> len = courant_lengths(m.g);
    for (int z = 0; z < m.g.nz; ++z)
      if (dt * (double)(1 << m.lev[z]) > len[z] * (1.0 + 1e-12))
        return fail(BTX_E_CFL, "a zone's time level takes it beyond its Courant limit");
  }
  return BTX_OK;
}

}  // namespace

// ------------------------------------------------------------ single context

struct btx_ctx {
  Model m;
  int device = 0;
  hipStream_t stream = nullptr;
  ModelDev *d_model = nullptr;       // descriptor of m on the device
  ModelDev h_model;                  // its host copy (dt of the last launch)
  int parity = 0;                    // buffer holding the current state
  // timing: three events per step recorded on the stream, resolved on query
  bool timing = false;
  double t_ms[2] = { 0, 0 };
  int64_t t_n[2] = { 0, 0 };
  std::vector<hipEvent_t> ev;      // pool, 3 per recorded step
  size_t ev_used = 0;              // events recorded and not yet resolved
};

namespace {

void free_ctx(btx_ctx *c)
{
  model_free(c->m);
  if (c->d_model) (void)hipFree(c->d_model);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

btx_status ctx_step(btx_ctx *c, double dt)
{
  Model &m = c->m;
  if (c->h_model.dt != dt) {                // kernels in flight read the descriptor
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->h_model.dt = dt;
    HIP_TRY(hipMemcpy(c->d_model, &c->h_model, sizeof(ModelDev), hipMemcpyHostToDevice));
  }
  if (!m.lev.empty()) {                       // time levels: 2^L substeps
    const int L = m.lmax;
    for (int k = 0; k < (1 << L); ++k) {
      const int lf = k == 0 ? L : std::min(L, __builtin_ctz(k));       // faces whose finer zone starts
      const int lz = std::min(L, __builtin_ctz(k + 1));                 // zones whose step ends
      // a substep with too few faces to fill the device takes one workgroup
      // per (face, species)
      const int rows = m.nf_lev[lf] < 2 * kFillFaces ? m.g.ns : 1;
      btx_status st = launch_faces(m.shape, m.tsize, c->d_model, m.d_fitems_lts, m.nf_lev[lf], face_threads(m),
                                   face_lds(m), 0, c->stream, k, rows);
      if (st != BTX_OK) return st;
      st = launch_zones(m.tsize, c->d_model, m.d_zitems_lts, m.nz_lev[lz], m.g.ns * m.g.ne, 0, c->stream,
                        m.g.ndir);
      if (st != BTX_OK) return st;
    }
    return BTX_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  const bool rec = c->timing && c->ev_used + 3 <= c->ev.size();
  if (rec) {
    e0 = c->ev[c->ev_used]; e1 = c->ev[c->ev_used + 1]; e2 = c->ev[c->ev_used + 2];
    c->ev_used += 3;
    HIP_TRY(hipEventRecord(e0, c->stream));
  }
  btx_status st = launch_faces(m.shape, m.tsize, c->d_model, m.d_fitems, (int)m.g.faces.size(), face_threads(m),
                               face_lds(m), c->parity, c->stream);
  if (st != BTX_OK) return st;
  if (rec) HIP_TRY(hipEventRecord(e1, c->stream));
  st = launch_zones(m.tsize, c->d_model, m.d_zitems, m.g.nz, m.g.ns * m.g.ne, c->parity, c->stream, m.g.ndir);
  if (st != BTX_OK) return st;
  if (rec) HIP_TRY(hipEventRecord(e2, c->stream));
  c->parity ^= 1;
  return BTX_OK;
}

}  // namespace

// ------------------------------------------------------------ batch

namespace {

// Face work items of the models that share one face shape: one launch each.
struct BatchGroup {
  FaceShape shape;
  int first = 0, count = 0;          // range in the group item array
  int first_lts = 0;                 // start in the level-sorted item array
  int threads = 64;
  size_t lds = 0;
};

}  // namespace

struct btx_batch {
  std::vector<Model> models;
  int device = 0;
  size_t tsize = 8;
  hipStream_t stream = nullptr;      // caller's stream: all work is ordered on it
  hipStream_t cap = nullptr;         // library stream used only to capture graphs
  ModelDev *d_models = nullptr;
  std::vector<ModelDev> h_models;
  std::vector<BatchGroup> groups;
  int2 *d_gitems = nullptr;          // face items of all groups, group after group
  int2 *d_zitems = nullptr;          // zone items of every model
  int nz_all = 0;
  double *d_tscratch = nullptr;      // tally target while shapes are timed
  int parity = 0;
  bool tuned = false, use_graph = true;
  hipGraphExec_t exec[2] = { nullptr, nullptr };
  std::string tune_path;
  // local time stepping: once a model is given time levels, every model
  // updates in place and a step is 2^L substeps (L the largest level);
  // face items sorted by level within each group, zone items by level
  bool lts = false, lts_dirty = true;
  int lts_L = 0;
  int2 *d_gitems_lts = nullptr, *d_zitems_lts = nullptr;
  std::vector<std::vector<int>> gf_lev;  // per group: items of level <= l
  std::vector<int> z_lev;                // zone items of level <= l
};

namespace {

void drop_graphs(btx_batch *b)
{
  for (auto &e : b->exec)
    if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
}

void free_batch(btx_batch *b)
{
  drop_graphs(b);
  for (Model &m : b->models) model_free(m);
  void *ptrs[] = { b->d_models, b->d_gitems, b->d_zitems, b->d_tscratch, b->d_gitems_lts, b->d_zitems_lts };
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

btx_status upload_descriptors(btx_batch *b)
{
  HIP_TRY(hipStreamSynchronize(b->stream));            // kernels in flight read them
  HIP_TRY(hipMemcpy(b->d_models, b->h_models.data(), b->h_models.size() * sizeof(ModelDev),
                    hipMemcpyHostToDevice));
  return BTX_OK;
}

std::string tune_key(const Model &m)
{
  return std::string(m.tsize == 8 ? "f64" : "f32") + ":nd" + std::to_string(m.g.ndir) + ":ne" +
         std::to_string(m.g.ne);
}

// tuning cache: a flat JSON object {"f32:nd16:ne12": 8, ...} (work items per
// direction of each model class)
std::vector<std::pair<std::string, int>> read_cache(const std::string &path)
{
  std::vector<std::pair<std::string, int>> out;
  if (path.empty()) return out;
  FILE *fp = std::fopen(path.c_str(), "r");
  if (!fp) return out;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, n);
  std::fclose(fp);
  size_t p = 0;
  while ((p = text.find('"', p)) != std::string::npos) {
    size_t q = text.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string key = text.substr(p + 1, q - p - 1);
    size_t c = text.find(':', q);
    if (c == std::string::npos) break;
    int v = std::atoi(text.c_str() + c + 1);
    if (v == 4 || v == 8) out.emplace_back(key, v);
    p = c + 1;
  }
  return out;
}

void write_cache(const std::string &path, const std::vector<std::pair<std::string, int>> &kv)
{
  if (path.empty()) return;
  FILE *fp = std::fopen(path.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{\n");
  for (size_t k = 0; k < kv.size(); ++k)
    std::fprintf(fp, "  \"%s\": %d%s\n", kv[k].first.c_str(), kv[k].second, k + 1 < kv.size() ? "," : "");
  std::fprintf(fp, "}\n");
  std::fclose(fp);
}

btx_status set_shape(btx_batch *b, Model &m, const FaceShape &f)
{
  m.shape = f;
  b->h_models[m.index].g.nch = f.nch;
  b->h_models[m.index].g.ce = f.ce;
  return BTX_OK;
}

// Groups models by face shape and uploads the grouped face items.
btx_status build_groups(btx_batch *b)
{
  drop_graphs(b);
  b->groups.clear();
  std::vector<int2> items;
  std::vector<bool> done(b->models.size(), false);
  for (size_t i = 0; i < b->models.size(); ++i) {
    if (done[i]) continue;
    BatchGroup gr;
    gr.shape = b->models[i].shape;
    gr.first = (int)items.size();
    for (size_t j = i; j < b->models.size(); ++j) {
      Model &m = b->models[j];
      if (done[j] || !(m.shape == gr.shape)) continue;
      done[j] = true;
      for (size_t k = 0; k < m.g.faces.size(); ++k) items.push_back(make_int2(m.index, (int)k));
      gr.threads = std::max(gr.threads, face_threads(m));
      gr.lds = std::max(gr.lds, face_lds(m));
    }
    gr.count = (int)items.size() - gr.first;
    btx_status st = set_face_lds(b->tsize, gr.shape, gr.lds);
    if (st != BTX_OK) return st;
    b->groups.push_back(gr);
  }
  b->lts_dirty = true;
  if (b->d_gitems) { (void)hipFree(b->d_gitems); b->d_gitems = nullptr; }
  return upload(&b->d_gitems, items.data(), items.size());
}

// Autotuner: FP32 models may run their faces with 8 or 4 work items per
// direction (groups per item follow); each model class (precision,
// directions, groups) takes the faster, timed on its own faces with the
// current state.  Choices persist in the tuning cache file.
btx_status tune(btx_batch *b)
{
  auto cache = read_cache(b->tune_path);
  auto lookup = [&](const std::string &k) {
    for (auto &kv : cache)
      if (kv.first == k) return kv.second;
    return 0;
  };
  // timing launches must not add to the boundary tallies
  size_t tmax = 1;
  for (Model &m : b->models) tmax = std::max(tmax, m.g.faces.size() * (size_t)m.g.ns);
  if (!b->d_tscratch) HIP_TRY(hipMalloc((void **)&b->d_tscratch, tmax * 8));
  std::vector<double *> tsave(b->models.size());
  for (Model &m : b->models) {
    tsave[m.index] = b->h_models[m.index].tally;
    b->h_models[m.index].tally = b->d_tscratch;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  btx_status st = BTX_OK;
  for (size_t i = 0; i < b->models.size() && st == BTX_OK; ++i) {
    const std::string key = tune_key(b->models[i]);
    if (b->tsize == 8 || lookup(key) || b->models[i].shape.gtab) continue;
    std::vector<Model *> cls;
    for (Model &m : b->models)
      if (tune_key(m) == key) cls.push_back(&m);
    float best = 1e30f;
    int best_nch = 8;
    for (int nch : { 8, 4 }) {
      const FaceShape f = make_shape(cls[0]->g.prec, cls[0]->g.ndir, cls[0]->g.ne, nch);
      if (f.ce == 0 || face_lds_bytes(cls[0]->g.ndir, cls[0]->g.ns, f.nch, f.ce, b->tsize) > 160 * 1024) continue;
      for (Model *m : cls) set_shape(b, *m, f);
      if ((st = upload_descriptors(b)) != BTX_OK) break;
      for (Model *m : cls)
        if ((st = build_tables(*m, b->d_models, b->stream)) != BTX_OK) break;
      if (st != BTX_OK || (st = set_face_lds(b->tsize, f, face_lds(*cls[0]))) != BTX_OK) break;
      float ms = 0.f;
      for (int rep = 0; rep < 4 && st == BTX_OK; ++rep) {
        if (rep == 1) HIP_TRY(hipEventRecord(e0, b->stream));
        for (Model *m : cls) {
          st = launch_faces(f, b->tsize, b->d_models, m->d_fitems, (int)m->g.faces.size(), face_threads(*m),
                            face_lds(*m), b->parity, b->stream);
          if (st != BTX_OK) break;
        }
      }
      if (st != BTX_OK) break;
      HIP_TRY(hipEventRecord(e1, b->stream));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; best_nch = nch; }
    }
    cache.emplace_back(key, best_nch);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (Model &m : b->models) b->h_models[m.index].tally = tsave[m.index];
  if (st != BTX_OK) return st;
  for (Model &m : b->models) {
    if (m.shape.gtab || b->tsize == 8) continue;     // tables through the caches, or FP64: as created
    const int nch = lookup(tune_key(m)) ? lookup(tune_key(m)) : 8;
    set_shape(b, m, make_shape(m.g.prec, m.g.ndir, m.g.ne, nch));
  }
  if ((st = upload_descriptors(b)) != BTX_OK) return st;
  for (Model &m : b->models)
    if ((st = build_tables(m, b->d_models, b->stream)) != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(b->stream));
  write_cache(b->tune_path, cache);
  if ((st = build_groups(b)) != BTX_OK) return st;
  b->tuned = true;
  return BTX_OK;
}

// one step of every model: one face launch per shape group, one zone launch
btx_status batch_launch(btx_batch *b, int parity, hipStream_t s)
{
  for (const BatchGroup &gr : b->groups) {
    btx_status st = launch_faces(gr.shape, b->tsize, b->d_models, b->d_gitems + gr.first, gr.count, gr.threads,
                                 gr.lds, parity, s);
    if (st != BTX_OK) return st;
  }
  int rows = 1, dirs = 0;
  for (const Model &m : b->models) {
    rows = std::max(rows, m.g.ns * m.g.ne);
    dirs = std::max(dirs, m.g.ndir);
  }
  return launch_zones(b->tsize, b->d_models, b->d_zitems, b->nz_all, rows, parity, s, dirs);
}

// Level-sorted work lists of a batch with time levels: per face-shape group
// the (model, face) items by the level of the face's finer zone, and every
// (model, zone) item by its zone's level, with the counts up to each level.
btx_status build_lts_lists(btx_batch *b)
{
  int L = 0;
  for (const Model &m : b->models) L = std::max(L, m.lmax);
  std::vector<int2> fit, zit;
  b->gf_lev.assign(b->groups.size(), std::vector<int>(L + 1, 0));
  std::vector<int> first(b->groups.size());
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const BatchGroup &gr = b->groups[gi];
    std::vector<std::pair<int, int2>> v;
    for (const Model &m : b->models) {
      if (!(m.shape == gr.shape)) continue;
      for (size_t f = 0; f < m.g.faces.size(); ++f) {
        const int lv = std::min(m.lev[m.g.faces[f].L.z], m.lev[m.g.faces[f].R.z]);
        v.emplace_back(lv, make_int2(m.index, (int)f));
      }
    }
    std::stable_sort(v.begin(), v.end(), [](const std::pair<int, int2> &x, const std::pair<int, int2> &y) {
      return x.first < y.first;
    });
    first[gi] = (int)fit.size();
    for (auto &e : v) {
      fit.push_back(e.second);
      for (int l = e.first; l <= L; ++l) ++b->gf_lev[gi][l];
    }
  }
  std::vector<std::pair<int, int2>> zv;
  for (const Model &m : b->models)
    for (int z = 0; z < m.g.nz; ++z) zv.emplace_back(m.lev[z], make_int2(m.index, z));
  std::stable_sort(zv.begin(), zv.end(), [](const std::pair<int, int2> &x, const std::pair<int, int2> &y) {
    return x.first < y.first;
  });
  b->z_lev.assign(L + 1, 0);
  for (auto &e : zv) {
    zit.push_back(e.second);
    for (int l = e.first; l <= L; ++l) ++b->z_lev[l];
  }
  if (b->d_gitems_lts) { (void)hipFree(b->d_gitems_lts); b->d_gitems_lts = nullptr; }
  if (b->d_zitems_lts) { (void)hipFree(b->d_zitems_lts); b->d_zitems_lts = nullptr; }
  btx_status st = upload(&b->d_gitems_lts, fit.data(), fit.size());
  if (st != BTX_OK) return st;
  if ((st = upload(&b->d_zitems_lts, zit.data(), zit.size())) != BTX_OK) return st;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) b->groups[gi].first_lts = first[gi];
  b->lts_L = L;
  b->lts_dirty = false;
  return BTX_OK;
}

// One step of a batch with time levels: 2^L substeps; at substep k the faces
// whose finer zone starts a step and then the zones whose step ends
btx_status batch_launch_lts(btx_batch *b, hipStream_t s)
{
  const int L = b->lts_L;
  int rows = 1, dirs = 0;
  for (const Model &m : b->models) {
    rows = std::max(rows, m.g.ns * m.g.ne);
    dirs = std::max(dirs, m.g.ndir);
  }
  for (int k = 0; k < (1 << L); ++k) {
    const int lf = k == 0 ? L : std::min(L, __builtin_ctz(k));
    const int lz = std::min(L, __builtin_ctz(k + 1));
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const BatchGroup &gr = b->groups[gi];
      btx_status st = launch_faces(gr.shape, b->tsize, b->d_models, b->d_gitems_lts + gr.first_lts,
                                   b->gf_lev[gi][lf], gr.threads, gr.lds, 0, s, k);
      if (st != BTX_OK) return st;
    }
    btx_status st = launch_zones(b->tsize, b->d_models, b->d_zitems_lts, b->z_lev[lz], rows, 0, s, dirs);
    if (st != BTX_OK) return st;
  }
  return BTX_OK;
}

// the step of each parity captured once as a graph on the library's stream
btx_status capture_graphs(btx_batch *b)
{
  for (int p = 0; p < 2; ++p) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    btx_status st = batch_launch(b, p, b->cap);
    hipError_t he = hipStreamEndCapture(b->cap, &g);
    if (st != BTX_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (he != hipSuccess) return fail(BTX_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
    he = hipGraphInstantiate(&b->exec[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) return fail(BTX_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  }
  return BTX_OK;
}

}  // namespace

// ---------------------------------------------------------------- the ABI

extern "C" {

const char *btx_last_error(void) { return g_err.c_str(); }

btx_status btx_create(const btx_grid_desc *d, int hip_device, void *hip_stream, btx_ctx **out)
{
  if (!d || !out) return fail(BTX_E_INVAL, "null argument");
  *out = nullptr;
  btx_status st = validate_desc(d);
  if (st != BTX_OK) return st;
  HIP_TRY(hipSetDevice(hip_device));
  size_t cap = 0;
  if ((st = device_lds_cap(hip_device, &cap)) != BTX_OK) return st;
  btx_ctx *c = new btx_ctx();
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  double *scr = nullptr;
  if ((st = scratch_base(hip_device, &scr)) != BTX_OK) return st;
  if ((st = model_init(c->m, d, 0, cap)) != BTX_OK) { delete c; return st; }
  c->h_model = model_dev(c->m, 0.0);
  if ((st = upload(&c->d_model, &c->h_model, 1)) != BTX_OK) { free_ctx(c); return st; }
  if ((st = set_face_lds(c->m.tsize, c->m.shape, face_lds(c->m))) != BTX_OK) { free_ctx(c); return st; }
  c->ev.resize(3 * 256);
  for (auto &e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) { free_ctx(c); return fail(BTX_E_DEVICE, "hipEventCreate failed"); }
  *out = c;
  return BTX_OK;
}

btx_status btx_set_background(btx_ctx *c, const btx_background *bg)
{
  if (!c) return fail(BTX_E_INVAL, "null argument");
  btx_status st = check_background(c->m, bg);
  if (st != BTX_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if ((st = upload_background(c->m, bg, c->stream)) != BTX_OK) return st;
  if ((st = build_tables(c->m, c->d_model, c->stream)) != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->m.have_bg = true;
  return BTX_OK;
}

btx_status btx_update_background(btx_ctx *c, const btx_background *bg)
{
  if (!c) return fail(BTX_E_INVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device));
  return model_update_background(c->m, bg, c->d_model, c->parity, c->stream);
}

btx_status btx_max_dt(const btx_ctx *c, double cfl, double *dt_out)
{
  if (!c || !dt_out) return fail(BTX_E_INVAL, "null argument");
  if (!(cfl > 0.0)) return fail(BTX_E_INVAL, "cfl must be positive");
  *dt_out = c->m.dt_max1 * cfl;
  return BTX_OK;
}

btx_status btx_set_state(btx_ctx *c, const void *f, int is_device_ptr)
{
  if (!c || !f) return fail(BTX_E_INVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device));
  return model_set_state(c->m, c->parity, f, is_device_ptr, c->stream);
}

btx_status btx_get_state(btx_ctx *c, void *f, int is_device_ptr)
{
  if (!c || !f) return fail(BTX_E_INVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device));
  return model_get_state(c->m, c->parity, f, is_device_ptr, c->stream);
}

btx_status btx_step(btx_ctx *c, double dt, int32_t n_steps)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  if (!c->m.have_bg || !c->m.have_state) return fail(BTX_E_STATE, "background and state must be set");
  if (n_steps < 0) return fail(BTX_E_INVAL, "n_steps must be >= 0");
  btx_status st = check_dt(c->m, dt);
  if (st != BTX_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  for (int t = 0; t < n_steps; ++t)
    if ((st = ctx_step(c, dt)) != BTX_OK) return st;
  return BTX_OK;
}

btx_status btx_time_levels(const btx_ctx *c, int32_t max_level, int32_t *levels)
{
  if (!c || !levels) return fail(BTX_E_INVAL, "null argument");
  if (max_level < 0 || max_level > 16) return fail(BTX_E_INVAL, "max_level must be in 0..16");
  std::vector<int> lev;
  assign_levels(c->m.g, max_level, lev);
  for (int z = 0; z < c->m.g.nz; ++z) levels[z] = lev[z];
  return BTX_OK;
}

btx_status btx_set_time_levels(btx_ctx *c, const int32_t *levels)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  btx_status st = model_set_levels(c->m, levels, c->parity, c->stream);
  c->h_model = model_dev(c->m, c->h_model.dt);
  HIP_TRY(hipMemcpy(c->d_model, &c->h_model, sizeof(ModelDev), hipMemcpyHostToDevice));
  return st;
}

btx_status btx_moments(btx_ctx *c, double *zone_moments, double *totals)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  return model_moments(c->m, c->d_model, c->parity, zone_moments, totals, c->stream);
}

btx_status btx_moments_device(btx_ctx *c, double *zone_moments, double *totals)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  double *scr = nullptr;
  btx_status st = scratch_base(c->device, &scr);
  if (st != BTX_OK) return st;
  return model_moments_device(c->m, c->d_model, c->parity, zone_moments, totals, scr, c->stream);
}

btx_status btx_source_terms(btx_ctx *c, double *q)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  return model_source_terms(c->m, q, c->stream);
}

btx_status btx_timing(btx_ctx *c, int enable, double *ms, int64_t *launches, int reset)
{
  if (!c) return fail(BTX_E_INVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  for (size_t k = 0; k + 3 <= c->ev_used; k += 3) {
    HIP_TRY(hipEventSynchronize(c->ev[k + 2]));
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, c->ev[k], c->ev[k + 1]));
    HIP_TRY(hipEventElapsedTime(&b, c->ev[k + 1], c->ev[k + 2]));
    c->t_ms[0] += a; c->t_ms[1] += b;
    c->t_n[0] += 1; c->t_n[1] += 1;
  }
  c->ev_used = 0;
  if (ms) { ms[0] = c->t_ms[0]; ms[1] = c->t_ms[1]; }
  if (launches) { launches[0] = c->t_n[0]; launches[1] = c->t_n[1]; }
  if (reset) { c->t_ms[0] = c->t_ms[1] = 0.0; c->t_n[0] = c->t_n[1] = 0; }
  c->timing = enable != 0;
  return BTX_OK;
}

btx_status btx_destroy(btx_ctx *c)
{
  if (!c) return BTX_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_ctx(c);
  return BTX_OK;
}

btx_status btx_batch_create(const btx_grid_desc *descs, int32_t n_models, int hip_device, void *hip_stream,
                            const char *tune_cache_path, btx_batch **out)
{
  if (!descs || !out || n_models < 1) return fail(BTX_E_INVAL, "null argument or no models");
  *out = nullptr;
  for (int i = 0; i < n_models; ++i) {
    btx_status st = validate_desc(&descs[i]);
    if (st != BTX_OK) return fail(st, "model " + std::to_string(i) + ": " + g_err);
    if (descs[i].precision != descs[0].precision)
      return fail(BTX_E_INVAL, "all models of a batch share one precision");
  }
  HIP_TRY(hipSetDevice(hip_device));
  size_t cap = 0;
  btx_status st = device_lds_cap(hip_device, &cap);
  if (st != BTX_OK) return st;
  btx_batch *b = new btx_batch();
  b->device = hip_device;
  b->stream = (hipStream_t)hip_stream;
  b->tsize = descs[0].precision == BTX_PREC_FP64 ? 8 : 4;
  b->tune_path = tune_cache_path ? tune_cache_path : "";
  b->models.resize(n_models);
  std::vector<int2> zit;
  for (int i = 0; i < n_models; ++i) {
    if ((st = model_init(b->models[i], &descs[i], i, cap)) != BTX_OK) {
      std::string why = g_err;
      free_batch(b);
      return fail(st, "model " + std::to_string(i) + ": " + why);
    }
    b->h_models.push_back(model_dev(b->models[i], 0.0));
    for (int z = 0; z < b->models[i].g.nz; ++z) zit.push_back(make_int2(i, z));
  }
  b->nz_all = (int)zit.size();
  if ((st = upload(&b->d_models, b->h_models.data(), b->h_models.size())) != BTX_OK ||
      (st = upload(&b->d_zitems, zit.data(), zit.size())) != BTX_OK) {
    free_batch(b);
    return st;
  }
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    free_batch(b);
    return fail(BTX_E_DEVICE, "hipStreamCreateWithFlags failed");
  }
  *out = b;
  return BTX_OK;
}

btx_status btx_batch_set_background(btx_batch *b, int32_t model, const btx_background *bg)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  Model &m = b->models[model];
  btx_status st = check_background(m, bg);
  if (st != BTX_OK) return st;
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if ((st = upload_background(m, bg, b->stream)) != BTX_OK) return st;
  if ((st = build_tables(m, b->d_models, b->stream)) != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(b->stream));
  m.have_bg = true;
  return BTX_OK;
}

btx_status btx_batch_update_background(btx_batch *b, int32_t model, const btx_background *bg)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_update_background(b->models[model], bg, b->d_models, b->parity, b->stream);
}

btx_status btx_batch_max_dt(const btx_batch *b, int32_t model, double cfl, double *dt_out)
{
  if (!b || !dt_out || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad argument");
  if (!(cfl > 0.0)) return fail(BTX_E_INVAL, "cfl must be positive");
  *dt_out = b->models[model].dt_max1 * cfl;
  return BTX_OK;
}

btx_status btx_batch_set_state(btx_batch *b, int32_t model, const void *f, int is_device_ptr)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_set_state(b->models[model], b->parity, f, is_device_ptr, b->stream);
}

btx_status btx_batch_get_state(btx_batch *b, int32_t model, void *f, int is_device_ptr)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_get_state(b->models[model], b->parity, f, is_device_ptr, b->stream);
}

btx_status btx_batch_step(btx_batch *b, const double *dt_per_model, int32_t n_steps)
{
  if (!b || !dt_per_model) return fail(BTX_E_INVAL, "null argument");
  if (n_steps < 0) return fail(BTX_E_INVAL, "n_steps must be >= 0");
  bool changed = false;
  for (Model &m : b->models) {
    if (!m.have_bg || !m.have_state)
      return fail(BTX_E_STATE, "model " + std::to_string(m.index) + ": background and state must be set");
    btx_status st = check_dt(m, dt_per_model[m.index]);
    if (st != BTX_OK) return fail(st, "model " + std::to_string(m.index) + ": " + g_err);
    changed |= b->h_models[m.index].dt != dt_per_model[m.index];
  }
  HIP_TRY(hipSetDevice(b->device));
  btx_status st = BTX_OK;
  if (changed) {
    for (Model &m : b->models) b->h_models[m.index].dt = dt_per_model[m.index];
    if ((st = upload_descriptors(b)) != BTX_OK) return st;
  }
  if (!b->tuned && (st = tune(b)) != BTX_OK) return st;
  if (b->lts) {                                      // time levels: in place, no graphs
    if (b->lts_dirty && (st = build_lts_lists(b)) != BTX_OK) return st;
    for (int t = 0; t < n_steps; ++t)
      if ((st = batch_launch_lts(b, b->stream)) != BTX_OK) return st;
    return BTX_OK;
  }
  if (b->use_graph && !b->exec[0] && (st = capture_graphs(b)) != BTX_OK) return st;
  for (int t = 0; t < n_steps; ++t) {
    if (b->use_graph) HIP_TRY(hipGraphLaunch(b->exec[b->parity], b->stream));
    else if ((st = batch_launch(b, b->parity, b->stream)) != BTX_OK) return st;
    b->parity ^= 1;
  }
  return BTX_OK;
}

btx_status btx_batch_use_graph(btx_batch *b, int enable)
{
  if (!b) return fail(BTX_E_INVAL, "null batch");
  b->use_graph = enable != 0;
  return BTX_OK;
}

btx_status btx_batch_shape(const btx_batch *b, int32_t model, int32_t *items_per_direction,
                           int32_t *groups_per_item)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  if (items_per_direction) *items_per_direction = b->models[model].shape.nch;
  if (groups_per_item) *groups_per_item = b->models[model].shape.ce;
  return BTX_OK;
}

btx_status btx_batch_moments(btx_batch *b, int32_t model, double *zone_moments, double *totals)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_moments(b->models[model], b->d_models, b->parity, zone_moments, totals, b->stream);
}

btx_status btx_batch_source_terms(btx_batch *b, int32_t model, double *q)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_source_terms(b->models[model], q, b->stream);
}

btx_status btx_batch_time_levels(const btx_batch *b, int32_t model, int32_t max_level, int32_t *levels)
{
  if (!b || !levels) return fail(BTX_E_INVAL, "null argument");
  if (model < 0 || model >= (int32_t)b->models.size()) return fail(BTX_E_INVAL, "model index out of range");
  if (max_level < 0 || max_level > 16) return fail(BTX_E_INVAL, "max_level must be in 0..16");
  std::vector<int> lev;
  assign_levels(b->models[model].g, max_level, lev);
  for (int z = 0; z < b->models[model].g.nz; ++z) levels[z] = lev[z];
  return BTX_OK;
}

btx_status btx_batch_set_time_levels(btx_batch *b, int32_t model, const int32_t *levels)
{
  if (!b) return fail(BTX_E_INVAL, "null batch");
  if (model < 0 || model >= (int32_t)b->models.size()) return fail(BTX_E_INVAL, "model index out of range");
  if (levels)
    for (int z = 0; z < b->models[model].g.nz; ++z)
      if (levels[z] < 0 || levels[z] > 16) return fail(BTX_E_INVAL, "time levels must be in 0..16");
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipStreamSynchronize(b->stream));
  drop_graphs(b);
  // every model steps in place from now on: its current state into buffer 0
  btx_status st = BTX_OK;
  for (Model &m : b->models) {
    int p = b->parity;
    const std::vector<int32_t> zeros(m.g.nz, 0);
    const int32_t *lv = m.index == model ? (levels ? levels : zeros.data())
                                         : (m.lev.empty() ? zeros.data() : nullptr);
    if (lv) st = model_set_levels(m, lv, p, b->stream);
    else if (p == 1)
      HIP_TRY(hipMemcpy(m.d_f[0], m.d_f[1], (size_t)m.g.nz * m.g.ns * m.g.ne * m.g.ndir * m.tsize,
                        hipMemcpyDeviceToDevice));
    if (st != BTX_OK) return st;
  }
  b->parity = 0;
  for (Model &m : b->models) {
    const FaceShape sh = m.shape;
    const double dt = b->h_models[m.index].dt;
    b->h_models[m.index] = model_dev(m, dt);
    b->h_models[m.index].g.nch = sh.nch;
    b->h_models[m.index].g.ce = sh.ce;
  }
  if ((st = upload_descriptors(b)) != BTX_OK) return st;
  b->lts = true;
  b->lts_dirty = true;
  return BTX_OK;
}

btx_status btx_batch_destroy(btx_batch *b)
{
  if (!b) return BTX_OK;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  free_batch(b);
  return BTX_OK;
}

}  // extern "C"
