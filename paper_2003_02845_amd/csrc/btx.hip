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

#include "btx_dev.h"

using btx::FaceDesc;
using btx::FaceShape;
using btx::SideDesc;

namespace {

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

}  // namespace

// ---------------------------------------------------------------- host side

// ---------------------------------------------------------------- host side

namespace {

// face workgroups that fill the device, one per CU (256 compute units)
constexpr int kFillFaces = 256;

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

const void *face_fn(size_t tsize, const FaceShape &f)
{
  return tsize == 8 ? btx::face_fn_f64(f) : btx::face_fn_f32(f);
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
  double *d_rconst = nullptr;        // q^k (k = -128 .. 128), cos and sin of the Phi nodes
  double *d_vr = nullptr, *d_vth = nullptr, *d_vph = nullptr, *d_alp = nullptr, *d_psi = nullptr;
  void *d_ka = nullptr, *d_ks = nullptr, *d_feq = nullptr, *d_f[2] = { nullptr, nullptr }, *d_dN = nullptr;
  char *d_tabs = nullptr;
  FaceAux *d_aux = nullptr;
  double *d_tally = nullptr, *d_zm = nullptr, *d_ze = nullptr, *d_stage = nullptr, *d_q = nullptr;
  double *d_nbg = nullptr;           // new v_r, v_theta, v_phi, alpha, psi of a background update
  int *d_err = nullptr;              // result of the device-side check of a background
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
  if (d->geometry == BTX_GEOM_COLUMN && !(d->dphi >= 0.0 && d->dphi <= 0.5 * kPi))
    return fail(BTX_E_INVAL, "a column's width dphi must be in [0, pi/2]");
  return BTX_OK;
}

void model_free(Model &m)
{
  void *ptrs[] = { m.d_rconst, m.d_mu, m.d_Phi, m.d_dOm, m.d_nvec, m.d_G, m.d_eps, m.d_vol, m.d_vr, m.d_vth, m.d_vph,
                   m.d_alp, m.d_psi, m.d_ka, m.d_ks, m.d_feq, m.d_f[0], m.d_f[1], m.d_dN, m.d_tally,
                   m.d_zm, m.d_ze, m.d_stage, m.d_faces, m.d_zf, m.d_tabs, m.d_aux, m.d_fitems, m.d_zitems,
                   m.d_nbg, m.d_q, m.d_zlev, m.d_fitems_lts, m.d_zitems_lts, m.d_bface, m.d_err };
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
  // the table build: one wave per table where the face kernel holds its
  // tables in LDS (the scratch of eight waves then fits too), else one
  // table at a time in global memory
  m.tab_lds = m.shape.gtab ? align16(5 * sizeof(FrameP)) + align16(scratch_bytes(g.ndir, m.tsize, 1)) +
                                 align16((size_t)g.nmu * 8) + align16((size_t)kQpow * 8) +
                                 align16((size_t)2 * g.nphi * 8)
                           : table_w_lds_bytes(g.ndir, g.nmu, g.nphi, m.tsize, 5 * sizeof(FrameP));
  if (m.tab_lds > lds_cap) return fail(BTX_E_UNSUPPORTED, "table build needs too much LDS");
  const size_t nz = g.nz, blk = (size_t)g.ns * g.ne * g.ndir, nk = nz * g.ns * g.ne, nf = g.faces.size();
  std::vector<int2> fit(nf), zit(nz);
  for (size_t k = 0; k < nf; ++k) fit[k] = make_int2(index, (int)k);
  for (size_t k = 0; k < nz; ++k) zit[k] = make_int2(index, (int)k);
  std::vector<double> zero(nz, 0.0), one(nz, 1.0);
#define TRY(x) do { st = (x); if (st != BTX_OK) { model_free(m); return st; } } while (0)
  TRY(upload(&m.d_mu, g.mu.data(), g.mu.size()));
  TRY(upload(&m.d_Phi, g.Phi.data(), g.Phi.size()));
  {
    std::vector<double> rc(kQpow + 2 * g.nphi);
    for (int k = -128; k <= 128; ++k) rc[k + 128] = std::exp(k * g.lnq);
    for (int k = 0; k < g.nphi; ++k) {
      rc[kQpow + k] = std::cos(g.Phi[k]);
      rc[kQpow + g.nphi + k] = std::sin(g.Phi[k]);
    }
    TRY(upload(&m.d_rconst, rc.data(), rc.size()));
  }
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
      !dmalloc(&m.d_dN, nf * 2 * blk * m.tsize) ||
      !dmalloc((void **)&m.d_tally, nf * g.ns * 8) ||
      !dmalloc((void **)&m.d_zm, nz * g.ns * 5 * 8) || !dmalloc((void **)&m.d_ze, nz * g.ns * 8) ||
      !dmalloc((void **)&m.d_stage, nk * 8) || !dmalloc((void **)&m.d_nbg, nz * 5 * 8) ||
      !dmalloc((void **)&m.d_q, nz * 5 * 8) || !dmalloc((void **)&m.d_err, 16) ||
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
  d.qpow = m.d_rconst; d.cphi = m.d_rconst + kQpow; d.sphi = m.d_rconst + kQpow + g.nphi;
  d.iq1 = 1.0 / (g.q - 1.0);
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

// Checks a background whose arrays are in device memory: every array must be
// device (or managed) memory of the model's device; the values are checked
// on the device (one synchronisation).
btx_status check_background_device(Model &m, const btx_background *bg, int device, hipStream_t s)
{
  if (!bg) return fail(BTX_E_INVAL, "null argument");
  if (!bg->v_r || !bg->v_theta || !bg->alpha || !bg->psi || !bg->kappa_a || !bg->kappa_s || !bg->f_eq)
    return fail(BTX_E_INVAL, "null background array");
  const double *arrs[8] = { bg->v_r, bg->v_theta, bg->alpha, bg->psi, bg->kappa_a, bg->kappa_s, bg->f_eq, bg->v_phi };
  for (const double *p : arrs) {
    if (!p) continue;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.device != device ||
        (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
      (void)hipGetLastError();
      return fail(BTX_E_INVAL, "background arrays must be device memory of the context's device");
    }
  }
  const size_t nz = m.g.nz, nk = nz * m.g.ns * m.g.ne;
  HIP_TRY(hipMemsetAsync(m.d_err, 0, sizeof(int), s));
  hipLaunchKernelGGL(bg_check_kernel, dim3(1024), dim3(256), 0, s, bg->v_r, bg->v_theta, bg->v_phi, bg->alpha,
                     bg->psi, nz, bg->kappa_a, bg->kappa_s, bg->f_eq, nk, m.d_err);
  HIP_TRY(hipGetLastError());
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, m.d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h & 1) return fail(BTX_E_INVAL, "background velocity/metric out of range (device arrays)");
  if (h & 2) return fail(BTX_E_INVAL, "opacities must be finite and >= 0 (device arrays)");
  return BTX_OK;
}

// copies the background into the model's buffers (storage precision); the
// arrays are host memory (synchronous copies) or, with on_device, device
// memory of the model's device (stream-ordered copies on s)
btx_status upload_background(Model &m, const btx_background *bg, hipStream_t s, bool on_device = false)
{
  const btx::Grid &g = m.g;
  const size_t nz = g.nz, nk = nz * g.ns * g.ne;
  auto copy = [&](void *dst, const void *src, size_t bytes) -> btx_status {
    if (on_device) HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
    else HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return BTX_OK;
  };
  btx_status st;
  const double *zsrc[4] = { bg->v_r, bg->v_theta, bg->alpha, bg->psi };
  double *zdst[4] = { m.d_vr, m.d_vth, m.d_alp, m.d_psi };
  for (int k = 0; k < 4; ++k)
    if ((st = copy(zdst[k], zsrc[k], nz * 8)) != BTX_OK) return st;
  if (bg->v_phi) {
    if ((st = copy(m.d_vph, bg->v_phi, nz * 8)) != BTX_OK) return st;
  } else {
    HIP_TRY(on_device ? hipMemsetAsync(m.d_vph, 0, nz * 8, s) : hipMemset(m.d_vph, 0, nz * 8));
  }
  const double *src[3] = { bg->kappa_a, bg->kappa_s, bg->f_eq };
  void *dst[3] = { m.d_ka, m.d_ks, m.d_feq };
  for (int k = 0; k < 3; ++k) {
    if (m.tsize == 8) {
      if ((st = copy(dst[k], src[k], nk * 8)) != BTX_OK) return st;
    } else {
      const double *from = src[k];
      if (!on_device) {
        HIP_TRY(hipMemcpy(m.d_stage, src[k], nk * 8, hipMemcpyHostToDevice));
        from = m.d_stage;
      }
      hipLaunchKernelGGL((cast_kernel<float>), dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s,
                         from, (float *)dst[k], nk);
      HIP_TRY(hipGetLastError());
      if (!on_device) HIP_TRY(hipStreamSynchronize(s));
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
  // one wave per table (m.tab_lds is sized for the kernel that runs)
  const void *tk = m.shape.gtab
                       ? (m.tsize == 8 ? (const void *)table_kernel_g<double> : (const void *)table_kernel_g<float>)
                       : (m.tsize == 8 ? (const void *)table_kernel_w<double> : (const void *)table_kernel_w<float>);
  btx_status st = raise_lds_limit(tk, m.tab_lds);
  if (st != BTX_OK) return st;
  const int2 *items = m.d_fitems;
  void *args[] = { &d_models, &items };
  // 512 threads: eight waves, one per table (the global-memory build was
  // measured at 21 ms against 26 ms with 384 threads and 32 ms with 256)
  HIP_TRY(hipLaunchKernel(tk, dim3(nf), dim3(512), args, m.tab_lds, s));
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

// zone kernel LDS: five FP64 row values per (species, group) row; per
// direction the weight 1/((1 + v.n) dOmega), dOmega and n (five FP64)
size_t zone_lds_bytes(int rows, int dirs) { return ((size_t)std::max(rows, 1) * 5 + (size_t)dirs * 5) * sizeof(double); }

btx_status launch_zones(size_t tsize, const ModelDev *d_models, const int2 *items, int n, int max_rows,
                        int parity, hipStream_t s, int max_dirs)
{
  if (n == 0) return BTX_OK;
  const void *zk = max_dirs > 256 ? (tsize == 8 ? (const void *)zone_kernel<double, 16> : (const void *)zone_kernel<float, 16>)
                                  : (tsize == 8 ? (const void *)zone_kernel<double, 4> : (const void *)zone_kernel<float, 4>);
  btx_status st = raise_lds_limit(zk, zone_lds_bytes(max_rows, max_dirs));
  if (st != BTX_OK) return st;
  void *args[] = { &d_models, &items, &parity };
  HIP_TRY(hipLaunchKernel(zk, dim3(n), dim3(256), args, zone_lds_bytes(max_rows, max_dirs), s));
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
// on_device: every array of bg is device memory of the model's device.
btx_status model_update_background(Model &m, const btx_background *bg, const ModelDev *d_models, int parity,
                                   hipStream_t s, int device = 0, bool on_device = false)
{
  btx_status st = on_device ? check_background_device(m, bg, device, s) : check_background(m, bg);
  if (st != BTX_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  if (m.have_bg && m.have_state) {
    const size_t nz = m.g.nz;
    // host arrays: synchronous copies; device arrays: stream-ordered on s
    auto copy = [&](double *dst, const double *src) -> btx_status {
      if (on_device) HIP_TRY(hipMemcpyAsync(dst, src, nz * 8, hipMemcpyDeviceToDevice, s));
      else HIP_TRY(hipMemcpy(dst, src, nz * 8, hipMemcpyHostToDevice));
      return BTX_OK;
    };
    if ((st = copy(m.d_nbg, bg->v_r)) != BTX_OK || (st = copy(m.d_nbg + nz, bg->v_theta)) != BTX_OK ||
        (st = copy(m.d_nbg + 3 * nz, bg->alpha)) != BTX_OK || (st = copy(m.d_nbg + 4 * nz, bg->psi)) != BTX_OK)
      return st;
    if (bg->v_phi) {
      if ((st = copy(m.d_nbg + 2 * nz, bg->v_phi)) != BTX_OK) return st;
    } else {
      HIP_TRY(on_device ? hipMemsetAsync(m.d_nbg + 2 * nz, 0, nz * 8, s) : hipMemset(m.d_nbg + 2 * nz, 0, nz * 8));
    }
    const void *tk = m.tsize == 8 ? (const void *)time_remap_kernel<double> : (const void *)time_remap_kernel<float>;
    const size_t lds = time_lds_bytes(m.g.ndir, m.g.ne, m.tsize);
    if ((st = raise_lds_limit(tk, lds)) != BTX_OK) return st;
    const int2 *items = m.d_zitems;
    const double *nbg = m.d_nbg;
    void *args[] = { &d_models, &items, &parity, &nbg };
    HIP_TRY(hipLaunchKernel(tk, dim3((unsigned)nz), dim3(256), args, lds, s));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
  }
  if ((st = upload_background(m, bg, s, on_device)) != BTX_OK) return st;
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

// Time levels (local time stepping, Sec. 5): zone z takes 2^l global steps
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
  // side streams and events of the captured graph's parallel branches (one
  // face launch per shape group each), created with the first capture
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
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
  hipGraphExec_t exec_lts = nullptr;  // the time-level step (2^L substeps), once captured
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
  if (b->exec_lts) { (void)hipGraphExecDestroy(b->exec_lts); b->exec_lts = nullptr; }
}

void free_batch(btx_batch *b)
{
  drop_graphs(b);
  for (Model &m : b->models) model_free(m);
  void *ptrs[] = { b->d_models, b->d_gitems, b->d_zitems, b->d_tscratch, b->d_gitems_lts, b->d_zitems_lts };
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (hipStream_t x : b->side) (void)hipStreamDestroy(x);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
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

// Groups models by face shape (and, without time levels, workgroup size)
// and uploads the grouped face items.
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
      // one launch per face shape and thread count: a model with fewer
      // directions than the group's widest would leave workgroup lanes idle
      // (1.75 against 2.14 ms per step of the 64-model batch).  With time
      // levels a step is many small launches, and fewer of them pay more:
      // one per shape (11.4 against 21.2 ms per 16 substeps).
      if (done[j] || !(m.shape == gr.shape) || (!b->lts && face_threads(m) != face_threads(b->models[i])))
        continue;
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
  if (b->exec_lts) { (void)hipGraphExecDestroy(b->exec_lts); b->exec_lts = nullptr; }
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

// One step as graph branches: the face launches of the shape groups run side
// by side (each writes only its own faces' changes), joined before the zone
// launch.  Called while b->cap is being captured.
btx_status batch_launch_branches(btx_batch *b, int parity)
{
  const size_t ng = b->groups.size();
  HIP_TRY(hipEventRecord(b->ev[ng], b->cap));
  for (size_t gi = 0; gi < ng; ++gi) {
    const BatchGroup &gr = b->groups[gi];
    HIP_TRY(hipStreamWaitEvent(b->side[gi], b->ev[ng], 0));
    btx_status st = launch_faces(gr.shape, b->tsize, b->d_models, b->d_gitems + gr.first, gr.count, gr.threads,
                                 gr.lds, parity, b->side[gi]);
    if (st != BTX_OK) return st;
    HIP_TRY(hipEventRecord(b->ev[gi], b->side[gi]));
    HIP_TRY(hipStreamWaitEvent(b->cap, b->ev[gi], 0));
  }
  int rows = 1, dirs = 0;
  for (const Model &m : b->models) {
    rows = std::max(rows, m.g.ns * m.g.ne);
    dirs = std::max(dirs, m.g.ndir);
  }
  return launch_zones(b->tsize, b->d_models, b->d_zitems, b->nz_all, rows, parity, b->cap, dirs);
}

// side streams and events for the branches of the captured graphs
btx_status branch_streams(btx_batch *b)
{
  const size_t ng = b->groups.size();
  while (b->side.size() < ng) {                        // default priority, like every stream here
    hipStream_t x;
    HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    b->side.push_back(x);
  }
  while (b->ev.size() < ng + 1) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->ev.push_back(e);
  }
  return BTX_OK;
}

// The time-level step (2^L substeps, as batch_launch_lts) captured once as a
// graph: each substep's face launches as branches, joined before its zone
// launch.  Recaptured when the level lists change.
btx_status capture_lts_graph(btx_batch *b)
{
  btx_status st = branch_streams(b);
  if (st != BTX_OK) return st;
  const size_t ng = b->groups.size();
  const int L = b->lts_L;
  int rows = 1, dirs = 0;
  for (const Model &m : b->models) {
    rows = std::max(rows, m.g.ns * m.g.ne);
    dirs = std::max(dirs, m.g.ndir);
  }
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < (1 << L) && st == BTX_OK; ++k) {
    const int lf = k == 0 ? L : std::min(L, __builtin_ctz(k));
    const int lz = std::min(L, __builtin_ctz(k + 1));
    hipError_t he = hipEventRecord(b->ev[ng], b->cap);
    for (size_t gi = 0; gi < ng && st == BTX_OK && he == hipSuccess; ++gi) {
      const BatchGroup &gr = b->groups[gi];
      if (b->gf_lev[gi][lf] == 0) continue;
      he = hipStreamWaitEvent(b->side[gi], b->ev[ng], 0);
      if (he == hipSuccess)
        st = launch_faces(gr.shape, b->tsize, b->d_models, b->d_gitems_lts + gr.first_lts, b->gf_lev[gi][lf],
                          gr.threads, gr.lds, 0, b->side[gi], k);
      if (st == BTX_OK && he == hipSuccess) he = hipEventRecord(b->ev[gi], b->side[gi]);
      if (st == BTX_OK && he == hipSuccess) he = hipStreamWaitEvent(b->cap, b->ev[gi], 0);
    }
    if (he != hipSuccess && st == BTX_OK) st = fail(BTX_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(he));
    if (st == BTX_OK) st = launch_zones(b->tsize, b->d_models, b->d_zitems_lts, b->z_lev[lz], rows, 0, b->cap, dirs);
  }
  hipError_t he = hipStreamEndCapture(b->cap, &g);
  if (st != BTX_OK) { if (g) (void)hipGraphDestroy(g); return st; }
  if (he != hipSuccess) return fail(BTX_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
  he = hipGraphInstantiate(&b->exec_lts, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (he != hipSuccess) return fail(BTX_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  return BTX_OK;
}

// the step of each parity captured once as a graph on the library's stream
btx_status capture_graphs(btx_batch *b)
{
  btx_status bst = branch_streams(b);
  if (bst != BTX_OK) return bst;
  for (int p = 0; p < 2; ++p) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    btx_status st = batch_launch_branches(b, p);
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

btx_status btx_update_background_device(btx_ctx *c, const btx_background *bg)
{
  if (!c) return fail(BTX_E_INVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device));
  return model_update_background(c->m, bg, c->d_model, c->parity, c->stream, c->device, true);
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

btx_status btx_batch_update_background_device(btx_batch *b, int32_t model, const btx_background *bg)
{
  if (!b || model < 0 || model >= (int)b->models.size()) return fail(BTX_E_INVAL, "bad batch or model index");
  HIP_TRY(hipSetDevice(b->device));
  return model_update_background(b->models[model], bg, b->d_models, b->parity, b->stream, b->device, true);
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
  if (b->lts) {                                      // time levels: in place
    if (b->lts_dirty && (st = build_lts_lists(b)) != BTX_OK) return st;
    // a graph of 2^L substeps only up to 64 of them; deeper hierarchies launch directly
    const bool graph = b->use_graph && b->lts_L <= 6;
    if (graph && !b->exec_lts && (st = capture_lts_graph(b)) != BTX_OK) return st;
    for (int t = 0; t < n_steps; ++t) {
      if (graph) HIP_TRY(hipGraphLaunch(b->exec_lts, b->stream));
      else if ((st = batch_launch_lts(b, b->stream)) != BTX_OK) return st;
    }
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
  const bool regroup = !b->lts && b->tuned;          // groups by shape alone from now on
  b->lts = true;
  b->lts_dirty = true;
  if (regroup && (st = build_groups(b)) != BTX_OK) return st;
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
