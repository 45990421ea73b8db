// Host layer of the rates library: argument checks, zone-independent tables (quadrature
// nodes, angular-weight coefficients), a per-device table cache and the C entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vtx_rates.h"
#include "hmass_gen.h"
#include "hpoly_gen.h"
#include "vtx_internal.h"

namespace vtx {
namespace {

// ---------------------------------------------------------------------------------------
// Gauss rules. Nodes: eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// three-term recurrence (Golub-Welsch), found by Sturm-sequence bisection, then polished
// by Newton steps on the orthogonal polynomial; weights from the polynomial's
// derivative at the node, which keeps the tiny Laguerre weights accurate to full relative
// precision.

// Number of eigenvalues below x of the symmetric tridiagonal matrix (diag d, off-diagonal
// e[k] coupling rows k-1 and k): the count of negative pivots of the LDL^T factorisation of
// J - x I (Sylvester's law of inertia).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int neg = 0;
  double q = 1.0;
  for (size_t k = 0; k < d.size(); ++k) {
    const double off = (k > 0) ? e[k] * e[k] / q : 0.0;
    q = d[k] - x - off;
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++neg;
  }
  return neg;
}

// All eigenvalues, ascending, by bisection on the Sturm count inside the Gershgorin bounds.
bool tridiag_eigenvalues(std::vector<double>& d, const std::vector<double>& e) {
  const int n = (int)d.size();
  double lo = 0.0, hi = 0.0;
  for (int k = 0; k < n; ++k) {
    const double r = (k > 0 ? std::fabs(e[k]) : 0.0) + (k + 1 < n ? std::fabs(e[k + 1]) : 0.0);
    lo = (k == 0) ? d[k] - r : std::fmin(lo, d[k] - r);
    hi = (k == 0) ? d[k] + r : std::fmax(hi, d[k] + r);
  }
  std::vector<double> ev(n);
  for (int m = 0; m < n; ++m) {
    // smallest x with at least m + 1 eigenvalues below it
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 4e-16 * std::fmax(1.0, std::fabs(a) + std::fabs(b)); ++it) {
      const double c = 0.5 * (a + b);
      if (sturm_count(d, e, c) > m) b = c; else a = c;
    }
    ev[m] = 0.5 * (a + b);
  }
  d = ev;
  return true;
}

// Legendre P_n and P_{n-1} at x.
void legendre_pn(int n, double x, double& pn, double& pn1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    pn1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// Laguerre L_n and L_{n-1} at x.
void laguerre_ln(int n, double x, double& ln, double& ln1) {
  double l0 = 1.0, l1 = 1.0 - x;
  if (n == 0) {
    ln = 1.0;
    ln1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double l2 = ((2 * k + 1 - x) * l1 - k * l0) / (k + 1);
    l0 = l1;
    l1 = l2;
  }
  ln = l1;
  ln1 = l0;
}

// kind 0: Gauss-Legendre on [0, 1]; kind 1: Gauss-Laguerre, weights times exp(x).
bool gauss_rule(int kind, int n, double* x, double* w) {
  std::vector<double> d(n), e(n, 0.0);
  for (int k = 0; k < n; ++k) {
    if (kind == 0) {
      d[k] = 0.0;
      if (k > 0) e[k] = k / std::sqrt(4.0 * k * k - 1.0);
    } else {
      d[k] = 2.0 * k + 1.0;
      if (k > 0) e[k] = k;
    }
  }
  if (!tridiag_eigenvalues(d, e)) return false;
  const std::vector<double>& r = d;
  for (int k = 0; k < n; ++k) {
    double xx = r[k];
    double der = 0.0;
    for (int it = 0; it < 4; ++it) {
      double pn, pn1;
      if (kind == 0) {
        legendre_pn(n, xx, pn, pn1);
        der = n * (xx * pn - pn1) / (xx * xx - 1.0);
      } else {
        laguerre_ln(n, xx, pn, pn1);
        der = n * (pn - pn1) / xx;
      }
      const double dx = pn / der;
      xx -= dx;
      if (std::fabs(dx) <= 1e-16 * std::fabs(xx)) break;
    }
    double pn, pn1;
    if (kind == 0) {
      legendre_pn(n, xx, pn, pn1);
      der = n * (xx * pn - pn1) / (xx * xx - 1.0);
      x[k] = 0.5 * (xx + 1.0);
      w[k] = 1.0 / ((1.0 - xx * xx) * der * der);   // (2/((1-x^2)P'^2)) / 2
    } else {
      laguerre_ln(n, xx, pn, pn1);
      der = n * (pn - pn1) / xx;
      x[k] = xx;
      w[k] = std::exp(xx - std::log(xx) - 2.0 * std::log(std::fabs(der)));
    }
  }
  return true;
}

// ---------------------------------------------------------------------------------------
// Angular-weight coefficient tables (zone independent), prefactor G_F^2/(pi e_i e_j) folded in.
// Pieces on a bounded variable u in [0, 1] are stored in the degree-7 Bernstein basis,
// p(u) = sum_k g_k u^k (1 - u)^(7-k) (binomials folded into g_k): the basis functions are
// nonnegative, so the kernels' FP32 moment sums carry no cancellation and the sign changes
// of the l = 1 weights are resolved in the FP64 contraction with g_k.

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// monomial coefficients c[0..7] (in u) -> folded Bernstein coefficients g[0..7]
void mono_to_bernstein7(const double* c, double* g) {
  for (int k = 0; k <= 7; ++k) {
    double b = 0.0;
    for (int j = 0; j <= k; ++j) b += binom(k, j) / binom(7, j) * c[j];
    g[k] = b * binom(7, k);
  }
}

// Bernstein form of a low piece (exact E^3 factor): its k = 0..2 coefficients vanish
// exactly, and only k = 3..7 are stored.
bool low_piece(const double* mono, double* out5) {
  double g[8];
  mono_to_bernstein7(mono, g);
  if (g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0) return false;
  for (int k = 0; k < 5; ++k) out5[k] = g[k + 3];
  return true;
}

bool nes_coefficients(double e, double ep, NesCoef& C) {
  double lo[4][8], hi[4][3];
  vtx_hpoly_nes(e, ep, lo, hi);
  const double pref = kGF * kGF / (M_PI * e * ep);
  bool ok = true;
  for (int c = 0; c < 4; ++c) {
    double m[8];
    for (int d = 0; d < 8; ++d) m[d] = pref * lo[c][d];
    ok = low_piece(m, C.lo[c]) && ok;
    for (int d = 0; d < 3; ++d) C.hi[c][d] = pref * hi[c][d];
  }
  return ok;
}

// H^{P,I}_l(e_i, e_j, .): for e_i >= e_j the generator's S = I comps, else its S = II comps
// with the arguments swapped (H^{P,I}(a, b, E) = H^{P,II}(b, a, E)).
bool pair_coefficients(double ei, double ej, PairCoef& C) {
  double A[4][8], B[4][3], Cc[4][8];
  const bool ordered = ei >= ej;
  vtx_hpoly_pair(ordered ? ei : ej, ordered ? ej : ei, A, B, Cc);
  const double pref = kGF * kGF / (M_PI * ei * ej);
  bool ok = true;
  for (int l = 0; l < 2; ++l) {
    const int comp = ordered ? l : 2 + l;
    double a[8], c[8];
    for (int d = 0; d < 8; ++d) {
      a[d] = pref * A[comp][d];
      c[d] = pref * Cc[comp][d];
    }
    ok = low_piece(a, C.A[l]) && ok;
    ok = low_piece(c, C.C[l]) && ok;
    for (int d = 0; d < 3; ++d) C.B[l][d] = pref * B[comp][d];
  }
  return ok;
}

double bernstein_low(const double* g5, double u) {
  const double v = 1.0 - u;
  double s = 0.0;
  for (int k = 3; k <= 7; ++k) s += g5[k - 3] * std::pow(u, k) * std::pow(v, 7 - k);
  return s;
}

// Electron-mass weights of scattering task (e >= ep) and pair {e, ep}: the generator's Laurent
// coefficients times the prefactor, the third structure with its sign in the rates (minus for
// scattering, plus for the pair), and the rule's breakpoints that depend on the task only.
//   scattering kink E_k: root of P + P' = e + ep, (sqrt(om^2 + 4 e ep + w^2 m^2/(e ep)) - om)/2;
//   pair: E = (w -+ y)/2 with y = |e - ep| sqrt(1 - m^2/(e ep)), open when e ep > m^2.
void mass_coefficients(double e, double ep, bool pair, MassCoef& C) {
  std::memset(&C, 0, sizeof(C));
  const double m = kMe, w = e + ep, om = e - ep;
  if (pair)
    vtx_hmass_pair(e, ep, m, C.c, C.c3);
  else
    vtx_hmass_nes(e, ep, m, C.c, C.c3);
  const double pref = kGF * kGF / (M_PI * e * ep);
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < 16; ++k) C.c[c][k] *= pref;
  const double s3 = pair ? pref : -pref;
  for (int l = 0; l < 2; ++l)
    for (int k = 0; k < 3; ++k) C.c3[l][k] *= s3;
  if (!pair) {
    const double ek = 0.5 * (std::sqrt(om * om + 4.0 * e * ep + w * w * m * m / (e * ep)) - om);
    C.k0 = std::fmax(ek, m);
  } else {
    const bool open = e * ep > m * m && w > 2.0 * m;
    const double y = open ? std::fabs(om) * std::sqrt(1.0 - m * m / (e * ep)) : 0.0;
    C.k0 = 0.5 * (w - y);
    C.k1 = 0.5 * (w + y);
    C.support = open ? 1.0 : 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// Table cache

struct Plan {
  int device;
  int ne, nquad, rule;
  double sin2w;
  std::vector<double> eps, w;
  DevPlan dp;              // pointers into the device buffer below
  void* dbuf = nullptr;
};

std::mutex g_mu;
std::vector<std::unique_ptr<Plan>> g_plans;
int g_block = 256;           // threads per workgroup of the rate kernels (vtx_set_workgroup_waves)
std::vector<int> g_dev_ok;   // per device: 0 unknown, 1 gfx950, -1 other

void couplings(double s2w, double beta[3][2], double beta3[3]) {
  const double cve = 0.5 + 2.0 * s2w;
  beta[0][0] = (cve + 0.5) * (cve + 0.5);
  beta[0][1] = (cve - 0.5) * (cve - 0.5);
  beta[1][0] = beta[0][1];
  beta[1][1] = beta[0][0];
  const double cvx = -0.5 + 2.0 * s2w;
  const double avg = 0.5 * ((cvx - 0.5) * (cvx - 0.5) + (cvx + 0.5) * (cvx + 0.5));
  beta[2][0] = beta[2][1] = avg;
  // beta_III = C_V^2 - C_A^2: unchanged by C_A -> -C_A, so shared by particle and antiparticle
  beta3[0] = beta3[1] = (cve - 0.5) * (cve + 0.5);
  beta3[2] = (cvx - 0.5) * (cvx + 0.5);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Task order for each k = #{eps_j < mu_e} (0..ne), over the tasks (i >= j). Where mu_e falls
// among the bins decides which side of the bins each quadrature group of a task lies on,
// hence its node-loop variant, the same way for scattering task (i, j) and pair tasks
// {(i, j), (j, i)}: eps_i < mu (i < k); eps_j < mu <= eps_i (j < k <= i); mu <= eps_j (k <= j),
// the last ordered by column so that the scattering tail's split at mu+ + 10 T stays
// contiguous. Each class is a contiguous run, so the waves that run the tasks see few
// mixed-variant groups.
void task_order(int ne, std::vector<uint16_t>& order) {
  const int ntn = ne * (ne + 1) / 2;
  order.assign(size_t(ne + 1) * ntn, 0);
  auto tri = [](int i, int j) { return i * (i + 1) / 2 + j; };
  for (int k = 0; k <= ne; ++k) {
    uint16_t* o = order.data() + size_t(k) * ntn;
    int n = 0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j <= i; ++j) o[n++] = (uint16_t)tri(i, j);
    for (int i = k; i < ne; ++i)
      for (int j = 0; j < k; ++j) o[n++] = (uint16_t)tri(i, j);
    for (int j = k; j < ne; ++j)
      for (int i = j; i < ne; ++i) o[n++] = (uint16_t)tri(i, j);
  }
}

int build_plan(int device, const vtx_grid* g, const vtx_opts* o, Plan** out) {
  std::unique_ptr<Plan> p(new Plan);
  p->device = device;
  p->ne = g->ne;
  p->nquad = o->nquad;
  p->rule = o->rule;
  p->sin2w = o->sin2w;
  p->eps.assign(g->eps, g->eps + g->ne);
  p->w.assign(g->w, g->w + g->ne);
  const int ne = g->ne, ntn = ne * (ne + 1) / 2, ntp = ne * ne, m4 = o->nquad / 4;
  const int nlag = (o->rule == VTX_RULE_LAGUERRE) ? o->nquad : m4;
  // host images
  std::vector<double> c0w(ne);
  const double c0 = 1.0 / (4.0 * M_PI * M_PI * kHbarC);
  for (int j = 0; j < ne; ++j) c0w[j] = c0 * g->w[j];
  std::vector<double> inv_eps(ne);
  for (int j = 0; j < ne; ++j) inv_eps[j] = 1.0 / g->eps[j];
  std::vector<int> nes_ij(ntn);
  std::vector<NesCoef> ncoef(ntn);
  bool ok = true;
  for (int i = 0, t = 0; i < ne; ++i)
    for (int j = 0; j <= i; ++j, ++t) {
      nes_ij[t] = i | (j << 8);
      ok = nes_coefficients(g->eps[i], g->eps[j], ncoef[t]) && ok;
    }
  std::vector<PairCoef> pcoef(ntp);
  for (int i = 0; i < ne; ++i)
    for (int j = 0; j < ne; ++j) ok = pair_coefficients(g->eps[i], g->eps[j], pcoef[i * ne + j]) && ok;
  if (!ok) return VTX_EINVAL;
  std::vector<MassCoef> mnes(ntn), mpair(ntn);
  for (int i = 0, t = 0; i < ne; ++i)
    for (int j = 0; j <= i; ++j, ++t) {
      mass_coefficients(g->eps[i], g->eps[j], false, mnes[t]);
      mass_coefficients(g->eps[i], g->eps[j], true, mpair[t]);
    }
  std::vector<double2> mgauss(kMassGauss);
  {
    double gx[kMassGauss], gw[kMassGauss];
    if (!gauss_rule(0, kMassGauss, gx, gw)) return VTX_EINVAL;
    for (int k = 0; k < kMassGauss; ++k) mgauss[k] = make_double2(gx[k], gw[k]);
  }
  std::vector<double> tx(m4), tw(m4), lx(nlag), lw(nlag);
  if (!gauss_rule(0, m4, tx.data(), tw.data()) || !gauss_rule(1, nlag, lx.data(), lw.data())) return VTX_EINVAL;
  std::vector<double4> leg64(m4), lag64(nlag);
  std::vector<float4> leg32(m4), lag32(nlag);
  for (int k = 0; k < m4; ++k) {
    leg64[k] = make_double4(tx[k], 1.0 - tx[k], tw[k], 0.0);
    leg32[k] = make_float4((float)tx[k], (float)(1.0 - tx[k]), (float)tw[k], 0.f);
  }
  for (int k = 0; k < nlag; ++k) {
    lag64[k] = make_double4(lx[k], lx[k], lw[k], 0.0);
    lag32[k] = make_float4((float)lx[k], (float)lx[k], (float)lw[k], 0.f);
  }
  // one device buffer
  size_t off = 0;
  auto place = [&](size_t bytes) {
    const size_t o0 = off;
    off = align256(off + bytes);
    return o0;
  };
  const size_t o_eps = place(sizeof(double) * ne), o_c0w = place(sizeof(double) * ne);
  const size_t o_ie = place(sizeof(double) * ne);
  const size_t o_ij = place(sizeof(int) * ntn), o_nc = place(sizeof(NesCoef) * ntn);
  const size_t o_pc = place(sizeof(PairCoef) * ntp);
  const size_t o_mn = place(sizeof(MassCoef) * ntn), o_mp = place(sizeof(MassCoef) * ntn);
  const size_t o_mg = place(sizeof(double2) * kMassGauss);
  const size_t o_l64 = place(sizeof(double4) * m4), o_g64 = place(sizeof(double4) * nlag);
  const size_t o_l32 = place(sizeof(float4) * m4), o_g32 = place(sizeof(float4) * nlag);
  std::vector<uint16_t> order;
  task_order(ne, order);
  const size_t o_to = place(sizeof(uint16_t) * order.size());
  std::vector<unsigned char> img(off, 0);
  auto put = [&](size_t o2, const void* src, size_t bytes) { std::memcpy(img.data() + o2, src, bytes); };
  put(o_eps, g->eps, sizeof(double) * ne);
  put(o_c0w, c0w.data(), sizeof(double) * ne);
  put(o_ie, inv_eps.data(), sizeof(double) * ne);
  put(o_ij, nes_ij.data(), sizeof(int) * ntn);
  put(o_nc, ncoef.data(), sizeof(NesCoef) * ntn);
  put(o_pc, pcoef.data(), sizeof(PairCoef) * ntp);
  put(o_mn, mnes.data(), sizeof(MassCoef) * ntn);
  put(o_mp, mpair.data(), sizeof(MassCoef) * ntn);
  put(o_mg, mgauss.data(), sizeof(double2) * kMassGauss);
  put(o_l64, leg64.data(), sizeof(double4) * m4);
  put(o_g64, lag64.data(), sizeof(double4) * nlag);
  put(o_l32, leg32.data(), sizeof(float4) * m4);
  put(o_g32, lag32.data(), sizeof(float4) * nlag);
  put(o_to, order.data(), sizeof(uint16_t) * order.size());
  if (hipMalloc(&p->dbuf, off) != hipSuccess) return VTX_ENOMEM;
  if (hipMemcpy(p->dbuf, img.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->dbuf);
    return VTX_EHIP;
  }
  unsigned char* b = (unsigned char*)p->dbuf;
  DevPlan& d = p->dp;
  d.ne = ne;
  d.ntn = ntn;
  d.ntp = ntp;
  d.m4 = m4;
  d.rule = o->rule;
  d.nlag = nlag;
  couplings(o->sin2w, d.beta, d.beta3);
  d.eps = (const double*)(b + o_eps);
  d.c0w = (const double*)(b + o_c0w);
  d.inv_eps = (const double*)(b + o_ie);
  d.nes_ij = (const int*)(b + o_ij);
  d.nes_coef = (const NesCoef*)(b + o_nc);
  d.pair_coef = (const PairCoef*)(b + o_pc);
  d.mass_nes = (const MassCoef*)(b + o_mn);
  d.mass_pair = (const MassCoef*)(b + o_mp);
  d.mass_gauss = (const double2*)(b + o_mg);
  d.leg64 = (const double4*)(b + o_l64);
  d.lag64 = (const double4*)(b + o_g64);
  d.leg32 = (const float4*)(b + o_l32);
  d.lag32 = (const float4*)(b + o_g32);
  d.task_order = (const uint16_t*)(b + o_to);
  *out = p.get();
  g_plans.push_back(std::move(p));
  return VTX_OK;
}

int check_args(const vtx_grid* g, const vtx_opts* o, int64_t nz) {
  if (!g || !o || nz < 0) return VTX_EINVAL;
  if (g->ne < 1 || g->ne > kMaxNE || !g->eps || !g->w) return VTX_EINVAL;
  for (int i = 0; i < g->ne; ++i) {
    if (!(g->eps[i] > 0.0) || !(g->w[i] > 0.0) || !std::isfinite(g->eps[i]) || !std::isfinite(g->w[i]))
      return VTX_EINVAL;
    if (i > 0 && !(g->eps[i] > g->eps[i - 1])) return VTX_EINVAL;
  }
  if (o->precision != VTX_FP64 && o->precision != VTX_MIXED) return VTX_EINVAL;
  if (o->nquad < 8 || o->nquad > kMaxNquad || (o->nquad % 4) != 0) return VTX_EINVAL;
  if (o->rule != VTX_RULE_LAGUERRE && o->rule != VTX_RULE_PANEL) return VTX_EINVAL;
  if (o->processes == 0 || (o->processes & ~7u) != 0) return VTX_EINVAL;
  if (!std::isfinite(o->sin2w) || !std::isfinite(o->eta_fp64)) return VTX_EINVAL;
  if (nz > 0x7fffffffLL) return VTX_EINVAL;
  return VTX_OK;
}

// Current device must be gfx950. Returns the device ordinal or a negative status.
int current_device(int* dev) {
  if (getenv("VTX_FAULT_INJECT_HIP")) return -VTX_EHIP;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return -VTX_EDEVICE;
  if (hipGetDevice(dev) != hipSuccess) return -VTX_EHIP;
  if ((int)g_dev_ok.size() < n) g_dev_ok.resize(n, 0);
  if (g_dev_ok[*dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return -VTX_EHIP;
    g_dev_ok[*dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
  }
  return g_dev_ok[*dev] == 1 ? 0 : -VTX_EDEVICE;
}

int get_plan(const vtx_grid* g, const vtx_opts* o, DevPlan* out) {
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  const int st = current_device(&dev);
  if (st < 0) return -st;
  Plan* hit = nullptr;
  for (auto& p : g_plans) {
    if (p->device == dev && p->ne == g->ne && p->nquad == o->nquad && p->rule == o->rule && p->sin2w == o->sin2w &&
        std::memcmp(p->eps.data(), g->eps, sizeof(double) * g->ne) == 0 &&
        std::memcmp(p->w.data(), g->w, sizeof(double) * g->ne) == 0) {
      hit = p.get();
      break;
    }
  }
  if (!hit) {
    const int rc = build_plan(dev, g, o, &hit);
    if (rc != VTX_OK) return rc;
  }
  *out = hit->dp;
  out->processes = (int)o->processes;
  out->precision = o->precision;
  out->eta_fp64 = o->eta_fp64;
  out->block = g_block;
  return VTX_OK;
}

}  // namespace
}  // namespace vtx

extern "C" {

void vtx_opts_default(vtx_opts* o) {
  if (!o) return;
  o->precision = VTX_FP64;
  o->nquad = 48;
  o->rule = VTX_RULE_PANEL;
  o->processes = VTX_NES | VTX_PAIR;
  o->sin2w = 0.2312;
  o->eta_fp64 = 30.0;
}

int vtx_rates_forward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                      const double* eta_e, const double* f, double* eta, double* chi, void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !f || !eta || !chi) return VTX_EINVAL;
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_forward(P, nzones, T, eta_e, f, eta, chi, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_rates_forward_mass(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                           const double* eta_e, const double* f, double* eta, double* chi, void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (opts->precision != VTX_FP64 || opts->rule != VTX_RULE_PANEL) return VTX_EINVAL;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !f || !eta || !chi) return VTX_EINVAL;
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_forward_mass(P, nzones, T, eta_e, f, eta, chi, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_rates_backward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                       const double* eta_e, const double* f, const double* g_eta, const double* g_chi, double* g_T,
                       double* g_eta_e, double* g_f, void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !f || !g_eta || !g_chi || !g_T || !g_eta_e || !g_f) return VTX_EINVAL;
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_backward(P, nzones, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f,
                                            (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_rates_jacobian(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                       const double* eta_e, const double* f, double* eta, double* chi, double* jac,
                       void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !jac) return VTX_EINVAL;
  const bool outs = f || eta || chi;
  if (outs && !(f && eta && chi)) return VTX_EINVAL;   // all three or none
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_jacobian(P, nzones, T, eta_e, f, eta, chi, jac, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_rates_forward_backward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                               const double* eta_e, const double* f, const double* g_eta, const double* g_chi,
                               double* eta, double* chi, double* g_T, double* g_eta_e, double* g_f,
                               void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !f || !g_eta || !g_chi || !eta || !chi || !g_T || !g_eta_e || !g_f) return VTX_EINVAL;
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_forward_backward(P, nzones, T, eta_e, f, g_eta, g_chi, eta, chi, g_T, g_eta_e,
                                                    g_f, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int64_t vtx_task_values(int32_t ne, uint32_t processes) {
  if (ne < 1 || ne > vtx::kMaxNE || processes == 0 || (processes & ~7u) != 0) return 0;
  return vtx::task_values(ne, processes);
}

namespace {
int rates_tasks(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T, const double* eta_e,
                double* tasks, bool rows, void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (nzones == 0) return VTX_OK;
  if (!T || !eta_e || !tasks) return VTX_EINVAL;
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e = vtx::launch_tasks(P, nzones, T, eta_e, tasks, rows, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}
}  // namespace

int vtx_rates_tasks(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                    const double* eta_e, double* tasks, void* hip_stream) {
  return rates_tasks(grid, opts, nzones, T, eta_e, tasks, false, hip_stream);
}

int vtx_rates_table_rows(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones, const double* T,
                         const double* eta_e, double* rows, void* hip_stream) {
  return rates_tasks(grid, opts, nzones, T, eta_e, rows, true, hip_stream);
}

int vtx_rates_forward_interp(const vtx_grid* grid, const vtx_opts* opts, const vtx_lattice* lat,
                             const double* table, int64_t table_len, int64_t nzones, const double* T,
                             const double* eta_e,
                             const double* f, double* eta, double* chi, void* hip_stream) {
  int rc = vtx::check_args(grid, opts, nzones);
  if (rc != VTX_OK) return rc;
  if (!lat || lat->nt < 2 || lat->nh < 2 || !(lat->dlnT > 0.0) || !(lat->deta > 0.0) ||
      !std::isfinite(lat->lnT0) || !std::isfinite(lat->eta0) || !std::isfinite(lat->dlnT) ||
      !std::isfinite(lat->deta))
    return VTX_EINVAL;
  if (table_len != int64_t(lat->nt) * lat->nh * vtx::task_values(grid->ne, opts->processes)) return VTX_EINVAL;
  if (nzones == 0) return VTX_OK;
  if (!table || !T || !eta_e || !f || !eta || !chi) return VTX_EINVAL;
  if ((reinterpret_cast<uintptr_t>(table) & 15) != 0) return VTX_EINVAL;   // rows are read in pairs
  vtx::DevPlan P;
  rc = vtx::get_plan(grid, opts, &P);
  if (rc != VTX_OK) return rc;
  const hipError_t e =
      vtx::launch_interp(P, *lat, table, nzones, T, eta_e, f, eta, chi, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_ray_system(int32_t ne, int64_t nrays, int32_t nzr, double dt, const double* jac, const double* f,
                   const double* f_n, const double* f_nm1, const double* eta, const double* chi, const double* lo,
                   const double* up, double* D, double* rhs, void* hip_stream) {
  if (ne < 1 || ne > vtx::kMaxNE || nrays < 0 || nzr < 1 || nzr > (1 << 22) || !(dt > 0.0) ||
      !std::isfinite(dt))
    return VTX_EINVAL;
  if (nrays > 0x7fffffffLL / nzr) return VTX_EINVAL;
  if (nrays == 0) return VTX_OK;
  if (!jac || !f || !f_n || !f_nm1 || !eta || !chi || !lo || !up || !D || !rhs) return VTX_EINVAL;
  {
    std::lock_guard<std::mutex> lock(vtx::g_mu);
    int dev = 0;
    const int st = vtx::current_device(&dev);
    if (st < 0) return -st;
  }
  const hipError_t e = vtx::launch_ray_system(ne, nrays * nzr, nzr, dt, jac, f, f_n, f_nm1, eta, chi, lo, up, D,
                                              rhs, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_ray_solve(int32_t nb, int64_t nrays, int32_t nzr, const double* lo, double* D, const double* up,
                  double* rhs, void* hip_stream) {
  if (nb < 1 || nb > vtx::max_block() || nrays < 0 || nzr < 1) return VTX_EINVAL;
  if (nrays > 0x7fffffffLL / nzr) return VTX_EINVAL;
  if (nrays == 0) return VTX_OK;
  if (!lo || !D || !up || !rhs) return VTX_EINVAL;
  {
    std::lock_guard<std::mutex> lock(vtx::g_mu);
    int dev = 0;
    const int st = vtx::current_device(&dev);
    if (st < 0) return -st;
  }
  const hipError_t e = vtx::launch_ray_solve(nb, nrays, nzr, lo, D, up, rhs, (hipStream_t)hip_stream);
  return e == hipSuccess ? VTX_OK : VTX_EHIP;
}

int vtx_ray_max_block(void) { return vtx::max_block(); }

const char* vtx_strerror(int code) {
  switch (code) {
    case VTX_OK: return "ok";
    case VTX_EINVAL: return "invalid argument";
    case VTX_EDEVICE: return "no gfx950 HIP device";
    case VTX_EHIP: return "HIP runtime error";
    case VTX_ENOMEM: return "device allocation failed";
    default: return "unknown status";
  }
}

int vtx_abi_version(void) { return VTX_ABI_VERSION; }

int vtx_set_workgroup_waves(int waves) {
  if (waves != 4 && waves != 8) return -VTX_EINVAL;
  std::lock_guard<std::mutex> lock(vtx::g_mu);
  const int prev = vtx::g_block / 64;
  vtx::g_block = 64 * waves;
  return prev;
}

void vtx_release(void) {
  std::lock_guard<std::mutex> lock(vtx::g_mu);
  for (auto& p : vtx::g_plans)
    if (p->dbuf) (void)hipFree(p->dbuf);
  vtx::g_plans.clear();
}

int vtx_eval_hmass(int process, int comp, double e, double ep, int n, const double* E, double* out) {
  if ((process != VTX_NES && process != VTX_PAIR) || comp < 0 || comp > 5 || n < 0 || (n > 0 && (!E || !out)))
    return VTX_EINVAL;
  if (!(e > 0.0) || !(ep > 0.0) || (process == VTX_NES && e < ep)) return VTX_EINVAL;
  const bool pair = process == VTX_PAIR;
  vtx::MassCoef C;
  vtx::mass_coefficients(e, ep, pair, C);
  const double m = vtx::kMe, w = e + ep, om = e - ep;
  // undo the prefactor and the third structure's sign: H itself
  const double pref = vtx::kGF * vtx::kGF / (M_PI * e * ep), s3 = pair ? pref : -pref;
  for (int q = 0; q < n; ++q) {
    const double x = E[q];
    double k0 = 0.0, k1 = 0.0;
    if (!pair) {
      const double xp = x + om;
      if (x > m && xp > m) {
        const double P = std::sqrt((x - m) * (x + m)), Pp = std::sqrt((xp - m) * (xp + m));
        k0 = (2.0 * x + om) * om / (P + Pp);
        k1 = std::fmin(w, P + Pp);
      }
    } else {
      const double xb = w - x;
      if (x > m && xb > m) {
        const double P = std::sqrt((x - m) * (x + m)), Pb = std::sqrt((xb - m) * (xb + m));
        k0 = std::fmax(std::fabs(om), std::fabs((2.0 * x - w) * w) / (P + Pb));
        k1 = P + Pb;
      }
    }
    const double L = k1 - k0;
    if (!(L > 0.0)) {
      out[q] = 0.0;
      continue;
    }
    // h_n = (k1^{n+1} - k0^{n+1}) / ((n + 1) L), n = -4, -2, 0, 2, 4, 6
    double sn[7] = {1.0, 0, 0, 0, 0, 0, 0};
    for (int a = 1; a <= 6; ++a) sn[a] = k1 * sn[a - 1] + std::pow(k0, a);
    const double ixy = k0 > 0.0 ? 1.0 / (k0 * k1) : 0.0;
    const double h[6] = {sn[2] * ixy * ixy * ixy / 3.0, ixy, 1.0, sn[2] / 3.0, sn[4] / 5.0, sn[6] / 7.0};
    double acc = 0.0;
    if (comp < 4) {
      for (int r = 0; r < 5; ++r)
        for (int a = 0; a < 3; ++a) acc += C.c[comp][3 * r + a] * std::pow(x, a) * h[r];
      acc += C.c[comp][15] * h[5];
      out[q] = L * acc / pref;
    } else {
      const int l = comp - 4;
      acc = C.c3[l][0] * h[2] + C.c3[l][1] * h[3] + C.c3[l][2] * h[4];
      out[q] = L * acc / s3;
    }
  }
  return VTX_OK;
}

int vtx_gauss_rule(int kind, int n, double* x, double* w) {
  if ((kind != 0 && kind != 1) || n < 1 || n > vtx::kMaxNquad || !x || !w) return VTX_EINVAL;
  return vtx::gauss_rule(kind, n, x, w) ? VTX_OK : VTX_EINVAL;
}

int vtx_task_coefficients(int process, double e, double ep, double* out) {
  if (!out || !(e > 0) || !(ep > 0)) return VTX_EINVAL;
  if (process == VTX_NES) {
    if (e < ep) return VTX_EINVAL;
    vtx::NesCoef C;
    if (!vtx::nes_coefficients(e, ep, C)) return VTX_EINVAL;
    std::memcpy(out, &C, sizeof(C));
    return VTX_OK;
  }
  if (process == VTX_PAIR) {
    vtx::PairCoef C;
    if (!vtx::pair_coefficients(e, ep, C)) return VTX_EINVAL;
    std::memcpy(out, &C, sizeof(C));
    return VTX_OK;
  }
  return VTX_EINVAL;
}

int vtx_eval_hpoly(int process, int comp, double e, double ep, int n, const double* E, double* out) {
  if (comp < 0 || comp > 3 || !(e > 0) || !(ep > 0) || n < 0 || (n > 0 && (!E || !out))) return VTX_EINVAL;
  if (process == VTX_NES) {
    if (e < ep) return VTX_EINVAL;
    vtx::NesCoef C;
    if (!vtx::nes_coefficients(e, ep, C)) return VTX_EINVAL;
    const double pref = vtx::kGF * vtx::kGF / (M_PI * e * ep);
    for (int k = 0; k < n; ++k) {
      const double u = E[k] / ep;
      double s = 0.0;
      if (u < 1.0)
        s = vtx::bernstein_low(C.lo[comp], u);
      else
        for (int d = 2; d >= 0; --d) s = s * u + C.hi[comp][d];
      out[k] = E[k] < 0 ? 0.0 : s / pref;
    }
    return VTX_OK;
  }
  if (process == VTX_PAIR) {
    // comp S = I/II, l; evaluated through the tables of the (e, ep) task for S = I and of
    // the (ep, e) task for S = II.
    const int S = comp >> 1, l = comp & 1;
    vtx::PairCoef C;
    const double a = S == 0 ? e : ep, b = S == 0 ? ep : e;
    if (!vtx::pair_coefficients(a, b, C)) return VTX_EINVAL;
    const double pref = vtx::kGF * vtx::kGF / (M_PI * e * ep);
    const double mn = std::fmin(e, ep), mx = std::fmax(e, ep), w = e + ep;
    for (int k = 0; k < n; ++k) {
      const double x = E[k];
      if (x <= 0 || x >= w) {
        out[k] = 0.0;
        continue;
      }
      double s;
      if (x <= mn) {
        s = vtx::bernstein_low(C.A[l], x / mn);
      } else if (x <= mx) {
        const double u = x / mx;
        s = (C.B[l][2] * u + C.B[l][1]) * u + C.B[l][0];
      } else {
        s = vtx::bernstein_low(C.C[l], (w - x) / mn);
      }
      out[k] = s / pref;
    }
    return VTX_OK;
  }
  return VTX_EINVAL;
}

}  // extern "C"
