// HIP kernels for gfx950: energy-coupled neutrino-matter interaction rates.
//
// A workgroup takes one zone and gives each lane whole (eps_i, eps_j) tasks: the
// scattering kernel integral for eps_i >= eps_j or the pair kernel integral for any (i, j).
// Tasks go to waves in units of 64 of one kind, so a wave never mixes the two kinds and
// each kind compiles to its own code path. A task's quadrature rule has four groups of nodes (Gauss-Legendre panels and,
// for scattering, a Gauss-Laguerre tail); every group is an affine image of one node table
// held in LDS. Per node a lane forms the piece variable u and the two Fermi-Dirac arguments
// from the table, evaluates the blocking factor with two exp and one reciprocal, and
// accumulates the moments sum_k w_k B_k b(u_k) of a nonnegative basis of the angular-weight
// piece. The moments are contracted in FP64 with the zone-independent angular-weight
// coefficients once per task. Task values stay in LDS: detailed-balance completion, species
// combination and the contraction with f run from LDS, and the only HBM writes are eta/chi
// (or the gradients). The work is VALU bound with no dense contraction, so MFMA has no role.
//
// Mixed precision runs the bulk in FP32 (node coordinates, Fermi-Dirac factors, angular-weight
// moments and their accumulation) with FP64 contractions and detailed-balance factors; zones
// with |eta_e| above a threshold run in FP64 (a second pass over the zones with the FP64 node
// loops, whose blocking factor takes one FP64 exponential).
#include <hip/hip_runtime.h>

#include "../../include/vtx_rates.h"
#include "vtx_internal.h"

namespace vtx {
namespace {

constexpr double kLog2e = 1.4426950408889634;
constexpr int kM4 = kMaxNquad / 4;
// Node table in LDS (entries of the bulk type): Gauss-Legendre x | 1 - x | w on [0, 1], then
// Gauss-Laguerre x | w e^x | 1. A map reads its node coordinate through a per-lane offset.
constexpr int kOffX = 0, kOffY = kM4, kOffW = 2 * kM4, kOffGX = 3 * kM4, kOffGW = 3 * kM4 + kMaxNquad;
constexpr int kOffOne = 3 * kM4 + 2 * kMaxNquad;
constexpr int kTabLen = 3 * kM4 + 3 * kMaxNquad;

// Workgroup size: four waves (DevPlan::block, 256 lanes), or eight as a diagnostic that the
// results do not depend on it. The task units of a zone spread over the waves, and four waves
// cover the per-zone contraction's 3 ne lanes up to 32 bins. Kernels accept either.
constexpr int kMaxBlock = 512;
constexpr int kSlotStride = 256;

// Lane modes of a group: every node in the low piece, every node in the high piece, or
// decided per node (u < split).
constexpr int kLow = 0, kHigh = 1, kGen = 2;

// Pair partner of species s: nu_e <-> anti-nu_e, nu_x <-> nu_x.
__device__ __forceinline__ int partner(int s) { return s == 2 ? 2 : 1 - s; }

// beta_S of species s, selected without indexing the by-value plan (keeps it in SGPRs).
__device__ __forceinline__ double beta_of(const DevPlan& P, int s, int S) {
  const double b0 = S ? P.beta[0][1] : P.beta[0][0];
  const double b1 = S ? P.beta[1][1] : P.beta[1][0];
  const double b2 = S ? P.beta[2][1] : P.beta[2][0];
  return s == 0 ? b0 : (s == 1 ? b1 : b2);
}

// 2^x in FP64 for x <= 1000 (callers cap larger arguments): x = n + f with n = rint(x),
// |f| <= 1/2, and 2^f from the degree-10 Chebyshev interpolant of 2^f on [-1/2, 1/2] in
// monomial form (derived by gen/exp2_coeffs.py; worst relative error of the whole evaluation
// 3.9e-16); 2^n enters through ldexp. x is clamped below at -2100, beyond which 2^x rounds to 0
// anyway, so -inf gives 0 too.
__device__ __forceinline__ double exp2_fp64(double x) {
  constexpr double kExpPoly[11] = {1.0, 0.69314718055995, 0.24022650695910097, 0.05550410866444772,
                                   0.009618129107606888, 0.0013333558230164974, 0.0001540353044173605,
                                   1.5252657260200837e-05, 1.321544258792169e-06, 1.0208690299958306e-07,
                                   7.072585949269223e-09};
  const double xc = fmax(x, -2100.0);
  const double n = rint(xc);
  const double t = xc - n;
  double p = kExpPoly[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) p = __builtin_fma(p, t, kExpPoly[k]);
  return ldexp(p, int(n));
}

// 1/x for x in [1, 2^1010]: the hardware estimate refined by two Newton steps, e = 1 - x r,
// r += r e (about 1 ulp).
__device__ __forceinline__ double recip_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Precision of a kernel: R, the bulk type (piece variable, node weights, angular-weight moments
// and their accumulation), and F, the type of the Fermi-Dirac arguments and blocking factors.
// The mixed path runs Fp32 on zones of moderate degeneracy and Fp64 on zones with |eta_e| above
// its threshold; the FP64 path runs Fp64 throughout.
struct Fp32 {
  using R = float;
  using F = float;   // the policies keep the two types apart; both use one type throughout
};
struct Fp64 {
  using R = double;
  using F = double;
};

// Arithmetic of a type. The Fermi-Dirac arguments are carried pre-scaled by log2(e), so
// exp(-z) is an exp2.
template <typename R> struct Num;
template <> struct Num<double> {
  __device__ static __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
};
template <> struct Num<float> {
  __device__ static __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

// Blocking factor B = sigma(z1) sigma(z2), sigma(z) = 1 / (1 + 2^-z), and (backward) the
// logarithmic derivatives r = 1 - sigma(z) of its two factors.
//
// FP32: two hardware exp2 and one reciprocal (two in the backward). Where 2^-z overflows to
// +inf the sums stay +inf (never inf x 0), so B = 0, sigma = 0 and r = 1 are the limits.
//
// FP64 (one exponential): the two arguments sum to the task constant K = D log2(e) / T >= 0
// (scattering D = eps_i - eps_j, pair D = eps_i + eps_j), so the smaller one, t, is at most K/2,
// and the other factor's 2^-(K - t) equals C a with a = 2^t and C = 2^-K (a task constant):
//   B = a / ((1 + a)(1 + C a)),  1 - sigma(t) = 1 / (1 + a),  1 - sigma(K - t) = C a / (1 + C a),
// all from one reciprocal. C a <= 1, and t is capped at 1000, where both factors are 1 to FP64
// precision (the other argument is then at least as large), so the denominator stays finite;
// a very negative t gives a = 0 and B = 0. Where C underflows (K above 1074), C a <= 2^(-K/2)
// and the second factor is 1 to FP64 precision.
__device__ __forceinline__ float blocking_fwd(float z1, float z2, float) {
  const float a = __builtin_amdgcn_exp2f(-z1), b = __builtin_amdgcn_exp2f(-z2);
  return __builtin_amdgcn_rcpf((1.0f + a) * (1.0f + b));
}
__device__ __forceinline__ double blocking_fwd(double z1, double z2, double C) {
  const double a = exp2_fp64(fmin(fmin(z1, z2), 1000.0));
  return a * recip_pos((1.0 + a) * __builtin_fma(C, a, 1.0));
}

template <typename R>
__device__ __forceinline__ void blocking_bwd(float z1, float z2, float, R& B, R& r1, R& r2) {
  const float i1 = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z1));
  const float i2 = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z2));
  B = i1 * i2;
  r1 = 1.0f - i1;
  r2 = 1.0f - i2;
}
template <typename R>
__device__ __forceinline__ void blocking_bwd(double z1, double z2, double C, R& B, R& r1, R& r2) {
  const bool first = z1 <= z2;
  const double a = exp2_fp64(fmin(fmin(z1, z2), 1000.0));
  const double ca = C * a, d1 = 1.0 + a, d2 = 1.0 + ca;
  const double q = recip_pos(d1 * d2);
  B = R(a * q);
  const R rt = R(d2 * q), ro = R(ca * (d1 * q));
  r1 = first ? rt : ro;
  r2 = first ? ro : rt;
}

// A breakpoint: value and its derivatives along T (eta_e fixed) and along eta_e (T fixed).
struct Tri {
  double v, dT, dE;
};

// Component-wise select (a struct select would become an address select into scratch).
__device__ __forceinline__ Tri sel(bool c, const Tri& a, const Tri& b) {
  return {c ? a.v : b.v, c ? a.dT : b.dT, c ? a.dE : b.dE};
}
__device__ __forceinline__ Tri pick4(int g, const Tri& a, const Tri& b, const Tri& c, const Tri& d) {
  return sel(g == 0, a, sel(g == 1, b, sel(g == 2, c, d)));
}

// Per-zone state shared by the lanes of a workgroup. A workgroup holds two: the zone, and its
// mirror (eta_e, mu_e negated) under which the scattering tasks become scattering on
// positrons, whose occupation is F(E; -mu_e).
struct Zone {
  double T, eta, invT, mu;
  int64_t z;   // zone index, or -1 for an empty slot
  int valid;
  int k;       // #{eps_j < mu_e}: selects the task order
};

// Node table of a kernel in LDS, in the kernel's type (piece variable, weights, Fermi-Dirac
// arguments).
__device__ __forceinline__ void fill_tab(const DevPlan& P, double* tab) {
  for (int k = threadIdx.x; k < P.m4; k += blockDim.x) {
    const double4 n = P.leg64[k];
    tab[kOffX + k] = n.x;
    tab[kOffY + k] = n.y;
    tab[kOffW + k] = n.z;
  }
  for (int k = threadIdx.x; k < P.nlag; k += blockDim.x) {
    const double4 n = P.lag64[k];
    tab[kOffGX + k] = n.x;
    tab[kOffGW + k] = n.z;
    tab[kOffOne + k] = 1.0;
  }
}
__device__ __forceinline__ void fill_tab(const DevPlan& P, float* tab) {
  for (int k = threadIdx.x; k < P.m4; k += blockDim.x) {
    const float4 n = P.leg32[k];
    tab[kOffX + k] = n.x;
    tab[kOffY + k] = n.y;
    tab[kOffW + k] = n.z;
  }
  for (int k = threadIdx.x; k < P.nlag; k += blockDim.x) {
    const float4 n = P.lag32[k];
    tab[kOffGX + k] = n.x;
    tab[kOffGW + k] = n.z;
    tab[kOffOne + k] = 1.0f;
  }
}

// The node table as read by the piece variable and weights (r) and by the Fermi-Dirac
// arguments (f): one table in LDS, in the kernel's type.
template <typename Pr>
struct Tabs {
  const typename Pr::R* r;
  const typename Pr::F* f;
};

template <typename Pr>
constexpr int tab_bytes() {
  return kTabLen * (int)sizeof(typename Pr::R);
}

template <typename Pr>
__device__ __forceinline__ Tabs<Pr> stage_tabs(const DevPlan& P, double* raw) {
  typename Pr::R* t = reinterpret_cast<typename Pr::R*>(raw);
  fill_tab(P, t);
  return {t, t};
}

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// ----------------------------------------------------------------------------------------
// Tasks and their quadrature groups.
//
// Scattering (eps_i >= eps_j): z1 = (mu - E)/T [F(E)], z2 = (E + Delta - mu)/T
// [1 - F(E + Delta)], Delta = eps_i - eps_j. Pair: z1 = (E - mu)/T [1 - F(E)],
// z2 = (w - E + mu)/T [1 - Fbar(w - E)], w = eps_i + eps_j. Both read
// z1 = sg (mu - E)/T and z2 = (D - sg (mu - E))/T with (sg, D) = (1, Delta) or (-1, w).
// The blocking factor is B = sigma(z1) sigma(z2), sigma(z) = 1 / (1 + exp(-z)).

struct Task {
  bool pair;
  int i, j;
  double e, ep, sg, D;
};

// Task t (i >= j). A pair task covers both (i, j) and (j, i): the two share the energy
// E + E' = eps_i + eps_j, the breakpoints, the blocking factor and the piece variables (which
// depend on min and max of the two energies only), so one node loop serves both and only
// the angular-weight coefficients differ.
template <bool PAIR>
__device__ __forceinline__ Task make_task(const DevPlan& P, int t) {
  Task K;
  const bool pair = PAIR;
  K.pair = pair;
  const int ij = P.nes_ij[t];
  K.i = ij & 0xff;
  K.j = ij >> 8;
  K.e = P.eps[K.i];
  K.ep = P.eps[K.j];
  K.sg = pair ? -1.0 : 1.0;
  K.D = pair ? K.e + K.ep : K.e - K.ep;
  return K;
}

// One group: a Gauss-Legendre panel E = lo + (hi - lo) x, or the Gauss-Laguerre tail
// E = lo + T x (table entries toff ...). The piece variable is u = E ub, or (w - E) ub for
// the pair's upper piece (c). mode: see kLow/kHigh/kGen; slot: moment slot of the piece.
struct GroupDesc {
  Tri lo, hi;
  bool lag, c;
  int toff, mode, slot, piece;
  double ub, w;
};

// Scattering breakpoints {0, (mu - Delta)+, mu+, min(eps_j, mu+ + KAPPA T)} in increasing
// order s1 <= s2 <= s3 (the first is 0). (mu - Delta)+ <= mu+ always, so only the cap is
// inserted.
__device__ __forceinline__ void nes_breakpoints(double ep, double delta, const Zone& Z, Tri& s1, Tri& s2,
                                                Tri& s3) {
  const double mu = Z.mu, T = Z.T, eta = Z.eta;
  const bool pm = mu - delta > 0.0, pu = mu > 0.0;
  const Tri b1 = {pm ? mu - delta : 0.0, pm ? eta : 0.0, pm ? T : 0.0};
  const Tri b2 = {pu ? mu : 0.0, pu ? eta : 0.0, pu ? T : 0.0};
  const double cap = b2.v + kKappa * T;
  const bool pp = ep <= cap;
  const Tri b3 = {pp ? ep : cap, pp ? 0.0 : b2.dT + kKappa, pp ? 0.0 : b2.dE};
  const bool c2 = b3.v < b2.v, c1 = b3.v < b1.v;
  s1 = sel(c1, b3, b1);
  s2 = sel(c1, b1, sel(c2, b3, b2));
  s3 = sel(c2, b2, b3);
}

// Pair breakpoints {0, b1, b2, b3, w}: {m, M} with c = clip(mu, 0, w) inserted after every
// one of {0, m, M} not above it.
__device__ __forceinline__ void pair_breakpoints(double mn, double mx, double w, const Zone& Z, Tri& b1, Tri& b2,
                                                 Tri& b3) {
  const double mu = Z.mu, T = Z.T, eta = Z.eta;
  const bool in = (mu > 0.0) && (mu <= w);
  const double cv = (mu > 0.0) ? fmin(mu, w) : 0.0, cT = in ? eta : 0.0, cE = in ? T : 0.0;
  const bool below_m = cv < mn, below_M = cv < mx;
  b1 = {below_m ? cv : mn, below_m ? cT : 0.0, below_m ? cE : 0.0};
  b2 = {below_m ? mn : (below_M ? cv : mx), (!below_m && below_M) ? cT : 0.0, (!below_m && below_M) ? cE : 0.0};
  b3 = {below_M ? mx : cv, below_M ? 0.0 : cT, below_M ? 0.0 : cE};
}

// The task's interior breakpoints, sorted (scattering: s1 <= s2 <= s3; pair: b1 <= b2 <= b3).
struct Brk {
  Tri b1, b2, b3;
};
template <bool PAIR>
__device__ __forceinline__ Brk task_breakpoints(const Task& K, const Zone& Z) {
  Brk B;
  if (!PAIR) {
    nes_breakpoints(K.ep, K.D, Z, B.b1, B.b2, B.b3);
  } else {
    const bool le = K.e <= K.ep;
    pair_breakpoints(le ? K.e : K.ep, le ? K.ep : K.e, K.D, Z, B.b1, B.b2, B.b3);
  }
  return B;
}

// Group g of a task (g is a constant once the group loop is unrolled). Scattering panels lie
// wholly below or wholly above eps_j (eps_j is a breakpoint whenever a panel could cross it),
// so only the tail can straddle u = 1. Each pair group lies in one piece: [0, m] (A),
// [m, M] (B), [M, w] (C).
// The ends of group g: (0, b1), (b1, b2), (b2, b3), then (b3, b3) for the scattering tail or
// (b3, w) for the pair's last panel.
template <bool PAIR>
__device__ __forceinline__ Tri group_hi(const Task& K, const Brk& Bk, int g) {
  const Tri last = PAIR ? Tri{K.D, 0.0, 0.0} : Bk.b3;
  return pick4(g, Bk.b1, Bk.b2, Bk.b3, last);
}

template <bool PAIR>
__device__ __forceinline__ GroupDesc describe(const DevPlan& P, const Task& K, const Brk& Bk, int g, const Tri& lo,
                                              const Tri& hi) {
  GroupDesc G;
  const Tri zero = {0.0, 0.0, 0.0};
  G.w = 0.0;
  G.c = false;
  G.slot = 0;
  G.piece = 0;
  if (!PAIR) {
    G.ub = P.inv_eps[K.j];
    if (P.rule == VTX_RULE_LAGUERRE) {
      G.lo = zero;
      G.hi = zero;
      G.lag = true;
      G.toff = g * P.m4;
      G.mode = kGen;
    } else {
      G.lo = lo;
      G.hi = hi;
      G.lag = (g == 3);
      G.toff = 0;
      G.mode = G.lag ? (Bk.b3.v >= K.ep ? kHigh : kGen) : (G.hi.v <= K.ep ? kLow : kHigh);
    }
  } else {
    const bool le = K.e <= K.ep;
    const double mn = le ? K.e : K.ep, mx = le ? K.ep : K.e, w = K.D;
    G.lo = lo;
    G.hi = hi;
    G.lag = false;
    G.toff = 0;
    const double mid = 0.5 * (G.lo.v + G.hi.v);
    const double imn = P.inv_eps[le ? K.i : K.j], imx = P.inv_eps[le ? K.j : K.i];
    // a zero-width group at m (diagonal tasks, or mu_e on a bin) counts as B like its
    // neighbours in the task order; it contributes nothing, and H is continuous at m
    G.piece = (mid < mn) ? 0 : ((mid <= mx) ? 1 : 2);
    G.ub = (G.piece == 1) ? imx : imn;
    G.c = (G.piece == 2);
    G.w = w;
    G.mode = (G.piece == 1) ? kHigh : kLow;
    G.slot = (G.piece == 2) ? 1 : 0;
  }
  return G;
}

// Values of the three maps at energy E.
struct EndV {
  double u, z1, z2;
};
__device__ __forceinline__ EndV end_values(const Task& K, const GroupDesc& G, const Zone& Z, double E) {
  const double d = Z.mu - E;
  return {G.c ? (G.w - E) * G.ub : E * G.ub, K.sg * d * Z.invT, (K.D - K.sg * d) * Z.invT};
}

// Node-loop parameters: value_k = c0 + c1 tab[off + k] per map; tab[ow + k] is the weight.
// A Legendre map is anchored at the end where it is smaller in magnitude (reading x or
// 1 - x), so that FP32 evaluation never subtracts two large numbers. Breakpoints sit on the
// zeros of the Fermi-Dirac arguments, so inside a group each argument keeps its sign. The
// Fermi-Dirac maps (a, b) are in the kernel's Fermi-Dirac type, with C = 2^-K the task constant
// of the one-exponential FP64 blocking factor (unused in FP32).
template <typename Pr>
struct Loop {
  using R = typename Pr::R;
  using F = typename Pr::F;
  R u0, u1, split;
  F a0, a1, b0, b1, C;
  int ou, o1, o2, ow;
  int oa, ob;   // backward: weights of the group's two end points, 1 - x and x (tail: 1 and x)
};

// Anchored map from its end values (already in the map's type): value = c0 + c1 x with x read
// from the column of x or 1 - x. The FP64 end values are rounded first, so c1 carries the
// rounding of the larger end, as the node values themselves would.
template <typename R>
__device__ __forceinline__ void anchor(R a, R b, R& c0, R& c1, int& off) {
  const bool rev = fabs(a) > fabs(b);
  const R d = b - a;
  c0 = rev ? b : a;
  c1 = rev ? -d : d;
  off = rev ? kOffY : kOffX;
}

// Returns the group's weight scale Es (nodes weigh Es w_k). The Fermi-Dirac arguments are
// formed in units of log2(e), so that exp(-z) is an exp2.
template <typename Pr>
__device__ __forceinline__ double make_loop(const Task& K, const GroupDesc& G, const Zone& Z, Loop<Pr>& L) {
  using R = typename Pr::R;
  using F = typename Pr::F;
  const double zs = kLog2e, its = Z.invT * zs;
  const double dA = Z.mu - G.lo.v;
  const double uA = G.c ? (G.w - G.lo.v) * G.ub : G.lo.v * G.ub;
  const double z1A = K.sg * dA * its, z2A = (K.D - K.sg * dA) * its;
  if constexpr (sizeof(F) == sizeof(double))
    L.C = exp2_fp64(-(K.D * its));
  else
    L.C = F(0);
  double Es;
  if (G.lag) {
    Es = Z.T;
    L.u0 = R(uA);
    L.u1 = R((G.c ? -G.ub : G.ub) * Z.T);
    L.a0 = F(z1A);
    L.a1 = F(-K.sg * zs);
    L.b0 = F(z2A);
    L.b1 = F(K.sg * zs);
    L.ou = L.o1 = L.o2 = kOffGX + G.toff;
    L.ow = kOffGW + G.toff;
    L.oa = kOffOne + G.toff;
    L.ob = kOffGX + G.toff;
  } else {
    Es = G.hi.v - G.lo.v;
    const double dB = Z.mu - G.hi.v;
    const double uB = G.c ? (G.w - G.hi.v) * G.ub : G.hi.v * G.ub;
    anchor<R>(R(uA), R(uB), L.u0, L.u1, L.ou);
    anchor<F>(F(z1A), F(K.sg * dB * its), L.a0, L.a1, L.o1);
    anchor<F>(F(z2A), F((K.D - K.sg * dB) * its), L.b0, L.b1, L.o2);
    L.ow = kOffW;
    L.oa = kOffY;
    L.ob = kOffX;
  }
  L.split = G.mode == kLow ? R(INFINITY) : (G.mode == kHigh ? R(-INFINITY) : R(1));
  return Es;
}

// A group of zero width whose end points do not move with T or eta_e (a clamped or coinciding
// breakpoint) adds exactly nothing to the task's values or derivatives. A wave skips its node
// loop when that holds on every lane, which leaves every result as it was.
__device__ __forceinline__ bool wave_skips(const GroupDesc& G) {
  const bool dead = !G.lag && G.hi.v == G.lo.v && G.hi.dT == G.lo.dT && G.hi.dE == G.lo.dE;
  return __all(dead);
}

// The variant a wave runs for a group: the lanes' common mode, else the general one. The
// general loop reproduces the low and high loops bit for bit on lanes of those modes
// (explicit fma, exact zeros), so results never depend on which lanes share a wave.
__device__ __forceinline__ int wave_mode(int m) {
  const bool gen = __any(m == kGen), lo = __any(m == kLow), hi = __any(m == kHigh);
  const int wm = (gen || (lo && hi)) ? kGen : (lo ? kLow : kHigh);
  return __builtin_amdgcn_readfirstlane(wm);
}

// ----------------------------------------------------------------------------------------
// Node loops.
//
// Low piece (degree-7 angular weight with a triple zero at u = 0): moments
//   M_j += w B u^3 q_j(u), q = (v^4, u v^3, u^2 v^2, u^3 v, u^4), v = 1 - u,
// i.e. the folded Bernstein basis u^k v^(7-k), k = 3..7. High piece: H_k += w B u^k,
// k = 0..2. Both bases are nonnegative on their ranges, so the FP32 sums are free of
// cancellation; sign changes of the l = 1 weights resolve in the FP64 contraction.

template <typename Pr, int MODE>
__device__ __forceinline__ void node_fwd(const Loop<Pr>& L, typename Pr::R xu, typename Pr::F x1,
                                         typename Pr::F x2, typename Pr::R w, typename Pr::R M[5],
                                         typename Pr::R H[3]) {
  using R = typename Pr::R;
  using F = typename Pr::F;
  using N = Num<R>;
  const R u = N::fma(L.u1, xu, L.u0);
  const F z1 = Num<F>::fma(L.a1, x1, L.a0), z2 = Num<F>::fma(L.b1, x2, L.b0);
  const R wB = w * R(blocking_fwd(z1, z2, L.C));
  R ul = u, wh = wB;
  if (MODE == kGen) {
    const bool lo = u < L.split;
    ul = lo ? u : R(0);
    wh = lo ? R(0) : wB;
  }
  if (MODE != kHigh) {
    // p q_j with the common factors taken first: p v^2 and p u^2 serve the five moments
    const R v = R(1) - ul, u2 = ul * ul, v2 = v * v, uv = ul * v;
    const R p = wB * (u2 * ul);
    const R pv2 = p * v2, pu2 = p * u2;
    M[0] = N::fma(pv2, v2, M[0]);
    M[1] = N::fma(pv2, uv, M[1]);
    M[2] = N::fma(pv2, u2, M[2]);
    M[3] = N::fma(pu2, uv, M[3]);
    M[4] = N::fma(pu2, u2, M[4]);
  }
  if (MODE != kLow) {
    H[0] = H[0] + wh;
    H[1] = N::fma(wh, u, H[1]);
    H[2] = N::fma(wh, u * u, H[2]);
  }
}

// Nodes in flight per lane: four in FP32; two where the bulk is FP64, whose exp2 chains are
// long and whose registers are twice as many.
template <typename Pr, int MODE>
__device__ __forceinline__ void nodes_fwd(const Loop<Pr>& L, int m, const Tabs<Pr>& tb, typename Pr::R M[5],
                                          typename Pr::R H[3]) {
  if constexpr (sizeof(typename Pr::R) == 8) {
#pragma unroll 2
    for (int k = 0; k < m; ++k)
      node_fwd<Pr, MODE>(L, tb.r[L.ou + k], tb.f[L.o1 + k], tb.f[L.o2 + k], tb.r[L.ow + k], M, H);
  } else {
#pragma unroll 4
    for (int k = 0; k < m; ++k)
      node_fwd<Pr, MODE>(L, tb.r[L.ou + k], tb.f[L.o1 + k], tb.f[L.o2 + k], tb.r[L.ow + k], M, H);
  }
}

template <typename Pr>
__device__ __forceinline__ void run_nodes_fwd(int mode, const Loop<Pr>& L, int m, const Tabs<Pr>& tb,
                                              typename Pr::R M[5], typename Pr::R H[3]) {
  const int wm = wave_mode(mode);
  if (wm == kLow)
    nodes_fwd<Pr, kLow>(L, m, tb, M, H);
  else if (wm == kHigh)
    nodes_fwd<Pr, kHigh>(L, m, tb, M, H);
  else
    nodes_fwd<Pr, kGen>(L, m, tb, M, H);
}

// Moment slots of a task: slot 0 low (scattering; pair piece A), high (scattering; pair
// piece B), slot 1 low (pair piece C). Groups add Es times their moments.
template <typename R>
struct Slots {
  R lo0[5], hi[3], lo1[5];
};

template <typename R>
__device__ __forceinline__ void add_group(const GroupDesc& G, double Es, const R M[5], const R H[3], Slots<R>& S) {
  const R es = R(Es);
  const R e0 = G.slot == 0 ? es : R(0), e1 = G.slot == 1 ? es : R(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    S.lo0[k] = Num<R>::fma(e0, M[k], S.lo0[k]);
    S.lo1[k] = Num<R>::fma(e1, M[k], S.lo1[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) S.hi[k] = Num<R>::fma(es, H[k], S.hi[k]);
}

// Task values (a struct, so that no array of them ever lives in scratch memory).
struct Q4 {
  double a, b, c, d;
};

// Coefficient tables are read through an opaque pointer at each use, so that the compiler
// reloads them (from cache) instead of keeping 26-32 doubles live across the node loops.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
  asm volatile("" : "+v"(p));
  return p;
}

template <typename R>
__device__ __forceinline__ void contract_pair(const PairCoef& C, const Slots<R>& S, double& q0, double& q1) {
  double q[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) a = fma(C.A[l][k], double(S.lo0[k]), a);
#pragma unroll
    for (int k = 0; k < 3; ++k) a = fma(C.B[l][k], double(S.hi[k]), a);
#pragma unroll
    for (int k = 0; k < 5; ++k) a = fma(C.C[l][k], double(S.lo1[k]), a);
    q[l] = a;
  }
  q0 = q[0];
  q1 = q[1];
}

// Task values from the slots (FP64 contraction with the coefficient tables): scattering
// (a, b, c, d) = (S, l) = (I,0), (I,1), (II,0), (II,1); pair (a, b) = l = 0, 1 of
// Phi_a,I(i, j) and (c, d) those of Phi_a,I(j, i).
template <typename R, bool PAIR>
__device__ __forceinline__ Q4 contract_task(const DevPlan& P, const Task& K, int t, const Slots<R>& S) {
  double q[4];
  if (!PAIR) {
    const NesCoef& C = *opaque(P.nes_coef + t);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) a = fma(C.lo[c][k], double(S.lo0[k]), a);
#pragma unroll
      for (int k = 0; k < 3; ++k) a = fma(C.hi[c][k], double(S.hi[k]), a);
      q[c] = a;
    }
  } else {
    contract_pair<R>(*opaque(P.pair_coef + K.i * P.ne + K.j), S, q[0], q[1]);
    contract_pair<R>(*opaque(P.pair_coef + K.j * P.ne + K.i), S, q[2], q[3]);
  }
  return {q[0], q[1], q[2], q[3]};
}

template <typename Pr, bool PAIR>
__device__ __forceinline__ Q4 task_forward(const DevPlan& P, const Tabs<Pr>& tb, const Zone& Z, int t) {
  using R = typename Pr::R;
  const Task K = make_task<PAIR>(P, t);
  const Brk Bk = task_breakpoints<PAIR>(K, Z);
  Slots<R> S = {};
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const Tri zero = {0.0, 0.0, 0.0};
    const Tri lo = g == 0 ? zero : group_hi<PAIR>(K, Bk, g - 1);
    const GroupDesc G = describe<PAIR>(P, K, Bk, g, lo, group_hi<PAIR>(K, Bk, g));
    if (wave_skips(G)) continue;
    Loop<Pr> L;
    const double Es = make_loop<Pr>(K, G, Z, L);
    R M[5] = {0, 0, 0, 0, 0}, H[3] = {0, 0, 0};
    run_nodes_fwd<Pr>(G.mode, L, P.m4, tb, M, H);
    add_group<R>(G, Es, M, H, S);
  }
  return contract_task<R, PAIR>(P, K, t, S);
}

// ----------------------------------------------------------------------------------------
// Workgroup layout: one zone per workgroup; in LDS (doubles): f [6 ne] | scattering task
// values [4 ntn] | pair task values [2 ntp] | exp(-|eps_i - eps_j|/T) [ne^2] |
// exp(-(eps_i + eps_j)/T) [ne^2] | contraction parts; the backward also holds g_eta, g_chi
// [12 ne] after f.

// Zone selection of a pass. The FP64 path takes every zone. The mixed path splits them into
// two classes by |eta_e|: up to its threshold (and values that do not compare) FP32, above it
// FP64. The threshold is capped at kFp32Range, which guards range, not accuracy: a task's whole
// integrand can sit near e^-|eta_e| (pair annihilation with mu_e above eps_i + eps_j), and FP32
// ends near e^-87.
constexpr int kSelAll = 0, kSelBulk = 1, kSelHigh = 2;
constexpr double kFp32Range = 64.0;

__device__ __forceinline__ bool selected(const DevPlan& P, int selm, double eta) {
  const bool high = fabs(eta) > fmin(P.eta_fp64, kFp32Range);
  return selm == kSelBulk ? !high : (selm == kSelHigh ? high : true);
}

// The zone of a pass's workgroup b. The FP64 path's single pass: zone b. The mixed path's class
// passes: the zones go in tiles of 64, and workgroup b takes tile t = b mod T (T tiles) and slot
// k = b div T, i.e. the k-th zone of the pass's class in that tile (in zone order), if the tile
// has more than k of them (-1 otherwise). Slot k is taken by workgroups k T .. k T + T - 1, so
// the workgroups that find a zone come first in the grid and those that find none last, with a
// band between them. Measured on the large workload's class passes (half the zones in each
// class), per step: a zone per workgroup in zone order, the two kinds alternating, 324 ms;
// these tiles 300 ms (tiles of 16 or 32 zones 306 and 303, of 512 zones 312; the slots of one
// tile on consecutive workgroups, 409; every chunk's zones sorted by class beforehand, 290).
// Every wave of the workgroup computes the same zone.
__device__ __forceinline__ int64_t pass_zone(const DevPlan& P, int selm, const double* etaz, int64_t nz) {
  const int64_t b = blockIdx.x;
  if (selm == kSelAll) return b < nz ? b : -1;
  const int64_t tiles = (nz + 63) >> 6, t = b % tiles;
  const int k = (int)(b / tiles);
  const int lane = threadIdx.x & 63;
  const int64_t zl = (t << 6) + lane;
  const bool in = zl < nz && selected(P, selm, etaz[zl]);
  const unsigned long long mask = __ballot(in);
  if (__popcll(mask) <= k) return -1;
  const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
  const unsigned long long hit = __ballot(in && (int)rank == k);
  return (t << 6) + (__ffsll((long long)hit) - 1);
}
__host__ __device__ constexpr int64_t pass_grid(int selm, int64_t nz) {
  return selm == kSelAll ? nz : ((nz + 63) >> 6) << 6;
}

__device__ void stage_zone_state(const DevPlan& P, int64_t z, const double* Tz, const double* etaz,
                                 Zone* zs) {   // zs[0]: the zone, zs[1]: its mirror
  if (threadIdx.x == 0) {
    Zone Z;
    Z.z = z;
    Z.valid = z >= 0;
    Z.T = Z.valid ? Tz[z] : 1.0;
    Z.eta = Z.valid ? etaz[z] : 0.0;
    Z.invT = 1.0 / Z.T;
    Z.mu = Z.eta * Z.T;
    Zone M = Z;
    M.eta = -Z.eta;
    M.mu = -Z.mu;
    Z.k = 0;
    M.k = 0;
    for (int j = 0; j < P.ne; ++j) {
      Z.k += P.eps[j] < Z.mu;
      M.k += P.eps[j] < M.mu;
    }
    zs[0] = Z;
    zs[1] = M;
  }
}

// LDS layout of a zone's task values (doubles), after `base` values of f (and gradients):
// scattering [4 ntn] | scattering on positrons [4 ntn, kernels built with NPS] | pair [2 ntp,
// slot of (i, j) at i ne + j] | detailed-balance factors [2 ne^2] | the rest.
//
// NPS (neutrino-positron scattering) is a template parameter of the kernels, chosen by the
// host from the process mask: kernels built without it carry none of its code, so the
// default processes run the smallest code.
struct Lay {
  int q, m, p, d;
};
template <bool NPS>
__device__ __forceinline__ Lay layout(const DevPlan& P, int base) {
  Lay L;
  L.q = base;
  L.m = L.q + 4 * P.ntn;
  L.p = L.m + (NPS ? 4 * P.ntn : 0);
  L.d = L.p + 2 * P.ntp;
  return L;
}

// Scattering kernel components of bin pair (i, j), electron and positron targets together in
// the electron-target coupling labels: the positron components (S, l) carry the couplings of
// (S', l), S' the other S (C_A -> -C_A), so they add to the other S. v[0..3] = (I,0), (I,1),
// (II,0), (II,1) of the down-scatter task tri(max, min).
__device__ __forceinline__ void scattering_values(const double* smem, const Lay& L, bool nes, bool nps, int tq,
                                                  double v[4]) {
  v[0] = v[1] = v[2] = v[3] = 0.0;
  if (nes) {
    const double* q = smem + L.q + tq;
    v[0] = q[0];
    v[1] = q[1];
    v[2] = q[2];
    v[3] = q[3];
  }
  if (nps) {
    const double* m = smem + L.m + tq;
    v[0] += m[2];
    v[1] += m[3];
    v[2] += m[0];
    v[3] += m[1];
  }
}

// Detailed-balance factors exp(-|eps_i - eps_j|/T) and exp(-(eps_i + eps_j)/T), FP64; both
// are symmetric in (i, j), so each is formed once for i >= j and stored twice.
__device__ void stage_factors(const DevPlan& P, const Zone& Z, double* s_d) {
  const int ne = P.ne, n2 = ne * ne;
  for (int r = threadIdx.x; r < P.ntn; r += blockDim.x) {
    const int ij = P.nes_ij[r], i = ij & 0xff, j = ij >> 8;
    const double ei = P.eps[i], ej = P.eps[j];
    const double d = exp(-(ei - ej) * Z.invT), pf = exp(-(ei + ej) * Z.invT);
    s_d[i * ne + j] = d;
    s_d[j * ne + i] = d;
    s_d[n2 + i * ne + j] = pf;
    s_d[n2 + j * ne + i] = pf;
  }
}

// Task units: units 0 .. nN-1 hold 64 scattering tasks each, the next nM 64 positron
// scattering tasks, the rest 64 pair tasks, each in its zone's task order (tasks whose groups
// take the same node-loop variants sit together). Wave w of workgroup b takes units
// (w + b) mod W, + W, ...; the rotation spreads the wave that holds one unit fewer over the
// SIMDs.
struct Units {
  int nN, nM, nU, first, step;
};
__device__ __forceinline__ Units task_units(int ntn, int ntm, int ntp) {
  Units U;
  U.nN = (ntn + 63) >> 6;
  U.nM = (ntm + 63) >> 6;
  U.nU = U.nN + U.nM + ((ntp + 63) >> 6);
  U.step = blockDim.x >> 6;
  U.first = __builtin_amdgcn_readfirstlane((int)(((threadIdx.x >> 6) + blockIdx.x) % U.step));
  return U;
}

// Parts of the per-zone contractions: lanes run (part, bin) and all three species, so that
// the lanes fill about one wave (64 / ne parts, from one to four).
__device__ __forceinline__ int bin_parts(int ne) {
  const int np = 64 / ne;
  return np < 1 ? 1 : (np > 4 ? 4 : np);
}

// Explicit Jacobian blocks of one zone, jac[s][p][o][i][j] (24 ne^2 doubles): the derivative
// of output o (eta0, chi0, eta1, chi1) of species s in bin i with respect to f_{o/2}(j) of
// species s (process p = 0, scattering) or of its pair partner (p = 1). The outputs are
// affine in f, so each block is a completed kernel times c0 w_j, the f-independent part of
// the Newton-Raphson Jacobian of the implicit transport step (Sect. 2.1). Lanes run bin
// pairs (i, j) and write each of the 24 blocks with consecutive j: every store of a wave is
// contiguous.
template <bool NPS>
__device__ void zone_jacobian(const DevPlan& P, const Zone& Z, const double* smem, double* __restrict__ jac) {
  const int ne = P.ne, n2 = ne * ne;
  const Lay L = layout<NPS>(P, 6 * ne);
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  double* out = jac + Z.z * (int64_t)(24 * n2);
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    const int i = e / ne, j = e - i * ne;
    const double cw = P.c0w[j];
    double v[4];
    scattering_values(smem, L, do_nes, do_nps, 4 * (i >= j ? tri(i, j) : tri(j, i)), v);
    const double q0 = v[0], q1 = v[1], q2 = v[2], q3 = v[3];
    const double dcw = cw * smem[L.d + e];
    const double cin = (i > j) ? dcw : cw, cout = (i < j) ? dcw : cw;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, pf = 0.0;
    if (do_pair) {
      const double* aij = smem + L.p + 2 * e;
      const double* aji = smem + L.p + 2 * (j * ne + i);
      a0 = aij[0];
      a1 = aij[1];
      b0 = aji[0];
      b1 = aji[1];
      pf = smem[L.d + n2 + e];
    }
    const double cwp = cw * pf, cwa = cw * (1.0 - pf);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
      const double k0 = bI * q0 + bII * q2, k1 = bI * q1 + bII * q3;
      const double ka0 = bI * a0 + bII * b0, ka1 = bI * a1 + bII * b1;
      double* o = out + s * 8 * n2 + e;
      o[0] = cin * k0;
      o[n2] = (cin - cout) * k0;
      o[2 * n2] = cin * k1;
      o[3 * n2] = (cin - cout) * k1;
      o[4 * n2] = -cwp * ka0;
      o[5 * n2] = cwa * ka0;
      o[6 * n2] = -cwp * ka1;
      o[7 * n2] = cwa * ka1;
    }
  }
}

// Completion, species combination and contraction of a zone's task values (LDS, layout L)
// with f (LDS, smem[0, 6 ne)) into eta, chi. One lane per (part, bin i) runs all three
// species over a part of j, so each (i, j) pair's task values, detailed-balance factors and
// weights are read and combined once; the parts (s_part, 12 npb ne doubles) are added in
// order.
template <bool NPS>
__device__ __forceinline__ void zone_contract(const DevPlan& P, const Zone& Z, const double* smem, const Lay& L,
                                              double* s_part, double* __restrict__ eta_out,
                                              double* __restrict__ chi_out) {
  const int ne = P.ne, n2 = ne * ne;
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  const int npb = bin_parts(ne);   // s_part: [part][i][species][eta0, chi0, eta1, chi1]
  for (int r = threadIdx.x; r < npb * ne; r += blockDim.x) {
    const int part = r / ne, i = r - part * ne;
    const int j0 = part * ne / npb, j1 = (part + 1) * ne / npb;
    const double* s_f = smem;
    const double* s_pa = smem + L.p;
    const double* s_d = smem + L.d;
    const double* s_p = s_d + n2;
    double acc[3][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    for (int j = j0; j < j1; ++j) {
      const double cw = P.c0w[j];
      const double dfac = s_d[i * ne + j];
      const double cin = (i > j) ? cw * dfac : cw, cout = (i < j) ? cw * dfac : cw;
      double fj[3][2];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        fj[s][0] = s_f[(2 * s) * ne + j];
        fj[s][1] = s_f[(2 * s + 1) * ne + j];
      }
      if (do_nes || do_nps) {
        double v[4];
        scattering_values(smem, L, do_nes, do_nps, 4 * (i >= j ? tri(i, j) : tri(j, i)), v);
        const double q0 = v[0], q1 = v[1], q2 = v[2], q3 = v[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
          const double k0 = bI * q0 + bII * q2, k1 = bI * q1 + bII * q3;
          const double t0 = fj[s][0] * k0, t1 = fj[s][1] * k1;
          acc[s][0] += cin * t0;
          acc[s][1] += cin * t0 + cout * (k0 - t0);
          acc[s][2] += cin * t1;
          acc[s][3] += (cin - cout) * t1;
        }
      }
      if (do_pair) {
        const double* aij = s_pa + 2 * (i * ne + j);
        const double* aji = s_pa + 2 * (j * ne + i);
        const double a0 = aij[0], a1 = aij[1], b0 = aji[0], b1 = aji[1];
        const double pf = s_p[i * ne + j], cwp = cw * pf;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          const int sb = partner(s);
          const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
          const double ka0 = bI * a0 + bII * b0, ka1 = bI * a1 + bII * b1;
          const double tp = fj[sb][0] * ka0, t1 = cw * fj[sb][1] * ka1;
          const double pr0 = cwp * (ka0 - tp);
          acc[s][0] += pr0;
          acc[s][1] += pr0 + cw * tp;
          acc[s][2] -= t1 * pf;
          acc[s][3] += t1 * (1.0 - pf);
        }
      }
    }
    double* pp = s_part + 12 * r;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      pp[4 * s] = acc[s][0];
      pp[4 * s + 1] = acc[s][1];
      pp[4 * s + 2] = acc[s][2];
      pp[4 * s + 3] = acc[s][3];
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 3 * ne; o += blockDim.x) {
    const int s = o / ne, i = o % ne;
    double e0 = 0.0, c0 = 0.0, e1 = 0.0, c1 = 0.0;
    for (int part = 0; part < npb; ++part) {
      const double* pp = s_part + 12 * (part * ne + i) + 4 * s;
      e0 += pp[0];
      c0 += pp[1];
      e1 += pp[2];
      c1 += pp[3];
    }
    const int64_t out = Z.z * 6 * ne + (2 * s) * ne + i;
    eta_out[out] = e0;
    chi_out[out] = c0;
    eta_out[out + ne] = e1;
    chi_out[out + ne] = c1;
  }
}

// Scattering task at position pos of the zone's task order: its four values into its slot.
template <typename Pr>
__device__ __forceinline__ void scattering_fwd(const DevPlan& P, const Tabs<Pr>& tb, const Zone& Z, double* slots,
                                               int pos) {
  const int t = P.task_order[Z.k * P.ntn + pos];
  const Q4 q = task_forward<Pr, false>(P, tb, Z, t);
  double* o = slots + 4 * t;
  o[0] = q.a;
  o[1] = q.b;
  o[2] = q.c;
  o[3] = q.d;
}

// Outputs of the forward kernels: eta, chi; the explicit Jacobian blocks (and eta, chi when
// eta_out is given); the task values themselves, packed (see export_tasks); or those in the
// interpolation variables of a table row.
constexpr int kOutRates = 0, kOutJac = 1, kOutTasks = 2, kOutTable = 3;

// Interpolation variables of a table row: each (task, S) pair (l = 0, l = 1), adjacent in the
// layout, as (ln x0, x1 / x0); x0 is positive and exponential in 1/T and eta_e, and
// |x1| <= x0 (|P_1| <= 1). x0 <= 0, only from underflow, is stored as (ln 1e-300, 0).
__device__ __forceinline__ void to_interp_vars(double x0, double x1, double& y0, double& y1) {
  const bool pos = x0 > 0.0;
  y0 = log(pos ? x0 : 1e-300);
  y1 = pos ? x1 / x0 : 0.0;
}

// A zone's task values from LDS to out[z][values], packed over the processes asked for:
// scattering [4 ntn] | positron scattering [4 ntn] | pair [2 ne^2] (the slot order of LDS);
// ROWS writes them in interpolation variables.
template <bool NPS, bool ROWS>
__device__ void export_tasks(const DevPlan& P, const Zone& Z, const double* smem, const Lay& L,
                             double* __restrict__ out) {
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  const int nv = (do_nes ? 4 * P.ntn : 0) + (do_nps ? 4 * P.ntn : 0) + (do_pair ? 2 * P.ntp : 0);
  double* o = out + Z.z * (int64_t)nv;
  int off = 0;
  for (int k = 0; k < 3; ++k) {
    const bool on = k == 0 ? do_nes : (k == 1 ? do_nps : do_pair);
    if (!on) continue;
    const int len = k == 2 ? 2 * P.ntp : 4 * P.ntn, src = k == 0 ? L.q : (k == 1 ? L.m : L.p);
    for (int r = threadIdx.x; r < len / 2; r += blockDim.x) {
      double y0 = smem[src + 2 * r], y1 = smem[src + 2 * r + 1];
      if (ROWS) to_interp_vars(y0, y1, y0, y1);
      o[off + 2 * r] = y0;
      o[off + 2 * r + 1] = y1;
    }
    off += len;
  }
}

// Forward of one zone: task values into LDS, then the contraction with f into eta, chi, or
// the explicit Jacobian blocks, which need no f (and the contraction as well when eta_out
// is given), or the task values themselves.
template <typename Pr, int OUT, bool NPS>
__device__ void zone_forward(const DevPlan& P, const Tabs<Pr>& tb, Zone* zs, double* smem, int64_t z,
                             const double* __restrict__ Tz, const double* __restrict__ etaz,
                             const double* __restrict__ f, double* __restrict__ eta_out,
                             double* __restrict__ chi_out, double* __restrict__ jac) {
  const int ne = P.ne, n2 = ne * ne;
  const Lay L = layout<NPS>(P, 6 * ne);
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  // task counts: scattering tasks (i >= j) on electrons and on positrons, pair tasks (one per
  // unordered pair {i, j})
  const int ntn = do_nes ? P.ntn : 0, ntm = do_nps ? P.ntn : 0, ntp = do_pair ? P.ntn : 0;
  stage_zone_state(P, z, Tz, etaz, zs);
  __syncthreads();
  const Zone& Z = zs[0];
  if (OUT == kOutRates || eta_out != nullptr)
    for (int r = threadIdx.x; r < 6 * ne; r += blockDim.x) smem[r] = f[Z.z * 6 * ne + r];
  stage_factors(P, Z, smem + L.d);
  const Units U = task_units(ntn, ntm, ntp);
  const int lane = threadIdx.x & 63;
  for (int u = U.first; u < U.nU; u += U.step) {
    // scattering on electrons, then on positrons (the mirrored zone); one call site serves
    // both, and without NPS the selection folds away
    if (u < U.nN + U.nM) {
      const bool mir = NPS && u >= U.nN;
      const int pos = ((mir ? u - U.nN : u) << 6) + lane;
      if (pos < (mir ? ntm : ntn)) scattering_fwd<Pr>(P, tb, zs[mir ? 1 : 0], smem + (mir ? L.m : L.q), pos);
    } else {
      const int pos = ((u - U.nN - U.nM) << 6) + lane;
      if (pos < ntp) {
        const int t = P.task_order[Z.k * P.ntn + pos], ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
        const Q4 q = task_forward<Pr, true>(P, tb, Z, t);
        double* o = smem + L.p + 2 * (i * ne + j);
        o[0] = q.a;
        o[1] = q.b;
        o = smem + L.p + 2 * (j * ne + i);   // the same slot on the diagonal, same values
        o[0] = q.c;
        o[1] = q.d;
      }
    }
  }
  __syncthreads();
  if (OUT == kOutTasks || OUT == kOutTable) {
    export_tasks<NPS, OUT == kOutTable>(P, Z, smem, L, jac);
    return;
  }
  if (OUT == kOutJac) {
    zone_jacobian<NPS>(P, Z, smem, jac);
    if (eta_out == nullptr) return;   // uniform: a kernel argument
  }
  zone_contract<NPS>(P, Z, smem, L, smem + L.d + 2 * n2, eta_out, chi_out);
}

// Workgroup b takes the zone pass_zone gives it. Occupancy targets (waves per SIMD): Fp32
// five (at most 102 VGPRs; five one-zone workgroups of 31 KB fill the 160 KB of LDS at 21
// bins), Fp64 three (four would spill); the FP64 export of task values for tables
// (built once per lattice) two, where three would spill.
template <typename Pr, int OUT>
constexpr int fwd_waves() {
  return sizeof(typename Pr::R) == 8 ? ((OUT == kOutTasks || OUT == kOutTable) ? 2 : 3) : 5;
}

template <typename Pr, int OUT, bool NPS>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(fwd_waves<Pr, OUT>())))
void rates_forward_kernel(DevPlan P, int64_t nz, int selm, const double* __restrict__ Tz,
                          const double* __restrict__ etaz, const double* __restrict__ f,
                          double* __restrict__ eta_out, double* __restrict__ chi_out, double* __restrict__ jac) {
  __shared__ double tab[(tab_bytes<Pr>() + 7) / 8];
  __shared__ Zone zs[2];
  extern __shared__ double smem[];
  const int64_t z = pass_zone(P, selm, etaz, nz);
  if (z < 0) return;   // uniform: one zone per workgroup
  const Tabs<Pr> tb = stage_tabs<Pr>(P, tab);
  zone_forward<Pr, OUT, NPS>(P, tb, zs, smem, z, Tz, etaz, f, eta_out, chi_out, jac);
}

// Interpolated forward: a zone's task values interpolated bilinearly from a table of task
// values on a regular lattice of zone states in (ln T, eta_e) (rows in the export layout, in
// interpolation variables), then completed and contracted with the zone's own T and f like
// the forward. Interpolation and contraction run in FP64 whatever precision built the table.
template <bool NPS>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(5))) void rates_interp_kernel(DevPlan P, vtx_lattice lat,
                                                                 const double* __restrict__ table, int64_t nz,
                                                                 const double* __restrict__ Tz,
                                                                 const double* __restrict__ etaz,
                                                                 const double* __restrict__ f,
                                                                 double* __restrict__ eta_out,
                                                                 double* __restrict__ chi_out) {
  __shared__ Zone zs[2];
  extern __shared__ double smem[];
  const int64_t z = blockIdx.x;
  stage_zone_state(P, z < nz ? z : -1, Tz, etaz, zs);
  __syncthreads();
  const Zone& Z = zs[0];
  if (!Z.valid) return;   // uniform
  const int ne = P.ne, n2 = ne * ne;
  const Lay L = layout<NPS>(P, 6 * ne);
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  const int nv = (do_nes ? 4 * P.ntn : 0) + (do_nps ? 4 * P.ntn : 0) + (do_pair ? 2 * P.ntp : 0);
  for (int r = threadIdx.x; r < 6 * ne; r += blockDim.x) smem[r] = f[Z.z * 6 * ne + r];
  stage_factors(P, Z, smem + L.d);
  // the cell (a, b) and the fractions (u, v); outside the lattice the edge cell extrapolates
  const double s = (log(Z.T) - lat.lnT0) / lat.dlnT, rr = (Z.eta - lat.eta0) / lat.deta;
  const double af = fmin(fmax(floor(s), 0.0), double(lat.nt - 2)), bf = fmin(fmax(floor(rr), 0.0), double(lat.nh - 2));
  const int a = int(af), b = int(bf);
  const double u = s - af, v = rr - bf;
  const double c00 = (1.0 - u) * (1.0 - v), c10 = u * (1.0 - v), c01 = (1.0 - u) * v, c11 = u * v;
  const double* t00 = table + ((int64_t)a * lat.nh + b) * nv;
  const double* t10 = table + ((int64_t)(a + 1) * lat.nh + b) * nv;
  const double* t01 = t00 + nv;
  const double* t11 = t10 + nv;
  // rows hold interpolation variables (ln x0, x1 / x0) per (task, S) pair; back by
  // x0 = exp(y0), x1 = y1 x0. Bilinear in them is exact for exponential dependence.
  int off = 0;
  for (int k = 0; k < 3; ++k) {
    const bool on = k == 0 ? do_nes : (k == 1 ? do_nps : do_pair);
    if (!on) continue;
    const int len = k == 2 ? 2 * P.ntp : 4 * P.ntn, dst = k == 0 ? L.q : (k == 1 ? L.m : L.p);
    for (int r = threadIdx.x; r < len / 2; r += blockDim.x) {
      const int q = off + 2 * r;
      const double2 a00 = *reinterpret_cast<const double2*>(t00 + q);
      const double2 a10 = *reinterpret_cast<const double2*>(t10 + q);
      const double2 a01 = *reinterpret_cast<const double2*>(t01 + q);
      const double2 a11 = *reinterpret_cast<const double2*>(t11 + q);
      const double y0 = c00 * a00.x + c10 * a10.x + c01 * a01.x + c11 * a11.x;
      const double y1 = c00 * a00.y + c10 * a10.y + c01 * a01.y + c11 * a11.y;
      const double x0 = exp(y0);
      smem[dst + 2 * r] = x0;
      smem[dst + 2 * r + 1] = y1 * x0;
    }
    off += len;
  }
  __syncthreads();
  zone_contract<NPS>(P, Z, smem, L, smem + L.d + 2 * n2, eta_out, chi_out);
}

// ---------------------------------------------------------------------------------------
// Backward (vector-Jacobian product). Recomputes every task's kernel values and, in the
// same node loop, the derivative of the adjoint-weighted kernel sum_c A_c q_c along T and
// eta_e, node motion included. A_c are the upstream weights of each task component.
//
// Each of the three maps m is affine along a group, m = m_A (1 - x) + m_B x on a panel (x the
// Legendre node on [0, 1]) or m_A + s_m x on the tail, so with the group weight Es w_k the
// derivative of Es sum_k w_k B_k H(u_k) along theta is
//   dEs/dtheta sum w B H + Es sum_m [dm_A/dtheta S_mA + dm_B/dtheta S_mB],
// S_zA = sum w B H r_z (1 - x), S_zB = sum w B H r_z x (r_z = d log sigma / dz = 1 - sigma(z))
// for the two Fermi-Dirac arguments and S_uA, S_uB likewise with w B dH/du (tail: weights 1
// and x, dm_B the slope's derivative). The node loop accumulates these sums; the group end
// applies the FP64 derivatives of the end points' map values.

struct Adj {
  const double* f;
  const double* ge;
  const double* gc;
  int ne;
  __device__ double F(int s, int m, int i) const { return f[(2 * s + m) * ne + i]; }
  __device__ double GE(int s, int m, int i) const { return ge[(2 * s + m) * ne + i]; }
  __device__ double GC(int s, int m, int i) const { return gc[(2 * s + m) * ne + i]; }
};

// Upstream weights of a scattering task (i >= j): for (S, l), the weight of Phi_out_{l,S}(a, b)
// plus that of Phi_in_{l,S}(b, a) in L is
//   ghat(a, b) = c0 w_b sum_s beta_S(s) gchi_l(s, a) ft_l(s, b) + c0 w_a sum_s beta_S(s) (geta + gchi)_l(s, b) f_l(s, a),
// ft_0 = 1 - f_0, ft_1 = -f_1. The task carries ghat(i, j) + d ghat(j, i) (d the detailed-balance
// factor, i > j); up receives d ghat(j, i). Each species' values at i and j are read once.
__device__ __forceinline__ void nes_adjoint(const DevPlan& P, const Adj& A, int i, int j, double d, double w[4],
                                            double up[4]) {
  const double cwi = P.c0w[i], cwj = P.c0w[j];
  const bool off = i > j;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    double oI = 0.0, oII = 0.0, iI = 0.0, iII = 0.0;   // (a, b) = (i, j): out and in sums
    double pI = 0.0, pII = 0.0, qI = 0.0, qII = 0.0;   // (a, b) = (j, i)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
      const double fi = A.F(s, l, i), fj = A.F(s, l, j);
      const double ci = A.GC(s, l, i), cj = A.GC(s, l, j);
      const double gi = A.GE(s, l, i) + ci, gj = A.GE(s, l, j) + cj;
      const double fti = l == 0 ? 1.0 - fi : -fi, ftj = l == 0 ? 1.0 - fj : -fj;
      const double o1 = ci * ftj, i1 = gj * fi, o2 = cj * fti, i2 = gi * fj;
      oI += bI * o1;
      oII += bII * o1;
      iI += bI * i1;
      iII += bII * i1;
      pI += bI * o2;
      pII += bII * o2;
      qI += bI * i2;
      qII += bII * i2;
    }
    const double uI = off ? d * (cwi * pI + cwj * qI) : 0.0, uII = off ? d * (cwi * pII + cwj * qII) : 0.0;
    up[l] = uI;
    up[2 + l] = uII;
    w[l] = cwj * oI + cwi * iI + uI;
    w[2 + l] = cwj * oII + cwi * iII + uII;
  }
}

// Upstream weights of a pair task {i, j}: for orientation (a, b) and l, the weight of
// Phi_a,I(a, b) collects Phi_a_{l,I}(a, b) and Phi_a_{l,II}(b, a). With partner species sb,
//   ponly_S(a, b) = c0 w_b sum_s beta_S(s) (geta + gchi)_l(s, a) ft_l(sb, b),
//   P2_S(a, b)    = c0 w_b sum_s beta_S(s) gchi_l(s, a) f_l(sb, b),
// the weight is p (ponly_I(a, b) + ponly_II(b, a)) + P2_I(a, b) + P2_II(b, a) and its
// p-coefficient (for d/dT of the production factor) ponly_I(a, b) + ponly_II(b, a).
__device__ __forceinline__ void pair_adjoint(const DevPlan& P, const Adj& A, int i, int j, double pf, double w[4],
                                             double pc[4]) {
  const double cwi = P.c0w[i], cwj = P.c0w[j];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    double fi[3], fj[3], ci[3], cj[3], gi[3], gj[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      fi[s] = A.F(s, l, i);
      fj[s] = A.F(s, l, j);
      ci[s] = A.GC(s, l, i);
      cj[s] = A.GC(s, l, j);
      gi[s] = A.GE(s, l, i) + ci[s];
      gj[s] = A.GE(s, l, j) + cj[s];
    }
    // sums over s with the partner's f at b: (a, b) = (i, j) -> 1, (j, i) -> 2
    double pI1 = 0.0, pII1 = 0.0, cI1 = 0.0, cII1 = 0.0, pI2 = 0.0, pII2 = 0.0, cI2 = 0.0, cII2 = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int sb = partner(s);
      const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
      const double ftj = l == 0 ? 1.0 - fj[sb] : -fj[sb], fti = l == 0 ? 1.0 - fi[sb] : -fi[sb];
      pI1 += bI * gi[s] * ftj;    // ponly_I(i, j) / c0 w_j
      pII1 += bII * gj[s] * fti;  // ponly_II(j, i) / c0 w_i
      cI1 += bI * ci[s] * fj[sb];
      cII1 += bII * cj[s] * fi[sb];
      pI2 += bI * gj[s] * fti;    // ponly_I(j, i) / c0 w_i
      pII2 += bII * gi[s] * ftj;  // ponly_II(i, j) / c0 w_j
      cI2 += bI * cj[s] * fi[sb];
      cII2 += bII * ci[s] * fj[sb];
    }
    const double p1 = cwj * pI1 + cwi * pII1, p2 = cwi * pI2 + cwj * pII2;
    pc[l] = p1;
    pc[2 + l] = p2;
    w[l] = pf * p1 + cwj * cI1 + cwi * cII1;
    w[2 + l] = pf * p2 + cwi * cI2 + cwj * cII2;
  }
}

// Adjoint-weighted angular weight of a piece and its u-derivative:
//   low:  H = u^3 sum_j hl_j q_j(u), dH/du = u^2 sum_j dl_j q_j(u);
//   high: H = hh0 + hh1 u + hh2 u^2, dH/du = dh0 + dh1 u.
template <typename R>
struct AdjPoly {
  R hl[5], dl[5], hh[3], dh[2];
};

// From folded Bernstein coefficients g_3..g_7 (g_k of u^k v^(7-k)), differentiating term by
// term: dH/du = sum_m D_m u^m v^(6-m), D_m = (m + 1) g_(m+1) - (7 - m) g_m, m = 2..6.
template <typename R>
__device__ __forceinline__ void make_adj_poly(const double lo[5], const double hi[3], AdjPoly<R>& Q) {
  Q.dl[0] = R(3.0 * lo[0]);
  Q.dl[1] = R(4.0 * lo[1] - 4.0 * lo[0]);
  Q.dl[2] = R(5.0 * lo[2] - 3.0 * lo[1]);
  Q.dl[3] = R(6.0 * lo[3] - 2.0 * lo[2]);
  Q.dl[4] = R(7.0 * lo[4] - lo[3]);
#pragma unroll
  for (int k = 0; k < 5; ++k) Q.hl[k] = R(lo[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) Q.hh[k] = R(hi[k]);
  Q.dh[0] = R(hi[1]);
  Q.dh[1] = R(2.0 * hi[2]);
}

// The same from coefficients already in the bulk type.
template <typename R>
__device__ __forceinline__ void make_adj_poly_r(const R lo[5], const R hi[3], AdjPoly<R>& Q) {
  Q.dl[0] = R(3) * lo[0];
  Q.dl[1] = R(4) * (lo[1] - lo[0]);
  Q.dl[2] = R(5) * lo[2] - R(3) * lo[1];
  Q.dl[3] = R(6) * lo[3] - R(2) * lo[2];
  Q.dl[4] = R(7) * lo[4] - lo[3];
#pragma unroll
  for (int k = 0; k < 5; ++k) Q.hl[k] = lo[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) Q.hh[k] = hi[k];
  Q.dh[0] = hi[1];
  Q.dh[1] = R(2) * hi[2];
}

// Sum over a group's nodes of x0 (node weight x blocking factor x adjoint-weighted angular
// weight): the adjoint coefficients applied to the group's moments, since x0 = p H_low + wh H_high
// node by node.
template <typename R>
__device__ __forceinline__ R adjoint_sum(const AdjPoly<R>& Q, const R M[5], const R H[3]) {
  using N = Num<R>;
  R s = Q.hh[0] * H[0];
  s = N::fma(Q.hh[1], H[1], s);
  s = N::fma(Q.hh[2], H[2], s);
#pragma unroll
  for (int k = 0; k < 5; ++k) s = N::fma(Q.hl[k], M[k], s);
  return s;
}

// Per node, x0 = w B H (H the adjoint-weighted angular weight) and yu = w B dH/du. S[1..4]
// collect x0 r1 and x0 r2 (r = d ln sigma / dz of each blocking factor) times the end weights
// pa and pb; S[5..6] collect yu times pa and pb; S[0] = sum x0 is adjoint_sum afterwards.
template <typename Pr, int MODE>
__device__ __forceinline__ void node_bwd(const Loop<Pr>& L, const AdjPoly<typename Pr::R>& Q, typename Pr::R xu,
                                         typename Pr::F x1, typename Pr::F x2, typename Pr::R w,
                                         typename Pr::R pa, typename Pr::R pb, typename Pr::R M[5],
                                         typename Pr::R H[3], typename Pr::R S[7]) {
  using R = typename Pr::R;
  using F = typename Pr::F;
  using N = Num<R>;
  const R u = N::fma(L.u1, xu, L.u0);
  const F z1 = Num<F>::fma(L.a1, x1, L.a0), z2 = Num<F>::fma(L.b1, x2, L.b0);
  // B = sigma(z1) sigma(z2) and r = 1 - sigma(z) of each factor; where exp(-z) overflows,
  // sigma = 0 and r = 1 are the limits, so no argument needs a clamp
  R B, r1, r2;
  blocking_bwd<R>(z1, z2, L.C, B, r1, r2);
  const R wB = w * B;
  R ul = u, wh = wB;
  if (MODE == kGen) {
    const bool lo = u < L.split;
    ul = lo ? u : R(0);
    wh = lo ? R(0) : wB;
  }
  R x0 = R(0), yu = R(0);
  if (MODE != kHigh) {
    const R v = R(1) - ul, u2 = ul * ul, v2 = v * v, uv = ul * v;
    const R q0 = v2 * v2, q1 = uv * v2, q2 = uv * uv, q3 = uv * u2, q4 = u2 * u2;
    const R w2 = wB * u2, p = w2 * ul;
    M[0] = N::fma(p, q0, M[0]);
    M[1] = N::fma(p, q1, M[1]);
    M[2] = N::fma(p, q2, M[2]);
    M[3] = N::fma(p, q3, M[3]);
    M[4] = N::fma(p, q4, M[4]);
    const R hq = N::fma(Q.hl[4], q4, N::fma(Q.hl[3], q3, N::fma(Q.hl[2], q2, N::fma(Q.hl[1], q1, Q.hl[0] * q0))));
    const R dq = N::fma(Q.dl[4], q4, N::fma(Q.dl[3], q3, N::fma(Q.dl[2], q2, N::fma(Q.dl[1], q1, Q.dl[0] * q0))));
    x0 = p * hq;
    yu = w2 * dq;
  }
  if (MODE != kLow) {
    H[0] = H[0] + wh;
    H[1] = N::fma(wh, u, H[1]);
    H[2] = N::fma(wh, u * u, H[2]);
    const R hh = N::fma(N::fma(Q.hh[2], u, Q.hh[1]), u, Q.hh[0]);
    const R dh = N::fma(Q.dh[1], u, Q.dh[0]);
    if (MODE == kHigh) {
      x0 = wh * hh;
      yu = wh * dh;
    } else {
      x0 = N::fma(wh, hh, x0);
      yu = N::fma(wh, dh, yu);
    }
  }
  const R y1 = x0 * r1, y2 = x0 * r2;
  S[1] = N::fma(y1, pa, S[1]);
  S[2] = N::fma(y1, pb, S[2]);
  S[3] = N::fma(y2, pa, S[3]);
  S[4] = N::fma(y2, pb, S[4]);
  S[5] = N::fma(yu, pa, S[5]);
  S[6] = N::fma(yu, pb, S[6]);
}

template <typename Pr, int MODE>
__device__ __forceinline__ void nodes_bwd(const Loop<Pr>& L, const AdjPoly<typename Pr::R>& Q, int m,
                                          const Tabs<Pr>& tb, typename Pr::R M[5], typename Pr::R H[3],
                                          typename Pr::R S[7]) {
#pragma unroll 2
  for (int k = 0; k < m; ++k)
    node_bwd<Pr, MODE>(L, Q, tb.r[L.ou + k], tb.f[L.o1 + k], tb.f[L.o2 + k], tb.r[L.ow + k], tb.r[L.oa + k],
                       tb.r[L.ob + k], M, H, S);
}

template <typename Pr>
__device__ __forceinline__ void run_nodes_bwd(int mode, const Loop<Pr>& L, const AdjPoly<typename Pr::R>& Q, int m,
                                              const Tabs<Pr>& tb, typename Pr::R M[5], typename Pr::R H[3],
                                              typename Pr::R S[7]) {
  const int wm = wave_mode(mode);
  if (wm == kLow)
    nodes_bwd<Pr, kLow>(L, Q, m, tb, M, H, S);
  else if (wm == kHigh)
    nodes_bwd<Pr, kHigh>(L, Q, m, tb, M, H, S);
  else
    nodes_bwd<Pr, kGen>(L, Q, m, tb, M, H, S);
}

// Derivatives of the map values at a group end E (a breakpoint with its derivatives):
// z1 = sg (mu - E)/T gives dz1/dT = sg (eta - E_T)/T - z1/T, dz1/deta = sg (1 - E_eta/T);
// z2 = D/T - z1 - ... gives dz2/dT = -sg (eta - E_T)/T - z2/T, dz2/deta = -dz1/deta;
// u = E ub (or (w - E) ub) gives du = +-ub dE.
struct EndD {
  double uT, uE, z1T, z1E, z2T, z2E;
};
__device__ __forceinline__ EndD end_derivs(const Task& K, const GroupDesc& G, const Zone& Z, const Tri& E,
                                           const EndV& v) {
  const double gT = K.sg * (Z.eta - E.dT) * Z.invT, gE = K.sg * (1.0 - E.dE * Z.invT);
  const double dudE = G.c ? -G.ub : G.ub;
  return {dudE * E.dT, dudE * E.dE, gT - v.z1 * Z.invT, gE, -gT - v.z2 * Z.invT, -gE};
}

// Group end of the backward: adds the group's d/dT and d/deta_e of the adjoint-weighted
// kernel. Along the group a map is A (1 - x) + B x (panel) or A + slope x (tail), so its
// derivative at a node is dA (1 - x) + dB x (or dA + dslope x), and the node sums weighted by
// those two end weights turn into the derivative with the end points' derivatives alone.
template <typename R>
__device__ __forceinline__ void group_grad(const Task& K, const GroupDesc& G, const Zone& Z, double Es, const R S[7],
                                           double& gT, double& gE) {
  const EndD dA = end_derivs(K, G, Z, G.lo, end_values(K, G, Z, G.lo.v));
  EndD dB;
  double EsT, EsE;
  if (G.lag) {
    dB = {G.c ? -G.ub : G.ub, 0.0, 0.0, 0.0, 0.0, 0.0};   // slopes: u's is ub T, the arguments' are constants
    EsT = 1.0;
    EsE = 0.0;
  } else {
    dB = end_derivs(K, G, Z, G.hi, end_values(K, G, Z, G.hi.v));
    EsT = G.hi.dT - G.lo.dT;
    EsE = G.hi.dE - G.lo.dE;
  }
  const double s0 = double(S[0]), s1 = double(S[1]), s2 = double(S[2]), s3 = double(S[3]), s4 = double(S[4]),
               s5 = double(S[5]), s6 = double(S[6]);
  gT += Es * (dA.uT * s5 + dB.uT * s6 + dA.z1T * s1 + dB.z1T * s2 + dA.z2T * s3 + dB.z2T * s4) + EsT * s0;
  gE += Es * (dA.uE * s5 + dB.uE * s6 + dA.z1E * s1 + dB.z1E * s2 + dA.z2E * s3 + dB.z2E * s4) + EsE * s0;
}

// Recompute one task with derivatives. adj: upstream weights of the task components
// (scattering: the four (S, l); pair: l = 0, 1 of both orientations). Returns the task
// values q and adds d/dT, d/deta_e to gT, gE. lq: the lane's LDS slot (13 values, stride
// kSlotStride) that holds a pair task's adjoint-weighted piece coefficients A[5] | B[3] | C[5].
template <typename Pr, bool PAIR>
__device__ __forceinline__ Q4 task_backward(const DevPlan& P, const Tabs<Pr>& tb, const Zone& Z, int t, const Q4& adj,
                                            typename Pr::R* lq, double& gT, double& gE) {
  using R = typename Pr::R;
  constexpr int bs = kSlotStride;
  const Task K = make_task<PAIR>(P, t);
  const Brk Bk = task_breakpoints<PAIR>(K, Z);
  Slots<R> Sl = {};
  AdjPoly<R> Q;
  if (!PAIR) {
    const NesCoef& C = *opaque(P.nes_coef + t);
    double lo[5], hi[3];
#pragma unroll
    for (int k = 0; k < 5; ++k)
      lo[k] = adj.a * C.lo[0][k] + adj.b * C.lo[1][k] + adj.c * C.lo[2][k] + adj.d * C.lo[3][k];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      hi[k] = adj.a * C.hi[0][k] + adj.b * C.hi[1][k] + adj.c * C.hi[2][k] + adj.d * C.hi[3][k];
    make_adj_poly<R>(lo, hi, Q);
  } else {
    // adjoint weights (a, b) of Phi_a,I(i, j) and (c, d) of Phi_a,I(j, i), l = 0, 1
    const PairCoef& C = *opaque(P.pair_coef + K.i * P.ne + K.j);
    const PairCoef& D = *opaque(P.pair_coef + K.j * P.ne + K.i);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      lq[k * bs] = R(adj.a * C.A[0][k] + adj.b * C.A[1][k] + adj.c * D.A[0][k] + adj.d * D.A[1][k]);
      lq[(8 + k) * bs] = R(adj.a * C.C[0][k] + adj.b * C.C[1][k] + adj.c * D.C[0][k] + adj.d * D.C[1][k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      lq[(5 + k) * bs] = R(adj.a * C.B[0][k] + adj.b * C.B[1][k] + adj.c * D.B[0][k] + adj.d * D.B[1][k]);
  }
  // kept rolled: unrolled, the four groups' live state exceeds the register budget; the lower
  // end of a group is the upper end of the one before
  Tri lo = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const Tri hi = group_hi<PAIR>(K, Bk, g);
    const GroupDesc G = describe<PAIR>(P, K, Bk, g, lo, hi);
    lo = hi;
    if (wave_skips(G)) continue;
    Loop<Pr> L;
    const double Es = make_loop<Pr>(K, G, Z, L);
    if (PAIR) {
      // the group's piece: A (slots 0-4), B (5-7) or C (8-12); the other part stays zero
      const R* pl = lq + (G.piece == 2 ? 8 : 0) * bs;
      R lo[5], hi[3];
#pragma unroll
      for (int k = 0; k < 5; ++k) lo[k] = G.piece == 1 ? R(0) : pl[k * bs];
#pragma unroll
      for (int k = 0; k < 3; ++k) hi[k] = G.piece == 1 ? lq[(5 + k) * bs] : R(0);
      make_adj_poly_r<R>(lo, hi, Q);
    }
    R M[5] = {0, 0, 0, 0, 0}, H[3] = {0, 0, 0}, S[7] = {0, 0, 0, 0, 0, 0, 0};
    run_nodes_bwd<Pr>(G.mode, L, Q, P.m4, tb, M, H, S);
    S[0] = adjoint_sum<R>(Q, M, H);
    add_group<R>(G, Es, M, H, Sl);
    group_grad<R>(K, G, Z, Es, S, gT, gE);
  }
  return contract_task<R, PAIR>(P, K, t, Sl);
}

// Sum over the 64 lanes of a wave (lane 0's value is the one used: its summation order
// depends only on lane positions).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Scattering task t in the backward: upstream weights of its components, recomputation with
// derivatives, and the T-derivative of its detailed-balance completion. The task's LDS slot
// holds the completion weights until the task values replace them. On positron targets
// (swap) the component (S, l) carries the couplings of the other S, so the weights of S = I
// and S = II trade places.
template <typename Pr>
__device__ __forceinline__ void nes_task_bwd(const DevPlan& P, const Tabs<Pr>& tb, const Zone& Z, const Adj& A,
                                             const double* s_d, double* s_u, bool swap, typename Pr::R* lq, int t,
                                             double& dT, double& dE) {
  const int ne = P.ne, ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
  double* o = s_u + 4 * t;
  double v[4], vu[4], w[4], up[4];
  nes_adjoint(P, A, i, j, s_d[i * ne + j], v, vu);
  const double v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3], u0 = vu[0], u1 = vu[1], u2 = vu[2], u3 = vu[3];
  w[0] = swap ? v2 : v0;
  w[1] = swap ? v3 : v1;
  w[2] = swap ? v0 : v2;
  w[3] = swap ? v1 : v3;
  up[0] = swap ? u2 : u0;
  up[1] = swap ? u3 : u1;
  up[2] = swap ? u0 : u2;
  up[3] = swap ? u1 : u3;
  o[0] = up[0];
  o[1] = up[1];
  o[2] = up[2];
  o[3] = up[3];
  const Q4 q = task_backward<Pr, false>(P, tb, Z, t, Q4{w[0], w[1], w[2], w[3]}, lq, dT, dE);
  // completion: Phi_out(j, i) = exp(-(eps_i - eps_j)/T) q, d/dT = (eps_i - eps_j)/T^2 times it
  dT += (q.a * o[0] + q.b * o[1] + q.c * o[2] + q.d * o[3]) * (P.eps[i] - P.eps[j]) * (Z.invT * Z.invT);
  o[0] = q.a;
  o[1] = q.b;
  o[2] = q.c;
  o[3] = q.d;
}

// Pair task t (i >= j) in the backward, covering Phi_a(i, j) and Phi_a(j, i) (once on the
// diagonal); the production factor's weights wait in the two tasks' LDS slots.
template <typename Pr>
__device__ __forceinline__ void pair_task_bwd(const DevPlan& P, const Tabs<Pr>& tb, const Zone& Z, const Adj& A,
                                              const double* s_p, double* s_pa, typename Pr::R* lq, int t, double& dT,
                                              double& dE) {
  const int ne = P.ne, ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
  const bool off = i != j;
  const double pf = s_p[i * ne + j];   // symmetric in (i, j)
  double* o1 = s_pa + 2 * (i * ne + j);
  double* o2 = s_pa + 2 * (j * ne + i);
  double w[4], pc[4];
  pair_adjoint(P, A, i, j, pf, w, pc);
  o1[0] = pc[0];
  o1[1] = pc[1];
  if (off) {
    o2[0] = pc[2];
    o2[1] = pc[3];
  }
  const Q4 q = task_backward<Pr, true>(P, tb, Z, t, Q4{w[0], w[1], off ? w[2] : 0.0, off ? w[3] : 0.0}, lq, dT, dE);
  // production factor p = exp(-(eps_i + eps_j)/T): d/dT = (eps_i + eps_j)/T^2 p
  const double pw = pf * (P.eps[i] + P.eps[j]) * (Z.invT * Z.invT);
  dT += (q.a * o1[0] + q.b * o1[1]) * pw;
  o1[0] = q.a;
  o1[1] = q.b;
  if (off) {
    dT += (q.c * o2[0] + q.d * o2[1]) * pw;
    o2[0] = q.c;
    o2[1] = q.d;
  }
}

// Task units of one zone, at most: 3 ceil(528/64) at 32 bins.
constexpr int kMaxUnits = 32;

// Backward of one zone; FUSED also contracts the recomputed task values with f into eta, chi
// (forward and backward in one pass).
template <typename Pr, bool NPS, bool FUSED>
__device__ void zone_backward(const DevPlan& P, const Tabs<Pr>& tb, Zone* zs, double* red, double* smem, int64_t z,
                              const double* __restrict__ Tz, const double* __restrict__ etaz,
                              const double* __restrict__ f, const double* __restrict__ g_eta,
                              const double* __restrict__ g_chi, double* __restrict__ gT_out,
                              double* __restrict__ gE_out, double* __restrict__ gf_out, double* __restrict__ eta_out,
                              double* __restrict__ chi_out) {
  const int ne = P.ne, n2 = ne * ne;
  const bool do_nes = P.processes & VTX_NES, do_nps = NPS && (P.processes & VTX_NPS),
             do_pair = P.processes & VTX_PAIR;
  const int ntn = do_nes ? P.ntn : 0, ntm = do_nps ? P.ntn : 0, ntp = do_pair ? P.ntn : 0;
  // f | g_eta | g_chi [6 ne each] | task values (layout(), full-size scattering and pair
  // regions whatever the process mask) | detailed-balance factors [2 ne^2]
  const int off_ge = 6 * ne, off_gc = 12 * ne;
  const Lay L = layout<NPS>(P, 18 * ne);
  stage_zone_state(P, z, Tz, etaz, zs);
  __syncthreads();
  const Zone& Z = zs[0];
  if (!Z.valid) return;   // uniform: every lane reads the same zone state
  for (int r = threadIdx.x; r < 6 * ne; r += blockDim.x) {
    const int64_t g = Z.z * 6 * ne + r;
    smem[r] = f[g];
    smem[off_ge + r] = g_eta[g];
    smem[off_gc + r] = g_chi[g];
  }
  stage_factors(P, Z, smem + L.d);
  __syncthreads();
  const Adj A{smem, smem + off_ge, smem + off_gc, ne};
  const Units U = task_units(ntn, ntm, ntp);
  const int lane = threadIdx.x & 63;
  // per-lane slots after the contraction parts: 13 bulk-type values per lane, stride
  // kSlotStride, in banks of kSlotStride lanes (a constant stride folds into the LDS offsets)
  using R = typename Pr::R;
  R* lq = reinterpret_cast<R*>(smem + L.d + 2 * n2 + 24 * ne) + (threadIdx.x % kSlotStride) +
          (threadIdx.x / kSlotStride) * (13 * kSlotStride);
  // d/dT and d/deta_e: summed per unit in the unit's wave, then over units in unit order, so
  // the result does not depend on which wave ran which unit
  for (int u = U.first; u < U.nU; u += U.step) {
    double dT = 0.0, dE = 0.0;
    if (u < U.nN + U.nM) {
      // positron targets: the mirrored zone, eta' = -eta_e, so d/deta_e = -d/deta'; without
      // NPS the selection folds away
      const bool mir = NPS && u >= U.nN;
      const Zone& ZS = zs[mir ? 1 : 0];
      const int pos = ((mir ? u - U.nN : u) << 6) + lane;
      if (pos < (mir ? ntm : ntn))
        nes_task_bwd<Pr>(P, tb, ZS, A, smem + L.d, smem + (mir ? L.m : L.q), mir, lq,
                        P.task_order[ZS.k * P.ntn + pos], dT, dE);
      if (mir) dE = -dE;
    } else {
      const int pos = ((u - U.nN - U.nM) << 6) + lane;
      if (pos < ntp)
        pair_task_bwd<Pr>(P, tb, Z, A, smem + L.d + n2, smem + L.p, lq, P.task_order[Z.k * P.ntn + pos], dT, dE);
    }
    dT = wave_sum(dT);
    dE = wave_sum(dE);
    if (lane == 0) {
      red[2 * u] = dT;
      red[2 * u + 1] = dE;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sT = 0.0, sE = 0.0;
    for (int u = 0; u < U.nU; ++u) {
      sT += red[2 * u];
      sE += red[2 * u + 1];
    }
    gT_out[Z.z] = sT;
    gE_out[Z.z] = sE;
  }
  // g_f: column contractions of the kernels from LDS, one lane per (part, bin j) for all three
  // species over a part of i (c0 w_j factors out of the sum); the parts are added in order
  const int npb = bin_parts(ne);
  double* s_part = smem + L.d + 2 * n2;   // [part][j][species][g_f0, g_f1]
  for (int r = threadIdx.x; r < npb * ne; r += blockDim.x) {
    const int part = r / ne, j = r - part * ne;
    const int i0 = part * ne / npb, i1 = (part + 1) * ne / npb;
    const double* s_pa = smem + L.p;
    const double* s_d = smem + L.d;
    const double* s_p = s_d + n2;
    double acc[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int i = i0; i < i1; ++i) {
      double ge[3][2], gc[3][2];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        ge[s][0] = A.GE(s, 0, i);
        ge[s][1] = A.GE(s, 1, i);
        gc[s][0] = A.GC(s, 0, i);
        gc[s][1] = A.GC(s, 1, i);
      }
      if (do_nes || do_nps) {
        double v[4];
        scattering_values(smem, L, do_nes, do_nps, 4 * (i >= j ? tri(i, j) : tri(j, i)), v);
        const double q0 = v[0], q1 = v[1], q2 = v[2], q3 = v[3];
        const double dfac = s_d[i * ne + j];
        const double a_in = (i > j) ? dfac : 1.0, a_out = (i < j) ? dfac : 1.0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
          const double k0 = bI * q0 + bII * q2, k1 = bI * q1 + bII * q3;
          acc[s][0] += k0 * ((ge[s][0] + gc[s][0]) * a_in - gc[s][0] * a_out);
          acc[s][1] += k1 * ((ge[s][1] + gc[s][1]) * a_in - gc[s][1] * a_out);
        }
      }
      if (do_pair) {
        const double* aij = s_pa + 2 * (i * ne + j);
        const double* aji = s_pa + 2 * (j * ne + i);
        const double a0 = aij[0], a1 = aij[1], b0 = aji[0], b1 = aji[1];
        const double pf = s_p[i * ne + j];
#pragma unroll
        for (int sg = 0; sg < 3; ++sg) {
          const int s = partner(sg);
          const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
          const double ka0 = bI * a0 + bII * b0, ka1 = bI * a1 + bII * b1;
          acc[sg][0] += ka0 * (gc[s][0] - (ge[s][0] + gc[s][0]) * pf);
          acc[sg][1] += ka1 * (gc[s][1] * (1.0 - pf) - ge[s][1] * pf);
        }
      }
    }
    const double cw = P.c0w[j];
    double* pp = s_part + 6 * r;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      pp[2 * s] = cw * acc[s][0];
      pp[2 * s + 1] = cw * acc[s][1];
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 3 * ne; o += blockDim.x) {
    const int sg = o / ne, j = o % ne;
    double a0 = 0.0, a1 = 0.0;
    for (int part = 0; part < npb; ++part) {
      const double* pp = s_part + 6 * (part * ne + j) + 2 * sg;
      a0 += pp[0];
      a1 += pp[1];
    }
    const int64_t zo = Z.z * 6 * ne;
    gf_out[zo + (2 * sg) * ne + j] = a0;
    gf_out[zo + (2 * sg + 1) * ne + j] = a1;
  }
  if (FUSED) {
    // the task values and f are still in LDS; the contraction parts reuse the g_f parts and
    // the per-lane slots behind them, once every lane has read its g_f parts
    __syncthreads();
    zone_contract<NPS>(P, Z, smem, L, smem + L.d + 2 * n2, eta_out, chi_out);
  }
}

// Occupancy targets (waves per SIMD): three for the Fp32 backward (at most 168
// VGPRs), two for the Fp64 one.
template <typename Pr>
constexpr int bwd_waves() {
  return sizeof(typename Pr::R) == 8 ? 2 : 3;
}

template <typename Pr, bool NPS, bool FUSED>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(bwd_waves<Pr>())))
void rates_backward_kernel(
    DevPlan P, int64_t nz, int selm, const double* __restrict__ Tz, const double* __restrict__ etaz,
    const double* __restrict__ f, const double* __restrict__ g_eta, const double* __restrict__ g_chi,
    double* __restrict__ gT_out, double* __restrict__ gE_out, double* __restrict__ gf_out,
    double* __restrict__ eta_out, double* __restrict__ chi_out) {
  __shared__ double tab[(tab_bytes<Pr>() + 7) / 8];
  __shared__ Zone zs[2];
  __shared__ double red[2 * kMaxUnits];
  extern __shared__ double smem[];
  const int64_t z = pass_zone(P, selm, etaz, nz);
  if (z < 0) return;   // uniform: one zone per workgroup
  const Tabs<Pr> tb = stage_tabs<Pr>(P, tab);
  zone_backward<Pr, NPS, FUSED>(P, tb, zs, red, smem, z, Tz, etaz, f, g_eta, g_chi, gT_out, gE_out, gf_out, eta_out,
                                chi_out);
}

// Per-zone LDS: the layouts above plus the contraction parts (at most 4 x ne x 3 x 4 doubles
// forward, 4 x ne x 3 x 2 backward).
int task_values(const DevPlan& P) {
  return 4 * P.ntn * ((P.processes & VTX_NPS) ? 2 : 1) + 2 * P.ntp;
}
size_t zone_lds_fwd(const DevPlan& P) {
  return sizeof(double) * (6 * P.ne + task_values(P) + 2 * P.ne * P.ne + 48 * P.ne);
}
// The backward adds 13 values per lane of the bulk type (elem bytes) for the pair tasks; the
// fused forward + backward reuses them for the forward's contraction parts (48 ne doubles).
size_t zone_lds_bwd(const DevPlan& P, size_t elem, bool fused) {
  const size_t head = sizeof(double) * (18 * P.ne + task_values(P) + 2 * P.ne * P.ne);
  const size_t bwd = head + sizeof(double) * 24 * P.ne + 13 * (size_t)P.block * elem;
  const size_t fwd = head + sizeof(double) * 48 * P.ne;
  return fused && fwd > bwd ? fwd : bwd;
}

// Dynamic LDS beyond the 64 KiB default must be requested per kernel.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Zones per launch: one workgroup per zone, and a dispatch holds fewer than 2^32 work-items.
// Larger calls are issued as consecutive slices on the same stream.
constexpr int64_t kSliceZones = int64_t(1) << 22;

template <typename Pr, bool NPS>
hipError_t forward_pass(const DevPlan& P, int64_t nz, int selm, const double* T, const double* eta_e,
                        const double* f, double* eta, double* chi, double* jac, int out, hipStream_t s) {
  auto k = out == kOutJac     ? rates_forward_kernel<Pr, kOutJac, NPS>
           : out == kOutTasks ? rates_forward_kernel<Pr, kOutTasks, NPS>
           : out == kOutTable ? rates_forward_kernel<Pr, kOutTable, NPS>
                              : rates_forward_kernel<Pr, kOutRates, NPS>;
  const size_t lds = zone_lds_fwd(P);
  hipError_t e;
  if ((e = allow_lds(k, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)pass_grid(selm, nz)), dim3(P.block), lds, s, P, nz, selm, T, eta_e, f, eta, chi,
                     jac);
  return hipGetLastError();
}

// The mixed path runs two passes over the zones, one per class (see selected()); a pass's
// workgroups find their zones by pass_zone, and those left without one leave at once. The FP64
// path is one pass.
template <bool NPS>
hipError_t forward_slice_t(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                           double* eta, double* chi, double* jac, int out, hipStream_t s) {
  if (P.precision == VTX_MIXED) {
    hipError_t e = forward_pass<Fp32, NPS>(P, nz, kSelBulk, T, eta_e, f, eta, chi, jac, out, s);
    if (e == hipSuccess) e = forward_pass<Fp64, NPS>(P, nz, kSelHigh, T, eta_e, f, eta, chi, jac, out, s);
    return e;
  }
  return forward_pass<Fp64, NPS>(P, nz, kSelAll, T, eta_e, f, eta, chi, jac, out, s);
}

hipError_t forward_slice(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                         double* eta, double* chi, double* jac, int out, hipStream_t s) {
  return (P.processes & VTX_NPS) ? forward_slice_t<true>(P, nz, T, eta_e, f, eta, chi, jac, out, s)
                                 : forward_slice_t<false>(P, nz, T, eta_e, f, eta, chi, jac, out, s);
}

template <bool NPS>
hipError_t interp_slice_t(const DevPlan& P, const vtx_lattice& lat, const double* table, int64_t nz,
                          const double* T, const double* eta_e, const double* f, double* eta, double* chi,
                          hipStream_t s) {
  const size_t lds = zone_lds_fwd(P);
  hipError_t e;
  if ((e = allow_lds(rates_interp_kernel<NPS>, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(rates_interp_kernel<NPS>, dim3((unsigned)nz), dim3(P.block), lds, s, P, lat, table, nz, T,
                     eta_e, f, eta, chi);
  return hipGetLastError();
}

template <typename Pr, bool NPS, bool FUSED>
hipError_t backward_pass(const DevPlan& P, int64_t nz, int selm, const double* T, const double* eta_e,
                         const double* f, const double* g_eta, const double* g_chi, double* g_T, double* g_eta_e,
                         double* g_f, double* eta, double* chi, hipStream_t s) {
  auto k = rates_backward_kernel<Pr, NPS, FUSED>;
  const size_t lds = zone_lds_bwd(P, sizeof(typename Pr::R), FUSED);
  hipError_t e;
  if ((e = allow_lds(k, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)pass_grid(selm, nz)), dim3(P.block), lds, s, P, nz, selm, T, eta_e, f, g_eta,
                     g_chi, g_T, g_eta_e, g_f, eta, chi);
  return hipGetLastError();
}

template <bool NPS, bool FUSED>
hipError_t backward_slice_t(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                            const double* g_eta, const double* g_chi, double* g_T, double* g_eta_e, double* g_f,
                            double* eta, double* chi, hipStream_t s) {
  if (P.precision == VTX_MIXED) {
    hipError_t e = backward_pass<Fp32, NPS, FUSED>(P, nz, kSelBulk, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f,
                                                   eta, chi, s);
    if (e == hipSuccess)
      e = backward_pass<Fp64, NPS, FUSED>(P, nz, kSelHigh, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s);
    return e;
  }
  return backward_pass<Fp64, NPS, FUSED>(P, nz, kSelAll, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s);
}

hipError_t backward_slice(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                          const double* g_eta, const double* g_chi, double* g_T, double* g_eta_e, double* g_f,
                          double* eta, double* chi, hipStream_t s) {
  const bool nps = P.processes & VTX_NPS;
  if (eta)
    return nps ? backward_slice_t<true, true>(P, nz, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s)
               : backward_slice_t<false, true>(P, nz, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s);
  return nps ? backward_slice_t<true, false>(P, nz, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s)
             : backward_slice_t<false, false>(P, nz, T, eta_e, f, g_eta, g_chi, g_T, g_eta_e, g_f, eta, chi, s);
}

}  // namespace

hipError_t launch_forward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                          double* eta, double* chi, hipStream_t s) {
  const int64_t zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = forward_slice(P, n, T + z0, eta_e + z0, f + z0 * zs, eta + z0 * zs, chi + z0 * zs,
                                       nullptr, kOutRates, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_jacobian(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                           double* eta, double* chi, double* jac, hipStream_t s) {
  const int64_t js = 24 * P.ne * P.ne, zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = eta ? forward_slice(P, n, T + z0, eta_e + z0, f + z0 * zs, eta + z0 * zs, chi + z0 * zs,
                                             jac + z0 * js, kOutJac, s)
                             : forward_slice(P, n, T + z0, eta_e + z0, nullptr, nullptr, nullptr, jac + z0 * js,
                                             kOutJac, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int64_t task_values(int ne, unsigned processes) {
  const int64_t ntn = int64_t(ne) * (ne + 1) / 2;
  return ((processes & VTX_NES) ? 4 * ntn : 0) + ((processes & VTX_NPS) ? 4 * ntn : 0) +
         ((processes & VTX_PAIR) ? 2 * int64_t(ne) * ne : 0);
}

hipError_t launch_tasks(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, double* tasks,
                        bool rows, hipStream_t s) {
  const int64_t nv = task_values(P.ne, P.processes);
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = forward_slice(P, n, T + z0, eta_e + z0, nullptr, nullptr, nullptr, tasks + z0 * nv,
                                       rows ? kOutTable : kOutTasks, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_interp(const DevPlan& P, const vtx_lattice& lat, const double* table, int64_t nz, const double* T,
                         const double* eta_e, const double* f, double* eta, double* chi, hipStream_t s) {
  const int64_t zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = (P.processes & VTX_NPS)
                             ? interp_slice_t<true>(P, lat, table, n, T + z0, eta_e + z0, f + z0 * zs, eta + z0 * zs,
                                                    chi + z0 * zs, s)
                             : interp_slice_t<false>(P, lat, table, n, T + z0, eta_e + z0, f + z0 * zs,
                                                     eta + z0 * zs, chi + z0 * zs, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                           const double* g_eta, const double* g_chi, double* g_T, double* g_eta_e, double* g_f,
                           hipStream_t s) {
  const int64_t zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = backward_slice(P, n, T + z0, eta_e + z0, f + z0 * zs, g_eta + z0 * zs, g_chi + z0 * zs,
                                        g_T + z0, g_eta_e + z0, g_f + z0 * zs, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_forward_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                                   const double* f, const double* g_eta, const double* g_chi, double* eta,
                                   double* chi, double* g_T, double* g_eta_e, double* g_f, hipStream_t s) {
  const int64_t zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kSliceZones) {
    const int64_t n = nz - z0 < kSliceZones ? nz - z0 : kSliceZones;
    const hipError_t e = backward_slice(P, n, T + z0, eta_e + z0, f + z0 * zs, g_eta + z0 * zs, g_chi + z0 * zs,
                                        g_T + z0, g_eta_e + z0, g_f + z0 * zs, eta + z0 * zs, chi + z0 * zs, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vtx
