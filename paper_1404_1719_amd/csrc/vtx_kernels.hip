// HIP kernels for gfx950: energy-coupled neutrino-matter interaction rates.
//
// One zone per workgroup (256 lanes = 4 wave64). The zone's work is split into items
// (task, group): a task is one (eps_i, eps_j) kernel integral -- scattering for
// eps_i >= eps_j, pair for every (i, j) -- and a group is one quarter of its quadrature
// rule (a Gauss-Legendre panel or a Gauss-Laguerre tail). The four groups of a task sit in
// four neighbouring lanes and are summed with two lane swaps. Per node a lane evaluates
// the two Fermi-Dirac blocking factors (two exp and one reciprocal) and accumulates the
// moments sum_k W_k B_k var_k^c of the piece variable; the moments are contracted with
// the zone-independent angular-weight coefficients in FP64 at the end of the group. Task
// results live in LDS only: detailed-balance completion, species combination and the
// contraction with f run from LDS, and the only HBM writes are eta/chi (or the gradients).
// The workload is VALU/transcendental bound (no dense contraction: no MFMA).
#include <hip/hip_runtime.h>

#include "../../include/vtx_rates.h"
#include "vtx_internal.h"

namespace vtx {
namespace {

// Pair partner of species s: nu_e <-> anti-nu_e, nu_x <-> nu_x.
__device__ __forceinline__ int partner(int s) { return s == 2 ? 2 : 1 - s; }

// beta_S of species s, selected without indexing the by-value plan (keeps it in SGPRs).
__device__ __forceinline__ double beta_of(const DevPlan& P, int s, int S) {
  const double b0 = S ? P.beta[0][1] : P.beta[0][0];
  const double b1 = S ? P.beta[1][1] : P.beta[1][0];
  const double b2 = S ? P.beta[2][1] : P.beta[2][0];
  return s == 0 ? b0 : (s == 1 ? b1 : b2);
}

template <typename R> struct V4;
template <> struct V4<double> { using T = double4; };
template <> struct V4<float> { using T = float4; };

__device__ __forceinline__ double exp_neg_abs(double z) { return exp(-fabs(z)); }
__device__ __forceinline__ float exp_neg_abs(float z) { return __expf(-fabsf(z)); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// A breakpoint: value and its derivatives along T (eta_e fixed) and along eta_e (T fixed).
struct Tri {
  double v, dT, dE;
};

__device__ __forceinline__ void cswap(Tri& a, Tri& b) {
  if (a.v > b.v) {
    Tri t = a;
    a = b;
    b = t;
  }
}

// value_k = c0 + c1 * (rev ? 1 - tau_k : tau_k)
struct Aff {
  double c0, c1;
  bool rev;
};

// Anchor an affine function of the node at the end of the group where it is smaller in
// magnitude, so that FP32 evaluation never subtracts two large numbers. Breakpoints sit on
// the zeros of the Fermi-Dirac arguments, so inside a group each argument keeps its sign.
__device__ __forceinline__ Aff anchor(double zA, double zB, bool lag, double slope_lag) {
  if (lag) return {zA, slope_lag, false};
  if (fabs(zA) <= fabs(zB)) return {zA, zB - zA, false};
  return {zB, zA - zB, true};
}

struct Group {
  bool lag;        // Laguerre table
  int toff;        // offset into the Laguerre table
  double Es;       // E = E0 + Es * tau; weight W = Es * w_table
  Aff var, z1, z2; // piece variable and the two Fermi-Dirac arguments
  double split;    // nodes with var < split go to the low piece
  Tri E0;          // group start (and its derivatives)
  double dEsT, dEsE;
  double s1, s2;   // d z / d eta_e
  double dvar;     // d var / dE
  int piece;       // pair: 0, 1, 2
};

// Scattering task eps_i >= eps_j, group g in 0..3.
//   z1 = (mu - E)/T  [F(E) = sigma(z1)],  z2 = (E + Delta - mu)/T  [1 - F(E + Delta) = sigma(z2)].
__device__ void nes_group(const DevPlan& P, double e, double ep, int g, double T, double eta, Group& G) {
  const double mu = eta * T, delta = e - ep;
  if (P.rule == VTX_RULE_LAGUERRE) {
    G.lag = true;
    G.toff = g * P.m4;
    G.E0 = {0.0, 0.0, 0.0};
    G.Es = T;
    G.dEsT = 1.0;
    G.dEsE = 0.0;
  } else {
    Tri b0 = {0.0, 0.0, 0.0};
    Tri bm = (mu - delta > 0.0) ? Tri{mu - delta, eta, T} : Tri{0.0, 0.0, 0.0};
    Tri bu = (mu > 0.0) ? Tri{mu, eta, T} : Tri{0.0, 0.0, 0.0};
    const double cap = bu.v + kKappa * T;
    Tri bp = (ep <= cap) ? Tri{ep, 0.0, 0.0} : Tri{cap, bu.dT + kKappa, bu.dE};
    cswap(b0, bm);
    cswap(bu, bp);
    cswap(b0, bu);
    cswap(bm, bp);
    cswap(bm, bu);
    // sorted breakpoints b0 <= bm <= bu <= bp; group g spans [b_g, b_{g+1}] (g = 3: tail)
    const Tri lo = (g == 0) ? b0 : (g == 1) ? bm : (g == 2) ? bu : bp;
    const Tri hi = (g == 0) ? bm : (g == 1) ? bu : bp;
    G.lag = (g == 3);
    G.toff = 0;
    G.E0 = lo;
    if (g < 3) {
      G.Es = hi.v - lo.v;
      G.dEsT = hi.dT - lo.dT;
      G.dEsE = hi.dE - lo.dE;
    } else {
      G.Es = T;
      G.dEsT = 1.0;
      G.dEsE = 0.0;
    }
  }
  const double Ea = G.E0.v, Eb = G.E0.v + G.Es;
  G.var = anchor(Ea / ep, Eb / ep, G.lag, T / ep);
  G.z1 = anchor((mu - Ea) / T, (mu - Eb) / T, G.lag, -1.0);
  G.z2 = anchor((Ea + delta - mu) / T, (Eb + delta - mu) / T, G.lag, 1.0);
  G.split = 1.0;
  G.s1 = 1.0;
  G.s2 = -1.0;
  G.dvar = 1.0 / ep;
  G.piece = 0;
}

// Pair task (e, ep), group g in 0..3: Gauss-Legendre panels between sorted {0, m, M, c, w}.
//   z1 = (E - mu)/T  [1 - F(E)],  z2 = (w - E + mu)/T  [1 - Fbar(w - E)].
__device__ void pair_group(double e, double ep, int g, double T, double eta, Group& G) {
  const double mu = eta * T, w = e + ep;
  const double mn = fmin(e, ep), mx = fmax(e, ep);
  Tri c = (mu > 0.0) ? (mu <= w ? Tri{mu, eta, T} : Tri{w, 0.0, 0.0}) : Tri{0.0, 0.0, 0.0};
  // sorted {0, m, M, c, w}: c goes after every one of {0, m, M} not above it (stable order)
  const int pos = 1 + (mn <= c.v ? 1 : 0) + (mx <= c.v ? 1 : 0);
  const Tri t0 = {0.0, 0.0, 0.0}, tm = {mn, 0.0, 0.0}, tM = {mx, 0.0, 0.0}, tw = {w, 0.0, 0.0};
  // element q of the sorted list: base element q for q < pos, c at pos, base element q-1 after
  auto elem = [&](int q) -> Tri {
    if (q == pos) return c;
    const int k = (q < pos) ? q : q - 1;
    return (k == 0) ? t0 : (k == 1) ? tm : (k == 2) ? tM : tw;
  };
  const Tri blo = elem(g), bhi = elem(g + 1);
  G.lag = false;
  G.toff = 0;
  G.E0 = blo;
  G.Es = bhi.v - blo.v;
  G.dEsT = bhi.dT - blo.dT;
  G.dEsE = bhi.dE - blo.dE;
  const double Ea = G.E0.v, Eb = Ea + G.Es;
  const double mid = Ea + 0.5 * G.Es;
  G.piece = (mid <= mn) ? 0 : ((mid <= mx) ? 1 : 2);
  if (G.piece == 0) {
    G.var = anchor(Ea / mn, Eb / mn, false, 0.0);
    G.dvar = 1.0 / mn;
  } else if (G.piece == 1) {
    G.var = anchor(Ea / mx, Eb / mx, false, 0.0);
    G.dvar = 1.0 / mx;
  } else {
    G.var = anchor((w - Ea) / mn, (w - Eb) / mn, false, 0.0);
    G.dvar = -1.0 / mn;
  }
  G.z1 = anchor((Ea - mu) / T, (Eb - mu) / T, false, 0.0);
  G.z2 = anchor((w - Ea + mu) / T, (w - Eb + mu) / T, false, 0.0);
  G.split = 1e30;
  G.s1 = -1.0;
  G.s2 = 1.0;
}

// LDS-staged node tables of one block.
struct Tables {
  double4 leg64[kMaxNquad / 4];
  double4 lag64[kMaxNquad];
  float4 leg32[kMaxNquad / 4];
  float4 lag32[kMaxNquad];
};

__device__ void stage_tables(const DevPlan& P, Tables& tb) {
  for (int k = threadIdx.x; k < P.m4; k += blockDim.x) {
    tb.leg64[k] = P.leg64[k];
    tb.leg32[k] = P.leg32[k];
  }
  for (int k = threadIdx.x; k < P.nlag; k += blockDim.x) {
    tb.lag64[k] = P.lag64[k];
    tb.lag32[k] = P.lag32[k];
  }
}

template <typename R> __device__ __forceinline__ const typename V4<R>::T* leg_tab(const Tables& tb);
template <> __device__ __forceinline__ const double4* leg_tab<double>(const Tables& tb) { return tb.leg64; }
template <> __device__ __forceinline__ const float4* leg_tab<float>(const Tables& tb) { return tb.leg32; }
template <typename R> __device__ __forceinline__ const typename V4<R>::T* lag_tab(const Tables& tb);
template <> __device__ __forceinline__ const double4* lag_tab<double>(const Tables& tb) { return tb.lag64; }
template <> __device__ __forceinline__ const float4* lag_tab<float>(const Tables& tb) { return tb.lag32; }

// Blocking factor sigma(z1) sigma(z2) from e_k = exp(-|z_k|).
template <typename RF>
__device__ __forceinline__ RF blocking(RF z1, RF z2, RF e1, RF e2) {
  const RF num = (z1 >= RF(0) ? RF(1) : e1) * (z2 >= RF(0) ? RF(1) : e2);
  return num * recip((RF(1) + e1) * (RF(1) + e2));
}

// Degree-7 Bernstein basis without binomials: b[k] = u^k (1 - u)^(7 - k).
template <typename R>
__device__ __forceinline__ void bernstein7(R u, R b[8]) {
  const R v = R(1) - u;
  const R u2 = u * u, u3 = u2 * u, u4 = u2 * u2, u5 = u4 * u, u6 = u3 * u3;
  const R v2 = v * v, v3 = v2 * v, v4 = v2 * v2, v5 = v4 * v, v6 = v3 * v3;
  b[0] = v6 * v;
  b[1] = u * v6;
  b[2] = u2 * v5;
  b[3] = u3 * v4;
  b[4] = u4 * v3;
  b[5] = u5 * v2;
  b[6] = u6 * v;
  b[7] = u6 * u;
}

// Forward node loop of one group: moments M[c] = sum W B u^c (1-u)^(7-c) of the low piece
// (nonnegative basis: positive sums, no cancellation in FP32) and Hm[c] = sum W B u^c of
// the high piece (c = 0..2). R: bulk precision; RF: Fermi-Dirac precision.
template <typename R, typename RF>
__device__ __forceinline__ void node_moments(const Group& G, int m4, const Tables& tb, R M[8], R Hm[3]) {
  const auto* tR = G.lag ? lag_tab<R>(tb) + G.toff : leg_tab<R>(tb);
  const auto* tF = G.lag ? lag_tab<RF>(tb) + G.toff : leg_tab<RF>(tb);
  const R v0 = R(G.var.c0), v1 = R(G.var.c1);
  const RF a0 = RF(G.z1.c0), a1 = RF(G.z1.c1), b0 = RF(G.z2.c0), b1 = RF(G.z2.c1);
  const R ws = R(G.Es), split = R(G.split);
  const bool vr = G.var.rev, ar = G.z1.rev, br = G.z2.rev;
#pragma unroll 4
  for (int k = 0; k < m4; ++k) {
    const auto nR = tR[k];
    const auto nF = tF[k];
    const R var = v0 + v1 * (vr ? nR.y : nR.x);
    const RF z1 = a0 + a1 * (ar ? nF.y : nF.x);
    const RF z2 = b0 + b1 * (br ? nF.y : nF.x);
    const RF B = blocking<RF>(z1, z2, exp_neg_abs(z1), exp_neg_abs(z2));
    const R wb = ws * nR.z * R(B);
    // select, never subtract: wb - wl would be contracted into fma(ws w, B, -wl), which
    // leaves the product's rounding residue in the other piece instead of zero
    const bool lo = var < split;
    const R wl = lo ? wb : R(0);
    const R wh = lo ? R(0) : wb;
    R b[8];
    bernstein7<R>(var, b);
#pragma unroll
    for (int c = 0; c < 8; ++c) M[c] += wl * b[c];
    Hm[0] += wh;
    Hm[1] += wh * var;
    Hm[2] += wh * (var * var);
  }
}

struct Q4 {
  double x, y, z, w;
};

// Task results (4 comps for scattering, 2 for pair) from the moments, in FP64.
template <typename R>
__device__ __forceinline__ Q4 contract_moments(const DevPlan& P, bool nes, int task, const Group& G,
                                               const R M[8], const R Hm[3]) {
  double m[8], h[3];
#pragma unroll
  for (int c = 0; c < 8; ++c) m[c] = double(M[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c) h[c] = double(Hm[c]);
  Q4 out = {0.0, 0.0, 0.0, 0.0};
  if (nes) {
    const NesCoef& C = P.nes_coef[task];
    double s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double a = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) a = fma(C.lo[q][c], m[c], a);
#pragma unroll
      for (int c = 0; c < 3; ++c) a = fma(C.hi[q][c], h[c], a);
      s[q] = a;
    }
    out = {s[0], s[1], s[2], s[3]};
  } else {
    const double* c0 = P.pair_coef[task].piece[G.piece][0];
    const double* c1 = P.pair_coef[task].piece[G.piece][1];
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      a = fma(c0[c], m[c], a);
      b = fma(c1[c], m[c], b);
    }
    out.x = a;
    out.y = b;
  }
  return out;
}

__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Detailed-balance factors exp(-|eps_i - eps_j|/T) and exp(-(eps_i + eps_j)/T), FP64.
__device__ void stage_factors(const DevPlan& P, double T, double* s_d, double* s_p) {
  const int ne = P.ne;
  for (int k = threadIdx.x; k < ne * ne; k += blockDim.x) {
    const int i = k / ne, j = k % ne;
    const double ei = P.eps[i], ej = P.eps[j];
    s_d[k] = exp(-fabs(ei - ej) / T);
    s_p[k] = exp(-(ei + ej) / T);
  }
}

// Item loop shared by forward and backward value passes: tasks' kernel integrals into LDS.
template <typename R, typename RF>
__device__ void items_forward(const DevPlan& P, const Tables& tb, double T, double eta, int ntn_used,
                              int ntp_used, double* s_qn, double* s_pa) {
  const int nitems = 4 * (ntn_used + ntp_used);
  for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
    const int task_any = it >> 2, g = it & 3;
    const bool nes = task_any < ntn_used;
    const int task = nes ? task_any : task_any - ntn_used;
    Group G;
    int i, j;
    if (nes) {
      const int ij = P.nes_ij[task];
      i = ij & 0xff;
      j = ij >> 8;
      nes_group(P, P.eps[i], P.eps[j], g, T, eta, G);
    } else {
      i = task / P.ne;
      j = task % P.ne;
      pair_group(P.eps[i], P.eps[j], g, T, eta, G);
    }
    R M[8] = {0, 0, 0, 0, 0, 0, 0, 0}, Hm[3] = {0, 0, 0};
    node_moments<R, RF>(G, P.m4, tb, M, Hm);
    Q4 o = contract_moments<R>(P, nes, task, G, M, Hm);
    o.x = quad_sum(o.x);
    o.y = quad_sum(o.y);
    o.z = quad_sum(o.z);
    o.w = quad_sum(o.w);
    if (g == 0) {
      if (nes) {
        double* q = s_qn + 4 * task;
        q[0] = o.x;
        q[1] = o.y;
        q[2] = o.z;
        q[3] = o.w;
      } else {
        s_pa[2 * task] = o.x;
        s_pa[2 * task + 1] = o.y;
      }
    }
  }
}

template <typename R>
__device__ void items_forward_dispatch(const DevPlan& P, const Tables& tb, double T, double eta, int ntn_used,
                                       int ntp_used, double* s_qn, double* s_pa) {
  if (sizeof(R) == sizeof(float) && eta > P.eta_fp64)
    items_forward<float, double>(P, tb, T, eta, ntn_used, ntp_used, s_qn, s_pa);
  else
    items_forward<R, R>(P, tb, T, eta, ntn_used, ntp_used, s_qn, s_pa);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void rates_forward_kernel(DevPlan P, const double* __restrict__ Tz,
                                                               const double* __restrict__ etaz,
                                                               const double* __restrict__ f,
                                                               double* __restrict__ eta_out,
                                                               double* __restrict__ chi_out) {
  __shared__ Tables tb;
  extern __shared__ double smem[];
  const int ne = P.ne;
  const int64_t z = blockIdx.x;
  const bool do_nes = P.processes & VTX_NES, do_pair = P.processes & VTX_PAIR;
  double* s_f = smem;                 // [6 ne]
  double* s_qn = s_f + 6 * ne;        // [4 ntn]
  double* s_pa = s_qn + 4 * P.ntn;    // [2 ntp]
  double* s_d = s_pa + 2 * P.ntp;     // [ne ne]
  double* s_p = s_d + ne * ne;        // [ne ne]
  const double T = Tz[z], eta = etaz[z];
  const double* fz = f + z * 6 * ne;
  for (int k = threadIdx.x; k < 6 * ne; k += blockDim.x) s_f[k] = fz[k];
  stage_tables(P, tb);
  stage_factors(P, T, s_d, s_p);
  __syncthreads();
  items_forward_dispatch<R>(P, tb, T, eta, do_nes ? P.ntn : 0, do_pair ? P.ntp : 0, s_qn, s_pa);
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < 3 * ne) {
    const int s = tid / ne, i = tid % ne, sb = partner(s);
    const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
    double e0 = 0.0, c0 = 0.0, e1 = 0.0, c1 = 0.0;
    for (int j = 0; j < ne; ++j) {
      const double cw = P.c0w[j];
      const double dfac = s_d[i * ne + j];
      if (do_nes) {
        const double* q = s_qn + 4 * (i >= j ? tri(i, j) : tri(j, i));
        const double k0 = bI * q[0] + bII * q[2];
        const double k1 = bI * q[1] + bII * q[3];
        const double a_in = (i > j) ? dfac : 1.0, a_out = (i < j) ? dfac : 1.0;
        const double f0 = s_f[(2 * s) * ne + j], f1 = s_f[(2 * s + 1) * ne + j];
        const double in0 = (cw * f0 * k0) * a_in, in1 = (cw * f1 * k1) * a_in;
        e0 += in0;
        c0 += in0 + (cw * (1.0 - f0) * k0) * a_out;
        e1 += in1;
        c1 += in1 - (cw * f1 * k1) * a_out;
      }
      if (do_pair) {
        const double* aij = s_pa + 2 * (i * ne + j);
        const double* aji = s_pa + 2 * (j * ne + i);
        const double ka0 = bI * aij[0] + bII * aji[0];
        const double ka1 = bI * aij[1] + bII * aji[1];
        const double pf = s_p[i * ne + j];
        const double g0 = s_f[(2 * sb) * ne + j], g1 = s_f[(2 * sb + 1) * ne + j];
        const double pr0 = (cw * (1.0 - g0) * ka0) * pf;
        const double t1 = cw * g1 * ka1;
        e0 += pr0;
        c0 += pr0 + cw * g0 * ka0;
        e1 -= t1 * pf;
        c1 += t1 - t1 * pf;
      }
    }
    const int64_t o = z * 6 * ne + (2 * s) * ne + i;
    eta_out[o] = e0;
    chi_out[o] = c0;
    eta_out[o + ne] = e1;
    chi_out[o + ne] = c1;
  }
}

// ---------------------------------------------------------------------------------------
// Backward (vector-Jacobian product). Recomputes every task's kernel values and, in the
// same node loop, the derivative of the adjoint-weighted kernel sum_c A_c q_c along T and
// eta_e (node motion included). A_c are the upstream weights of each task component.

struct Adj {
  const double* f;
  const double* ge;
  const double* gc;
  int ne;
  __device__ double F(int s, int m, int i) const { return f[(2 * s + m) * ne + i]; }
  __device__ double GE(int s, int m, int i) const { return ge[(2 * s + m) * ne + i]; }
  __device__ double GC(int s, int m, int i) const { return gc[(2 * s + m) * ne + i]; }
};

// Scattering: weight of Phi_out_{l,S}(a, b) plus that of Phi_in_{l,S}(b, a) in L.
__device__ double nes_ghat(const DevPlan& P, const Adj& A, int S, int l, int a, int b) {
  double go = 0.0, gi = 0.0;
  for (int s = 0; s < 3; ++s) {
    const double bs = beta_of(P, s, S);
    if (l == 0) {
      go += bs * A.GC(s, 0, a) * (1.0 - A.F(s, 0, b));
      gi += bs * (A.GE(s, 0, b) + A.GC(s, 0, b)) * A.F(s, 0, a);
    } else {
      go -= bs * A.GC(s, 1, a) * A.F(s, 1, b);
      gi += bs * (A.GE(s, 1, b) + A.GC(s, 1, b)) * A.F(s, 1, a);
    }
  }
  return P.c0w[b] * go + P.c0w[a] * gi;
}

// Pair: weight of Phi_a_{l,S}(a, b) in L (pf = p_ab), or only its p-coefficient.
__device__ double pair_gw(const DevPlan& P, const Adj& A, int S, int l, int a, int b, double pf, bool ponly) {
  double acc = 0.0;
  for (int s = 0; s < 3; ++s) {
    const double bs = beta_of(P, s, S);
    const int sb = partner(s);
    if (l == 0) {
      const double ge = A.GE(s, 0, a) + A.GC(s, 0, a);
      const double f0 = A.F(sb, 0, b);
      acc += ponly ? bs * ge * (1.0 - f0) : bs * (ge * (1.0 - f0) * pf + A.GC(s, 0, a) * f0);
    } else {
      const double f1 = A.F(sb, 1, b);
      acc += ponly ? -bs * f1 * (A.GE(s, 1, a) + A.GC(s, 1, a))
                   : bs * f1 * (-A.GE(s, 1, a) * pf + A.GC(s, 1, a) * (1.0 - pf));
    }
  }
  return P.c0w[b] * acc;
}

template <typename R, typename RF>
__device__ __forceinline__ void node_loop_bwd(const Group& G, int m4, const Tables& tb, double T, double eta,
                                              const R hl[8], const R hh[3], const R dl[8], const R dh[2],
                                              R M[8], R Hm[3], R& accT, R& accE) {
  const auto* tR = G.lag ? lag_tab<R>(tb) + G.toff : leg_tab<R>(tb);
  const auto* tF = G.lag ? lag_tab<RF>(tb) + G.toff : leg_tab<RF>(tb);
  const R v0 = R(G.var.c0), v1 = R(G.var.c1);
  const RF a0 = RF(G.z1.c0), a1 = RF(G.z1.c1), b0 = RF(G.z2.c0), b1 = RF(G.z2.c1);
  const R ws = R(G.Es), split = R(G.split);
  const bool vr = G.var.rev, ar = G.z1.rev, br = G.z2.rev;
  const R s1 = R(G.s1), s2 = R(G.s2);
  const R invT = R(1.0 / T), etaR = R(eta);
  const R dE0T = R(G.E0.dT), dEsT = R(G.dEsT), dE0E = R(G.E0.dE), dEsE = R(G.dEsE);
#pragma unroll 2
  for (int k = 0; k < m4; ++k) {
    const auto nR = tR[k];
    const auto nF = tF[k];
    const R var = v0 + v1 * (vr ? nR.y : nR.x);
    const RF z1 = a0 + a1 * (ar ? nF.y : nF.x);
    const RF z2 = b0 + b1 * (br ? nF.y : nF.x);
    const RF e1 = exp_neg_abs(z1), e2 = exp_neg_abs(z2);
    const RF i1 = recip(RF(1) + e1), i2 = recip(RF(1) + e2);
    const RF sg1 = (z1 >= RF(0) ? RF(1) : e1) * i1, sg2 = (z2 >= RF(0) ? RF(1) : e2) * i2;
    const RF r1 = (z1 >= RF(0) ? e1 : RF(1)) * i1, r2 = (z2 >= RF(0) ? e2 : RF(1)) * i2;
    const R B = R(sg1 * sg2);
    const R wt = nR.z;
    const R wb = ws * wt * B;
    // value moments
    const bool lo = var < split;
    const R wl = lo ? wb : R(0);
    const R wh = lo ? R(0) : wb;   // select, never subtract (see node_moments)
    R b[8];
    bernstein7<R>(var, b);
    R Hlo = R(0), Dlo = R(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      M[c] += wl * b[c];
      Hlo += hl[c] * b[c];
      Dlo += dl[c] * b[c];
    }
    Hm[0] += wh;
    Hm[1] += wh * var;
    Hm[2] += wh * (var * var);
    // derivatives of log B at fixed E, and along E
    const R rr1 = R(r1), rr2 = R(r2);
    const R dlE = s1 * rr1 + s2 * rr2;                                    // d/deta
    const R dlT = -(rr1 * R(z1) + rr2 * R(z2) - etaR * dlE) * invT;       // d/dT
    const R dlX = -dlE * invT;                                            // d/dE
    // node motion
    const R tau = nR.x;
    const R dET = dE0T + dEsT * tau, dEE = dE0E + dEsE * tau;
    // adjoint-weighted angular weight and its E-derivative (low piece: Bernstein above)
    const R Hhi = (hh[2] * var + hh[1]) * var + hh[0];
    const R Dhi = dh[1] * var + dh[0];
    const R H = lo ? Hlo : Hhi;
    const R D = lo ? Dlo : Dhi;
    const R wtB = wt * B;
    const R aT = dEsT * wtB + wb * (dlT + dlX * dET);
    const R aE = dEsE * wtB + wb * (dlE + dlX * dEE);
    accT += aT * H + wb * dET * D;
    accE += aE * H + wb * dEE * D;
  }
}

template <typename R, typename RF>
__device__ void items_backward(const DevPlan& P, const Tables& tb, double T, double eta, int ntn_used,
                               int ntp_used, const double* s_adj, const double* s_uadj, double* s_qn,
                               double* s_pa, double& gT, double& gE) {
  const int nitems = 4 * (ntn_used + ntp_used);
  for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
    const int task_any = it >> 2, g = it & 3;
    const bool nes = task_any < ntn_used;
    const int task = nes ? task_any : task_any - ntn_used;
    Group G;
    int i, j;
    double hl64[8], hh64[3];
    if (nes) {
      const int ij = P.nes_ij[task];
      i = ij & 0xff;
      j = ij >> 8;
      nes_group(P, P.eps[i], P.eps[j], g, T, eta, G);
      const NesCoef& C = P.nes_coef[task];
      const double* a = s_adj + 4 * task;
      for (int c = 0; c < 8; ++c) hl64[c] = a[0] * C.lo[0][c] + a[1] * C.lo[1][c] + a[2] * C.lo[2][c] + a[3] * C.lo[3][c];
      for (int c = 0; c < 3; ++c) hh64[c] = a[0] * C.hi[0][c] + a[1] * C.hi[1][c] + a[2] * C.hi[2][c] + a[3] * C.hi[3][c];
    } else {
      i = task / P.ne;
      j = task % P.ne;
      pair_group(P.eps[i], P.eps[j], g, T, eta, G);
      const PairCoef& C = P.pair_coef[task];
      const double* a = s_adj + 4 * P.ntn + 2 * task;
      for (int c = 0; c < 8; ++c) hl64[c] = a[0] * C.piece[G.piece][0][c] + a[1] * C.piece[G.piece][1][c];
      for (int c = 0; c < 3; ++c) hh64[c] = 0.0;
    }
    // d/dE of the low piece, in the same folded degree-7 Bernstein basis: with beta_k =
    // g_k / C(7,k), dH/du has degree-6 coefficients d_k = 7 (beta_{k+1} - beta_k); degree
    // elevation gives D_k = (k/7) d_{k-1} + (1 - k/7) d_k; fold C(7,k) back and scale by du/dE.
    constexpr double kBin7[8] = {1.0, 7.0, 21.0, 35.0, 35.0, 21.0, 7.0, 1.0};
    double d6[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) d6[c] = 7.0 * (hl64[c + 1] / kBin7[c + 1] - hl64[c] / kBin7[c]);
    R hl[8], hh[3], dl[8], dh[2];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double lower = (c > 0) ? (c / 7.0) * d6[c - 1] : 0.0;
      const double upper = (c < 7) ? (1.0 - c / 7.0) * d6[c] : 0.0;
      hl[c] = R(hl64[c]);
      dl[c] = R((lower + upper) * kBin7[c] * G.dvar);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) hh[c] = R(hh64[c]);
#pragma unroll
    for (int c = 0; c < 2; ++c) dh[c] = R(hh64[c + 1] * (c + 1) * G.dvar);
    R M[8] = {0, 0, 0, 0, 0, 0, 0, 0}, Hm[3] = {0, 0, 0};
    R accT = 0, accE = 0;
    node_loop_bwd<R, RF>(G, P.m4, tb, T, eta, hl, hh, dl, dh, M, Hm, accT, accE);
    gT += double(accT);
    gE += double(accE);
    Q4 o = contract_moments<R>(P, nes, task, G, M, Hm);
    o.x = quad_sum(o.x);
    o.y = quad_sum(o.y);
    o.z = quad_sum(o.z);
    o.w = quad_sum(o.w);
    if (g == 0) {
      if (nes) {
        const double* u = s_uadj + 4 * task;
        const double de = (P.eps[i] - P.eps[j]) / (T * T);
        gT += (o.x * u[0] + o.y * u[1] + o.z * u[2] + o.w * u[3]) * de;
        double* q = s_qn + 4 * task;   // same slot: read above, overwritten now
        q[0] = o.x;
        q[1] = o.y;
        q[2] = o.z;
        q[3] = o.w;
      } else {
        const double* u = s_uadj + 4 * P.ntn + 2 * task;
        const double u0 = u[0], u1 = u[1];
        s_pa[2 * task] = o.x;
        s_pa[2 * task + 1] = o.y;
        gT += o.x * u0 + o.y * u1;
      }
    }
  }
}

__device__ double block_sum(double v, double* scratch) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += scratch[k];
  return t;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void rates_backward_kernel(
    DevPlan P, const double* __restrict__ Tz, const double* __restrict__ etaz, const double* __restrict__ f,
    const double* __restrict__ g_eta, const double* __restrict__ g_chi, double* __restrict__ gT_out,
    double* __restrict__ gE_out, double* __restrict__ gf_out) {
  __shared__ Tables tb;
  __shared__ double red[8];
  extern __shared__ double smem[];
  const int ne = P.ne;
  const int64_t z = blockIdx.x;
  const bool do_nes = P.processes & VTX_NES, do_pair = P.processes & VTX_PAIR;
  const int ntn = do_nes ? P.ntn : 0, ntp = do_pair ? P.ntp : 0;
  // Task slots: [4 ntn] scattering comps, then [2 ntp] pair comps (full-size offsets
  // whatever the process mask). s_uadj holds each task's completion-factor weight until the
  // lane that owns the task has read it; the same lane then stores the task's kernel values
  // in that slot (s_qn / s_pa alias s_uadj).
  double* s_f = smem;
  double* s_ge = s_f + 6 * ne;
  double* s_gc = s_ge + 6 * ne;
  double* s_adj = s_gc + 6 * ne;                    // adjoint weights of task comps
  double* s_uadj = s_adj + 4 * P.ntn + 2 * P.ntp;   // completion-factor T-derivative weights
  double* s_qn = s_uadj;
  double* s_pa = s_uadj + 4 * P.ntn;
  double* s_d = s_uadj + 4 * P.ntn + 2 * P.ntp;
  double* s_p = s_d + ne * ne;
  const double T = Tz[z], eta = etaz[z];
  const int64_t zo = z * 6 * ne;
  for (int k = threadIdx.x; k < 6 * ne; k += blockDim.x) {
    s_f[k] = f[zo + k];
    s_ge[k] = g_eta[zo + k];
    s_gc[k] = g_chi[zo + k];
  }
  stage_tables(P, tb);
  stage_factors(P, T, s_d, s_p);
  __syncthreads();
  const Adj A{s_f, s_ge, s_gc, ne};
  // adjoint weights per task component
  for (int t = threadIdx.x; t < ntn + ntp; t += blockDim.x) {
    if (t < ntn) {
      const int ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
      const double d = s_d[i * ne + j];
      for (int c = 0; c < 4; ++c) {
        const int S = c >> 1, l = c & 1;
        const double up = (i > j) ? d * nes_ghat(P, A, S, l, j, i) : 0.0;
        s_adj[4 * t + c] = nes_ghat(P, A, S, l, i, j) + up;
        s_uadj[4 * t + c] = up;
      }
    } else {
      const int p = t - ntn, i = p / ne, j = p % ne;
      const double pf = s_p[i * ne + j];
      const double dpf = pf * (P.eps[i] + P.eps[j]) / (T * T);
      for (int l = 0; l < 2; ++l) {
        s_adj[4 * P.ntn + 2 * p + l] = pair_gw(P, A, 0, l, i, j, pf, false) + pair_gw(P, A, 1, l, j, i, pf, false);
        s_uadj[4 * P.ntn + 2 * p + l] = (pair_gw(P, A, 0, l, i, j, pf, true) + pair_gw(P, A, 1, l, j, i, pf, true)) * dpf;
      }
    }
  }
  __syncthreads();
  double gT = 0.0, gE = 0.0;
  if (sizeof(R) == sizeof(float) && eta > P.eta_fp64)
    items_backward<float, double>(P, tb, T, eta, ntn, ntp, s_adj, s_uadj, s_qn, s_pa, gT, gE);
  else
    items_backward<R, R>(P, tb, T, eta, ntn, ntp, s_adj, s_uadj, s_qn, s_pa, gT, gE);
  const double sT = block_sum(gT, red);
  const double sE = block_sum(gE, red + 4);
  if (threadIdx.x == 0) {
    gT_out[z] = sT;
    gE_out[z] = sE;
  }
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < 3 * ne) {
    const int sg = tid / ne, j = tid % ne;
    const double cw = P.c0w[j];
    double a0 = 0.0, a1 = 0.0;
    if (do_nes) {
      const double bI = beta_of(P, sg, 0), bII = beta_of(P, sg, 1);
      for (int i = 0; i < ne; ++i) {
        const double* q = s_qn + 4 * (i >= j ? tri(i, j) : tri(j, i));
        const double k0 = bI * q[0] + bII * q[2], k1 = bI * q[1] + bII * q[3];
        const double dfac = s_d[i * ne + j];
        const double a_in = (i > j) ? dfac : 1.0, a_out = (i < j) ? dfac : 1.0;
        const double ge0 = cw * A.GE(sg, 0, i), gc0 = cw * A.GC(sg, 0, i);
        const double ge1 = cw * A.GE(sg, 1, i), gc1 = cw * A.GC(sg, 1, i);
        a0 += ((ge0 + gc0) * k0) * a_in - (gc0 * k0) * a_out;
        a1 += ((ge1 + gc1) * k1) * a_in - (gc1 * k1) * a_out;
      }
    }
    if (do_pair) {
      const int s = partner(sg);
      const double bI = beta_of(P, s, 0), bII = beta_of(P, s, 1);
      for (int i = 0; i < ne; ++i) {
        const double* aij = s_pa + 2 * (i * ne + j);
        const double* aji = s_pa + 2 * (j * ne + i);
        const double ka0 = bI * aij[0] + bII * aji[0];
        const double ka1 = bI * aij[1] + bII * aji[1];
        const double pf = s_p[i * ne + j];
        const double ge0 = cw * A.GE(s, 0, i), gc0 = cw * A.GC(s, 0, i);
        const double ge1 = cw * A.GE(s, 1, i), gc1 = cw * A.GC(s, 1, i);
        a0 += -((ge0 + gc0) * ka0) * pf + gc0 * ka0;
        a1 += -(ge1 * ka1) * pf + gc1 * ka1 - (gc1 * ka1) * pf;
      }
    }
    gf_out[zo + (2 * sg) * ne + j] = a0;
    gf_out[zo + (2 * sg + 1) * ne + j] = a1;
  }
}

size_t fwd_smem(const DevPlan& P) {
  return sizeof(double) * (6 * P.ne + 4 * P.ntn + 2 * P.ntp + 2 * P.ne * P.ne);
}
size_t bwd_smem(const DevPlan& P) {
  return sizeof(double) * (18 * P.ne + 2 * (4 * P.ntn + 2 * P.ntp) + 2 * P.ne * P.ne);
}

// Dynamic LDS beyond the 64 KiB default must be requested per kernel.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace

hipError_t launch_forward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                          double* eta, double* chi, hipStream_t s) {
  if (nz <= 0) return hipSuccess;
  const dim3 grid((unsigned)nz), block(kBlock);
  const size_t lds = fwd_smem(P);
  hipError_t e;
  if (P.precision == VTX_MIXED) {
    if ((e = allow_lds(rates_forward_kernel<float>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(rates_forward_kernel<float>, grid, block, lds, s, P, T, eta_e, f, eta, chi);
  } else {
    if ((e = allow_lds(rates_forward_kernel<double>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(rates_forward_kernel<double>, grid, block, lds, s, P, T, eta_e, f, eta, chi);
  }
  return hipGetLastError();
}

hipError_t launch_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                           const double* g_eta, const double* g_chi, double* g_T, double* g_eta_e, double* g_f,
                           hipStream_t s) {
  if (nz <= 0) return hipSuccess;
  const dim3 grid((unsigned)nz), block(kBlock);
  const size_t lds = bwd_smem(P);
  hipError_t e;
  if (P.precision == VTX_MIXED) {
    if ((e = allow_lds(rates_backward_kernel<float>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(rates_backward_kernel<float>, grid, block, lds, s, P, T, eta_e, f, g_eta, g_chi, g_T,
                       g_eta_e, g_f);
  } else {
    if ((e = allow_lds(rates_backward_kernel<double>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(rates_backward_kernel<double>, grid, block, lds, s, P, T, eta_e, f, g_eta, g_chi, g_T,
                       g_eta_e, g_f);
  }
  return hipGetLastError();
}

}  // namespace vtx
