// Interaction rates with the electron mass (FP64): the accuracy variant of the forward pass
// for low temperatures and neutrino energies, where m_e is not small against the electron
// energies (the rates of Sect. 2.1's list of model components, with massive e+-).
//
// What changes against the massless kernels:
// * the spin-summed matrix element gains a third structure m^2 (q.q') with coupling
//   beta_III = C_V^2 - C_A^2, minus for scattering and plus for the pair;
// * the electron momentum P = sqrt(E^2 - m^2) replaces E in the kinematics, so the angular
//   weights H are no longer polynomials in E: each node evaluates them afresh;
// * the electron energy starts at m (and the positron's at m), so the quadrature rule changes
//   (below).
//
// Angular weight at a node. For fixed E the azimuth-averaged integrand is f(k) =
// sum c_{n,a} E^a k^n with n even in -4..6 (Laurent coefficients per task, host tables), and
// H = Integral_{k0}^{k1} f dk. Two routes, by the length L = k1 - k0 of the momentum-transfer
// interval against its distance k0 from k = 0 (the only singular point):
//   long  (L > k0/16): exact, H = L sum c_{n,a} E^a h_n with h_n = (k1^{n+1} - k0^{n+1})/((n+1) L)
//         formed from positive terms only; the node accumulates W B L E^a h_n into 16 moments
//         and the task contracts them with its coefficients once, at the end;
//   short (L <= k0/16): the Laurent terms cancel there, so f is evaluated directly from the
//         cosines of the kinematics at 5 Gauss-Legendre points on [k0, k1] (the singular point
//         lies at least 16 L away, Bernstein-ellipse radius >= 33 + 8 sqrt 17, error ~1e-15).
// The third structure, m^2 (q.q')/(e e') P_l(x), is a polynomial in k (n = 0, 2, 4): exact
// on both routes.
//
// Rule (panels of nquad/4 Gauss-Legendre nodes, as the massless PANEL rule with the electron
// threshold in place of E = 0 and the mass-shifted kink of H in place of eps_j):
//   scattering (eps_i >= eps_j, omega = eps_i - eps_j): breakpoints sort(m, max(m, mu - omega),
//     max(m, mu), min(E_k, max(m, mu) + 10 T)); panels in s with E = m + (b_3 - m) s^2 (H grows
//     like sqrt(E - m) at threshold, linear in s), then a Gauss-Laguerre tail of scale T;
//   pair: breakpoints sort(m, E_lo, E_hi, clip(mu, m, w - m), w - m) (w = eps_i + eps_j);
//     panels in theta with E = m + (w - 2m) sin^2(pi theta/2), quadratic at both thresholds.
// Layout, completion, species sums and contraction follow the massless forward, with the
// third structure beside the other two.
#include <hip/hip_runtime.h>

#include "vtx_internal.h"

namespace vtx {
namespace {

constexpr int kMassBlock = 256;
constexpr double kShortRatio = 0.0625;   // short route when L <= kShortRatio k0
constexpr int64_t kMassSlice = int64_t(1) << 22;   // zones per launch (grid x-dimension)

// 1/x for finite x > 0: the hardware reciprocal refined by two Newton steps, to FP64
// rounding, instead of the division sequence.
__device__ __forceinline__ double recip_m(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}

__device__ __forceinline__ int m_partner(int s) { return s == 2 ? 2 : 1 - s; }
__device__ __forceinline__ int m_tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Blocking factor sigma(z) sigma(K - z) of a node, sigma(z) = 1/(1 + e^-z): the two Fermi-Dirac
// arguments of a task sum to the task constant K = D/T >= 0 (scattering D = omega, pair
// D = eps_i + eps_j). With t the smaller argument (t <= K/2), a = e^t and C = e^-K,
//   B = a / ((1 + a)(1 + C a)),
// one exponential per node; C a <= 1 and t is capped at 700 (both factors are then 1 to FP64
// precision), a very negative t gives a = 0 and B = 0.
__device__ __forceinline__ double blocking_m(double z, double K, double C) {
  const double a = exp(fmin(fmin(z, K - z), 700.0));
  return a * recip_m((1.0 + a) * (1.0 + C * a));
}

__device__ __forceinline__ void sort3(double& a, double& b, double& c) {
  double t;
  if (b < a) { t = a; a = b; b = t; }
  if (c < b) { t = b; b = c; c = t; }
  if (b < a) { t = a; a = b; b = t; }
}

// h_n = (x^{n+1} - y^{n+1}) / ((n + 1)(x - y)), x = k1 > y = k0 >= 0, for n = -4, -2, 0, 2, 4, 6
// (h[0..5]); sums of positive terms s_n = sum_{a <= n} x^a y^{n-a}. Where y = 0 the negative
// powers' coefficients vanish (diagonal task), and their h is set to 0.
__device__ __forceinline__ void laurent_means(double x, double y, double h[6]) {
  const double y2 = y * y, y3 = y2 * y;
  const double s1 = x + y, s2 = x * s1 + y2, s3 = x * s2 + y3, s4 = x * s3 + y2 * y2, s5 = x * s4 + y2 * y3,
               s6 = x * s5 + y3 * y3;
  const bool pos = y > 0.0;
  const double ixy = pos ? recip_m(x * y) : 0.0;
  h[0] = s2 * ixy * ixy * ixy * (1.0 / 3.0);
  h[1] = ixy;
  h[2] = 1.0;
  h[3] = s2 * (1.0 / 3.0);
  h[4] = s4 * 0.2;
  h[5] = s6 * (1.0 / 7.0);
}

// Accumulators of one task: long-route moments M[slot] (slot 3 (n + 4)/2 + a, 15 for (6, 0)),
// the short route's third-structure moments and direct sums.
struct Acc {
  double M[16];
  double M3[3];
  double Q[4];
};

__device__ __forceinline__ void acc_zero(Acc& A) {
#pragma unroll
  for (int s = 0; s < 16; ++s) A.M[s] = 0.0;
  A.M3[0] = A.M3[1] = A.M3[2] = 0.0;
  A.Q[0] = A.Q[1] = A.Q[2] = A.Q[3] = 0.0;
}

__device__ __forceinline__ void add_long(Acc& A, double wbl, double E, const double h[6]) {
  const double t1 = wbl * E, t2 = t1 * E;
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    A.M[3 * r] += wbl * h[r];
    A.M[3 * r + 1] += t1 * h[r];
    A.M[3 * r + 2] += t2 * h[r];
  }
  A.M[15] += wbl * h[5];
}

// Azimuth-averaged integrand f_{S,l}(k) / (e e') for S = I, II and l = 0, 1 at momentum
// transfer k: v[0..3] = (I,0), (I,1), (II,0), (II,1). pca = P cos(alpha), side +1 for
// scattering (q, q' on one side of k) and -1 for the pair; Mx the (S = I, S = II) structures.
struct Kin {
  double e, ep, E, P2;
  double ie, iep, iee;   // 1/e, 1/e', 1/(e e'): task constants
};

__device__ __forceinline__ void averages(const Kin& K, double pca, double cb, double cbp, double sbsb, double side,
                                         double& qp, double& qpp, double& qqp) {
  qp = K.e * (K.E - cb * pca);
  qpp = K.ep * (K.E - cbp * pca);
  qqp = K.e * K.ep *
        (K.E * K.E - K.E * (cb + cbp) * pca + cb * cbp * pca * pca + side * 0.5 * sbsb * (K.P2 - pca * pca));
}

__device__ __forceinline__ void nes_direct(const Kin& K, double om, double w, double A_, double k, double v[4]) {
  const double ik = recip_m(k);
  const double Q2 = (k - om) * (k + om);
  const double iee = K.iee;
  const double x = 1.0 - 0.5 * Q2 * iee;
  const double pca = 0.5 * (A_ - k * k) * ik;
  const double cb = 0.5 * (w * om + k * k) * ik * K.ie, cbp = 0.5 * (w * om - k * k) * ik * K.iep;
  const double sbsb = 0.25 * Q2 * (w - k) * (w + k) * iee * ik * ik;
  double qp, qpp, qqp;
  averages(K, pca, cb, cbp, sbsb, 1.0, qp, qpp, qqp);
  const double M1 = (qqp + 0.5 * Q2 * qp) * iee, M2 = (qqp - 0.5 * Q2 * qpp) * iee;
  v[0] = M1;
  v[1] = x * M1;
  v[2] = M2;
  v[3] = x * M2;
}

__device__ __forceinline__ void pair_direct(const Kin& K, double d, double w, double k, double v[4]) {
  const double ik = recip_m(k);
  const double s = (w - k) * (w + k);
  const double iee = K.iee;
  const double x = 1.0 - 0.5 * s * iee;
  const double ad = fabs(d);
  const double pca = 0.5 * (k * k + (2.0 * K.E - w) * w) * ik;
  const double cb = 0.5 * (d * w + k * k) * ik * K.ie, cbp = 0.5 * (k * k - d * w) * ik * K.iep;
  const double sbsb = 0.25 * s * (k - ad) * (k + ad) * iee * ik * ik;
  double qp, qpp, qqp;
  averages(K, pca, cb, cbp, sbsb, -1.0, qp, qpp, qqp);
  const double M1 = (0.5 * s * qpp - qqp) * iee, M2 = (0.5 * s * qp - qqp) * iee;
  v[0] = M1;
  v[1] = x * M1;
  v[2] = M2;
  v[3] = x * M2;
}

// One node of a task: weight wb = W B, interval [k0, k1]; PAIR picks the integrand.
template <bool PAIR>
__device__ __forceinline__ void node_mass(const DevPlan& P, Acc& A, const Kin& K, double wb, double k0, double k1,
                                          double om_or_d, double w, double A_) {
  const double L = k1 - k0;
  if (!(L > 0.0) || wb == 0.0) return;
  const double wbl = wb * L;
  double h[6];
  laurent_means(k1, k0, h);
  if (L > kShortRatio * k0) {
    add_long(A, wbl, K.E, h);
  } else {
    A.M3[0] += wbl;
    A.M3[1] += wbl * h[3];
    A.M3[2] += wbl * h[4];
#pragma unroll 1
    for (int g = 0; g < kMassGauss; ++g) {
      const double2 gk = P.mass_gauss[g];   // (t, w) on [0, 1]
      const double k = k0 + L * gk.x;
      double v[4];
      if (PAIR)
        pair_direct(K, om_or_d, w, k, v);
      else
        nes_direct(K, om_or_d, w, A_, k, v);
      const double c = wbl * gk.y;
      A.Q[0] += c * v[0];
      A.Q[1] += c * v[1];
      A.Q[2] += c * v[2];
      A.Q[3] += c * v[3];
    }
  }
}

// Task values from the accumulators: q[0..3] = (I,0), (I,1), (II,0), (II,1), q[4..5] = (III,0),
// (III,1), the prefactor and the third structure's sign folded into the coefficients.
__device__ __forceinline__ void finish(const MassCoef& C, const Acc& A, double pref, double q[6]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = pref * A.Q[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) s += C.c[c][k] * A.M[k];
    q[c] = s;
  }
#pragma unroll
  for (int l = 0; l < 2; ++l)
    q[4 + l] = C.c3[l][0] * (A.M[6] + A.M3[0]) + C.c3[l][1] * (A.M[9] + A.M3[1]) + C.c3[l][2] * (A.M[12] + A.M3[2]);
}

// Scattering task (i >= j) in a zone of temperature T and chemical potential mu (the mirrored
// zone, mu -> -mu, for scattering on positrons).
__device__ void nes_task(const DevPlan& P, int t, double T, double mu, double q[6]) {
  const int ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
  const MassCoef& C = P.mass_nes[t];
  const double m = kMe, e = P.eps[i], ep = P.eps[j], om = e - ep, w = e + ep;
  const double invT = 1.0 / T;
  double b1 = fmax(m, mu - om), b2 = fmax(m, mu), b3 = fmin(C.k0, b2 + kKappa * T);
  sort3(b1, b2, b3);
  const double Lr = b3 - m, Ls = Lr > 0.0 ? Lr : 1.0;
  const double s[4] = {0.0, sqrt(fmax(b1 - m, 0.0) / Ls), sqrt(fmax(b2 - m, 0.0) / Ls), sqrt(fmax(b3 - m, 0.0) / Ls)};
  Acc A;
  acc_zero(A);
  Kin K;
  K.e = e;
  K.ep = ep;
  K.ie = P.inv_eps[i];
  K.iep = P.inv_eps[j];
  K.iee = K.ie * K.iep;
  const double Kt = om * invT, Ct = exp(-Kt);
  auto node = [&](double E, double W) {
    const double B = blocking_m((mu - E) * invT, Kt, Ct);
    const double Ep = E + om;
    const double Pn = sqrt((E - m) * (E + m)), Pp = sqrt((Ep - m) * (Ep + m));
    const double sp = Pn + Pp;
    const double A_ = (2.0 * E + om) * om;
    const double k0 = sp > 0.0 ? A_ * recip_m(sp) : 0.0;
    K.E = E;
    K.P2 = (E - m) * (E + m);
    node_mass<false>(P, A, K, W * B, k0, fmin(w, sp), om, w, A_);
  };
  for (int p = 0; p < 3; ++p) {
    const double sa = s[p], ds = s[p + 1] - s[p];
    for (int k = 0; k < P.m4; ++k) {
      const double4 g = P.leg64[k];
      const double v = sa + ds * g.x;
      node(m + Lr * v * v, ds * g.z * 2.0 * Lr * v);
    }
  }
  for (int k = 0; k < P.m4; ++k) {
    const double4 g = P.lag64[k];
    node(b3 + T * g.x, T * g.z);
  }
  finish(C, A, kGF * kGF / (M_PI * e * ep), q);
}

// Pair task {i, j} (i >= j): structures I and II of (i, j) (II of (i, j) = I of (j, i)) and
// the symmetric third one.
__device__ void pair_task(const DevPlan& P, int t, double T, double mu, double q[6]) {
  const int ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
  const MassCoef& C = P.mass_pair[t];
  const double m = kMe, e = P.eps[i], ep = P.eps[j], d = e - ep, w = e + ep;
  if (!(C.support > 0.0)) {
#pragma unroll
    for (int c = 0; c < 6; ++c) q[c] = 0.0;
    return;
  }
  const double invT = 1.0 / T, span = w - 2.0 * m, top = w - m;
  const double Kp = w * invT, Cp = exp(-Kp);
  double b1 = fmin(fmax(C.k0, m), top), b2 = fmin(fmax(C.k1, m), top), b3 = fmin(fmax(mu, m), top);
  sort3(b1, b2, b3);
  auto theta = [&](double b) { return acos(fmin(fmax(1.0 - 2.0 * (b - m) / span, -1.0), 1.0)) / M_PI; };
  const double th[5] = {0.0, theta(b1), theta(b2), theta(b3), 1.0};
  Acc A;
  acc_zero(A);
  Kin K;
  K.e = e;
  K.ep = ep;
  K.ie = P.inv_eps[i];
  K.iep = P.inv_eps[j];
  K.iee = K.ie * K.iep;
  for (int p = 0; p < 4; ++p) {
    const double ta = th[p], dt = th[p + 1] - th[p];
    for (int k = 0; k < P.m4; ++k) {
      const double4 g = P.leg64[k];
      const double v = ta + dt * g.x;
      const double sh = sinpi(0.5 * v);
      const double E = m + span * sh * sh, Eb = w - E;
      const double W = dt * g.z * span * 0.5 * M_PI * sinpi(v);
      const double B = blocking_m((E - mu) * invT, Kp, Cp);
      const double Pn = sqrt((E - m) * (E + m)), Pb = sqrt((Eb - m) * (Eb + m));
      const double sp = Pn + Pb;
      const double k0 = fmax(fabs(d), fabs((2.0 * E - w) * w) * recip_m(sp));
      K.E = E;
      K.P2 = (E - m) * (E + m);
      node_mass<true>(P, A, K, W * B, k0, sp, d, w, 0.0);
    }
  }
  finish(C, A, kGF * kGF / (M_PI * e * ep), q);
}

// LDS (doubles): f [6 ne] | scattering [6 ntn] | positron scattering [6 ntn] | pair, structure
// I of (i, j) at slot i ne + j [2 ne^2] | pair, third structure [2 ne^2] | exp(-|eps_i - eps_j|/T)
// [ne^2] | exp(-(eps_i + eps_j)/T) [ne^2].
struct MLay {
  int q, m, p, p3, d;
};
__device__ __forceinline__ MLay mass_layout(const DevPlan& P) {
  MLay L;
  const int ne = P.ne, n2 = ne * ne;
  L.q = 6 * ne;
  L.m = L.q + 6 * P.ntn;
  L.p = L.m + 6 * P.ntn;
  L.p3 = L.p + 2 * n2;
  L.d = L.p3 + 2 * n2;
  return L;
}

}  // namespace

size_t mass_lds_bytes(int ne) {
  const int ntn = ne * (ne + 1) / 2, n2 = ne * ne;
  return sizeof(double) * (size_t)(6 * ne + 12 * ntn + 6 * n2);
}

__global__ __launch_bounds__(kMassBlock) void rates_mass_kernel(DevPlan P, int64_t nz, const double* __restrict__ Tz,
                                                                const double* __restrict__ etaz,
                                                                const double* __restrict__ f,
                                                                double* __restrict__ eta_out,
                                                                double* __restrict__ chi_out) {
  extern __shared__ double smem[];
  const int64_t z = blockIdx.x;
  if (z >= nz) return;   // uniform
  const int ne = P.ne, n2 = ne * ne, ntn = P.ntn;
  const MLay L = mass_layout(P);
  const double T = Tz[z], mu = etaz[z] * T, invT = 1.0 / T;
  const bool do_nes = P.processes & VTX_NES, do_nps = P.processes & VTX_NPS, do_pair = P.processes & VTX_PAIR;
  for (int r = threadIdx.x; r < 6 * ne; r += blockDim.x) smem[r] = f[z * 6 * ne + r];
  for (int r = threadIdx.x; r < ntn; r += blockDim.x) {
    const int ij = P.nes_ij[r], i = ij & 0xff, j = ij >> 8;
    const double ei = P.eps[i], ej = P.eps[j];
    const double dd = exp(-(ei - ej) * invT), pf = exp(-(ei + ej) * invT);
    smem[L.d + i * ne + j] = dd;
    smem[L.d + j * ne + i] = dd;
    smem[L.d + n2 + i * ne + j] = pf;
    smem[L.d + n2 + j * ne + i] = pf;
  }
  // tasks: scattering on electrons, on positrons (mirrored zone), pair; a lane per task
  for (int u = threadIdx.x; u < 3 * ntn; u += blockDim.x) {
    const int kind = u / ntn, t = u - kind * ntn;
    double q[6];
    if (kind == 0) {
      if (!do_nes) continue;
      nes_task(P, t, T, mu, q);
      double* o = smem + L.q + 6 * t;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = q[c];
    } else if (kind == 1) {
      if (!do_nps) continue;
      nes_task(P, t, T, -mu, q);
      double* o = smem + L.m + 6 * t;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = q[c];
    } else {
      if (!do_pair) continue;
      pair_task(P, t, T, mu, q);
      const int ij = P.nes_ij[t], i = ij & 0xff, j = ij >> 8;
      smem[L.p + 2 * (i * ne + j)] = q[0];
      smem[L.p + 2 * (i * ne + j) + 1] = q[1];
      smem[L.p + 2 * (j * ne + i)] = q[2];
      smem[L.p + 2 * (j * ne + i) + 1] = q[3];
      smem[L.p3 + 2 * (i * ne + j)] = q[4];
      smem[L.p3 + 2 * (i * ne + j) + 1] = q[5];
      smem[L.p3 + 2 * (j * ne + i)] = q[4];
      smem[L.p3 + 2 * (j * ne + i) + 1] = q[5];
    }
  }
  __syncthreads();
  // completion, species sums and contraction: a lane per (species, bin i)
  for (int r = threadIdx.x; r < 3 * ne; r += blockDim.x) {
    const int s = r / ne, i = r - s * ne, sb = m_partner(s);
    const double bI = P.beta[s][0], bII = P.beta[s][1], bIII = P.beta3[s];
    double e0 = 0.0, c0 = 0.0, e1 = 0.0, c1 = 0.0;
    for (int j = 0; j < ne; ++j) {
      const double cw = P.c0w[j];
      const double dfac = smem[L.d + i * ne + j];
      const double cin = (i > j) ? cw * dfac : cw, cout = (i < j) ? cw * dfac : cw;
      const double f0 = smem[(2 * s) * ne + j], f1 = smem[(2 * s + 1) * ne + j];
      if (do_nes || do_nps) {
        const int tq = 6 * (i >= j ? m_tri(i, j) : m_tri(j, i));
        double k0 = 0.0, k1 = 0.0;
        if (do_nes) {
          const double* q = smem + L.q + tq;
          k0 += bI * q[0] + bII * q[2] + bIII * q[4];
          k1 += bI * q[1] + bII * q[3] + bIII * q[5];
        }
        if (do_nps) {   // positron target: beta_I <-> beta_II
          const double* q = smem + L.m + tq;
          k0 += bII * q[0] + bI * q[2] + bIII * q[4];
          k1 += bII * q[1] + bI * q[3] + bIII * q[5];
        }
        const double t0 = f0 * k0, t1 = f1 * k1;
        e0 += cin * t0;
        c0 += cin * t0 + cout * (k0 - t0);
        e1 += cin * t1;
        c1 += (cin - cout) * t1;
      }
      if (do_pair) {
        const double* aij = smem + L.p + 2 * (i * ne + j);
        const double* aji = smem + L.p + 2 * (j * ne + i);
        const double* a3 = smem + L.p3 + 2 * (i * ne + j);
        const double ka0 = bI * aij[0] + bII * aji[0] + bIII * a3[0];
        const double ka1 = bI * aij[1] + bII * aji[1] + bIII * a3[1];
        const double pf = smem[L.d + n2 + i * ne + j], cwp = cw * pf;
        const double g0 = smem[(2 * sb) * ne + j], g1 = smem[(2 * sb + 1) * ne + j];
        const double tp = g0 * ka0, u1 = cw * g1 * ka1;
        const double pr0 = cwp * (ka0 - tp);
        e0 += pr0;
        c0 += pr0 + cw * tp;
        e1 -= u1 * pf;
        c1 += u1 * (1.0 - pf);
      }
    }
    const int64_t o = z * 6 * ne + (2 * s) * ne + i;
    eta_out[o] = e0;
    chi_out[o] = c0;
    eta_out[o + ne] = e1;
    chi_out[o + ne] = c1;
  }
}

hipError_t launch_forward_mass(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                               double* eta, double* chi, hipStream_t s) {
  const size_t lds = mass_lds_bytes(P.ne);
  hipError_t e = hipFuncSetAttribute((const void*)rates_mass_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int64_t zs = 6 * P.ne;
  for (int64_t z0 = 0; z0 < nz; z0 += kMassSlice) {
    const int64_t n = nz - z0 < kMassSlice ? nz - z0 : kMassSlice;
    hipLaunchKernelGGL(rates_mass_kernel, dim3((unsigned)n), dim3(kMassBlock), lds, s, P, n, T + z0, eta_e + z0,
                       f + z0 * zs, eta + z0 * zs, chi + z0 * zs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vtx
