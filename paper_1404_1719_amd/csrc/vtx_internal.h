// Internal declarations shared by the host layer (vtx_host.cpp) and the kernels
// (vtx_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vtx {

constexpr int kMaxNE = 32;
constexpr int kMaxNquad = 64;
constexpr int kBlock = 256;
// Decay panel above mu_e is capped at KAPPA * T; the rest of the decay goes to the tail.
constexpr double kKappa = 10.0;
constexpr double kGF = 1.1663787e-11;        // MeV^-2
constexpr double kHbarC = 1.973269804e-11;   // MeV cm

// Angular-weight coefficients of one scattering task (eps_i >= eps_j), comps
// (S, l) = (I,0), (I,1), (II,0), (II,1); variable u = E / eps_j; lo: E < eps_j, hi: E >= eps_j.
// lo: degree-7 Bernstein, H = sum_k lo[k] u^k (1-u)^(7-k) (binomials folded in);
// hi: monomials, H = sum_k hi[k] u^k. The task prefactor G_F^2 / (pi eps_i eps_j) is folded in.
struct NesCoef {
  double lo[4][8];
  double hi[4][4];   // [3] unused
};

// Pair task (i, j): H^{P,I}_l(eps_i, eps_j, .) on the three pieces
// A: [0, m] var E/m,  B: [m, M] var E/M,  C: [M, w] var (w - E)/m  (m, M = min, max),
// each in the folded degree-7 Bernstein basis of its variable. Prefactor folded in.
struct PairCoef {
  double piece[3][2][8];
};

// Everything a kernel needs about the zone-independent tables; passed by value.
struct DevPlan {
  int ne;
  int ntn;          // scattering tasks  ne (ne + 1) / 2
  int ntp;          // pair tasks        ne * ne
  int m4;           // nodes per group   nquad / 4
  int rule;         // VTX_RULE_*
  int processes;    // VTX_NES | VTX_PAIR
  int precision;    // VTX_FP64 / VTX_MIXED
  int nlag;         // entries of the Laguerre table (m4 for PANEL, nquad for LAGUERRE)
  double eta_fp64;
  double beta[3][2];
  const double* eps;        // [ne]
  const double* c0w;        // [ne] c0 w_j
  const int* nes_ij;        // [ntn] i | (j << 8)
  const NesCoef* nes_coef;  // [ntn]
  const PairCoef* pair_coef;// [ntp]  task p = i * ne + j
  const double4* leg64;     // [m4]   {t, 1 - t, w, 0} on [0, 1]
  const double4* lag64;     // [nlag] {x, x, w exp(x), 0}
  const float4* leg32;
  const float4* lag32;
};

hipError_t launch_forward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                          const double* f, double* eta, double* chi, hipStream_t s);
hipError_t launch_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                           const double* f, const double* g_eta, const double* g_chi,
                           double* g_T, double* g_eta_e, double* g_f, hipStream_t s);

}  // namespace vtx
