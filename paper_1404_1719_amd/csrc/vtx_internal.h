// Internal declarations shared by the host layer (vtx_host.cpp) and the kernels
// (vtx_kernels.hip, vtx_newton.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vtx_rates.h"

namespace vtx {

constexpr int kMaxNE = 32;
constexpr int kMaxNquad = 64;
// Decay panel above mu_e is capped at KAPPA * T; the rest of the decay goes to the tail.
constexpr double kKappa = 10.0;
constexpr double kGF = 1.1663787e-11;        // MeV^-2
constexpr double kHbarC = 1.973269804e-11;   // MeV cm
constexpr double kMe = 0.51099895;           // electron mass, MeV
constexpr int kMassGauss = 5;                // points of the short momentum-transfer route

// Angular-weight coefficients of one scattering task (eps_i >= eps_j), comps
// (S, l) = (I,0), (I,1), (II,0), (II,1); variable u = E / eps_j.
// lo (E < eps_j): H = sum_{k=3..7} lo[k-3] u^k (1-u)^(7-k), the degree-7 Bernstein form with
//   binomials folded in; its k = 0..2 coefficients vanish exactly (H ~ E^3 near E = 0).
// hi (E >= eps_j): H = sum_{k=0..2} hi[k] u^k.
// The task prefactor G_F^2 / (pi eps_i eps_j) is folded in.
struct NesCoef {
  double lo[4][5];
  double hi[4][3];
};

// Pair task (i, j): H^{P,I}_l(eps_i, eps_j, .), l = 0, 1, on its three pieces (m, M = min,
// max of eps_i, eps_j; w = eps_i + eps_j):
//   A on [0, m], u = E/m:        folded Bernstein k = 3..7 (factor E^3);
//   B on [m, M], u = E/M:        monomials k = 0..2;
//   C on [M, w], u = (w - E)/m:  folded Bernstein k = 3..7 (factor (w - E)^3).
// Prefactor folded in.
struct PairCoef {
  double A[2][5];
  double B[2][3];
  double C[2][5];
};

// Electron-mass weights of one task (i >= j; for the pair, the unordered pair {i, j}):
// c[comp][slot], comps (S, l) = (I,0), (I,1), (II,0), (II,1), are the Laurent coefficients of
// the azimuth-averaged integrand in E^a k^n (slot 3 (n + 4)/2 + a for n = -4..4, slot 15 for
// (6, 0)) and c3[l][n/2] the third structure's (n = 0, 2, 4), with the prefactor
// G_F^2/(pi e_i e_j) folded in and the third structure's sign in the rates (minus for
// scattering, plus for the pair). k0: scattering E_k, the kink of H (>= m); pair E_lo;
// k1: pair E_hi; support: pair, 1 when the pair is open (e_i e_j > m^2, e_i + e_j > 2m).
struct MassCoef {
  double c[4][16];
  double c3[2][3];
  double k0, k1, support, pad;
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
  int block;        // threads per workgroup of the rate kernels: 256, or 512 (diagnostic)
  double eta_fp64;
  double beta[3][2];
  const double* eps;        // [ne]
  const double* inv_eps;    // [ne] 1 / eps
  const double* c0w;        // [ne] c0 w_j
  const int* nes_ij;        // [ntn] i | (j << 8)
  const NesCoef* nes_coef;  // [ntn]
  const PairCoef* pair_coef;// [ntp]  task p = i * ne + j
  // Task order by the zone's k = #{eps_j < mu_e}: row k lists the (i >= j) tasks so that those
  // whose groups take the same node-loop variants are contiguous (see task_order in
  // vtx_host.cpp). Scattering tasks and pair tasks (one per unordered pair) share it.
  const uint16_t* task_order; // [ne + 1][ntn]
  const MassCoef* mass_nes;   // [ntn] electron-mass weights, scattering task t
  const MassCoef* mass_pair;  // [ntn] electron-mass weights, pair {i, j} of task t
  const double2* mass_gauss;  // [kMassGauss] {t, w} on [0, 1]
  double beta3[3];            // beta_III = C_V^2 - C_A^2 per species
  const double4* leg64;     // [m4]   {t, 1 - t, w, 0} on [0, 1]
  const double4* lag64;     // [nlag] {x, x, w exp(x), 0}
  const float4* leg32;
  const float4* lag32;
};

hipError_t launch_forward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                          const double* f, double* eta, double* chi, hipStream_t s);
hipError_t launch_jacobian(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                           double* eta, double* chi, double* jac, hipStream_t s);
int64_t task_values(int ne, unsigned processes);   // doubles per zone of the packed task values
hipError_t launch_tasks(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, double* tasks,
                        bool rows, hipStream_t s);
hipError_t launch_interp(const DevPlan& P, const vtx_lattice& lat, const double* table, int64_t nz, const double* T,
                         const double* eta_e, const double* f, double* eta, double* chi, hipStream_t s);
hipError_t launch_forward_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                                   const double* f, const double* g_eta, const double* g_chi, double* eta,
                                   double* chi, double* g_T, double* g_eta_e, double* g_f, hipStream_t s);
hipError_t launch_backward(const DevPlan& P, int64_t nz, const double* T, const double* eta_e,
                           const double* f, const double* g_eta, const double* g_chi,
                           double* g_T, double* g_eta_e, double* g_f, hipStream_t s);

// Newton step of the radial sweep (vtx_newton.hip).
hipError_t launch_ray_system(int ne, int64_t nz, int nzr, double dt, const double* jac, const double* f,
                             const double* f_n, const double* f_nm1, const double* eta, const double* chi,
                             const double* lo, const double* up, double* D, double* rhs, hipStream_t s);
hipError_t launch_ray_solve(int nb, int64_t nrays, int nzr, const double* lo, double* D, const double* up,
                            double* rhs, hipStream_t s);
int max_block();   // largest diagonal block the solve holds in LDS

// Forward with the electron mass (vtx_massive.hip), FP64, PANEL rule.
hipError_t launch_forward_mass(const DevPlan& P, int64_t nz, const double* T, const double* eta_e, const double* f,
                               double* eta, double* chi, hipStream_t s);
size_t mass_lds_bytes(int ne);

}  // namespace vtx
