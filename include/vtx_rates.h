/*
 * vtx_rates.h -- C ABI of the MI355X (gfx950) neutrino-matter interaction-rate library.
 *
 * What it computes (per spatial zone): the energy-coupled interaction kernels of
 * neutrino-electron scattering and e+e- pair annihilation/production, Legendre moments
 * l = 0, 1, each a quadrature over the electron energy of Fermi-Dirac products, for every
 * (eps_i, eps_j) energy-bin pair, contracted at once with the neutrino distribution into
 * emissivities eta and opacities chi. The paper (Marek, Rampp, Hanke, Janka, "Towards
 * Petaflops Capability of the VERTEX Supernova Code") lists these rates as the model
 * component that feeds the transport source terms (Sect. 2.1) and the Jacobian of the
 * implicit ray-by-ray Newton-Raphson solve (Sect. 2.1, radial sweep); the moments J, H of
 * its Eq. 1 are the f0, f1 moments used here, with the (2 pi hbar c)^3 phase-space
 * normalisation of its intensity definition.
 *
 * Definitions (massless e+-, V-A couplings; G_F = 1.1663787e-11 MeV^-2,
 * hbar c = 1.973269804e-11 MeV cm, c0 = 1/(4 pi^2 hbar c)):
 *   Phi_out_l(i,j) = G_F^2/(pi eps_i eps_j) Int dE F(E)[1-F(E+eps_i-eps_j)] sum_S beta_S H^N_{l,S}
 *   Phi_a_l(i,j)   = G_F^2/(pi eps_i eps_j) Int dE [1-F(E)][1-Fbar(eps_i+eps_j-E)] sum_S beta_S H^P_{l,S}
 *   computed by quadrature for eps_i >= eps_j (scattering) and all pairs (pair), completed
 *   by detailed balance: Phi_out(i<j) = exp(-(eps_j-eps_i)/T) Phi_out(j,i),
 *   Phi_in(i,j) = Phi_out(j,i), Phi_p = exp(-(eps_i+eps_j)/T) Phi_a;
 *   eta/chi for species s (partner sbar), m = 0, 1, summed over both processes:
 *     eta0 = c0 sum_j w_j [Phi_in_0 f0(j) + Phi_p_0 (1 - f0sbar(j))]
 *     chi0 = c0 sum_j w_j [Phi_in_0 f0 + Phi_out_0 (1 - f0) + Phi_p_0 (1 - f0sbar) + Phi_a_0 f0sbar]
 *     eta1 = c0 sum_j w_j [Phi_in_1 f1(j) - Phi_p_1 f1sbar(j)]
 *     chi1 = c0 sum_j w_j [(Phi_in_1 - Phi_out_1) f1 + (Phi_a_1 - Phi_p_1) f1sbar]
 *   Quadrature rule (both rules keep n/4 nodes per group, continuous in T and eta_e):
 *     PANEL: scattering: Gauss-Legendre panels between sorted {0, max(0, mu-Delta), max(0, mu),
 *            min(eps_j, max(0, mu) + 10 T)} plus a Gauss-Laguerre tail of scale T;
 *            pair: Gauss-Legendre panels between sorted {0, min, max, clip(mu, 0, w), w}.
 *     LAGUERRE: scattering uses one n-point Gauss-Laguerre rule E = T x; pair as PANEL.
 *
 * Array layouts (row-major, FP64, DEVICE memory owned by the caller):
 *   T[nz] (MeV, > 0), eta_e[nz] (mu_e/T, finite; |eta_e| <= 700),
 *   f[nz][3][2][ne]   species (nu_e, anti-nu_e, nu_x) x moment (f0, f1) x bin,
 *   eta, chi, g_eta, g_chi, g_f: same [nz][3][2][ne] layout; g_T, g_eta_e: [nz].
 * The energy grid (vtx_grid) is HOST memory: ne bin centres (strictly increasing, > 0) and
 * ne bin volumes w_j = (e_{j+1}^3 - e_j^3)/3 in MeV^3.
 *
 * Execution: calls enqueue kernels on hip_stream (a hipStream_t; NULL = default stream) and
 * return without synchronising. The first call for a given (device, grid, nquad, rule,
 * sin2w) builds zone-independent tables (quadrature nodes, angular-weight coefficients)
 * and uploads them with synchronous copies; they live until vtx_release() or process exit.
 * Later calls allocate nothing. Calls are thread-safe.
 *
 * Errors: return VTX_OK (0) or a positive code; vtx_strerror() names it. Invalid arguments
 * are detected on the host before any launch. Values outside the input domain are not
 * checked on the device: they produce non-finite results confined to the offending zone.
 */
#ifndef VTX_RATES_H
#define VTX_RATES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VTX_ABI_VERSION 1

enum vtx_status {
  VTX_OK = 0,
  VTX_EINVAL = 1,   /* null pointer, bad sizes/options, unsorted or non-positive grid */
  VTX_EDEVICE = 2,  /* no HIP device, or the current device is not gfx950 */
  VTX_EHIP = 3,     /* a HIP runtime call or kernel launch failed */
  VTX_ENOMEM = 4    /* table allocation failed */
};

enum vtx_precision {
  VTX_FP64 = 0,   /* every step in FP64 */
  VTX_MIXED = 1   /* FP32 quadrature bulk (node coordinates, Fermi-Dirac factors, angular-weight
                     moments and their accumulation); FP64 angular-weight contraction,
                     detailed-balance factors and the per-zone contraction. Zones with
                     |eta_e| > eta_fp64 run entirely in FP64, their Fermi-Dirac factors among
                     the rest; the threshold is capped at 64, where a task's whole integrand can
                     sit near exp(-|eta_e|) and FP32 ends near exp(-87). Each class of zones is
                     computed by its own pass over the call's zones */
};

enum vtx_rule { VTX_RULE_LAGUERRE = 0, VTX_RULE_PANEL = 1 };

/* Processes: neutrino-electron scattering, pair annihilation/production, and (optional)
 * neutrino-positron scattering: the scattering kernels with the positron occupation
 * Fbar(E) = F(E; -mu_e) and the antiparticle-target couplings (C_A -> -C_A, which swaps
 * beta_I and beta_II); its Phi_in, Phi_out add to the electron ones in eta, chi and in the
 * scattering Jacobian block. */
enum vtx_process { VTX_NES = 1, VTX_PAIR = 2, VTX_NPS = 4 };

typedef struct {
  int32_t ne;          /* number of energy bins, 1..32 */
  const double* eps;   /* [ne] bin centres, MeV, host memory */
  const double* w;     /* [ne] bin volumes, MeV^3, host memory */
} vtx_grid;

typedef struct {
  int32_t precision;   /* vtx_precision */
  int32_t nquad;       /* nodes per kernel integral: multiple of 4 in [8, 64] */
  int32_t rule;        /* vtx_rule */
  uint32_t processes;  /* bitmask of vtx_process, nonzero (default VTX_NES | VTX_PAIR) */
  double sin2w;        /* weak mixing angle sin^2(theta_W), default 0.2312 */
  double eta_fp64;     /* mixed precision: zones with |eta_e| > min(eta_fp64, 64) run in FP64,
                          Fermi-Dirac factors included (default 30) */
} vtx_opts;

/* Fill *opts with the defaults: FP64, 48 nodes, PANEL, both processes, 0.2312, 30. */
void vtx_opts_default(vtx_opts* opts);

/*
 * Forward: the emissivities eta and opacities chi of nzones zones, i.e. the interaction rates
 * that the paper lists among the model's components and that enter the source terms of the
 * moment equations for J and H (Sect. 2.1, Eq. 1), computed by the definitions and the rule
 * above.
 *   grid, opts: host structs, read during the call only.
 *   T, eta_e [nz], f [nz][3][2][ne]: device inputs, read only.
 *   eta, chi [nz][3][2][ne]: device outputs; every entry of the nz zones is overwritten. They
 *   must not overlap the inputs or each other.
 *   nzones: 0 <= nzones <= 2^31 - 1; 0 is a no-op (pointers unused).
 * Errors, all detected before any launch: VTX_EINVAL (null grid/opts, a null array with
 * nzones > 0, bad grid or options, nzones out of range), VTX_EDEVICE (no gfx950 device
 * current), VTX_ENOMEM (tables could not be allocated). VTX_EHIP: a launch failed; outputs
 * are then unspecified.
 */
int vtx_rates_forward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                      const double* T, const double* eta_e, const double* f,
                      double* eta, double* chi, void* hip_stream);

/*
 * Forward with the electron mass m = 0.51099895 MeV: the accuracy variant for low T and eps,
 * where m is not small against the electron energies (the rates of Sect. 2.1's list of model
 * components with massive e+-). Same arguments, layouts, outputs and error behaviour as
 * vtx_rates_forward; opts->precision must be VTX_FP64 and opts->rule VTX_RULE_PANEL (else
 * VTX_EINVAL). What changes:
 *   - electrons and positrons have total energy E >= m and momentum P = sqrt(E^2 - m^2); the
 *     chemical potential mu_e = eta_e T includes the rest mass (positrons at -mu_e);
 *   - the spin-summed matrix element gains m^2 (q.q') beta_III, beta_III = C_V^2 - C_A^2
 *     (the same for a species and its antiparticle), with a minus sign for scattering and a
 *     plus sign for the pair; H^{N,P}_{l,III} = 1/(eps eps') Int dk P_l(x) m^2 (q.q');
 *   - the rule: scattering panels between sorted {m, max(m, mu-Delta), max(m, mu),
 *     min(E_k, max(m, mu) + 10 T)} in s with E = m + (b_3 - m) s^2, then the Gauss-Laguerre
 *     tail; E_k = (sqrt(Delta^2 + 4 eps_i eps_j + (eps_i+eps_j)^2 m^2/(eps_i eps_j)) - Delta)/2
 *     is the kink of H. Pair panels between sorted {m, E_lo, E_hi, clip(mu, m, w-m), w-m} in
 *     theta with E = m + (w - 2m) sin^2(pi theta/2), E_lo,hi = (w -+ |eps_i - eps_j|
 *     sqrt(1 - m^2/(eps_i eps_j)))/2; the pair kernel vanishes unless eps_i eps_j > m^2.
 * Only the forward exists in this form (no backward, Jacobian or mixed precision).
 */
int vtx_rates_forward_mass(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                           const double* T, const double* eta_e, const double* f,
                           double* eta, double* chi, void* hip_stream);

/*
 * Backward (vector-Jacobian product): given upstream gradients g_eta, g_chi of a scalar L,
 * writes g_T = dL/dT (at fixed eta_e), g_eta_e = dL/deta_e (at fixed T) and g_f = dL/df:
 * the derivatives of the rates that the implicit ray-by-ray Newton-Raphson solve needs
 * (Sect. 2.1, radial sweep). They are the exact derivatives of the discrete rule above,
 * including the motion of the quadrature nodes with T and mu_e = eta_e T. The kernels are
 * recomputed; nothing is saved from the forward call.
 *   T, eta_e [nz], f, g_eta, g_chi [nz][3][2][ne]: device inputs, read only.
 *   g_T, g_eta_e [nz], g_f [nz][3][2][ne]: device outputs, overwritten; no overlaps.
 *   grid, opts, nzones and the error codes as for vtx_rates_forward.
 */
int vtx_rates_backward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                       const double* T, const double* eta_e, const double* f,
                       const double* g_eta, const double* g_chi,
                       double* g_T, double* g_eta_e, double* g_f, void* hip_stream);

/*
 * Explicit Jacobian blocks with respect to f (the f-part of the Newton-Raphson Jacobian of
 * the implicit ray-by-ray transport solve, Sect. 2.1). The outputs are affine in f, so the
 * blocks depend on T and eta_e only:
 *   jac[nz][3 species s][2 process p][4 output o][ne i][ne j] = d out_o^s(i) / d f_m^{s'}(j),
 *   o = eta0, chi0, eta1, chi1 with m = o / 2; s' = s for p = 0 (scattering) and the pair
 *   partner of s (nu_e <-> anti-nu_e, nu_x <-> nu_x) for p = 1 (pair). For nu_x both blocks act
 *   on the same f and add. Entries, with the kernels completed as above:
 *     p = 0: c0 w_j [Phi_in_0, Phi_in_0 - Phi_out_0, Phi_in_1, Phi_in_1 - Phi_out_1](i, j)
 *            (scattering on electrons, plus on positrons with VTX_NPS)
 *     p = 1: c0 w_j [-Phi_p_0, Phi_a_0 - Phi_p_0, -Phi_p_1, Phi_a_1 - Phi_p_1](i, j)
 *   A process left out of opts->processes gives zero blocks. Same precision rules as the
 *   forward. jac (device memory, 192 ne^2 bytes per zone) is overwritten; T, eta_e as above.
 * f, eta, chi: all NULL, or all given; then the same call also writes eta, chi for f (the
 *   residual and its Jacobian at one zone state, from the same kernel values, bit-identical
 *   to vtx_rates_forward).
 */
int vtx_rates_jacobian(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                       const double* T, const double* eta_e, const double* f,
                       double* eta, double* chi, double* jac, void* hip_stream);

/*
 * Forward and backward in one pass: eta, chi as vtx_rates_forward and g_T, g_eta_e, g_f as
 * vtx_rates_backward (bit-identical to it), for callers that hold the upstream gradients
 * g_eta, g_chi before the forward values, e.g. a Newton-Krylov solve that needs a residual
 * and a transposed Jacobian product at one state. The backward recomputes the kernels
 * anyway, so eta, chi cost one extra contraction. eta, chi agree with vtx_rates_forward to
 * rounding (the kernels come from the backward's quadrature loop).
 */
int vtx_rates_forward_backward(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                               const double* T, const double* eta_e, const double* f,
                               const double* g_eta, const double* g_chi,
                               double* eta, double* chi,
                               double* g_T, double* g_eta_e, double* g_f, void* hip_stream);

/*
 * Tabulated kernels (a production alternative, kept as a comparison point): the quadratures
 * of each zone are interpolated from a table over a regular lattice of zone states instead of
 * being evaluated. Completion and contraction still take the zone's own T and f, so detailed
 * balance stays exact; the interpolation error sits in the quadratures alone.
 *
 * Task values of one zone (doubles, packed over the processes asked for), the quadratures
 * before completion, prefactor G_F^2/(pi eps_i eps_j) included:
 *   VTX_NES:  q[t][S][l], t = i (i + 1)/2 + j for i >= j, (S, l) = (I,0), (I,1), (II,0), (II,1)
 *   VTX_NPS:  the same on positrons
 *   VTX_PAIR: A[i][j][l] = Phi_a,I,l(i, j) for all i, j
 * vtx_task_values gives their count per zone.
 */
typedef struct {
  int32_t nt, nh;      /* lattice nodes along ln T and eta_e, >= 2 each */
  double lnT0, dlnT;   /* node a at ln T = lnT0 + a dlnT (dlnT > 0), T in MeV */
  double eta0, deta;   /* node b at eta_e = eta0 + b deta (deta > 0) */
} vtx_lattice;

int64_t vtx_task_values(int32_t ne, uint32_t processes);

/* Task values tasks[nz][vtx_task_values(ne, processes)] of nzones zone states (device
 * memory). */
int vtx_rates_tasks(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                    const double* T, const double* eta_e, double* tasks, void* hip_stream);

/* The same in interpolation variables: each adjacent (l = 0, l = 1) pair (x0, x1) of the
 * layout as (ln x0, x1/x0) (x0 <= 0, only from underflow, as (ln 1e-300, 0)); Phi_0 is
 * positive and exponential in 1/T and eta_e, and |Phi_1| <= Phi_0. Run over the lattice
 * states (row a nh + b) it builds the table of vtx_rates_forward_interp. */
int vtx_rates_table_rows(const vtx_grid* grid, const vtx_opts* opts, int64_t nzones,
                         const double* T, const double* eta_e, double* rows, void* hip_stream);

/* eta, chi with the zone's task values interpolated bilinearly from table[nt nh][values]
 * (device memory, rows of vtx_rates_table_rows): s = (ln T - lnT0)/dlnT, r = (eta_e - eta0)/deta, cell
 * a = clip(floor(s), 0, nt - 2), b = clip(floor(r), 0, nh - 2), fractions u = s - a,
 * v = r - b, weights (1-u)(1-v), u(1-v), (1-u) v, u v on t[a][b], t[a+1][b], t[a][b+1],
 * t[a+1][b+1] (linear extrapolation outside the lattice), then each pair mapped back by
 * x0 = exp(y0), x1 = y1 x0. FP64 throughout. table_len is the table's length in doubles; it
 * must equal nt nh vtx_task_values(ne, opts->processes) (the table's processes), and table
 * must be 16-byte aligned (VTX_EINVAL otherwise). */
int vtx_rates_forward_interp(const vtx_grid* grid, const vtx_opts* opts, const vtx_lattice* lattice,
                             const double* table, int64_t table_len, int64_t nzones, const double* T,
                             const double* eta_e, const double* f, double* eta, double* chi,
                             void* hip_stream);

/*
 * Newton step of an implicit radial sweep along rays. The paper's radial transport sweep is
 * implicit and ray by ray, BDF2 in time, solved by Newton-Raphson with an explicitly built
 * Jacobian and a direct solution of the linearised system (Sect. 2.1, radial sweep). These two
 * calls give that step for a minimal stated system that consumes the rates (the transport
 * terms proper are outside this library). Per ray, zones r = 0 .. nzr-1 (zones laid out ray by
 * ray, nrays * nzr in all), unknowns F_r = f[r][3][2][ne] (nb = 6 ne values, in f's layout):
 *   G_r = (3/2 F_r - 2 F_r^n + 1/2 F_r^{n-1}) / dt + (lo_r + up_r) F_r - lo_r F_{r-1} - up_r F_{r+1} - S_r
 * (componentwise; F_{-1} = F_nzr = 0; lo, up >= 0 a three-point radial coupling of each
 * component, e.g. upwind advection lo = v/dr, up = 0, or diffusion lo = up = D/dr^2), with the
 * moment sources of the rates S0 = eta0 - chi0 f0 - 3 chi1 f1, S1 = eta1 - chi1 f0 - chi0 f1
 * (per species and bin; time in units of length). The Jacobian is block tridiagonal:
 * D_r = dG_r/dF_r = (3/(2 dt)) I + diag(lo_r + up_r) - dS_r/dF_r, dG_r/dF_{r-1} = -diag(lo_r),
 * dG_r/dF_{r+1} = -diag(up_r); dS/dF comes from the rates' explicit blocks (vtx_rates_jacobian).
 *
 * vtx_ray_system: from jac [nz][3][2][4][ne][ne] (vtx_rates_jacobian), f, f_n, f_nm1, eta, chi
 *   (eta, chi of the rates at f; all [nz][3][2][ne]) and lo, up [nz][nb], writes the diagonal
 *   blocks D [nz][nb][nb] (row = (species, moment, bin) of G, column = that of F) and
 *   rhs = -G [nz][nb]. dt > 0. All device memory; D and rhs are overwritten.
 * vtx_ray_solve: solves -diag(lo_r) x_{r-1} + D_r x_r - diag(up_r) x_{r+1} = rhs_r along each ray
 *   (any nb x nb blocks, 1 <= nb <= vtx_ray_max_block(), 140), in place: rhs becomes x, and D
 *   is overwritten by the inverses of the eliminated diagonal blocks; nothing else is allocated.
 *   One ray per workgroup, Gauss-Jordan elimination with partial pivoting in FP64. A singular
 *   block gives non-finite x on its ray. The Newton update is F += x with rhs = -G.
 * Errors as for the rates (VTX_EINVAL for bad sizes or null pointers, checked on the host).
 */
int vtx_ray_system(int32_t ne, int64_t nrays, int32_t nzr, double dt, const double* jac, const double* f,
                   const double* f_n, const double* f_nm1, const double* eta, const double* chi,
                   const double* lo, const double* up, double* D, double* rhs, void* hip_stream);
int vtx_ray_solve(int32_t nb, int64_t nrays, int32_t nzr, const double* lo, double* D, const double* up,
                  double* rhs, void* hip_stream);
int vtx_ray_max_block(void);

/* Human-readable name of a status code (static storage). */
const char* vtx_strerror(int code);

/* VTX_ABI_VERSION of the built library. */
int vtx_abi_version(void);

/* Diagnostic: the rate kernels run one zone per workgroup of 4 waves (the default); waves = 8
 * runs them with 8. The results do not depend on it, bit for bit (a zone's task units are summed
 * in unit order whatever wave ran them); only the speed does. Returns the previous setting, or
 * -VTX_EINVAL for waves other than 4 or 8. Process-wide; affects later calls. */
int vtx_set_workgroup_waves(int waves);

/* Free every cached table on every device (no call may be in flight). */
void vtx_release(void);

/*
 * Host-side inspection of the zone-independent tables (no GPU needed; for tests).
 * vtx_gauss_rule: kind 0 = Gauss-Legendre on [0, 1] (x, w), kind 1 = Gauss-Laguerre with
 *   weights already multiplied by exp(x) (x, w exp(x)); n in [1, 64]. Arrays of n, host.
 * vtx_eval_hpoly: evaluates the angular weight H from the library's coefficient tables:
 *   process VTX_NES (requires e >= ep) or VTX_PAIR, comp = 2*(S-1) + l (S = 1, 2 for I, II),
 *   at n energies E[] (host), into out[] (host).
 * vtx_eval_hmass: the angular weight with the electron mass from the library's Laurent
 *   coefficient tables, on the exact route of long momentum-transfer intervals (the kernels
 *   switch to Gauss points on the integrand where the interval is short against its distance
 *   from k = 0; this hook does not); comp = 2*(S-1) + l for S = I, II and 4 + l for the
 *   third structure m^2 (q.q'). Same arguments otherwise; 0 outside the kinematic range.
 */
int vtx_gauss_rule(int kind, int n, double* x, double* w);
int vtx_eval_hpoly(int process, int comp, double e, double ep, int n, const double* E, double* out);
int vtx_eval_hmass(int process, int comp, double e, double ep, int n, const double* E, double* out);

/*
 * Host-side copy of one task's coefficient table, prefactor G_F^2/(pi e ep) included:
 *   VTX_NES (e >= ep): 32 doubles, lo[4 comps][5] then hi[4][3]; H = sum_{k=3..7} lo[k-3]
 *     u^k (1-u)^(7-k) for u = E/ep < 1 (folded Bernstein form; its k < 3 terms vanish) and
 *     H = sum_{k<3} hi[k] u^k for u >= 1;
 *   VTX_PAIR: 26 doubles, A[2 l][5], B[2][3], C[2][5]: folded Bernstein k = 3..7 in E/m on
 *     [0, m], monomials in E/M on [m, M], folded Bernstein in (e + ep - E)/m on [M, e + ep].
 * out must hold 32 doubles.
 */
int vtx_task_coefficients(int process, double e, double ep, double* out);

#ifdef __cplusplus
}
#endif

#endif /* VTX_RATES_H */
