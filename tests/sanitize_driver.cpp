// Host-only driver of the library's host layer (vtx_host.cpp) for an AddressSanitizer and
// UndefinedBehaviorSanitizer build with g++ (no device code). It exercises every host path that
// runs without a GPU: the Gauss rules for every size, the angular-weight tables and their
// evaluation over a grid of energies, the option defaults, and every entry point's argument
// checks (invalid arguments, then valid ones that stop at the missing device). The kernel
// launchers are stubs that must never be reached without a device.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hip/hip_runtime.h>

#include "../include/vtx_rates.h"
#include "../paper_1404_1719_amd/csrc/vtx_internal.h"

namespace vtx {
[[noreturn]] static void unreachable(const char* what) {
  std::fprintf(stderr, "launcher reached without a device: %s\n", what);
  std::abort();
}
hipError_t launch_forward(const DevPlan&, int64_t, const double*, const double*, const double*, double*, double*,
                          hipStream_t) { unreachable("forward"); }
hipError_t launch_jacobian(const DevPlan&, int64_t, const double*, const double*, const double*, double*, double*,
                           double*, hipStream_t) { unreachable("jacobian"); }
int64_t task_values(int ne, unsigned processes) {
  const int64_t ntn = int64_t(ne) * (ne + 1) / 2;
  return ((processes & VTX_NES) ? 4 * ntn : 0) + ((processes & VTX_NPS) ? 4 * ntn : 0) +
         ((processes & VTX_PAIR) ? 2 * int64_t(ne) * ne : 0);
}
hipError_t launch_tasks(const DevPlan&, int64_t, const double*, const double*, double*, bool, hipStream_t) {
  unreachable("tasks");
}
hipError_t launch_interp(const DevPlan&, const vtx_lattice&, const double*, int64_t, const double*, const double*,
                         const double*, double*, double*, hipStream_t) { unreachable("interp"); }
hipError_t launch_forward_backward(const DevPlan&, int64_t, const double*, const double*, const double*,
                                   const double*, const double*, double*, double*, double*, double*, double*,
                                   hipStream_t) { unreachable("forward_backward"); }
hipError_t launch_backward(const DevPlan&, int64_t, const double*, const double*, const double*, const double*,
                           const double*, double*, double*, double*, hipStream_t) { unreachable("backward"); }
hipError_t launch_ray_system(int, int64_t, int, double, const double*, const double*, const double*, const double*,
                             const double*, const double*, const double*, const double*, double*, double*,
                             hipStream_t) { unreachable("ray_system"); }
hipError_t launch_ray_solve(int, int64_t, int, const double*, double*, const double*, double*, hipStream_t) {
  unreachable("ray_solve");
}
int max_block() { return 140; }
hipError_t launch_forward_mass(const DevPlan&, int64_t, const double*, const double*, const double*, double*, double*,
                               hipStream_t) { unreachable("forward_mass"); }
size_t mass_lds_bytes(int) { unreachable("mass_lds_bytes"); }
}  // namespace vtx

static int failures = 0;
#define EXPECT(c)                                                        \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "expectation failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

int main() {
  // Gauss rules of every size: weights sum to the measure, nodes increase
  for (int kind = 0; kind < 2; ++kind)
    for (int n = 1; n <= 64; ++n) {
      std::vector<double> x(n), w(n);
      EXPECT(vtx_gauss_rule(kind, n, x.data(), w.data()) == VTX_OK);
      for (int k = 1; k < n; ++k) EXPECT(x[k] > x[k - 1]);
      if (kind == 0) {
        double s = 0;
        for (double v : w) s += v;
        EXPECT(std::fabs(s - 1.0) < 1e-12);
      }
    }
  double x1, w1;
  EXPECT(vtx_gauss_rule(2, 4, &x1, &w1) == VTX_EINVAL);
  EXPECT(vtx_gauss_rule(0, 65, &x1, &w1) == VTX_EINVAL);
  EXPECT(vtx_gauss_rule(0, 0, &x1, &w1) == VTX_EINVAL);
  // angular-weight tables and their evaluation
  std::vector<double> E(97), out(97), coef(32);
  for (int k = 0; k < 97; ++k) E[k] = -1.0 + 0.7 * k;
  const double es[] = {2.0, 5.5, 20.0, 140.0, 380.0};
  for (double e : es)
    for (double ep : es) {
      for (int comp = 0; comp < 4; ++comp) {
        if (e >= ep) EXPECT(vtx_eval_hpoly(VTX_NES, comp, e, ep, 97, E.data(), out.data()) == VTX_OK);
        EXPECT(vtx_eval_hpoly(VTX_PAIR, comp, e, ep, 97, E.data(), out.data()) == VTX_OK);
        for (double v : out) EXPECT(std::isfinite(v));
      }
      if (e >= ep) EXPECT(vtx_task_coefficients(VTX_NES, e, ep, coef.data()) == VTX_OK);
      EXPECT(vtx_task_coefficients(VTX_PAIR, e, ep, coef.data()) == VTX_OK);
    }
  EXPECT(vtx_eval_hpoly(VTX_NES, 4, 3.0, 2.0, 1, E.data(), out.data()) == VTX_EINVAL);
  EXPECT(vtx_eval_hpoly(VTX_NES, 0, 2.0, 3.0, 1, E.data(), out.data()) == VTX_EINVAL);
  EXPECT(vtx_task_coefficients(VTX_NPS, 3.0, 2.0, coef.data()) == VTX_EINVAL);
  // electron-mass weights: thresholds, the diagonal and energies far outside the range
  const double esm[] = {0.3, 0.6, 2.0, 20.0, 380.0};
  for (double e : esm)
    for (double ep : esm)
      for (int comp = 0; comp < 6; ++comp) {
        if (e >= ep) EXPECT(vtx_eval_hmass(VTX_NES, comp, e, ep, 97, E.data(), out.data()) == VTX_OK);
        EXPECT(vtx_eval_hmass(VTX_PAIR, comp, e, ep, 97, E.data(), out.data()) == VTX_OK);
        for (double v : out) EXPECT(std::isfinite(v));
      }
  EXPECT(vtx_eval_hmass(VTX_NES, 6, 3.0, 2.0, 1, E.data(), out.data()) == VTX_EINVAL);
  EXPECT(vtx_eval_hmass(VTX_NES, 0, 2.0, 3.0, 1, E.data(), out.data()) == VTX_EINVAL);
  EXPECT(vtx_task_coefficients(VTX_PAIR, -1.0, 2.0, coef.data()) == VTX_EINVAL);
  // options and argument checks of every entry point
  vtx_opts o;
  vtx_opts_default(&o);
  EXPECT(o.precision == VTX_FP64 && o.nquad == 48 && o.eta_fp64 == 30.0);
  vtx_opts_default(nullptr);
  const int ne = 21;
  std::vector<double> eps(ne), wv(ne);
  for (int j = 0; j < ne; ++j) {
    eps[j] = 2.0 * std::pow(190.0, (j + 0.5) / ne);
    wv[j] = eps[j] * eps[j];
  }
  vtx_grid g{ne, eps.data(), wv.data()};
  double dummy[8] = {1, 1, 1, 1, 1, 1, 1, 1};
  double* d = dummy;
  EXPECT(vtx_rates_forward(nullptr, &o, 1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_rates_forward(&g, &o, -1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_rates_forward(&g, &o, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == VTX_OK);
  EXPECT(vtx_rates_forward(&g, &o, 1, nullptr, d, d, d, d, nullptr) == VTX_EINVAL);
  vtx_opts bad = o;
  bad.nquad = 30;
  EXPECT(vtx_rates_backward(&g, &bad, 1, d, d, d, d, d, d, d, d, nullptr) == VTX_EINVAL);
  bad = o;
  bad.processes = 8;
  EXPECT(vtx_rates_jacobian(&g, &bad, 1, d, d, nullptr, nullptr, nullptr, d, nullptr) == VTX_EINVAL);
  bad = o;
  bad.eta_fp64 = NAN;
  EXPECT(vtx_rates_forward_backward(&g, &bad, 1, d, d, d, d, d, d, d, d, d, d, nullptr) == VTX_EINVAL);
  vtx_grid g0{0, eps.data(), wv.data()};
  EXPECT(vtx_rates_forward(&g0, &o, 1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  std::vector<double> eps_bad(eps);
  eps_bad[3] = eps_bad[2];
  vtx_grid gb{ne, eps_bad.data(), wv.data()};
  const int rc_unsorted = vtx_rates_forward(&gb, &o, 1, d, d, d, d, d, nullptr);
  EXPECT(rc_unsorted == VTX_EINVAL || rc_unsorted == VTX_EDEVICE);
  EXPECT(vtx_rates_forward_mass(&g, &o, -1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_rates_forward_mass(&g, &o, 1, d, nullptr, d, d, d, nullptr) == VTX_EINVAL);
  bad = o;
  bad.precision = VTX_MIXED;
  EXPECT(vtx_rates_forward_mass(&g, &bad, 1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  bad = o;
  bad.rule = VTX_RULE_LAGUERRE;
  EXPECT(vtx_rates_forward_mass(&g, &bad, 1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  // valid arguments stop at the device check (no GPU here)
  const int rc = vtx_rates_forward(&g, &o, 1, d, d, d, d, d, nullptr);
  EXPECT(rc == VTX_EDEVICE || rc == VTX_EHIP);
  EXPECT(vtx_task_values(ne, VTX_NES | VTX_PAIR) == 4 * 231 + 2 * 441);
  EXPECT(vtx_task_values(0, 1) == 0);
  vtx_lattice lat{1, 4, 0.0, 0.1, 0.0, 0.25};
  EXPECT(vtx_rates_forward_interp(&g, &o, &lat, d, 8, 1, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_system(0, 1, 1, 1.0, d, d, d, d, d, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_system(4, 1, 1, -1.0, d, d, d, d, d, d, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_system(4, 0, 1, 1.0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                        nullptr, nullptr, nullptr) == VTX_OK);
  EXPECT(vtx_ray_solve(141, 1, 1, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_solve(4, 1, 0, d, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_solve(4, 1, 1, nullptr, d, d, d, nullptr) == VTX_EINVAL);
  EXPECT(vtx_ray_max_block() == 140);
  for (int code = -1; code < 6; ++code) EXPECT(vtx_strerror(code) != nullptr);
  EXPECT(vtx_abi_version() == VTX_ABI_VERSION);
  vtx_release();
  std::printf("host layer ok, %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
