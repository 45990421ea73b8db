// HIP kernels for gfx950: one Newton step of an implicit radial sweep along rays.
//
// The paper's radial transport sweep is implicit, ray by ray (BDF2 in time), solved by
// Newton-Raphson with an explicitly built Jacobian and a direct solution of the linearised
// system (Sect. 2.1, radial sweep). The system here is a minimal stated one that consumes the
// interaction rates: per ray zone r the unknowns F_r are the 6 ne values f[species][moment][bin],
//   G_r = (3/2 F_r - 2 F_r^n + 1/2 F_r^{n-1}) / dt + (lo_r + up_r) F_r - lo_r F_{r-1} - up_r F_{r+1} - S_r,
//   S0 = eta0 - chi0 f0 - 3 chi1 f1,  S1 = eta1 - chi1 f0 - chi0 f1,
// (componentwise products; F_{-1} = F_N = 0). Its Jacobian is block tridiagonal with dense
// diagonal blocks D_r = (3/(2 dt)) I + diag(lo_r + up_r) - dS_r/dF_r, dS from the rates' explicit
// blocks, and diagonal neighbours -diag(lo_r), -diag(up_r).
//
// ray_system_kernel assembles D_r and -G_r (one zone per workgroup; HBM-write bound, like the
// Jacobian blocks). ray_solve_kernel eliminates along each ray (one ray per workgroup): the
// Schur complement M_r = D_r - diag(lo_r) M_{r-1}^{-1} diag(up_{r-1}) is built in LDS and inverted
// there by Gauss-Jordan elimination with partial pivoting (FP64), M_r^{-1} overwrites D_r for
// the back substitution x_r = y_r + M_r^{-1} (up_r x_{r+1}). The blocks are small dense
// inversions with pivoting, one after another along the ray: FP64 vector arithmetic in LDS.
#include <hip/hip_runtime.h>

#include "../../include/vtx_rates.h"
#include "vtx_internal.h"

namespace vtx {
namespace {

constexpr int kNBlock = 256;

__device__ __forceinline__ int partner_of(int s) { return s == 2 ? 2 : 1 - s; }

// D_r and rhs_r = -G_r of zone z (ray z / nzr, radial index z % nzr). Entry (row, col) with
// row = (s, m, i), col = (s2, m2, j): the rates' blocks jac[s][p][o][i][j] act on f_{o/2} of
// species s (p = 0, scattering) or of its partner (p = 1, pair).
__global__ __launch_bounds__(kNBlock) void ray_system_kernel(int ne, int64_t nz, int nzr, double dt,
                                                             const double* __restrict__ jac,
                                                             const double* __restrict__ f,
                                                             const double* __restrict__ f_n,
                                                             const double* __restrict__ f_nm1,
                                                             const double* __restrict__ eta,
                                                             const double* __restrict__ chi,
                                                             const double* __restrict__ lo,
                                                             const double* __restrict__ up, double* __restrict__ D,
                                                             double* __restrict__ rhs) {
  const int64_t z = blockIdx.x;
  if (z >= nz) return;
  const int nb = 6 * ne, n2 = ne * ne;
  const int r = (int)(z % nzr);
  extern __shared__ double sm[];
  double* sf = sm;            // f, eta, chi of the zone [3][2][ne] each
  double* se = sf + nb;
  double* sc = se + nb;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    sf[k] = f[z * nb + k];
    se[k] = eta[z * nb + k];
    sc[k] = chi[z * nb + k];
  }
  __syncthreads();
  const double* J = jac + z * (int64_t)(24 * n2);
  const double c0 = 1.5 / dt;
  double* Dz = D + z * (int64_t)nb * nb;
  // columns run over consecutive lanes: reads of J along j and writes of D along col coalesce
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int row = e / nb, col = e - row * nb;
    const int s = row / (2 * ne), m = (row / ne) & 1, i = row % ne;
    const int s2 = col / (2 * ne), m2 = (col / ne) & 1, j = col % ne;
    const double f0 = sf[(2 * s) * ne + i], f1 = sf[(2 * s + 1) * ne + i];
    double dS = 0.0;
    for (int p = 0; p < 2; ++p) {
      if (s2 != (p == 0 ? s : partner_of(s))) continue;
      const double* Jp = J + ((s * 2 + p) * 4) * n2 + i * ne + j;   // [o][i][j] of (s, p)
      if (m == 0)
        dS += m2 == 0 ? Jp[0] - f0 * Jp[n2] : -3.0 * f1 * Jp[3 * n2];
      else
        dS += m2 == 0 ? -f1 * Jp[n2] : Jp[2 * n2] - f0 * Jp[3 * n2];
    }
    double d = -dS;
    if (s2 == s && j == i) {
      const double x0 = sc[(2 * s) * ne + i], x1 = sc[(2 * s + 1) * ne + i];
      d += m == 0 ? (m2 == 0 ? x0 : 3.0 * x1) : (m2 == 0 ? x1 : x0);
      if (m2 == m) d += c0 + lo[z * nb + row] + up[z * nb + row];
    }
    Dz[e] = d;
  }
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    const int s = k / (2 * ne), m = (k / ne) & 1, i = k % ne;
    const double f0 = sf[(2 * s) * ne + i], f1 = sf[(2 * s + 1) * ne + i];
    const double x0 = sc[(2 * s) * ne + i], x1 = sc[(2 * s + 1) * ne + i];
    const double S = m == 0 ? se[k] - x0 * f0 - 3.0 * x1 * f1 : se[k] - x1 * f0 - x0 * f1;
    const double F = sf[k], l = lo[z * nb + k], u = up[z * nb + k];
    double G = (1.5 * F - 2.0 * f_n[z * nb + k] + 0.5 * f_nm1[z * nb + k]) / dt + (l + u) * F - S;
    if (r > 0) G -= l * f[(z - 1) * nb + k];
    if (r < nzr - 1) G -= u * f[(z + 1) * nb + k];
    rhs[z * nb + k] = -G;
  }
}

// Sum over the 64 lanes of a wave.
__device__ __forceinline__ double wave_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// In-place inverse of the nb x nb matrix M (row-major, LDS) by Gauss-Jordan elimination with
// partial (row) pivoting: column k takes the row of largest |M[i][k]|, i >= k (the first on ties);
// the row swaps are undone on the columns of the result at the end. col: nb doubles of LDS.
__device__ void invert_in_lds(double* M, int nb, double* col, int* perm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = 0; k < nb; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i < nb; i += 64) {
        const double a = fabs(M[i * nb + k]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) perm[k] = bi;
    }
    __syncthreads();
    const int p = perm[k];
    if (p != k) {   // uniform
      for (int j = tid; j < nb; j += blockDim.x) {
        const double t = M[k * nb + j];
        M[k * nb + j] = M[p * nb + j];
        M[p * nb + j] = t;
      }
      __syncthreads();
    }
    const double pinv = 1.0 / M[k * nb + k];
    __syncthreads();   // every lane has read the pivot before row k changes
    for (int t = tid; t < 2 * nb; t += blockDim.x) {
      if (t < nb) {
        if (t != k) col[t] = M[t * nb + k];
      } else {
        const int j = t - nb;
        M[k * nb + j] = (j == k ? 1.0 : M[k * nb + j]) * pinv;
      }
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e - i * nb;
      if (i != k) M[e] = (j == k ? 0.0 : M[e]) - col[i] * M[k * nb + j];
    }
    __syncthreads();
  }
  for (int k = nb - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {   // uniform
      for (int i = tid; i < nb; i += blockDim.x) {
        const double t = M[i * nb + k];
        M[i * nb + k] = M[i * nb + p];
        M[i * nb + p] = t;
      }
      __syncthreads();
    }
  }
}

// out[i] = sum_j A[i][j] w[j] + add[i] for an nb x nb row-major A (LDS or global): wave w takes
// rows w, w + 4, ...; its lanes split j and sum by shuffles.
__device__ __forceinline__ void matvec(const double* A, const double* w, const double* add, double* out, int nb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wave; i < nb; i += nw) {
    double s = 0.0;
    for (int j = lane; j < nb; j += 64) s += A[(int64_t)i * nb + j] * w[j];
    s = wave_sum64(s);
    if (lane == 0) out[i] = s + add[i];
  }
}

constexpr int kMaxNb = 140;   // nb^2 + 4 nb doubles and the pivot rows within the 160 KiB of LDS

__global__ __launch_bounds__(kNBlock) void ray_solve_kernel(int nb, int64_t nrays, int nzr,
                                                            const double* __restrict__ lo, double* __restrict__ D,
                                                            const double* __restrict__ up,
                                                            double* __restrict__ rhs) {
  const int64_t ray = blockIdx.x;
  if (ray >= nrays) return;
  extern __shared__ double sm[];
  __shared__ int perm[kMaxNb];
  const int nb2 = nb * nb;
  double* M = sm;          // [nb][nb]
  double* v = M + nb2;     // right-hand side of the zone, then x of the zone above
  double* y = v + nb;      // y_r
  double* w = y + nb;      // scaled vector of the back substitution
  double* col = w + nb;    // pivot column
  const int tid = threadIdx.x;
  double* Dray = D + ray * nzr * (int64_t)nb2;
  double* bray = rhs + ray * nzr * (int64_t)nb;
  const double* lray = lo + ray * nzr * (int64_t)nb;
  const double* uray = up + ray * nzr * (int64_t)nb;
  for (int r = 0; r < nzr; ++r) {
    double* Dr = Dray + (int64_t)r * nb2;
    const double* lr = lray + (int64_t)r * nb;
    const double* um = uray + (int64_t)(r - 1) * nb;
    // M holds M_{r-1}^{-1}: M_r = D_r - diag(lo_r) M_{r-1}^{-1} diag(up_{r-1}), in place
    for (int e = tid; e < nb2; e += blockDim.x) {
      const int i = e / nb, j = e - i * nb;
      double m = Dr[e];
      if (r > 0) m -= lr[i] * M[e] * um[j];
      M[e] = m;
    }
    for (int i = tid; i < nb; i += blockDim.x) v[i] = bray[(int64_t)r * nb + i] + (r > 0 ? lr[i] * y[i] : 0.0);
    __syncthreads();
    invert_in_lds(M, nb, col, perm);
    // y_r = M_r^{-1} v; M_r^{-1} replaces D_r for the back substitution, y_r the right-hand side
    for (int i = tid; i < nb; i += blockDim.x) w[i] = 0.0;
    __syncthreads();
    matvec(M, v, w, y, nb);
    for (int e = tid; e < nb2; e += blockDim.x) Dr[e] = M[e];
    __syncthreads();
    for (int i = tid; i < nb; i += blockDim.x) bray[(int64_t)r * nb + i] = y[i];
    __syncthreads();
  }
  // back substitution: x_{N-1} = y_{N-1}; x_r = y_r + M_r^{-1} (up_r x_{r+1}); x kept in v
  for (int i = tid; i < nb; i += blockDim.x) v[i] = y[i];
  __syncthreads();
  for (int r = nzr - 2; r >= 0; --r) {
    const double* ur = uray + (int64_t)r * nb;
    for (int i = tid; i < nb; i += blockDim.x) {
      w[i] = ur[i] * v[i];
      y[i] = bray[(int64_t)r * nb + i];
    }
    __syncthreads();
    matvec(Dray + (int64_t)r * nb2, w, y, v, nb);
    __syncthreads();
    for (int i = tid; i < nb; i += blockDim.x) bray[(int64_t)r * nb + i] = v[i];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_ray_system(int ne, int64_t nz, int nzr, double dt, const double* jac, const double* f,
                             const double* f_n, const double* f_nm1, const double* eta, const double* chi,
                             const double* lo, const double* up, double* D, double* rhs, hipStream_t s) {
  const size_t lds = sizeof(double) * 18 * ne;
  // slices of whole rays (a zone's radial index is its launch index modulo nzr), under 2^22
  // workgroups per dispatch
  const int64_t slice = ((int64_t(1) << 22) / nzr) * nzr;
  for (int64_t z0 = 0; z0 < nz; z0 += slice) {
    const int64_t n = nz - z0 < slice ? nz - z0 : slice;
    const int64_t nb = 6 * ne;
    hipLaunchKernelGGL(ray_system_kernel, dim3((unsigned)n), dim3(kNBlock), lds, s, ne, n, nzr, dt,
                       jac + z0 * 24 * ne * ne, f + z0 * nb, f_n + z0 * nb, f_nm1 + z0 * nb, eta + z0 * nb,
                       chi + z0 * nb, lo + z0 * nb, up + z0 * nb, D + z0 * nb * nb, rhs + z0 * nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int max_block() { return kMaxNb; }

hipError_t launch_ray_solve(int nb, int64_t nrays, int nzr, const double* lo, double* D, const double* up,
                            double* rhs, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)nb * nb + 4 * (size_t)nb);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(ray_solve_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (int64_t r0 = 0; r0 < nrays; r0 += (int64_t(1) << 22)) {
    const int64_t n = nrays - r0 < (int64_t(1) << 22) ? nrays - r0 : (int64_t(1) << 22);
    const int64_t per = (int64_t)nzr * nb;
    hipLaunchKernelGGL(ray_solve_kernel, dim3((unsigned)n), dim3(kNBlock), lds, s, nb, n, nzr, lo + r0 * per,
                       D + r0 * per * nb, up + r0 * per, rhs + r0 * per);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vtx
