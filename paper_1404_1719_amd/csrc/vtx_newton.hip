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
// Schur complement M_r = D_r - diag(lo_r) M_{r-1}^{-1} diag(up_{r-1}) is built in registers and
// inverted there by Gauss-Jordan elimination with partial pivoting (FP64), M_r^{-1} overwrites D_r
// for the back substitution x_r = y_r + M_r^{-1} (up_r x_{r+1}). The blocks are small dense
// inversions with pivoting, one after another along the ray: FP64 vector arithmetic, the block
// held in the registers of a 1024-lane workgroup, pivot columns exchanged through LDS and pivot
// rows read across lanes.
#include <hip/hip_runtime.h>

#include "../../include/vtx_rates.h"
#include "vtx_internal.h"

namespace vtx {
namespace {

constexpr int kNBlock = 256;
constexpr int kSysCols = (6 * kMaxNE + 63) / 64;   // columns per lane of a zone's block

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
  // rows go to waves, columns to consecutive lanes: reads of J along j and writes of D along col
  // coalesce; a lane's columns and a wave's row are decomposed into (species, moment, bin) once
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int cs[kSysCols], cm[kSysCols], cj[kSysCols];
#pragma unroll
  for (int u = 0; u < kSysCols; ++u) {
    const int col = lane + 64 * u;
    cs[u] = col / (2 * ne);
    cm[u] = (col / ne) & 1;
    cj[u] = col % ne;
  }
  for (int row = wave; row < nb; row += nw) {
    const int s = row / (2 * ne), m = (row / ne) & 1, i = row % ne, sp = partner_of(s);
    const double f0 = sf[(2 * s) * ne + i], f1 = sf[(2 * s + 1) * ne + i];
    const double x0 = sc[(2 * s) * ne + i], x1 = sc[(2 * s + 1) * ne + i];
    const double diag = c0 + lo[z * nb + row] + up[z * nb + row];
    double* Drow = Dz + (int64_t)row * nb;
#pragma unroll
    for (int u = 0; u < kSysCols; ++u) {
      const int col = lane + 64 * u;
      if (col >= nb) continue;
      const int s2 = cs[u], m2 = cm[u], j = cj[u];
      double dS = 0.0;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (s2 != (p == 0 ? s : sp)) continue;
        const double* Jp = J + ((s * 2 + p) * 4) * n2 + i * ne + j;   // [o][i][j] of (s, p)
        if (m == 0)
          dS += m2 == 0 ? Jp[0] - f0 * Jp[n2] : -3.0 * f1 * Jp[3 * n2];
        else
          dS += m2 == 0 ? -f1 * Jp[n2] : Jp[2 * n2] - f0 * Jp[3 * n2];
      }
      double d = -dS;
      if (s2 == s && j == i) {
        d += m == 0 ? (m2 == 0 ? x0 : 3.0 * x1) : (m2 == 0 ? x1 : x0);
        if (m2 == m) d += diag;
      }
      Drow[col] = d;
    }
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

// Block elimination along a ray (one ray per 1024-lane workgroup). The Schur complement
// M_r = D_r - diag(lo_r) M_{r-1}^{-1} diag(up_{r-1}) lives in registers: lane l of wave w holds
// the entries (i, j) with i = l + 64 h (h < ROWS, ROWS = ceil(nb / 64)) and j = 9 w + c (c < 9),
// so wave w holds the block's 9-column panel w whole and a row is spread over one lane of every
// wave. Entries outside the nb x nb block are zeros and stay zeros, so no step needs a bounds
// test on them. The block is inverted in place by Gauss-Jordan elimination with partial
// pivoting done implicitly: step k takes, among the rows not yet used, the one with the largest
// |M[i][k]| (the lowest index on ties) and eliminates column k from every other row, without
// moving any row. That is the in-place elimination of P M (P the pivot order, row k of P M = row
// pi(k) of M), so the registers end with Z[pi(a)][j] = ((P M)^-1)[a][j] = M^-1[a][pi(j)]: entry
// (i, j) of Z is M^-1[pi^-1(i)][pi(j)].
//
// The steps go by panels: the wave holding panel q runs its 9 steps alone (pivot search by DPP
// and readlane, pivot row by readlane, no barrier between them) and publishes the factored panel
// G in LDS; one barrier; every other wave then applies the 9 steps at once. The 9 steps act on a
// column x as x + U x[pivots] (they only mix in the pivot rows), and the factored panel holds
// G[i][t] = delta(i, p_t) + U[i][t], so the other columns take x'[i] = (i a pivot row ? 0 :
// x[i]) + sum_t G[i][t] x[p_t]. A wave reads its own pivot rows x[p_t] through a small LDS area
// of its own. The wave of the next panel applies the current one first. The inverse is staged
// in LDS in its own order (the panels' buffers share that space while the block is in
// registers), copied to D_r for the back substitution and used for the next zone's Schur
// complement and for y_r.
constexpr int kSolveBlock = 1024, kSolveWaves = kSolveBlock / 64;
constexpr int kPanel = 9;     // columns per wave (a multiple of 3: the update reads them in threes)
constexpr int kMaxNb = 140;   // nb^2 + 3 nb doubles of LDS and the pivot maps within 160 KiB
static_assert(kMaxNb <= kPanel * kSolveWaves, "the waves' panels cover the largest block");
constexpr int kFormRows = 3;   // rows per wave whose loads are in flight while forming the block

// LDS doubles the panels need inside the block's space: two factored panels (alternate
// panels) and each wave's 9 x 9 pivot rows.
constexpr int panel_space(int rows) { return 2 * kPanel * 64 * rows + kSolveWaves * kPanel * kPanel; }

// out[i] = sum_j A[i][j] w[j] + add[i] for an nb x nb row-major A (LDS or global): wave w takes
// rows w, w + 16, ...; its lanes split j and sum by shuffles. The loads of all its rows are issued
// before their sums, so a global A costs one memory latency, not one per row.
constexpr int kMatvecRows = (kMaxNb + kSolveWaves - 1) / kSolveWaves;   // rows per wave
constexpr int kMatvecCols = (kMaxNb + 63) / 64;                         // entries per lane and row
__device__ __forceinline__ void matvec(const double* A, const double* w, const double* add, double* out, int nb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s[kMatvecRows];
#pragma unroll
  for (int t = 0; t < kMatvecRows; ++t) {
    const int i = wave + kSolveWaves * t;
    s[t] = 0.0;
#pragma unroll
    for (int u = 0; u < kMatvecCols; ++u) {
      const int j = lane + 64 * u;
      if (i < nb && j < nb) s[t] = __builtin_fma(A[(int64_t)i * nb + j], w[j], s[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < kMatvecRows; ++t) {
    const int i = wave + kSolveWaves * t;
    const double r = wave_sum64(s[t]);
    if (lane == 0 && i < nb) out[i] = r + add[i];
  }
}

// The rows of A that matvec gives this lane (wave w: rows w, w + 16, ...), loaded ahead of
// their use; and the product from them.
template <int COLS>
__device__ __forceinline__ void matvec_load(const double* A, int nb, double (&m)[kMatvecRows][COLS]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < kMatvecRows; ++t) {
    const int i = wave + kSolveWaves * t;
#pragma unroll
    for (int u = 0; u < COLS; ++u) {
      const int j = lane + 64 * u;
      m[t][u] = (i < nb && j < nb) ? A[(int64_t)i * nb + j] : 0.0;
    }
  }
}
template <int COLS>
__device__ __forceinline__ void matvec_partial(const double (&m)[kMatvecRows][COLS], const double* w, int nb,
                                               double (&s)[kMatvecRows]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kMatvecRows; ++t) {
    s[t] = 0.0;
#pragma unroll
    for (int u = 0; u < COLS; ++u) {
      const int j = lane + 64 * u;
      if (j < nb) s[t] = __builtin_fma(m[t][u], w[j], s[t]);
    }
  }
}
__device__ __forceinline__ void matvec_finish(double (&s)[kMatvecRows], const double* add, double* out, int nb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < kMatvecRows; ++t) {
    const int i = wave + kSolveWaves * t;
    const double r = wave_sum64(s[t]);
    if (lane == 0 && i < nb) out[i] = r + add[i];
  }
}

// The value of a double in lane src of the wave (uniform).
__device__ __forceinline__ double read_lane(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The pivot search's order: a larger key first, on equal keys the lower row.
__device__ __forceinline__ void pivot_better(double& key, int& row, double okey, int orow) {
  const bool take = okey > key || (okey == key && orow < row);
  key = take ? okey : key;
  row = take ? orow : row;
}

// v from another lane of the same row of 16 (DPP, no memory access): CTRL is a quad permutation
// or a rotation within the row, so every source lane exists.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ void pivot_dpp(double& key, int& row) {
  pivot_better(key, row, dpp_double<CTRL>(key), __builtin_amdgcn_update_dpp(0, row, CTRL, 0xf, 0xf, false));
}

// The best (key, row) over the wave, uniform: within each row of 16 lanes by DPP (lane order
// xor 1, xor 2, then rotations by 4 and 8), then over the four rows' results.
__device__ __forceinline__ int wave_pivot(double key, int row) {
  constexpr int kXor1 = 0xb1, kXor2 = 0x4e, kRor4 = 0x124, kRor8 = 0x128;
  pivot_dpp<kXor1>(key, row);
  pivot_dpp<kXor2>(key, row);
  pivot_dpp<kRor4>(key, row);
  pivot_dpp<kRor8>(key, row);
  double bk = read_lane(key, 0);
  int br = __builtin_amdgcn_readlane(row, 0);
#pragma unroll
  for (int q = 16; q < 64; q += 16) pivot_better(bk, br, read_lane(key, q), __builtin_amdgcn_readlane(row, q));
  return __builtin_amdgcn_readfirstlane(br);
}

// The same pivot, first by the keys' upper 32 bits: for keys >= 0 they order as the keys do,
// up to ties. Where one lane alone holds the largest upper word, its (key, row) is the best
// (each lane's pair is already its own best); otherwise the full comparison decides.
__device__ __forceinline__ int wave_pivot_fast(double key, int row) {
  const long long b = __builtin_bit_cast(long long, key);
  const unsigned int hi = key >= 0.0 ? (unsigned int)(b >> 32) : 0u;
  constexpr int kXor1 = 0xb1, kXor2 = 0x4e, kRor4 = 0x124, kRor8 = 0x128;
  unsigned int m = hi;
  m = max(m, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)m, kXor1, 0xf, 0xf, false));
  m = max(m, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)m, kXor2, 0xf, 0xf, false));
  m = max(m, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)m, kRor4, 0xf, 0xf, false));
  m = max(m, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)m, kRor8, 0xf, 0xf, false));
  unsigned int top = (unsigned int)__builtin_amdgcn_readlane((int)m, 0);
#pragma unroll
  for (int q = 16; q < 64; q += 16) top = max(top, (unsigned int)__builtin_amdgcn_readlane((int)m, q));
  const unsigned long long at = __ballot(hi == top);
  if (__popcll(at) == 1) return __builtin_amdgcn_readlane(row, __ffsll((long long)at) - 1);
  return wave_pivot(key, row);
}

// The wave holding panel q runs the panel's steps k = 9 q + s on its columns and publishes the
// factored panel: G[s][i] (row i = lane + 64 h) into g_out, the pivots into piv and step.
template <int ROWS>
__device__ __forceinline__ void panel_factor(double (&a)[ROWS][kPanel], int q, int nb, int lane, double* g_out,
                                             int* piv, int* step) {
  bool used[ROWS];
#pragma unroll
  for (int h = 0; h < ROWS; ++h) {
    const int i = lane + 64 * h;
    used[h] = i >= nb || step[i] >= 0;
  }
#pragma unroll
  for (int s = 0; s < kPanel; ++s) {
    const int k = kPanel * q + s;
    if (k >= nb) break;
    // the unused row of largest |M[i][k]|, the lowest index on ties (NaN counts as largest)
    double best = -1.0;
    int bi = nb;
#pragma unroll
    for (int h = 0; h < ROWS; ++h)
      if (!used[h]) {
        const double ax = fabs(a[h][s]);
        pivot_better(best, bi, ax == ax ? ax : INFINITY, lane + 64 * h);
      }
    const int p = wave_pivot_fast(best, bi);
    const int hp = p >> 6, lp = p & 63;
    double rw[kPanel];
    if (ROWS == 1 || hp == 0) {
#pragma unroll
      for (int c = 0; c < kPanel; ++c) rw[c] = read_lane(a[0][c], lp);
    } else if (ROWS == 2 || hp == 1) {
#pragma unroll
      for (int c = 0; c < kPanel; ++c) rw[c] = read_lane(a[ROWS > 1 ? 1 : 0][c], lp);
    } else {
#pragma unroll
      for (int c = 0; c < kPanel; ++c) rw[c] = read_lane(a[ROWS - 1][c], lp);
    }
    const double pinv = 1.0 / rw[s];
    // factors f_i / pivot; row p becomes the pivot row times 1/pivot (zeroed, factor -1/pivot),
    // column k becomes -f_i / pivot and 1/pivot in row p (zeroed, the pivot row's entry taken as 1)
    double g[ROWS];
#pragma unroll
    for (int h = 0; h < ROWS; ++h) g[h] = a[h][s] * pinv;
    if (lane == lp) {
#pragma unroll
      for (int h = 0; h < ROWS; ++h)
        if (h == hp) {
          g[h] = -pinv;
          used[h] = true;
#pragma unroll
          for (int c = 0; c < kPanel; ++c) a[h][c] = 0.0;
        }
    }
    rw[s] = 1.0;
#pragma unroll
    for (int h = 0; h < ROWS; ++h) a[h][s] = 0.0;
#pragma unroll
    for (int h = 0; h < ROWS; ++h)
#pragma unroll
      for (int c = 0; c < kPanel; ++c) a[h][c] = __builtin_fma(-g[h], rw[c], a[h][c]);
    if (lane == 0) {
      piv[k] = p;
      step[p] = k;
    }
  }
#pragma unroll
  for (int s = 0; s < kPanel; ++s)
#pragma unroll
    for (int h = 0; h < ROWS; ++h) g_out[s * 64 * ROWS + lane + 64 * h] = a[h][s];
}

// Another wave applies panel q's steps to its columns: x'[i] = (i a pivot row of the panel ? 0 :
// x[i]) + sum_t G[t][i] x[p_t]. cw: the wave's own 9 x 9 area, x[p_t] on its columns.
template <int ROWS>
__device__ __forceinline__ void panel_apply(double (&a)[ROWS][kPanel], int q, int nb, int lane, const double* g_in,
                                            double* cw, const int* step) {
  const int k0 = kPanel * q;
  const int ns = nb - k0 < kPanel ? nb - k0 : kPanel;
  double keep[ROWS];
#pragma unroll
  for (int h = 0; h < ROWS; ++h) {
    const int i = lane + 64 * h;
    const int t = i < nb ? step[i] - k0 : -1;
    const bool pv = t >= 0 && t < ns;
    keep[h] = pv ? 0.0 : 1.0;
    if (pv) {
#pragma unroll
      for (int c = 0; c < kPanel; ++c) cw[t * kPanel + c] = a[h][c];
    }
  }
  // the pivot rows reach the whole wave through its own LDS area (in order within the wave)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int c = 0; c < kPanel; ++c) a[h][c] *= keep[h];
#pragma unroll
  for (int t = 0; t < kPanel; ++t) {
    if (t >= ns) break;
    double gt[ROWS];
#pragma unroll
    for (int h = 0; h < ROWS; ++h) gt[h] = g_in[t * 64 * ROWS + lane + 64 * h];
#pragma unroll
    for (int c0 = 0; c0 < kPanel; c0 += 3) {
      double x[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c] = cw[t * kPanel + c0 + c];
#pragma unroll
      for (int h = 0; h < ROWS; ++h)
#pragma unroll
        for (int c = 0; c < 3; ++c) a[h][c0 + c] = __builtin_fma(gt[h], x[c], a[h][c0 + c]);
    }
  }
  // the area is written again at the next panel, after this wave's reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// A workgroup barrier for LDS only: it waits for the wave's LDS operations, not for its global
// stores, which the elimination never reads back before its closing full barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int ROWS>
__global__ __launch_bounds__(kSolveBlock) void ray_solve_kernel(int nb, int64_t nrays, int nzr,
                                                                const double* __restrict__ lo,
                                                                double* __restrict__ D,
                                                                const double* __restrict__ up,
                                                                double* __restrict__ rhs) {
  const int64_t ray = blockIdx.x;
  if (ray >= nrays) return;
  extern __shared__ double sm[];
  __shared__ int piv[kMaxNb];    // piv[k]: the row pivoted at step k
  __shared__ int step[kMaxNb];   // step[i]: the step that pivoted row i, -1 while unused
  const int nb2 = nb * nb;
  const int space = nb2 > panel_space(ROWS) ? nb2 : panel_space(ROWS);
  double* Inv = sm;              // [nb][nb] the inverse of the zone's block, logical order
  double* gbuf = sm;             // while the block is in registers: 2 factored panels | pivot rows
  double* v = sm + space;        // right-hand side of the zone, then x of the zone above
  double* y = v + nb;            // y_r
  double* w = y + nb;            // zeros, then up_r x_{r+1} of the back substitution
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* cw = gbuf + 2 * kPanel * 64 * ROWS + wave * kPanel * kPanel;
  double* Dray = D + ray * nzr * (int64_t)nb2;
  double* bray = rhs + ray * nzr * (int64_t)nb;
  const double* lray = lo + ray * nzr * (int64_t)nb;
  const double* uray = up + ray * nzr * (int64_t)nb;
  const int npanels = (nb + kPanel - 1) / kPanel;
  double a[ROWS][kPanel];
  for (int r = 0; r < nzr; ++r) {
    double* Dr = Dray + (int64_t)r * nb2;
    const double* lr = lray + (int64_t)r * nb;
    const double* um = uray + (int64_t)(r - 1) * nb;
    // M_r, formed in LDS over M_{r-1}^{-1}: waves take rows, lanes columns (coalesced reads of D_r,
    // a wave's rows' loads issued before their first use). At three rows per lane, entry by entry,
    // with fewer registers: the elimination there needs every one.
    if constexpr (ROWS < 3) {
#pragma unroll 1
      for (int i0 = wave; i0 < nb; i0 += kSolveWaves * kFormRows) {
        double dv[kFormRows][ROWS];   // columns per lane: ceil(nb / 64), as rows
#pragma unroll
        for (int t = 0; t < kFormRows; ++t) {
          const int i = i0 + kSolveWaves * t;
#pragma unroll
          for (int u = 0; u < ROWS; ++u) {
            const int j = lane + 64 * u;
            dv[t][u] = (i < nb && j < nb) ? Dr[(int64_t)i * nb + j] : 0.0;
          }
        }
#pragma unroll
        for (int t = 0; t < kFormRows; ++t) {
          const int i = i0 + kSolveWaves * t;
          if (i >= nb) break;
          const double li = r > 0 ? lr[i] : 0.0;
#pragma unroll
          for (int u = 0; u < ROWS; ++u) {
            const int j = lane + 64 * u;
            if (j < nb) Inv[i * nb + j] = r > 0 ? dv[t][u] - li * Inv[i * nb + j] * um[j] : dv[t][u];
          }
        }
      }
    } else {
      for (int e = tid; e < nb2; e += blockDim.x) {
        double m = Dr[e];
        if (r > 0) {
          const int i = e / nb, j = e - i * nb;
          m -= lr[i] * Inv[e] * um[j];
        }
        Inv[e] = m;
      }
    }
    for (int i = tid; i < nb; i += blockDim.x) {
      v[i] = bray[(int64_t)r * nb + i] + (r > 0 ? lr[i] * y[i] : 0.0);
      w[i] = 0.0;
      step[i] = -1;
    }
    lds_barrier();
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      const int i = lane + 64 * h;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const int j = kPanel * wave + c;
        a[h][c] = (i < nb && j < nb) ? Inv[i * nb + j] : 0.0;
      }
    }
    lds_barrier();   // the panels' buffers take the block's space
    for (int q = 0; q < npanels; ++q) {
      if (q > 0 && wave != q - 1)
        panel_apply<ROWS>(a, q - 1, nb, lane, gbuf + ((q - 1) & 1) * kPanel * 64 * ROWS, cw, step);
      if (wave == q) panel_factor<ROWS>(a, q, nb, lane, gbuf + (q & 1) * kPanel * 64 * ROWS, piv, step);
      lds_barrier();
    }
    if (wave != npanels - 1)
      panel_apply<ROWS>(a, npanels - 1, nb, lane, gbuf + ((npanels - 1) & 1) * kPanel * 64 * ROWS, cw, step);
    lds_barrier();
    // Inv[a][b] = Z[pi(a)][pi^-1(b)]: entry (i, j) of the registers goes to Inv[step[i]][piv[j]]
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      const int i = lane + 64 * h;
      if (i >= nb) continue;
      const int ai = step[i];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const int j = kPanel * wave + c;
        if (j < nb) Inv[ai * nb + piv[j]] = a[h][c];
      }
    }
    lds_barrier();
    // y_r = M_r^{-1} v; M_r^{-1} replaces D_r for the back substitution, y_r the right-hand side
    for (int e = tid; e < nb2; e += blockDim.x) Dr[e] = Inv[e];
    matvec(Inv, v, w, y, nb);
    lds_barrier();
    for (int i = tid; i < nb; i += blockDim.x) bray[(int64_t)r * nb + i] = y[i];
    lds_barrier();
  }
  // back substitution: x_{N-1} = y_{N-1}; x_r = y_r + M_r^{-1} (up_r x_{r+1}); x kept in v
  for (int i = tid; i < nb; i += blockDim.x) v[i] = y[i];
  __syncthreads();   // also makes the sweep's writes of D and rhs visible to the whole workgroup
  // the rows of the next zone's M_r^{-1} are loaded while this zone's sums and barriers run
  // (at three rows per lane, zone by zone: the prefetch would spill the elimination's registers)
  constexpr int kPre = ROWS < 3 ? ROWS : 1;
  double mrow[kMatvecRows][kPre];
  if (ROWS < 3 && nzr > 1) matvec_load(Dray + (int64_t)(nzr - 2) * nb2, nb, mrow);
  for (int r = nzr - 2; r >= 0; --r) {
    const double* ur = uray + (int64_t)r * nb;
    for (int i = tid; i < nb; i += blockDim.x) {
      w[i] = ur[i] * v[i];
      y[i] = bray[(int64_t)r * nb + i];
    }
    lds_barrier();
    if constexpr (ROWS < 3) {
      double sums[kMatvecRows];
      matvec_partial(mrow, w, nb, sums);
      if (r > 0) matvec_load(Dray + (int64_t)(r - 1) * nb2, nb, mrow);
      matvec_finish(sums, y, v, nb);
    } else {
      matvec(Dray + (int64_t)r * nb2, w, y, v, nb);
    }
    lds_barrier();
    for (int i = tid; i < nb; i += blockDim.x) bray[(int64_t)r * nb + i] = v[i];
    lds_barrier();
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

template <int ROWS>
hipError_t launch_ray_solve_t(int nb, int64_t nrays, int nzr, const double* lo, double* D, const double* up,
                              double* rhs, hipStream_t s) {
  const size_t nb2 = (size_t)nb * nb, ps = (size_t)panel_space(ROWS);
  const size_t lds = sizeof(double) * ((nb2 > ps ? nb2 : ps) + 3 * (size_t)nb);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(ray_solve_kernel<ROWS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (int64_t r0 = 0; r0 < nrays; r0 += (int64_t(1) << 22)) {
    const int64_t n = nrays - r0 < (int64_t(1) << 22) ? nrays - r0 : (int64_t(1) << 22);
    const int64_t per = (int64_t)nzr * nb;
    hipLaunchKernelGGL(ray_solve_kernel<ROWS>, dim3((unsigned)n), dim3(kSolveBlock), lds, s, nb, n, nzr,
                       lo + r0 * per, D + r0 * per * nb, up + r0 * per, rhs + r0 * per);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Rows per lane: the fewest that cover the block (nb <= kMaxNb, checked by the caller).
hipError_t launch_ray_solve(int nb, int64_t nrays, int nzr, const double* lo, double* D, const double* up,
                            double* rhs, hipStream_t s) {
  static_assert(kMaxNb <= 3 * 64, "three rows per lane cover the largest block");
  if (nb <= 64) return launch_ray_solve_t<1>(nb, nrays, nzr, lo, D, up, rhs, s);
  if (nb <= 128) return launch_ray_solve_t<2>(nb, nrays, nzr, lo, D, up, rhs, s);
  return launch_ray_solve_t<3>(nb, nrays, nzr, lo, D, up, rhs, s);
}

}  // namespace vtx
