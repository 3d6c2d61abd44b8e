// Derivatives of an eigenpair (E, psi) of Eq. (1) with respect to the fields
// h_j, through one linear solve with the same MINRES kernels.
//
// dH/dh_j = -S^z_j is diagonal with entries -s_j(a), s_j = bit_{j-1}(a) - 1/2.
// * Hellmann-Feynman: dE/dh_j = <psi| dH/dh_j |psi> = -sum_a c_a^2 s_j(a).
// * Twist overlap z = sum_a c_a^2 u_a (App. B): d|z|^2/dc_a = g_a =
//   4 c_a Re(conj(z) u_a). With P = I - psi psi^T and lambda the solution
//   orthogonal to psi of (H - E) lambda = P g (one MINRES solve, sigma = E),
//   d|z|^2/dh_j = -lambda^T (dH/dh_j) psi = sum_a lambda_a c_a s_j(a).
//   This is the adjoint of the L forward solves (H - E) x_j = -P dH/dh_j psi.
#include "rows.h"

#include <cmath>
#include <vector>

namespace mbl {

// partials[g * (L + 1) + j] = sum over rows of a_i b_i bit_j(state_i) (j < L),
// partials[g * (L + 1) + L] = sum of a_i b_i
__global__ __launch_bounds__(kWG) void k_site_sums(DevBasis B, const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldArgs F{};
  const RowTables t = setup_tables(B, F, smem);
  __shared__ double red[kWavesPerWG][kMaxL + 1];
  __syncthreads();
  double acc[kMaxL + 1];
#pragma unroll
  for (int j = 0; j <= kMaxL; ++j) acc[j] = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t st) {
    const double w = a[row] * b[row];
#pragma unroll
    for (int j = 0; j < kMaxL; ++j)
      if ((st >> j) & 1u) acc[j] += w;
    acc[kMaxL] += w;
  });
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j <= kMaxL; ++j) {
    double v = acc[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  const int L = B.L;
  if (threadIdx.x <= (unsigned)L) {
    const int j = (threadIdx.x == (unsigned)L) ? kMaxL : threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < kWavesPerWG; ++w) s += red[w][j];
    partials[(size_t)blockIdx.x * (L + 1) + threadIdx.x] = s;
  }
}

struct GradTab {
  double c[2 * kMaxL];
  double s[2 * kMaxL];
};

// g_a = 4 c_a (Re z cos(theta_a) + Im z sin(theta_a)), u_a = exp(i theta_a)
__global__ __launch_bounds__(kWG) void k_twist_grad(DevBasis B, GradTab T, double zre, double zim,
                                                    const double* __restrict__ psi,
                                                    double* __restrict__ g) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldArgs F{};
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  const int twoL = 2 * B.L, base = (B.L * (B.L + 1)) / 2;
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      uint32_t w = 0;
      for (int p = 0; p < 32; ++p)
        if (((p + 1) >> k) & 1) w |= (1u << p);
      sum += __popc(a & w) << k;
    }
    int m = (2 * sum - base) % twoL;
    if (m < 0) m += twoL;
    g[row] = 4.0 * psi[row] * (zre * T.c[m] + zim * T.s[m]);
  });
}

mbl_status twist_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* psi, int64_t ld,
                     int nvec, double* z, hipStream_t s);

static mbl_status site_sums(mbl_basis_s* b, mbl_workspace_s* ws, const double* a,
                            const double* c, std::vector<double>& out, hipStream_t s) {
  const int G = row_grid(b);
  const int L = b->L;
  hipLaunchKernelGGL(k_site_sums, dim3(G), dim3(kWG), row_lds_bytes(b), s, b->dev(), a, c,
                     ws->partials2);
  MBL_HIP(hipGetLastError());
  out.assign(L + 1, 0.0);
  return reduce_to_host(ws, ws->partials2, G, L + 1, L + 1, out.data(), s);
}

static mbl_status dot_h(mbl_workspace_s* ws, int64_t n, const double* x, const double* y,
                        double* out, hipStream_t s) {
  int np = 0;
  MBL_HIP(launch_dot(n, x, y, ws->partials1, &np, s));
  return reduce_to_host(ws, ws->partials1, np, 1, 1, out, s);
}

mbl_status eig_grad_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* h, double E,
                        const double* psi, double tol, int64_t kmax, int precond, double* dE,
                        double* dz2, double* zout, mbl_minres_info* info, hipStream_t s) {
  const int L = b->L;
  const int64_t n = b->n;
  // Hellmann-Feynman: dE/dh_j = -(sum c^2 b_j - (1/2) sum c^2)
  std::vector<double> sums;
  MBL_TRY(site_sums(b, ws, psi, psi, sums, s));
  const double norm2 = sums[L];
  for (int j = 0; j < L; ++j) dE[j] = -(sums[j] - 0.5 * norm2);
  // z and g = d|z|^2 / dc
  double z[2];
  MBL_TRY(twist_run(b, ws, psi, n, 1, z, s));
  if (zout) {
    zout[0] = z[0];
    zout[1] = z[1];
  }
  GradTab T{};
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < 2 * L; ++m) {
    T.c[m] = std::cos(pi * m / L);
    T.s[m] = std::sin(pi * m / L);
  }
  double* g = ws->w;
  double* lam = ws->x;
  hipLaunchKernelGGL(k_twist_grad, dim3(row_grid(b)), dim3(kWG), row_lds_bytes(b), s, b->dev(), T,
                     z[0], z[1], psi, g);
  MBL_HIP(hipGetLastError());
  // P g = g - psi (psi . g) / (psi . psi)
  double pg = 0;
  MBL_TRY(dot_h(ws, n, psi, g, &pg, s));
  MBL_HIP(launch_axpby(n, -pg / norm2, psi, 1.0, g, s));
  // (H - E + theta psi psi^T / |psi|^2) lambda = P g: the rank-one term lifts
  // the near-null direction psi of H - E (its rounding components would
  // otherwise be amplified by 1 / (E_true - E)) and leaves the solution for a
  // right-hand side orthogonal to psi unchanged; then lambda orthogonal to psi
  mbl_minres_info mi{};
  const mbl_status st = minres_run(b, h, E, g, lam, tol, kmax, MBL_FP64, precond, true, ws, &mi,
                                   s, psi, 1.0 / norm2);
  if (st < 0) return st;
  double pl = 0;
  MBL_TRY(dot_h(ws, n, psi, lam, &pl, s));
  MBL_HIP(launch_axpby(n, -pl / norm2, psi, 1.0, lam, s));
  // d|z|^2/dh_j = sum lambda c s_j = sum lambda c b_j - (1/2) sum lambda c
  MBL_TRY(site_sums(b, ws, lam, psi, sums, s));
  for (int j = 0; j < L; ++j) dz2[j] = sums[j] - 0.5 * sums[L];
  if (info) *info = mi;
  return st;
}

}  // namespace mbl

using namespace mbl;

extern "C" mbl_status mbl_eig_grad(mbl_basis b, const double* h_host, double E,
                                   const double* psi_dev, double tol, int64_t kmax, int precond,
                                   mbl_workspace ws, double* dE_dh_host, double* dz2_dh_host,
                                   double* z_host, mbl_minres_info* info, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && psi_dev && ws && dE_dh_host && dz2_dh_host, "NULL argument");
  MBL_ARG(ws->basis == b, "workspace belongs to another basis");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(E), "non-finite h or E");
  MBL_ARG(tol > 0 && kmax >= 1, "bad tol or kmax");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  return eig_grad_run(b, ws, h_host, E, psi_dev, tol, kmax, precond, dE_dh_host, dz2_dh_host,
                      z_host, info, reinterpret_cast<hipStream_t>(stream));
}
