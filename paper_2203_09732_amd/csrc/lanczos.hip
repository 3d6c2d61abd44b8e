// Shift-invert Lanczos (Sec. II, Alg. 1) with MINRES inner solves, the
// sigma = (E_min + E_max)/2 helper (Sec. IV A), the twist overlap
// (Sec. III, App. B) and explicit eigen-residuals, on gfx950.
//
// The Lanczos basis V stays in HBM (n x (mmax+1) FP64, column-major): only
// alpha_k, beta_{k+1} and a few norms cross to the host per step. Full
// reorthogonalisation against the earlier basis vectors is two passes of
// classical Gram-Schmidt, each a tall-skinny V^T w (tiles of 8 columns per
// workgroup, w read once per tile) followed by w -= V c.
#include "mbl_internal.h"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <mutex>
#include <numeric>

namespace mbl {

constexpr int kTile = 8;   // columns per CGS / Ritz tile
constexpr int kLanczosGrid = 512;

__device__ __forceinline__ double wsum_l(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partials[g * k + c] = sum over this workgroup's rows of V[i, c] * w[i],
// for the tile of columns c in [8 * blockIdx.y, 8 * blockIdx.y + 8) and c < k.
__global__ __launch_bounds__(kWG) void k_multidot(int64_t n, const double* __restrict__ V,
                                                  int64_t ld, int k, const double* __restrict__ w,
                                                  double* __restrict__ partials) {
  __shared__ double red[kWavesPerWG][kTile];
  const int c0 = blockIdx.y * kTile;
  const int nc = min(kTile, k - c0);
  double acc[kTile];
#pragma unroll
  for (int t = 0; t < kTile; ++t) acc[t] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
#pragma unroll
    for (int t = 0; t < kTile; ++t)
      if (t < nc) acc[t] += V[(size_t)(c0 + t) * ld + i] * wi;
  }
#pragma unroll
  for (int t = 0; t < kTile; ++t) acc[t] = wsum_l(acc[t]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int t = 0; t < kTile; ++t) red[threadIdx.x >> 6][t] = acc[t];
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    double s = 0.0;
    for (int wv = 0; wv < kWavesPerWG; ++wv) s += red[wv][threadIdx.x];
    partials[(size_t)blockIdx.x * k + c0 + threadIdx.x] = s;
  }
}

// w[i] -= sum_{c < k} V[i, c] coef[c]
__global__ __launch_bounds__(kWG) void k_cgs_update(int64_t n, const double* __restrict__ V,
                                                    int64_t ld, int k,
                                                    const double* __restrict__ coef,
                                                    double* __restrict__ w) {
  extern __shared__ double sc[];
  for (int c = threadIdx.x; c < k; c += blockDim.x) sc[c] = coef[c];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += V[(size_t)c * ld + i] * sc[c];
    w[i] -= s;
  }
}

// U[i, t] = sum_{c < k} V[i, c] Y[c, t] for the tile t in [8 by, 8 by + 8), t < nev
__global__ __launch_bounds__(kWG) void k_ritz(int64_t n, const double* __restrict__ V, int64_t ld,
                                              int k, const double* __restrict__ Y, int nev,
                                              double* __restrict__ U, int64_t ldu) {
  extern __shared__ double sy[];   // k x kTile
  const int t0 = blockIdx.y * kTile;
  const int nt = min(kTile, nev - t0);
  for (int e = threadIdx.x; e < k * kTile; e += blockDim.x) {
    const int c = e / kTile, t = e % kTile;
    sy[e] = (t < nt) ? Y[(size_t)(t0 + t) * k + c] : 0.0;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[kTile];
#pragma unroll
    for (int t = 0; t < kTile; ++t) acc[t] = 0.0;
    for (int c = 0; c < k; ++c) {
      const double v = V[(size_t)c * ld + i];
#pragma unroll
      for (int t = 0; t < kTile; ++t) acc[t] += v * sy[c * kTile + t];
    }
#pragma unroll
    for (int t = 0; t < kTile; ++t)
      if (t < nt) U[(size_t)(t0 + t) * ldu + i] = acc[t];
  }
}

static int lgrid(int64_t n) {
  int64_t g = (n + kWG - 1) / kWG;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kLanczosGrid));
}

// ---------------------------------------------------------------------------
// host symmetric tridiagonal eigensolver: the symmetric QR algorithm of
// Golub & Van Loan (Matrix Computations, Sec. 8.3, the implicit symmetric QR
// step with Wilkinson shift, Alg. 8.3.2, inside the deflating driver of
// Alg. 8.3.3). Off-diagonal entries below eps (|d_i| + |d_{i+1}|) are set to
// zero; the trailing unreduced block [lo, hi] gets one implicit QR step: the
// Wilkinson shift mu from its trailing 2 x 2 block, a Givens rotation in the
// plane (lo, lo+1) chosen from the first column of T - mu I, and the bulge it
// creates chased down to hi by further rotations. The rotations are
// accumulated into the eigenvector matrix. alpha[0..k-1] diagonal,
// beta[0..k-2] off-diagonal. evals ascending, evecs k x k column-major
// (column i belongs to evals[i]); with evecs NULL only the eigenvalues are
// formed. Returns 0 on success, -1 if a block needed more than 60 QR steps
// per eigenvalue.
int tridiag_eig(int k, const double* alpha, const double* beta, double* evals, double* evecs) {
  const bool vec = evecs != nullptr;
  const double eps = 2.220446049250313e-16;
  std::vector<double> d(alpha, alpha + k), e(k > 1 ? k - 1 : 1, 0.0),
      Z(vec ? (size_t)k * k : 0, 0.0);
  for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
  if (vec)
    for (int i = 0; i < k; ++i) Z[(size_t)i * k + i] = 1.0;
  int hi = k - 1, steps = 0;
  while (hi > 0) {
    // deflation: negligible couplings become exact zeros
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])) ||
          std::fabs(e[i]) <= 1e-300)
        e[i] = 0.0;
    while (hi > 0 && e[hi - 1] == 0.0) {   // d[hi] has converged
      --hi;
      steps = 0;
    }
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++steps > 60) return -1;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer d[hi]
    const double half = 0.5 * (d[hi - 1] - d[hi]), bh = e[hi - 1];
    const double root = std::hypot(half, bh);
    const double mu = d[hi] - bh * (bh / (half + (half >= 0.0 ? root : -root)));
    // the first rotation from the first column of T - mu I, then the bulge
    // (x, z) = (T[j][j-1], T[j+1][j-1]) chased to the bottom of the block
    double x = d[lo] - mu, z = e[lo];
    for (int j = lo; j < hi; ++j) {
      const double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = z / r;
      }
      if (j > lo) e[j - 1] = r;
      // T <- G^T T G in the plane (j, j+1), G = [[c, -s], [s, c]]
      const double a = d[j], bb = e[j], cc = d[j + 1];
      const double cs = c * s;
      d[j] = c * c * a + 2.0 * cs * bb + s * s * cc;
      d[j + 1] = s * s * a - 2.0 * cs * bb + c * c * cc;
      e[j] = cs * (cc - a) + (c * c - s * s) * bb;
      if (j + 1 < hi) {
        z = s * e[j + 1];      // the new bulge at (j + 2, j)
        e[j + 1] *= c;
        x = e[j];
      }
      if (vec) {
        double* zj = &Z[(size_t)j * k];
        double* zj1 = &Z[(size_t)(j + 1) * k];
        for (int row = 0; row < k; ++row) {
          const double t0 = zj[row], t1 = zj1[row];
          zj[row] = c * t0 + s * t1;
          zj1[row] = c * t1 - s * t0;
        }
      }
    }
  }
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int i = 0; i < k; ++i) {
    evals[i] = d[order[i]];
    if (vec)
      std::copy(&Z[(size_t)order[i] * k], &Z[(size_t)order[i] * k] + k, &evecs[(size_t)i * k]);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// host-side helpers with a workspace

mbl_status reduce_to_host(mbl_workspace_s* ws, const double* partials, int nparts, int stride,
                          int nvals, double* out_host, hipStream_t s) {
  MBL_HIP(launch_reduce(partials, nparts, stride, nvals, ws->red_out, s));
  MBL_HIP(hipMemcpyAsync(ws->h_red, ws->red_out, sizeof(double) * nvals, hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  std::copy(ws->h_red, ws->h_red + nvals, out_host);
  return MBL_OK;
}

static mbl_status dot_ws(mbl_workspace_s* ws, int64_t n, const double* x, const double* y,
                         double* out, hipStream_t s) {
  int np = 0;
  MBL_HIP(launch_dot(n, x, y, ws->partials1, &np, s));
  return reduce_to_host(ws, ws->partials1, np, 1, 1, out, s);
}

// coef[0..k) = V_k^T w on the device (ws->coef)
static mbl_status multidot(mbl_workspace_s* ws, int64_t n, const double* V, int64_t ld, int k,
                           const double* w, hipStream_t s) {
  const int G = lgrid(n);
  hipLaunchKernelGGL(k_multidot, dim3(G, (k + kTile - 1) / kTile), dim3(kWG), 0, s, n, V, ld, k,
                     w, ws->partials2);
  MBL_HIP(hipGetLastError());
  MBL_HIP(launch_reduce(ws->partials2, G, k, k, ws->coef, s));
  return MBL_OK;
}

static mbl_status cgs_pass(mbl_workspace_s* ws, int64_t n, const double* V, int64_t ld, int k,
                           double* w, hipStream_t s) {
  MBL_TRY(multidot(ws, n, V, ld, k, w, s));
  hipLaunchKernelGGL(k_cgs_update, dim3(lgrid(n)), dim3(kWG), sizeof(double) * k, s, n, V, ld, k,
                     ws->coef, w);
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

// ||(H - shift) v||_2
static mbl_status apply_norm(mbl_basis_s* b, mbl_workspace_s* ws, const double* h, double shift,
                             const double* v, double* tmp, double* out, hipStream_t s) {
  const FieldArgs F = make_fields(b, h, shift);
  int np = 0;
  MBL_HIP(launch_apply<double>(b, F, v, tmp, 2, ws->partials1, &np, s));
  double ss = 0;
  MBL_TRY(reduce_to_host(ws, ws->partials1, np, 1, 1, &ss, s));
  *out = std::sqrt(ss);
  return MBL_OK;
}

double gershgorin_bound(const mbl_basis_s* b, const double* h) {
  double sh = 0.0;
  for (int j = 0; j < b->L; ++j) sh += std::fabs(h[j]);
  return 0.25 * b->L + 0.5 * sh + 0.5 * b->L;
}

// ---------------------------------------------------------------------------
mbl_status si_lanczos_run(mbl_basis_s* b, const double* h, double sigma, int nev, int mmax,
                          double minres_tol, int64_t minres_kmax, double eig_tol, double gap_tol,
                          double escale, const double* v0, uint64_t seed, int precision,
                          int precond, mbl_workspace_s* ws, double* evals, double* evecs,
                          int64_t ldu, double* resid, mbl_si_info* info, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t n = b->n;
  const int64_t ld = n;
  double* V = ws->V;
  if (escale <= 0) escale = gershgorin_bound(b, h);

  // v_1 = v / ||v||
  if (v0)
    MBL_HIP(hipMemcpyAsync(V, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  else
    MBL_HIP(launch_splitmix(n, seed, V, s));
  double nv = 0;
  MBL_TRY(dot_ws(ws, n, V, V, &nv, s));
  nv = std::sqrt(nv);
  if (!(nv > 0) || !std::isfinite(nv)) {
    set_error("start vector has zero or non-finite norm");
    return MBL_ERR_ARG;
  }
  MBL_HIP(launch_scale_copy(n, 1.0 / nv, V, V, s));

  std::vector<double> alphas, betas;   // betas[k-1] = beta_{k+1}
  std::vector<double> theta, Y;
  std::vector<int> sel;
  int64_t total_iters = 0;
  // MBL_VERBOSE=1: one line per Lanczos step on stderr (long runs)
  const bool verbose = std::getenv("MBL_VERBOSE") != nullptr;
  bool breakdown = false, converged = false, minres_warn = false;
  int k = 0;
  double beta_k = 0.0;   // beta_k multiplying v_{k-1}; v_0 = 0
  for (k = 1; k <= mmax; ++k) {
    double* vk = V + (size_t)(k - 1) * ld;
    // x = (H - sigma)^{-1} v_k by MINRES from x0 = 0
    mbl_minres_info mi{};
    mbl_status st = minres_run(b, h, sigma, vk, ws->x, minres_tol, minres_kmax, precision,
                               precond, true, ws, &mi, s);
    if (st < 0) return st;
    if (st == MBL_WARN_NOCONV) minres_warn = true;
    total_iters += mi.iters;
    // w = x - beta_k v_{k-1}; alpha_k = v_k . w; w -= alpha_k v_k
    MBL_HIP(hipMemcpyAsync(ws->w, ws->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (k > 1) MBL_HIP(launch_axpby(n, -beta_k, V + (size_t)(k - 2) * ld, 1.0, ws->w, s));
    double alpha = 0;
    MBL_TRY(dot_ws(ws, n, vk, ws->w, &alpha, s));
    MBL_HIP(launch_axpby(n, -alpha, vk, 1.0, ws->w, s));
    // full reorthogonalisation: two classical Gram-Schmidt passes against v_1..v_k
    MBL_TRY(cgs_pass(ws, n, V, ld, k, ws->w, s));
    MBL_TRY(cgs_pass(ws, n, V, ld, k, ws->w, s));
    double bb = 0;
    MBL_TRY(dot_ws(ws, n, ws->w, ws->w, &bb, s));
    const double beta_next = std::sqrt(bb);
    alphas.push_back(alpha);
    betas.push_back(beta_next);
    if (!std::isfinite(alpha) || !std::isfinite(beta_next)) {
      set_error("non-finite Lanczos coefficient");
      return MBL_ERR_NUMERIC;
    }
    // Ritz values of T_k
    theta.assign(k, 0.0);
    Y.assign((size_t)k * k, 0.0);
    if (tridiag_eig(k, alphas.data(), betas.data(), theta.data(), Y.data()) != 0) {
      set_error("tridiagonal eigensolver did not converge");
      return MBL_ERR_NUMERIC;
    }
    double tmax = 0.0;
    for (double t : theta) tmax = std::max(tmax, std::fabs(t));
    breakdown = beta_next <= 1e-14 * tmax;
    // v_{k+1} = w / beta_{k+1}
    double* vn = V + (size_t)k * ld;
    if (!breakdown) MBL_HIP(launch_scale_copy(n, 1.0 / beta_next, ws->w, vn, s));
    if (k >= nev) {
      // the nev Ritz values of largest |theta| are the eigenvalues nearest sigma
      std::vector<int> idx(k);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int a, int c) { return std::fabs(theta[a]) > std::fabs(theta[c]); });
      sel.assign(idx.begin(), idx.begin() + nev);
      // ||H u - lambda u|| = |beta_{k+1} y_k / theta| * ||(H - sigma) v_{k+1}||
      double nav = 0.0;
      if (!breakdown) MBL_TRY(apply_norm(b, ws, h, sigma, vn, ws->t64, &nav, s));
      converged = true;
      for (int i : sel) {
        const double est = std::fabs(beta_next * Y[(size_t)i * k + (k - 1)] / theta[i]) * nav;
        const double lam = sigma + 1.0 / theta[i];
        double gap = INFINITY;
        for (int j = 0; j < k; ++j)
          if (j != i) gap = std::min(gap, std::fabs(sigma + 1.0 / theta[j] - lam));
        bool ok = est <= eig_tol * escale;
        if (gap_tol > 0) ok = ok && est <= gap_tol * gap;
        if (!ok) converged = false;
      }
    }
    if (verbose)
      std::fprintf(stderr, "[mbl] si_lanczos step %d: minres %lld iterations (total %lld), %s\n", k,
                   (long long)mi.iters, (long long)total_iters,
                   converged ? "converged" : (breakdown ? "breakdown" : "continuing"));
    if (converged || breakdown) break;
    beta_k = beta_next;
  }
  if (k > mmax) k = mmax;
  if ((int)sel.size() < nev) {
    set_error("Krylov space became invariant after " + std::to_string(k) +
              " steps, fewer than nev");
    return MBL_ERR_NUMERIC;
  }
  // order the selected pairs by eigenvalue
  std::vector<double> lam(nev);
  std::sort(sel.begin(), sel.end(), [&](int a, int c) {
    return sigma + 1.0 / theta[a] < sigma + 1.0 / theta[c];
  });
  std::vector<double> Ysel((size_t)k * nev);
  for (int t = 0; t < nev; ++t) {
    lam[t] = sigma + 1.0 / theta[sel[t]];
    std::copy(&Y[(size_t)sel[t] * k], &Y[(size_t)sel[t] * k] + k, &Ysel[(size_t)t * k]);
  }
  MBL_HIP(hipMemcpyAsync(ws->ycoef, Ysel.data(), sizeof(double) * Ysel.size(),
                         hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_ritz, dim3(lgrid(n), (nev + kTile - 1) / kTile), dim3(kWG),
                     sizeof(double) * k * kTile, s, n, V, ld, k, ws->ycoef, nev, evecs, ldu);
  MBL_HIP(hipGetLastError());
  // normalise, then explicit residuals in FP64
  int nconv = 0;
  double maxrel = 0.0;
  for (int t = 0; t < nev; ++t) {
    double* u = evecs + (size_t)t * ldu;
    double nn = 0;
    MBL_TRY(dot_ws(ws, n, u, u, &nn, s));
    MBL_HIP(launch_scale_copy(n, 1.0 / std::sqrt(nn), u, u, s));
    double r = 0;
    MBL_TRY(apply_norm(b, ws, h, lam[t], u, ws->t64, &r, s));
    evals[t] = lam[t];
    if (resid) resid[t] = r;
    maxrel = std::max(maxrel, r / escale);
    if (r <= eig_tol * escale) ++nconv;
  }
  MBL_HIP(hipStreamSynchronize(s));
  if (info) {
    info->steps = k;
    info->nconv = nconv;
    info->minres_iters = total_iters;
    info->max_rel_resid = maxrel;
    info->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (nconv < nev) {
    if (breakdown) return MBL_WARN_BREAKDOWN;
    set_error(minres_warn ? "eigenpairs not converged (MINRES hit kmax)"
                          : "eigenpairs not converged within mmax steps");
    return MBL_WARN_NOCONV;
  }
  return MBL_OK;
}

// ---------------------------------------------------------------------------
// sigma = (E_min + E_max) / 2: Lanczos on H without reorthogonalisation
// (extremal Ritz values converge first and are unaffected by the copies that
// loss of orthogonality creates); three n-vectors.
mbl_status sigma_midpoint_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* h,
                              double rel_tol, int mmax, double* emin, double* emax,
                              hipStream_t s) {
  const int64_t n = b->n;
  double *v_prev = ws->r64, *v = ws->t64, *w = ws->w;
  MBL_HIP(launch_splitmix(n, 0x5eed5eedULL, v, s));
  double nv = 0;
  MBL_TRY(dot_ws(ws, n, v, v, &nv, s));
  MBL_HIP(launch_scale_copy(n, 1.0 / std::sqrt(nv), v, v, s));
  MBL_HIP(launch_fill(n, 0.0, v_prev, s));
  const FieldArgs F = make_fields(b, h, 0.0);
  std::vector<double> al, be, th, Y;
  double beta = 0.0;
  double lo = 0, hi = 0;
  bool conv = false;
  for (int k = 1; k <= mmax; ++k) {
    MBL_HIP(launch_apply<double>(b, F, v, w, 0, nullptr, nullptr, s));
    if (k > 1) MBL_HIP(launch_axpby(n, -beta, v_prev, 1.0, w, s));
    double a = 0;
    MBL_TRY(dot_ws(ws, n, v, w, &a, s));
    MBL_HIP(launch_axpby(n, -a, v, 1.0, w, s));
    double bb = 0;
    MBL_TRY(dot_ws(ws, n, w, w, &bb, s));
    const double bn = std::sqrt(bb);
    al.push_back(a);
    be.push_back(bn);
    th.assign(k, 0.0);
    Y.assign((size_t)k * k, 0.0);
    if (tridiag_eig(k, al.data(), be.data(), th.data(), Y.data()) != 0) {
      set_error("tridiagonal eigensolver did not converge");
      return MBL_ERR_NUMERIC;
    }
    lo = th[0];
    hi = th[k - 1];
    const double sc = std::max(std::fabs(lo), std::fabs(hi));
    const double r_lo = std::fabs(bn * Y[(size_t)0 * k + (k - 1)]);
    const double r_hi = std::fabs(bn * Y[(size_t)(k - 1) * k + (k - 1)]);
    if (k >= 4 && r_lo <= rel_tol * sc && r_hi <= rel_tol * sc) {
      conv = true;
      break;
    }
    if (bn <= 1e-14 * sc) {
      conv = true;
      break;
    }
    // v_prev <- v, v <- w / bn
    std::swap(v_prev, v);
    MBL_HIP(launch_scale_copy(n, 1.0 / bn, w, v, s));
    beta = bn;
  }
  *emin = lo;
  *emax = hi;
  return conv ? MBL_OK : MBL_WARN_NOCONV;
}

// ---------------------------------------------------------------------------
mbl_status twist_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* psi, int64_t ld,
                     int nvec, double* z, hipStream_t s) {
  const int L = b->L;
  std::vector<double> ct(2 * L), st(2 * L);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < 2 * L; ++m) {
    ct[m] = std::cos(pi * m / L);
    st[m] = std::sin(pi * m / L);
  }
  int done = 0;
  while (done < nvec) {
    const int nb = std::min(nvec - done, 32);
    int G = 0;
    MBL_HIP(launch_twist(b, psi + (size_t)done * ld, ld, nb, ct.data(), st.data(), ws->partials2,
                         &G, s));
    // out[t * 2 + v] = sum_g partials[(t * G + g) * 2 + v]
    std::vector<double> out(2 * nb);
    for (int t = 0; t < nb; ++t)
      MBL_TRY(reduce_to_host(ws, ws->partials2 + (size_t)t * G * 2, G, 2, 2, &out[2 * t], s));
    std::copy(out.begin(), out.end(), z + 2 * done);
    done += nb;
  }
  return MBL_OK;
}

mbl_status eig_residual_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* h,
                            const double* E, const double* psi, int64_t ld, int nvec,
                            double* resid, hipStream_t s) {
  for (int t = 0; t < nvec; ++t)
    MBL_TRY(apply_norm(b, ws, h, E[t], psi + (size_t)t * ld, ws->t64, &resid[t], s));
  return MBL_OK;
}

}  // namespace mbl
