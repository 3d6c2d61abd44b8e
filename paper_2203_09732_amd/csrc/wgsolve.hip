// Many disorder realizations of uneven chain length in one persistent launch:
// shift-invert Lanczos (Alg. 1) with preconditioned MINRES inner solves
// (Alg. 2), the Ritz extraction, explicit residuals and the twist overlap
// (Sec. III), all on the device, one realization per workgroup at a time.
//
// Workgroups claim problems from a device counter (atomicAdd) until the queue
// is empty, so every workgroup reaches the exit and the grid drains. A
// workgroup (8 waves) keeps every vector of its realization in its own slot
// of device memory and every scalar in registers or LDS; the reductions are
// workgroup reductions (LDS, fixed order), so there is no grid barrier and no
// host round trip between the steps. The launch serves L <= kWgMaxL = 16:
// there the MINRES vectors of all realizations in flight (256 x 10 x 103 KB
// at L = 16) about fill the last-level cache, so most gathers of a neighbour
// amplitude hit it. At L = 18 they are about 0.7 GB; a gather then fetches a
// whole line from HBM for one double, and a mixed set of 171 realizations
// had mostly not finished after 800 s, where a lockstep batch of 32 (whose
// interleaved layout turns each gather into 256 contiguous bytes) takes
// about 7 s of the whole chip per realization. Longer chains therefore go to
// the batched form inside the same call: 32 streaming lanes, each running its
// own realization's Lanczos steps (batched.hip). The solver is inlined into the
// kernel for each chain length (the problem's basis selects the instance), so
// every problem-wide value stays in scalar registers; it needs 229 VGPRs, so
// a workgroup is 512 threads and a CU runs one.
//
// Per realization:
//  1. sigma = (E_min + E_max) / 2 (Sec. IV A) unless given: Lanczos on H
//     without reorthogonalisation from a seeded start vector; every 8 steps
//     the extreme eigenvalues of T_j by Sturm bisection and their residual
//     estimates |beta_{j+1} y_j| by inverse iteration on T_j;
//  2. SI-Lanczos: x = (H - sigma)^{-1} v_k by MINRES from x0 = 0 (two row
//     passes per iteration: p = A q_k with the d/x update of iteration k - 1,
//     then z_{k+1}, q_{k+1}), three-term recurrence, two classical
//     Gram-Schmidt passes against v_1..v_k, the tridiagonal T_k
//     eigendecomposition by the symmetric QR algorithm (one wave), the
//     convergence test of the single-realization solver;
//  3. the Ritz vectors V_k y_i of the nev pairs nearest sigma, normalised,
//     their explicit residuals ||H u - lambda u|| and twist overlaps.
#include "rows.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

namespace mbl {

constexpr int kWgThreads = 512;     // 229 VGPRs: one workgroup of 8 waves per CU
constexpr int kWgWaves = kWgThreads / 64;
constexpr int kWgMaxNev = 32;
constexpr int kWgMaxM = 128;          // Lanczos steps per realization
constexpr int kWgSigmaSteps = 320;    // Lanczos steps of the sigma search
constexpr int kWgVecs = 8;            // MINRES vectors in a slot
constexpr int kWgMaxL = 16;           // longest chain of the persistent launch

struct WgProblem {
  double h[kMaxL];
  double sigma;       // NaN: the spectral midpoint is computed here
  double escale;      // > 0: energy scale of the stopping rule; else max(|E_min|, |E_max|)
  int L, basis, nev, mmax;
  double* evecs;      // n x nev column-major (ld = n), caller-owned device memory
};

struct WgResult {
  double evals[kWgMaxNev];
  double resid[kWgMaxNev];
  double z[2 * kWgMaxNev];
  double sigma, emin, emax, escale;
  int64_t minres_iters;
  int32_t steps, nconv, status, minres_noconv;
};

struct WgPhase {
  double c[2 * kMaxL];
  double s[2 * kMaxL];
};

struct WgParams {
  const WgProblem* probs;
  WgResult* results;
  const DevBasis* bases;
  const WgPhase* phases;    // per basis
  double* slots;
  int64_t slot_stride;      // doubles per workgroup slot
  int64_t vs;               // doubles per n-vector inside a slot (>= max n)
  unsigned int* counter;
  unsigned int* done;       // host-mapped, one per workgroup: realizations it finished
  int nprob;
  int precond;
  double minres_tol, eig_tol, gap_tol, sigma_rel_tol;
  int64_t minres_kmax;
  uint64_t seed;
};

// ---------------------------------------------------------------------------
// workgroup reductions: every thread gets the sum, fixed order
__device__ __forceinline__ double wg_sum(double v, double* red) { return block_sum_all(v, red); }

// eight sums at once; red8: [kWgWaves][8]
__device__ __forceinline__ void wg_sum8(double (&v)[8], double* red8) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = wave_sum(v[j]);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) red8[wave * 8 + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double s = 0.0;
    for (int w = 0; w < kWgWaves; ++w) s += red8[w * 8 + j];
    v[j] = s;
  }
  __syncthreads();
}

// SplitMix64 (Steele, Lea & Flood 2014) of seed + (i + 1) * golden gamma,
// top 53 bits mapped to [-1/2, 1/2): the seeded start vectors of the library.
__device__ __forceinline__ double wg_splitmix(uint64_t seed, int64_t i) {
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal eigenproblems on one wave (wave 0 calls these). All 64
// lanes run the same scalar recurrence and every lane writes the shared
// arrays itself (the same values): a lane never reads a value another lane
// wrote without a barrier between them. The eigenvector rows are split over
// the lanes.

// Number of eigenvalues of T (d, e, size k) below x (Sturm sequence count).
__device__ __forceinline__ int sturm_count(const double* d, const double* e, int k, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    const double qq = q != 0.0 ? q : 1e-300;
    q = d[i] - x - e[i - 1] * e[i - 1] / qq;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// The idx-th smallest eigenvalue of T by bisection on [lo, hi].
__device__ double sturm_eigenvalue(const double* d, const double* e, int k, int idx, double lo,
                                   double hi) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, k, mid) > idx) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for the eigenvalue lam: two
// steps of inverse iteration (tridiagonal elimination with partial pivoting);
// y and scratch in work[0 .. 5k).
__device__ double last_component(const double* d, const double* e, int k, double lam,
                                 double* work) {
  double* y = work;
  double* a = work + k;       // sub-diagonal
  double* b = work + 2 * k;   // diagonal
  double* c = work + 3 * k;   // super-diagonal
  double* f = work + 4 * k;   // second super-diagonal after pivoting
  for (int i = 0; i < k; ++i) y[i] = 1.0;
  const double shift_eps = 1e-300;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = 0; i < k; ++i) {
      b[i] = d[i] - lam;
      a[i] = i > 0 ? e[i - 1] : 0.0;
      c[i] = i + 1 < k ? e[i] : 0.0;
      f[i] = 0.0;
    }
    // forward elimination with row interchanges
    for (int i = 0; i + 1 < k; ++i) {
      if (fabs(a[i + 1]) > fabs(b[i])) {
        // swap rows i and i + 1
        double t = b[i]; b[i] = a[i + 1]; a[i + 1] = t;
        t = c[i]; c[i] = b[i + 1]; b[i + 1] = t;
        t = f[i]; f[i] = c[i + 1]; c[i + 1] = t;
        t = y[i]; y[i] = y[i + 1]; y[i + 1] = t;
      }
      const double piv = b[i] != 0.0 ? b[i] : shift_eps;
      const double m = a[i + 1] / piv;
      b[i + 1] -= m * c[i];
      c[i + 1] -= m * f[i];
      y[i + 1] -= m * y[i];
    }
    // back substitution
    for (int i = k - 1; i >= 0; --i) {
      double s = y[i];
      if (i + 1 < k) s -= c[i] * y[i + 1];
      if (i + 2 < k) s -= f[i] * y[i + 2];
      y[i] = s / (b[i] != 0.0 ? b[i] : shift_eps);
    }
    double nn = 0.0;
    for (int i = 0; i < k; ++i) nn += y[i] * y[i];
    nn = sqrt(nn);
    for (int i = 0; i < k; ++i) y[i] /= nn;
  }
  return fabs(y[k - 1]);
}

// Eigendecomposition of T (d, e in LDS, size k) by the symmetric QR algorithm
// (Golub & Van Loan Sec. 8.3: implicit steps with Wilkinson shift, bulge
// chasing, deflation from the bottom), rotations accumulated into Z (k x k,
// column-major, global memory, column i the eigenvector of d[i] on return).
// d and e are overwritten (d: the eigenvalues, unsorted). Returns 0, or -1
// if a block needs more than 60 steps per eigenvalue. Wave 0 only.
__device__ int wave_tridiag_qr(double* d, double* e, int k, double* Z) {
  const int lane = threadIdx.x & 63;
  for (int col = 0; col < k; ++col)
    for (int row = lane; row < k; row += 64) Z[(size_t)col * k + row] = row == col ? 1.0 : 0.0;
  const double eps = 2.220446049250313e-16;
  int hi = k - 1, steps = 0;
  while (hi > 0) {
    for (int i = 0; i < hi; ++i) {
      const double ei = e[i];
      if (fabs(ei) <= eps * (fabs(d[i]) + fabs(d[i + 1])) || fabs(ei) <= 1e-300) e[i] = 0.0;
    }
    while (hi > 0 && e[hi - 1] == 0.0) {
      --hi;
      steps = 0;
    }
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++steps > 60) return -1;
    const double half = 0.5 * (d[hi - 1] - d[hi]), bh = e[hi - 1];
    const double root = hypot(half, bh);
    const double mu = d[hi] - bh * (bh / (half + (half >= 0.0 ? root : -root)));
    double x = d[lo] - mu, zb = e[lo];
    for (int j = lo; j < hi; ++j) {
      const double r = hypot(x, zb);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = zb / r;
      }
      const double a = d[j], bb = e[j], cc = d[j + 1];
      const double cs = c * s;
      const double dj = c * c * a + 2.0 * cs * bb + s * s * cc;
      const double dj1 = s * s * a - 2.0 * cs * bb + c * c * cc;
      const double ej = cs * (cc - a) + (c * c - s * s) * bb;
      double ej1 = 0.0;
      if (j + 1 < hi) {
        ej1 = e[j + 1];
        zb = s * ej1;
        ej1 *= c;
        x = ej;
      }
      if (j > lo) e[j - 1] = r;
      d[j] = dj;
      d[j + 1] = dj1;
      e[j] = ej;
      if (j + 1 < hi) e[j + 1] = ej1;
      double* zj = Z + (size_t)j * k;
      double* zj1 = Z + (size_t)(j + 1) * k;
      for (int row = lane; row < k; row += 64) {
        const double t0 = zj[row], t1 = zj1[row];
        zj[row] = c * t0 + s * t1;
        zj1[row] = c * t1 - s * t0;
      }
    }
  }
  return 0;
}

// a_aa - sigma (c0 = L/4 + sum h / 2 - sigma) and N_anti of state a, the
// diagonal of the row kernels written for a runtime c0
template <int L>
__device__ __forceinline__ double wg_diag(const DevBasis& B, const RowTables& t, double c0,
                                          uint32_t a, int& nanti) {
  const int LL = L ? L : B.L;
  const uint32_t mask = (LL == 32) ? 0xffffffffu : ((1u << LL) - 1u);
  nanti = __popc(a ^ (((a << 1) | (a >> (LL - 1))) & mask));
  double f = 0.0;
  if constexpr (L > 0) {
    constexpr int NNIB = (L + 3) >> 2;
    double fv[NNIB];
#pragma unroll
    for (int k = 0; k < NNIB; ++k) fv[k] = t.lut[(k << 4) + ((a >> (4 * k)) & 15u)];
#pragma unroll
    for (int k = 0; k < NNIB; ++k) f += fv[k];
  } else {
    const int nnib = (B.L + 3) >> 2;
    for (int k = 0; k < nnib; ++k) f += t.lut[(k << 4) + ((a >> (4 * k)) & 15u)];
  }
  return c0 - 0.5 * (double)nanti - f;
}

// ---------------------------------------------------------------------------
// One realization on one workgroup.
struct WgShared {
  double alpha[kWgMaxM + kWgSigmaSteps];
  double beta[kWgMaxM + kWgSigmaSteps];
  double d[kWgSigmaSteps];
  double e[kWgSigmaSteps];
  double coef[kWgMaxM + 8];
  double red8[kWgWaves * 8];
  double work[5 * kWgSigmaSteps];
  int sel[kWgMaxNev];
  FieldArgs F;
  int pid;
  int flag;
};

template <int L, int NLO>
__device__ __attribute__((always_inline)) void wg_solve(const WgParams& P, const WgProblem& pr, WgResult& res, double* slot,
                         WgShared& S, unsigned char* smem) {
  const DevBasis B = P.bases[pr.basis];
  const int64_t n = B.n;
  const int tid = threadIdx.x;
  const uint32_t wave = threadIdx.x >> 6;
  const int64_t vs = P.vs;
  double* qv[2] = {slot, slot + vs};
  double* zv[2] = {slot + 2 * vs, slot + 3 * vs};
  double* pv = slot + 4 * vs;
  double* dv[2] = {slot + 5 * vs, slot + 6 * vs};
  double* xv = slot + 7 * vs;
  double* V = slot + kWgVecs * vs;                 // (mmax + 1) columns
  double* Z = V + (size_t)(pr.mmax + 1) * vs;      // mmax x mmax
  double* Ysel = Z + (size_t)kWgMaxM * kWgMaxM;    // mmax x nev
  const int nev = pr.nev, mmax = pr.mmax;

  // fields into LDS, then the row tables
  if (tid < kMaxL) S.F.h[tid] = tid < pr.L ? pr.h[tid] : 0.0;
  __syncthreads();
  if (tid == 0) {
    double sh = 0.0;
    for (int j = 0; j < pr.L; ++j) sh += S.F.h[j];
    S.F.c0 = 0.25 * pr.L + 0.5 * sh;
    S.F.sigma = 0.0;
  }
  __syncthreads();
  const RowTables t = setup_tables<L>(B, S.F, smem);
  __syncthreads();
  const double c0_h = S.F.c0;   // shift 0

  auto dense = [&](auto f) {
    for (int64_t i = tid; i < n; i += kWgThreads) f(i);
  };
  auto rows = [&](auto f) { for_rows_range(B, t, wave, kWgWaves, f); };
  // ||(H - shift) v||^2 over the rows
  auto apply_norm2 = [&](const double* v, double c0) -> double {
    double acc = 0.0;
    rows([&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0, uint32_t a) {
      const double off = RowOps<double, L, NLO>::offdiag(B, t, v, hi, lo, j, block0);
      int na;
      const double dsh = wg_diag<L>(B, t, c0, a, na);
      const double y = dsh * v[row] + 0.5 * off;
      acc += y * y;
    });
    return wg_sum(acc, t.red);
  };

  // ---- 1. sigma ------------------------------------------------------------
  double sigma = pr.sigma, emin = NAN, emax = NAN;
  int status = 0;
  if (isnan(sigma)) {
    double* vp = qv[0];
    double* vc = qv[1];
    double* w = pv;
    double acc = 0.0;
    dense([&](int64_t i) {
      const double v = wg_splitmix(0x5eed5eedULL, i);
      vc[i] = v;
      vp[i] = 0.0;
      acc += v * v;
    });
    const double nv = sqrt(wg_sum(acc, t.red));
    dense([&](int64_t i) { vc[i] /= nv; });
    __syncthreads();
    double beta = 0.0;
    bool conv = false;
    int j = 0;
    for (j = 1; j <= kWgSigmaSteps; ++j) {
      // w = H v - beta v_prev; alpha = v . w
      double aw = 0.0;
      rows([&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t jj, uint32_t block0, uint32_t a) {
        const double off = RowOps<double, L, NLO>::offdiag(B, t, vc, hi, lo, jj, block0);
        int na;
        const double dg = wg_diag<L>(B, t, c0_h, a, na);
        const double y = dg * vc[row] + 0.5 * off - beta * vp[row];
        w[row] = y;
        aw += vc[row] * y;
      });
      const double alpha = wg_sum(aw, t.red);
      double ww = 0.0;
      dense([&](int64_t i) {
        const double y = w[i] - alpha * vc[i];
        w[i] = y;
        ww += y * y;
      });
      const double bn = sqrt(wg_sum(ww, t.red));
      if (tid == 0) {
        S.alpha[j - 1] = alpha;
        S.beta[j - 1] = bn;
      }
      __syncthreads();
      if (j >= 4 && (j % 8 == 0 || j == kWgSigmaSteps || !(bn > 0))) {
        // extremes of T_j by bisection, residual estimates by inverse iteration
        if (wave == 0) {
          double gl = INFINITY, gh = -INFINITY;
          for (int i = 0; i < j; ++i) {
            const double r = (i > 0 ? fabs(S.beta[i - 1]) : 0.0) + (i + 1 < j ? fabs(S.beta[i]) : 0.0);
            gl = fmin(gl, S.alpha[i] - r);
            gh = fmax(gh, S.alpha[i] + r);
          }
          const double lo_e = sturm_eigenvalue(S.alpha, S.beta, j, 0, gl, gh);
          const double hi_e = sturm_eigenvalue(S.alpha, S.beta, j, j - 1, gl, gh);
          const double sc = fmax(fabs(lo_e), fabs(hi_e));
          double r_lo = 0.0, r_hi = 0.0;
          if (bn > 1e-14 * sc) {
            r_lo = fabs(bn) * last_component(S.alpha, S.beta, j, lo_e, S.work);
            r_hi = fabs(bn) * last_component(S.alpha, S.beta, j, hi_e, S.work);
          }
          if ((threadIdx.x & 63) == 0) {
            S.d[0] = lo_e;
            S.d[1] = hi_e;
            S.flag = (r_lo <= P.sigma_rel_tol * sc && r_hi <= P.sigma_rel_tol * sc) ? 1 : 0;
          }
        }
        __syncthreads();
        emin = S.d[0];
        emax = S.d[1];
        conv = S.flag != 0;
        __syncthreads();
        if (conv) break;
      }
      if (!(bn > 0)) break;
      // v_prev <- v, v <- w / bn
      dense([&](int64_t i) {
        vp[i] = vc[i];
        vc[i] = w[i] / bn;
      });
      __syncthreads();
      beta = bn;
    }
    if (!conv) status = MBL_WARN_NOCONV;
    sigma = 0.5 * (emin + emax);
  }
  double escale = pr.escale;
  if (!(escale > 0)) {
    if (!isnan(emin)) {
      escale = fmax(fabs(emin), fabs(emax));
    } else {
      double sh = 0.0;
      for (int jj = 0; jj < pr.L; ++jj) sh += fabs(S.F.h[jj]);
      escale = 0.25 * pr.L + 0.5 * sh + 0.5 * pr.L;   // Gershgorin bound on ||H||
    }
  }
  const double c0 = c0_h - sigma;

  // ---- 2. shift-invert Lanczos --------------------------------------------
  {
    double acc = 0.0;
    dense([&](int64_t i) {
      const double v = wg_splitmix(P.seed, i);
      V[i] = v;
      acc += v * v;
    });
    const double nv = sqrt(wg_sum(acc, t.red));
    dense([&](int64_t i) { V[i] /= nv; });
    __syncthreads();
  }
  int64_t total_iters = 0;
  int minres_noconv = 0;
  int k = 0, ksel = 0;
  bool converged = false, breakdown = false, numeric = false;
  double beta_k = 0.0;
  const double tol = P.minres_tol;
  for (k = 1; k <= mmax; ++k) {
    const double* vk = V + (size_t)(k - 1) * vs;
    // -- MINRES for (H - sigma) x = v_k from x0 = 0 (Alg. 2)
    double qz = 0.0;
    rows([&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
      int na;
      const double dg = wg_diag<L>(B, t, c0, a, na);
      const double b = vk[row];
      const double q = b / precond_value(P.precond, dg, na);
      zv[0][row] = 0.0;    // z_0
      zv[1][row] = b;      // z_1
      qv[1][row] = q;      // q_1 (slot of odd k)
      dv[0][row] = 0.0;
      dv[1][row] = 0.0;
      xv[row] = 0.0;
      qz += q * b;
    });
    double beta = sqrt(wg_sum(qz, t.red));
    double beta_prev = 1.0, cc = 1.0, ss = 0.0, dhat = 0.0, eps = 0.0, phi = beta;
    // d/x coefficients of the previous iteration
    double co_ib = 0.0, co_de = 0.0, co_ep = 0.0, co_ig = 0.0, co_tau = 0.0;
    int64_t it = 0;
    bool bad = !isfinite(beta);
    while (!bad && fabs(phi) >= tol && it < P.minres_kmax) {
      ++it;
      double* qk = qv[it & 1];
      double* qo = qv[(it + 1) & 1];       // q_{k-1}, then q_{k+1}
      double* zk = zv[it & 1];
      double* zo = zv[(it + 1) & 1];       // z_{k-1}, then z_{k+1}
      double* dprev = dv[(it + 1) & 1];    // d_{k-2} slot receives d_{k-1}
      double* dprev2 = dv[it & 1];
      // pass 1: the d/x update of iteration k - 1, then p = A q_k and q_k . p
      const bool dx = it > 1;
      double qp = 0.0;
      rows([&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0, uint32_t a) {
        if (dx) {
          const double dd = (qo[row] * co_ib - co_de * dprev2[row] - co_ep * dprev[row]) * co_ig;
          dprev[row] = dd;
          xv[row] += co_tau * dd;
        }
        const double off = RowOps<double, L, NLO>::offdiag(B, t, qk, hi, lo, j, block0);
        int na;
        const double dg = wg_diag<L>(B, t, c0, a, na);
        const double pr_ = dg * qk[row] + 0.5 * off;
        pv[row] = pr_;
        qp += qk[row] * pr_;
      });
      const double alpha = wg_sum(qp, t.red) / (beta * beta);
      // pass 2: z_{k+1} (over z_{k-1}), q_{k+1} = M^{-1} z_{k+1} (over q_{k-1})
      const double c1 = 1.0 / beta, c2 = alpha / beta, c3 = beta / beta_prev;
      double qzn = 0.0;
      rows([&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
        const double zn = c1 * pv[row] - c2 * zk[row] - c3 * zo[row];
        int na;
        const double dg = wg_diag<L>(B, t, c0, a, na);
        const double qn = zn / precond_value(P.precond, dg, na);
        zo[row] = zn;
        qo[row] = qn;
        qzn += qn * zn;
      });
      const double beta_next = sqrt(wg_sum(qzn, t.red));
      // Givens step
      const double delta = cc * dhat + ss * alpha;
      const double gamma_hat = -ss * dhat + cc * alpha;
      const double eps_next = ss * beta_next;
      const double dhat_next = cc * beta_next;
      const double gamma = sqrt(gamma_hat * gamma_hat + beta_next * beta_next);
      const double cn = gamma_hat / gamma, sn = beta_next / gamma;
      co_ib = 1.0 / beta;
      co_de = delta;
      co_ep = eps;
      co_ig = 1.0 / gamma;
      co_tau = cn * phi;
      phi = -sn * phi;
      beta_prev = beta;
      beta = beta_next;
      cc = cn;
      ss = sn;
      dhat = dhat_next;
      eps = eps_next;
      bad = !isfinite(phi) || !isfinite(alpha) || !isfinite(beta_next);
    }
    if (it >= 1) {
      // the d/x update of the last iteration K: q_K in qv[K & 1], d_j in
      // dv[j & 1], so d_{K-1} in dv[(K + 1) & 1] and d_K over d_{K-2}
      const double* qK = qv[it & 1];
      const double* dKm1 = dv[(it + 1) & 1];
      double* dK = dv[it & 1];
      dense([&](int64_t i) {
        const double dd = (qK[i] * co_ib - co_de * dKm1[i] - co_ep * dK[i]) * co_ig;
        dK[i] = dd;
        xv[i] += co_tau * dd;
      });
      __syncthreads();
    }
    total_iters += it;
    if (bad) {
      numeric = true;
      break;
    }
    if (fabs(phi) >= tol) minres_noconv = 1;
    // -- w = x - beta_k v_{k-1}; alpha_k = v_k . w; w -= alpha_k v_k (w in p)
    double* w = pv;
    const double* vkm1 = k > 1 ? V + (size_t)(k - 2) * vs : nullptr;
    double aw = 0.0;
    dense([&](int64_t i) {
      const double y = xv[i] - (vkm1 ? beta_k * vkm1[i] : 0.0);
      w[i] = y;
      aw += vk[i] * y;
    });
    const double alpha = wg_sum(aw, t.red);
    dense([&](int64_t i) { w[i] -= alpha * vk[i]; });
    __syncthreads();
    // -- two classical Gram-Schmidt passes against v_1 .. v_k
    for (int pass = 0; pass < 2; ++pass) {
      for (int c0t = 0; c0t < k; c0t += 8) {
        double dots[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int nc = min(8, k - c0t);
        dense([&](int64_t i) {
          const double wi = w[i];
#pragma unroll
          for (int jj = 0; jj < 8; ++jj)
            if (jj < nc) dots[jj] += V[(size_t)(c0t + jj) * vs + i] * wi;
        });
        wg_sum8(dots, S.red8);
        if (tid == 0) {
#pragma unroll
          for (int jj = 0; jj < 8; ++jj)
            if (jj < nc) S.coef[c0t + jj] = dots[jj];
        }
      }
      __syncthreads();
      dense([&](int64_t i) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += V[(size_t)c * vs + i] * S.coef[c];
        w[i] -= s;
      });
      __syncthreads();
    }
    double bb = 0.0;
    dense([&](int64_t i) { bb += w[i] * w[i]; });
    const double beta_next = sqrt(wg_sum(bb, t.red));
    if (!isfinite(alpha) || !isfinite(beta_next)) {
      numeric = true;
      break;
    }
    if (tid == 0) {
      S.alpha[k - 1] = alpha;
      S.beta[k - 1] = beta_next;
    }
    __syncthreads();
    // -- eigendecomposition of T_k (wave 0)
    if (wave == 0) {
      for (int i = threadIdx.x; i < k; i += 64) {
        S.d[i] = S.alpha[i];
        S.e[i] = i + 1 < k ? S.beta[i] : 0.0;
      }
      // lanes read the arrays their wave wrote: LDS ops of a wave are in order
      const int qr = wave_tridiag_qr(S.d, S.e, k, Z);
      if ((threadIdx.x & 63) == 0) S.flag = qr;
    }
    __syncthreads();
    if (S.flag != 0) {
      numeric = true;
      break;
    }
    double tmax = 0.0;
    for (int i = 0; i < k; ++i) tmax = fmax(tmax, fabs(S.d[i]));
    breakdown = beta_next <= 1e-14 * tmax;
    double* vn = V + (size_t)k * vs;
    if (!breakdown) {
      dense([&](int64_t i) { vn[i] = w[i] / beta_next; });
      __syncthreads();
    }
    if (k >= nev) {
      // the nev Ritz values of largest |theta| (first index on ties)
      if (tid == 0) {
        for (int s = 0; s < nev; ++s) {
          int best = -1;
          for (int i = 0; i < k; ++i) {
            bool used = false;
            for (int u = 0; u < s; ++u) used = used || S.sel[u] == i;
            if (used) continue;
            if (best < 0 || fabs(S.d[i]) > fabs(S.d[best])) best = i;
          }
          S.sel[s] = best;
        }
      }
      __syncthreads();
      ksel = k;
      const double nav = breakdown ? 0.0 : sqrt(apply_norm2(vn, c0));
      bool conv = true;
      for (int s = 0; s < nev; ++s) {
        const int i = S.sel[s];
        const double th = S.d[i];
        const double est = fabs(beta_next * Z[(size_t)i * k + (k - 1)] / th) * nav;
        const double lam = sigma + 1.0 / th;
        double gap = INFINITY;
        for (int jj = 0; jj < k; ++jj)
          if (jj != i) gap = fmin(gap, fabs(sigma + 1.0 / S.d[jj] - lam));
        bool ok = est <= P.eig_tol * escale;
        if (P.gap_tol > 0) ok = ok && est <= P.gap_tol * gap;
        conv = conv && ok;
      }
      converged = conv;
    }
    if (converged || breakdown) break;
    beta_k = beta_next;
  }
  if (k > mmax) k = mmax;
  // ---- 3. Ritz vectors, residuals, twist ----------------------------------
  int nconv = 0;
  if (!numeric && ksel == k && k >= nev) {
    // selected pairs ordered by eigenvalue
    if (tid == 0) {
      for (int a = 1; a < nev; ++a)
        for (int b = a; b > 0; --b) {
          const double la = sigma + 1.0 / S.d[S.sel[b - 1]], lb = sigma + 1.0 / S.d[S.sel[b]];
          if (lb < la) {
            const int tmp = S.sel[b - 1];
            S.sel[b - 1] = S.sel[b];
            S.sel[b] = tmp;
          }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < k * nev; idx += kWgThreads) {
      const int tt = idx / k, c = idx % k;
      Ysel[(size_t)tt * k + c] = Z[(size_t)S.sel[tt] * k + c];
    }
    __syncthreads();
    double* U = pr.evecs;
    for (int tt = 0; tt < nev; ++tt) {
      double* u = U + (size_t)tt * n;
      const double* y = Ysel + (size_t)tt * k;
      double nn = 0.0;
      dense([&](int64_t i) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += V[(size_t)c * vs + i] * y[c];
        u[i] = s;
        nn += s * s;
      });
      const double inv = 1.0 / sqrt(wg_sum(nn, t.red));
      dense([&](int64_t i) { u[i] *= inv; });
      __syncthreads();
      const double lam = sigma + 1.0 / S.d[S.sel[tt]];
      const double r = sqrt(apply_norm2(u, c0_h - lam));
      // twist overlap: phase index m(a) = 2 sum_{set bits p} (p + 1) - L(L+1)/2 mod 2L
      const WgPhase& ph = P.phases[pr.basis];
      const int twoL = 2 * pr.L, base = (pr.L * (pr.L + 1)) / 2;
      double zr = 0.0, zi = 0.0;
      rows([&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
        int sum = 0;
        for (uint32_t m = a; m; m &= m - 1) sum += __ffs(m);
        int mm = (2 * sum - base) % twoL;
        if (mm < 0) mm += twoL;
        const double c2 = u[row] * u[row];
        zr += c2 * ph.c[mm];
        zi += c2 * ph.s[mm];
      });
      zr = wg_sum(zr, t.red);
      zi = wg_sum(zi, t.red);
      if (tid == 0) {
        res.evals[tt] = lam;
        res.resid[tt] = r;
        res.z[2 * tt] = zr;
        res.z[2 * tt + 1] = zi;
      }
      if (r <= P.eig_tol * escale) ++nconv;
    }
  }
  if (tid == 0) {
    res.sigma = sigma;
    res.emin = emin;
    res.emax = emax;
    res.escale = escale;
    res.minres_iters = total_iters;
    res.steps = k;
    res.nconv = nconv;
    res.minres_noconv = minres_noconv;
    if (numeric) status = MBL_ERR_NUMERIC;
    else if (ksel != k || k < nev) status = MBL_ERR_NUMERIC;   // invariant subspace below nev
    else if (nconv < nev) status = breakdown ? MBL_WARN_BREAKDOWN : MBL_WARN_NOCONV;
    res.status = status;
  }
  __syncthreads();
}

#define MBL_WG_SPLITS(X) X(12, 9) X(14, 10) X(16, 10)

__global__ __launch_bounds__(kWgThreads) void k_si_campaign(WgParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ WgShared S;
  double* slot = P.slots + (size_t)blockIdx.x * P.slot_stride;
  unsigned int finished = 0;
  for (;;) {
    if (threadIdx.x == 0) S.pid = (int)atomicAdd(P.counter, 1u);
    __syncthreads();
    const int pid = S.pid;
    __syncthreads();
    if (pid >= P.nprob) break;
    const WgProblem& pr = P.probs[pid];
    WgResult& res = P.results[pid];
    const DevBasis& B = P.bases[pr.basis];
    switch (B.L * 64 + B.nlo) {
#define MBL_CASE(LL, NN)                                       \
  case LL * 64 + NN:                                          \
    wg_solve<LL, NN>(P, pr, res, slot, S, smem);              \
    break;
      MBL_WG_SPLITS(MBL_CASE)
#undef MBL_CASE
      default:
        wg_solve<0, 0>(P, pr, res, slot, S, smem);
        break;
    }
    ++finished;
    if (threadIdx.x == 0 && P.done)   // a plain store to this workgroup's own slot
      __hip_atomic_store(P.done + blockIdx.x, finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void k_set_counter(unsigned int* p, unsigned int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// dst[t * n + i] = src[(t * n + i) * R + r]: realization r out of interleaved blocks
__global__ __launch_bounds__(kWG) void k_deinterleave(int64_t n, int R, int nev, int r,
                                                      const double* __restrict__ src,
                                                      double* __restrict__ dst) {
  const int64_t total = n * nev;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e * R + r];
}

// ===========================================================================
// host side

static int device_cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  return v;
}

// RAII for the device buffers of one call
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

static mbl_status alloc_dev(DevBuf& b, size_t bytes) {
  if (hipMalloc(&b.p, std::max<size_t>(bytes, 64)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
    return MBL_ERR_NOMEM;
  }
  return MBL_OK;
}

static uint64_t nchoosek(int n, int k) {
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

// Problems with L <= kWgMaxL: one persistent launch, one realization per
// workgroup, claimed from a device counter.
// Mean square field of a realization: the width of its spectrum grows with
// it, and the MINRES iterations per solve fall (a cost proxy for scheduling).
static double disorder_strength(const mbl_problem& pr) {
  double s2 = 0.0;
  for (int j = 0; j < pr.L; ++j) s2 += pr.h_host[j] * pr.h_host[j];
  return s2 / pr.L;
}

static mbl_status campaign_small(mbl_problem* probs, const std::vector<int>& idx,
                                 const std::vector<int>& mm, double minres_tol,
                                 int64_t minres_kmax, double eig_tol, double gap_tol,
                                 uint64_t seed, int precond, hipStream_t s) {
  if (idx.empty()) return MBL_OK;
  // one basis per chain length
  std::map<int, mbl_basis> bases;
  struct Guard {
    std::map<int, mbl_basis>& b;
    ~Guard() {
      for (auto& kv : b) mbl_basis_free(kv.second);
    }
  } guard{bases};
  for (int i : idx) {
    const int L = probs[i].L;
    if (!bases.count(L)) {
      mbl_basis b = nullptr;
      MBL_TRY(mbl_build_basis(L, 0, s, &b));
      bases[L] = b;
    }
  }
  std::vector<DevBasis> hb;
  std::vector<WgPhase> hph;
  std::map<int, int> bidx;
  int64_t nmax = 0;
  int nlo_max = 1;
  for (auto& kv : bases) {
    bidx[kv.first] = (int)hb.size();
    hb.push_back(kv.second->dev());
    nmax = std::max<int64_t>(nmax, kv.second->n);
    nlo_max = std::max(nlo_max, kv.second->nlo);
    WgPhase ph{};
    const int L = kv.first;
    const double pi = 3.14159265358979323846;
    for (int m = 0; m < 2 * L; ++m) {
      ph.c[m] = std::cos(pi * m / L);
      ph.s[m] = std::sin(pi * m / L);
    }
    hph.push_back(ph);
  }
  // problems, most expensive first: longest chains, then weakest disorder
  // (a narrower spectrum, so smaller gaps at sigma and longer MINRES solves)
  std::vector<int> order(idx);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (probs[a].L != probs[b].L) return probs[a].L > probs[b].L;
    return disorder_strength(probs[a]) < disorder_strength(probs[b]);
  });
  std::vector<WgProblem> hp(order.size());
  int mmax_max = 1;
  for (size_t q = 0; q < order.size(); ++q) {
    const mbl_problem& pr = probs[order[q]];
    WgProblem& w = hp[q];
    std::memset(&w, 0, sizeof(w));
    for (int j = 0; j < pr.L; ++j) w.h[j] = pr.h_host[j];
    w.sigma = pr.sigma;
    w.escale = pr.escale;
    w.L = pr.L;
    w.basis = bidx[pr.L];
    w.nev = pr.nev;
    w.mmax = mm[order[q]];
    w.evecs = pr.evecs_dev;
    mmax_max = std::max(mmax_max, w.mmax);
  }
  const int nprob = (int)hp.size();
  const int G = std::max(1, std::min(nprob, device_cu_count()));
  const int64_t vs = (nmax + 63) / 64 * 64;
  const int64_t slot_stride = (int64_t)(kWgVecs + mmax_max + 1) * vs + (int64_t)kWgMaxM * kWgMaxM +
                              (int64_t)kWgMaxM * kWgMaxNev;
  DevBuf d_probs, d_res, d_bases, d_ph, d_slots, d_cnt;
  MBL_TRY(alloc_dev(d_probs, sizeof(WgProblem) * hp.size()));
  MBL_TRY(alloc_dev(d_res, sizeof(WgResult) * hp.size()));
  MBL_TRY(alloc_dev(d_bases, sizeof(DevBasis) * hb.size()));
  MBL_TRY(alloc_dev(d_ph, sizeof(WgPhase) * hph.size()));
  MBL_TRY(alloc_dev(d_slots, sizeof(double) * (size_t)slot_stride * G));
  MBL_TRY(alloc_dev(d_cnt, sizeof(unsigned int)));
  MBL_HIP(hipMemcpyAsync(d_probs.p, hp.data(), sizeof(WgProblem) * hp.size(), hipMemcpyHostToDevice, s));
  MBL_HIP(hipMemcpyAsync(d_bases.p, hb.data(), sizeof(DevBasis) * hb.size(), hipMemcpyHostToDevice, s));
  MBL_HIP(hipMemcpyAsync(d_ph.p, hph.data(), sizeof(WgPhase) * hph.size(), hipMemcpyHostToDevice, s));
  WgParams P{};
  P.probs = static_cast<const WgProblem*>(d_probs.p);
  P.results = static_cast<WgResult*>(d_res.p);
  P.bases = static_cast<const DevBasis*>(d_bases.p);
  P.phases = static_cast<const WgPhase*>(d_ph.p);
  P.slots = static_cast<double*>(d_slots.p);
  P.slot_stride = slot_stride;
  P.vs = vs;
  P.counter = static_cast<unsigned int*>(d_cnt.p);
  // progress counter in host-mapped pinned memory
  unsigned int* done_host = nullptr;
  struct HostGuard {
    unsigned int*& p;
    ~HostGuard() {
      if (p) (void)hipHostFree(p);
    }
  } hguard{done_host};
  if (hipHostMalloc((void**)&done_host, sizeof(unsigned int) * G, hipHostMallocMapped) != hipSuccess) {
    (void)hipGetLastError();
    done_host = nullptr;
  }
  P.done = nullptr;
  if (done_host) {
    for (int g = 0; g < G; ++g) done_host[g] = 0;
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, done_host, 0) == hipSuccess) P.done = static_cast<unsigned int*>(dp);
    else (void)hipGetLastError();
  }
  P.nprob = nprob;
  P.precond = precond;
  P.minres_tol = minres_tol;
  P.eig_tol = eig_tol;
  P.gap_tol = gap_tol;
  P.sigma_rel_tol = 1e-12;
  P.minres_kmax = minres_kmax;
  P.seed = seed;
  const size_t lds = row_lds_for(nlo_max);
  // the two launches (counter reset, persistent solver) as one captured graph
  hipStream_t cap = nullptr;
  MBL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t st;
    ~StreamGuard() { (void)hipStreamDestroy(st); }
  } sg{cap};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  MBL_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, cap, P.counter, 0u);
  hipLaunchKernelGGL(k_si_campaign, dim3(G), dim3(kWgThreads), lds, cap, P);
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  MBL_HIP(e);
  e = hipGraphLaunch(exec, s);
  // wait for the launch; with MBL_VERBOSE set, report the realizations done
  // (counted by the kernel in host-mapped memory) every 30 s
  if (e == hipSuccess) {
    const bool verbose = std::getenv("MBL_VERBOSE") != nullptr;
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, s);
    const auto t0 = std::chrono::steady_clock::now();
    auto last = t0;
    while (e == hipSuccess) {
      const hipError_t q = hipEventQuery(ev);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) {
        e = q;
        break;
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(20));
      const auto now = std::chrono::steady_clock::now();
      if (verbose && done_host && std::chrono::duration<double>(now - last).count() >= 30.0) {
        last = now;
        unsigned int total = 0;
        for (int g = 0; g < G; ++g) total += __atomic_load_n(done_host + g, __ATOMIC_RELAXED);
        std::fprintf(stderr, "[mbl] problems: %u of %d done (%.0f s)\n", total, nprob,
                     std::chrono::duration<double>(now - t0).count());
      }
    }
    if (ev) (void)hipEventDestroy(ev);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (verbose && e == hipSuccess)
      std::fprintf(stderr, "[mbl] persistent launch: %d problems in %.1f s\n", nprob,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  }
  (void)hipGraphExecDestroy(exec);
  MBL_HIP(e);
  std::vector<WgResult> hr(hp.size());
  MBL_HIP(hipMemcpy(hr.data(), d_res.p, sizeof(WgResult) * hr.size(), hipMemcpyDeviceToHost));
  for (size_t q = 0; q < order.size(); ++q) {
    mbl_problem& pr = probs[order[q]];
    const WgResult& r = hr[q];
    for (int t = 0; t < pr.nev; ++t) {
      pr.evals_host[t] = r.evals[t];
      if (pr.resid_host) pr.resid_host[t] = r.resid[t];
      if (pr.z_host) {
        pr.z_host[2 * t] = r.z[2 * t];
        pr.z_host[2 * t + 1] = r.z[2 * t + 1];
      }
    }
    pr.sigma_out = r.sigma;
    pr.info.steps = r.steps;
    pr.info.nconv = r.nconv;
    pr.info.minres_iters = r.minres_iters;
    double mx = 0.0;
    for (int t = 0; t < pr.nev; ++t) mx = std::max(mx, r.resid[t] / r.escale);
    pr.info.max_rel_resid = mx;
    pr.status = r.status;
  }
  return MBL_OK;
}

double gershgorin_bound(const mbl_basis_s* b, const double* h);

// Problems with L > kWgMaxL: the streaming batched form, one run per chain
// length on up to 32 lanes. Each lane runs its own realization's Lanczos
// steps and takes the next realization when its own has converged, so no
// lane waits for the slowest solve of a step. The realizations of each chain
// length are queued by disorder strength, weakest (most expensive) first, so
// the long ones start early and the last lanes to drain hold short ones.
static mbl_status campaign_large(mbl_problem* probs, const std::vector<int>& idx,
                                 const std::vector<int>& mm, double minres_tol,
                                 int64_t minres_kmax, double eig_tol, double gap_tol,
                                 uint64_t seed, int precond, hipStream_t s) {
  std::map<int, std::vector<int>> byL;
  for (int i : idx) byL[probs[i].L].push_back(i);
  for (auto& kv : byL)
    std::stable_sort(kv.second.begin(), kv.second.end(), [&](int a, int c) {
      return disorder_strength(probs[a]) < disorder_strength(probs[c]);
    });
  for (auto& kv : byL) {
    const int L = kv.first;
    const std::vector<int>& all = kv.second;
    mbl_basis b = nullptr;
    MBL_TRY(mbl_build_basis(L, 0, s, &b));
    struct BG {
      mbl_basis b;
      ~BG() { mbl_basis_free(b); }
    } bg{b};
    int R = 2;
    while (R < 32 && R < (int)all.size()) R *= 2;
    int nev = 1, mmax = 1;
    for (int i : all) {
      nev = std::max(nev, probs[i].nev);
      mmax = std::max(mmax, mm[i]);
    }
    mbl_batch bt = nullptr;
    mbl_status st = mbl_batch_create(b, R, mmax, nev, &bt);
    while (st < 0 && R > 2) {   // too wide for this L: halve
      R /= 2;
      st = mbl_batch_create(b, R, mmax, nev, &bt);
    }
    MBL_TRY(st);
    struct BTG {
      mbl_batch b;
      ~BTG() { mbl_batch_free(b); }
    } btg{bt};
    std::vector<StreamProblem> sp(all.size());
    for (size_t q = 0; q < all.size(); ++q) {
      mbl_problem& pr = probs[all[q]];
      double emin = 0, emax = 0, sg = pr.sigma, es = pr.escale;
      if (std::isnan(sg)) {
        MBL_TRY(mbl_sigma_midpoint(b, pr.h_host, 1e-12, 0, &emin, &emax, &sg, s));
        if (!(es > 0)) es = std::max(std::fabs(emin), std::fabs(emax));
      } else if (!(es > 0)) {
        es = gershgorin_bound(b, pr.h_host);
      }
      StreamProblem& p = sp[q];
      p.h = pr.h_host;
      p.sigma = sg;
      p.escale = es;
      p.nev = pr.nev;
      p.seed = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(all[q] + 1);
      p.evals = pr.evals_host;
      p.resid = pr.resid_host;
      p.z = pr.z_host;
      p.evecs_dev = pr.evecs_dev;
      pr.sigma_out = sg;
    }
    MBL_TRY(bstream_si_lanczos(b, bt, sp.data(), (int)sp.size(), nev, mmax, minres_tol,
                               minres_kmax, eig_tol, gap_tol, precond, s));
    for (size_t q = 0; q < all.size(); ++q) {
      mbl_problem& pr = probs[all[q]];
      const StreamProblem& p = sp[q];
      pr.info.steps = p.steps;
      pr.info.nconv = p.nconv;
      pr.info.minres_iters = p.minres_iters;
      pr.info.max_rel_resid = p.max_rel;
      pr.status = p.status;
    }
  }
  return MBL_OK;
}

}  // namespace mbl

using namespace mbl;

extern "C" mbl_status mbl_si_lanczos_problems(mbl_problem* probs, int nprob, int mmax,
                                              double minres_tol, int64_t minres_kmax,
                                              double eig_tol, double gap_tol, uint64_t seed,
                                              int precond, void* stream) {
  clear_error();
  MBL_ARG(probs != nullptr && nprob >= 1, "need a problem array with nprob >= 1");
  MBL_ARG(minres_tol > 0 && std::isfinite(minres_tol) && minres_kmax >= 1, "bad MINRES tolerance or kmax");
  MBL_ARG(eig_tol > 0 && std::isfinite(eig_tol), "eig_tol must be positive");
  MBL_ARG(std::isfinite(gap_tol), "gap_tol must be finite");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  MBL_ARG(mmax == 0 || (mmax >= 1 && mmax <= kWgMaxM), "mmax must be 0 or in [1, 128]");
  // the longest chain of the persistent launch: 16, or MBL_PERSISTENT_MAX_L
  // (even, 10..16) to send shorter chains to the streaming batches as well
  // (the batched kernels have instances from L = 12 on)
  int max_small = kWgMaxL;
  if (const char* e = std::getenv("MBL_PERSISTENT_MAX_L")) {
    const int v = std::atoi(e);
    MBL_ARG(v >= 10 && v <= kWgMaxL && v % 2 == 0, "MBL_PERSISTENT_MAX_L must be even in [10, 16]");
    max_small = v;
  }
  std::vector<int> small, large, mm(nprob);
  for (int i = 0; i < nprob; ++i) {
    const mbl_problem& pr = probs[i];
    MBL_ARG(pr.L >= 4 && pr.L <= kMaxL && pr.L % 2 == 0, "problem L must be even with 4 <= L <= 32");
    MBL_ARG(pr.h_host && pr.evals_host && pr.evecs_dev, "NULL field, eigenvalue or eigenvector pointer");
    MBL_ARG(fields_finite(pr.L, pr.h_host), "non-finite field");
    MBL_ARG(!std::isinf(pr.sigma), "sigma must be finite or NaN (computed)");
    const uint64_t n = nchoosek(pr.L, pr.L / 2);
    MBL_ARG(pr.nev >= 1 && pr.nev <= kWgMaxNev && (uint64_t)pr.nev <= n, "nev must be in [1, min(32, n)]");
    int m = mmax ? mmax : std::min(kWgMaxM, 3 * pr.nev + 40);
    m = (int)std::min<uint64_t>((uint64_t)m, n);
    MBL_ARG(m >= pr.nev, "mmax must be >= nev");
    mm[i] = m;
    (pr.L <= max_small ? small : large).push_back(i);
  }
  for (int i = 0; i < nprob; ++i) {
    probs[i].status = MBL_OK;
    probs[i].info = mbl_si_info{};
    probs[i].sigma_out = NAN;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  MBL_TRY(campaign_small(probs, small, mm, minres_tol, minres_kmax, eig_tol, gap_tol, seed, precond, s));
  MBL_TRY(campaign_large(probs, large, mm, minres_tol, minres_kmax, eig_tol, gap_tol, seed, precond, s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  mbl_status worst = MBL_OK;
  for (int i = 0; i < nprob; ++i) {
    probs[i].info.seconds = secs;
    if (probs[i].status < 0) worst = probs[i].status;
    else if (worst >= 0 && probs[i].status > worst) worst = probs[i].status;
  }
  if (worst != MBL_OK) set_error("some problems did not converge (see their status)");
  return worst < 0 ? MBL_WARN_NOCONV : worst;
}
