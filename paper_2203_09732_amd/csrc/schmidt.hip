// Bipartite entanglement entropy of eigenvectors (Sec. IV, entanglement and
// level spacing): S = -Tr rho_A ln rho_A for subsystem A = sites 1..la
// (bits 0..la-1 of the state), and the level-spacing ratio r_k.
//
// In the S^z = 0 sector the coefficients psi(a, b) (a: the bits of A, b: the
// bits of B) vanish unless a has k and b has L/2 - k up spins, so the
// coefficient matrix is block diagonal in k, block k being dA_k x dB_k with
// dA_k = C(la, k) and dB_k = C(L - la, L/2 - k), and rho_A is the direct sum
// of the Gram matrices of the blocks. On the device:
//   1. k_schmidt_scatter permutes the n coefficients into the blocks (one
//      coalesced pass over the rows). Block k is stored column-major with its
//      rows on the smaller side, so its Gram matrix G_k is m_k x m_k with
//      m_k = min(dA_k, dB_k). A state's place inside its block is its rank
//      among the states of the same width and popcount in ascending order
//      (combinatorial number system); any bijection would do, since the
//      spectrum of G_k does not depend on the order of rows and columns.
//   2. k_schmidt_gram forms G_k = X_k X_k^T on the FP64 matrix cores, one
//      wavefront per 16 x 16 tile (v_mfma_f64_16x16x4f64).
// On the host the eigenvalues of every G_k (Householder tridiagonalisation,
// then symmetric QR, eigenvalues only) are divided by Tr rho_A = sum_k tr G_k
// and S = -sum p ln p; (vector, block) tasks run on up to 16 threads and
// are combined in a fixed order.
#include "rows.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

namespace mbl {

constexpr int kSchmidtMaxK = 33;   // k = 0..32

struct SchmidtArgs {
  int la;
  int64_t n;                     // elements per vector in X
  int64_t gtot;                  // elements per vector in G
  int64_t xoff[kSchmidtMaxK];    // block k in X
  int64_t goff[kSchmidtMaxK];    // block k in G
  uint32_t m[kSchmidtMaxK];      // rows of X_k (the smaller side)
  uint32_t c[kSchmidtMaxK];      // columns of X_k (the larger side)
  uint32_t a_rows[kSchmidtMaxK]; // 1: rows are the states of A
};

// C(n, r) exactly (each partial product is itself a binomial coefficient)
__device__ __forceinline__ uint32_t sbinom(uint32_t n, uint32_t r) {
  if (r > n) return 0;
  uint64_t v = 1;
  for (uint32_t t = 1; t <= r; ++t) v = v * (uint64_t)(n - r + t) / t;
  return (uint32_t)v;
}

// rank of a bit pattern among the patterns of its width and popcount, in
// ascending order: sum over its set bits p_1 < p_2 < ... of C(p_i, i)
__device__ __forceinline__ uint32_t cns_rank(uint32_t bits) {
  uint32_t r = 0, i = 0;
  while (bits) {
    const uint32_t p = (uint32_t)__ffs(bits) - 1u;
    ++i;
    r += sbinom(p, i);
    bits &= bits - 1u;
  }
  return r;
}

// vector v = t R + r of the input (t < nvec, r < R) has its element i at
// psi[t ld + i rstride + r]: ld = n, rstride = R = 1 for column-major
// vectors, ld = n R, rstride = R for R interleaved realizations
__global__ __launch_bounds__(kWG) void k_schmidt_scatter(DevBasis B, SchmidtArgs A,
                                                         const double* __restrict__ psi,
                                                         int64_t ld, int64_t rstride, int R,
                                                         int64_t v0, int nv,
                                                         double* __restrict__ X) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldArgs F{};
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  const uint32_t maskA = (1u << A.la) - 1u;   // la <= L - 1 <= 31
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    const uint32_t sa = a & maskA, sb = a >> A.la;
    const int k = __popc(sa);
    const int64_t ia = cns_rank(sa), ib = cns_rank(sb);
    const int64_t dst = A.xoff[k] + (A.a_rows[k] ? ib * A.m[k] + ia : ia * A.m[k] + ib);
    for (int j = 0; j < nv; ++j) {
      const int64_t v = v0 + j, t = v / R, r = v % R;
      X[(size_t)j * A.n + dst] = psi[(size_t)t * ld + (size_t)row * rstride + r];
    }
  });
}

typedef double v4d __attribute__((ext_vector_type(4)));

// G_k = X_k X_k^T, tile (k, ti, tj) of 16 x 16 per wavefront, vector
// blockIdx.y. X_k is column-major (m_k rows): element (i, t) at t * m_k + i.
// MFMA operands: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16) of the
// 16 x 4 and 4 x 16 slices, and receives D(l / 16 + 4 v, l % 16), v < 4
// (the layout of this instruction on gfx950, measured).
__global__ __launch_bounds__(kWG) void k_schmidt_gram(SchmidtArgs A, const uint4* __restrict__ tiles,
                                                      int ntiles, const double* __restrict__ X,
                                                      double* __restrict__ Gm) {
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int tix = (int)blockIdx.x * (kWG / 64) + wave;
  if (tix >= ntiles) return;   // the whole wavefront
  const uint4 tl = tiles[tix];
  const int k = (int)tl.x;
  const uint32_t m = A.m[k], c = A.c[k];
  const double* Xk = X + (size_t)blockIdx.y * A.n + A.xoff[k];
  double* Gk = Gm + (size_t)blockIdx.y * A.gtot + A.goff[k];
  const uint32_t i0 = tl.y * 16u, j0 = tl.z * 16u;
  const uint32_t li = (uint32_t)lane & 15u, lk = (uint32_t)lane >> 4;
  const bool in_i = i0 + li < m, in_j = j0 + li < m;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t t0 = 0; t0 < c; t0 += 4) {
    const uint32_t tt = t0 + lk;
    const bool in_t = tt < c;
    const double av = (in_i && in_t) ? Xk[(size_t)tt * m + i0 + li] : 0.0;
    const double bv = (in_j && in_t) ? Xk[(size_t)tt * m + j0 + li] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t row = i0 + lk + 4u * (uint32_t)v, col = j0 + li;
    if (row < m && col < m) Gk[(size_t)row * m + col] = acc[v];
  }
}

// ---------------------------------------------------------------------------
// host: eigenvalues of a symmetric matrix (row-major, overwritten) by
// Householder reduction to tridiagonal form (Golub & Van Loan, Sec. 8.3.1),
// then the symmetric QR iterations of tridiag_eig without eigenvectors. A
// column whose entries are all below 1e-20 max|A| is taken as zero (the
// eigenvalues move by less than that); otherwise a rank-deficient block is
// reduced to a tridiagonal graded down into the subnormal range, where the
// deflation test no longer works. The reduction leaves the large entries at
// the top of the tridiagonal and the small ones at the bottom, the grading
// the QR iteration (shifted and deflated from the bottom) converges on.
static int sym_eigenvalues(int m, std::vector<double>& A, std::vector<double>& w) {
  w.assign(m, 0.0);
  if (m == 1) {
    w[0] = A[0];
    return 0;
  }
  std::vector<double> d(m), e(m, 0.0), v(m), p(m);
  double amax = 0.0;
  for (double x : A) amax = std::max(amax, std::fabs(x));
  const double negligible = 1e-20 * amax;
  for (int k = 0; k + 2 < m; ++k) {
    d[k] = A[(size_t)k * m + k];
    // the column below the diagonal, scaled by its largest entry so that
    // neither its norm nor the reflector overflows or underflows
    double sc = 0.0;
    for (int i = k + 1; i < m; ++i) sc = std::max(sc, std::fabs(A[(size_t)i * m + k]));
    if (sc <= negligible) {
      e[k] = 0.0;
      continue;
    }
    double xx = 0.0;
    for (int i = k + 1; i < m; ++i) {
      v[i] = A[(size_t)i * m + k] / sc;
      xx += v[i] * v[i];
    }
    const double xn = std::sqrt(xx);
    const double r = v[k + 1] >= 0.0 ? -xn : xn;   // H x = r sc e_1
    v[k + 1] -= r;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    for (int i = k + 1; i < m; ++i) v[i] /= vn;    // unit reflector: H = I - 2 v v^T
    // trailing block B <- H B H: p = 2 B v, w = p - (v^T p) v, B -= v w^T + w v^T
    double vp = 0.0;
    for (int i = k + 1; i < m; ++i) {
      const double* Ai = &A[(size_t)i * m];
      double sum = 0.0;
      for (int j = k + 1; j < m; ++j) sum += Ai[j] * v[j];
      p[i] = 2.0 * sum;
      vp += v[i] * p[i];
    }
    for (int i = k + 1; i < m; ++i) p[i] -= vp * v[i];
    for (int i = k + 1; i < m; ++i) {
      double* Ai = &A[(size_t)i * m];
      const double vi = v[i], pi = p[i];
      for (int j = k + 1; j < m; ++j) Ai[j] -= vi * p[j] + pi * v[j];
    }
    e[k] = r * sc;
  }
  d[m - 2] = A[(size_t)(m - 2) * m + (m - 2)];
  e[m - 2] = A[(size_t)(m - 1) * m + (m - 2)];
  if (std::fabs(e[m - 2]) <= negligible) e[m - 2] = 0.0;
  d[m - 1] = A[(size_t)(m - 1) * m + (m - 1)];
  return tridiag_eig(m, d.data(), e.data(), w.data(), nullptr);
}

static uint64_t hbinom(int n, int k) {
  if (k < 0 || k > n) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

mbl_status entropy_run(mbl_basis_s* b, const double* psi, int64_t ld, int64_t rstride, int R,
                       int nvec, int la, double* S, hipStream_t s) {
  const int L = b->L, half = b->half;
  SchmidtArgs A{};
  A.la = la;
  A.n = b->n;
  int64_t xo = 0, go = 0;
  std::vector<int> ks;
  std::vector<uint4> tiles;
  for (int k = 0; k <= la && k < kSchmidtMaxK; ++k) {
    const uint64_t dA = hbinom(la, k), dB = hbinom(L - la, half - k);
    if (dA == 0 || dB == 0) continue;
    A.xoff[k] = xo;
    A.goff[k] = go;
    A.a_rows[k] = dA <= dB ? 1u : 0u;
    A.m[k] = (uint32_t)std::min(dA, dB);
    A.c[k] = (uint32_t)std::max(dA, dB);
    xo += (int64_t)(dA * dB);
    go += (int64_t)A.m[k] * A.m[k];
    ks.push_back(k);
    const uint32_t nt = (A.m[k] + 15u) / 16u;
    for (uint32_t ti = 0; ti < nt; ++ti)
      for (uint32_t tj = 0; tj < nt; ++tj) tiles.push_back(make_uint4((uint32_t)k, ti, tj, 0u));
  }
  if (xo != b->n) {
    set_error("Schmidt blocks do not cover the sector");
    return MBL_ERR_ARG;
  }
  A.gtot = go;
  // vectors per device pass: X and G of every vector of the pass in HBM (at
  // most 4 GiB), and at most 64 (the Gram launch's y dimension, host copies)
  const int chunk = (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)nvec, (int64_t)64, ((int64_t)4 << 30) / (8 * (b->n + go))}));
  double *X = nullptr, *Gd = nullptr;
  uint4* td = nullptr;
  auto release = [&] {
    if (X) (void)hipFree(X);
    if (Gd) (void)hipFree(Gd);
    if (td) (void)hipFree(td);
  };
  if (hipMalloc((void**)&X, sizeof(double) * (size_t)chunk * b->n) != hipSuccess ||
      hipMalloc((void**)&Gd, sizeof(double) * (size_t)chunk * go) != hipSuccess ||
      hipMalloc((void**)&td, sizeof(uint4) * tiles.size()) != hipSuccess) {
    (void)hipGetLastError();
    release();
    set_error("device allocation for the Schmidt blocks failed");
    return MBL_ERR_NOMEM;
  }
  mbl_status st = MBL_OK;
  std::vector<double> Gh((size_t)chunk * go);
  const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (hipMemcpy(td, tiles.data(), sizeof(uint4) * tiles.size(), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipGetLastError();
    set_error("copy of the Gram tile table failed");
    st = MBL_ERR_HIP;
  }
  for (int v0 = 0; v0 < nvec && st == MBL_OK; v0 += chunk) {
    const int nv = std::min(chunk, nvec - v0);
    hipLaunchKernelGGL(k_schmidt_scatter, dim3(row_grid(b)), dim3(kWG), row_lds_bytes(b), s,
                       b->dev(), A, psi, ld, rstride, R, (int64_t)v0, nv, X);
    const int ntiles = (int)tiles.size();
    hipLaunchKernelGGL(k_schmidt_gram, dim3((ntiles + 3) / 4, nv), dim3(kWG), 0, s, A, td,
                       ntiles, X, Gd);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(Gh.data(), Gd, sizeof(double) * (size_t)nv * go, hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("HIP error in the entanglement entropy kernels");
      st = MBL_ERR_HIP;
      break;
    }
    // tasks (vector, block), largest blocks first; partial sums in a table
    const int nb = (int)ks.size();
    std::vector<std::pair<int, int>> tasks;
    for (int v = 0; v < nv; ++v)
      for (int q = 0; q < nb; ++q) tasks.emplace_back(v, q);
    std::stable_sort(tasks.begin(), tasks.end(), [&](const auto& x, const auto& y) {
      return A.m[ks[x.second]] > A.m[ks[y.second]];
    });
    std::vector<double> trace((size_t)nv * nb, 0.0), plogp((size_t)nv * nb, 0.0);
    std::vector<std::vector<double>> evals((size_t)nv * nb);
    std::atomic<size_t> next{0};
    std::atomic<int> failed{0};
    auto worker = [&] {
      std::vector<double> M;
      for (;;) {
        const size_t t = next.fetch_add(1);
        if (t >= tasks.size()) break;
        const int v = tasks[t].first, q = tasks[t].second, k = ks[q];
        const int m = (int)A.m[k];
        const double* G = &Gh[(size_t)v * go + A.goff[k]];
        M.assign(G, G + (size_t)m * m);
        double tr = 0.0;
        for (int i = 0; i < m; ++i) tr += M[(size_t)i * m + i];
        trace[(size_t)v * nb + q] = tr;
        if (sym_eigenvalues(m, M, evals[(size_t)v * nb + q]) != 0) failed = 1;
      }
    };
    std::vector<std::thread> pool;
    for (int i = 1; i < nthreads; ++i) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    if (failed) {
      set_error("eigenvalues of a Schmidt block did not converge");
      st = MBL_ERR_NUMERIC;
      break;
    }
    for (int v = 0; v < nv; ++v) {
      double T = 0.0;
      for (int q = 0; q < nb; ++q) T += trace[(size_t)v * nb + q];
      if (!(T > 0.0) || !std::isfinite(T)) {
        set_error("entanglement entropy of a zero or non-finite vector");
        st = MBL_ERR_NUMERIC;
        break;
      }
      double Sv = 0.0;
      for (int q = 0; q < nb; ++q)
        for (double lam : evals[(size_t)v * nb + q]) {
          const double pr = lam / T;
          if (pr > 0.0) Sv -= pr * std::log(pr);
        }
      S[v0 + v] = Sv;
    }
  }
  release();
  return st;
}

mbl_status symmetric_eigenvalues_run(int m, const double* A, double* w) {
  std::vector<double> M(A, A + (size_t)m * m), ev;
  if (sym_eigenvalues(m, M, ev) != 0) {
    set_error("symmetric eigenvalues did not converge");
    return MBL_ERR_NUMERIC;
  }
  std::copy(ev.begin(), ev.end(), w);
  return MBL_OK;
}

mbl_status spacing_ratio_run(int count, const double* E, double* r, double* r_mean) {
  std::vector<double> e(E, E + count);
  std::sort(e.begin(), e.end());
  double sum = 0.0;
  int used = 0;
  for (int k = 1; k + 1 < count; ++k) {
    const double d0 = e[k] - e[k - 1], d1 = e[k + 1] - e[k];
    const double hi = std::max(d0, d1), lo = std::min(d0, d1);
    const double rk = hi > 0.0 ? lo / hi : std::nan("");
    if (r) r[k - 1] = rk;
    if (hi > 0.0) {
      sum += rk;
      ++used;
    }
  }
  *r_mean = used ? sum / used : std::nan("");
  return MBL_OK;
}

}  // namespace mbl
