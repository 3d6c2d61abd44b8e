// Row kernels of the matrix-free Hamiltonian (Eq. (1)) on gfx950, and the
// dense vector helpers around them.
//
// Work decomposition. A state a = (hi << nlo) | lo. Rows sharing hi are one
// contiguous block; a chunk is up to 64 consecutive rows of one block and is
// processed by one wavefront, one row per lane. Inside a wavefront hi is
// uniform, so everything that depends on hi alone (block offsets of the
// neighbour blocks, which high bonds are antiparallel) is scalar work, and a
// hop on a bond inside the high bits reads a contiguous run of x from the
// neighbour block: a coalesced load. Hops on bonds inside the low bits stay
// in the same block (a few KB, cache resident); their targets come from the
// low-pattern rank table held in LDS. The two bonds that cross the split (the
// one between bit nlo-1 and bit nlo, and the periodic bond between bit L-1
// and bit 0) change the popcount of both halves and use both tables.
//
// Diagonal: a_aa - sigma = L/4 - N_anti/2 + (1/2) sum_j h_j - F(a) - sigma,
// where N_anti = popcount(a xor rotl_L(a, 1)) counts antiparallel bonds and
// F(a) = sum of h_j over set bits, summed from a per-nibble table in LDS.
//
// Reductions are per-workgroup partial sums written in a fixed order and
// reduced again in a fixed order, so results are bitwise reproducible.
#include "rows.h"

#include <algorithm>
#include <cstdlib>

namespace mbl {

// ---------------------------------------------------------------------------
// y = (H - sigma) x. MODE 0: plain; 1: partial sums of x.y; 2: partial sums of
// y.y. GUARD: the product of MINRES iteration k, which first takes the Givens
// step of iteration k - 1 (G; every workgroup the same, workgroup 0 stores
// it) and returns at once when the state is then done. (L, NLO) = (0, 0) is
// the runtime-split form.
template <typename T, int MODE, bool GUARD, int L, int NLO>
__global__ __launch_bounds__(kWG) void k_apply(DevBasis B, FieldArgs F, MinresGivens G,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               double* __restrict__ partials, Defl D) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the MINRES scalars and partial sums are loaded before the table fill, so
  // that the two latencies overlap
  PartialsPrefetch pq, pc;
  MinresState sp{};
  double al = 0.0;
  if (GUARD) {
    if (G.active) {
      prefetch_partials(G.part2, G.P2, pq);
      sp = *G.Sprev;
      al = *G.alpha;
    } else if (G.Scur->done) {
      return;
    }
    if (D.v) prefetch_partials(D.c_part, D.P, pc);
  }
  const RowTables t = setup_tables<L>(B, F, smem);
  __syncthreads();
  if (GUARD && G.active) {
    const double qz = reduce_prefetched(pq, G.P2, t.red);
    const MinresState so = minres_givens_step(sp, al, qz, G.tol, G.kmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) *G.Scur = so;
    if (so.done) return;
  }
  // rank-one term theta v (v . x) of a deflated MINRES operator
  double dcoef = 0.0;
  if (GUARD && D.v) dcoef = D.theta * reduce_prefetched(pc, D.P, t.red);
  double acc = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0,
                     uint32_t a) {
    const double xi = (double)x[row];
    const double off = RowOps<T, L, NLO>::offdiag(B, t, x, hi, lo, j, block0);
    int na;
    const double dsh = row_diag<L>(B, F, t, a, na);
    double yv = dsh * xi + 0.5 * off;
    if (GUARD && D.v) yv += dcoef * D.v[row];
    const T yt = (T)yv;
    y[row] = yt;
    if (MODE == 1) acc += xi * (double)yt;
    if (MODE == 2) acc += (double)yt * (double)yt;
  });
  if (MODE != 0) {
    const double s = block_sum_all(acc, t.red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kWG) void k_precond(DevBasis B, FieldArgs F, int kind,
                                                 const double* z, double* q) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    int na;
    const double dsh = row_diag<0>(B, F, t, a, na);
    q[row] = z[row] / precond_value(kind, dsh, na);
  });
}

// r = rhs - (H - sigma) x, partials[2g] = sum r^2 / m, partials[2g+1] = sum r^2
template <int L, int NLO>
__global__ __launch_bounds__(kWG) void k_residual(DevBasis B, FieldArgs F, int kind,
                                                  const double* __restrict__ rhs,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ r,
                                                  double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RowTables t = setup_tables<L>(B, F, smem);
  __syncthreads();
  double am = 0.0, a2 = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0,
                     uint32_t a) {
    const double off = RowOps<double, L, NLO>::offdiag(B, t, x, hi, lo, j, block0);
    int na;
    const double dsh = row_diag<L>(B, F, t, a, na);
    const double ri = rhs[row] - (dsh * x[row] + 0.5 * off);
    r[row] = ri;
    am += ri * ri / precond_value(kind, dsh, na);
    a2 += ri * ri;
  });
  const double sm = block_sum_all(am, t.red);
  const double s2 = block_sum_all(a2, t.red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sm;
    partials[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(kWG) void k_states(DevBasis B, uint32_t* states) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldArgs F{};
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    states[row] = a;
  });
}

__global__ __launch_bounds__(kWG) void k_rank(DevBasis B, const uint32_t* states, int64_t count,
                                              int64_t* ranks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t a = states[i];
  const uint64_t top = (uint64_t)a >> B.L;
  int64_t out = -1;
  if (top == 0 && __popc(a) == B.half) {
    const uint32_t hi = a >> B.nlo, lo = a & ((1u << B.nlo) - 1u);
    out = (int64_t)B.hi_off[hi] + B.lo_rank[lo];
  }
  ranks[i] = out;
}

// Twist overlap partial sums. m(a) = 2 sum_{set bits p} (p + 1) - L(L+1)/2,
// u_a = exp(i pi m / L) from a 2L-entry table.
struct TwistTables {
  double c[2 * kMaxL];
  double s[2 * kMaxL];
};

__global__ __launch_bounds__(kWG) void k_twist(DevBasis B, TwistTables T, const double* psi,
                                               int64_t ld, double* partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  FieldArgs F{};
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  const double* v = psi + (size_t)blockIdx.y * ld;
  const int twoL = 2 * B.L;
  const int base = (B.L * (B.L + 1)) / 2;
  double are = 0.0, aim = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    int sum = 0;   // sum over set bits of (p + 1)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      uint32_t w = 0;
      for (int p = 0; p < 32; ++p)
        if (((p + 1) >> k) & 1) w |= (1u << p);
      sum += __popc(a & w) << k;
    }
    int m = (2 * sum - base) % twoL;
    if (m < 0) m += twoL;
    const double c2 = v[row] * v[row];
    are += c2 * T.c[m];
    aim += c2 * T.s[m];
  });
  const double sr = block_sum_all(are, t.red);
  const double si = block_sum_all(aim, t.red);
  if (threadIdx.x == 0) {
    const size_t g = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[2 * g] = sr;
    partials[2 * g + 1] = si;
  }
}

// ---------------------------------------------------------------------------
// dense helpers

constexpr int kDenseGrid = 512;

__global__ __launch_bounds__(kWG) void k_dot(int64_t n, const double* __restrict__ x,
                                             const double* __restrict__ y,
                                             double* __restrict__ partials) {
  __shared__ double red[kWavesPerWG];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  const double s = block_sum_all(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[v] = sum_{g < nparts} partials[g * stride + v], one workgroup per v.
__global__ __launch_bounds__(kWG) void k_reduce(const double* __restrict__ partials, int nparts,
                                                int stride, double* __restrict__ out) {
  __shared__ double red[kWavesPerWG];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int g = threadIdx.x; g < nparts; g += blockDim.x) acc += partials[(size_t)g * stride + v];
  const double s = block_sum_all(acc, red);
  if (threadIdx.x == 0) out[v] = s;
}

__global__ __launch_bounds__(kWG) void k_axpby(int64_t n, double a, const double* __restrict__ x,
                                               double b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // BLAS convention: a zero coefficient does not read its operand
    const double ax = a != 0.0 ? a * x[i] : 0.0;
    y[i] = b != 0.0 ? ax + b * y[i] : ax;
  }
}

__global__ __launch_bounds__(kWG) void k_scale_copy(int64_t n, double a, const double* __restrict__ x,
                                                    double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ __launch_bounds__(kWG) void k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

// SplitMix64 (Steele, Lea & Flood 2014) of seed + (i + 1) * golden gamma,
// top 53 bits mapped to [-1/2, 1/2).
__global__ __launch_bounds__(kWG) void k_splitmix(int64_t n, uint64_t seed, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    y[i] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
  }
}

// ---------------------------------------------------------------------------
// host launch wrappers

int row_grid(const mbl_basis_s* b) {
  int g = (b->nchunks + kWavesPerWG - 1) / kWavesPerWG;
  if (g > kMaxPartials) g = kMaxPartials;
  if (g < 1) g = 1;
  return g >= 64 ? (g / 8) * 8 : g;   // whole XCD slices once the grid is large
}

size_t row_lds_bytes(const mbl_basis_s* b) { return row_lds_for(b->nlo); }

static int dense_grid(int64_t n) {
  int64_t g = (n + kWG - 1) / kWG;
  return (int)(g < 1 ? 1 : (g > kDenseGrid ? kDenseGrid : g));
}

// launch the (L, NLO) instance matching the basis, else the runtime form
template <typename T, int MODE, bool GUARD>
static hipError_t apply_dispatch(const mbl_basis_s* b, const FieldArgs& F, const MinresGivens& S,
                                 const T* x, T* y, double* partials, hipStream_t s,
                                 const Defl& D = Defl{}) {
  const dim3 g(row_grid(b)), blk(kWG);
  const size_t lds = row_lds_bytes(b);
  const DevBasis B = b->dev();
  switch (b->L * 64 + b->nlo) {
#define MBL_CASE(LL, NN)                                                                     \
  case LL * 64 + NN:                                                                        \
    hipLaunchKernelGGL((k_apply<T, MODE, GUARD, LL, NN>), g, blk, lds, s, B, F, S, x, y,  \
                       partials, D);                                                        \
    return hipGetLastError();
    MBL_FAST_SPLITS(MBL_CASE)
#undef MBL_CASE
    default:
      hipLaunchKernelGGL((k_apply<T, MODE, GUARD, 0, 0>), g, blk, lds, s, B, F, S, x, y,
                         partials, D);
      return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_apply(const mbl_basis_s* b, const FieldArgs& F, const T* x, T* y, int mode,
                        double* partials, int* nparts, hipStream_t s) {
  if (nparts) *nparts = row_grid(b);
  if (mode == 0) return apply_dispatch<T, 0, false>(b, F, MinresGivens{}, x, y, partials, s);
  if (mode == 1) return apply_dispatch<T, 1, false>(b, F, MinresGivens{}, x, y, partials, s);
  return apply_dispatch<T, 2, false>(b, F, MinresGivens{}, x, y, partials, s);
}
template hipError_t launch_apply<double>(const mbl_basis_s*, const FieldArgs&, const double*,
                                         double*, int, double*, int*, hipStream_t);
template hipError_t launch_apply<float>(const mbl_basis_s*, const FieldArgs&, const float*, float*,
                                        int, double*, int*, hipStream_t);

template <typename T>
hipError_t launch_minres_apply(const mbl_basis_s* b, const FieldArgs& F, const MinresGivens& G,
                               const T* q, T* p, double* partials, const Defl& D, hipStream_t s) {
  return apply_dispatch<T, 1, true>(b, F, G, q, p, partials, s, D);
}
template hipError_t launch_minres_apply<double>(const mbl_basis_s*, const FieldArgs&,
                                                const MinresGivens&, const double*, double*,
                                                double*, const Defl&, hipStream_t);
template hipError_t launch_minres_apply<float>(const mbl_basis_s*, const FieldArgs&,
                                               const MinresGivens&, const float*, float*, double*,
                                               const Defl&, hipStream_t);

hipError_t launch_precond(const mbl_basis_s* b, const FieldArgs& F, int kind, const double* z,
                          double* q, hipStream_t s) {
  hipLaunchKernelGGL(k_precond, dim3(row_grid(b)), dim3(kWG), row_lds_bytes(b), s, b->dev(), F,
                     kind, z, q);
  return hipGetLastError();
}

hipError_t launch_residual(const mbl_basis_s* b, const FieldArgs& F, int precond,
                           const double* rhs, const double* x, double* r, double* partials,
                           int* nparts, hipStream_t s) {
  const int g = row_grid(b);
  if (nparts) *nparts = g;
  const size_t lds = row_lds_bytes(b);
  switch (b->L * 64 + b->nlo) {
#define MBL_CASE(LL, NN)                                                                    \
  case LL * 64 + NN:                                                                       \
    hipLaunchKernelGGL((k_residual<LL, NN>), dim3(g), dim3(kWG), lds, s, b->dev(), F,     \
                       precond, rhs, x, r, partials);                                      \
    return hipGetLastError();
    MBL_FAST_SPLITS(MBL_CASE)
#undef MBL_CASE
    default:
      hipLaunchKernelGGL((k_residual<0, 0>), dim3(g), dim3(kWG), lds, s, b->dev(), F, precond,
                         rhs, x, r, partials);
      return hipGetLastError();
  }
}

hipError_t launch_states(const mbl_basis_s* b, uint32_t* states, hipStream_t s) {
  hipLaunchKernelGGL(k_states, dim3(row_grid(b)), dim3(kWG), row_lds_bytes(b), s, b->dev(),
                     states);
  return hipGetLastError();
}

hipError_t launch_rank(const mbl_basis_s* b, const uint32_t* states, int64_t count,
                       int64_t* ranks, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int64_t g = (count + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_rank, dim3((unsigned)g), dim3(kWG), 0, s, b->dev(), states, count, ranks);
  return hipGetLastError();
}

hipError_t launch_twist(const mbl_basis_s* b, const double* psi, int64_t ld, int nvec,
                        const double* costab, const double* sintab, double* partials, int* nparts,
                        hipStream_t s) {
  TwistTables T{};
  for (int m = 0; m < 2 * b->L; ++m) {
    T.c[m] = costab[m];
    T.s[m] = sintab[m];
  }
  int g = row_grid(b);
  if (g * nvec > kMaxPartials * 32) g = (kMaxPartials * 32) / nvec;
  if (g < 1) g = 1;
  if (nparts) *nparts = g;
  hipLaunchKernelGGL(k_twist, dim3(g, nvec), dim3(kWG), row_lds_bytes(b), s, b->dev(), T, psi, ld,
                     partials);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double* x, const double* y, double* partials, int* nparts,
                      hipStream_t s) {
  const int g = dense_grid(n);
  if (nparts) *nparts = g;
  hipLaunchKernelGGL(k_dot, dim3(g), dim3(kWG), 0, s, n, x, y, partials);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int stride, int nvals, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nvals), dim3(kWG), 0, s, partials, nparts, stride, out);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(dense_grid(n)), dim3(kWG), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

hipError_t launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(dense_grid(n)), dim3(kWG), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(dense_grid(n)), dim3(kWG), 0, s, n, v, y);
  return hipGetLastError();
}

hipError_t launch_splitmix(int64_t n, uint64_t seed, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_splitmix, dim3(dense_grid(n)), dim3(kWG), 0, s, n, seed, y);
  return hipGetLastError();
}

}  // namespace mbl
