// Preconditioned MINRES for (H - sigma I) x = b (App. A, Alg. 2) on gfx950.
//
// Iteration k is two row launches on the same stream:
//   1. the product p = A q_k with partial sums of q_k . p; it first takes the
//      Givens step of iteration k - 1 (beta_k from the partials of q_k . z_k,
//      the rotation, phi_{k-1}, the d/x coefficients of iteration k - 1) and
//      returns at once when the solve is done (kernels.hip, k_apply GUARD);
//   2. the d/x update of iteration k - 1, d_{k-1} and x_{k-1} += tau d_{k-1}
//      (a flat elementwise pass); then alpha_k = q_k . p / beta_k^2; z_{k+1} =
//      p/beta_k - (alpha_k/beta_k) z_k - (beta_k/beta_{k-1}) z_{k-1}; q_{k+1} =
//      M^{-1} z_{k+1} with M regenerated from the state bits; partial sums of
//      q_{k+1} . z_{k+1} (a pass over the rows). Two passes in one launch keep
//      fewer vectors streaming at a time than one fused pass (measured faster
//      at every L, 5 % at L = 26 in FP64 and 14 % in FP32).
// Every workgroup reduces the partial sums itself in the same fixed order,
// so all workgroups hold bitwise identical scalars without a host round
// trip. The scalar states live in device memory in two slots (k & 1); the
// host checks them one chunk of iterations behind, and after the last
// iteration one small launch takes its Givens step and d/x update.
//
// Vector slots: z_{k-1}/z_{k+1} share a buffer (updated in place), so do
// d_{k-3}/d_{k-1}; q_{k-1}, q_k, q_{k+1} use a ring of three. With p and x
// that is 9 n-vectors besides b.
#include "rows.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>
#include <type_traits>
#include <cstring>

namespace mbl {

// ---- initialisation: z_0 = 0, z_1 = scale * (src - Ax0), q_1 = M^{-1} z_1,
// d_{-1} = d_0 = 0, e = 0 (if given); partial sums of q_1 . z_1.
template <typename T>
__global__ __launch_bounds__(kWG) void k_minres_init(DevBasis B, FieldArgs F, int kind,
                                                     const double* __restrict__ src,
                                                     const T* __restrict__ ax0, double scale,
                                                     T* z0, T* z1, T* q1, T* d0, T* d1, T* e,
                                                     double* __restrict__ partials,
                                                     const double* __restrict__ dv,
                                                     double* __restrict__ part3) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RowTables t = setup_tables(B, F, smem);
  __syncthreads();
  double acc = 0.0, acc3 = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    double zi = src[row];
    if (ax0) zi -= (double)ax0[row];
    const T zt = (T)(scale * zi);
    int na;
    const double dsh = row_diag<0>(B, F, t, a, na);
    const T qt = (T)((double)zt / precond_value(kind, dsh, na));
    z0[row] = (T)0;
    z1[row] = zt;
    q1[row] = qt;
    d0[row] = (T)0;
    d1[row] = (T)0;
    if (e) e[row] = (T)0;
    acc += (double)qt * (double)zt;
    if (dv) acc3 += dv[row] * (double)qt;
  });
  const double s = block_sum_all(acc, t.red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (dv) {
    const double s3 = block_sum_all(acc3, t.red);
    if (threadIdx.x == 0) part3[blockIdx.x] = s3;
  }
}

__global__ void k_minres_init_state(const double* __restrict__ partials, int P, double tol,
                                    int64_t kmax, MinresState* S) {
  __shared__ double red[kWavesPerWG];
  const double qz = reduce_partials(partials, P, red);
  if (threadIdx.x == 0) {
    const double beta = sqrt(qz);
    MinresState s0;
    s0.beta_prev = 1.0;
    s0.beta = beta;
    s0.c = 1.0;
    s0.s = 0.0;
    s0.dhat = 0.0;
    s0.eps = 0.0;
    s0.phi = beta;
    s0.k = 0;
    s0.bad = !isfinite(beta);
    s0.done = !(fabs(beta) >= tol && 0 < kmax);
    S[0] = s0;
  }
}

// ---- step 2: alpha_k; z_{k+1}, q_{k+1}, partial sums of q_{k+1} . z_{k+1};
// the d/x update of iteration k - 1 --------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_minres_zqdx(
    DevBasis B, FieldArgs F, int kind, const MinresState* __restrict__ Sprev,
    const MinresState* __restrict__ Scur, const double* __restrict__ part1, int P1,
    double* __restrict__ alpha_out, const T* __restrict__ p, const T* __restrict__ zk,
    T* __restrict__ zkm1, T* __restrict__ qnext, double* __restrict__ part2,
    const double* __restrict__ dv, double* __restrict__ part3, const T* __restrict__ qprev,
    T* __restrict__ dprev, const T* __restrict__ dprev2, T* __restrict__ x) {
  const bool zq = !Scur->done;                 // iteration k is taken
  const bool dx = Sprev && !Sprev->done;       // iteration k - 1 was taken
  if (!zq && !dx) return;
  extern __shared__ __align__(16) unsigned char smem[];
  PartialsPrefetch pp;   // loaded before the table fill (overlapping latencies)
  if (zq) prefetch_partials(part1, P1, pp);
  const MinresState sc = *Scur;
  // d_{k-1} = (q_{k-1} / beta_{k-1} - delta d_{k-2} - eps d_{k-3}) / gamma and
  // x_{k-1} = x_{k-2} + tau d_{k-1}, from the Givens step of iteration k - 1
  // (the state sc): elementwise, so a flat grid-stride pass
  if (dx) {
    const double ib = sc.d_inv_beta, de = sc.d_delta, ep = sc.d_eps, ig = sc.d_inv_gamma,
                 tau = sc.d_tau;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B.n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double d = ((double)qprev[i] * ib - de * (double)dprev2[i] -
                        ep * (double)dprev[i]) * ig;
      const T dt = (T)d;
      dprev[i] = dt;
      x[i] = (T)((double)x[i] + tau * (double)dt);
    }
  }
  if (!zq) return;
  const RowTables t = setup_tables(B, F, smem);
  const double qp = reduce_prefetched(pp, P1, t.red);
  const double alpha = qp / (sc.beta * sc.beta);
  if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
  const double c1 = 1.0 / sc.beta, c2 = alpha / sc.beta, c3 = sc.beta / sc.beta_prev;
  double acc = 0.0, acc3 = 0.0;
  for_rows(B, t, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a) {
    {
      const double zn = c1 * (double)p[row] - c2 * (double)zk[row] - c3 * (double)zkm1[row];
      const T zt = (T)zn;
      int na;
      const double dsh = row_diag<0>(B, F, t, a, na);
      const T qt = (T)((double)zt / precond_value(kind, dsh, na));
      zkm1[row] = zt;
      qnext[row] = qt;
      acc += (double)qt * (double)zt;
      if (dv) acc3 += dv[row] * (double)qt;
    }
  });
  const double s = block_sum_all(acc, t.red);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
  if (dv) {
    const double s3 = block_sum_all(acc3, t.red);
    if (threadIdx.x == 0) part3[blockIdx.x] = s3;
  }
}

// ---- after the last issued iteration K: its Givens step (one workgroup) ----
__global__ __launch_bounds__(kWG) void k_minres_givens_last(MinresGivens G) {
  __shared__ double red[kWavesPerWG];
  const double qz = reduce_partials(G.part2, G.P2, red);
  if (threadIdx.x == 0) *G.Scur = minres_givens_step(*G.Sprev, *G.alpha, qz, G.tol, G.kmax);
}

// ---- and its d/x update: d_K, x_K (flat kernel) ------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_minres_dx_last(int64_t n, const MinresState* __restrict__ Sprev,
                                                        const MinresState* __restrict__ Scur,
                                                        const T* __restrict__ qk,
                                                        T* __restrict__ dk,
                                                        const T* __restrict__ dkm1,
                                                        T* __restrict__ x) {
  if (Sprev->done) return;
  const MinresState sc = *Scur;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = ((double)qk[i] * sc.d_inv_beta - sc.d_delta * (double)dkm1[i] -
                      sc.d_eps * (double)dk[i]) * sc.d_inv_gamma;
    const T dt = (T)d;
    dk[i] = dt;
    x[i] = (T)((double)x[i] + sc.d_tau * (double)dt);
  }
}

// ---- the whole solve in one cooperative launch ------------------------------
// Every workgroup owns the rows of its chunks (grid-stride over chunks) for
// every vector update, and meets the others at two grid barriers per
// iteration:
//   phase A: d_{k-1}, x_{k-1} update of the previous iteration on own rows;
//            p = A q_k on own rows (gathers read all of q_k); partial q_k.p
//   -- barrier --
//   phase B: alpha_k from all partials; z_{k+1}, q_{k+1} on own rows; partial
//            q_{k+1}.z_{k+1}
//   -- barrier --
//   phase C: beta_{k+1} and the Givens rotation from all partials (every
//            workgroup computes the same scalars in the same order, so all
//            leave the loop at the same k)
// A barrier is an arrival counter; a workgroup that waits longer than about
// one second marks the launch failed and leaves, so the launch always ends.
template <typename T>
struct PersistArgs {
  T* z[2];
  T* q[2];
  T* d[2];
  T* p;
  T* x;
  double* part1;
  double* part2;
  GridSync gs;           // arrival counter, release generation, result, failure flag
  MinresState* S;        // S[0]: state after initialisation; final state written back
  double tol;
  int64_t kmax;
  int kind;
};

constexpr uint64_t kBarrierTimeoutTicks = 100000000ull;   // ~1 s of the 100 MHz clock

// Grid-wide sum of one partial per workgroup at a barrier. Each workgroup
// publishes its partial and arrives on a 64-bit counter; the last to arrive
// sums the G partials in the fixed order of reduce_partials (so the result
// does not depend on arrival order) and releases the others by advancing a
// generation word. One reduction per barrier instead of one per workgroup.
// A workgroup that waits longer than about one second sets the failure flag
// and every workgroup leaves, so the launch always ends.
__device__ __forceinline__ bool reduce_barrier(const GridSync& g, const double* partials, int G,
                                               unsigned long long epoch, double* red, int* sflag,
                                               double* sval, double& out) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned long long prev = atomicAdd(g.count, 1ull);
    *sflag = (prev == (epoch + 1ull) * (unsigned long long)G - 1ull) ? 1 : 0;
  }
  __syncthreads();
  if (*sflag) {   // the last arrival reduces (uniform in the workgroup)
    __threadfence();
    const double sum = reduce_partials(partials, G, red);
    if (threadIdx.x == 0) {
      __hip_atomic_store(g.result, __builtin_bit_cast(unsigned long long, sum), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(g.gen, epoch + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0) {
    const uint64_t t0 = wall_clock64();
    int bad = 0;
    while (__hip_atomic_load(g.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < epoch + 1ull) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          wall_clock64() - t0 > kBarrierTimeoutTicks) {
        bad = 1;
        atomicExch(g.fail, 1);
        break;
      }
    }
    *sval = __builtin_bit_cast(double, __hip_atomic_load(g.result, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT));
    *sflag = bad;
  }
  __syncthreads();
  out = *sval;
  return *sflag == 0;
}

template <typename T, int L, int NLO>
__global__ __launch_bounds__(kWG) void k_minres_persistent(DevBasis B, FieldArgs F,
                                                           PersistArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sflag;
  __shared__ double sval;
  const RowTables t = setup_tables<L>(B, F, smem);
  __syncthreads();
  MinresState st = a.S[0];
  const int G = gridDim.x;
  unsigned long long epoch = 0;
  // previous iteration's d/x update, applied at the start of the next phase A
  bool pending = false;
  double pv_inv_beta = 0, pv_delta = 0, pv_eps = 0, pv_inv_gamma = 0, pv_tau = 0;
  const uint32_t wpg = kWavesPerWG;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t first = blockIdx.x * wpg + wave, stride = G * wpg;
  int64_t k = st.k;
  bool done = st.done != 0;
  while (!done) {
    ++k;
    T* qk = a.q[k & 1];
    T* qn = a.q[(k + 1) & 1];
    T* zk = a.z[k & 1];
    T* zkm1 = a.z[(k + 1) & 1];
    // ---- phase A
    {
      T* dprev = a.d[(k - 1) & 1];        // receives d_{k-1} (holds d_{k-3})
      const T* dpp = a.d[k & 1];          // d_{k-2}
      const T* qprev = qn;                // q_{k-1} (overwritten only in phase B)
      double acc = 0.0;
      for_rows_range(B, t, first, stride,
                     [&](uint32_t row, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0,
                         uint32_t s_a) {
                       if (pending) {
                         const double dd = ((double)qprev[row] * pv_inv_beta -
                                            pv_delta * (double)dpp[row] -
                                            pv_eps * (double)dprev[row]) *
                                           pv_inv_gamma;
                         const T dt = (T)dd;
                         dprev[row] = dt;
                         a.x[row] = (T)((double)a.x[row] + pv_tau * (double)dt);
                       }
                       const double xi = (double)qk[row];
                       const double off = RowOps<T, L, NLO>::offdiag(B, t, qk, hi, lo, j, block0);
                       int na;
                       const double dsh = row_diag<L>(B, F, t, s_a, na);
                       const T pt = (T)(dsh * xi + 0.5 * off);
                       a.p[row] = pt;
                       acc += xi * (double)pt;
                     });
      const double sblk = block_sum_all(acc, t.red);
      if (threadIdx.x == 0) a.part1[blockIdx.x] = sblk;
    }
    double qp = 0.0;
    if (!reduce_barrier(a.gs, a.part1, G, epoch++, t.red, &sflag, &sval, qp)) return;
    // ---- phase B
    const double beta = st.beta, beta_prev = st.beta_prev;
    const double alpha = qp / (beta * beta);
    {
      const double c1 = 1.0 / beta, c2 = alpha / beta, c3 = beta / beta_prev;
      double acc = 0.0;
      for_rows_range(B, t, first, stride,
                     [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t s_a) {
                       const double zn = c1 * (double)a.p[row] - c2 * (double)zk[row] -
                                         c3 * (double)zkm1[row];
                       const T zt = (T)zn;
                       int na;
                       const double dsh = row_diag<L>(B, F, t, s_a, na);
                       const T qt = (T)((double)zt / precond_value(a.kind, dsh, na));
                       zkm1[row] = zt;
                       qn[row] = qt;
                       acc += (double)qt * (double)zt;
                     });
      const double sblk = block_sum_all(acc, t.red);
      if (threadIdx.x == 0) a.part2[blockIdx.x] = sblk;
    }
    double qz = 0.0;
    if (!reduce_barrier(a.gs, a.part2, G, epoch++, t.red, &sflag, &sval, qz)) return;
    // ---- phase C (scalars, identical in every workgroup)
    const double beta_next = sqrt(qz);
    const double delta = st.c * st.dhat + st.s * alpha;
    const double gamma_hat = -st.s * st.dhat + st.c * alpha;
    const double eps_next = st.s * beta_next;
    const double dhat_next = st.c * beta_next;
    const double gamma = sqrt(gamma_hat * gamma_hat + beta_next * beta_next);
    const double c = gamma_hat / gamma;
    const double s = beta_next / gamma;
    const double tau = c * st.phi;
    const double phi = -s * st.phi;
    pending = true;
    pv_inv_beta = 1.0 / beta;
    pv_delta = delta;
    pv_eps = st.eps;
    pv_inv_gamma = 1.0 / gamma;
    pv_tau = tau;
    st.beta_prev = beta;
    st.beta = beta_next;
    st.c = c;
    st.s = s;
    st.dhat = dhat_next;
    st.eps = eps_next;
    st.phi = phi;
    st.k = k;
    st.bad = !isfinite(phi) || !isfinite(alpha) || !isfinite(beta_next);
    done = st.bad || !(fabs(phi) >= a.tol && k < a.kmax);
    st.done = done;
  }
  // the last iteration's d/x update (q_k is still in q[k & 1])
  if (pending) {
    T* dk = a.d[k & 1];                  // holds d_{k-2}
    const T* dkm1 = a.d[(k - 1) & 1];
    const T* qk = a.q[k & 1];
    for_rows_range(B, t, first, stride,
                   [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t) {
                     const double dd = ((double)qk[row] * pv_inv_beta -
                                        pv_delta * (double)dkm1[row] - pv_eps * (double)dk[row]) *
                                       pv_inv_gamma;
                     const T dt = (T)dd;
                     dk[row] = dt;
                     a.x[row] = (T)((double)a.x[row] + pv_tau * (double)dt);
                   });
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.S[1] = st;
}

__global__ void k_zero_u32(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// x64 += scale * e
__global__ __launch_bounds__(kWG) void k_add_scaled_f32(int64_t n, double scale,
                                                        const float* __restrict__ e,
                                                        double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += scale * (double)e[i];
}


static int flat_grid(int64_t n) {
  int64_t g = (n + kWG - 1) / kWG;
  if (g > 2048) g = 2048;
  return (int)(g < 1 ? 1 : g);
}

static size_t mlds(const mbl_basis_s* b) { return row_lds_for(b->nlo); }

// One cooperative launch for the whole solve. Returns MBL_ERR_HIP with
// *refused = true when the runtime declines the cooperative launch (the
// caller then uses the per-iteration launches).
template <typename T>
static mbl_status persistent_solve(mbl_basis_s* b, const FieldArgs& F, int precond,
                                   mbl_workspace_s* ws, T* x, double tol, int64_t kmax,
                                   hipStream_t s, MinresState* out, bool* refused) {
  *refused = false;
  const void* fn = nullptr;
  switch (b->L * 64 + b->nlo) {
#define MBL_CASE(LL, NN)                                        \
  case LL * 64 + NN:                                           \
    fn = (const void*)&k_minres_persistent<T, LL, NN>;         \
    break;
    MBL_FAST_SPLITS(MBL_CASE)
#undef MBL_CASE
    default:
      fn = (const void*)&k_minres_persistent<T, 0, 0>;
  }
  const size_t lds = row_lds_for(b->nlo);
  int dev = 0, ncu = 0, per_cu = 0;
  MBL_HIP(hipGetDevice(&dev));
  MBL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MBL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWG, lds));
  int G = std::min(ncu * std::max(per_cu, 0), (b->nchunks + kWavesPerWG - 1) / kWavesPerWG);
  G = std::min(G, kMaxPartials);
  if (G < 1) {
    *refused = true;
    return MBL_ERR_HIP;
  }
  PersistArgs<T> a;
  for (int i = 0; i < 2; ++i) {
    a.z[i] = (T*)ws->z[i];
    a.q[i] = (T*)ws->q[i];
    a.d[i] = (T*)ws->d[i];
  }
  a.p = (T*)ws->p;
  a.x = x;
  a.part1 = ws->partials1;
  a.part2 = ws->partials2;
  a.gs = grid_sync(ws->sync);
  a.S = ws->state;
  a.tol = tol;
  a.kmax = kmax;
  a.kind = precond;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws->sync, kSyncWords);
  MBL_HIP(hipGetLastError());
  DevBasis B = b->dev();
  FieldArgs Fc = F;
  void* args[] = {&B, &Fc, &a};
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(kWG), args, (unsigned)lds, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *refused = true;
    return MBL_ERR_HIP;
  }
  MBL_HIP(hipMemcpyAsync(&ws->h_state[2], ws->state + 1, sizeof(MinresState),
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipMemcpyAsync(&ws->h_state[3], ws->sync, sizeof(unsigned int) * kSyncWords,
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  const int fail = reinterpret_cast<const int*>(&ws->h_state[3])[kSyncFailWord];
  if (fail) {
    set_error("grid barrier timed out in the persistent MINRES launch");
    return MBL_ERR_HIP;
  }
  *out = ws->h_state[2];
  return MBL_OK;
}

// The single cooperative launch pays two grid barriers per iteration. On a
// GPU whose L2 caches are private to each XCD, a barrier that makes one
// workgroup's vector writes visible to the others needs device-scope release
// and acquire fences, which write back and invalidate L2; measured, the
// launches per iteration are faster from L = 16 up (11.8 against 17.2 us
// per iteration at L = 16, 14.7 against 35 at L = 18) and the cooperative launch
// wins only on the smallest grids. MBL_MINRES_LAUNCH=iter|persistent forces
// a form.
constexpr int kPersistentMaxGrid = 32;
static bool use_persistent(const mbl_basis_s* b) {
  static int forced = -2;
  if (forced == -2) {
    const char* e = getenv("MBL_MINRES_LAUNCH");
    forced = !e ? -1 : (std::string(e) == "iter" ? 0 : (std::string(e) == "persistent" ? 1 : -1));
  }
  if (forced >= 0) return forced == 1;
  return (b->nchunks + kWavesPerWG - 1) / kWavesPerWG <= kPersistentMaxGrid;
}

// Runs Alg. 2 on vectors of type T. src: FP64 right-hand side (scaled by
// scale on entry). x: T solution (x0 on entry unless x0_zero).
template <typename T>
static mbl_status minres_core(mbl_basis_s* b, const FieldArgs& F, const double* src,
                              double scale, T* x, bool x0_zero, double tol, int64_t kmax,
                              int precond, mbl_workspace_s* ws, int64_t* iters, double* phi,
                              hipStream_t s, const double* defl = nullptr, double theta = 0.0) {
  const int64_t n = b->n;
  T* Z[2] = {(T*)ws->z[0], (T*)ws->z[1]};
  T* Q[2] = {(T*)ws->q[0], (T*)ws->q[1]};
  T* D[2] = {(T*)ws->d[0], (T*)ws->d[1]};
  T* P = (T*)ws->p;
  const int G = row_grid(b);
  const size_t lds = mlds(b);
  const DevBasis B = b->dev();
  MinresState* S = ws->state;

  // p = A x0 (skipped when x0 = 0; a deflated solve starts from x0 = 0)
  if (!x0_zero) MBL_HIP(launch_apply<T>(b, F, x, P, 0, nullptr, nullptr, s));
  Defl dfl;
  if (defl) {
    dfl.v = defl;
    dfl.theta = theta;
    dfl.c_part = ws->partials3;
    dfl.P = G;
  }
  // z_0 = 0 in Z[0], z_1 in Z[1], q_1 in Q[1], d_{-1} in D[1], d_0 in D[0]
  hipLaunchKernelGGL((k_minres_init<T>), dim3(G), dim3(kWG), lds, s, B, F, precond, src,
                     x0_zero ? (const T*)nullptr : (const T*)P, scale, Z[0], Z[1], Q[1], D[0],
                     D[1], x0_zero ? x : (T*)nullptr, ws->partials2, defl, ws->partials3);
  MBL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_minres_init_state, dim3(1), dim3(kWG), 0, s, ws->partials2, G, tol, kmax,
                     S);
  MBL_HIP(hipGetLastError());

  if (use_persistent(b) && !defl) {
    MinresState fin{};
    bool refused = false;
    mbl_status ps = persistent_solve<T>(b, F, precond, ws, x, tol, kmax, s, &fin, &refused);
    if (ps == MBL_OK) {
      *iters = fin.k;
      *phi = fin.phi;
      if (fin.bad) {
        set_error("MINRES met a non-finite value (singular preconditioner or breakdown)");
        return MBL_ERR_NUMERIC;
      }
      return (fabs(fin.phi) < tol) ? MBL_OK : MBL_WARN_NOCONV;
    }
    if (!refused) return ps;
    clear_error();
  }

  T* Qr[3] = {(T*)ws->q[0], (T*)ws->q[1], (T*)ws->q[2]};   // q_k in Qr[k % 3]
  const int FG = flat_grid(n);
  MinresGivens gbase;
  gbase.part2 = ws->partials2;
  gbase.P2 = G;
  gbase.tol = tol;
  gbase.kmax = kmax;
  // the Givens step of iteration k - 1: state k - 1 into slot (k - 1) & 1,
  // alpha_{k-1} in ws->alpha[(k - 1) & 1]
  auto givens_args = [&](int64_t k) {
    MinresGivens g = gbase;
    g.alpha = ws->alpha + ((k - 1) & 1);
    g.Sprev = S + (k & 1);
    g.Scur = S + ((k - 1) & 1);
    g.active = k >= 2;
    return g;
  };
  // iteration k: the product (after the Givens step of k - 1), then the z/q
  // update of k with the d/x update of k - 1
  auto iteration = [&](int64_t k, hipStream_t st) -> mbl_status {
    const MinresGivens g = givens_args(k);
    MBL_HIP(launch_minres_apply<T>(b, F, g, Qr[k % 3], P, ws->partials1, dfl, st));
    hipLaunchKernelGGL((k_minres_zqdx<T>), dim3(G), dim3(kWG), lds, st, B, F, precond,
                       k >= 2 ? (const MinresState*)g.Sprev : (const MinresState*)nullptr,
                       (const MinresState*)g.Scur, ws->partials1, G, ws->alpha + (k & 1), P,
                       Z[k & 1], Z[(k + 1) & 1], Qr[(k + 1) % 3], ws->partials2, defl,
                       ws->partials3, Qr[(k + 2) % 3], D[(k + 1) & 1], D[k & 1], x);
    MBL_HIP(hipGetLastError());
    return MBL_OK;
  };
  // after the last issued iteration K: its Givens step and its d/x update
  auto finish = [&](int64_t K, hipStream_t st) -> mbl_status {
    const MinresGivens g = givens_args(K + 1);
    hipLaunchKernelGGL(k_minres_givens_last, dim3(1), dim3(kWG), 0, st, g);
    hipLaunchKernelGGL((k_minres_dx_last<T>), dim3(FG), dim3(kWG), 0, st, n,
                       (const MinresState*)g.Sprev, (const MinresState*)g.Scur, Qr[K % 3],
                       D[K & 1], (const T*)D[(K + 1) & 1], x);
    MBL_HIP(hipGetLastError());
    return MBL_OK;
  };
  // Iteration 1 runs eagerly; then blocks of kGraphIters iterations (2..13,
  // 14..25, ...), whose buffers and state slots depend only on k mod 6 and
  // whose kernels read their scalars and done flags from device memory, are
  // captured once (on the workspace's own stream) and replayed on the
  // caller's stream; a replay after convergence is a sequence of no-op
  // launches. The graph holds its kernel arguments (fields and shift, tol,
  // kmax, x, the preconditioner, the deflation vector), so it is captured
  // again when any of them changes.
  constexpr int64_t kGraphIters = 12;
  const int64_t kChunkIters = 4 * kGraphIters;
  if (ws->graph_mode < 0) {
    const char* e = getenv("MBL_MINRES_GRAPHS");
    ws->graph_mode = (e && std::string(e) == "0") ? 0 : 1;
  }
  const bool use_graph = ws->graph_mode == 1 && kmax > kChunkIters;
  const int ti = std::is_same<T, float>::value ? 1 : 0;
  if (use_graph) {
    std::vector<unsigned char> key(sizeof(FieldArgs) + 2 * sizeof(double) + sizeof(int64_t) +
                                   2 * sizeof(void*) + sizeof(int));
    unsigned char* kp = key.data();
    auto put = [&](const void* v, size_t sz) {
      std::memcpy(kp, v, sz);
      kp += sz;
    };
    put(&F, sizeof(FieldArgs));
    put(&tol, sizeof(double));
    put(&theta, sizeof(double));
    put(&kmax, sizeof(int64_t));
    const void* xp = x;
    const void* dp = defl;
    put(&xp, sizeof(void*));
    put(&dp, sizeof(void*));
    put(&precond, sizeof(int));
    hipGraphExec_t& gx = ws->graph[ti];
    if (gx && ws->graph_key[ti] != key) {
      (void)hipGraphExecDestroy(gx);
      gx = nullptr;
    }
    if (!gx) {
      if (!ws->cap) MBL_HIP(hipStreamCreateWithFlags(&ws->cap, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      MBL_HIP(hipStreamBeginCapture(ws->cap, hipStreamCaptureModeThreadLocal));
      mbl_status cst = MBL_OK;
      for (int64_t k = 2; k <= kGraphIters + 1 && cst == MBL_OK; ++k) cst = iteration(k, ws->cap);
      hipError_t ee = hipStreamEndCapture(ws->cap, &g);
      if (cst != MBL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return cst;
      }
      MBL_HIP(ee);
      ee = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      MBL_HIP(ee);
      ws->graph_key[ti] = key;
    }
  }
  int64_t issued = 0;
  int pending = 0;       // status copies in flight (0..2)
  int slot = 0;
  bool done = false;
  // a status copy for the chunk ending at iteration k goes to h_state[slot]
  auto check = [&](int which) -> mbl_status {
    MBL_HIP(hipEventSynchronize(ws->ev[which]));
    if (ws->h_state[which].done) done = true;
    return MBL_OK;
  };
  if (kmax >= 1) {
    MBL_TRY(iteration(1, s));
    issued = 1;
  }
  while (!done && issued < kmax) {
    const int64_t k_end = std::min(kmax, issued + kChunkIters);
    if (use_graph && k_end - issued == kChunkIters) {
      for (int64_t rep = 0; rep < kChunkIters / kGraphIters; ++rep)
        MBL_HIP(hipGraphLaunch(ws->graph[ti], s));
    } else {
      for (int64_t k = issued + 1; k <= k_end; ++k) MBL_TRY(iteration(k, s));
    }
    issued = k_end;
    // the newest state on the device is the one after iteration issued - 1
    MBL_HIP(hipMemcpyAsync(&ws->h_state[slot], S + ((issued - 1) & 1), sizeof(MinresState),
                           hipMemcpyDeviceToHost, s));
    MBL_HIP(hipEventRecord(ws->ev[slot], s));
    ++pending;
    if (pending == 2) {     // wait for the previous chunk's status, keep one chunk queued
      MBL_TRY(check(slot ^ 1));
      --pending;
    }
    slot ^= 1;
  }
  if (pending > 0) MBL_TRY(check(slot ^ 1));
  if (issued >= 1) MBL_TRY(finish(issued, s));
  MBL_HIP(hipMemcpyAsync(&ws->h_state[0], S + (issued & 1), sizeof(MinresState),
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  const MinresState last = ws->h_state[0];
  *iters = last.k;
  *phi = last.phi;
  if (last.bad) {
    set_error("MINRES met a non-finite value (singular preconditioner or breakdown)");
    return MBL_ERR_NUMERIC;
  }
  return (fabs(last.phi) < tol) ? MBL_OK : MBL_WARN_NOCONV;
}

mbl_status minres_run(mbl_basis_s* b, const double* h_host, double sigma, const double* rhs,
                      double* x, double tol, int64_t kmax, int precision, int precond,
                      bool x0_zero, mbl_workspace_s* ws, mbl_minres_info* info, hipStream_t s,
                      const double* defl, double theta) {
  const FieldArgs F = make_fields(b, h_host, sigma);
  const int64_t n = b->n;
  mbl_minres_info inf{};
  mbl_status st = MBL_OK;
  if (precision == MBL_FP64) {
    int64_t it = 0;
    double phi = 0;
    st = minres_core<double>(b, F, rhs, 1.0, x, x0_zero, tol, kmax, precond, ws, &it, &phi, s,
                             defl, theta);
    if (st < 0) return st;
    inf.iters = it;
    inf.phi = phi;
  } else {
    // FP32 inner solves, FP64 residual recomputation and restart. Each cycle
    // solves A e = r / ||r||_{M^-1} in FP32 to a relative tolerance eta and
    // updates x += ||r||_{M^-1} e in FP64. The FP32 recurrence drifts from
    // the true residual by roughly u_32 times the squared condition number,
    // so a cycle can report its tolerance without having reduced the true
    // residual; a cycle that does not cut the FP64 residual by kMinCycleGain
    // ends the FP32 phase and the solve is finished by FP64 MINRES on the
    // same residual.
    const double eta = 1e-3;
    const double kMinCycleGain = 10.0;
    const int max_restarts = 60;
    // MBL_VERBOSE=1: one line per cycle on stderr
    const bool verbose = std::getenv("MBL_VERBOSE") != nullptr;
    int64_t total = 0;
    int restarts = 0;
    double rM = 0.0, rM_prev = INFINITY;
    bool first = true, fp64_finish = false;
    for (;;) {
      int np = 0;
      if (first && x0_zero) MBL_HIP(launch_fill(n, 0.0, x, s));
      MBL_HIP(launch_residual(b, F, precond, rhs, x, ws->r64, ws->partials1, &np, s));
      double sums[2];
      MBL_TRY(reduce_to_host(ws, ws->partials1, np, 2, 2, sums, s));
      rM = std::sqrt(sums[0]);
      first = false;
      if (verbose)
        std::fprintf(stderr, "[mbl] fp32-inner cycle %d: ||r||_M^-1 = %.3e after %lld iterations\n",
                     restarts, rM, (long long)total);
      if (!std::isfinite(rM)) {
        set_error("non-finite residual in FP32-inner MINRES");
        return MBL_ERR_NUMERIC;
      }
      if (!(rM >= tol) || total >= kmax) break;
      if (restarts >= max_restarts || rM > rM_prev / kMinCycleGain) {
        fp64_finish = true;
        break;
      }
      rM_prev = rM;
      const double inner_tol = std::max(eta, 0.5 * tol / rM);
      int64_t it = 0;
      double phi = 0;
      mbl_status s2 = minres_core<float>(b, F, ws->r64, 1.0 / rM, (float*)ws->e, true, inner_tol,
                                         kmax - total, precond, ws, &it, &phi, s);
      if (s2 < 0) return s2;
      if (verbose)
        std::fprintf(stderr, "[mbl]   inner FP32 solve: %lld iterations, phi %.3e (target %.1e)\n",
                     (long long)it, phi, inner_tol);
      total += it;
      hipLaunchKernelGGL(k_add_scaled_f32, dim3(flat_grid(n)), dim3(kWG), 0, s, n, rM,
                         (const float*)ws->e, x);
      MBL_HIP(hipGetLastError());
      ++restarts;
    }
    if (fp64_finish) {
      // FP64 MINRES on A e = r (r = rhs - A x is in r64), then x += e
      int64_t it = 0;
      double phi = 0;
      double* e64 = ws->t64;
      mbl_status s3 = minres_core<double>(b, F, ws->r64, 1.0, e64, true, tol, kmax - total,
                                          precond, ws, &it, &phi, s);
      if (s3 < 0) return s3;
      if (verbose)
        std::fprintf(stderr, "[mbl]   FP64 finish: %lld iterations, phi %.3e, status %d\n",
                     (long long)it, phi, (int)s3);
      total += it;
      MBL_HIP(launch_axpby(n, 1.0, e64, 1.0, x, s));
      int np = 0;
      MBL_HIP(launch_residual(b, F, precond, rhs, x, ws->r64, ws->partials1, &np, s));
      double sums[2];
      MBL_TRY(reduce_to_host(ws, ws->partials1, np, 2, 2, sums, s));
      rM = std::sqrt(sums[0]);
      if (verbose)
        std::fprintf(stderr, "[mbl]   after the FP64 finish: ||r||_M^-1 = %.3e\n", rM);
    }
    inf.iters = total;
    inf.restarts = restarts;
    inf.phi = rM;
    st = (rM < tol) ? MBL_OK : MBL_WARN_NOCONV;
  }
  // true residual ||b - (H - sigma) x||_2 in FP64
  {
    int np = 0;
    MBL_HIP(launch_residual(b, F, precond, rhs, x, ws->r64, ws->partials1, &np, s));
    double sums[2];
    MBL_TRY(reduce_to_host(ws, ws->partials1, np, 2, 2, sums, s));
    inf.true_res = std::sqrt(sums[1]);
  }
  if (info) *info = inf;
  return st;
}

}  // namespace mbl
