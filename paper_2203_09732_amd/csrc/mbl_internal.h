// Internal declarations of the MI355X library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mbl.h"

namespace mbl {

constexpr int kMaxL = 32;
constexpr int kMaxLoBits = 13;   // LDS tables: 2 x 2^13 x 2 B = 32 KB
constexpr int kMaxLanczos = 1000; // mmax bound (CGS and Ritz tiles are staged in LDS)
constexpr int kWG = 256;             // threads per workgroup (4 waves of 64)
constexpr int kWavesPerWG = kWG / 64;
constexpr int kMaxPartials = 1024;   // upper bound on workgroups of a reducing launch
constexpr int kChunk = 64;           // rows per chunk = one wave

// ---------------------------------------------------------------------------
// Error reporting (thread-local message, C ABI status codes).
void set_error(const std::string& msg);
void clear_error();

#define MBL_HIP(call)                                                               \
  do {                                                                              \
    hipError_t _e = (call);                                                         \
    if (_e != hipSuccess) {                                                         \
      ::mbl::set_error(std::string(#call) + ": " + hipGetErrorString(_e));          \
      return MBL_ERR_HIP;                                                           \
    }                                                                               \
  } while (0)

#define MBL_TRY(expr)                \
  do {                               \
    mbl_status _s = (expr);          \
    if (_s < 0) return _s;           \
  } while (0)

#define MBL_ARG(cond, msg)                       \
  do {                                           \
    if (!(cond)) {                               \
      ::mbl::set_error(msg);                     \
      return MBL_ERR_ARG;                        \
    }                                            \
  } while (0)

// ---------------------------------------------------------------------------
// Sector basis in (high bits, low bits) form.
//
// A state a = (hi << nlo) | lo. Ascending integer order is (hi, lo)
// lexicographic order, so the states sharing hi form one contiguous block
// starting at hi_off[hi]; inside it lo runs over the nlo-bit patterns with
// popcount L/2 - popcount(hi) in ascending order, at offset lo_rank[lo].
// A chunk is up to 64 consecutive rows of one block: one wavefront.
struct DevBasis {
  int L, nlo, nhi, half;
  int64_t n;
  int nchunks;
  const uint32_t* hi_off;    // [1 << nhi], 0xffffffff for empty blocks
  const uint16_t* lo_rank;   // [1 << nlo]
  const uint16_t* lo_state;  // [1 << nlo], sorted by (popcount, value)
  const uint32_t* lo_coff;   // [nlo + 2], start of popcount class c in lo_state
  const uint4* chunks;       // {hi, j0, count, row0}
};

// Fields and shift, by value in kernel arguments.
struct FieldArgs {
  double h[kMaxL];
  double c0;      // L/4 + (1/2) sum_j h_j - sigma
  double sigma;
};

// Rank-one term theta * v v^T added to the operator of a MINRES solve
// (deflation of a known near-null vector v). c_part holds per-workgroup
// partial sums of v . q for the current q.
struct Defl {
  const double* v = nullptr;
  double theta = 0.0;
  const double* c_part = nullptr;
  int P = 0;
};

// Words of the grid-barrier block of a workspace (device, zeroed before a
// cooperative launch): 64-bit arrival counter, 64-bit release generation,
// the published sum (a double), the failure flag.
constexpr int kSyncWords = 8;
constexpr int kSyncFailWord = 6;
struct GridSync {
  unsigned long long* count;
  unsigned long long* gen;
  unsigned long long* result;
  int* fail;
};
inline GridSync grid_sync(unsigned int* words) {
  return GridSync{reinterpret_cast<unsigned long long*>(words),
                  reinterpret_cast<unsigned long long*>(words + 2),
                  reinterpret_cast<unsigned long long*>(words + 4),
                  reinterpret_cast<int*>(words + kSyncFailWord)};
}

// MINRES scalar state after iteration k (two slots, k & 1).
struct MinresState {
  double beta_prev, beta, c, s, dhat, eps, phi;
  int64_t k;
  int32_t done;
  int32_t bad;     // non-finite value met
  // coefficients of the d/x update of iteration k: d_k = (q_k d_inv_beta -
  // d_delta d_{k-1} - d_eps d_{k-2}) d_inv_gamma, x_k = x_{k-1} + d_tau d_k
  double d_inv_beta, d_delta, d_eps, d_inv_gamma, d_tau;
};

// The Givens step of iteration k - 1 that the MINRES product of iteration k
// takes first (the same in every workgroup; workgroup 0 stores it).
struct MinresGivens {
  const double* part2 = nullptr;   // q_k . z_k partials of the previous z/q update
  int P2 = 0;
  const double* alpha = nullptr;   // alpha_{k-1}
  const MinresState* Sprev = nullptr;   // state after iteration k - 2
  MinresState* Scur = nullptr;          // receives the state after iteration k - 1
  double tol = 0.0;
  int64_t kmax = 0;
  int active = 0;                  // 0 at k = 1: Scur holds the initial state
};

}  // namespace mbl

struct mbl_basis_s {
  int L, nlo, nhi, half;
  int64_t n;
  int nchunks;
  int device;
  uint32_t* d_hi_off = nullptr;
  uint16_t* d_lo_rank = nullptr;
  uint16_t* d_lo_state = nullptr;
  uint32_t* d_lo_coff = nullptr;
  uint4* d_chunks = nullptr;
  mbl::DevBasis dev() const {
    return mbl::DevBasis{L, nlo, nhi, half, n, nchunks, d_hi_off, d_lo_rank, d_lo_state,
                         d_lo_coff, d_chunks};
  }
};

struct mbl_workspace_s {
  mbl_basis basis;
  int mmax;
  int precision;
  int64_t n;
  int64_t bytes = 0;
  // MINRES vectors: FP64 set or FP32 set (+ FP64 residual for restarts)
  void* z[2] = {nullptr, nullptr};
  void* q[3] = {nullptr, nullptr, nullptr};   // ring: q_{k-1}, q_k, q_{k+1}
  void* d[2] = {nullptr, nullptr};
  void* p = nullptr;
  void* e = nullptr;         // FP32 correction (FP32 inner form)
  double* r64 = nullptr;     // FP64 residual / scratch vector
  double* t64 = nullptr;     // FP64 scratch vector
  // Lanczos
  double* V = nullptr;       // n x (mmax + 1)
  double* w = nullptr;       // n
  double* x = nullptr;       // n
  double* coef = nullptr;    // device, mmax + 64 doubles
  double* ycoef = nullptr;   // device, selected Ritz coefficients
  // reductions and MINRES state
  double* partials1 = nullptr;   // kMaxPartials * 64
  double* partials2 = nullptr;   // kMaxPartials * 64
  double* partials3 = nullptr;   // kMaxPartials
  double* red_out = nullptr;     // 256 doubles
  mbl::MinresState* state = nullptr;  // 2 slots
  double* alpha = nullptr;            // 2 slots: MINRES alpha_k by the parity of k
  unsigned int* sync = nullptr;       // kSyncWords: grid barrier words (GridSync)
  mbl::MinresState* h_state = nullptr;  // pinned host, 4 slots
  double* h_red = nullptr;              // pinned host, 256 doubles
  hipEvent_t ev[2] = {nullptr, nullptr};
  // captured MINRES iterations per vector type (0: FP64, 1: FP32) and the
  // kernel arguments they were captured with
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  std::vector<unsigned char> graph_key[2];
  hipStream_t cap = nullptr;            // capture stream
  int graph_mode = -1;                  // -1: unset (environment), 0: eager, 1: graphs
};

namespace mbl {

// field arguments for a call
FieldArgs make_fields(const mbl_basis_s* b, const double* h_host, double sigma);
bool fields_finite(int L, const double* h_host);

// launch geometry for row (chunk) kernels
int row_grid(const mbl_basis_s* b);
size_t row_lds_bytes(const mbl_basis_s* b);

// ---- kernels launched from other translation units (defined in kernels.hip)
template <typename T>
hipError_t launch_apply(const mbl_basis_s* b, const FieldArgs& F, const T* x, T* y, int mode,
                        double* partials, int* nparts, hipStream_t s);
template <typename T>
hipError_t launch_minres_apply(const mbl_basis_s* b, const FieldArgs& F, const MinresGivens& G,
                               const T* q, T* p, double* partials, const Defl& D, hipStream_t s);
hipError_t launch_precond(const mbl_basis_s* b, const FieldArgs& F, int kind, const double* z,
                          double* q, hipStream_t s);
hipError_t launch_states(const mbl_basis_s* b, uint32_t* states, hipStream_t s);
hipError_t launch_rank(const mbl_basis_s* b, const uint32_t* states, int64_t count,
                       int64_t* ranks, hipStream_t s);
hipError_t launch_twist(const mbl_basis_s* b, const double* psi, int64_t ld, int nvec,
                        const double* costab, const double* sintab, double* partials, int* nparts,
                        hipStream_t s);
// residual r = b - (H - sigma) x in FP64 with partial sums of r^2 / m_i (M^{-1}-norm)
// and r^2 into partials[2 * g], partials[2 * g + 1]
hipError_t launch_residual(const mbl_basis_s* b, const FieldArgs& F, int precond,
                           const double* rhs, const double* x, double* r, double* partials,
                           int* nparts, hipStream_t s);

// generic dense vector helpers
hipError_t launch_dot(int64_t n, const double* x, const double* y, double* partials, int* nparts,
                      hipStream_t s);
hipError_t launch_reduce(const double* partials, int nparts, int stride, int nvals, double* out,
                         hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y,
                        hipStream_t s);       // y = a x + b y
hipError_t launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s);
hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s);
hipError_t launch_splitmix(int64_t n, uint64_t seed, double* y, hipStream_t s);

// reduce on device and copy nvals results to host (synchronizes the stream)
mbl_status reduce_to_host(mbl_workspace_s* ws, const double* partials, int nparts, int stride,
                          int nvals, double* out_host, hipStream_t s);

// MINRES driver (minres.hip)
mbl_status minres_run(mbl_basis_s* b, const double* h_host, double sigma, const double* rhs,
                      double* x, double tol, int64_t kmax, int precision, int precond,
                      bool x0_zero, mbl_workspace_s* ws, mbl_minres_info* info, hipStream_t s,
                      const double* defl = nullptr, double theta = 0.0);

// host symmetric tridiagonal eigensolver (symmetric QR with Wilkinson shifts)
int tridiag_eig(int k, const double* alpha, const double* beta, double* evals, double* evecs);

// One realization for the streaming batched SI-Lanczos (batched.hip): inputs,
// then outputs.
struct StreamProblem {
  const double* h;      // L fields (host)
  double sigma;         // shift
  double escale;        // energy scale of the stopping rule (> 0)
  int nev;              // pairs kept: the nev nearest sigma, ascending (<= the run's nev)
  uint64_t seed;        // start vector: the SplitMix64 stream of this seed, normalised
  double* evals;        // nev (host)
  double* resid;        // nev explicit residuals (host) or null
  double* z;            // 2 nev twist overlaps (host) or null
  double* evecs_dev;    // n x nev column-major (device)
  int steps = 0, nconv = 0;
  int64_t minres_iters = 0;
  double max_rel = 0.0;
  mbl_status status = MBL_OK;
};

// Alg. 1 for many realizations of one L on the R lanes of a batch workspace,
// each lane running its own Lanczos steps: when a lane's MINRES solve ends,
// its Lanczos step is taken and its next solve starts while the other lanes
// iterate on, and a lane whose realization has converged takes the next one.
// FP64. The workspace's mmax and nevmax bound mmax and nev.
mbl_status bstream_si_lanczos(mbl_basis b, mbl_batch w, StreamProblem* probs, int nprob, int nev,
                              int mmax, double minres_tol, int64_t minres_kmax, double eig_tol,
                              double gap_tol, int precond, hipStream_t s);

}  // namespace mbl
