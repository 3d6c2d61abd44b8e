// C ABI entry points: argument validation, basis tables, workspace, and the
// calls into the kernel drivers. No exception crosses the ABI.
#include "mbl_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

namespace mbl {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

bool fields_finite(int L, const double* h) {
  for (int j = 0; j < L; ++j)
    if (!std::isfinite(h[j])) return false;
  return true;
}

FieldArgs make_fields(const mbl_basis_s* b, const double* h, double sigma) {
  FieldArgs F{};
  double sh = 0.0;
  for (int j = 0; j < b->L; ++j) {
    F.h[j] = h[j];
    sh += h[j];
  }
  F.c0 = 0.25 * b->L + 0.5 * sh - sigma;
  F.sigma = sigma;
  return F;
}

// declared in lanczos.hip
mbl_status si_lanczos_run(mbl_basis_s* b, const double* h, double sigma, int nev, int mmax,
                          double minres_tol, int64_t minres_kmax, double eig_tol, double gap_tol,
                          double escale, const double* v0, uint64_t seed, int precision,
                          int precond, mbl_workspace_s* ws, double* evals, double* evecs,
                          int64_t ldu, double* resid, mbl_si_info* info, hipStream_t s);
mbl_status sigma_midpoint_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* h,
                              double rel_tol, int mmax, double* emin, double* emax,
                              hipStream_t s);
mbl_status twist_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* psi, int64_t ld,
                     int nvec, double* z, hipStream_t s);
mbl_status eig_residual_run(mbl_basis_s* b, mbl_workspace_s* ws, const double* h,
                            const double* E, const double* psi, int64_t ld, int nvec,
                            double* resid, hipStream_t s);
// declared in schmidt.hip
mbl_status entropy_run(mbl_basis_s* b, const double* psi, int64_t ld, int64_t rstride, int R,
                       int nvec, int la, double* S, hipStream_t s);
mbl_status spacing_ratio_run(int count, const double* E, double* r, double* r_mean);
mbl_status symmetric_eigenvalues_run(int m, const double* A, double* w);

static uint64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

// Fraction of lanes doing useful work for a given split.
static double lane_efficiency(int L, int nlo) {
  const int half = L / 2, nhi = L - nlo;
  uint64_t rows = 0, lanes = 0;
  for (int c_hi = 0; c_hi <= nhi; ++c_hi) {
    const int c_lo = half - c_hi;
    if (c_lo < 0 || c_lo > nlo) continue;
    const uint64_t bs = binom(nlo, c_lo), nb = binom(nhi, c_hi);
    rows += nb * bs;
    lanes += nb * ((bs + kChunk - 1) / kChunk) * kChunk;
  }
  return lanes ? (double)rows / (double)lanes : 0.0;
}

static int default_lo_bits(int L) {
  int best = std::max(1, L / 2);
  double be = -1;
  for (int nlo = std::max(1, L / 2 - 1); nlo <= std::min(kMaxLoBits, L - 1); ++nlo) {
    if (nlo > L / 2 + 3) break;
    const double e = lane_efficiency(L, nlo);
    if (e > be + 1e-3) {
      be = e;
      best = nlo;
    }
  }
  return best;
}

static void free_basis(mbl_basis_s* b) {
  if (!b) return;
  hipFree(b->d_hi_off);
  hipFree(b->d_lo_rank);
  hipFree(b->d_lo_state);
  hipFree(b->d_lo_coff);
  hipFree(b->d_chunks);
  delete b;
}

template <typename T>
static mbl_status dalloc(T** p, size_t count, int64_t* bytes) {
  const size_t nb = std::max<size_t>(count, 1) * sizeof(T);
  if (hipMalloc((void**)p, nb) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(nb) + " bytes failed");
    return MBL_ERR_NOMEM;
  }
  if (bytes) *bytes += (int64_t)nb;
  return MBL_OK;
}

static void free_ws(mbl_workspace_s* w) {
  if (!w) return;
  for (int i = 0; i < 2; ++i) {
    hipFree(w->z[i]);
    hipFree(w->d[i]);
  }
  for (int i = 0; i < 3; ++i) hipFree(w->q[i]);
  hipFree(w->alpha);
  hipFree(w->p);
  hipFree(w->e);
  hipFree(w->r64);
  hipFree(w->t64);
  hipFree(w->V);
  hipFree(w->w);
  hipFree(w->x);
  hipFree(w->coef);
  hipFree(w->ycoef);
  hipFree(w->partials1);
  hipFree(w->partials2);
  hipFree(w->partials3);
  hipFree(w->red_out);
  hipFree(w->state);
  hipFree(w->sync);
  if (w->h_state) hipHostFree(w->h_state);
  if (w->h_red) hipHostFree(w->h_red);
  for (int i = 0; i < 2; ++i) {
    if (w->ev[i]) hipEventDestroy(w->ev[i]);
    if (w->graph[i]) hipGraphExecDestroy(w->graph[i]);
  }
  if (w->cap) hipStreamDestroy(w->cap);
  delete w;
}

// minres_vectors: allocate the MINRES recurrence vectors (8 bytes per
// element, usable by both precisions)
static mbl_status create_ws(mbl_basis_s* b, int mmax, int precision, bool minres_vectors,
                            mbl_workspace_s** out) {
  mbl_workspace_s* w = new (std::nothrow) mbl_workspace_s();
  if (!w) {
    set_error("host allocation failed");
    return MBL_ERR_NOMEM;
  }
  w->basis = b;
  w->mmax = mmax;
  w->precision = precision;
  w->n = b->n;
  const size_t n = (size_t)b->n;
  mbl_status st = MBL_OK;
  auto A = [&](auto** p, size_t count) {
    if (st == MBL_OK) st = dalloc(p, count, &w->bytes);
  };
  if (minres_vectors) {
    for (int i = 0; i < 2; ++i) {
      A((double**)&w->z[i], n);
      A((double**)&w->d[i], n);
    }
    for (int i = 0; i < 3; ++i) A((double**)&w->q[i], n);
    A((double**)&w->p, n);
    A((double**)&w->e, n);
  }
  A(&w->r64, n);
  A(&w->t64, n);
  A(&w->w, n);
  A(&w->x, n);
  if (mmax > 0) A(&w->V, n * (size_t)(mmax + 1));
  A(&w->coef, (size_t)mmax + 64);
  A(&w->ycoef, std::max<size_t>(64, (size_t)(mmax + 1) * (size_t)(mmax + 1)));
  A(&w->partials1, (size_t)kMaxPartials * 64);
  A(&w->partials2, std::max<size_t>((size_t)kMaxPartials * 64, (size_t)512 * (mmax + 1)));
  A(&w->partials3, (size_t)kMaxPartials);
  A(&w->red_out, 256);
  A(&w->state, 2);
  A(&w->alpha, 2);
  A(&w->sync, kSyncWords);
  if (st == MBL_OK) {
    if (hipHostMalloc((void**)&w->h_state, 4 * sizeof(MinresState)) != hipSuccess ||
        hipHostMalloc((void**)&w->h_red, 256 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      st = MBL_ERR_NOMEM;
    }
  }
  if (st == MBL_OK) {
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&w->ev[i], hipEventDisableTiming) != hipSuccess) {
        set_error("hipEventCreate failed");
        st = MBL_ERR_HIP;
      }
  }
  if (st != MBL_OK) {
    free_ws(w);
    return st;
  }
  *out = w;
  return MBL_OK;
}

// per-basis scratch workspace for calls that take none (created on first use)
struct ScratchHolder {
  std::mutex mu;
  mbl_workspace_s* ws = nullptr;
};

}  // namespace mbl

using namespace mbl;

struct BasisExtra {
  ScratchHolder scratch;
};

// the scratch holder lives beside the basis; keyed by pointer
#include <unordered_map>
static std::mutex g_extra_mu;
static std::unordered_map<const mbl_basis_s*, BasisExtra*> g_extra;

static BasisExtra* extra_of(const mbl_basis_s* b) {
  std::lock_guard<std::mutex> lk(g_extra_mu);
  auto it = g_extra.find(b);
  if (it != g_extra.end()) return it->second;
  auto* e = new BasisExtra();
  g_extra[b] = e;
  return e;
}

static mbl_status with_scratch(mbl_basis_s* b, mbl_workspace_s** ws, std::unique_lock<std::mutex>* lk) {
  BasisExtra* e = extra_of(b);
  *lk = std::unique_lock<std::mutex>(e->scratch.mu);
  if (!e->scratch.ws) MBL_TRY(create_ws(b, 0, MBL_FP64, false, &e->scratch.ws));
  *ws = e->scratch.ws;
  return MBL_OK;
}

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

const char* mbl_last_error(void) { return g_err.c_str(); }
const char* mbl_version(void) { return "mbl-mi355x 0.1 (gfx950)"; }

mbl_status mbl_build_basis(int L, int lo_bits, void* stream, mbl_basis* out) {
  clear_error();
  MBL_ARG(out != nullptr, "out is NULL");
  MBL_ARG(L >= 4 && L <= kMaxL && L % 2 == 0, "L must be even with 4 <= L <= 32");
  MBL_ARG(lo_bits == 0 || (lo_bits >= 1 && lo_bits <= kMaxLoBits && lo_bits < L),
          "lo_bits must be 0 or in [1, min(13, L-1)]");
  const int nlo = lo_bits ? lo_bits : default_lo_bits(L);
  const int nhi = L - nlo, half = L / 2;
  const uint32_t nlo_states = 1u << nlo;
  std::vector<uint16_t> lo_state(nlo_states), lo_rank(nlo_states);
  std::vector<uint32_t> lo_coff(nlo + 2, 0);
  {
    uint32_t pos = 0;
    for (int c = 0; c <= nlo; ++c) {
      lo_coff[c] = pos;
      for (uint32_t v = 0; v < nlo_states; ++v)
        if (__builtin_popcount(v) == c) {
          lo_state[pos] = (uint16_t)v;
          lo_rank[v] = (uint16_t)(pos - lo_coff[c]);
          ++pos;
        }
    }
    lo_coff[nlo + 1] = pos;
  }
  const size_t nhi_states = (size_t)1 << nhi;
  std::vector<uint32_t> hi_off(nhi_states, 0xffffffffu);
  std::vector<uint4> chunks;
  uint64_t running = 0;
  for (size_t hi = 0; hi < nhi_states; ++hi) {
    const int c_lo = half - __builtin_popcountll(hi);
    if (c_lo < 0 || c_lo > nlo) continue;
    const uint64_t bs = binom(nlo, c_lo);
    hi_off[hi] = (uint32_t)running;
    for (uint64_t j0 = 0; j0 < bs; j0 += kChunk)
      chunks.push_back(make_uint4((uint32_t)hi, (uint32_t)j0,
                                  (uint32_t)std::min<uint64_t>(kChunk, bs - j0),
                                  (uint32_t)(running + j0)));
    running += bs;
  }
  if (running != binom(L, half)) {
    set_error("internal: sector dimension mismatch");
    return MBL_ERR_ARG;
  }
  mbl_basis_s* b = new (std::nothrow) mbl_basis_s();
  if (!b) {
    set_error("host allocation failed");
    return MBL_ERR_NOMEM;
  }
  b->L = L;
  b->nlo = nlo;
  b->nhi = nhi;
  b->half = half;
  b->n = (int64_t)running;
  b->nchunks = (int)chunks.size();
  hipGetDevice(&b->device);
  mbl_status st = MBL_OK;
  if (st == MBL_OK) st = dalloc(&b->d_hi_off, nhi_states, nullptr);
  if (st == MBL_OK) st = dalloc(&b->d_lo_rank, nlo_states, nullptr);
  if (st == MBL_OK) st = dalloc(&b->d_lo_state, nlo_states, nullptr);
  if (st == MBL_OK) st = dalloc(&b->d_lo_coff, lo_coff.size(), nullptr);
  if (st == MBL_OK) st = dalloc(&b->d_chunks, chunks.size(), nullptr);
  if (st != MBL_OK) {
    free_basis(b);
    return st;
  }
  hipStream_t s = S(stream);
  hipError_t e = hipSuccess;
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_hi_off, hi_off.data(), sizeof(uint32_t) * nhi_states,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_lo_rank, lo_rank.data(), sizeof(uint16_t) * nlo_states,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_lo_state, lo_state.data(), sizeof(uint16_t) * nlo_states,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_lo_coff, lo_coff.data(), sizeof(uint32_t) * lo_coff.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_chunks, chunks.data(), sizeof(uint4) * chunks.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error(std::string("basis upload: ") + hipGetErrorString(e));
    free_basis(b);
    return MBL_ERR_HIP;
  }
  *out = b;
  return MBL_OK;
}

void mbl_basis_free(mbl_basis b) {
  if (!b) return;
  {
    std::lock_guard<std::mutex> lk(g_extra_mu);
    auto it = g_extra.find(b);
    if (it != g_extra.end()) {
      free_ws(it->second->scratch.ws);
      delete it->second;
      g_extra.erase(it);
    }
  }
  free_basis(b);
}

mbl_status mbl_basis_dim(mbl_basis b, int64_t* n) {
  clear_error();
  MBL_ARG(b && n, "NULL argument");
  *n = b->n;
  return MBL_OK;
}

mbl_status mbl_basis_lo_bits(mbl_basis b, int* lo_bits) {
  clear_error();
  MBL_ARG(b && lo_bits, "NULL argument");
  *lo_bits = b->nlo;
  return MBL_OK;
}

mbl_status mbl_basis_states(mbl_basis b, uint32_t* states_dev, void* stream) {
  clear_error();
  MBL_ARG(b && states_dev, "NULL argument");
  MBL_HIP(launch_states(b, states_dev, S(stream)));
  return MBL_OK;
}

mbl_status mbl_basis_rank(mbl_basis b, const uint32_t* states_dev, int64_t count,
                          int64_t* ranks_dev, void* stream) {
  clear_error();
  MBL_ARG(b && count >= 0, "NULL basis or negative count");
  MBL_ARG(count == 0 || (states_dev && ranks_dev), "NULL buffer");
  MBL_HIP(launch_rank(b, states_dev, count, ranks_dev, S(stream)));
  return MBL_OK;
}

mbl_status mbl_workspace_create(mbl_basis b, int mmax, int precision, mbl_workspace* ws) {
  clear_error();
  MBL_ARG(b && ws, "NULL argument");
  MBL_ARG(mmax >= 0 && mmax <= kMaxLanczos, "mmax must be in [0, 1000]");
  MBL_ARG(precision == MBL_FP64 || precision == MBL_FP32_INNER, "unknown precision");
  return create_ws(b, mmax, precision, true, ws);
}

void mbl_workspace_free(mbl_workspace ws) { free_ws(ws); }

mbl_status mbl_workspace_bytes(mbl_workspace ws, int64_t* bytes) {
  clear_error();
  MBL_ARG(ws && bytes, "NULL argument");
  *bytes = ws->bytes;
  return MBL_OK;
}

mbl_status mbl_apply_H(mbl_basis b, const double* h_host, double sigma, const double* x_dev,
                       double* y_dev, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && x_dev && y_dev, "NULL argument");
  MBL_ARG(x_dev != y_dev, "x and y must not alias");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(sigma), "non-finite h or sigma");
  MBL_HIP(launch_apply<double>(b, make_fields(b, h_host, sigma), x_dev, y_dev, 0, nullptr,
                               nullptr, S(stream)));
  return MBL_OK;
}

mbl_status mbl_apply_H_f32(mbl_basis b, const double* h_host, double sigma, const float* x_dev,
                           float* y_dev, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && x_dev && y_dev, "NULL argument");
  MBL_ARG(x_dev != y_dev, "x and y must not alias");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(sigma), "non-finite h or sigma");
  MBL_HIP(launch_apply<float>(b, make_fields(b, h_host, sigma), x_dev, y_dev, 0, nullptr, nullptr,
                              S(stream)));
  return MBL_OK;
}

mbl_status mbl_precond_apply(mbl_basis b, const double* h_host, double sigma, int precond,
                             const double* z_dev, double* q_dev, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && z_dev && q_dev, "NULL argument");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(sigma), "non-finite h or sigma");
  MBL_HIP(launch_precond(b, make_fields(b, h_host, sigma), precond, z_dev, q_dev, S(stream)));
  return MBL_OK;
}

mbl_status mbl_minres_solve(mbl_basis b, const double* h_host, double sigma,
                            const double* rhs_dev, double* x_dev, double tol, int64_t kmax,
                            int precision, int precond, mbl_workspace ws, mbl_minres_info* info,
                            void* stream) {
  clear_error();
  MBL_ARG(b && h_host && rhs_dev && x_dev && ws, "NULL argument");
  MBL_ARG(ws->basis == b, "workspace belongs to another basis");
  MBL_ARG(rhs_dev != x_dev, "rhs and x must not alias");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(sigma), "non-finite h or sigma");
  MBL_ARG(tol > 0 && std::isfinite(tol), "tol must be positive");
  MBL_ARG(kmax >= 1, "kmax must be >= 1");
  MBL_ARG(precision == MBL_FP64 || precision == MBL_FP32_INNER, "unknown precision");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  return minres_run(b, h_host, sigma, rhs_dev, x_dev, tol, kmax, precision, precond, false, ws,
                    info, S(stream));
}

mbl_status mbl_si_lanczos(mbl_basis b, const double* h_host, double sigma, int nev, int mmax,
                          double minres_tol, int64_t minres_kmax, double eig_tol, double gap_tol,
                          double escale, const double* v0_dev, uint64_t seed, int precision,
                          int precond, mbl_workspace ws, double* evals_host, double* evecs_dev,
                          int64_t ld, double* resid_host, mbl_si_info* info, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && ws && evals_host && evecs_dev, "NULL argument");
  MBL_ARG(ws->basis == b, "workspace belongs to another basis");
  MBL_ARG(fields_finite(b->L, h_host) && std::isfinite(sigma), "non-finite h or sigma");
  MBL_ARG(nev >= 1 && nev <= b->n, "nev must be in [1, n]");
  MBL_ARG(mmax >= nev && mmax <= ws->mmax, "need nev <= mmax <= workspace mmax");
  MBL_ARG(mmax <= b->n, "mmax must not exceed n");
  MBL_ARG(minres_tol > 0 && minres_kmax >= 1, "bad MINRES tolerance or kmax");
  MBL_ARG(eig_tol > 0 && std::isfinite(eig_tol), "eig_tol must be positive");
  MBL_ARG(ld >= b->n, "ld must be >= n");
  MBL_ARG(precision == MBL_FP64 || precision == MBL_FP32_INNER, "unknown precision");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  return si_lanczos_run(b, h_host, sigma, nev, mmax, minres_tol, minres_kmax, eig_tol, gap_tol,
                        escale, v0_dev, seed, precision, precond, ws, evals_host, evecs_dev, ld,
                        resid_host, info, S(stream));
}

mbl_status mbl_twist_expect(mbl_basis b, const double* psi_dev, int64_t ld, int nvec,
                            double* z_host, void* stream) {
  clear_error();
  MBL_ARG(b && psi_dev && z_host, "NULL argument");
  MBL_ARG(nvec >= 1 && ld >= b->n, "need nvec >= 1 and ld >= n");
  mbl_workspace_s* ws = nullptr;
  std::unique_lock<std::mutex> lk;
  MBL_TRY(with_scratch(b, &ws, &lk));
  return twist_run(b, ws, psi_dev, ld, nvec, z_host, S(stream));
}

mbl_status mbl_entanglement_entropy(mbl_basis b, const double* psi_dev, int64_t ld, int nvec,
                                    int la, double* S_host, void* stream) {
  clear_error();
  MBL_ARG(b && psi_dev && S_host, "NULL argument");
  MBL_ARG(nvec >= 1 && ld >= b->n, "need nvec >= 1 and ld >= n");
  MBL_ARG(la >= 1 && la <= b->L - 1, "need 1 <= la <= L - 1");
  return entropy_run(b, psi_dev, ld, 1, 1, nvec, la, S_host, S(stream));
}

mbl_status mbl_entanglement_entropy_interleaved(mbl_basis b, const double* psi_dev, int R,
                                                int nvec, int la, double* S_host, void* stream) {
  clear_error();
  MBL_ARG(b && psi_dev && S_host, "NULL argument");
  MBL_ARG(R >= 1 && nvec >= 1, "need R >= 1 and nvec >= 1");
  MBL_ARG((int64_t)R * nvec <= (int64_t)1 << 30, "R * nvec too large");
  MBL_ARG(la >= 1 && la <= b->L - 1, "need 1 <= la <= L - 1");
  std::vector<double> Sv((size_t)R * nvec);
  MBL_TRY(entropy_run(b, psi_dev, b->n * (int64_t)R, R, R, R * nvec, la, Sv.data(), S(stream)));
  for (int t = 0; t < nvec; ++t)
    for (int r = 0; r < R; ++r) S_host[(size_t)r * nvec + t] = Sv[(size_t)t * R + r];
  return MBL_OK;
}

mbl_status mbl_symmetric_eigenvalues(int m, const double* a_host, double* w_host) {
  clear_error();
  MBL_ARG(a_host && w_host, "NULL argument");
  MBL_ARG(m >= 1 && m <= 20000, "need 1 <= m <= 20000");
  for (size_t i = 0; i < (size_t)m * m; ++i) MBL_ARG(std::isfinite(a_host[i]), "non-finite entry");
  return symmetric_eigenvalues_run(m, a_host, w_host);
}

mbl_status mbl_spacing_ratio(int count, const double* evals_host, double* r_host,
                             double* r_mean) {
  clear_error();
  MBL_ARG(evals_host && r_mean, "NULL argument");
  MBL_ARG(count >= 3, "need at least 3 eigenvalues");
  for (int i = 0; i < count; ++i) MBL_ARG(std::isfinite(evals_host[i]), "non-finite eigenvalue");
  return spacing_ratio_run(count, evals_host, r_host, r_mean);
}

mbl_status mbl_eig_residual(mbl_basis b, const double* h_host, const double* E_host,
                            const double* psi_dev, int64_t ld, int nvec, double* resid_host,
                            void* stream) {
  clear_error();
  MBL_ARG(b && h_host && E_host && psi_dev && resid_host, "NULL argument");
  MBL_ARG(nvec >= 1 && ld >= b->n, "need nvec >= 1 and ld >= n");
  MBL_ARG(fields_finite(b->L, h_host), "non-finite h");
  mbl_workspace_s* ws = nullptr;
  std::unique_lock<std::mutex> lk;
  MBL_TRY(with_scratch(b, &ws, &lk));
  return eig_residual_run(b, ws, h_host, E_host, psi_dev, ld, nvec, resid_host, S(stream));
}

mbl_status mbl_sigma_midpoint(mbl_basis b, const double* h_host, double rel_tol, int mmax,
                              double* emin, double* emax, double* sigma, void* stream) {
  clear_error();
  MBL_ARG(b && h_host && emin && emax && sigma, "NULL argument");
  MBL_ARG(fields_finite(b->L, h_host), "non-finite h");
  MBL_ARG(rel_tol > 0, "rel_tol must be positive");
  if (mmax <= 0) mmax = 300;
  mbl_workspace_s* ws = nullptr;
  std::unique_lock<std::mutex> lk;
  MBL_TRY(with_scratch(b, &ws, &lk));
  mbl_status st = sigma_midpoint_run(b, ws, h_host, rel_tol, mmax, emin, emax, S(stream));
  if (st < 0) return st;
  *sigma = 0.5 * (*emin + *emax);
  if (st == MBL_WARN_NOCONV) set_error("extremal eigenvalues not converged within mmax steps");
  return st;
}

mbl_status mbl_dot(int64_t n, const double* x_dev, const double* y_dev, double* out_host,
                   void* stream) {
  clear_error();
  MBL_ARG(n >= 0 && out_host, "bad argument");
  MBL_ARG(n == 0 || (x_dev && y_dev), "NULL buffer");
  if (n == 0) {
    *out_host = 0.0;
    return MBL_OK;
  }
  static std::mutex mu;
  static double* parts = nullptr;
  static double* red = nullptr;
  static double* hred = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!parts) {
    MBL_HIP(hipMalloc((void**)&parts, sizeof(double) * 1024));
    MBL_HIP(hipMalloc((void**)&red, sizeof(double) * 8));
    MBL_HIP(hipHostMalloc((void**)&hred, sizeof(double) * 8));
  }
  hipStream_t s = S(stream);
  int np = 0;
  MBL_HIP(launch_dot(n, x_dev, y_dev, parts, &np, s));
  MBL_HIP(launch_reduce(parts, np, 1, 1, red, s));
  MBL_HIP(hipMemcpyAsync(hred, red, sizeof(double), hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  *out_host = hred[0];
  return MBL_OK;
}

mbl_status mbl_tridiag_eig(int k, const double* alpha, const double* beta, double* evals,
                           double* evecs) {
  clear_error();
  MBL_ARG(k >= 1 && alpha && evals && evecs && (k == 1 || beta), "bad argument");
  if (tridiag_eig(k, alpha, beta, evals, evecs) != 0) {
    set_error("tridiagonal eigensolver did not converge");
    return MBL_ERR_NUMERIC;
  }
  return MBL_OK;
}

}  // extern "C"
