// Device-side row machinery of the batched form (R realizations of one L in
// lockstep): the interleaved layout, LDS tables, buffer-resource access and
// the row traversal shared by the batched kernels.
#pragma once

#include "rows.h"

namespace mbl {

constexpr int kBWG = 1024;   // threads per workgroup of the batched row kernels
constexpr int kBMaxR = 32;
constexpr int kBGrid = 512;  // upper bound on workgroups (partials per realization)

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// Per-realization MINRES state, double-buffered by iteration parity.
struct BState {
  double beta_prev, beta, c, s, dhat, eps, phi;
  double alpha;                 // alpha_k of the current iteration
  double d_inv_beta, d_delta, d_eps, d_inv_gamma, d_tau;   // d/x update coefficients
  int64_t k;
  int32_t done, bad;
  int32_t fresh;                // a restarted solve: the next Givens step carries this state
  int32_t pad_;
};

struct BatchDev {
  const double* h;     // R x L fields
  const double* c0;    // R: L/4 + (1/2) sum h - sigma
  int R;
  int grid;            // workgroups of the row kernels; 0: one per compute unit (host only)
};

// LDS layout (bytes): lo_rank (2^nlo uint16) at offset 0, so a rank read is
// addressed by (lo << 1) ^ (mask << 1) alone; lo_state (2^nlo uint16); the
// field table lut[(k * 16 + v) * R + r] = sum of h_r over the set bits of
// nibble value v at nibble position k, so a lane reads its realization pair
// with one 16-byte access; c0[R]; reduction scratch; per-realization values
// shared by the workgroup (done flags, MINRES alpha).
__host__ __device__ constexpr size_t blds_bytes(int R, int L, int nlo) {
  return ((size_t)4 << nlo) + (size_t)R * (((L + 3) >> 2) * 16) * sizeof(double) +
         (size_t)R * sizeof(double) + kLdsRed * kBMaxR * sizeof(double) +
         kBMaxR * sizeof(double);
}

struct BTables {
  const unsigned char* rank;  // lo_rank, byte-addressed
  const uint16_t* state;
  const double* lut;          // [nnib][16][R]
  const double* c0;           // [R]
  double* red;                // [waves][R]
  double* shared_r;           // [kBMaxR] per-realization values for the workgroup
  int rsh;                    // log2 R
};

__device__ __forceinline__ BTables bsetup(const DevBasis& B, const BatchDev& Q, unsigned char* smem) {
  const int R = Q.R, nnib = (B.L + 3) >> 2;
  uint16_t* rank = reinterpret_cast<uint16_t*>(smem);
  uint16_t* state = rank + (1u << B.nlo);
  double* lut = reinterpret_cast<double*>(smem + ((size_t)4 << B.nlo));
  double* c0 = lut + (size_t)R * nnib * 16;
  double* red = c0 + R;
  for (int t = threadIdx.x; t < R * nnib * 16; t += blockDim.x) {
    const int r = t % R, kv = t / R, k = kv >> 4, v = kv & 15;
    double acc = 0.0;
    for (int b = 0; b < 4; ++b) {
      const int site = 4 * k + b;
      if (site < B.L && ((v >> b) & 1)) acc += Q.h[r * B.L + site];
    }
    lut[t] = acc;
  }
  for (int t = threadIdx.x; t < R; t += blockDim.x) c0[t] = Q.c0[t];
  const int words = (1 << B.nlo) >> 1;
  const uint32_t* gr = reinterpret_cast<const uint32_t*>(B.lo_rank);
  const uint32_t* gs = reinterpret_cast<const uint32_t*>(B.lo_state);
  uint32_t* sr = reinterpret_cast<uint32_t*>(rank);
  uint32_t* ss = reinterpret_cast<uint32_t*>(state);
  for (int t = threadIdx.x; t < words; t += blockDim.x) {
    sr[t] = gr[t];
    ss[t] = gs[t];
  }
  return BTables{reinterpret_cast<const unsigned char*>(rank), state, lut, c0, red,
                 red + kLdsRed * kBMaxR, 31 - __builtin_clz((unsigned)R)};
}

// a_aa - sigma_r for the lane's realization pair (2p, 2p + 1); the field sum
// is taken nibble by nibble in increasing position, as in the single form.
template <int L>
__device__ __forceinline__ void bdiag2(const BTables& t, int p, uint32_t a, int nanti, double& d0,
                                       double& d1) {
  constexpr int NNIB = (L + 3) >> 2;
  double2 fv[NNIB];
#pragma unroll
  for (int k = 0; k < NNIB; ++k)
    fv[k] = *reinterpret_cast<const double2*>(
        t.lut + ((((uint32_t)k << 4) + ((a >> (4 * k)) & 15u)) << t.rsh) + 2 * p);
  double f0 = 0.0, f1 = 0.0;
#pragma unroll
  for (int k = 0; k < NNIB; ++k) {
    f0 += fv[k].x;
    f1 += fv[k].y;
  }
  d0 = t.c0[2 * p] - 0.5 * (double)nanti - f0;
  d1 = t.c0[2 * p + 1] - 0.5 * (double)nanti - f1;
}

template <int L>
__device__ __forceinline__ int bnanti(uint32_t a) {
  constexpr uint32_t mask = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
  return __popc(a ^ (((a << 1) | (a >> (L - 1))) & mask));
}

// Vector access through buffer resources: the byte offset of an element is a
// 32-bit per-lane part (voffset) plus a wave-uniform part (soffset, a block
// offset), so no 64-bit address arithmetic is needed per gather. Batch
// buffers are below 2^31 bytes.
constexpr int kBufFlags = 0x00020000;   // buffer resource word 3 for gfx9 data formats
constexpr int kStoreStream = 2;         // cache policy of a streaming (nontemporal) store

__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* ptr, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(ptr), (short)0, (int)bytes, kBufFlags);
}

template <typename T> struct BIO;
template <> struct BIO<double> {
  static constexpr int kShift = 4;   // log2 bytes of a pair
  __device__ static __forceinline__ double2 ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, 0);
    double2 d;
    __builtin_memcpy(&d, &u, sizeof(d));
    return d;
  }
  template <int AUX>
  __device__ static __forceinline__ void st(double2 d, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                            uint32_t s) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    U u;
    __builtin_memcpy(&u, &d, sizeof(d));
    __builtin_amdgcn_raw_buffer_store_b128(u, r, (int)v, (int)s, AUX);
  }
};
template <> struct BIO<float> {
  static constexpr int kShift = 3;
  __device__ static __forceinline__ float2 ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0);
    float2 d;
    __builtin_memcpy(&d, &u, sizeof(d));
    return d;
  }
  template <int AUX>
  __device__ static __forceinline__ void st(float2 d, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                            uint32_t s) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    U u;
    __builtin_memcpy(&u, &d, sizeof(d));
    __builtin_amdgcn_raw_buffer_store_b64(u, r, (int)v, (int)s, AUX);
  }
};

// Byte offsets of one row for one lane: rows are 2^rs bytes (R values of
// T), the lane's pair sits at lane_off inside the row.
struct BRowAddr {
  uint32_t rs;        // log2 row bytes
  uint32_t lane_off;  // pair offset inside a row
  uint32_t jv;        // (j << rs) + lane_off: position j in a block
  uint32_t sb;        // block start (uniform), bytes
};

// Off-diagonal sums for the lane's realization pair of one row. Every gather
// is issued before any is summed. A low-bond, boundary or wrap gather is
// predicated per lane (masked lanes cost no memory traffic); hi is uniform in
// the wave, so a high bond that is not antiparallel skips its load for the
// whole wave.
template <typename T, int L, int NLO>
__device__ __forceinline__ void boffdiag(const DevBasis& B, const BTables& t,
                                         __amdgpu_buffer_rsrc_t rx, const BRowAddr& ad,
                                         uint32_t hi, uint32_t lo, double& o0, double& o1) {
  using T2 = typename Pair<T>::type;
  constexpr int NHI = L - NLO;
  constexpr int NLB = NLO - 1 > 0 ? NLO - 1 : 1;
  constexpr int NHB = NHI - 1 > 0 ? NHI - 1 : 1;
  const uint32_t rs = ad.rs;
  const uint32_t hb_bnd = uni(B.hi_off[hi ^ 1u]) << rs;
  const uint32_t hb_wrap = uni(B.hi_off[hi ^ (1u << (NHI - 1))]) << rs;
  uint32_t hb[NHB];
#pragma unroll
  for (int b = 0; b + 1 < NHI; ++b) hb[b] = uni(B.hi_off[hi ^ (3u << b)]) << rs;
  const uint32_t lo2 = lo << 1;
  uint32_t r[NLB];
#pragma unroll
  for (int b = 0; b + 1 < NLO; ++b)
    r[b] = *reinterpret_cast<const uint16_t*>(t.rank + (lo2 ^ (6u << b)));
  const uint32_t r_bnd = *reinterpret_cast<const uint16_t*>(t.rank + (lo2 ^ (2u << (NLO - 1))));
  const uint32_t r_wrap = *reinterpret_cast<const uint16_t*>(t.rank + (lo2 ^ 2u));
  const uint32_t flips = lo ^ (lo >> 1);
  const uint32_t hflips = uni(hi ^ (hi >> 1));
  const T2 zero = {(T)0, (T)0};
  T2 v[NLB];
#pragma unroll
  for (int b = 0; b + 1 < NLO; ++b) {
    v[b] = zero;
    if ((flips >> b) & 1u) v[b] = BIO<T>::ld(rx, (r[b] << rs) + ad.lane_off, ad.sb);
  }
  T2 v_bnd = zero;
  if (((lo >> (NLO - 1)) ^ hi) & 1u) v_bnd = BIO<T>::ld(rx, (r_bnd << rs) + ad.lane_off, hb_bnd);
  T2 vh[NHB];
#pragma unroll
  for (int b = 0; b + 1 < NHI; ++b) {
    vh[b] = zero;
    if ((hflips >> b) & 1u) vh[b] = BIO<T>::ld(rx, ad.jv, hb[b]);
  }
  T2 v_wrap = zero;
  if (((hi >> (NHI - 1)) ^ lo) & 1u) v_wrap = BIO<T>::ld(rx, (r_wrap << rs) + ad.lane_off, hb_wrap);
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int b = 0; b + 1 < NLO; ++b) {
    a0 += (double)v[b].x;
    a1 += (double)v[b].y;
  }
  a0 += (double)v_bnd.x;
  a1 += (double)v_bnd.y;
#pragma unroll
  for (int b = 0; b + 1 < NHI; ++b) {
    a0 += (double)vh[b].x;
    a1 += (double)vh[b].y;
  }
  a0 += (double)v_wrap.x;
  a1 += (double)v_wrap.y;
  o0 = a0;
  o1 = a1;
}

// Visit rows: body(row, hi, lo, j, block0, a, p) for lanes with a valid row.
// The waves of a workgroup cooperate on consecutive chunks: a chunk (up to 64
// rows) needs PR waves of RPW rows each, so one workgroup step covers
// wpg / PR chunks. Workgroups of one XCD sweep that XCD's contiguous slice of
// chunks side by side, so the XCD's live window is about 32 workgroups x 64
// rows and the rows' low-bond and near high-bond neighbours stay in its L2.
template <typename Body>
__device__ __forceinline__ void bfor_rows(const DevBasis& B, const BTables& t, int R, Body body) {
  const uint32_t PR = (uint32_t)R >> 1, RPW = 64 / PR;
  const uint32_t lane = threadIdx.x & 63u;
  const int p = lane % PR;
  const uint32_t slot = lane / PR;
  const uint32_t wpg = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t cps = max(1u, wpg / PR);           // chunks per workgroup step
  const uint32_t my_chunk = wave / PR;              // this wave's chunk in the step
  const uint32_t my_row0 = (wave % PR) * RPW;       // this wave's first row in the chunk
  const bool wave_on = my_chunk < cps;
  const uint32_t G = gridDim.x, nch = (uint32_t)B.nchunks;
  uint32_t c_lo = 0, c_hi = nch, k = blockIdx.x, per = G;
  if (G % kXcds == 0) {
    const uint32_t span = (nch + kXcds - 1) / kXcds;
    c_lo = min(nch, (blockIdx.x % kXcds) * span);
    c_hi = min(nch, c_lo + span);
    k = blockIdx.x / kXcds;
    per = G / kXcds;
  }
  for (uint32_t base = c_lo + k * cps; base < c_hi; base += per * cps) {
    const uint32_t c = base + my_chunk;
    if (!wave_on || c >= c_hi) continue;
    const uint4 ch = B.chunks[c];
    const uint32_t hi = uni(ch.x), j0 = uni(ch.y), cnt = uni(ch.z), row0 = uni(ch.w);
    const uint32_t coff = uni(B.lo_coff[B.half - __popc(hi)]);
    const uint32_t rl = my_row0 + slot;
    if (rl < cnt) {
      const uint32_t j = j0 + rl;
      const uint32_t lo = t.state[coff + j];
      body(row0 + rl, hi, lo, j, row0 - j0, (hi << B.nlo) | lo, p);
    }
  }
}

// Per-realization block reduction of (acc0, acc1) for pair p; thread r < R of
// the workgroup ends with the sum for realization r (returned), others 0.
__device__ __forceinline__ double bblock_sum(double acc0, double acc1, double* red, int R) {
  const int PR = R >> 1;
#pragma unroll
  for (int o = PR; o < 64; o <<= 1) {
    acc0 += __shfl_xor(acc0, o, 64);
    acc1 += __shfl_xor(acc1, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane < PR) {
    red[wave * R + 2 * lane] = acc0;
    red[wave * R + 2 * lane + 1] = acc1;
  }
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < R) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) s += red[w * R + threadIdx.x];
  }
  return s;
}


// Per-realization sums of the G workgroup partials partials[g * R + r], the
// same in every workgroup that calls it: thread t adds g = t / R, t / R +
// nt / R, ... of realization r = t % R; lanes of one realization inside a
// wave are combined by a butterfly, then the waves in index order. Thread
// r < R returns the sum for realization r, the others 0. red: [waves][R].
__device__ __forceinline__ double bsum_combine(double v, int R, double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1)
    if (o >= R) v += __shfl_xor(v, o, 64);
  const int lane = t & 63, wave = t >> 6;
  __syncthreads();
  if (lane < R) red[wave * R + lane] = v;
  __syncthreads();
  double sum = 0.0;
  if (t < R) {
    const int nw = (int)blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) sum += red[w * R + t];
  }
  __syncthreads();
  return sum;
}

__device__ __forceinline__ double bsum_partials(const double* __restrict__ partials, int G, int R,
                                                double* red) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int r = t % R, per = nt / R;
  double v = 0.0;
  for (int g = t / R; g < G; g += per) v += partials[(size_t)g * R + r];
  return bsum_combine(v, R, red);
}

// bsum_partials split in two for kBWG-thread workgroups: the loads, issued
// at kernel entry so that their latency overlaps the LDS table fill, and
// later the same fixed-order sum (G <= kBGrid, R <= kBMaxR).
constexpr int kBPrefetch = kBGrid * kBMaxR / kBWG;
struct BPrefetch {
  double v[kBPrefetch];
};
__device__ __forceinline__ void bprefetch_partials(const double* __restrict__ partials, int G,
                                                   int R, BPrefetch& f) {
  const int t = threadIdx.x, r = t % R, per = kBWG / R;
#pragma unroll
  for (int j = 0; j < kBPrefetch; ++j) {
    const int g = t / R + j * per;
    f.v[j] = g < G ? partials[(size_t)g * R + r] : 0.0;
  }
}
__device__ __forceinline__ double bsum_prefetched(const BPrefetch& f, int G, int R, double* red) {
  const int t = threadIdx.x, per = kBWG / R;
  double v = 0.0;
#pragma unroll
  for (int j = 0; j < kBPrefetch; ++j)
    if (t / R + j * per < G) v += f.v[j];
  return bsum_combine(v, R, red);
}

// One step of the MINRES scalar recurrence of Alg. 2 for one realization:
// from the state after iteration k - 1, alpha_k and q_{k+1} . z_{k+1}, the
// state after iteration k (beta_{k+1}, the Givens rotation, the d/x
// coefficients of iteration k, phi_k, done). A done state is carried with a
// zero step. A fresh state (a solve restarted for one realization while the
// others run on) is carried unchanged, as the state after the iteration
// before its first one.
__device__ __forceinline__ BState bgivens_step(const BState& si, double alpha, double qz,
                                               double tol, int64_t kmax) {
  BState so = si;
  if (si.fresh) {
    so.fresh = 0;
    return so;
  }
  if (si.done) {
    so.d_tau = 0.0;
    return so;
  }
  const double beta = si.beta;
  const double beta_next = sqrt(qz);
  const double delta = si.c * si.dhat + si.s * alpha;
  const double gamma_hat = -si.s * si.dhat + si.c * alpha;
  const double eps_next = si.s * beta_next;
  const double dhat_next = si.c * beta_next;
  const double gamma = sqrt(gamma_hat * gamma_hat + beta_next * beta_next);
  const double c = gamma_hat / gamma, s = beta_next / gamma;
  const double tau = c * si.phi, phi = -s * si.phi;
  so.alpha = alpha;
  so.d_inv_beta = 1.0 / beta;
  so.d_delta = delta;
  so.d_eps = si.eps;
  so.d_inv_gamma = 1.0 / gamma;
  so.d_tau = tau;
  so.beta_prev = beta;
  so.beta = beta_next;
  so.c = c;
  so.s = s;
  so.dhat = dhat_next;
  so.eps = eps_next;
  so.phi = phi;
  so.k = si.k + 1;
  so.bad = !isfinite(phi) || !isfinite(alpha) || !isfinite(beta_next);
  so.done = so.bad || !(fabs(phi) >= tol && so.k < kmax);
  return so;
}

// Arguments of the Givens step of iteration k - 1 that the MINRES product of
// iteration k computes first (every workgroup the same; workgroup 0 stores it).
struct BGivens {
  const double* part2;   // q_k . z_k partials of the previous z/q update
  const double* alpha;   // alpha_{k-1} per realization
  const BState* Sprev;   // state after iteration k - 2
  BState* Scur;          // receives the state after iteration k - 1
  int G;
  int active;            // 0 at k = 1: Scur already holds the initial state
  double tol;
  int64_t kmax;
};

}  // namespace mbl
