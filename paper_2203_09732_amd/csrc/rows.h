// Device-side row machinery shared by the kernels: the (high, low) block
// decomposition of the S^z = 0 sector, the LDS tables, the diagonal of
// Eq. (1) and the spin-swap neighbours of a row.
//
// A state a = (hi << nlo) | lo. A chunk (up to 64 consecutive rows of one
// block) is one wavefront, one row per lane; hi is uniform in the wave.
//
// Two forms of the off-diagonal gather share one contract:
//  * RowOps<T, L, NLO> with compile-time L and NLO: every bond loop is
//    unrolled, all neighbour indices are formed first (scalar block offsets,
//    then the LDS rank reads), then all gathers are issued (predicated on the
//    bond being antiparallel) and only then summed, so a row costs one
//    memory latency instead of one per bond;
//  * RowOps<T, 0, 0>: runtime L and nlo, for splits without an instance.
// Both sum the neighbours in the same order: low bonds b = 0..nlo-2, the
// bond across the split, high bonds, then the periodic bond.
#pragma once

#include "mbl_internal.h"

namespace mbl {

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup, returned to every thread; red holds one double per
// wave. Fixed order: butterfly inside the wave, then waves in index order.
__device__ __forceinline__ double block_sum_all(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// every workgroup: the same fixed-order sum of P partials
__device__ __forceinline__ double reduce_partials(const double* __restrict__ p, int P,
                                                  double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < P; i += blockDim.x) v += p[i];
  return block_sum_all(v, red);
}

// reduce_partials split in two for kWG-thread workgroups: the loads, issued
// at kernel entry so that their latency overlaps the LDS table fill, and
// later the same fixed-order sum (P <= kMaxPartials)
struct PartialsPrefetch {
  double v[kMaxPartials / kWG];
};
__device__ __forceinline__ void prefetch_partials(const double* __restrict__ p, int P,
                                                  PartialsPrefetch& f) {
#pragma unroll
  for (int j = 0; j < kMaxPartials / kWG; ++j) {
    const int i = (int)threadIdx.x + j * kWG;
    f.v[j] = i < P ? p[i] : 0.0;
  }
}
__device__ __forceinline__ double reduce_prefetched(const PartialsPrefetch& f, int P,
                                                    double* red) {
  double v = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxPartials / kWG; ++j)
    if ((int)threadIdx.x + j * kWG < P) v += f.v[j];
  return block_sum_all(v, red);
}

constexpr int kLdsLut = 128;   // doubles: field table, 16 entries per nibble, 8 nibbles
constexpr int kLdsRed = 16;    // doubles: reduction scratch (up to 16 waves)

struct RowTables {
  const double* lut;       // F over a nibble, per nibble position
  double* red;             // reduction scratch
  const uint16_t* rank;    // lo_rank in LDS
  const uint16_t* state;   // lo_state in LDS
};

__host__ __device__ constexpr size_t row_lds_for(int nlo) {
  return (kLdsLut + kLdsRed) * sizeof(double) + 2 * sizeof(uint16_t) * ((size_t)1 << nlo);
}

// Fill the LDS tables (caller synchronises before use). With a compile-time
// L the field table is formed from kernel-argument loads at fixed offsets.
template <int L = 0>
__device__ __forceinline__ RowTables setup_tables(const DevBasis& B, const FieldArgs& F,
                                                  unsigned char* smem) {
  double* lut = reinterpret_cast<double*>(smem);
  double* red = lut + kLdsLut;
  uint16_t* rank = reinterpret_cast<uint16_t*>(red + kLdsRed);
  uint16_t* state = rank + (1u << B.nlo);
  if constexpr (L > 0) {
    constexpr int NNIB = (L + 3) >> 2;
    if (threadIdx.x < NNIB * 16) {
      const int k = threadIdx.x >> 4, v = threadIdx.x & 15;
      double acc = 0.0;
#pragma unroll
      for (int kk = 0; kk < NNIB; ++kk) {
        if (kk == k) {
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (4 * kk + b < L && ((v >> b) & 1)) acc += F.h[4 * kk + b];
        }
      }
      lut[threadIdx.x] = acc;
    }
  } else {
    const int nnib = (B.L + 3) >> 2;
    for (int t = threadIdx.x; t < nnib * 16; t += blockDim.x) {
      const int k = t >> 4, v = t & 15;
      double acc = 0.0;
      for (int b = 0; b < 4; ++b) {
        const int site = 4 * k + b;
        if (site < B.L && ((v >> b) & 1)) acc += F.h[site];
      }
      lut[t] = acc;
    }
  }
  // both uint16 tables as 16-byte words, four loads in flight per thread
  const int vec = (1 << B.nlo) >> 3;   // uint4 per table (nlo >= 3), else word copy
  if (vec >= 1) {
    const uint4* gr = reinterpret_cast<const uint4*>(B.lo_rank);
    const uint4* gs = reinterpret_cast<const uint4*>(B.lo_state);
    uint4* sr = reinterpret_cast<uint4*>(rank);
    uint4* ss = reinterpret_cast<uint4*>(state);
    for (int t0 = threadIdx.x; t0 < vec; t0 += 2 * blockDim.x) {
      const int t1 = t0 + blockDim.x;
      const uint4 a0 = gr[t0], b0 = gs[t0];
      uint4 a1{}, b1{};
      if (t1 < vec) {
        a1 = gr[t1];
        b1 = gs[t1];
      }
      sr[t0] = a0;
      ss[t0] = b0;
      if (t1 < vec) {
        sr[t1] = a1;
        ss[t1] = b1;
      }
    }
  } else {
    for (int t = threadIdx.x; t < (1 << B.nlo); t += blockDim.x) {
      rank[t] = B.lo_rank[t];
      state[t] = B.lo_state[t];
    }
  }
  return RowTables{lut, red, rank, state};
}

// a_aa - sigma and the number of antiparallel bonds of state a:
// L/4 - N_anti/2 + (1/2) sum h - F(a) - sigma, with c0 = L/4 + (1/2) sum h - sigma.
template <int L>
__device__ __forceinline__ double row_diag(const DevBasis& B, const FieldArgs& F,
                                           const RowTables& t, uint32_t a, int& nanti) {
  const int LL = L ? L : B.L;
  const uint32_t mask = (LL == 32) ? 0xffffffffu : ((1u << LL) - 1u);
  const uint32_t rot = ((a << 1) | (a >> (LL - 1))) & mask;
  nanti = __popc(a ^ rot);
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
  return F.c0 - 0.5 * (double)nanti - f;
}

// preconditioner value m_a (Sec. II): row norm, |a_aa - sigma| or 1
__device__ __forceinline__ double precond_value(int kind, double dsh, int nanti) {
  if (kind == MBL_PRECOND_ROW) return sqrt(dsh * dsh + 0.25 * (double)nanti);
  if (kind == MBL_PRECOND_JACOBI) return fabs(dsh);
  return 1.0;
}

// Sum of x over the states reached by one spin swap on an antiparallel bond.
template <typename T, int L, int NLO>
struct RowOps {
  static_assert(NLO >= 1 && L - NLO >= 1, "split must leave bits on both sides");
  static constexpr int NHI = L - NLO;
  static constexpr int NLB = NLO - 1 > 0 ? NLO - 1 : 1;   // low bonds (array size)
  static constexpr int NHB = NHI - 1 > 0 ? NHI - 1 : 1;   // high bonds (array size)

  __device__ static __forceinline__ double offdiag(const DevBasis& B, const RowTables& t,
                                                   const T* __restrict__ x, uint32_t hi,
                                                   uint32_t lo, uint32_t j, uint32_t block0) {
    // 1. uniform block offsets of the neighbour blocks (scalar loads)
    const uint32_t hb_bnd = uni(B.hi_off[hi ^ 1u]);
    const uint32_t hb_wrap = uni(B.hi_off[hi ^ (1u << (NHI - 1))]);
    uint32_t hb[NHB];
#pragma unroll
    for (int b = 0; b + 1 < NHI; ++b) hb[b] = uni(B.hi_off[hi ^ (3u << b)]);
    // 2. LDS ranks of the low-pattern neighbours
    uint32_t r[NLB];
#pragma unroll
    for (int b = 0; b + 1 < NLO; ++b) r[b] = t.rank[lo ^ (3u << b)];
    const uint32_t r_bnd = t.rank[lo ^ (1u << (NLO - 1))];
    const uint32_t r_wrap = t.rank[lo ^ 1u];
    // 3. all gathers, each predicated on its bond being antiparallel; raw T
    //    values, converted only in the sum so no load is waited on early
    T v[NLB];
#pragma unroll
    for (int b = 0; b + 1 < NLO; ++b) {
      v[b] = (T)0;
      if (((lo >> b) ^ (lo >> (b + 1))) & 1u) v[b] = x[(size_t)block0 + r[b]];
    }
    T v_bnd = (T)0;
    if (((lo >> (NLO - 1)) ^ hi) & 1u) v_bnd = x[(size_t)hb_bnd + r_bnd];
    T vh[NHB];
#pragma unroll
    for (int b = 0; b + 1 < NHI; ++b) {
      vh[b] = (T)0;
      if (((hi >> b) ^ (hi >> (b + 1))) & 1u) vh[b] = x[(size_t)hb[b] + j];
    }
    T v_wrap = (T)0;
    if (((hi >> (NHI - 1)) ^ lo) & 1u) v_wrap = x[(size_t)hb_wrap + r_wrap];
    // 4. fixed-order sum in FP64
    double off = 0.0;
#pragma unroll
    for (int b = 0; b + 1 < NLO; ++b) off += (double)v[b];
    off += (double)v_bnd;
#pragma unroll
    for (int b = 0; b + 1 < NHI; ++b) off += (double)vh[b];
    off += (double)v_wrap;
    return off;
  }
};

template <typename T>
struct RowOps<T, 0, 0> {
  __device__ static __forceinline__ double offdiag(const DevBasis& B, const RowTables& t,
                                                   const T* __restrict__ x, uint32_t hi,
                                                   uint32_t lo, uint32_t j, uint32_t block0) {
    const int nlo = B.nlo, nhi = B.nhi;
    double off = 0.0;
    for (int b = 0; b + 1 < nlo; ++b)
      if (((lo >> b) ^ (lo >> (b + 1))) & 1u) off += (double)x[(size_t)block0 + t.rank[lo ^ (3u << b)]];
    {
      const uint32_t hb = uni(B.hi_off[hi ^ 1u]);
      if (((lo >> (nlo - 1)) ^ hi) & 1u)
        off += (double)x[(size_t)hb + t.rank[lo ^ (1u << (nlo - 1))]];
    }
    for (int b = 0; b + 1 < nhi; ++b)
      if (((hi >> b) ^ (hi >> (b + 1))) & 1u) {
        const uint32_t hb = uni(B.hi_off[hi ^ (3u << b)]);
        off += (double)x[(size_t)hb + j];
      }
    {
      const uint32_t hb = uni(B.hi_off[hi ^ (1u << (nhi - 1))]);
      if (((hi >> (nhi - 1)) ^ lo) & 1u) off += (double)x[(size_t)hb + t.rank[lo ^ 1u]];
    }
    return off;
  }
};

// Chunks c = first, first + stride, ... of this wave; body(row, hi, lo, j, block0, a)
// for the valid lanes.
template <typename Body>
__device__ __forceinline__ void for_rows_range(const DevBasis& B, const RowTables& t,
                                               uint32_t first, uint32_t stride, Body body) {
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t c = first; c < (uint32_t)B.nchunks; c += stride) {
    const uint4 ch = B.chunks[c];
    const uint32_t hi = uni(ch.x), j0 = uni(ch.y), cnt = uni(ch.z), row0 = uni(ch.w);
    const uint32_t coff = uni(B.lo_coff[B.half - __popc(hi)]);
    if (lane < cnt) {
      const uint32_t j = j0 + lane;
      const uint32_t lo = t.state[coff + j];
      body(row0 + lane, hi, lo, j, row0 - j0, (hi << B.nlo) | lo);
    }
  }
}

// XCD-aware placement. Workgroups are dispatched round-robin over the 8 XCDs
// (workgroup b runs on XCD b % 8), each XCD with its own L2. XCD x takes the
// x-th contiguous eighth of the chunks, so the rows of a block and the
// nearby neighbour blocks are read through one L2.
constexpr int kXcds = 8;
// Walk of this workgroup's chunks: the XCD's slice of chunks is swept by all
// of its workgroups together (grid-stride inside the slice), so at any time
// one XCD works on one window of the state space and its L2 holds the window
// and its near neighbour blocks. Calls body(c) for each chunk of this wave.
template <typename F>
__device__ __forceinline__ void for_chunks(int nchunks, F f) {
  const uint32_t G = gridDim.x, wpg = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  if (G % kXcds) {
    for (uint32_t c = blockIdx.x * wpg + wave; c < (uint32_t)nchunks; c += G * wpg) f(c);
    return;
  }
  const uint32_t per_xcd = G / kXcds;
  const uint32_t xcd = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
  const uint32_t span = ((uint32_t)nchunks + kXcds - 1) / kXcds;
  const uint32_t c_lo = min((uint32_t)nchunks, xcd * span);
  const uint32_t c_hi = min((uint32_t)nchunks, c_lo + span);
  for (uint32_t c = c_lo + k * wpg + wave; c < c_hi; c += per_xcd * wpg) f(c);
}

template <typename Body>
__device__ __forceinline__ void for_rows(const DevBasis& B, const RowTables& t, Body body) {
  const uint32_t lane = threadIdx.x & 63u;
  for_chunks(B.nchunks, [&](uint32_t c) {
    const uint4 ch = B.chunks[c];
    const uint32_t hi = uni(ch.x), j0 = uni(ch.y), cnt = uni(ch.z), row0 = uni(ch.w);
    const uint32_t coff = uni(B.lo_coff[B.half - __popc(hi)]);
    if (lane < cnt) {
      const uint32_t j = j0 + lane;
      const uint32_t lo = t.state[coff + j];
      body(row0 + lane, hi, lo, j, row0 - j0, (hi << B.nlo) | lo);
    }
  });
}

// Compile-time (L, NLO) instances: the library's default split for each L.
// X(L, NLO)
// The default split of each L first, then the smaller-block splits the
// tuner may choose for the batched form.
#define MBL_FAST_SPLITS(X) \
  X(12, 9)                 \
  X(14, 10)                \
  X(16, 10)                \
  X(18, 12)                \
  X(20, 13)                \
  X(22, 13)                \
  X(24, 13)                \
  X(26, 13)                \
  X(28, 13)                \
  X(30, 13)                \
  X(32, 13)                \
  X(14, 7)                 \
  X(16, 8)                 \
  X(18, 9)                 \
  X(20, 9)                 \
  X(20, 11)                \
  X(22, 10)                \
  X(22, 9)                 \
  X(22, 11)                \
  X(24, 9)                 \
  X(24, 11)                \
  X(26, 9)                 \
  X(26, 11)


// One step of the MINRES scalar recurrence of Alg. 2: from the state after
// iteration k - 1, alpha_k and q_{k+1} . z_{k+1}, the state after iteration k
// (beta_{k+1}, the Givens rotation, phi_k, the d/x coefficients of iteration
// k, done). A done state is carried with a zero step.
__device__ __forceinline__ MinresState minres_givens_step(const MinresState& si, double alpha,
                                                          double qz, double tol, int64_t kmax) {
  MinresState so = si;
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
  const double c = gamma_hat / gamma;
  const double s = beta_next / gamma;
  so.d_inv_beta = 1.0 / beta;
  so.d_delta = delta;
  so.d_eps = si.eps;
  so.d_inv_gamma = 1.0 / gamma;
  so.d_tau = c * si.phi;
  so.beta_prev = beta;
  so.beta = beta_next;
  so.c = c;
  so.s = s;
  so.dhat = dhat_next;
  so.eps = eps_next;
  so.phi = -s * si.phi;
  so.k = si.k + 1;
  so.bad = !isfinite(so.phi) || !isfinite(alpha) || !isfinite(beta_next);
  so.done = so.bad || !(fabs(so.phi) >= tol && so.k < kmax);
  return so;
}

}  // namespace mbl
