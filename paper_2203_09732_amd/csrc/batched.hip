// Batched form: R disorder realizations of one chain length L solved in
// lockstep. Vectors are interleaved, element (i, r) at i * R + r, so every
// gather of a neighbour row fetches R contiguous values, and the index work
// of a row (its state, neighbour ranks, block offsets) is shared by all R
// realizations.
//
// Lane mapping (R a power of two, 2 <= R <= 32): PR = R / 2 lanes per row,
// each lane owns the realization pair (2p, 2p + 1) and moves it with one
// 8- or 16-byte access; a wavefront covers RPW = 64 / PR consecutive rows of
// one chunk per step. Each realization keeps its own fields, shift, MINRES
// scalars and done flag; per-realization dot products are reduced per
// workgroup and then by one workgroup per realization, in a fixed order.
#include "brows.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

namespace mbl {

// ---------------------------------------------------------------------------
// y = (H_r - sigma_r) x_r for every realization. MODE 1 is the product of
// MINRES iteration k: it first takes the Givens step of iteration k - 1 for
// every realization (gv; the same in every workgroup, stored by workgroup
// 0), skips realizations whose state is then done (GUARD), and writes
// partial sums of x.y per realization.
template <typename T, int MODE, bool GUARD, int L, int NLO>
__global__ __launch_bounds__(kBWG) void k_bapply(DevBasis B, BatchDev Q, BGivens gv,
                                                 const T* __restrict__ x, T* __restrict__ y,
                                                 double* __restrict__ partials) {
  using T2 = typename Pair<T>::type;
  const int R = Q.R;
  extern __shared__ __align__(16) unsigned char smem[];
  // the Givens step's inputs are loaded before the table fill, so that the
  // two latencies overlap
  BPrefetch pf;
  BState sp{};
  double al = 0.0;
  if (GUARD && gv.active) {
    bprefetch_partials(gv.part2, gv.G, R, pf);
    if (threadIdx.x < R) {
      sp = gv.Sprev[threadIdx.x];
      al = gv.alpha[threadIdx.x];
    }
  }
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  const uint32_t rs = (uint32_t)t.rsh + (sizeof(T) == 8 ? 3u : 2u);
  const uint32_t bytes = (uint32_t)B.n << rs;
  const __amdgpu_buffer_rsrc_t rx = brsrc(x, bytes), ry = brsrc(y, bytes);
  const int lane_p = (threadIdx.x & 63) % (R >> 1);
  bool live = true;
  if (GUARD) {
    if (gv.active) {
      const double qz = bsum_prefetched(pf, gv.G, R, t.red);
      if (threadIdx.x < R) {
        const int r = threadIdx.x;
        const BState so = bgivens_step(sp, al, qz, gv.tol, gv.kmax);
        if (blockIdx.x == 0) gv.Scur[r] = so;
        t.shared_r[r] = so.done ? 1.0 : 0.0;
      }
    } else if (threadIdx.x < R) {
      t.shared_r[threadIdx.x] = gv.Scur[threadIdx.x].done ? 1.0 : 0.0;
    }
    __syncthreads();
    live = !(t.shared_r[2 * lane_p] != 0.0 && t.shared_r[2 * lane_p + 1] != 0.0);
  }
  double acc0 = 0.0, acc1 = 0.0;
  if (live) {
    bfor_rows(B, t, R, [&](uint32_t, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0,
                           uint32_t a, int p) {
      BRowAddr ad;
      ad.rs = rs;
      ad.lane_off = (uint32_t)p << BIO<T>::kShift;
      ad.jv = (j << rs) + ad.lane_off;
      ad.sb = uni(block0) << rs;
      double o0, o1;
      boffdiag<T, L, NLO>(B, t, rx, ad, hi, lo, o0, o1);
      const int na = bnanti<L>(a);
      double d0, d1;
      bdiag2<L>(t, p, a, na, d0, d1);
      const T2 xv = BIO<T>::ld(rx, ad.jv, ad.sb);
      T2 yv;
      yv.x = (T)(d0 * (double)xv.x + 0.5 * o0);
      yv.y = (T)(d1 * (double)xv.y + 0.5 * o1);
      // streaming stores also for the MINRES product: p is far larger than
      // L2, and stores that allocate there evict the x lines the gathers
      // reuse (measured: the product, z/q and d/x kernels all run faster)
      BIO<T>::template st<kStoreStream>(yv, ry, ad.jv, ad.sb);
      if (MODE == 1) {
        acc0 += (double)xv.x * (double)yv.x;
        acc1 += (double)xv.y * (double)yv.y;
      }
    });
  }
  if (MODE == 1) {
    const double s = bblock_sum(acc0, acc1, t.red, R);
    if (threadIdx.x < R) partials[(size_t)blockIdx.x * R + threadIdx.x] = s;
  }
}

// r = rhs - (H_r - sigma_r) x in FP64; partials[(g * R + r) * 2 + {0, 1}] =
// sum r^2 / m (row-norm or chosen preconditioner) and sum r^2.
template <int L, int NLO>
__global__ __launch_bounds__(kBWG) void k_bresidual(DevBasis B, BatchDev Q, int kind,
                                                    const double* __restrict__ rhs,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ res,
                                                    double* __restrict__ partials) {
  const int R = Q.R;
  extern __shared__ __align__(16) unsigned char smem[];
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  const uint32_t rs = (uint32_t)t.rsh + 3u;
  const uint32_t bytes = (uint32_t)B.n << rs;
  const __amdgpu_buffer_rsrc_t rx = brsrc(x, bytes), rb = brsrc(rhs, bytes), rr = brsrc(res, bytes);
  double m0 = 0, m1 = 0, q0 = 0, q1 = 0;
  bfor_rows(B, t, R, [&](uint32_t, uint32_t hi, uint32_t lo, uint32_t j, uint32_t block0,
                         uint32_t a, int p) {
    BRowAddr ad;
    ad.rs = rs;
    ad.lane_off = (uint32_t)p << 4;
    ad.jv = (j << rs) + ad.lane_off;
    ad.sb = uni(block0) << rs;
    double o0, o1;
    boffdiag<double, L, NLO>(B, t, rx, ad, hi, lo, o0, o1);
    const int na = bnanti<L>(a);
    double d0, d1;
    bdiag2<L>(t, p, a, na, d0, d1);
    const double2 xv = BIO<double>::ld(rx, ad.jv, ad.sb), bv = BIO<double>::ld(rb, ad.jv, ad.sb);
    double2 rv;
    rv.x = bv.x - (d0 * xv.x + 0.5 * o0);
    rv.y = bv.y - (d1 * xv.y + 0.5 * o1);
    BIO<double>::st<0>(rv, rr, ad.jv, ad.sb);
    m0 += rv.x * rv.x / precond_value(kind, d0, na);
    m1 += rv.y * rv.y / precond_value(kind, d1, na);
    q0 += rv.x * rv.x;
    q1 += rv.y * rv.y;
  });
  const double sm = bblock_sum(m0, m1, t.red, R);
  const double sq = bblock_sum(q0, q1, t.red, R);
  if (threadIdx.x < R) {
    partials[((size_t)blockIdx.x * R + threadIdx.x) * 2] = sm;
    partials[((size_t)blockIdx.x * R + threadIdx.x) * 2 + 1] = sq;
  }
}

// MINRES initialisation per realization from x0 = 0: z_0 = 0, z_1 = scale_r
// src_r, q_1 = M_r^{-1} z_1, d = 0, x = 0; partial sums of q_1 . z_1.
template <typename T, int L>
__global__ __launch_bounds__(kBWG) void k_binit(DevBasis B, BatchDev Q, int kind,
                                                const double* __restrict__ src,
                                                const double* __restrict__ scale, T* z0, T* z1,
                                                T* q1, T* d0, T* d1, T* x,
                                                double* __restrict__ partials) {
  using T2 = typename Pair<T>::type;
  const int R = Q.R, PR = R >> 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  const double2* s2 = reinterpret_cast<const double2*>(src);
  double a0 = 0, a1 = 0;
  const T2 zero = {(T)0, (T)0};
  bfor_rows(B, t, R, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a, int p) {
    const size_t e = (size_t)row * PR + p;
    const int na = bnanti<L>(a);
    double d0v, d1v;
    bdiag2<L>(t, p, a, na, d0v, d1v);
    const double2 sv = s2[e];
    T2 zt, qt;
    // a zero scale (realization not solved) gives z = 0 whatever src holds
    const double sc0 = scale[2 * p], sc1 = scale[2 * p + 1];
    zt.x = (T)(sc0 != 0.0 ? sc0 * sv.x : 0.0);
    zt.y = (T)(sc1 != 0.0 ? sc1 * sv.y : 0.0);
    qt.x = (T)((double)zt.x / precond_value(kind, d0v, na));
    qt.y = (T)((double)zt.y / precond_value(kind, d1v, na));
    reinterpret_cast<T2*>(z0)[e] = zero;
    reinterpret_cast<T2*>(z1)[e] = zt;
    reinterpret_cast<T2*>(q1)[e] = qt;
    reinterpret_cast<T2*>(d0)[e] = zero;
    reinterpret_cast<T2*>(d1)[e] = zero;
    reinterpret_cast<T2*>(x)[e] = zero;
    a0 += (double)qt.x * (double)zt.x;
    a1 += (double)qt.y * (double)zt.y;
  });
  const double s = bblock_sum(a0, a1, t.red, R);
  if (threadIdx.x < R) partials[(size_t)blockIdx.x * R + threadIdx.x] = s;
}

// z_{k+1}, q_{k+1} and partial sums of q_{k+1} . z_{k+1}, for live
// realizations. A realization that is done gets z_{k+1} = q_{k+1} = 0 (never
// read by its own recurrence again), so the old q_{k+1} slot is not read.
template <typename T, int L>
__global__ __launch_bounds__(kBWG) void k_bzq(DevBasis B, BatchDev Q, int kind,
                                              const BState* __restrict__ S,
                                              const double* __restrict__ part1, int G,
                                              double* __restrict__ alpha_out,
                                              const T* __restrict__ p, const T* __restrict__ zk,
                                              T* __restrict__ zkm1, T* __restrict__ qn,
                                              double* __restrict__ partials) {
  using T2 = typename Pair<T>::type;
  const int R = Q.R, PR = R >> 1;
  extern __shared__ __align__(16) unsigned char smem[];
  BPrefetch pf;   // loaded before the table fill (overlapping latencies)
  bprefetch_partials(part1, G, R, pf);
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  // alpha_k = q_k . p_k / beta_k^2 from the product's partials (the same in
  // every workgroup; workgroup 0 keeps it for the Givens step)
  const double qp = bsum_prefetched(pf, G, R, t.red);
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    const double beta = S[r].beta;
    const double alpha = qp / (beta * beta);
    t.shared_r[r] = alpha;
    if (blockIdx.x == 0) alpha_out[r] = alpha;
  }
  __syncthreads();
  const uint32_t rs = (uint32_t)t.rsh + (sizeof(T) == 8 ? 3u : 2u);
  const uint32_t bytes = (uint32_t)B.n << rs;
  const __amdgpu_buffer_rsrc_t rp = brsrc(p, bytes), rz = brsrc(zk, bytes),
                               rzo = brsrc(zkm1, bytes), rq = brsrc(qn, bytes);
  const int lp = (threadIdx.x & 63) % PR;
  const BState s0 = S[2 * lp], s1 = S[2 * lp + 1];
  const double al0 = t.shared_r[2 * lp], al1 = t.shared_r[2 * lp + 1];
  const bool live0 = !s0.done, live1 = !s1.done;
  const double c10 = 1.0 / s0.beta, c20 = al0 / s0.beta, c30 = s0.beta / s0.beta_prev;
  const double c11 = 1.0 / s1.beta, c21 = al1 / s1.beta, c31 = s1.beta / s1.beta_prev;
  double a0 = 0, a1 = 0;
  if (live0 || live1) {
    bfor_rows(B, t, R, [&](uint32_t, uint32_t, uint32_t, uint32_t j, uint32_t block0, uint32_t a,
                           int pp) {
      const uint32_t jv = (j << rs) + ((uint32_t)pp << BIO<T>::kShift);
      const uint32_t sb = uni(block0) << rs;
      const int na = bnanti<L>(a);
      const T2 pv = BIO<T>::ld(rp, jv, sb);
      const T2 zv = BIO<T>::ld(rz, jv, sb);
      const T2 zm = BIO<T>::ld(rzo, jv, sb);
      double dg0, dg1;
      bdiag2<L>(t, pp, a, na, dg0, dg1);
      T2 zo = {(T)0, (T)0}, qo = {(T)0, (T)0};
      if (live0) {
        const double zn = c10 * (double)pv.x - c20 * (double)zv.x - c30 * (double)zm.x;
        zo.x = (T)zn;
        qo.x = (T)((double)zo.x / precond_value(kind, dg0, na));
        a0 += (double)qo.x * (double)zo.x;
      }
      if (live1) {
        const double zn = c11 * (double)pv.y - c21 * (double)zv.y - c31 * (double)zm.y;
        zo.y = (T)zn;
        qo.y = (T)((double)zo.y / precond_value(kind, dg1, na));
        a1 += (double)qo.y * (double)zo.y;
      }
      BIO<T>::template st<0>(zo, rzo, jv, sb);
      BIO<T>::template st<0>(qo, rq, jv, sb);
    });
  }
  const double s = bblock_sum(a0, a1, t.red, R);
  if (threadIdx.x < R) partials[(size_t)blockIdx.x * R + threadIdx.x] = s;
}

// One workgroup per realization: beta_1 and the initial state.
__global__ void k_binit_state(const double* __restrict__ partials, int G, int R, double tol,
                              int64_t kmax, BState* S0) {
  __shared__ double red[kWavesPerWG];
  const int r = blockIdx.x;
  double v = 0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) v += partials[(size_t)g * R + r];
  const double qz = block_sum_all(v, red);
  if (threadIdx.x == 0) {
    BState s{};
    s.beta_prev = 1.0;
    s.beta = sqrt(qz);
    s.c = 1.0;
    s.s = 0.0;
    s.dhat = 0.0;
    s.eps = 0.0;
    s.phi = s.beta;
    s.k = 0;
    s.bad = !isfinite(s.beta);
    s.done = s.bad || !(fabs(s.beta) >= tol && 0 < kmax);
    S0[r] = s;
  }
}

// ---- block-staged product (split nlo = 10, R = 32, FP64) --------------------
// y_r = (H_r - sigma_r) x_r with the terms of k_bapply<double, 0, false>
// (the off-diagonal ones summed in another order: low bonds, split bond, high
// bonds, wrap bond), for bases split at nlo = 10 (a hi block holds at most
// C(10, 5) = 252 rows, 252 x 256 B of x at R = 32).
// Each workgroup owns a host-built list of whole blocks: the blocks of one
// eighth of the rows go to that eighth's XCD, balanced by rows between its
// workgroups. While it computes block i, the workgroup stages block i + 1 of x
// in LDS by LDS DMA (buffer_load ... lds); the low-bond neighbours then come
// from LDS, the split-bond, wrap-bond and high-bond neighbours from memory,
// the far ones (high bonds b >= kStageFar and the wrap bond) by non-temporal
// loads, since they are not reused before their lines leave L2.
constexpr int kStageNlo = 10, kStageR = 32, kStageCap = 252, kStageFar = 7;

struct StagedBlock {
  uint32_t hi, row0, cnt, coff;   // block, its first row and row count, lo_state offset
  uint32_t sb_bnd, sb_wrap;       // byte offsets of the blocks hi ^ 1 and hi ^ 2^(nhi - 1)
  uint32_t pad0, pad1;
  uint32_t sbh[24];               // byte offsets of the blocks hi ^ (3 << b), b < nhi - 1
};

__device__ __forceinline__ double2 bld_nt(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t so) {
  const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)so, 2);   // nt
  double2 d;
  __builtin_memcpy(&d, &u, sizeof(d));
  return d;
}

typedef __attribute__((address_space(3))) void lds_void_t;

// MODE 1 is the product of MINRES iteration k, as k_bapply<double, 1, true>:
// the Givens step of iteration k - 1 first (every workgroup the same, stored
// by workgroup 0), realization pairs that are then both done skipped, and
// per-workgroup partial sums of x . y per realization (the grid is the row
// kernels' grid, so the next kernels read as many partials).
template <int L, int MODE>
__global__ __launch_bounds__(kBWG) void k_bapply_staged(DevBasis B, BatchDev Q, BGivens gv,
                                                        const StagedBlock* __restrict__ blocks,
                                                        const int* __restrict__ wg_first,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y,
                                                        double* __restrict__ partials) {
  constexpr int NLO = kStageNlo, R = kStageR, NHI = L - NLO;
  constexpr int PR = R / 2, RPW = 64 / PR, ROWB = R * 8, NW = kBWG / 64;
  constexpr int NNIB = (NLO + 3) / 4;
  __shared__ __align__(16) double bufA[kStageCap * R];
  __shared__ __align__(16) double bufB[kStageCap * R];
  __shared__ __align__(16) uint16_t s_rank[1 << NLO];
  __shared__ __align__(16) uint16_t s_state[1 << NLO];
  __shared__ __align__(16) double s_lut[NNIB * 16 * R];   // low-bit field sums
  __shared__ __align__(16) double s_c0[R];
  __shared__ __align__(16) double s_fA[R];                // high-bit field sum of a block
  __shared__ __align__(16) double s_fB[R];
  __shared__ __align__(16) double s_h[R * L];
  __shared__ double s_red[MODE == 1 ? NW * R : 1];
  __shared__ double s_done[MODE == 1 ? R : 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = uni(tid >> 6);
  const int first = wg_first[blockIdx.x], last = wg_first[blockIdx.x + 1];
  if (MODE == 1) {
    if (gv.active) {
      BState sp{};
      double al = 0.0;
      if (tid < R) {
        sp = gv.Sprev[tid];
        al = gv.alpha[tid];
      }
      const double qz = bsum_partials(gv.part2, gv.G, R, s_red);
      if (tid < R) {
        const BState so = bgivens_step(sp, al, qz, gv.tol, gv.kmax);
        if (blockIdx.x == 0) gv.Scur[tid] = so;
        s_done[tid] = so.done ? 1.0 : 0.0;
      }
    } else if (tid < R) {
      s_done[tid] = gv.Scur[tid].done ? 1.0 : 0.0;
    }
  }
  for (int t = tid; t < (1 << NLO); t += kBWG) {
    s_rank[t] = B.lo_rank[t];
    s_state[t] = B.lo_state[t];
  }
  for (int t = tid; t < NNIB * 16 * R; t += kBWG) {
    const int r = t % R, kv = t / R, k = kv >> 4, v = kv & 15;
    double acc = 0.0;
    for (int bb = 0; bb < 4; ++bb) {
      const int site = 4 * k + bb;
      if (site < NLO && ((v >> bb) & 1)) acc += Q.h[r * L + site];
    }
    s_lut[t] = acc;
  }
  if (tid < R) s_c0[tid] = Q.c0[tid];
  for (int t = tid; t < R * L; t += kBWG) s_h[t] = Q.h[t];
  const uint32_t nbytes = (uint32_t)B.n * ROWB;
  const __amdgpu_buffer_rsrc_t rx = brsrc(x, nbytes), ry = brsrc(y, nbytes);
  // issue the LDS DMA of block blk into buf (1 KB per wave instruction) and
  // the block's high-bit field sums
  auto stage = [&](const StagedBlock& blk, double* buf, double* fh) {
    const uint32_t hi = uni(blk.hi), row0 = uni(blk.row0), cnt = uni(blk.cnt);
    const uint32_t nb = cnt * ROWB, ninst = (nb + 1023) >> 10;
    for (uint32_t i = wave; i < ninst; i += NW) {
      const uint32_t off = i * 1024 + lane * 16;
      if (off < nb)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_t*)((char*)buf + i * 1024), 16,
                                                 row0 * ROWB + off, 0, 0, 0);
    }
    if (tid < R) {
      double f = 0.0;
      for (int bb = 0; bb < NHI; ++bb)
        if ((hi >> bb) & 1u) f += s_h[tid * L + NLO + bb];
      fh[tid] = f;
    }
  };
  double acc0 = 0.0, acc1 = 0.0;   // MODE 1: x . y of this lane's pair
  bool live = true;
  auto compute = [&](const StagedBlock& o, const double* buf, const double* fh) {
    if (!live) return;
    const uint32_t hi = uni(o.hi), cnt = uni(o.cnt), coff = uni(o.coff);
    const uint32_t sb_bnd = uni(o.sb_bnd), sb_wrap = uni(o.sb_wrap);
    uint32_t sbh[NHI - 1];
#pragma unroll
    for (int bb = 0; bb + 1 < NHI; ++bb) sbh[bb] = uni(o.sbh[bb]);
    const uint32_t hflips = uni(hi ^ (hi >> 1));
    const int p = lane % PR;
    const uint32_t slot = lane / PR;
    const double f0 = fh[2 * p], f1 = fh[2 * p + 1];
    const double cc0 = s_c0[2 * p], cc1 = s_c0[2 * p + 1];
    const uint32_t loff = (uint32_t)p * 16;
    for (uint32_t j0 = wave * RPW; j0 < cnt; j0 += NW * RPW) {
      const uint32_t j = j0 + slot;
      if (j >= cnt) continue;
      const uint32_t lo = s_state[coff + j];
      const uint32_t a = (hi << NLO) | lo;
      const uint32_t rbnd = s_rank[lo ^ (1u << (NLO - 1))], rwrap = s_rank[lo ^ 1u];
      // the gathers from memory first (their latency overlaps the LDS work)
      double2 vb = {0.0, 0.0}, vw = {0.0, 0.0};
      if (((lo >> (NLO - 1)) ^ hi) & 1u) vb = BIO<double>::ld(rx, rbnd * ROWB + loff, sb_bnd);
      double2 vh[NHI - 1];
#pragma unroll
      for (int bb = 0; bb + 1 < NHI; ++bb) {
        vh[bb] = double2{0.0, 0.0};
        if ((hflips >> bb) & 1u)
          vh[bb] = bb >= kStageFar ? bld_nt(rx, j * ROWB + loff, sbh[bb])
                                   : BIO<double>::ld(rx, j * ROWB + loff, sbh[bb]);
      }
      if (((hi >> (NHI - 1)) ^ lo) & 1u) vw = bld_nt(rx, rwrap * ROWB + loff, sb_wrap);
      const double2 own = *reinterpret_cast<const double2*>(buf + j * R + 2 * p);
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int bb = 0; bb + 1 < NLO; ++bb) {
        const uint32_t rk = s_rank[lo ^ (3u << bb)];
        const double2 v = *reinterpret_cast<const double2*>(buf + rk * R + 2 * p);
        const bool f = ((lo >> bb) ^ (lo >> (bb + 1))) & 1u;
        a0 += f ? v.x : 0.0;
        a1 += f ? v.y : 0.0;
      }
      a0 += vb.x;
      a1 += vb.y;
#pragma unroll
      for (int bb = 0; bb + 1 < NHI; ++bb) {
        a0 += vh[bb].x;
        a1 += vh[bb].y;
      }
      a0 += vw.x;
      a1 += vw.y;
      constexpr uint32_t mask = (1u << L) - 1u;
      const int na = __popc(a ^ (((a << 1) | (a >> (L - 1))) & mask));
      double F0 = f0, F1 = f1;
#pragma unroll
      for (int k = 0; k < NNIB; ++k) {
        const double2 fv = *reinterpret_cast<const double2*>(
            s_lut + (((k << 4) + ((lo >> (4 * k)) & 15u)) * R) + 2 * p);
        F0 += fv.x;
        F1 += fv.y;
      }
      const double d0 = cc0 - 0.5 * (double)na - F0, d1 = cc1 - 0.5 * (double)na - F1;
      double2 yv;
      yv.x = d0 * own.x + 0.5 * a0;
      yv.y = d1 * own.y + 0.5 * a1;
      BIO<double>::st<kStoreStream>(yv, ry, (uni(o.row0) + j) * ROWB + loff, 0);
      if (MODE == 1) {
        acc0 += own.x * yv.x;
        acc1 += own.y * yv.y;
      }
    }
  };
  __syncthreads();
  if (MODE == 1) {
    const int lp = lane % PR;
    live = !(s_done[2 * lp] != 0.0 && s_done[2 * lp + 1] != 0.0);
  }
  if (first >= last) {
    if (MODE == 1) {   // no blocks: zero partials
      const double sm = bblock_sum(0.0, 0.0, s_red, R);
      if (tid < R) partials[(size_t)blockIdx.x * R + tid] = sm;
    }
    return;
  }
  stage(blocks[first], bufA, s_fA);
  for (int i = first; i < last; i += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's DMA into the buffer landed
    __syncthreads();                      // every wave's did; the other buffer is free
    if (i + 1 < last) stage(blocks[i + 1], bufB, s_fB);
    compute(blocks[i], bufA, s_fA);
    if (i + 1 >= last) break;
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (i + 2 < last) stage(blocks[i + 2], bufA, s_fA);
    compute(blocks[i + 1], bufB, s_fB);
  }
  if (MODE == 1) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // no DMA left in flight past the kernel's end
    const double sm = bblock_sum(acc0, acc1, s_red, R);
    if (tid < R) partials[(size_t)blockIdx.x * R + tid] = sm;
  }
}

// ---- the streaming form: one realization's solve restarted in flight ----

// MINRES restart of the realizations with mask[r] != 0 from x0 = 0: z_K =
// src_r, z_{K-1} = 0, q_K = M_r^{-1} z_K, d = x = 0 (the buffers passed are
// the ones iteration K uses); partial sums of q_K . z_K. Other realizations
// are not touched.
template <int L>
__global__ __launch_bounds__(kBWG) void k_blane_init(DevBasis B, BatchDev Q, int kind,
                                                     const int* __restrict__ mask,
                                                     const double* __restrict__ src, double* zk,
                                                     double* zkm1, double* qk, double* d0,
                                                     double* d1, double* x,
                                                     double* __restrict__ partials) {
  const int R = Q.R;
  extern __shared__ __align__(16) unsigned char smem[];
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  const int lp = (threadIdx.x & 63) % (R >> 1);
  const bool m0 = mask[2 * lp] != 0, m1 = mask[2 * lp + 1] != 0;
  double a0 = 0, a1 = 0;
  if (m0 || m1) {
    bfor_rows(B, t, R, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a, int p) {
      const size_t e = (size_t)row * R + 2 * p;
      const int na = bnanti<L>(a);
      double dg0, dg1;
      bdiag2<L>(t, p, a, na, dg0, dg1);
      if (m0) {
        const double z = src[e], q = z / precond_value(kind, dg0, na);
        zk[e] = z;
        zkm1[e] = 0.0;
        qk[e] = q;
        d0[e] = 0.0;
        d1[e] = 0.0;
        x[e] = 0.0;
        a0 += q * z;
      }
      if (m1) {
        const double z = src[e + 1], q = z / precond_value(kind, dg1, na);
        zk[e + 1] = z;
        zkm1[e + 1] = 0.0;
        qk[e + 1] = q;
        d0[e + 1] = 0.0;
        d1[e + 1] = 0.0;
        x[e + 1] = 0.0;
        a1 += q * z;
      }
    });
  }
  const double sm = bblock_sum(a0, a1, t.red, R);
  if (threadIdx.x < R) partials[(size_t)blockIdx.x * R + threadIdx.x] = sm;
}

// One workgroup per realization: beta_1 and the initial state of each
// restarted solve, marked fresh, into the slot that the Givens step of the
// restart iteration reads (it carries the state on unchanged).
__global__ void k_blane_state(const double* __restrict__ partials, int G, int R,
                              const int* __restrict__ mask, double tol, int64_t kmax,
                              BState* Sslot) {
  __shared__ double red[kWavesPerWG];
  const int r = blockIdx.x;
  if (!mask[r]) return;
  double v = 0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) v += partials[(size_t)g * R + r];
  const double qz = block_sum_all(v, red);
  if (threadIdx.x == 0) {
    BState st{};
    st.beta_prev = 1.0;
    st.beta = sqrt(qz);
    st.c = 1.0;
    st.phi = st.beta;
    st.k = 0;
    st.bad = !isfinite(st.beta);
    st.done = st.bad || !(fabs(st.beta) >= tol && 0 < kmax);
    st.fresh = 1;
    Sslot[r] = st;
  }
}

// out[i, r] = V_{kidx[r]}[i, r] (0 where kidx[r] < 0)
__global__ __launch_bounds__(kWG) void k_blane_gather(int64_t n, int R, const double* __restrict__ V,
                                                      int64_t vstride, const int* __restrict__ kidx,
                                                      double* __restrict__ out) {
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = kidx[e & (R - 1)];
    out[e] = c >= 0 ? V[(size_t)c * vstride + e] : 0.0;
  }
}

// V_{kidx[r]}[i, r] = src[i, r] where kidx[r] >= 0
__global__ __launch_bounds__(kWG) void k_blane_scatter(int64_t n, int R,
                                                       const double* __restrict__ src, double* V,
                                                       int64_t vstride,
                                                       const int* __restrict__ kidx) {
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = kidx[e & (R - 1)];
    if (c >= 0) V[(size_t)c * vstride + e] = src[e];
  }
}

// column `lane` of blocks 0 .. nblk - 1 of V set to 0, then block 0 of it to
// src (contiguous n), if src is given
__global__ __launch_bounds__(kWG) void k_blane_reset(int64_t n, int R, int lane, double* V,
                                                     int64_t vstride, int nblk,
                                                     const double* __restrict__ src) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const size_t e = (size_t)i * R + lane;
    for (int c = 0; c < nblk; ++c) V[(size_t)c * vstride + e] = 0.0;
    if (src) V[e] = src[i];
  }
}

// dst (n contiguous) = column `lane` of src (interleaved n x R)
__global__ __launch_bounds__(kWG) void k_blane_get(int64_t n, int R, int lane,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[(size_t)i * R + lane];
}

// The Givens step of the last issued iteration (one workgroup of kBWG
// threads; the same arithmetic as the product's prologue).
__global__ __launch_bounds__(kBWG) void k_bgivens_last(BGivens gv, int R) {
  __shared__ double red[kLdsRed * kBMaxR];
  const double qz = bsum_partials(gv.part2, gv.G, R, red);
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    gv.Scur[r] = bgivens_step(gv.Sprev[r], gv.alpha[r], qz, gv.tol, gv.kmax);
  }
}

// The d/x update of Alg. 2 for kDxGroup consecutive iterations in one pass:
// each element walks d_k = (q_k / beta_k - delta_k d_{k-1} - eps_k d_{k-2}) /
// gamma_k, x += tau_k d_k for k = k_first .. k_first + count - 1 with the same
// per-element arithmetic as one update per iteration, reading q_k from the
// ring and the coefficients from the ring of states, and stores only the last
// two d's and x. Iterations in which a realization was already done are
// skipped for it.
constexpr int kDxGroup = 4;   // the longest d/x pass (the schedule may use 1 or 2)
constexpr int kRing = 8;   // q vectors and iteration states kept; a divisor of the graph length

template <typename T>
struct QRing {
  const T* q[kRing];
};

template <typename T>
__global__ __launch_bounds__(kWG) void k_bdx_group(int64_t n, int R, const BState* __restrict__ S,
                                                   QRing<T> Qr, int64_t k_first, int count,
                                                   T* __restrict__ d_a, T* __restrict__ d_b,
                                                   T* __restrict__ x) {
  // d_a holds d_{k} for even k, d_b for odd k
  __shared__ double co[kDxGroup][kBMaxR][5];
  __shared__ int act[kDxGroup][kBMaxR];
  for (int t = threadIdx.x; t < count * R; t += blockDim.x) {
    const int j = t / R, r = t % R;
    const int64_t k = k_first + j;
    const BState sk = S[(size_t)(k % kRing) * R + r];
    co[j][r][0] = sk.d_inv_beta;
    co[j][r][1] = sk.d_delta;
    co[j][r][2] = sk.d_eps;
    co[j][r][3] = sk.d_inv_gamma;
    co[j][r][4] = sk.d_tau;
    act[j][r] = !S[(size_t)((k - 1) % kRing) * R + r].done;
  }
  __syncthreads();
  T* dk1 = ((k_first - 1) & 1) ? d_b : d_a;   // d_{k_first - 1}
  T* dk2 = ((k_first - 1) & 1) ? d_a : d_b;   // d_{k_first - 2}
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e & (R - 1));
    if (!act[0][r]) continue;
    double dm1 = (double)dk1[e], dm2 = (double)dk2[e];
    T xv = x[e];
    int last = -1;
#pragma unroll
    for (int j = 0; j < kDxGroup; ++j) {
      if (j >= count || !act[j][r]) break;
      const int64_t k = k_first + j;
      const double d = ((double)Qr.q[k % kRing][e] * co[j][r][0] - co[j][r][1] * dm1 -
                        co[j][r][2] * dm2) * co[j][r][3];
      const T dt = (T)d;
      xv = (T)((double)xv + co[j][r][4] * (double)dt);
      dm2 = dm1;
      dm1 = (double)dt;
      last = j;
    }
    if (last >= 0) {
      const int64_t kl = k_first + last;            // d_kl in dm1, d_{kl-1} in dm2
      ((kl & 1) ? d_b : d_a)[e] = (T)dm1;
      ((kl & 1) ? d_a : d_b)[e] = (T)dm2;
      x[e] = xv;
    }
  }
}

// per-realization reduction: out[r * nv + v] = sum_g partials[(g * R + r) * nv + v]
__global__ void k_breduce(const double* __restrict__ partials, int G, int R, int nv,
                          double* __restrict__ out) {
  __shared__ double red[kWavesPerWG];
  const int r = blockIdx.x / nv, v = blockIdx.x % nv;
  double a = 0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) a += partials[((size_t)g * R + r) * nv + v];
  const double s = block_sum_all(a, red);
  if (threadIdx.x == 0) out[r * nv + v] = s;
}

// x64 += scale_r * e (interleaved)
__global__ __launch_bounds__(kWG) void k_badd_scaled(int64_t n, int R, const double* __restrict__ scale,
                                                     const float* __restrict__ e,
                                                     double* __restrict__ x) {
  const int64_t total = n * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double sc = scale[i & (R - 1)];
    if (sc != 0.0) x[i] += sc * (double)e[i];   // a zero scale leaves x untouched
  }
}

// ---------------------------------------------------------------------------
// dense batched helpers for the Lanczos recurrences (interleaved n x R)

// partials[(g * k + c) * R + r] = sum_i V_c[i, r] w[i, r] over this group's
// rows, c in the tile [4 by, 4 by + 4) with c < k
__global__ __launch_bounds__(kWG) void k_bmultidot(int64_t n, int R, const double* __restrict__ V,
                                                   int64_t vstride, int k,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ partials) {
  constexpr int TC = 4;
  __shared__ double red[kWavesPerWG][TC][kBMaxR];
  const int c0 = blockIdx.y * TC;
  const int nc = min(TC, k - c0);
  // each thread owns one realization r = tid % R and rows strided by 256/R
  const int r = threadIdx.x % R;
  const int rows_per = blockDim.x / R;
  const int rl = threadIdx.x / R;
  double acc[TC] = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * rows_per + rl; i < n; i += (int64_t)gridDim.x * rows_per) {
    const double wi = w[i * R + r];
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
      if (tc < nc) acc[tc] += V[(size_t)(c0 + tc) * vstride + i * R + r] * wi;
  }
  // reduce over lanes with the same r inside the wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int tc = 0; tc < TC; ++tc)
    for (int o = R; o < 64; o <<= 1) acc[tc] += __shfl_xor(acc[tc], o, 64);
  if (lane < R) {
#pragma unroll
    for (int tc = 0; tc < TC; ++tc) red[wave][tc][lane] = acc[tc];
  }
  __syncthreads();
  if (threadIdx.x < nc * R) {
    const int tc = threadIdx.x / R, rr = threadIdx.x % R;
    double s = 0;
    for (int wv = 0; wv < kWavesPerWG; ++wv) s += red[wv][tc][rr];
    partials[((size_t)blockIdx.x * k + c0 + tc) * R + rr] = s;
  }
}

// w[i, r] -= sum_{c < k} V_c[i, r] coef[c * R + r]
__global__ __launch_bounds__(kWG) void k_bcgs_update(int64_t n, int R, const double* __restrict__ V,
                                                     int64_t vstride, int k,
                                                     const double* __restrict__ coef,
                                                     double* __restrict__ w) {
  extern __shared__ double sc[];
  for (int e = threadIdx.x; e < k * R; e += blockDim.x) sc[e] = coef[e];
  __syncthreads();
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % R);
    double s = 0;
    for (int c = 0; c < k; ++c) s += V[(size_t)c * vstride + e] * sc[c * R + r];
    w[e] -= s;
  }
}

// y[i, r] = a[r] * x[i, r] + b[r] * y[i, r]
__global__ __launch_bounds__(kWG) void k_baxpby(int64_t n, int R, const double* __restrict__ a,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b, double* y) {
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % R);
    // BLAS convention: a zero coefficient does not read its operand, so
    // stale or unset entries of x or y never reach the result
    const double ar = a[r], br = b[r];
    const double ax = ar != 0.0 ? ar * x[e] : 0.0;
    y[e] = br != 0.0 ? ax + br * y[e] : ax;
  }
}

// partials[(g * R + r)] = sum_i x[i, r] y[i, r]
__global__ __launch_bounds__(kWG) void k_bdot(int64_t n, int R, const double* __restrict__ x,
                                              const double* __restrict__ y,
                                              double* __restrict__ partials) {
  __shared__ double red[kWavesPerWG][kBMaxR];
  const int r = threadIdx.x % R, rl = threadIdx.x / R, rows_per = blockDim.x / R;
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * rows_per + rl; i < n; i += (int64_t)gridDim.x * rows_per)
    acc += x[i * R + r] * y[i * R + r];
  for (int o = R; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < R) red[wave][lane] = acc;
  __syncthreads();
  if (threadIdx.x < R) {
    double s = 0;
    for (int wv = 0; wv < kWavesPerWG; ++wv) s += red[wv][threadIdx.x];
    partials[(size_t)blockIdx.x * R + threadIdx.x] = s;
  }
}

// U_t[i, r] = sum_c V_c[i, r] Y[(r * k + c) * nev + t]   (Y per realization)
__global__ __launch_bounds__(kWG) void k_britz(int64_t n, int R, const double* __restrict__ V,
                                               int64_t vstride, int k,
                                               const double* __restrict__ Y, int nev,
                                               double* __restrict__ U, int64_t ustride) {
  const int t = blockIdx.y;
  const int64_t total = n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % R);
    double s = 0;
    for (int c = 0; c < k; ++c) s += V[(size_t)c * vstride + e] * Y[((size_t)r * k + c) * nev + t];
    U[(size_t)t * ustride + e] = s;
  }
}


// twist partial sums per (vector t, realization r): partials[((t * G + g) * R + r) * 2 + {0, 1}]
struct BTwistTab {
  double c[2 * kMaxL];
  double s[2 * kMaxL];
};
template <int L>
__global__ __launch_bounds__(kBWG) void k_btwist(DevBasis B, BatchDev Q, BTwistTab T,
                                                 const double* __restrict__ psi, int64_t vstride,
                                                 double* __restrict__ partials) {
  const int R = Q.R, PR = R >> 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const BTables t = bsetup(B, Q, smem);
  __syncthreads();
  const double2* v2 = reinterpret_cast<const double2*>(psi + (size_t)blockIdx.y * vstride);
  double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
  constexpr int base = (L * (L + 1)) / 2;
  bfor_rows(B, t, R, [&](uint32_t row, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t a, int p) {
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      uint32_t w = 0;
      for (int q = 0; q < 32; ++q)
        if (((q + 1) >> k) & 1) w |= (1u << q);
      sum += __popc(a & w) << k;
    }
    int m = (2 * sum - base) % (2 * L);
    if (m < 0) m += 2 * L;
    const double2 v = v2[(size_t)row * PR + p];
    r0 += v.x * v.x * T.c[m];
    i0 += v.x * v.x * T.s[m];
    r1 += v.y * v.y * T.c[m];
    i1 += v.y * v.y * T.s[m];
  });
  const double sr = bblock_sum(r0, r1, t.red, R);
  const double si = bblock_sum(i0, i1, t.red, R);
  if (threadIdx.x < R) {
    const size_t g = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * R + threadIdx.x;
    partials[2 * g] = sr;
    partials[2 * g + 1] = si;
  }
}

}  // namespace mbl

// ===========================================================================
// host side

struct mbl_batch_s {
  mbl_basis basis = nullptr;
  int R = 0, mmax = 0, nevmax = 0;
  int64_t n = 0, bytes = 0;
  double* h = nullptr;       // R * L
  double* c0 = nullptr;      // R
  mbl::BState* S = nullptr;  // kRing * R
  double* z[2] = {nullptr, nullptr};
  double* q[mbl::kRing] = {};
  double* d[2] = {nullptr, nullptr};
  double* p = nullptr;
  double* e = nullptr;
  double* r64 = nullptr;
  double* t64 = nullptr;
  double* w = nullptr;
  double* x = nullptr;
  double* V = nullptr;       // (mmax + 1) blocks of n * R
  double* coef = nullptr;    // (mmax + 1) * R
  double* ycoef = nullptr;   // R * (mmax + 1) * nevmax
  double* partials1 = nullptr;
  double* partials2 = nullptr;
  double* red = nullptr;     // R * 64
  double* scale = nullptr;   // R
  double* scale2 = nullptr;  // R
  double* alph = nullptr;    // 2 * R: MINRES alpha_k by the parity of k
  mbl::BState* h_state = nullptr;   // pinned, 4 * R
  double* h_red = nullptr;          // pinned, R * 64
  double* h_stage = nullptr;        // pinned, R * (L + 1) + 4 R
  hipEvent_t ev[2] = {nullptr, nullptr};
  size_t part_elems = 0;
  std::vector<double> last_up;      // host copy of the last uploaded (h, c0)
  // captured MINRES loop (16 iterations) per (vector type, preconditioner)
  hipGraphExec_t graph[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  double graph_tol[2][3] = {{0, 0, 0}, {0, 0, 0}};
  int64_t graph_kmax[2][3] = {{0, 0, 0}, {0, 0, 0}};
  void* graph_x[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int graph_mode = -1;              // -1: unset (env), 0: eager launches, 1: graphs
  // launch schedule (mbl_batch_set_schedule): row-kernel workgroups (0: one
  // per CU), MINRES iterations per captured graph, iterations per d/x pass
  int sched_grid = 0, sched_graph = 16, sched_dx = 4;
  // block lists of the staged plain product (nlo = 10, R = 32), built on first use
  void* stage_blocks = nullptr;
  int* stage_first = nullptr;
  int stage_G = 0;
  hipStream_t cap = nullptr;        // capture stream (the caller's may be the null stream)
};

namespace mbl {

// Workgroups of the batched row kernels: enough 16-wave workgroups for every
// chunk to get its R / 2 waves (a chunk of 64 rows needs R / 2 wave-steps),
// at most one 1024-thread workgroup per compute unit (measured: a second
// resident workgroup per CU slows the gather-bound apply), whole XCD slices
// once large.
static int device_cus(int device) {
  // per-device cache; calls from several host threads may fill it at once
  // (they store the same value)
  static std::atomic<int> cached[64];
  if (device < 0 || device >= 64) return 256;
  int c = cached[device].load(std::memory_order_relaxed);
  if (c == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        v <= 0) {
      (void)hipGetLastError();
      v = 256;
    }
    cached[device].store(v, std::memory_order_relaxed);
    c = v;
  }
  return c;
}

static int bgrid(const mbl_basis_s* b, int R, int grid = 0) {
  if (grid > 0) return grid;   // a tuned schedule (a multiple of 8, <= kBGrid)
  const int64_t wave_steps = (int64_t)b->nchunks * std::max(1, R / 2);
  int64_t g = (wave_steps + (kBWG / 64) - 1) / (kBWG / 64);
  g = std::max<int64_t>(1, std::min<int64_t>({g, kBGrid, device_cus(b->device)}));
  return g >= 64 ? (int)(g / 8) * 8 : (int)g;
}

static bool batched_split_supported(const mbl_basis_s* b) {
  switch (b->L * 64 + b->nlo) {
#define MBL_CASE(LL, NN) case LL * 64 + NN:
    MBL_FAST_SPLITS(MBL_CASE)
#undef MBL_CASE
    return true;
    default:
      return false;
  }
}

#define MBL_BDISPATCH(KERNEL_TEMPLATE_CALL)                                   \
  switch (b->L * 64 + b->nlo) {                                              \
    MBL_FAST_SPLITS(KERNEL_TEMPLATE_CALL)                                    \
    default:                                                                 \
      set_error("batched form has no instance for this (L, lo_bits)");      \
      return MBL_ERR_ARG;                                                    \
  }

template <typename T, int MODE, bool GUARD>
static mbl_status launch_bapply(const mbl_basis_s* b, const BatchDev& Q, const BGivens& gv,
                                const T* x, T* y, double* partials, hipStream_t s) {
  const size_t lds = blds_bytes(Q.R, b->L, b->nlo);
  const dim3 g(bgrid(b, Q.R, Q.grid)), blk(kBWG);
  const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                    \
  case LL * 64 + NN:                                                                       \
    hipLaunchKernelGGL((k_bapply<T, MODE, GUARD, LL, NN>), g, blk, lds, s, B, Q, gv, x, y, \
                       partials);                                                          \
    break;
  MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

static mbl_status launch_bresidual(const mbl_basis_s* b, const BatchDev& Q, int kind,
                                   const double* rhs, const double* x, double* res,
                                   double* partials, hipStream_t s) {
  const size_t lds = blds_bytes(Q.R, b->L, b->nlo);
  const dim3 g(bgrid(b, Q.R, Q.grid)), blk(kBWG);
  const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                       \
  case LL * 64 + NN:                                                                          \
    hipLaunchKernelGGL((k_bresidual<LL, NN>), g, blk, lds, s, B, Q, kind, rhs, x, res,       \
                       partials);                                                             \
    break;
  MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

template <typename T>
static mbl_status launch_binit(const mbl_basis_s* b, const BatchDev& Q, int kind,
                               const double* src, const double* scale, T* z0, T* z1, T* q1, T* d0,
                               T* d1, T* x, double* partials, hipStream_t s) {
  const size_t lds = blds_bytes(Q.R, b->L, b->nlo);
  const dim3 g(bgrid(b, Q.R, Q.grid)), blk(kBWG);
  const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                        \
  case LL * 64 + NN:                                                                           \
    hipLaunchKernelGGL((k_binit<T, LL>), g, blk, lds, s, B, Q, kind, src, scale, z0, z1, q1,  \
                       d0, d1, x, partials);                                                   \
    break;
  MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

template <typename T>
static mbl_status launch_bzq(const mbl_basis_s* b, const BatchDev& Q, int kind, const BState* S,
                             const double* part1, double* alpha_out, const T* p, const T* zk,
                             T* zkm1, T* qn, double* partials, hipStream_t s) {
  const size_t lds = blds_bytes(Q.R, b->L, b->nlo);
  const dim3 g(bgrid(b, Q.R, Q.grid)), blk(kBWG);
  const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                        \
  case LL * 64 + NN:                                                                           \
    hipLaunchKernelGGL((k_bzq<T, LL>), g, blk, lds, s, B, Q, kind, S, part1, (int)g.x,      \
                       alpha_out, p, zk, zkm1, qn, partials);                                  \
    break;
  MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

static int bflat_grid(int64_t total) {
  int64_t g = (total + kWG - 1) / kWG;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

// upload fields and shifts of the R realizations (c0_r = L/4 + sum h_r / 2 - sigma_r)
static mbl_status bupload(mbl_batch_s* bw, const double* h_host, const double* sigma_host,
                          hipStream_t s) {
  const int R = bw->R, L = bw->basis->L;
  std::vector<double> up((size_t)R * (L + 1));
  std::copy(h_host, h_host + (size_t)R * L, up.begin());
  for (int r = 0; r < R; ++r) {
    double sh = 0;
    for (int j = 0; j < L; ++j) sh += h_host[(size_t)r * L + j];
    up[(size_t)R * L + r] = 0.25 * L + 0.5 * sh - sigma_host[r];
  }
  if (up == bw->last_up) return MBL_OK;   // already on the device
  double* st = bw->h_stage;
  MBL_HIP(hipStreamSynchronize(s));   // staging buffer reuse
  std::copy(up.begin(), up.end(), st);
  bw->last_up = up;
  MBL_HIP(hipMemcpyAsync(bw->h, st, sizeof(double) * R * L, hipMemcpyHostToDevice, s));
  MBL_HIP(hipMemcpyAsync(bw->c0, st + (size_t)R * L, sizeof(double) * R, hipMemcpyHostToDevice,
                         s));
  return MBL_OK;
}

// per-realization sums to host: out[r * nv + v] = sum_g partials[((g * R) + r) * nv + v]
static mbl_status breduce_host(mbl_batch_s* bw, const double* partials, int G, int nv,
                               double* out, hipStream_t s) {
  const int R = bw->R;
  hipLaunchKernelGGL(k_breduce, dim3(R * nv), dim3(kWG), 0, s, partials, G, R, nv, bw->red);
  MBL_HIP(hipGetLastError());
  MBL_HIP(hipMemcpyAsync(bw->h_red, bw->red, sizeof(double) * R * nv, hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  std::copy(bw->h_red, bw->h_red + R * nv, out);
  return MBL_OK;
}

static bool staged_instance(const mbl_basis_s* b, int R) {
  return R == kStageR && b->nlo == kStageNlo && (b->L == 14 || b->L == 16 || b->L == 22);
}

// The staged product's block lists for the workspace's grid: the blocks of
// one eighth of the rows go to the workgroups of one XCD (workgroup g runs on
// XCD g % 8), each block to that XCD's workgroup with the fewest rows so far.
static mbl_status staged_plan(mbl_basis_s* b, mbl_batch_s* w, hipStream_t s) {
  // the row kernels' grid, so that the MINRES product's partial sums are as
  // many as the kernels after it read
  const int G = bgrid(b, w->R, w->sched_grid);
  if (w->stage_blocks && w->stage_G == G) return MBL_OK;
  if (w->stage_blocks) (void)hipFree(w->stage_blocks);
  if (w->stage_first) (void)hipFree(w->stage_first);
  w->stage_blocks = nullptr;
  w->stage_first = nullptr;
  const int nhi = b->nhi, nlo = b->nlo;
  std::vector<uint32_t> hi_off((size_t)1 << nhi), coff(nlo + 2);
  MBL_HIP(hipMemcpyAsync(hi_off.data(), b->d_hi_off, sizeof(uint32_t) * hi_off.size(),
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipMemcpyAsync(coff.data(), b->d_lo_coff, sizeof(uint32_t) * coff.size(),
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  struct Blk {
    uint32_t hi, row0, cnt, coff;
  };
  std::vector<Blk> all;
  for (size_t hi = 0; hi < hi_off.size(); ++hi) {
    if (hi_off[hi] == 0xffffffffu) continue;
    const int c = b->half - __builtin_popcountll(hi);
    if (c < 0 || c > nlo) continue;
    const uint32_t cnt = coff[c + 1] - coff[c];
    if (cnt == 0) continue;
    if (cnt > (uint32_t)kStageCap) {
      set_error("internal: staged block larger than its LDS buffer");
      return MBL_ERR_NUMERIC;
    }
    all.push_back(Blk{(uint32_t)hi, hi_off[hi], cnt, coff[c]});
  }
  const int X = kXcds, per = std::max(1, G / X);
  std::vector<std::vector<Blk>> wl(G);
  const uint64_t n = (uint64_t)b->n;
  size_t bi = 0;
  for (int xcd = 0; xcd < X; ++xcd) {
    const uint64_t lim = n * (uint64_t)(xcd + 1) / X;
    std::vector<uint64_t> load(per, 0);
    while (bi < all.size() && (all[bi].row0 < lim || xcd == X - 1)) {
      int best = 0;
      for (int q = 1; q < per; ++q)
        if (load[q] < load[best]) best = q;
      load[best] += all[bi].cnt;
      wl[std::min(G - 1, xcd + X * best)].push_back(all[bi]);
      ++bi;
    }
  }
  std::vector<StagedBlock> list;
  std::vector<int> first(1, 0);
  const uint32_t ROWB = kStageR * 8;
  for (int g = 0; g < G; ++g) {
    for (const Blk& v : wl[g]) {
      StagedBlock d{};
      d.hi = v.hi;
      d.row0 = v.row0;
      d.cnt = v.cnt;
      d.coff = v.coff;
      // neighbour blocks that do not exist are only addressed by masked gathers
      d.sb_bnd = hi_off[v.hi ^ 1u] * ROWB;
      d.sb_wrap = hi_off[v.hi ^ (1u << (nhi - 1))] * ROWB;
      for (int bb = 0; bb + 1 < nhi; ++bb) d.sbh[bb] = hi_off[v.hi ^ (3u << bb)] * ROWB;
      list.push_back(d);
    }
    first.push_back((int)list.size());
  }
  if (hipMalloc(&w->stage_blocks, sizeof(StagedBlock) * std::max<size_t>(list.size(), 1)) !=
          hipSuccess ||
      hipMalloc((void**)&w->stage_first, sizeof(int) * first.size()) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed (staged block lists)");
    return MBL_ERR_NOMEM;
  }
  MBL_HIP(hipMemcpyAsync(w->stage_blocks, list.data(), sizeof(StagedBlock) * list.size(),
                         hipMemcpyHostToDevice, s));
  MBL_HIP(hipMemcpyAsync(w->stage_first, first.data(), sizeof(int) * first.size(),
                         hipMemcpyHostToDevice, s));
  MBL_HIP(hipStreamSynchronize(s));
  w->stage_G = G;
  return MBL_OK;
}

// The staged product; its block lists must exist (staged_plan, which
// synchronizes and so runs before any graph capture).
template <int MODE>
static mbl_status launch_bapply_staged(mbl_basis_s* b, mbl_batch_s* w, const BatchDev& Q,
                                       const BGivens& gv, const double* x, double* y,
                                       double* partials, hipStream_t s) {
  if (!w->stage_blocks || w->stage_G != bgrid(b, w->R, w->sched_grid)) {
    set_error("internal: staged product launched without its block lists");
    return MBL_ERR_ARG;
  }
  const DevBasis B = b->dev();
  const StagedBlock* blk = static_cast<const StagedBlock*>(w->stage_blocks);
  switch (b->L) {
    case 14:
      hipLaunchKernelGGL((k_bapply_staged<14, MODE>), dim3(w->stage_G), dim3(kBWG), 0, s, B, Q,
                         gv, blk, w->stage_first, x, y, partials);
      break;
    case 16:
      hipLaunchKernelGGL((k_bapply_staged<16, MODE>), dim3(w->stage_G), dim3(kBWG), 0, s, B, Q,
                         gv, blk, w->stage_first, x, y, partials);
      break;
    case 22:
      hipLaunchKernelGGL((k_bapply_staged<22, MODE>), dim3(w->stage_G), dim3(kBWG), 0, s, B, Q,
                         gv, blk, w->stage_first, x, y, partials);
      break;
    default:
      set_error("internal: no staged instance for this L");
      return MBL_ERR_ARG;
  }
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

// The streaming form's view of a running batched MINRES. After each chunk of
// iterations has been issued, the hook receives the states after iteration
// `iter` of an earlier chunk (the snapshot lags one chunk, so the d/x updates
// of every realization done in it have been issued too) and `next_k`, the
// iteration the next chunk starts with. It may restart the solve of any
// realization that is done: restart[r] = 1 with right-hand side column r of
// *rhs (x0 = 0, from iteration next_k on). keep_going = false ends the loop.
struct MinresHook {
  std::function<mbl_status(const BState* st, int64_t iter, int64_t next_k, std::vector<int>& restart,
                           const double** rhs, bool& keep_going)>
      on_snapshot;
  int* mask_dev = nullptr;       // R ints, device
  double* part_dev = nullptr;    // bgrid * R doubles, device
};

// Alg. 2 on all realizations, from x0 = 0 with z_1 = scale_r src_r (a zero
// scale makes realization r done at once). x: T, n * R. With a hook (FP64
// only), the loop runs until the hook stops it and per-realization solves are
// restarted in flight.
template <typename T>
static mbl_status bminres_core(mbl_basis_s* b, mbl_batch_s* bw, const BatchDev& Q, int precond,
                               const double* src, const double* scale_dev, T* x, double tol,
                               int64_t kmax, hipStream_t s, std::vector<BState>& fin,
                               MinresHook* hook = nullptr) {
  const int R = bw->R;
  const int64_t n = b->n;
  T* Z[2] = {(T*)bw->z[0], (T*)bw->z[1]};
  T* Qv[kRing];
  QRing<T> qr;
  for (int i = 0; i < kRing; ++i) qr.q[i] = Qv[i] = (T*)bw->q[i];
  T* D[2] = {(T*)bw->d[0], (T*)bw->d[1]};
  T* P = (T*)bw->p;
  const int G = bgrid(b, R, Q.grid);
  const int dxg = bw->sched_dx;   // iterations per d/x pass (1, 2 or 4)
  BState* S = bw->S;
  // z_0 in Z[0], z_1 in Z[1], q_1 in Qv[1], d_0 in D[0], d_{-1} in D[1]
  MBL_TRY(launch_binit<T>(b, Q, precond, src, scale_dev, Z[0], Z[1], Qv[1], D[0], D[1], x,
                          bw->partials2, s));
  hipLaunchKernelGGL(k_binit_state, dim3(R), dim3(kWG), 0, s, bw->partials2, G, R, tol, kmax, S);
  MBL_HIP(hipGetLastError());
  const int FG = bflat_grid(n * R);
  // d/x updates of iterations k_first .. k_first + count - 1
  auto dx_group = [&](int64_t k_first, int count, hipStream_t st) -> mbl_status {
    hipLaunchKernelGGL((k_bdx_group<T>), dim3(FG), dim3(kWG), 0, st, n, R, S, qr, k_first, count,
                       D[0], D[1], x);
    MBL_HIP(hipGetLastError());
    return MBL_OK;
  };
  // The Givens step of iteration k - 1 (state k - 1 in slot (k - 1) % kRing,
  // alpha_{k-1} in alph[(k - 1) & 1]).
  auto givens_args = [&](int64_t k) {
    BGivens gv;
    gv.part2 = bw->partials2;
    gv.alpha = bw->alph + ((k - 1) & 1) * R;
    gv.Sprev = S + ((k + kRing - 2) % kRing) * R;
    gv.Scur = S + ((k - 1) % kRing) * R;
    gv.G = G;
    gv.active = k >= 2;
    gv.tol = tol;
    gv.kmax = kmax;
    return gv;
  };
  // Iteration k of Alg. 2 for all realizations, two row launches: the
  // product p = A q_k, which first takes the Givens step of iteration k - 1
  // (and skips realizations that are then done), and the z/q update, which
  // first forms alpha_k. The d/x update of iterations k - 4 .. k - 1 runs
  // between them once their Givens steps are known.
  // FP64 products at split 10 with R = 32 run block-staged (the block lists
  // are built here, outside any graph capture)
  const bool staged = std::is_same<T, double>::value && staged_instance(b, R);
  if (staged) MBL_TRY(staged_plan(b, bw, s));
  auto iteration = [&](int64_t k, hipStream_t st) -> mbl_status {
    const BGivens gv = givens_args(k);
    if (staged)
      MBL_TRY(launch_bapply_staged<1>(b, bw, Q, gv, (const double*)Qv[k % kRing], (double*)P,
                                      bw->partials1, st));
    else
      MBL_TRY((launch_bapply<T, 1, true>(b, Q, gv, Qv[k % kRing], P, bw->partials1, st)));
    if (k > dxg && (k - 1) % dxg == 0) MBL_TRY(dx_group(k - dxg, dxg, st));
    MBL_TRY(launch_bzq<T>(b, Q, precond, gv.Scur, bw->partials1, bw->alph + (k & 1) * R, P,
                          Z[k & 1], Z[(k + 1) & 1], Qv[(k + 1) % kRing], bw->partials2, st));
    return MBL_OK;
  };
  // After the last issued iteration K: its Givens step, then the d/x update
  // of the iterations not yet covered (those after the last full group).
  auto finish = [&](int64_t K, hipStream_t st) -> mbl_status {
    BGivens gv = givens_args(K + 1);
    hipLaunchKernelGGL(k_bgivens_last, dim3(1), dim3(kBWG), 0, st, gv, R);
    MBL_HIP(hipGetLastError());
    const int64_t covered = K >= 1 ? dxg * ((K - 1) / dxg) : 0;
    if (K > covered) MBL_TRY(dx_group(covered + 1, (int)(K - covered), st));
    return MBL_OK;
  };
  // Iteration 1 runs eagerly; then blocks of kGraphIters iterations (2..17,
  // 18..33, ...), which use buffers and state slots that depend only on k mod
  // kRing and read their scalars and done flags from device memory, are
  // captured once per workspace and replayed (a replay after convergence is
  // a sequence of no-op launches). tol and kmax are kernel arguments, so the
  // graph is captured again when they change.
  const int64_t kGraphIters = bw->sched_graph;
  const int ti = std::is_same<T, float>::value ? 1 : 0;
  if (bw->graph_mode < 0) {
    const char* e = getenv("MBL_BATCH_GRAPHS");
    bw->graph_mode = (e && std::string(e) == "0") ? 0 : 1;
  }
  const bool use_graph = bw->graph_mode == 1;
  hipGraphExec_t& gx = bw->graph[ti][precond];
  if (use_graph && (bw->graph_tol[ti][precond] != tol || bw->graph_kmax[ti][precond] != kmax ||
                    bw->graph_x[ti][precond] != (void*)x) && gx) {
    (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  }
  if (use_graph && !gx) {
    // captured on the workspace's own stream (nothing runs during capture),
    // launched on the caller's stream
    hipGraph_t g = nullptr;
    MBL_HIP(hipStreamBeginCapture(bw->cap, hipStreamCaptureModeThreadLocal));
    mbl_status cst = MBL_OK;
    for (int64_t k = 2; k <= kGraphIters + 1 && cst == MBL_OK; ++k) cst = iteration(k, bw->cap);
    hipError_t ee = hipStreamEndCapture(bw->cap, &g);
    if (cst != MBL_OK) {
      if (g) (void)hipGraphDestroy(g);
      return cst;
    }
    MBL_HIP(ee);
    ee = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MBL_HIP(ee);
    bw->graph_tol[ti][precond] = tol;
    bw->graph_kmax[ti][precond] = kmax;
    bw->graph_x[ti][precond] = (void*)x;
  }
  const int64_t kChunkIters = 2 * kGraphIters;
  int64_t issued = 0;
  int pending = 0, slot = 0;
  bool done = false;
  int64_t snap_iter[2] = {0, 0};
  // restart the realizations in `restart` at iteration K = issued + 1: z_K =
  // rhs, z_{K-1} = 0, q_K = M^{-1} z_K, d = x = 0, and their initial state
  // (marked fresh) in the slot the Givens step of iteration K reads
  auto restart_lanes = [&](const std::vector<int>& restart, const double* rhs) -> mbl_status {
    const int64_t K = issued + 1;
    if (K % dxg != 2 % dxg || kGraphIters % kRing != 0) {
      set_error("internal: streaming restart off the iteration grid");
      return MBL_ERR_NUMERIC;
    }
    MBL_HIP(hipMemcpyAsync(hook->mask_dev, restart.data(), sizeof(int) * R, hipMemcpyHostToDevice,
                           s));
    const size_t lds = blds_bytes(R, b->L, b->nlo);
    const dim3 g(G), blk(kBWG);
    const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                        \
  case LL * 64 + NN:                                                                           \
    hipLaunchKernelGGL((k_blane_init<LL>), g, blk, lds, s, B, Q, precond, hook->mask_dev, rhs, \
                       (double*)Z[K & 1], (double*)Z[(K + 1) & 1], (double*)Qv[K % kRing],     \
                       (double*)D[0], (double*)D[1], (double*)x, hook->part_dev);            \
    break;
    MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
    MBL_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_blane_state, dim3(R), dim3(kWG), 0, s, hook->part_dev, G, R,
                       hook->mask_dev, tol, kmax, S + ((K + kRing - 2) % kRing) * R);
    MBL_HIP(hipGetLastError());
    return MBL_OK;
  };
  auto check = [&](int which) -> mbl_status {
    MBL_HIP(hipEventSynchronize(bw->ev[which]));
    if (hook) {
      std::vector<int> restart(R, 0);
      const double* rhs = nullptr;
      bool keep = true;
      MBL_TRY(hook->on_snapshot(bw->h_state + which * R, snap_iter[which], issued + 1, restart,
                                &rhs, keep));
      bool any = false;
      for (int r = 0; r < R; ++r) any = any || restart[r];
      if (any) MBL_TRY(restart_lanes(restart, rhs));
      if (!keep) done = true;
      return MBL_OK;
    }
    bool all = true;
    for (int r = 0; r < R; ++r) all = all && bw->h_state[which * R + r].done;
    if (all) done = true;
    return MBL_OK;
  };
  if (hook && (!use_graph || !std::is_same<T, double>::value)) {
    set_error("internal: the streaming form needs FP64 and captured graphs");
    return MBL_ERR_ARG;
  }
  if (kmax >= 1) {
    MBL_TRY(iteration(1, s));
    issued = 1;
  }
  while (!done && (hook || issued < kmax)) {
    const int64_t k_end = hook ? issued + kChunkIters : std::min(kmax, issued + kChunkIters);
    if (use_graph && k_end - issued == kChunkIters) {
      for (int64_t rep = 0; rep < kChunkIters / kGraphIters; ++rep)
        MBL_HIP(hipGraphLaunch(gx, s));
    } else {
      for (int64_t k = issued + 1; k <= k_end; ++k) MBL_TRY(iteration(k, s));
    }
    issued = k_end;
    // the state after iteration issued - 1 is the newest one on the device
    MBL_HIP(hipMemcpyAsync(bw->h_state + slot * R, S + ((issued - 1) % kRing) * R,
                           sizeof(BState) * R, hipMemcpyDeviceToHost, s));
    MBL_HIP(hipEventRecord(bw->ev[slot], s));
    snap_iter[slot] = issued - 1;
    ++pending;
    if (pending == 2) {
      MBL_TRY(check(slot ^ 1));
      --pending;
    }
    slot ^= 1;
  }
  if (hook) {
    MBL_HIP(hipStreamSynchronize(s));
    return MBL_OK;
  }
  if (pending > 0) MBL_TRY(check(slot ^ 1));
  if (issued >= 1) MBL_TRY(finish(issued, s));
  MBL_HIP(hipMemcpyAsync(bw->h_state, S + (issued % kRing) * R, sizeof(BState) * R,
                         hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  fin.assign(bw->h_state, bw->h_state + R);
  for (const BState& st : fin)
    if (st.bad) {
      set_error("batched MINRES met a non-finite value");
      return MBL_ERR_NUMERIC;
    }
  return MBL_OK;
}

static mbl_status baxpby(mbl_batch_s* bw, int64_t n, const std::vector<double>& a, const double* x,
                         const std::vector<double>& bb, double* y, hipStream_t s);

// Batched MINRES for (H_r - sigma_r) x_r = b_r from x0 = 0 (fields and shifts
// already uploaded). FP64, or FP32 inner solves with FP64 residual restarts.
// active[r] = 0 skips realization r (its x is left at 0).
static mbl_status bminres_run(mbl_basis_s* b, mbl_batch_s* bw, int precision, int precond,
                              const double* rhs, double* x, double tol, int64_t kmax,
                              const std::vector<int>& active, hipStream_t s,
                              std::vector<int64_t>& iters, std::vector<double>& phi) {
  const int R = bw->R;
  const int64_t n = b->n;
  BatchDev Q{bw->h, bw->c0, R, bw->sched_grid};
  iters.assign(R, 0);
  phi.assign(R, 0.0);
  std::vector<double> sc(R);
  if (precision == MBL_FP64) {
    for (int r = 0; r < R; ++r) sc[r] = active[r] ? 1.0 : 0.0;
    MBL_HIP(hipMemcpyAsync(bw->scale, sc.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    std::vector<BState> fin;
    MBL_TRY(bminres_core<double>(b, bw, Q, precond, rhs, bw->scale, x, tol, kmax, s, fin));
    for (int r = 0; r < R; ++r) {
      iters[r] = fin[r].k;
      phi[r] = std::fabs(fin[r].phi);
    }
    return MBL_OK;
  }
  // FP32 inner solves: x64 starts at 0, restart from the FP64 residual. A
  // realization whose cycle fails to cut its FP64 residual by kMinCycleGain
  // leaves the FP32 phase; those are finished together by FP64 MINRES on the
  // residual (see the single-realization solver for the reasoning).
  const double eta = 1e-3;
  const double kMinCycleGain = 10.0;
  const int max_cycles = 60;
  MBL_HIP(hipMemsetAsync(x, 0, sizeof(double) * n * R, s));
  std::vector<double> sums(2 * R), prev(R, INFINITY);
  std::vector<int> fp32_phase(R, 1);
  for (int cycle = 0;; ++cycle) {
    MBL_TRY(launch_bresidual(b, Q, precond, rhs, x, bw->r64, bw->partials1, s));
    MBL_TRY(breduce_host(bw, bw->partials1, bgrid(b, R, Q.grid), 2, sums.data(), s));
    bool any = false, any_fp64 = false;
    double worst = 0;
    for (int r = 0; r < R; ++r) {
      const double rM = std::sqrt(sums[2 * r]);
      phi[r] = rM;
      if (!std::isfinite(rM) && active[r]) {
        set_error("non-finite residual in batched FP32-inner MINRES");
        return MBL_ERR_NUMERIC;
      }
      const bool open = active[r] && rM >= tol && iters[r] < kmax;
      if (open && fp32_phase[r] && (cycle >= max_cycles || rM > prev[r] / kMinCycleGain))
        fp32_phase[r] = 0;
      if (open && !fp32_phase[r]) any_fp64 = true;
      const bool go = open && fp32_phase[r];
      sc[r] = go ? 1.0 / rM : 0.0;
      bw->h_stage[r] = go ? rM : 0.0;
      if (go) prev[r] = rM;
      any = any || go;
      if (go) worst = std::max(worst, tol / rM);
    }
    if (!any) {
      if (any_fp64) {
        // FP64 finish: A e = r for the realizations that left the FP32 phase
        for (int r = 0; r < R; ++r)
          sc[r] = (active[r] && phi[r] >= tol && !fp32_phase[r]) ? 1.0 : 0.0;
        MBL_HIP(hipMemcpyAsync(bw->scale, sc.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
        std::vector<BState> fin;
        MBL_TRY(bminres_core<double>(b, bw, Q, precond, bw->r64, bw->scale, bw->t64, tol, kmax, s,
                                     fin));
        for (int r = 0; r < R; ++r) iters[r] += fin[r].k;
        std::vector<double> ones(R, 1.0);
        MBL_TRY(baxpby(bw, n, ones, bw->t64, ones, x, s));
        MBL_TRY(launch_bresidual(b, Q, precond, rhs, x, bw->r64, bw->partials1, s));
        MBL_TRY(breduce_host(bw, bw->partials1, bgrid(b, R, Q.grid), 2, sums.data(), s));
        for (int r = 0; r < R; ++r) phi[r] = std::sqrt(sums[2 * r]);
      }
      break;
    }
    MBL_HIP(hipMemcpyAsync(bw->scale, sc.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    MBL_HIP(hipMemcpyAsync(bw->scale2, bw->h_stage, sizeof(double) * R, hipMemcpyHostToDevice, s));
    const double inner_tol = std::max(eta, 0.5 * worst);
    std::vector<BState> fin;
    MBL_TRY(bminres_core<float>(b, bw, Q, precond, bw->r64, bw->scale, (float*)bw->e, inner_tol,
                                kmax, s, fin));
    for (int r = 0; r < R; ++r) iters[r] += fin[r].k;
    hipLaunchKernelGGL(k_badd_scaled, dim3(bflat_grid(n * R)), dim3(kWG), 0, s, n, R, bw->scale2,
                       (const float*)bw->e, x);
    MBL_HIP(hipGetLastError());
    MBL_HIP(hipStreamSynchronize(s));
  }
  return MBL_OK;
}

static mbl_status bdot_host(mbl_batch_s* bw, int64_t n, const double* x, const double* y,
                            double* out, hipStream_t s) {
  const int R = bw->R;
  const int G = std::max<int>(1, std::min<int64_t>(512, (n + 255) / 256));
  hipLaunchKernelGGL(k_bdot, dim3(G), dim3(kWG), 0, s, n, R, x, y, bw->partials1);
  MBL_HIP(hipGetLastError());
  return breduce_host(bw, bw->partials1, G, 1, out, s);
}

static mbl_status baxpby(mbl_batch_s* bw, int64_t n, const std::vector<double>& a, const double* x,
                         const std::vector<double>& bb, double* y, hipStream_t s) {
  const int R = bw->R;
  MBL_HIP(hipStreamSynchronize(s));
  std::copy(a.begin(), a.end(), bw->h_stage);
  std::copy(bb.begin(), bb.end(), bw->h_stage + R);
  MBL_HIP(hipMemcpyAsync(bw->scale, bw->h_stage, sizeof(double) * R, hipMemcpyHostToDevice, s));
  MBL_HIP(hipMemcpyAsync(bw->scale2, bw->h_stage + R, sizeof(double) * R, hipMemcpyHostToDevice,
                         s));
  hipLaunchKernelGGL(k_baxpby, dim3(bflat_grid(n * R)), dim3(kWG), 0, s, n, R, bw->scale, x,
                     bw->scale2, y);
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

static mbl_status bcgs_pass(mbl_batch_s* bw, int64_t n, int k, double* w, hipStream_t s) {
  const int R = bw->R;
  const int G = std::max<int>(1, std::min<int64_t>(256, (n + 255) / 256));
  const int64_t vstride = n * R;
  hipLaunchKernelGGL(k_bmultidot, dim3(G, (k + 3) / 4), dim3(kWG), 0, s, n, R, bw->V, vstride, k,
                     w, bw->partials2);
  MBL_HIP(hipGetLastError());
  // coef[c * R + r] = sum_g partials[(g * k + c) * R + r]: per-realization reduce with k*R values
  hipLaunchKernelGGL(k_breduce, dim3(k * R), dim3(kWG), 0, s, bw->partials2, G, k * R, 1,
                     bw->coef);
  MBL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bcgs_update, dim3(bflat_grid(n * R)), dim3(kWG), sizeof(double) * k * R, s,
                     n, R, bw->V, vstride, k, bw->coef, w);
  MBL_HIP(hipGetLastError());
  return MBL_OK;
}

double gershgorin_bound(const mbl_basis_s* b, const double* h);

// norms ||(H_r - shift_r) v_r|| for all r (fields uploaded with shifts)
static mbl_status bapply_norms(mbl_basis_s* b, mbl_batch_s* bw, const double* v, double* out,
                               hipStream_t s) {
  BatchDev Q{bw->h, bw->c0, bw->R, bw->sched_grid};
  MBL_TRY((launch_bapply<double, 0, false>(b, Q, BGivens{}, v, bw->t64, nullptr, s)));
  MBL_TRY(bdot_host(bw, b->n, bw->t64, bw->t64, out, s));
  for (int r = 0; r < bw->R; ++r) out[r] = std::sqrt(out[r]);
  return MBL_OK;
}

static mbl_status bsi_lanczos_run(mbl_basis_s* b, mbl_batch_s* bw, const double* h,
                                  const double* sigma, int nev, int mmax, double minres_tol,
                                  int64_t minres_kmax, double eig_tol, double gap_tol,
                                  const double* escale_in, const double* v0, uint64_t seed,
                                  int precision, int precond, double* evals, double* evecs,
                                  double* resid, mbl_si_info* info, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int R = bw->R, L = b->L;
  const int64_t n = b->n, NR = n * R;
  std::vector<double> escale(R);
  for (int r = 0; r < R; ++r)
    escale[r] = (escale_in && escale_in[r] > 0) ? escale_in[r]
                                                : gershgorin_bound(b, h + (size_t)r * L);
  MBL_TRY(bupload(bw, h, sigma, s));
  double* V = bw->V;
  if (v0)
    MBL_HIP(hipMemcpyAsync(V, v0, sizeof(double) * NR, hipMemcpyDeviceToDevice, s));
  else
    MBL_HIP(launch_splitmix(NR, seed, V, s));
  std::vector<double> nv(R), ones(R, 1.0), zeros(R, 0.0);
  MBL_TRY(bdot_host(bw, n, V, V, nv.data(), s));
  std::vector<double> inv(R);
  for (int r = 0; r < R; ++r) {
    if (!(nv[r] > 0) || !std::isfinite(nv[r])) {
      set_error("start vector has zero or non-finite norm");
      return MBL_ERR_ARG;
    }
    inv[r] = 1.0 / std::sqrt(nv[r]);
  }
  MBL_TRY(baxpby(bw, n, inv, V, zeros, V, s));
  std::vector<std::vector<double>> al(R), be(R), theta(R), Y(R);
  std::vector<std::vector<int>> sel(R);
  std::vector<int> active(R, 1), ksteps(R, 0);
  std::vector<double> beta_k(R, 0.0);
  int64_t total_iters = 0, lockstep_iters = 0;
  std::vector<int64_t> its, rits(R, 0);
  std::vector<double> phis;
  int k = 0;
  std::vector<double> alpha(R), bb(R), nav(R);
  for (k = 1; k <= mmax; ++k) {
    double* vk = V + (size_t)(k - 1) * NR;
    MBL_TRY(bupload(bw, h, sigma, s));
    MBL_TRY(bminres_run(b, bw, precision, precond, vk, bw->x, minres_tol, minres_kmax, active, s,
                        its, phis));
    int64_t most = 0;
    for (int r = 0; r < R; ++r) {
      total_iters += its[r];
      rits[r] += its[r];
      most = std::max(most, its[r]);
    }
    lockstep_iters += most;   // the iterations the batch launched for this step
    // w = x - beta_k v_{k-1}
    MBL_HIP(hipMemcpyAsync(bw->w, bw->x, sizeof(double) * NR, hipMemcpyDeviceToDevice, s));
    if (k > 1) {
      std::vector<double> mb(R);
      for (int r = 0; r < R; ++r) mb[r] = -beta_k[r];
      MBL_TRY(baxpby(bw, n, mb, V + (size_t)(k - 2) * NR, ones, bw->w, s));
    }
    MBL_TRY(bdot_host(bw, n, vk, bw->w, alpha.data(), s));
    {
      std::vector<double> ma(R);
      for (int r = 0; r < R; ++r) ma[r] = -alpha[r];
      MBL_TRY(baxpby(bw, n, ma, vk, ones, bw->w, s));
    }
    MBL_TRY(bcgs_pass(bw, n, k, bw->w, s));
    MBL_TRY(bcgs_pass(bw, n, k, bw->w, s));
    MBL_TRY(bdot_host(bw, n, bw->w, bw->w, bb.data(), s));
    std::vector<double> invb(R, 0.0);
    for (int r = 0; r < R; ++r) {
      if (!active[r]) continue;
      const double bn = std::sqrt(bb[r]);
      al[r].push_back(alpha[r]);
      be[r].push_back(bn);
      ksteps[r] = k;
      if (!std::isfinite(alpha[r]) || !std::isfinite(bn)) {
        set_error("non-finite Lanczos coefficient (batched)");
        return MBL_ERR_NUMERIC;
      }
      theta[r].assign(k, 0.0);
      Y[r].assign((size_t)k * k, 0.0);
      if (tridiag_eig(k, al[r].data(), be[r].data(), theta[r].data(), Y[r].data()) != 0) {
        set_error("tridiagonal eigensolver did not converge (batched)");
        return MBL_ERR_NUMERIC;
      }
      double tmax = 0;
      for (double t : theta[r]) tmax = std::max(tmax, std::fabs(t));
      invb[r] = (bn > 1e-14 * tmax) ? 1.0 / bn : 0.0;
      beta_k[r] = bn;
    }
    // v_{k+1} = w / beta_{k+1} (zero for realizations that stopped or broke down)
    double* vn = V + (size_t)k * NR;
    MBL_TRY(baxpby(bw, n, invb, bw->w, zeros, vn, s));
    MBL_TRY(bapply_norms(b, bw, vn, nav.data(), s));
    bool all_conv = true;
    for (int r = 0; r < R; ++r) {
      if (!active[r]) continue;
      if (k < nev) {
        all_conv = false;
        continue;
      }
      const int kr = k;
      std::vector<int> idx(kr);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
        return std::fabs(theta[r][a]) > std::fabs(theta[r][c]);
      });
      sel[r].assign(idx.begin(), idx.begin() + nev);
      bool conv = true;
      const bool broke = invb[r] == 0.0;
      for (int i : sel[r]) {
        const double est = broke ? 0.0
                                 : std::fabs(be[r].back() * Y[r][(size_t)i * kr + (kr - 1)] /
                                             theta[r][i]) * nav[r];
        const double lam = sigma[r] + 1.0 / theta[r][i];
        double gap = INFINITY;
        for (int jj = 0; jj < kr; ++jj)
          if (jj != i) gap = std::min(gap, std::fabs(sigma[r] + 1.0 / theta[r][jj] - lam));
        bool ok = est <= eig_tol * escale[r];
        if (gap_tol > 0) ok = ok && est <= gap_tol * gap;
        conv = conv && ok;
      }
      if (conv || broke) active[r] = 0;
      else all_conv = false;
    }
    if (std::getenv("MBL_VERBOSE")) {   // one line per lockstep Lanczos step (long runs)
      int live = 0;
      for (int r = 0; r < R; ++r) live += active[r];
      std::fprintf(stderr, "[mbl] batched si_lanczos step %d: %d of %d realizations still "
                   "stepping, minres total %lld, lockstep %lld\n", k, live, R,
                   (long long)total_iters, (long long)lockstep_iters);
    }
    if (all_conv) break;
  }
  if (k > mmax) k = mmax;
  const int kmaxr = *std::max_element(ksteps.begin(), ksteps.end());
  // Ritz vectors: U_t[:, r] = V[:, :k_r, r] Y_r[:, sel_t]; Y padded to kmaxr rows
  std::vector<double> Ys((size_t)R * kmaxr * nev, 0.0);
  std::vector<double> lam((size_t)R * nev);
  for (int r = 0; r < R; ++r) {
    const int kr = ksteps[r];
    if ((int)sel[r].size() < nev) {
      set_error("Krylov space became invariant before nev steps (batched)");
      return MBL_ERR_NUMERIC;
    }
    std::sort(sel[r].begin(), sel[r].end(), [&](int a, int c) {
      return sigma[r] + 1.0 / theta[r][a] < sigma[r] + 1.0 / theta[r][c];
    });
    for (int t = 0; t < nev; ++t) {
      lam[(size_t)r * nev + t] = sigma[r] + 1.0 / theta[r][sel[r][t]];
      for (int c = 0; c < kr; ++c)
        Ys[((size_t)r * kmaxr + c) * nev + t] = Y[r][(size_t)sel[r][t] * kr + c];
    }
  }
  MBL_HIP(hipMemcpyAsync(bw->ycoef, Ys.data(), sizeof(double) * Ys.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_britz, dim3(bflat_grid(NR), nev), dim3(kWG), 0, s, n, R, V, NR, kmaxr,
                     bw->ycoef, nev, evecs, NR);
  MBL_HIP(hipGetLastError());
  // normalise and explicit residuals ||H_r u - lambda u||
  std::vector<double> nn(R), invn(R), lt(R);
  for (int t = 0; t < nev; ++t) {
    double* u = evecs + (size_t)t * NR;
    MBL_TRY(bdot_host(bw, n, u, u, nn.data(), s));
    for (int r = 0; r < R; ++r) invn[r] = 1.0 / std::sqrt(nn[r]);
    MBL_TRY(baxpby(bw, n, invn, u, zeros, u, s));
    for (int r = 0; r < R; ++r) lt[r] = lam[(size_t)r * nev + t];
    MBL_TRY(bupload(bw, h, lt.data(), s));
    std::vector<double> rn(R);
    MBL_TRY(bapply_norms(b, bw, u, rn.data(), s));
    for (int r = 0; r < R; ++r) {
      evals[(size_t)r * nev + t] = lam[(size_t)r * nev + t];
      if (resid) resid[(size_t)r * nev + t] = rn[r];
    }
  }
  MBL_HIP(hipStreamSynchronize(s));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  int all_ok = 1;
  for (int r = 0; r < R; ++r) {
    int nconv = 0;
    double mx = 0;
    for (int t = 0; t < nev; ++t) {
      const double rr = resid ? resid[(size_t)r * nev + t] : 0.0;
      mx = std::max(mx, rr / escale[r]);
      if (rr <= eig_tol * escale[r]) ++nconv;
    }
    if (nconv < nev) all_ok = 0;
    if (info) {
      info[r].steps = ksteps[r];
      info[r].nconv = nconv;
      info[r].minres_iters = rits[r];
      info[r].max_rel_resid = mx;
      info[r].seconds = secs;
    }
  }
  if (!all_ok) {
    set_error("some batched eigenpairs did not converge");
    return MBL_WARN_NOCONV;
  }
  return MBL_OK;
}

// ---- streaming form ---------------------------------------------------------
// Each lane of the batch runs its own realization through Alg. 1. The lanes
// share the MINRES launches (one batched iteration serves every lane), but a
// lane's solve ends on its own: the hook below takes that lane's Lanczos
// step (w = x - beta_k v_{k-1}, alpha_k, two classical Gram-Schmidt passes,
// beta_{k+1}, v_{k+1}, the eigenpairs of T_k and the stopping rule of the
// lockstep form) and restarts its MINRES on v_{k+1} while the other lanes
// iterate on. A lane whose realization has converged writes its Ritz pairs,
// residuals and twist overlaps and takes the next realization. The lockstep
// form instead launches, per Lanczos step, as many iterations as the
// slowest lane needs.
struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

static mbl_status dev_alloc(DevMem& m, size_t bytes) {
  if (hipMalloc(&m.p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed (streaming batch)");
    return MBL_ERR_NOMEM;
  }
  return MBL_OK;
}

mbl_status bstream_si_lanczos(mbl_basis b, mbl_batch bw, StreamProblem* P, int nprob, int nev,
                              int mmax, double minres_tol, int64_t minres_kmax, double eig_tol,
                              double gap_tol, int precond, hipStream_t s) {
  const int R = bw->R, L = b->L;
  const int64_t n = b->n, NR = n * R, vstride = NR;
  if (nprob <= 0) return MBL_OK;
  if (mmax < 1 || mmax > bw->mmax || nev < 1 || nev > bw->nevmax || nev > mmax) {
    set_error("streaming batch: mmax or nev beyond the workspace");
    return MBL_ERR_ARG;
  }
  const bool verbose = std::getenv("MBL_VERBOSE") != nullptr;
  const int G = bgrid(b, R, bw->sched_grid);
  const int GC = std::max<int>(1, std::min<int64_t>(256, (n + 255) / 256));   // CGS groups
  DevMem mask, part, kidx, part3, U, vtmp;
  MBL_TRY(dev_alloc(mask, sizeof(int) * R));
  MBL_TRY(dev_alloc(part, sizeof(double) * (size_t)G * R));
  MBL_TRY(dev_alloc(kidx, sizeof(int) * R));
  MBL_TRY(dev_alloc(part3, sizeof(double) * (size_t)GC * (mmax + 1) * R));
  MBL_TRY(dev_alloc(U, sizeof(double) * (size_t)NR * nev));
  MBL_TRY(dev_alloc(vtmp, sizeof(double) * (size_t)n));
  double* T1 = bw->r64;   // v_k, then v_{k+1}, then the next right-hand sides
  double* T2 = bw->e;     // v_{k-1}
  double* Ub = static_cast<double*>(U.p);

  struct Lane {
    int prob = -1;          // realization, -1: idle
    int k = 0;              // Lanczos vectors v_1 .. v_k in V blocks 0 .. k-1
    bool solving = false;   // MINRES on v_k in flight
    int64_t K0 = 1;         // iteration its solve started at
    double beta_k = 0.0;
    std::vector<double> al, be, theta, Y;
    int64_t iters = 0;
    int noconv = 0;
  };
  std::vector<Lane> lane(R);
  std::vector<double> Hh((size_t)R * L, 0.0), C0(R, 0.0);
  int next = 0, done_probs = 0;
  const auto t0 = std::chrono::steady_clock::now();
  auto secs = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };

  auto lane_shift = [&](int r, double shift) {
    double sh = 0;
    for (int j = 0; j < L; ++j) sh += Hh[(size_t)r * L + j];
    C0[r] = 0.25 * L + 0.5 * sh - shift;
  };
  auto upload = [&]() -> mbl_status {
    MBL_HIP(hipStreamSynchronize(s));   // staging buffer reuse
    std::copy(Hh.begin(), Hh.end(), bw->h_stage);
    std::copy(C0.begin(), C0.end(), bw->h_stage + (size_t)R * L);
    MBL_HIP(hipMemcpyAsync(bw->h, bw->h_stage, sizeof(double) * R * L, hipMemcpyHostToDevice, s));
    MBL_HIP(hipMemcpyAsync(bw->c0, bw->h_stage + (size_t)R * L, sizeof(double) * R,
                           hipMemcpyHostToDevice, s));
    MBL_HIP(hipStreamSynchronize(s));
    bw->last_up.clear();   // the lockstep form's upload cache no longer holds
    return MBL_OK;
  };
  auto put_kidx = [&](const std::vector<int>& kv) -> mbl_status {
    MBL_HIP(hipStreamSynchronize(s));
    MBL_HIP(hipMemcpyAsync(kidx.p, kv.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
    MBL_HIP(hipStreamSynchronize(s));
    return MBL_OK;
  };
  // lane r takes realization p: fields, shift, and V column (all blocks 0,
  // block 0 the raw start vector; normalised by normalise_new)
  auto assign = [&](int r, int p) -> mbl_status {
    Lane& ln = lane[r];
    ln = Lane();
    ln.prob = p;
    ln.k = 1;
    std::copy(P[p].h, P[p].h + L, Hh.begin() + (size_t)r * L);
    lane_shift(r, P[p].sigma);
    MBL_HIP(launch_splitmix(n, P[p].seed, static_cast<double*>(vtmp.p), s));
    hipLaunchKernelGGL(k_blane_reset, dim3(bflat_grid(n)), dim3(kWG), 0, s, n, R, r, bw->V,
                       vstride, mmax + 1, static_cast<const double*>(vtmp.p));
    MBL_HIP(hipGetLastError());
    return MBL_OK;
  };
  auto normalise_new = [&](const std::vector<int>& fresh) -> mbl_status {
    std::vector<double> nv(R), a(R, 1.0), zero(R, 0.0);
    MBL_TRY(bdot_host(bw, n, bw->V, bw->V, nv.data(), s));
    for (int r = 0; r < R; ++r) {
      if (!fresh[r]) continue;
      if (!(nv[r] > 0) || !std::isfinite(nv[r])) {
        set_error("start vector has zero or non-finite norm");
        return MBL_ERR_NUMERIC;
      }
      a[r] = 1.0 / std::sqrt(nv[r]);
    }
    return baxpby(bw, n, a, bw->V, zero, bw->V, s);
  };

  // finish the realizations of the lanes in fin: Ritz vectors of the pairs
  // nearest sigma, normalised; explicit residuals; twist overlaps; outputs
  auto finish = [&](const std::vector<int>& fin, std::vector<std::vector<int>>& sel)
      -> mbl_status {
    for (int r = 0; r < R; ++r) {   // the selected pairs in ascending eigenvalue
      if (!fin[r]) continue;
      const double sg = P[lane[r].prob].sigma;
      const std::vector<double>& th = lane[r].theta;
      std::sort(sel[r].begin(), sel[r].end(),
                [&](int a, int c) { return sg + 1.0 / th[a] < sg + 1.0 / th[c]; });
    }
    int kmaxr = 1;
    for (int r = 0; r < R; ++r)
      if (fin[r]) kmaxr = std::max(kmaxr, (int)lane[r].al.size());
    std::vector<double> Ys((size_t)R * kmaxr * nev, 0.0), lam((size_t)R * nev, 0.0);
    for (int r = 0; r < R; ++r) {
      if (!fin[r]) continue;
      const Lane& ln = lane[r];
      const int kr = (int)ln.al.size();
      for (int t = 0; t < nev; ++t) {
        lam[(size_t)r * nev + t] = P[ln.prob].sigma + 1.0 / ln.theta[sel[r][t]];
        for (int c = 0; c < kr; ++c)
          Ys[((size_t)r * kmaxr + c) * nev + t] = ln.Y[(size_t)sel[r][t] * kr + c];
      }
    }
    MBL_HIP(hipStreamSynchronize(s));
    MBL_HIP(hipMemcpyAsync(bw->ycoef, Ys.data(), sizeof(double) * Ys.size(),
                           hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_britz, dim3(bflat_grid(NR), nev), dim3(kWG), 0, s, n, R, bw->V, vstride,
                       kmaxr, bw->ycoef, nev, Ub, NR);
    MBL_HIP(hipGetLastError());
    std::vector<double> nn(R), invn(R), zero(R, 0.0), rn((size_t)R * nev), rr(R);
    for (int t = 0; t < nev; ++t) {
      double* u = Ub + (size_t)t * NR;
      MBL_TRY(bdot_host(bw, n, u, u, nn.data(), s));
      for (int r = 0; r < R; ++r) invn[r] = (fin[r] && nn[r] > 0) ? 1.0 / std::sqrt(nn[r]) : 0.0;
      MBL_TRY(baxpby(bw, n, invn, u, zero, u, s));
    }
    // residuals ||H u - lambda u||: the finishing lanes' shifts set to lambda_t
    for (int t = 0; t < nev; ++t) {
      for (int r = 0; r < R; ++r)
        if (fin[r]) lane_shift(r, lam[(size_t)r * nev + t]);
      MBL_TRY(upload());
      MBL_TRY(bapply_norms(b, bw, Ub + (size_t)t * NR, rr.data(), s));
      for (int r = 0; r < R; ++r) rn[(size_t)r * nev + t] = rr[r];
    }
    std::vector<double> zz((size_t)R * nev * 2);
    {
      const mbl_status st = mbl_twist_expect_batched(b, bw, Ub, nev, zz.data(), s);
      if (st != MBL_OK) return st;
    }
    for (int r = 0; r < R; ++r) {
      if (!fin[r]) continue;
      Lane& ln = lane[r];
      StreamProblem& pr = P[ln.prob];
      const double sg = pr.sigma;
      // the pr.nev of the nev pairs nearest sigma, ascending
      std::vector<int> o(nev);
      std::iota(o.begin(), o.end(), 0);
      std::stable_sort(o.begin(), o.end(), [&](int a, int c) {
        return std::fabs(lam[(size_t)r * nev + a] - sg) < std::fabs(lam[(size_t)r * nev + c] - sg);
      });
      o.resize(pr.nev);
      std::sort(o.begin(), o.end());
      int nconv = 0;
      double mx = 0.0;
      for (int t = 0; t < pr.nev; ++t) {
        const int src = o[t];
        pr.evals[t] = lam[(size_t)r * nev + src];
        const double res = rn[(size_t)r * nev + src];
        if (pr.resid) pr.resid[t] = res;
        if (pr.z) {
          pr.z[2 * t] = zz[((size_t)r * nev + src) * 2];
          pr.z[2 * t + 1] = zz[((size_t)r * nev + src) * 2 + 1];
        }
        hipLaunchKernelGGL(k_blane_get, dim3(bflat_grid(n)), dim3(kWG), 0, s, n, R, r,
                           Ub + (size_t)src * NR, pr.evecs_dev + (size_t)t * n);
        MBL_HIP(hipGetLastError());
        mx = std::max(mx, res / pr.escale);
        if (res <= eig_tol * pr.escale) ++nconv;
      }
      pr.steps = (int)ln.al.size();
      pr.nconv = nconv;
      pr.minres_iters = ln.iters;
      pr.max_rel = mx;
      if (pr.status == MBL_OK && nconv < pr.nev) pr.status = MBL_WARN_NOCONV;
      ++done_probs;
      if (verbose)
        std::fprintf(stderr,
                     "[mbl] stream L=%d: realization %d done (%d steps, %lld MINRES iterations), "
                     "%d of %d (%.0f s)\n",
                     L, ln.prob, pr.steps, (long long)ln.iters, done_probs, nprob, secs());
      ln.prob = -1;
      ln.solving = false;
    }
    MBL_HIP(hipStreamSynchronize(s));
    return MBL_OK;
  };

  // the Lanczos step of the lanes in M (their solves x = (H - sigma)^{-1} v_k
  // are final in bw->x); sets conv[r] for lanes that stop, with their pair
  // selection in sel[r]
  auto lanczos_step = [&](const std::vector<int>& M, std::vector<int>& stop,
                          std::vector<std::vector<int>>& sel) -> mbl_status {
    std::vector<int> k1(R, -1), k2(R, -1);
    int kM = 1;
    for (int r = 0; r < R; ++r) {
      if (!M[r]) continue;
      k1[r] = lane[r].k - 1;
      k2[r] = lane[r].k >= 2 ? lane[r].k - 2 : -1;
      kM = std::max(kM, lane[r].k);
    }
    MBL_TRY(put_kidx(k1));
    hipLaunchKernelGGL(k_blane_gather, dim3(bflat_grid(NR)), dim3(kWG), 0, s, n, R, bw->V,
                       vstride, static_cast<const int*>(kidx.p), T1);
    MBL_TRY(put_kidx(k2));
    hipLaunchKernelGGL(k_blane_gather, dim3(bflat_grid(NR)), dim3(kWG), 0, s, n, R, bw->V,
                       vstride, static_cast<const int*>(kidx.p), T2);
    MBL_HIP(hipGetLastError());
    MBL_HIP(hipMemcpyAsync(bw->w, bw->x, sizeof(double) * NR, hipMemcpyDeviceToDevice, s));
    std::vector<double> a(R, 0.0), one(R, 1.0), zero(R, 0.0), alpha(R), bb(R);
    for (int r = 0; r < R; ++r)
      if (M[r] && lane[r].k >= 2) a[r] = -lane[r].beta_k;
    MBL_TRY(baxpby(bw, n, a, T2, one, bw->w, s));
    MBL_TRY(bdot_host(bw, n, T1, bw->w, alpha.data(), s));
    for (int r = 0; r < R; ++r) a[r] = M[r] ? -alpha[r] : 0.0;
    MBL_TRY(baxpby(bw, n, a, T1, one, bw->w, s));
    for (int pass = 0; pass < 2; ++pass) {   // CGS2 against v_1 .. v_k (zero blocks beyond)
      hipLaunchKernelGGL(k_bmultidot, dim3(GC, (kM + 3) / 4), dim3(kWG), 0, s, n, R, bw->V,
                         vstride, kM, bw->w, static_cast<double*>(part3.p));
      MBL_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_breduce, dim3(kM * R), dim3(kWG), 0, s,
                         static_cast<const double*>(part3.p), GC, kM * R, 1, bw->coef);
      MBL_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_bcgs_update, dim3(bflat_grid(NR)), dim3(kWG), sizeof(double) * kM * R,
                         s, n, R, bw->V, vstride, kM, bw->coef, bw->w);
      MBL_HIP(hipGetLastError());
    }
    MBL_TRY(bdot_host(bw, n, bw->w, bw->w, bb.data(), s));
    std::vector<double> invb(R, 0.0);
    for (int r = 0; r < R; ++r) {
      if (!M[r]) continue;
      Lane& ln = lane[r];
      const double bn = std::sqrt(bb[r]);
      if (!std::isfinite(alpha[r]) || !std::isfinite(bn)) {
        set_error("non-finite Lanczos coefficient (streaming batch)");
        return MBL_ERR_NUMERIC;
      }
      ln.al.push_back(alpha[r]);
      ln.be.push_back(bn);
      const int k = ln.k;
      ln.theta.assign(k, 0.0);
      ln.Y.assign((size_t)k * k, 0.0);
      if (tridiag_eig(k, ln.al.data(), ln.be.data(), ln.theta.data(), ln.Y.data()) != 0) {
        set_error("tridiagonal eigensolver did not converge (streaming batch)");
        return MBL_ERR_NUMERIC;
      }
      double tmax = 0;
      for (double t : ln.theta) tmax = std::max(tmax, std::fabs(t));
      invb[r] = (bn > 1e-14 * tmax) ? 1.0 / bn : 0.0;
      ln.beta_k = bn;
    }
    // v_{k+1} = w / beta_{k+1} into T1 and V block k
    MBL_TRY(baxpby(bw, n, invb, bw->w, zero, T1, s));
    std::vector<int> kn(R, -1);
    for (int r = 0; r < R; ++r)
      if (M[r] && lane[r].k <= mmax && invb[r] != 0.0) kn[r] = lane[r].k;
    MBL_TRY(put_kidx(kn));
    hipLaunchKernelGGL(k_blane_scatter, dim3(bflat_grid(NR)), dim3(kWG), 0, s, n, R, T1, bw->V,
                       vstride, static_cast<const int*>(kidx.p));
    MBL_HIP(hipGetLastError());
    std::vector<double> nav(R);
    MBL_TRY(bapply_norms(b, bw, T1, nav.data(), s));
    for (int r = 0; r < R; ++r) {
      if (!M[r]) continue;
      Lane& ln = lane[r];
      const int kr = ln.k;
      const bool broke = invb[r] == 0.0;
      bool conv = false;
      if (kr >= nev) {
        std::vector<int> idx(kr);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int x1, int x2) {
          return std::fabs(ln.theta[x1]) > std::fabs(ln.theta[x2]);
        });
        sel[r].assign(idx.begin(), idx.begin() + nev);
        const double sg = P[ln.prob].sigma, es = P[ln.prob].escale;
        conv = true;
        for (int i : sel[r]) {
          const double est = broke ? 0.0
                                   : std::fabs(ln.be.back() * ln.Y[(size_t)i * kr + (kr - 1)] /
                                               ln.theta[i]) * nav[r];
          const double lam = sg + 1.0 / ln.theta[i];
          double gap = INFINITY;
          for (int jj = 0; jj < kr; ++jj)
            if (jj != i) gap = std::min(gap, std::fabs(sg + 1.0 / ln.theta[jj] - lam));
          bool ok = est <= eig_tol * es;
          if (gap_tol > 0) ok = ok && est <= gap_tol * gap;
          conv = conv && ok;
        }
      }
      if (conv || broke || kr >= mmax) {
        if ((int)sel[r].size() < nev) {
          set_error("Krylov space became invariant before nev steps (streaming batch)");
          return MBL_ERR_NUMERIC;
        }
        if (broke) P[ln.prob].status = MBL_WARN_BREAKDOWN;
        stop[r] = 1;
      } else {
        ln.k = kr + 1;
      }
    }
    return MBL_OK;
  };

  // start: every lane takes a realization (or idles), all V blocks zero
  MBL_HIP(hipMemsetAsync(bw->V, 0, sizeof(double) * (size_t)NR * (mmax + 1), s));
  std::vector<int> fresh(R, 0);
  for (int r = 0; r < R && next < nprob; ++r) {
    MBL_TRY(assign(r, next++));
    fresh[r] = 1;
  }
  MBL_TRY(normalise_new(fresh));
  MBL_TRY(upload());
  std::vector<double> sc(R);
  for (int r = 0; r < R; ++r) {
    sc[r] = fresh[r] ? 1.0 : 0.0;
    lane[r].solving = fresh[r] != 0;
    lane[r].K0 = 1;
  }
  MBL_HIP(hipMemcpyAsync(bw->scale, sc.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));

  MinresHook hook;
  hook.mask_dev = static_cast<int*>(mask.p);
  hook.part_dev = static_cast<double*>(part.p);
  double last_report = 0.0;
  hook.on_snapshot = [&](const BState* st, int64_t iter, int64_t next_k, std::vector<int>& restart,
                         const double** rhs, bool& keep_going) -> mbl_status {
    std::vector<int> M(R, 0);
    bool anyM = false;
    for (int r = 0; r < R; ++r) {
      Lane& ln = lane[r];
      if (!ln.solving || iter < ln.K0 || !st[r].done) continue;
      if (st[r].bad) {
        set_error("batched MINRES met a non-finite value (streaming)");
        return MBL_ERR_NUMERIC;
      }
      ln.iters += st[r].k;
      if (st[r].k >= minres_kmax) ++ln.noconv;
      M[r] = 1;
      anyM = true;
    }
    if (anyM) {
      std::vector<int> stop(R, 0);
      std::vector<std::vector<int>> sel(R);
      MBL_TRY(lanczos_step(M, stop, sel));
      bool anystop = false;
      for (int r = 0; r < R; ++r) anystop = anystop || stop[r];
      std::vector<int> nw(R, 0);
      if (anystop) {
        MBL_TRY(finish(stop, sel));
        bool anynew = false;
        for (int r = 0; r < R; ++r)
          if (stop[r] && next < nprob) {
            MBL_TRY(assign(r, next++));
            nw[r] = 1;
            anynew = true;
          }
        if (anynew) MBL_TRY(normalise_new(nw));
        MBL_TRY(upload());   // fields of new lanes (and shifts of finished ones)
      }
      // the right-hand sides v_k of every lane that starts a solve
      std::vector<int> kv(R, -1);
      for (int r = 0; r < R; ++r) {
        if ((M[r] && !stop[r]) || nw[r]) {
          restart[r] = 1;
          kv[r] = lane[r].k - 1;
          lane[r].solving = true;
          lane[r].K0 = next_k;
        } else if (M[r]) {
          lane[r].solving = lane[r].prob >= 0;
        }
      }
      MBL_TRY(put_kidx(kv));
      hipLaunchKernelGGL(k_blane_gather, dim3(bflat_grid(NR)), dim3(kWG), 0, s, n, R, bw->V,
                         vstride, static_cast<const int*>(kidx.p), T1);
      MBL_HIP(hipGetLastError());
      *rhs = T1;
    }
    bool any = false;
    for (int r = 0; r < R; ++r) any = any || lane[r].solving;
    keep_going = any;
    if (verbose && secs() - last_report >= 30.0) {
      last_report = secs();
      int live = 0;
      for (int r = 0; r < R; ++r) live += lane[r].solving;
      std::fprintf(stderr, "[mbl] stream L=%d: %d of %d realizations done, %d lanes busy (%.0f s)\n",
                   L, done_probs, nprob, live, secs());
    }
    return MBL_OK;
  };
  BatchDev Q{bw->h, bw->c0, R, bw->sched_grid};
  std::vector<BState> fin;
  MBL_TRY(bminres_core<double>(b, bw, Q, precond, bw->V, bw->scale, bw->x, minres_tol,
                               minres_kmax, s, fin, &hook));
  if (done_probs != nprob) {
    set_error("internal: streaming batch ended with realizations left");
    return MBL_ERR_NUMERIC;
  }
  return MBL_OK;
}

static void free_batch(mbl_batch_s* w) {
  if (!w) return;
  double* bufs[] = {w->h, w->c0, w->z[0], w->z[1], w->d[0], w->d[1], w->p,
                    w->e, w->r64, w->t64, w->w, w->x, w->V, w->coef, w->ycoef, w->partials1,
                    w->partials2, w->red, w->scale, w->scale2, w->alph};
  for (double* p : bufs) (void)hipFree(p);
  for (double* p : w->q) (void)hipFree(p);
  if (w->stage_blocks) (void)hipFree(w->stage_blocks);
  if (w->stage_first) (void)hipFree(w->stage_first);
  (void)hipFree(w->S);
  for (auto& row : w->graph)
    for (auto& gx : row)
      if (gx) (void)hipGraphExecDestroy(gx);
  if (w->cap) (void)hipStreamDestroy(w->cap);
  if (w->h_state) hipHostFree(w->h_state);
  if (w->h_red) hipHostFree(w->h_red);
  if (w->h_stage) hipHostFree(w->h_stage);
  for (int i = 0; i < 2; ++i)
    if (w->ev[i]) hipEventDestroy(w->ev[i]);
  delete w;
}

static mbl_status create_batch(mbl_basis_s* b, int R, int mmax, int nevmax, mbl_batch_s** out) {
  mbl_batch_s* w = new (std::nothrow) mbl_batch_s();
  if (!w) {
    set_error("host allocation failed");
    return MBL_ERR_NOMEM;
  }
  w->basis = b;
  w->R = R;
  w->mmax = mmax;
  w->nevmax = nevmax;
  w->n = b->n;
  const size_t NR = (size_t)b->n * R;
  mbl_status st = MBL_OK;
  auto A = [&](double** p, size_t cnt) {
    if (st != MBL_OK) return;
    if (hipMalloc((void**)p, std::max<size_t>(cnt, 1) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("device allocation failed (batched workspace)");
      st = MBL_ERR_NOMEM;
      return;
    }
    w->bytes += (int64_t)(cnt * sizeof(double));
  };
  A(&w->h, (size_t)R * b->L);
  A(&w->c0, R);
  for (int i = 0; i < 2; ++i) {
    A(&w->z[i], NR);
    A(&w->d[i], NR);
  }
  for (int i = 0; i < kRing; ++i) A(&w->q[i], NR);
  A(&w->p, NR);
  A(&w->e, NR);
  A(&w->r64, NR);
  A(&w->t64, NR);
  A(&w->w, NR);
  A(&w->x, NR);
  if (mmax > 0) A(&w->V, NR * (size_t)(mmax + 1));
  A(&w->coef, (size_t)(mmax + 1) * R);
  A(&w->ycoef, (size_t)R * (mmax + 1) * std::max(nevmax, 1));
  w->part_elems = std::max<size_t>((size_t)kBGrid * R * 2, (size_t)256 * (mmax + 1) * R);
  A(&w->partials1, w->part_elems);
  A(&w->partials2, w->part_elems);
  A(&w->red, (size_t)std::max(R * 64, (mmax + 1) * R));
  A(&w->scale, R);
  A(&w->scale2, R);
  A(&w->alph, 2 * (size_t)R);
  if (st == MBL_OK && hipMalloc((void**)&w->S, sizeof(BState) * kRing * R) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed (batched state)");
    st = MBL_ERR_NOMEM;
  }
  if (st == MBL_OK &&
      (hipHostMalloc((void**)&w->h_state, sizeof(BState) * 4 * R) != hipSuccess ||
       hipHostMalloc((void**)&w->h_red, sizeof(double) * std::max(R * 64, (mmax + 1) * R)) !=
           hipSuccess ||
       hipHostMalloc((void**)&w->h_stage, sizeof(double) * ((size_t)R * (b->L + 1) + 4 * R)) !=
           hipSuccess)) {
    (void)hipGetLastError();
    set_error("pinned host allocation failed (batched)");
    st = MBL_ERR_NOMEM;
  }
  for (int i = 0; i < 2 && st == MBL_OK; ++i)
    if (hipEventCreateWithFlags(&w->ev[i], hipEventDisableTiming) != hipSuccess) {
      set_error("hipEventCreate failed");
      st = MBL_ERR_HIP;
    }
  if (st == MBL_OK && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess) {
    set_error("hipStreamCreate failed");
    st = MBL_ERR_HIP;
  }
  if (st != MBL_OK) {
    free_batch(w);
    return st;
  }
  *out = w;
  return MBL_OK;
}

static bool pow2(int R) { return R >= 2 && R <= kBMaxR && (R & (R - 1)) == 0; }

}  // namespace mbl

using namespace mbl;

extern "C" {

mbl_status mbl_batch_create(mbl_basis b, int R, int mmax, int nevmax, mbl_batch* out) {
  clear_error();
  MBL_ARG(b && out, "NULL argument");
  MBL_ARG(pow2(R), "R must be a power of two in [2, 32]");
  MBL_ARG(mmax >= 0 && mmax <= kMaxLanczos && nevmax >= 0 && nevmax <= std::max(mmax, 1),
          "need 0 <= nevmax <= mmax <= 1000");
  MBL_ARG(batched_split_supported(b), "batched form needs the library's default lo_bits for L");
  MBL_ARG(blds_bytes(R, b->L, b->nlo) <= 65536, "R too large for this L (LDS)");
  MBL_ARG((uint64_t)b->n * (uint64_t)R * sizeof(double) < ((uint64_t)1 << 31),
          "n * R * 8 bytes must stay below 2^31 (32-bit buffer offsets); use a smaller R");
  return create_batch(b, R, mmax, nevmax, out);
}

void mbl_batch_free(mbl_batch w) { free_batch(w); }

mbl_status mbl_batch_bytes(mbl_batch w, int64_t* bytes) {
  clear_error();
  MBL_ARG(w && bytes, "NULL argument");
  *bytes = w->bytes;
  return MBL_OK;
}

mbl_status mbl_batch_set_schedule(mbl_batch w, int grid, int graph_iters, int dx_group) {
  clear_error();
  MBL_ARG(w, "NULL argument");
  MBL_ARG(grid == 0 || (grid >= 8 && grid <= kBGrid && grid % 8 == 0),
          "grid must be 0 or a multiple of 8 in [8, 512]");
  MBL_ARG(graph_iters == 0 || graph_iters == 8 || graph_iters == 16 || graph_iters == 32,
          "graph_iters must be 0, 8, 16 or 32");
  MBL_ARG(dx_group == 0 || dx_group == 1 || dx_group == 2 || dx_group == 4,
          "dx_group must be 0, 1, 2 or 4");
  const int g = graph_iters ? graph_iters : 16, d = dx_group ? dx_group : 4;
  if (grid != w->sched_grid || g != w->sched_graph || d != w->sched_dx) {
    // captured MINRES graphs hold the old launch shapes
    for (auto& row : w->graph)
      for (auto& gx : row)
        if (gx) {
          (void)hipGraphExecDestroy(gx);
          gx = nullptr;
        }
  }
  w->sched_grid = grid;
  w->sched_graph = g;
  w->sched_dx = d;
  return MBL_OK;
}

mbl_status mbl_apply_H_batched(mbl_basis b, mbl_batch w, const double* h_host,
                               const double* sigma_host, const double* x_dev, double* y_dev,
                               void* stream) {
  clear_error();
  MBL_ARG(b && w && h_host && sigma_host && x_dev && y_dev, "NULL argument");
  MBL_ARG(w->basis == b, "batch workspace belongs to another basis");
  MBL_ARG(x_dev != y_dev, "x and y must not alias");
  for (int r = 0; r < w->R; ++r)
    MBL_ARG(fields_finite(b->L, h_host + (size_t)r * b->L) && std::isfinite(sigma_host[r]),
            "non-finite h or sigma");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  MBL_TRY(bupload(w, h_host, sigma_host, s));
  BatchDev Q{w->h, w->c0, w->R, w->sched_grid};
  if (staged_instance(b, w->R)) {
    MBL_TRY(staged_plan(b, w, s));
    return launch_bapply_staged<0>(b, w, Q, BGivens{}, x_dev, y_dev, nullptr, s);
  }
  return launch_bapply<double, 0, false>(b, Q, BGivens{}, x_dev, y_dev, nullptr, s);
}

mbl_status mbl_apply_H_batched_f32(mbl_basis b, mbl_batch w, const double* h_host,
                                   const double* sigma_host, const float* x_dev, float* y_dev,
                                   void* stream) {
  clear_error();
  MBL_ARG(b && w && h_host && sigma_host && x_dev && y_dev, "NULL argument");
  MBL_ARG(w->basis == b, "batch workspace belongs to another basis");
  MBL_ARG((const void*)x_dev != (const void*)y_dev, "x and y must not alias");
  for (int r = 0; r < w->R; ++r)
    MBL_ARG(fields_finite(b->L, h_host + (size_t)r * b->L) && std::isfinite(sigma_host[r]),
            "non-finite h or sigma");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  MBL_TRY(bupload(w, h_host, sigma_host, s));
  BatchDev Q{w->h, w->c0, w->R, w->sched_grid};
  return launch_bapply<float, 0, false>(b, Q, BGivens{}, x_dev, y_dev, nullptr, s);
}

mbl_status mbl_minres_solve_batched(mbl_basis b, mbl_batch w, const double* h_host,
                                    const double* sigma_host, const double* rhs_dev,
                                    double* x_dev, double tol, int64_t kmax, int precision,
                                    int precond, int64_t* iters_host, double* phi_host,
                                    void* stream) {
  clear_error();
  MBL_ARG(b && w && h_host && sigma_host && rhs_dev && x_dev, "NULL argument");
  MBL_ARG(w->basis == b, "batch workspace belongs to another basis");
  MBL_ARG(rhs_dev != x_dev, "rhs and x must not alias");
  MBL_ARG(tol > 0 && kmax >= 1, "bad tol or kmax");
  MBL_ARG(precision == MBL_FP64 || precision == MBL_FP32_INNER, "unknown precision");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  for (int r = 0; r < w->R; ++r)
    MBL_ARG(fields_finite(b->L, h_host + (size_t)r * b->L) && std::isfinite(sigma_host[r]),
            "non-finite h or sigma");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  MBL_TRY(bupload(w, h_host, sigma_host, s));
  std::vector<int> active(w->R, 1);
  std::vector<int64_t> its;
  std::vector<double> phi;
  MBL_TRY(bminres_run(b, w, precision, precond, rhs_dev, x_dev, tol, kmax, active, s, its, phi));
  MBL_HIP(hipStreamSynchronize(s));
  bool all = true;
  for (int r = 0; r < w->R; ++r) {
    if (iters_host) iters_host[r] = its[r];
    if (phi_host) phi_host[r] = phi[r];
    all = all && phi[r] < tol;
  }
  return all ? MBL_OK : MBL_WARN_NOCONV;
}

mbl_status mbl_si_lanczos_batched(mbl_basis b, mbl_batch w, const double* h_host,
                                  const double* sigma_host, int nev, int mmax, double minres_tol,
                                  int64_t minres_kmax, double eig_tol, double gap_tol,
                                  const double* escale_host, const double* v0_dev, uint64_t seed,
                                  int precision, int precond, double* evals_host,
                                  double* evecs_dev, double* resid_host, mbl_si_info* info_host,
                                  void* stream) {
  clear_error();
  MBL_ARG(b && w && h_host && sigma_host && evals_host && evecs_dev, "NULL argument");
  MBL_ARG(w->basis == b, "batch workspace belongs to another basis");
  MBL_ARG(nev >= 1 && nev <= w->nevmax, "need 1 <= nev <= nevmax of the batch workspace");
  MBL_ARG(mmax >= nev && mmax <= w->mmax && mmax <= b->n, "need nev <= mmax <= workspace mmax");
  MBL_ARG(minres_tol > 0 && minres_kmax >= 1 && eig_tol > 0, "bad tolerances");
  MBL_ARG(precision == MBL_FP64 || precision == MBL_FP32_INNER, "unknown precision");
  MBL_ARG(precond >= 0 && precond <= 2, "unknown preconditioner");
  for (int r = 0; r < w->R; ++r)
    MBL_ARG(fields_finite(b->L, h_host + (size_t)r * b->L) && std::isfinite(sigma_host[r]),
            "non-finite h or sigma");
  return bsi_lanczos_run(b, w, h_host, sigma_host, nev, mmax, minres_tol, minres_kmax, eig_tol,
                         gap_tol, escale_host, v0_dev, seed, precision, precond, evals_host,
                         evecs_dev, resid_host, info_host, reinterpret_cast<hipStream_t>(stream));
}

mbl_status mbl_twist_expect_batched(mbl_basis b, mbl_batch w, const double* psi_dev, int nvec,
                                    double* z_host, void* stream) {
  clear_error();
  MBL_ARG(b && w && psi_dev && z_host, "NULL argument");
  MBL_ARG(w->basis == b, "batch workspace belongs to another basis");
  MBL_ARG(nvec >= 1, "nvec must be >= 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int R = w->R, L = b->L;
  const int G = bgrid(b, R, w->sched_grid);
  MBL_ARG((size_t)G * R * 2 <= w->part_elems, "internal: partials too small");
  BTwistTab T{};
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < 2 * L; ++m) {
    T.c[m] = std::cos(pi * m / L);
    T.s[m] = std::sin(pi * m / L);
  }
  BatchDev Q{w->h, w->c0, R, w->sched_grid};
  const size_t lds = blds_bytes(R, L, b->nlo);
  const int64_t NR = b->n * R;
  for (int t = 0; t < nvec; ++t) {
    const DevBasis B = b->dev();
#define MBL_CASE(LL, NN)                                                                      \
  case LL * 64 + NN:                                                                         \
    hipLaunchKernelGGL((k_btwist<LL>), dim3(G, 1), dim3(kBWG), lds, s, B, Q, T,              \
                       psi_dev + (size_t)t * NR, NR, w->partials1);                          \
    break;
    MBL_BDISPATCH(MBL_CASE)
#undef MBL_CASE
    MBL_HIP(hipGetLastError());
    std::vector<double> out(2 * R);
    MBL_TRY(breduce_host(w, w->partials1, G, 2, out.data(), s));
    for (int r = 0; r < R; ++r) {
      z_host[((size_t)r * nvec + t) * 2] = out[2 * r];
      z_host[((size_t)r * nvec + t) * 2 + 1] = out[2 * r + 1];
    }
  }
  return MBL_OK;
}

}  // extern "C"
