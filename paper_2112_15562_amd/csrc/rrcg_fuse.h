// Pieces of the joint CG step (Sec. 2.4, eqs. RRCG:2-7) shared by the solver's own
// kernels and the product kernels that carry them as prologues and epilogues:
//   * the device-resident scalar layout;
//   * block partial sums of FP64 dot products, one value per block and slot;
//   * the finishing sums (beta of RRCG:5, the step s of RRCG:6, the Gramian scalars of
//     RRCG:2-3), done by every block of the kernel that consumes them: the launch
//     boundary makes the producer's partials visible without fences or atomics, and
//     every block sums the same partials in the same order, so all blocks hold the
//     same scalars;
//   * Fuse<T>, the arguments of the fused forms of the row transforms.
// The results are bitwise repeatable for a given launch configuration.
#pragma once
#include "common.h"

namespace bttb {

// Scalar array layout (doubles).
enum {
  S_ALPHA = 0, S_LPREV = 2, S_PHI = 4, S_THR = 6, S_BETA = 7, S_STEP = 9, S_GRAM = 11, S_FROZEN = 12,
  S_K = 14, S_CONV = 15, S_NONFIN = 16, S_G11 = 17, S_G22 = 18, S_G12 = 19, S_L = 20, S_PL = 22,
  S_PP = 24, S_QQ = 26, S_SIM = 28, S_COUNT = 32
};

// Partial-sum slots: ||l_i||^2; (p_i, l_i) and ||p_i||^2; ||q_i||^2 (q = A~ p); the Gramian
// sums (m1,m1), (m2,m2), (m1,m2); the misfits ||r~_i||^2.
enum {
  PB_L0 = 0, PB_L1, PB_PL0, PB_PP0, PB_PL1, PB_PP1, PB_Q0, PB_Q1, PB_G11, PB_G22, PB_G12, PB_F0, PB_F1,
  PB_NSLOT = 16
};
// Fused forms of the row transforms.
enum { FUSE_NONE = 0, FUSE_DIR = 1, FUSE_GRAD = 2, FUSE_QQ = 3, FUSE_RUPD = 4 };

template <typename T>
struct Fuse {
  int self;     // data set of this launch (0, 1)
  int lead;     // 1: block 0 of this launch records the finished scalars (first data set)
  int restart;  // beta = 0 in this step
  int coupled;  // joint beta and s (else per data set)
  int gram_w;   // Gramian on w m instead of m
  double lam[2];
  const T* l;     // DIR: gradient of this data set
  T* p;           // DIR: direction of this data set (the previous one, read)
  T* pout;        // DIR: where the new direction goes: p itself in the solve; a scratch copy in
                  //      the timing repeats, which thereby read and write the same values each time
  const T* m[2];  // GRAD: models of both data sets (original space)
  const T* w[2];  // GRAD: weights of both data sets
  const T* ma;    // GRAD: the regulariser's anchor of this data set in the original space (m_apr,
                  //       or m_prev for the previous-iterate anchor), or NULL for zero
  T* r;           // RUPD: weighted residual r~ of this data set, updated in place
  const T* q;     // RUPD: q = A~ p of this data set
  double* sc;     // scalars
  double* pb;     // [PB_NSLOT][pbs] partials
  int* pbn;       // [PB_NSLOT] number of partials in each slot
  int pbs;        // partials per slot (>= blocks of any reducing launch)
};

// Sum of x over the 64 lanes of a full wave, in the last lane (63): an exchange butterfly
// inside each row of 16 lanes through DPP moves (quad swaps by 1 and 2, then the mirrors of
// 8 and 16 lanes; both partners add the same two values), then the row sums r0..r3 carried
// up by the row broadcasts, leaving (r3 + r2) + (r1 + r0) in lane 63.
__device__ __forceinline__ double wave_sum_last(double x) {
  x += __builtin_amdgcn_update_dpp(0.0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x140, 0xF, 0xF, false);  // row_mirror
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// Per-wave sums of K values, each written by one lane to sh[k][wave]: with DPP and full
// waves the DPP sum, from lane 63; otherwise an xor butterfly through lane shuffles whose
// partners stay among the active lanes (blocks below 64 threads are a power of two), from
// lane 0.  The DPP form is faster; the butterfly needs fewer registers where a kernel has
// loads in flight.
template <int K, bool DPP>
__device__ __forceinline__ void wave_sums_to(double (&v)[K], double (&sh)[K][16]) {
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (DPP && blockDim.x >= 64) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_last(v[k]);
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
    }
  } else {
    // one level of all K butterflies at a time: their lane exchanges are in flight together,
    // so a level costs one LDS round trip rather than K (each sum adds the same terms in the
    // same order as K butterflies one after another)
    const int wsz = blockDim.x < 64 ? (int)blockDim.x : 64;
    for (int off = wsz >> 1; off >= 1; off >>= 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
    }
  }
}

// Sum of v over the block (every thread calls; blockDim a multiple of 64 or a power of two
// below 64, at most 1024) stored at pb[(slot0 + k) * pbs + bid]; block 0 of the nb blocks
// records their number.
template <int K, bool DPP = true>
__device__ __forceinline__ void block_partials(double (&v)[K], double* pb, int* pbn, int pbs, int slot0, int bid,
                                               int nb) {
  __shared__ double sh[K][16];
  wave_sums_to<K, DPP>(v, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[k][w];
      gstore(pb + (slot0 + k) * pbs + bid, s);
      if (bid == 0) gstore(pbn + slot0 + k, nb);
    }
  }
}

// Sums of K values over the block, left in v of every thread (blockDim a multiple of 64
// or a power of two below 64, at most 1024).  All lanes of a wave hold the same sum after
// the wave sum, and the waves' sums are added in a fixed order.
template <int K>
__device__ __forceinline__ void block_allreduce(double (&v)[K]) {
  __shared__ double sh[K][16];
  // (the xor butterfly: this runs in kernel prologues with their loads in flight, where the
  // DPP form's temporaries cost registers)
  wave_sums_to<K, false>(v, sh);
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Fixed-order totals of K slots' partials, in two stages so that a kernel can issue the
// loads before its own bulk loads and take the totals after them.  The counts and the first
// two partials of each thread go out together, in one round trip: those loads do not wait
// for the count (every index below pbs is allocated), and the ones past it add zero.  Each
// thread adds its partials in index order, as a plain strided loop would.
template <int K>
struct SlotSums {
  static constexpr int U = 2;
  const double* src[K];
  int n[K];
  double x[K][U];

  __device__ __forceinline__ void load(const double* pb, const int* pbn, int pbs, const int (&slot)[K]) {
    const int nt = blockDim.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      n[k] = gload(pbn + slot[k]);
      src[k] = pb + (long long)slot[k] * pbs;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = threadIdx.x + u * nt;
        x[k][u] = gload_or(src[k], i, i < pbs);
      }
    }
  }
  __device__ __forceinline__ void total(double (&out)[K]) {
    const int nt = blockDim.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) s += (int)threadIdx.x + u * nt < n[k] ? x[k][u] : 0.0;  // a select, not a branch
      for (int i = threadIdx.x + U * nt; i < n[k]; i += nt) s += gload(src[k] + i);
      out[k] = s;
    }
    block_allreduce<K>(out);
  }
};

template <int K>
__device__ __forceinline__ void slot_totals(const double* pb, const int* pbn, int pbs, const int (&slot)[K],
                                            double (&out)[K]) {
  SlotSums<K> ss;
  ss.load(pb, pbn, pbs, slot);
  ss.total(out);
}

// RRCG:5 from the partials of ||l_i||^2: L_i and beta (joint when coupled; 0 at a restart).
__device__ __forceinline__ void beta_load(SlotSums<2>& ss, const double* pb, const int* pbn, int pbs) {
  const int sl[2] = {PB_L0, PB_L1};
  ss.load(pb, pbn, pbs, sl);
}
__device__ __forceinline__ void beta_finish(const double* sc, SlotSums<2>& ss, int restart, int coupled,
                                            double (&beta)[2], double (&L)[2]) {
  ss.total(L);
  const double P0 = gload(sc + S_LPREV), P1 = gload(sc + S_LPREV + 1);
  if (coupled) {
    const double Lp = P0 + P1;
    beta[0] = beta[1] = (restart || Lp == 0.0) ? 0.0 : (L[0] + L[1]) / Lp;
  } else {
    beta[0] = (restart || P0 == 0.0) ? 0.0 : L[0] / P0;
    beta[1] = (restart || P1 == 0.0) ? 0.0 : L[1] / P1;
  }
}
__device__ __forceinline__ void beta_from(const double* sc, const double* pb, const int* pbn, int pbs,
                                          int restart, int coupled, double (&beta)[2], double (&L)[2]) {
  SlotSums<2> ss;
  beta_load(ss, pb, pbn, pbs);
  beta_finish(sc, ss, restart, coupled, beta, L);
}

__device__ __forceinline__ void record_beta(double* sc, const double (&beta)[2], const double (&L)[2]) {
  gstore(sc + S_L, L[0]);
  gstore(sc + S_L + 1, L[1]);
  gstore(sc + S_BETA, beta[0]);
  gstore(sc + S_BETA + 1, beta[1]);
  if (!isfinite(L[0]) || !isfinite(L[1])) gstore(sc + S_NONFIN, 1.0);
}

// RRCG:6: s = sum (p,l) / sum (||A~ p||^2 + (alpha + lambda) ||p||^2), joint when coupled.
// The block-0 thread 0 of the consumer records it (and L_prev <- L for the next beta) when
// `record` is set.
__device__ __forceinline__ void step_load(SlotSums<6>& ss, const double* pb, const int* pbn, int pbs) {
  const int sl[6] = {PB_PL0, PB_PL1, PB_PP0, PB_PP1, PB_Q0, PB_Q1};
  ss.load(pb, pbn, pbs, sl);
}
__device__ __forceinline__ void step_finish(double* sc, SlotSums<6>& ss, double lam0, double lam1, int coupled,
                                            bool record, double (&s)[2]) {
  double t[6];
  ss.total(t);
  const double den0 = t[4] + (gload(sc + S_ALPHA) + lam0) * t[2];
  const double den1 = t[5] + (gload(sc + S_ALPHA + 1) + lam1) * t[3];
  // a zero denominator means p = 0, where (p, l) = 0 too: the quadratic of this reweighting
  // step is at its minimum and the step is 0 (no update), as a CG iteration ends
  if (coupled) {
    const double D = den0 + den1;
    s[0] = s[1] = D == 0.0 ? 0.0 : (t[0] + t[1]) / D;
  } else {
    s[0] = den0 == 0.0 ? 0.0 : t[0] / den0;
    s[1] = den1 == 0.0 ? 0.0 : t[1] / den1;
  }
  if (record && threadIdx.x == 0) {
    gstore(sc + S_STEP, s[0]);
    gstore(sc + S_STEP + 1, s[1]);
    gstore(sc + S_PL, t[0]);
    gstore(sc + S_PL + 1, t[1]);
    gstore(sc + S_PP, t[2]);
    gstore(sc + S_PP + 1, t[3]);
    gstore(sc + S_QQ, t[4]);
    gstore(sc + S_QQ + 1, t[5]);
    gstore(sc + S_LPREV, gload(sc + S_L));
    gstore(sc + S_LPREV + 1, gload(sc + S_L + 1));
    if (!isfinite(s[0]) || !isfinite(s[1])) gstore(sc + S_NONFIN, 1.0);
  }
}
__device__ __forceinline__ void step_from(double* sc, const double* pb, const int* pbn, int pbs, double lam0,
                                          double lam1, int coupled, bool record, double (&s)[2]) {
  SlotSums<6> ss;
  step_load(ss, pb, pbn, pbs);
  step_finish(sc, ss, lam0, lam1, coupled, record, s);
}

// RRCG:2-3 scalars (m1,m1), (m2,m2), (m1,m2) from their partials.
__device__ __forceinline__ void gram_load(SlotSums<3>& ss, const double* pb, const int* pbn, int pbs) {
  const int sl[3] = {PB_G11, PB_G22, PB_G12};
  ss.load(pb, pbn, pbs, sl);
}
__device__ __forceinline__ void gram_finish(double* sc, SlotSums<3>& ss, bool record, double (&g)[3]) {
  ss.total(g);
  if (record && threadIdx.x == 0) {
    gstore(sc + S_G11, g[0]);
    gstore(sc + S_G22, g[1]);
    gstore(sc + S_G12, g[2]);
    if (!isfinite(g[0]) || !isfinite(g[1]) || !isfinite(g[2])) gstore(sc + S_NONFIN, 1.0);
  }
}
__device__ __forceinline__ void gram_from(double* sc, const double* pb, const int* pbn, int pbs, bool record,
                                          double (&g)[3]) {
  SlotSums<3> ss;
  gram_load(ss, pb, pbn, pbs);
  gram_finish(sc, ss, record, g);
}

// RRCG:4 for one element of data set `self`, given z = (A^T W_d r~)_j, the models a = m1_j,
// b = m2_j, the weights ws (this data set) and wo (the other; read only when gram_w) and
// ma = m_apr of this data set (0 when there is none):
//   l = z / w + alpha (w m - w m_apr) + lambda l_G,
//   l_G = (m2,m2) m1 - (m1,m2) m2 for data set 0, (m1,m1) m2 - (m1,m2) m1 for data set 1
// (on w m instead of m when gram_w).
template <typename T>
__device__ __forceinline__ T grad_value(bool s0, int gram_w, T z, double a, double b, double Ws, double Wo,
                                        double ma, double al, double lam, double g11, double g22, double g12) {
  double u0 = a, u1 = b;
  if (gram_w) {
    u0 = s0 ? Ws * a : Wo * a;
    u1 = s0 ? Wo * b : Ws * b;
  }
  const double lg = s0 ? g22 * u0 - g12 * u1 : g11 * u1 - g12 * u0;
  const double ms = s0 ? a : b;
  const double mt = Ws * ms, mta = Ws * ma;
  // z / w: in FP32 a product with the hardware reciprocal (within 1 ulp), as the other
  // multiplies of the FP32 form; in FP64 the division
  double zw;
  if constexpr (sizeof(T) == 4) zw = (double)(z * __builtin_amdgcn_rcpf((float)Ws));
  else zw = (double)z / Ws;
  return (T)(zw + al * (mt - mta) + lam * lg);
}

// The same in the common form (no m_apr, Gramian on m), with the data set's choices made once
// per block: ms = this data set's model, mo = the other's, gs = (m2,m2) for data set 0 and
// (m1,m1) for data set 1, so that l_G = gs ms - (m1,m2) mo.  Same operations in the same
// order as above (w m_apr is zero), hence the same result.
template <typename T>
__device__ __forceinline__ T grad_value_plain(T z, double ms, double mo, double Ws, double al, double lam, double gs,
                                              double g12) {
  const double lg = gs * ms - g12 * mo;
  const double mt = Ws * ms;
  double zw;
  if constexpr (sizeof(T) == 4) zw = (double)(z * __builtin_amdgcn_rcpf((float)Ws));
  else zw = (double)z / Ws;
  return (T)(zw + al * mt + lam * lg);
}

}  // namespace bttb
