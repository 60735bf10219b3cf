// Elementwise pieces of the joint RRCG step (Sec. 2.4 eqs. RRCG:1-8, Sec. 2.5 bounds,
// Sec. 2.6 chi^2 test, Sec. 2.8 alpha schedule) as device functions over blocks
// bid = 0 .. nb-1 of blockDim.x threads, shared by the one-inversion solver (one launch of
// RGRID blocks of RB threads) and the group solver (one launch over the blocks of many
// inversions, eb_threads per block).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "rrcg_fuse.h"

namespace bttb {

constexpr int RB = 256;       // threads per elementwise block of the one-inversion solver
// threads per elementwise block of the group solver: the loads of a whole block are in
// flight together, and an inversion's blocks (hence its partials) stay at most RGRID
#ifndef RRCG_EB32
#define RRCG_EB32 512
#endif
#ifndef RRCG_EB64
#define RRCG_EB64 512
#endif
constexpr int eb_threads(int esz) { return esz == 4 ? RRCG_EB32 : RRCG_EB64; }
#ifndef RRCG_RGRID
#define RRCG_RGRID 512
#endif
constexpr int RGRID = RRCG_RGRID;  // most elementwise blocks per inversion
#ifndef RRCG_EW_UNROLL
#define RRCG_EW_UNROLL 4
#endif
constexpr int EW_UNROLL = RRCG_EW_UNROLL;  // elements per thread whose loads are issued together

struct Red {  // where a reducing kernel puts its partials
  double* pb;
  int* pbn;
  int pbs;
};

template <typename T>
__device__ __forceinline__ void weights_body(long long n, const T* m0, const T* m1, const T* ma0, const T* ma1,
                                             const T* wz0, const T* wz1, const T* wh0, const T* wh1, double eps2,
                                             int p_norm, int gram_w, T* w0, T* w1, T* wi0, T* wi1, double* sc,
                                             Red rd, int bid, int nb) {
  const int nt = blockDim.x;
  double v[3] = {0.0, 0.0, 0.0};
  for (long long j0 = bid * (long long)nt * EW_UNROLL + threadIdx.x; j0 < n; j0 += (long long)nb * nt * EW_UNROLL) {
    T a_[EW_UNROLL], b_[EW_UNROLL], z0[EW_UNROLL], z1[EW_UNROLL], h0[EW_UNROLL], h1[EW_UNROLL], c0[EW_UNROLL],
        c1[EW_UNROLL];
#pragma unroll
    for (int u = 0; u < EW_UNROLL; ++u) {  // every load before the first store
      const long long j = j0 + (long long)u * nt;
      const bool ok = j < n;
      a_[u] = gload_or(m0, j, ok);
      b_[u] = gload_or(m1, j, ok);
      z0[u] = gload_or(wz0, j, ok);
      z1[u] = gload_or(wz1, j, ok);
      h0[u] = wh0 ? gload_or(wh0, j, ok, T(1)) : T(1);
      h1[u] = wh1 ? gload_or(wh1, j, ok, T(1)) : T(1);
      c0[u] = ma0 ? gload_or(ma0, j, ok) : T(0);
      c1[u] = ma1 ? gload_or(ma1, j, ok) : T(0);
    }
#pragma unroll
    for (int u = 0; u < EW_UNROLL; ++u) {
      const long long j = j0 + (long long)u * nt;
      if (j >= n) continue;
      const double a = a_[u], b = b_[u];
      double W0 = z0[u], W1 = z1[u];
      if (wh0) W0 *= (double)h0[u];
      if (wh1) W1 *= (double)h1[u];
      if (p_norm == 1) {  // (d^2 + eps^2)^(-1/4)
        const double d0 = a - (double)c0[u], d1 = b - (double)c1[u];
        W0 *= 1.0 / sqrt(sqrt(d0 * d0 + eps2));
        W1 *= 1.0 / sqrt(sqrt(d1 * d1 + eps2));
      }
      const T W0t = (T)W0, W1t = (T)W1;
      gstore(w0 + j, W0t);
      gstore(w1 + j, W1t);
      gstore(wi0 + j, (T)(1.0 / (double)W0t));
      gstore(wi1 + j, (T)(1.0 / (double)W1t));
      const double u0 = gram_w ? (double)W0t * a : a, u1 = gram_w ? (double)W1t * b : b;
      v[0] += u0 * u0;
      v[1] += u1 * u1;
      v[2] += u0 * u1;
    }
  }
  block_partials<3>(v, rd.pb, rd.pbn, rd.pbs, PB_G11, bid, nb);
}

// l = A~^T r~ (already in l) + alpha (w m - w ma) + lambda l_G, ma the anchor in the original
// space (m_apr or m_prev; NULL: zero);  partials of ||l_i||^2.
template <typename T>
__device__ __forceinline__ void grad_body(long long n, T* l0, T* l1, const T* m0, const T* m1, const T* w0,
                                          const T* w1, const T* ma0, const T* ma1, double* sc, double lam0,
                                          double lam1, int gram_w, Red rd, int bid, int nb) {
  double gg[3];
  gram_from(sc, rd.pb, rd.pbn, rd.pbs, bid == 0, gg);
  const double g11 = gg[0], g22 = gg[1], g12 = gg[2];
  const double al0 = gload(sc + S_ALPHA), al1 = gload(sc + S_ALPHA + 1);
  double v[2] = {0.0, 0.0};
  for (long long j = bid * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)nb * blockDim.x) {
    const double a = gload(m0 + j), b = gload(m1 + j), W0 = gload(w0 + j), W1 = gload(w1 + j);
    const double u0 = gram_w ? W0 * a : a, u1 = gram_w ? W1 * b : b;
    const double lg0 = g22 * u0 - g12 * u1, lg1 = g11 * u1 - g12 * u0;
    const double mt0 = W0 * a, mt1 = W1 * b;
    const double mta0 = ma0 ? W0 * (double)gload(ma0 + j) : 0.0, mta1 = ma1 ? W1 * (double)gload(ma1 + j) : 0.0;
    const T r0 = (T)((double)gload(l0 + j) + al0 * (mt0 - mta0) + lam0 * lg0);
    const T r1 = (T)((double)gload(l1 + j) + al1 * (mt1 - mta1) + lam1 * lg1);
    gstore(l0 + j, r0);
    gstore(l1 + j, r1);
    v[0] += (double)r0 * (double)r0;
    v[1] += (double)r1 * (double)r1;
  }
  block_partials<2>(v, rd.pb, rd.pbn, rd.pbs, PB_L0, bid, nb);
}

// beta from ||l||^2; p = l + beta p; partials (p, l)_i and ||p_i||^2.
template <typename T>
__device__ __forceinline__ void dir_body(long long n, const T* l0, const T* l1, T* p0, T* p1, double* sc,
                                         int restart_now, int coupled, Red rd, int bid, int nb) {
  double bt[2], L[2];
  beta_from(sc, rd.pb, rd.pbn, rd.pbs, restart_now, coupled, bt, L);
  if (bid == 0 && threadIdx.x == 0) record_beta(sc, bt, L);
  const double b0 = bt[0], b1 = bt[1];
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // (p0,l0), ||p0||^2, (p1,l1), ||p1||^2
  for (long long j = bid * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)nb * blockDim.x) {
    const double la = gload(l0 + j), lb = gload(l1 + j);
    const T pa = (T)(la + b0 * (double)gload(p0 + j));
    const T pbv = (T)(lb + b1 * (double)gload(p1 + j));
    gstore(p0 + j, pa);
    gstore(p1 + j, pbv);
    v[0] += (double)pa * la;
    v[1] += (double)pa * (double)pa;
    v[2] += (double)pbv * lb;
    v[3] += (double)pbv * (double)pbv;
  }
  block_partials<4>(v, rd.pb, rd.pbn, rd.pbs, PB_PL0, bid, nb);
}

// partials of ||q_i||^2.
template <typename T>
__device__ __forceinline__ void sumsq2_body(long long n, const T* a0, const T* a1, Red rd, int bid, int nb) {
  double v[2] = {0.0, 0.0};
  for (long long j = bid * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)nb * blockDim.x) {
    const double x = gload(a0 + j), y = gload(a1 + j);
    v[0] += x * x;
    v[1] += y * y;
  }
  block_partials<2>(v, rd.pb, rd.pbn, rd.pbs, PB_Q0, bid, nb);
}

// s from the partials (RRCG:6); m <- m - s p / w (i.e. m~ <- m~ - s p, then m = m~ / w);
// r~ <- r~ - s q (for nd > 0); Gramian partials of the new m (on m or on w m); with the
// previous-iterate anchor (mp0 non-NULL) the model before the update into mp.  Block 0
// records the step length unless `record` is off (another part of the launch records it).
// Every load of an iteration goes out before its first store: vector memory operations
// complete in issue order, so a load issued after a store could only be waited for together
// with it.
template <typename T>
__device__ __forceinline__ void update_body(long long n, long long nd, T* m0, T* m1, const T* p0, const T* p1,
                                            const T* w0, const T* w1, T* r0, T* r1, const T* q0, const T* q1,
                                            double* sc, double lam0, double lam1, int coupled, int gram_w,
                                            T* mp0, T* mp1, Red rd, int bid, int nb, bool record = true) {
  constexpr int U = EW_UNROLL;
  const int nt = blockDim.x;
  double st[2];
  step_from(sc, rd.pb, rd.pbn, rd.pbs, lam0, lam1, coupled, record && bid == 0, st);
  const double s0 = uniform(st[0]), s1 = uniform(st[1]);
  double v[3] = {0.0, 0.0, 0.0};
  const long long top = n > nd ? n : nd;
  const long long step = (long long)nb * nt * U;
  for (long long j0 = bid * (long long)nt * U + threadIdx.x; j0 < top; j0 += step) {
    const bool data = j0 - threadIdx.x < nd;  // this block's iteration reaches the data vectors
    T M0[U], M1[U], P0[U], P1[U], V0[U], V1[U], R0[U], R1[U], Q0[U], Q1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * nt;
      const bool ok = j < n;
      M0[u] = gload_or(m0, j, ok);
      M1[u] = gload_or(m1, j, ok);
      P0[u] = gload_or(p0, j, ok);
      P1[u] = gload_or(p1, j, ok);
      V0[u] = gload_or(w0, j, ok, T(1));
      V1[u] = gload_or(w1, j, ok, T(1));
    }
    if (data) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long j = j0 + (long long)u * nt;
        const bool okd = j < nd;
        R0[u] = gload_or(r0, j, okd);
        R1[u] = gload_or(r1, j, okd);
        Q0[u] = gload_or(q0, j, okd);
        Q1[u] = gload_or(q1, j, okd);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * nt;
      if (j < n) {
        const double W0 = V0[u], W1 = V1[u];
        const T a = (T)((W0 * (double)M0[u] - s0 * (double)P0[u]) / W0);
        const T b = (T)((W1 * (double)M1[u] - s1 * (double)P1[u]) / W1);
        if (mp0) {
          gstore(mp0 + j, M0[u]);
          gstore(mp1 + j, M1[u]);
        }
        gstore(m0 + j, a);
        gstore(m1 + j, b);
        const double u0 = gram_w ? W0 * (double)a : (double)a, u1 = gram_w ? W1 * (double)b : (double)b;
        v[0] += u0 * u0;
        v[1] += u1 * u1;
        v[2] += u0 * u1;
      }
    }
    if (data) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long j = j0 + (long long)u * nt;
        if (j < nd) {
          gstore(r0 + j, (T)((double)R0[u] - s0 * (double)Q0[u]));
          gstore(r1 + j, (T)((double)R1[u] - s1 * (double)Q1[u]));
        }
      }
    }
  }
  block_partials<3>(v, rd.pb, rd.pbn, rd.pbs, PB_G11, bid, nb);
}

// m <- clip(m, lo, hi); Gramian partials of the projected m (original space).
template <typename T>
__device__ __forceinline__ void clip_body(long long n, T* m0, T* m1, double lo0, double hi0, double lo1,
                                          double hi1, Red rd, int bid, int nb) {
  constexpr int U = EW_UNROLL;
  const int nt = blockDim.x;
  double v[3] = {0.0, 0.0, 0.0};
  for (long long j0 = bid * (long long)nt * U + threadIdx.x; j0 < n; j0 += (long long)nb * nt * U) {
    T A[U], B[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * nt;
      A[u] = gload_or(m0, j, j < n);
      B[u] = gload_or(m1, j, j < n);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * nt;
      if (j >= n) continue;
      const T at = (T)fmin(fmax((double)A[u], lo0), hi0), bt = (T)fmin(fmax((double)B[u], lo1), hi1);
      gstore(m0 + j, at);
      gstore(m1 + j, bt);
      v[0] += (double)at * (double)at;
      v[1] += (double)bt * (double)bt;
      v[2] += (double)at * (double)bt;
    }
  }
  block_partials<3>(v, rd.pb, rd.pbn, rd.pbs, PB_G11, bid, nb);
}

// r~ = W_d (A m - d) (A m already in r); partials of ||r~_i||^2.
template <typename T>
__device__ __forceinline__ void resid_body(long long nd, T* r0, T* r1, const T* d0, const T* d1, const T* wd0,
                                           const T* wd1, Red rd, int bid, int nb) {
  double v[2] = {0.0, 0.0};
  for (long long j = bid * (long long)blockDim.x + threadIdx.x; j < nd; j += (long long)nb * blockDim.x) {
    const T a = (T)((double)gload(wd0 + j) * ((double)gload(r0 + j) - (double)gload(d0 + j)));
    const T b = (T)((double)gload(wd1 + j) * ((double)gload(r1 + j) - (double)gload(d1 + j)));
    gstore(r0 + j, a);
    gstore(r1 + j, b);
    v[0] += (double)a * (double)a;
    v[1] += (double)b * (double)b;
  }
  block_partials<2>(v, rd.pb, rd.pbn, rd.pbs, PB_F0, bid, nb);
}

// Phi, S_G, and (advance = 1) the chi^2 test, freeze flags and alpha schedule (Sec. 2.6, 2.8);
// one block.
__device__ __forceinline__ void fin_outer_body(double* sc, Red rd, double q0, double q1, double amin0,
                                               double amin1, int advance, int bid, int nb) {
  const int sl[5] = {PB_G11, PB_G22, PB_G12, PB_F0, PB_F1};
  double t[5];
  slot_totals<5>(rd.pb, rd.pbn, rd.pbs, sl, t);
  const double g11 = t[0], g22 = t[1], g12 = t[2], f0 = t[3], f1 = t[4];
  if (threadIdx.x == 0) {
    gstore(sc + S_PHI, f0);
    gstore(sc + S_PHI + 1, f1);
    gstore(sc + S_GRAM, g11 * g22 - g12 * g12);
    // the cosine of the two models, |(m1, m2)| / (||m1|| ||m2||), 0 when a model is zero
    gstore(sc + S_SIM, (g11 > 0.0 && g22 > 0.0) ? fabs(g12) / sqrt(g11 * g22) : 0.0);
    if (!isfinite(f0) || !isfinite(f1) || !isfinite(g11) || !isfinite(g22)) gstore(sc + S_NONFIN, 1.0);
    if (advance) {
      const double thr = gload(sc + S_THR);
      const bool p0 = f0 <= thr, p1 = f1 <= thr;
      const bool fr0 = gload(sc + S_FROZEN) != 0.0 || p0, fr1 = gload(sc + S_FROZEN + 1) != 0.0 || p1;
      gstore(sc + S_FROZEN, fr0 ? 1.0 : 0.0);
      gstore(sc + S_FROZEN + 1, fr1 ? 1.0 : 0.0);
      gstore(sc + S_CONV, (p0 && p1) ? 1.0 : 0.0);
      if (!fr0) gstore(sc + S_ALPHA, fmax(q0 * gload(sc + S_ALPHA), amin0));
      if (!fr1) gstore(sc + S_ALPHA + 1, fmax(q1 * gload(sc + S_ALPHA + 1), amin1));
      gstore(sc + S_K, gload(sc + S_K) + 1.0);
    }
  }
}

}  // namespace bttb
