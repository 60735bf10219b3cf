// Kernel bodies of the power-of-two path (register-resident FFT, fft_reg.h), written as
// device functions of explicit block coordinates so that the one-plan kernels and the
// group kernels (one launch over many plans) share them.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "fft_reg.h"
#include "rrcg_fuse.h"

namespace bttb {

// Orders the LDS accesses of one wave: LDS requests of a wave complete in issue order,
// so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LANES>
struct GroupSync {  // a group of LANES (a power of two) lanes: inside one wave up to 64
  __device__ __forceinline__ void operator()() const {
    if constexpr (LANES <= 64) wave_sync();
    else __syncthreads();
  }
};

template <int N>
constexpr int row_buf() {  // per-group LDS elements of the row kernels (exchange and [2][K2] staging)
  return Len<N>::BUF > N + 2 ? Len<N>::BUF : N + 2;
}

#ifndef BTTB_ROW_WAVES32
#define BTTB_ROW_WAVES32 8
#endif
#ifndef BTTB_GRAD_WAVES32
#define BTTB_GRAD_WAVES32 6
#endif
// Waves per SIMD the row kernels are compiled for: in FP32 up to 512 points, eight, so that the
// registers (at most 64) let four blocks of 512 threads share a CU and a whole product's row
// blocks are resident at once, except the direction form in the full form, whose loads in
// flight need more than 64 registers (six waves).  Longer transforms hold more twiddles and
// keep the default.
template <typename T, int N, int MODE, bool HALF>
constexpr int row_waves() {
  // (a 5-smooth size's direction form holds a composite radix's values as well: six waves)
  return sizeof(T) != 4 || N > 512                                         ? 2
         : MODE == FUSE_DIR && (!HALF || (N & (N - 1)) != 0) ? BTTB_GRAD_WAVES32
                                                             : BTTB_ROW_WAVES32;
}
// The inverse row transforms: the model-row ones as above, except the gradient form in the
// full form, which needs more than 64 registers (six waves, three blocks per CU); the data-row
// ones launch few blocks and keep their registers.
template <typename T, int N, bool ROWIN, int MODE, bool HALF>
constexpr int c2r_waves() {
  return sizeof(T) != 4 || N > 512 || ROWIN ? 2 : MODE == FUSE_GRAD && !HALF ? BTTB_GRAD_WAVES32 : BTTB_ROW_WAVES32;
}

// ------------------------------------------------------------------------------------
// Row transforms
// ------------------------------------------------------------------------------------
template <typename T>
struct FRowArgs {
  const T* in;
  long long in_bs;
  const T* scale;
  cx<T>* out;
  long long out_bs;
  long long in_cs;  // c2r: stride between summed partials
  int nsum;
  int L, nrows, ncols, ld, K2, fpb, tiles;
  const cx<T>* tw;
};

// ROWOUT = false: half spectra stored column-major out[l][k2][row] (ld = padded rows) through an
// LDS transpose; ROWOUT = true: row-major out[l][row][k2] (ld = padded K2) straight from registers.
// MODE = FUSE_DIR (ROWOUT = false, the forward product inside the CG step): beta is summed from
// the partials of ||l||^2 at the start, the input is the new direction p = l + beta p (RRCG:5),
// written back, and the block partials of (p, l) and ||p||^2 are stored for the step length.
// Block (bx, by) of the launch: bx = layer * tiles + tile, by = batch entry; pid and pcount
// are this block's index and the block count for the partial sums of the fused form.
// HALF (a.ncols <= N/2): a lane's upper four inputs (index >= N/2) are zero padding, known
// at compile time, so the first radix-8 pass folds them away.
template <typename T, int N, bool ROWOUT, int MODE, bool HALF>
__device__ __forceinline__ void frow_r2c_body(const FRowArgs<T>& a, const Fuse<T>& fz, int bx, int by, int pid,
                                              int pcount, unsigned char* smem_raw) {
  static_assert(MODE == FUSE_NONE || (MODE == FUSE_DIR && !ROWOUT) || (MODE == FUSE_RUPD && ROWOUT), "fused form");
  using P = Len<N>;
  constexpr int TPF = P::TPF, LANES = P::LANES, BS = row_buf<N>(), K2 = N / 2 + 1;
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / LANES, tl = threadIdx.x - f * LANES;
  // a 5-smooth size's lanes past TPF hold no values: they index as lane 0 and store nothing
  const bool live = P::POW2 || tl < TPF;
  const int t = P::POW2 ? tl : (live ? tl : 0);
  const int l = bx / a.tiles, tile = bx - l * a.tiles;
  const int b = by;
  const int RT = 2 * a.fpb;
  const int r0 = tile * RT + 2 * f;
  cx<T>* buf = smem + f * BS;
  GroupSync<LANES> gsync;
  FFTOf<T, N> F;
  const long long lofs = (long long)l * a.nrows * a.ncols;
  const T* src = a.in + b * a.in_bs + lofs;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  const bool ra = live && r0 < a.nrows, rb = live && r0 + 1 < a.nrows;
  cx<T> v[8];
  double acc[2] = {0.0, 0.0};
  if constexpr (MODE == FUSE_DIR) {
    // The loads of the prologue go out before any store of the new direction (vector memory
    // operations complete in issue order, so a load issued after a store could only be
    // waited for together with it), half of a thread's entries (4 h .. 4 h + 3, both rows)
    // at a time; the first half before the partial sums of beta, whose loads then overlap
    // them.  The half form has no upper half: a row fills at most half the transform.
    const T* lv = fz.l + lofs;
    const T* pv = fz.p + lofs;
    T* po = fz.pout + lofs;
    T LA[4], LB[4], PA[4], PB[4], SA[4], SB[4];
    auto dir_load = [&](int h) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = t + (4 * h + i) * TPF;
        const bool ok = n < a.ncols;
        const long long oa = (long long)r0 * a.ncols + n;
        LA[i] = gload_or(lv, oa, ok & ra);
        PA[i] = gload_or(pv, oa, ok & ra);
        SA[i] = gload_or(sc, oa, ok & ra);
        LB[i] = gload_or(lv, oa + a.ncols, ok & rb);
        PB[i] = gload_or(pv, oa + a.ncols, ok & rb);
        SB[i] = gload_or(sc, oa + a.ncols, ok & rb);
      }
    };
    dir_load(0);
    double bt[2], L[2];
    beta_from(fz.sc, fz.pb, fz.pbn, fz.pbs, fz.restart, fz.coupled, bt, L);
    if (fz.lead && pid == 0 && threadIdx.x == 0) record_beta(fz.sc, bt, L);
    const double beta = fz.self == 0 ? bt[0] : bt[1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1) {
        if constexpr (HALF) {  // the upper half of the transform input is zero padding
#pragma unroll
          for (int i = 4; i < 8; ++i) v[i] = cx<T>{T(0), T(0)};
          break;
        }
        if (t + 4 * TPF < a.ncols) dir_load(1);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = t + (4 * h + i) * TPF;
        T xa = T(0), xb = T(0);
        if (n < a.ncols) {
          const long long oa = (long long)r0 * a.ncols + n;
          if (ra) {
            const double lo = LA[i];
            const T pn = (T)(lo + beta * (double)PA[i]);
            gstore(po + oa, pn);
            acc[0] += (double)pn * lo;
            acc[1] += (double)pn * (double)pn;
            xa = pn * SA[i];
          }
          if (rb) {
            const double lo = LB[i];
            const T pn = (T)(lo + beta * (double)PB[i]);
            gstore(po + oa + a.ncols, pn);
            acc[0] += (double)pn * lo;
            acc[1] += (double)pn * (double)pn;
            xb = pn * SB[i];
          }
        }
        v[4 * h + i] = cx<T>{xa, xb};
      }
    }
  } else if constexpr (MODE == FUSE_RUPD) {
    // The residual update of the previous CG step, r~ <- r~ - s q (RRCG:7, data space), carried
    // by the transform of W_d r~ that starts the next step: the loads of four entries per row
    // first, then (once) the step length s from its partials (RRCG:6), the stores of r~ and
    // the transform input; the full form takes its upper four entries the same way after.
    // (without a scale the factors are ones, read from r~'s first entry and discarded)
    const T* zbase = sc ? sc : fz.r;
    const bool scaled = sc != nullptr;
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < (HALF ? 1 : 2); ++h) {
      T RA[4], RB[4], QA[4], QB[4], ZA[4], ZB[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = t + (4 * h + i) * TPF;
        const bool ok = n < a.ncols;
        const long long oa = (long long)r0 * a.ncols + n;
        RA[i] = gload_or<T>(fz.r, oa, ok & ra);
        QA[i] = gload_or(fz.q, oa, ok & ra);
        ZA[i] = gload_or(zbase, oa, ok & ra & scaled, T(1));
        RB[i] = gload_or<T>(fz.r, oa + a.ncols, ok & rb);
        QB[i] = gload_or(fz.q, oa + a.ncols, ok & rb);
        ZB[i] = gload_or(zbase, oa + a.ncols, ok & rb & scaled, T(1));
      }
      if (h == 0) {
        double st[2];
        step_from(fz.sc, fz.pb, fz.pbn, fz.pbs, fz.lam[0], fz.lam[1], fz.coupled, fz.lead && pid == 0, st);
        s = uniform(fz.self == 0 ? st[0] : st[1]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = t + (4 * h + i) * TPF;
        T xa = T(0), xb = T(0);
        if (n < a.ncols) {
          const long long oa = (long long)r0 * a.ncols + n;
          if (ra) {
            const T rn = (T)((double)RA[i] - s * (double)QA[i]);
            gstore(fz.r + oa, rn);
            xa = rn * ZA[i];
          }
          if (rb) {
            const T rn = (T)((double)RB[i] - s * (double)QB[i]);
            gstore(fz.r + oa + a.ncols, rn);
            xb = rn * ZB[i];
          }
        }
        v[4 * h + i] = cx<T>{xa, xb};
      }
    }
    if constexpr (HALF) {
#pragma unroll
      for (int i = 4; i < 8; ++i) v[i] = cx<T>{T(0), T(0)};
    }
  } else {
    // every load first, branch-free: entries out of range read the layer's first entry and
    // give zero; without a scale the factors are ones
    const T* sbase = sc ? sc : src;
    const bool scaled = sc != nullptr;
    T XA[8], XB[8], SA[8], SB[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int n = t + i * TPF;
      const bool ok = (!HALF || i < 4) & (n < a.ncols);
      const long long oa = (long long)r0 * a.ncols + n;
      XA[i] = gload_or(src, oa, ok & ra);
      SA[i] = gload_or(sbase, oa, ok & ra & scaled, T(1));
      XB[i] = gload_or(src, oa + a.ncols, ok & rb);
      SB[i] = gload_or(sbase, oa + a.ncols, ok & rb & scaled, T(1));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = cx<T>{XA[i] * SA[i], XB[i] * SB[i]};
  }
  F.init(a.tw, t);  // twiddles loaded here: not live during the prologue
  if constexpr (!P::POW2) F.live = live;
  F.template run<false>(v, buf, t, gsync);
  // X_a[k] = (Z[k] + conj Z[N-k]) / 2,  X_b[k] = (Z[k] - conj Z[N-k]) / (2i),  k <= N/2
  if (live) {
#pragma unroll
    for (int i = 0; i < 8; ++i) buf[lds_pad(t + i * TPF)] = v[i];
  }
  gsync();
  const T h = T(0.5);
  cx<T> xa[5], xb[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int k = t + i * TPF;
    if (k <= N / 2) {
      const cx<T> A = v[i];
      const cx<T> C = buf[lds_pad(P::POW2 ? ((N - k) & (N - 1)) : (k == 0 ? 0 : N - k))];
      xa[i] = cx<T>{h * (A.re + C.re), h * (A.im - C.im)};
      xb[i] = cx<T>{h * (A.im + C.im), h * (C.re - A.re)};
    }
  }
  if constexpr (ROWOUT) {
    cx<T>* dst = a.out + b * a.out_bs + ((long long)l * a.nrows + r0) * a.ld;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int k = t + i * TPF;
      if (k <= N / 2) {
        if (ra) gstore(dst + k, xa[i]);
        if (rb) gstore(dst + a.ld + k, xb[i]);
      }
    }
    return;
  }
  gsync();
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int k = t + i * TPF;
    if (live && k <= N / 2) {
      buf[k] = xa[i];
      buf[K2 + k] = xb[i];
    }
  }
  __syncthreads();
  // (the direction's partial sums first: their registers are then free for the stores; the
  // butterfly form, with which the kernel's prologue stays within its registers)
  if constexpr (MODE == FUSE_DIR) block_partials<2, false>(acc, fz.pb, fz.pbn, fz.pbs, fz.self ? PB_PL1 : PB_PL0, pid, pcount);
  // rows beyond nrows are not stored: a tile may be taller than the padded row count ld
  cx<T>* dst = a.out + b * a.out_bs + (long long)l * K2 * a.ld + tile * RT;
  const int rows = min(RT, a.nrows - tile * RT);
  if (TPF >= 2 && 2 * (int)blockDim.x == RT * TPF) {
    // every LDS read first, then the stores.  With blockDim = RT TPF / 2 (one transform of two
    // rows per TPF threads, TPF >= 2) a thread keeps its row rr and steps TPF / 2 columns per
    // pass, and ITER passes cover the K2 RT entries.
    constexpr int ITER = (2 * K2 + TPF - 1) / TPF;
    const int rr = threadIdx.x % RT, k0 = threadIdx.x / RT;
    const cx<T>* srow = smem + (rr >> 1) * BS + (rr & 1) * K2;
    // k0 < TPF / 2: only the last pass reaches past K2, where the k0 = 0 lane holds the
    // Nyquist column; the others store from one per-thread base with a uniform stride.
    cx<T> ov[ITER];
#pragma unroll
    for (int it = 0; it < ITER - 1; ++it) ov[it] = srow[k0 + it * (TPF / 2)];
    if (k0 == 0) ov[ITER - 1] = srow[K2 - 1];
    if (rr < rows) {
      cx<T>* dp = dst + rr + (long long)k0 * a.ld;
      const long long st = (long long)(TPF / 2) * a.ld;
#pragma unroll
      for (int it = 0; it < ITER - 1; ++it) gstore(dp + it * st, ov[it]);
      if (k0 == 0) gstore(dp + (ITER - 1) * st, ov[ITER - 1]);
    }
    return;
  }
  for (int idx = threadIdx.x; idx < K2 * RT; idx += blockDim.x) {
    const int k2 = idx / RT, rr = idx - k2 * RT;
    if (rr < rows) gstore(dst + (long long)k2 * a.ld + rr, smem[(rr >> 1) * BS + (rr & 1) * K2 + k2]);
  }
}

template <typename T, int N, bool ROWOUT, int MODE, bool HALF>
__global__ void __launch_bounds__(512, (row_waves<T, N, MODE, HALF>())) k_frow_r2c(FRowArgs<T> a, Fuse<T> fz) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  frow_r2c_body<T, N, ROWOUT, MODE, HALF>(a, fz, blockIdx.x, blockIdx.y, blockIdx.x + gridDim.x * blockIdx.y,
                                          gridDim.x * gridDim.y, smem_raw);
}

// ROWIN = false: half spectra read column-major in[l][k2][row] (ld = padded rows, nsum = 1)
// through an LDS transpose; ROWIN = true: row-major in[c][l][row][k2] (ld = padded K2) summed
// over the nsum partials, read straight into the strided layout.
// MODE = FUSE_QQ (ROWIN = true, the forward product inside the CG step): block partials of
// ||q||^2 for the output q (for the step length of RRCG:6).
// MODE = FUSE_GRAD (ROWIN = false, the transpose product inside the CG step): the output is the
// gradient l of RRCG:4, from the Gramian scalars summed at the start, with its block partials
// of ||l||^2 (for beta of RRCG:5).
// HALF (a.ncols <= N/2): a lane's upper four outputs are never stored, known at compile time,
// so the last pass does not compute them.
template <typename T, int N, bool ROWIN, int MODE, bool HALF>
__device__ __forceinline__ void frow_c2r_body(const FRowArgs<T>& a, const Fuse<T>& fz, int bx, int by, int pid,
                                              int pcount, unsigned char* smem_raw) {
  static_assert(MODE == FUSE_NONE || (MODE == FUSE_QQ && ROWIN) || (MODE == FUSE_GRAD && !ROWIN), "fused form");
  using P = Len<N>;
  constexpr int TPF = P::TPF, LANES = P::LANES, BS = row_buf<N>(), K2 = N / 2 + 1;
  // the row-split staging below needs groups of exactly TPF lanes
  constexpr bool SPLIT = TPF >= 2 && P::POW2;
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / LANES, tl = threadIdx.x - f * LANES;
  const bool live = P::POW2 || tl < TPF;  // as in the forward row transform
  const int t = P::POW2 ? tl : (live ? tl : 0);
  const int l = bx / a.tiles, tile = bx - l * a.tiles;
  const int b = by;
  const int RT = 2 * a.fpb;
  cx<T>* buf = smem + f * BS;
  GroupSync<LANES> gsync;
  FFTOf<T, N> F;
  const int r0 = tile * RT + 2 * f;
  const bool ra = live && r0 < a.nrows, rb = live && r0 + 1 < a.nrows;
  const long long lofs = (long long)l * a.nrows * a.ncols;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  cx<T> v[8];
  double gg[3] = {0.0, 0.0, 0.0};  // Gramian scalars for the gradient form
  if constexpr (ROWIN) {
    // base: the start of this batch entry (valid for every lane); rows r0, r0 + 1 may lie
    // beyond nrows, where the guarded loads read the base instead
    const cx<T>* base = reinterpret_cast<const cx<T>*>(a.in) + b * a.in_bs;
    const long long off = ((long long)l * a.nrows + r0) * a.ld;
    cx<T> ha[8], hb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = t + i * TPF;
      const int kk = k <= N / 2 ? k : N - k;
      ha[i] = gload_or(base, off + kk, ra);
      hb[i] = gload_or(base, off + a.ld + kk, rb);
    }
    for (int c = 1; c < a.nsum; ++c) {  // partials of the layer chunks, summed in order
      const cx<T>* pbase = base + c * a.in_cs;  // chunk c of this batch entry
      cx<T> pa[8], pb[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {  // every load of the chunk before the first sum
        const int k = t + i * TPF;
        const int kk = k <= N / 2 ? k : N - k;
        pa[i] = gload_or(pbase, off + kk, ra);
        pb[i] = gload_or(pbase, off + a.ld + kk, rb);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        ha[i] = cadd(ha[i], pa[i]);
        hb[i] = cadd(hb[i], pb[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = t + i * TPF;
      const int kk = k <= N / 2 ? k : N - k;
      if (kk == 0 || kk == N / 2) {  // DC and Nyquist of a real row are real
        ha[i].im = T(0);
        hb[i].im = T(0);
      }
      v[i] = k <= N / 2 ? cx<T>{ha[i].re - hb[i].im, ha[i].im + hb[i].re}
                        : cx<T>{ha[i].re + hb[i].im, hb[i].re - ha[i].im};
    }
  } else {
    // `in` is complex [L][K2][ld] (nsum = 1).  Each thread loads its ITER values first, then
    // stages them in LDS, so the loads are in flight together.
    // blockDim = RT TPF / 2, so ITER passes cover the K2 RT entries; from TPF = 2 on, a thread
    // keeps its row rr and steps TPF / 2 columns per pass.
    constexpr int ITER = (2 * K2 + TPF - 1) / TPF;
    const cx<T>* src = reinterpret_cast<const cx<T>*>(a.in) + b * a.in_bs + (long long)l * K2 * a.ld + tile * RT;
    const int rows = min(RT, a.nrows - tile * RT);
    const int rr0 = threadIdx.x % RT, k0 = threadIdx.x / RT;
    auto pos = [&](int it, int& k2, int& rr) {
      if constexpr (SPLIT) {
        k2 = k0 + it * (TPF / 2);
        rr = rr0;
      } else {
        const int idx = threadIdx.x + it * blockDim.x;
        k2 = idx / RT;
        rr = idx - k2 * RT;
      }
    };
    cx<T> hv[ITER];
    if constexpr (SPLIT) {
      // k0 < TPF / 2, so only the last pass can reach past K2 (its k0 = 0 lane holds the
      // Nyquist column); a row past `rows` reads row 0 (in range) and is zeroed when staged.
      const bool okr = rr0 < rows;
      const cx<T>* sp = src + (okr ? (long long)k0 * a.ld + rr0 : 0);
      const long long st = (long long)(TPF / 2) * a.ld;
#pragma unroll
      for (int it = 0; it < ITER - 1; ++it) hv[it] = gload(sp + it * st);
      hv[ITER - 1] = gload_or(sp, (ITER - 1) * st, k0 == 0);
    } else {
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        int k2, rr;
        pos(it, k2, rr);
        hv[it] = gload_or(src, (long long)k2 * a.ld + rr, (k2 < K2) & (rr < rows));
      }
    }
    // the Gramian scalars' partials, loaded while the spectra are in flight
    if constexpr (MODE == FUSE_GRAD) {
      gram_from(fz.sc, fz.pb, fz.pbn, fz.pbs, fz.lead && pid == 0, gg);
#pragma unroll
      for (int k = 0; k < 3; ++k) gg[k] = uniform(gg[k]);  // scalar registers across the transform
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      int k2, rr;
      pos(it, k2, rr);
      if (k2 < K2) {
        cx<T> h = hv[it];
        if constexpr (SPLIT) {
          if (rr0 >= rows) h = cx<T>{T(0), T(0)};
        }
        if (k2 == 0 || k2 == K2 - 1) h.im = T(0);  // DC and Nyquist of a real row are real
        smem[(rr >> 1) * BS + (rr & 1) * K2 + k2] = h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = t + i * TPF;
      if (k <= N / 2) {
        const cx<T> ha = buf[k], hb = buf[K2 + k];
        v[i] = cx<T>{ha.re - hb.im, ha.im + hb.re};
      } else {
        const cx<T> ha = buf[N - k], hb = buf[K2 + N - k];
        v[i] = cx<T>{ha.re + hb.im, hb.re - ha.im};
      }
    }
  }
  gsync();
  F.init(a.tw, t);  // twiddles loaded here: not live while the input is staged
  if constexpr (!P::POW2) F.live = live;
  F.template run<true>(v, buf, t, gsync);
  T* dst = reinterpret_cast<T*>(a.out) + b * a.out_bs + lofs;
  if constexpr (MODE == FUSE_GRAD) {
    const bool s0 = fz.self == 0;
    // block-wide scalars, in scalar registers
    const double al = uniform(gload(fz.sc + S_ALPHA + fz.self)), lam = uniform(s0 ? fz.lam[0] : fz.lam[1]);
    const double g11 = gg[0], g22 = gg[1], g12 = gg[2];
    const T* m0p = fz.m[0] + lofs;
    const T* m1p = fz.m[1] + lofs;
    const T* wsp = (s0 ? fz.w[0] : fz.w[1]) + lofs;
    const T* wop = (s0 ? fz.w[1] : fz.w[0]) + lofs;
    const T* map = fz.ma ? fz.ma + lofs : nullptr;
    // (the weight divides the transform here: the weights' reciprocals are not read)
    auto grad_at = [&](long long o, T z) -> T {
      return grad_value<T>(s0, fz.gram_w, z, gload(m0p + o), gload(m1p + o), gload(wsp + o),
                           fz.gram_w ? gload(wop + o) : T(0), map ? gload(map + o) : T(0), al, lam, g11, g22, g12);
    };
    double acc[1] = {0.0};
    if (!fz.gram_w && !map) {
      // The common form: the operands of CH entries per row go out together before any
      // store (a load issued after a store could only be waited for together with it); the
      // full form takes them in smaller groups, within its registers.
      constexpr int CH = HALF ? 4 : 2;
      const T* msp = s0 ? m0p : m1p;  // this data set's model and the other's
      const T* mop = s0 ? m1p : m0p;
      const double gs = s0 ? g22 : g11;
#pragma unroll
      for (int c = 0; c < (HALF ? 4 : 8); c += CH) {
        T AS[CH], AO[CH], AW[CH], BS_[CH], BO[CH], BW[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int q = t + (c + i) * TPF;
          const bool ok = q < a.ncols;
          const long long o = (long long)r0 * a.ncols + q;
          AS[i] = gload_or(msp, o, ok & ra);
          AO[i] = gload_or(mop, o, ok & ra);
          AW[i] = gload_or(wsp, o, ok & ra, T(1));
          BS_[i] = gload_or(msp, o + a.ncols, ok & rb);
          BO[i] = gload_or(mop, o + a.ncols, ok & rb);
          BW[i] = gload_or(wsp, o + a.ncols, ok & rb, T(1));
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int q = t + (c + i) * TPF;
          if (q < a.ncols) {
            const long long o = (long long)r0 * a.ncols + q;
            if (ra) {
              const T g = grad_value_plain<T>(v[c + i].re, AS[i], AO[i], AW[i], al, lam, gs, g12);
              gstore(dst + o, g);
              acc[0] += (double)g * (double)g;
            }
            if (rb) {
              const T g = grad_value_plain<T>(v[c + i].im, BS_[i], BO[i], BW[i], al, lam, gs, g12);
              gstore(dst + o + a.ncols, g);
              acc[0] += (double)g * (double)g;
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < (HALF ? 4 : 8); ++i) {
        const int q = t + i * TPF;
        if (q < a.ncols) {
          const long long o = (long long)r0 * a.ncols + q;
          if (ra) {
            const T g = grad_at(o, v[i].re);
            gstore(dst + o, g);
            acc[0] += (double)g * (double)g;
          }
          if (rb) {
            const T g = grad_at(o + a.ncols, v[i].im);
            gstore(dst + o + a.ncols, g);
            acc[0] += (double)g * (double)g;
          }
        }
      }
    }
    block_partials<1>(acc, fz.pb, fz.pbn, fz.pbs, fz.self ? PB_L1 : PB_L0, pid, pcount);
    return;
  }
  double acc[1] = {0.0};
  // The scale factors of four entries per row go out together before any store; without a
  // scale they are ones, read from the output's first entry and discarded (no branch).
  const T* sbase = sc ? sc : dst;
  const bool scaled = sc != nullptr;
#pragma unroll
  for (int c = 0; c < (HALF ? 4 : 8); c += 4) {
    T SA[4], SB[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = t + (c + i) * TPF;
      const bool ok = (q < a.ncols) & scaled;
      const long long o = (long long)r0 * a.ncols + q;
      SA[i] = gload_or(sbase, o, ok & ra, T(1));
      SB[i] = gload_or(sbase, o + a.ncols, ok & rb, T(1));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = t + (c + i) * TPF;
      if (q < a.ncols) {
        const long long o = (long long)r0 * a.ncols + q;
        if (ra) {
          const T y = v[c + i].re * SA[i];
          gstore(dst + o, y);
          if constexpr (MODE == FUSE_QQ) acc[0] += (double)y * (double)y;
        }
        if (rb) {
          const T y = v[c + i].im * SB[i];
          gstore(dst + o + a.ncols, y);
          if constexpr (MODE == FUSE_QQ) acc[0] += (double)y * (double)y;
        }
      }
    }
  }
  if constexpr (MODE == FUSE_QQ) block_partials<1>(acc, fz.pb, fz.pbn, fz.pbs, fz.self ? PB_Q1 : PB_Q0, pid, pcount);
}

template <typename T, int N, bool ROWIN, int MODE, bool HALF>
__global__ void __launch_bounds__(512, (c2r_waves<T, N, ROWIN, MODE, HALF>())) k_frow_c2r(FRowArgs<T> a, Fuse<T> fz) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  frow_c2r_body<T, N, ROWIN, MODE, HALF>(a, fz, blockIdx.x, blockIdx.y, blockIdx.x + gridDim.x * blockIdx.y,
                                         gridDim.x * gridDim.y, smem_raw);
}

// ------------------------------------------------------------------------------------
// Column passes
// ------------------------------------------------------------------------------------
template <typename T>
struct FColArgs {
  const cx<T>* in;
  long long in_bs;
  const cx<T>* eig;  // complex [L][K2][N], or with eig_even real [L][K2][N/2 + 1]
  cx<T>* out;
  long long out_bs;
  long long out_cs;  // forward: stride between layer-chunk partials
  int L, nin, nout, ldin, ldout, K2, fpb, nchunk;
  const cx<T>* tw;
  int eig_even;  // the eigenvalues are real and even along x: lambda[N - k] = lambda[k]
};

// Eigenvalue k of a column of length N starting at `col` (EVEN: real and even, stored for
// k <= N/2 only; else complex, interleaved), as loaded: no select on it, since a prefetched
// value that is selected at once is waited for at once.
template <typename T, int N, bool EVEN>
__device__ __forceinline__ cx<T> eig_at(const T* col, int k) {
  if constexpr (EVEN) return cx<T>{gload(col + (k <= N / 2 ? k : N - k)), T(0)};
  return gload(reinterpret_cast<const cx<T>*>(col) + k);
}
// Start of the stored eigenvalue column k2 of layer l.
template <typename T, int N, bool EVEN>
__device__ __forceinline__ const T* eig_col(const cx<T>* eig, int K2, int l, int k2) {
  constexpr int R = EVEN ? N / 2 + 1 : 2 * N;  // reals per column
  return reinterpret_cast<const T*>(eig) + ((long long)l * K2 + k2) * R;
}

// Column jobs: job k2 in [0, K2) is column k2 of the row spectra.  The two real columns
// (k2 = 0 and Py/2) are ordinary complex jobs with zero imaginary parts: combining them into
// one transform saves one job in K2 but needs a separate path whose registers every block
// would then reserve.

// Accumulator of the forward layer sum: the plan's type (the sum is part of the product,
// whose FFTs and multiplies run in that type), or FP64 when built with BTTB_LAYER_SUM_F64=1.
#ifndef BTTB_LAYER_SUM_F64
#define BTTB_LAYER_SUM_F64 0
#endif
template <typename T>
struct LayerAcc {
  using type = typename std::conditional<BTTB_LAYER_SUM_F64 != 0, double, T>::type;
};
template <typename A>
struct AccPair {
  A x, y;
};

// One layer's prefetched operands of a column pass.
template <typename T, bool COL>
struct ColBuf {
  cx<T> un[COL ? 8 : 1], en[8];
};

// Layer loop of the forward column pass for one group: acc += eig_l . FFT_x(column_l).  The
// next layer's eigenvalues (and in FP32 its column) are loaded while the current one is
// transformed; FP64 keeps the column load in place to stay within 256 registers.  (A second
// layer in flight was measured slower: the extra registers cost more than the latency they
// hide.)
template <typename T, int N, bool EVEN, bool HALF>
__device__ __forceinline__ void fwd_layers(const FColArgs<T>& a, const FFTOf<T, N>& F, cx<T>* buf, int t, int f,
                                           int G, int k2, int l0, int l1, int b,
                                           typename LayerAcc<T>::type (&ar)[8],
                                           typename LayerAcc<T>::type (&ai)[8]) {
  using Acc = typename LayerAcc<T>::type;
  constexpr int TPF = N / 8;
  constexpr bool PF_IN = sizeof(T) == 4;
  GroupSync<Len<N>::LANES> gsync;
  const cx<T>* src = a.in + b * a.in_bs + (long long)k2 * a.ldin;
  const long long lstride_in = (long long)a.K2 * a.ldin;
  const int nit = (l1 - l0 + G - 1) / G;
  using Buf = ColBuf<T, PF_IN>;
  auto load_col = [&](int l, int i) -> cx<T> {
    if (HALF && i >= 4) return cx<T>{T(0), T(0)};  // zero padding, known at compile time
    const int n = t + i * TPF;
    return gload_or(src, l * lstride_in + n, l < l1 && n < a.nin);  // (a branch here measures faster)
  };
  // The next layer's loads go into B as loaded: the zero padding past nin is applied when the
  // layer is used (a select right after the load would wait for it there), and a layer past
  // l1 loads layer l0 and is discarded (its products are not accumulated).
  auto fetch = [&](Buf& B, int l) {
    const int le = l < l1 ? l : l0;
    const T* ecol = eig_col<T, N, EVEN>(a.eig, a.K2, le, k2);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int n = t + i * TPF;
      if constexpr (PF_IN) {
        if (!(HALF && i >= 4)) B.un[i] = gload(src + le * lstride_in + (n < a.nin ? n : 0));
      }
      B.en[i] = eig_at<T, N, EVEN>(ecol, n);
    }
  };
  auto layer = [&](int it, Buf& B) {
    const int l = l0 + it * G + f;
    const bool act = l < l1;
    cx<T> v[8], e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (PF_IN) {
        v[i] = (HALF && i >= 4) || t + i * TPF >= a.nin ? cx<T>{T(0), T(0)} : B.un[i];
      } else {
        v[i] = load_col(l, i);
      }
      e[i] = B.en[i];
    }
    if (it + 1 < nit) fetch(B, l + G);
    F.template run<false>(v, buf, t, gsync);
    if (act) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Acc xr = v[i].re, xi = v[i].im, wr = e[i].re, wi = e[i].im;
        ar[i] += wr * xr - wi * xi;
        ai[i] += wr * xi + wi * xr;
      }
    }
  };
  Buf B;
  fetch(B, l0 + f);
  for (int it = 0; it < nit; ++it) layer(it, B);
}

// Forward: partial over the layers of chunk c of sum_l eig_l . FFT_x(U_l column), then the
// inverse FFT_x; rows p < nout are written row-major to out[c][p][k2] (ldout = padded K2).
// FP64 column blocks are limited to 256 threads so that the registers beyond 256 per lane
// (the accumulation registers) can hold what does not fit, instead of scratch memory.
constexpr int col_threads(int esz) { return esz == 4 ? 512 : 256; }

// Block of column job k2, layer chunk c, batch entry b.
// HALF (nin, nout <= N/2): the upper four inputs of a lane are zero padding and its upper four
// outputs are not stored, both known at compile time.
template <typename T, int N, bool HALF>
__device__ __forceinline__ void fcol_fwd_body(const FColArgs<T>& a, int k2, int c, int b, unsigned char* smem_raw) {
  using P = Len<N>;
  constexpr int TPF = P::TPF, LANES = P::LANES;
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / LANES, tl = threadIdx.x - f * LANES;
  // a 5-smooth size's lanes past TPF hold no values: they index as lane 0 and store nothing
  const bool live = P::POW2 || tl < TPF;
  const int t = P::POW2 ? tl : (live ? tl : 0);
  const int G = a.fpb;
  const int l0 = (c * a.L) / a.nchunk, l1 = ((c + 1) * a.L) / a.nchunk;
  cx<T>* buf = smem + f * P::BUF;
  GroupSync<LANES> gsync;
  FFTOf<T, N> F;
  F.init(a.tw, t);
  if constexpr (!P::POW2) F.live = live;
  using Acc = typename LayerAcc<T>::type;
  Acc ar[8], ai[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) ar[i] = ai[i] = Acc(0);
  if (a.eig_even) fwd_layers<T, N, true, HALF>(a, F, buf, t, f, G, k2, l0, l1, b, ar, ai);
  else fwd_layers<T, N, false, HALF>(a, F, buf, t, f, G, k2, l0, l1, b, ar, ai);
  // tree reduction of the groups' accumulators (G is a power of two)
  AccPair<Acc>* red = reinterpret_cast<AccPair<Acc>*>(smem_raw);
  for (int half = G >> 1; half >= 1; half >>= 1) {
    __syncthreads();
    if (live && f >= half && f < 2 * half) {
#pragma unroll
      for (int i = 0; i < 8; ++i) red[(f - half) * N + t + i * TPF] = AccPair<Acc>{ar[i], ai[i]};
    }
    __syncthreads();
    if (f < half) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const AccPair<Acc> u = red[f * N + t + i * TPF];
        ar[i] += u.x;
        ai[i] += u.y;
      }
    }
  }
  __syncthreads();
  if (LANES > 64 || f == 0) {  // groups wider than a wave run the transform together
    cx<T> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = cx<T>{(T)ar[i], (T)ai[i]};
    F.template run<true>(v, buf, t, gsync);
    if (live && f == 0) {
      cx<T>* dst = a.out + b * a.out_bs + c * a.out_cs;
#pragma unroll
      for (int i = 0; i < (HALF ? 4 : 8); ++i) {
        const int p = t + i * TPF;
        if (p < a.nout) gstore(dst + (long long)p * a.ldout + k2, v[i]);
      }
    }
  }
}

template <typename T, int N, bool HALF>
__global__ void __launch_bounds__(col_threads(sizeof(T))) k_fcol_fwd(FColArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fcol_fwd_body<T, N, HALF>(a, blockIdx.x, blockIdx.y, blockIdx.z, smem_raw);
}

// Layer loop of the transpose column pass for one group: per layer conj(eig_l) R, inverse
// FFT_x, rows a < nout stored.  The next layer's eigenvalues are loaded while the current one
// is transformed.
template <typename T, int N, bool EVEN, bool HALF>
__device__ __forceinline__ void adj_layers(const FColArgs<T>& a, const FFTOf<T, N>& F, cx<T>* buf, int t, int f,
                                           int G, int k2, int l0, int l1, int b, const cx<T> (&R)[8],
                                           bool live) {
  constexpr int TPF = N / 8;
  GroupSync<Len<N>::LANES> gsync;
  cx<T>* dst = a.out + b * a.out_bs + (long long)k2 * a.ldout;
  const long long lstride_out = (long long)a.K2 * a.ldout;
  const int nit = (l1 - l0 + G - 1) / G;
  using Buf = ColBuf<T, false>;
  // the next layer's eigenvalues as loaded (a layer past l1 loads layer l0; it is not stored)
  auto fetch = [&](Buf& B, int l) {
    const T* ecol = eig_col<T, N, EVEN>(a.eig, a.K2, l < l1 ? l : l0, k2);
#pragma unroll
    for (int i = 0; i < 8; ++i) B.en[i] = eig_at<T, N, EVEN>(ecol, t + i * TPF);
  };
  // (live: false for a 5-smooth size's lanes past TPF, which store nothing)
  auto layer = [&](int it, Buf& B) {
    const int l = l0 + it * G + f;
    const bool act = live && l < l1;
    cx<T> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = cmulc(R[i], B.en[i]);
    if (it + 1 < nit) fetch(B, l + G);
    F.template run<true>(v, buf, t, gsync);
    if (act) {
#pragma unroll
      for (int i = 0; i < (HALF ? 4 : 8); ++i) {
        const int p = t + i * TPF;
        if (p < a.nout) gstore(dst + l * lstride_out + p, v[i]);
      }
    }
  };
  Buf B;
  fetch(B, l0 + f);
  for (int it = 0; it < nit; ++it) layer(it, B);
}

// Transpose: R = FFT_x(Rrow column) once per block (group 0, shared through LDS), then for
// each layer of chunk c, conj(eig_l) R and the inverse FFT_x; rows a < nout are written
// to out[l][k2][a] (ldout = padded rows).  Rrow is row-major Rrow[p][k2] (ldin = padded K2).
template <typename T, int N, bool HALF>
__device__ __forceinline__ void fcol_adj_body(const FColArgs<T>& a, int k2, int c, int b, unsigned char* smem_raw) {
  using P = Len<N>;
  constexpr int TPF = P::TPF, LANES = P::LANES;
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / LANES, tl = threadIdx.x - f * LANES;
  const bool live = P::POW2 || tl < TPF;  // as in the forward pass
  const int t = P::POW2 ? tl : (live ? tl : 0);
  const int G = a.fpb;
  const int l0 = (c * a.L) / a.nchunk, l1 = ((c + 1) * a.L) / a.nchunk;
  cx<T>* buf = smem + f * P::BUF;
  cx<T>* Rs = smem + G * P::BUF;  // the shared column spectrum, N values
  GroupSync<LANES> gsync;
  FFTOf<T, N> F;
  F.init(a.tw, t);
  if constexpr (!P::POW2) F.live = live;
  const cx<T>* col = a.in + b * a.in_bs;
  if (LANES > 64 || f == 0) {
    cx<T> R[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int n = t + i * TPF;
      R[i] = (HALF && i >= 4) || n >= a.nin ? cx<T>{T(0), T(0)} : gload(col + (long long)n * a.ldin + k2);
    }
    F.template run<false>(R, buf, t, gsync);
    if (live && f == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) Rs[t + i * TPF] = R[i];
    }
  }
  __syncthreads();
  cx<T> R[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) R[i] = Rs[t + i * TPF];
  if (a.eig_even) adj_layers<T, N, true, HALF>(a, F, buf, t, f, G, k2, l0, l1, b, R, live);
  else adj_layers<T, N, false, HALF>(a, F, buf, t, f, G, k2, l0, l1, b, R, live);
}

template <typename T, int N, bool HALF>
__global__ void __launch_bounds__(col_threads(sizeof(T))) k_fcol_adj(FColArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fcol_adj_body<T, N, HALF>(a, blockIdx.x, blockIdx.y, blockIdx.z, smem_raw);
}

}  // namespace bttb
