// Register-resident FFT of a power-of-two length N (8 <= N <= 2048) for gfx950.
//
// A transform is held by a group of TPF = N/8 lanes, 8 values per lane, in the
// "strided" layout v[i] = x[t + i TPF] (t = lane within the group).  The passes are
// radix 8 (log2 N / 3 of them) followed, when log2 N is not a multiple of 3, by one
// radix-2 or radix-4 pass.  A pass with radix R runs 8/R butterflies per lane; the
// butterfly j = t + b TPF reads x[j + r N/R] = v[b + (8/R) r], which is already the
// strided layout, multiplies input r by w^(r k) with k = j mod Ns (Ns the product of
// the earlier radices; w = exp(-+2 pi i/(Ns R))), applies the R-point DFT and produces
// y[(j - k) R + k + r Ns].  For the last pass Ns = N/R, so y lands back on index
// b + (8/R) r of the same lane; between the other passes the values go through LDS
// (write at their output position, group barrier, read the strided layout).
// Each lane's twiddles are the same for every transform it runs, so they are read
// once from the table into registers.
//
// The first pass therefore reads the input straight from global memory (lane t loads
// x[t + i TPF]: consecutive lanes, consecutive addresses) and the output of the last
// pass is directly usable for elementwise products and coalesced stores.
// LDS addresses are padded by one element every 8 to avoid bank conflicts.
#pragma once
#include "fft_engine.h"

namespace bttb {

__host__ __device__ __forceinline__ constexpr int lds_pad(int i) { return i + (i >> 3); }

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <int N>
struct Pow2 {
  static_assert(N >= 8 && N <= 2048 && (N & (N - 1)) == 0, "power of two in [8, 2048]");
  static constexpr int TPF = N / 8;
  static constexpr int LG = ilog2(N);
  static constexpr int NFULL = LG / 3;
  static constexpr int REM = LG % 3;
  static constexpr int NPASS = NFULL + (REM ? 1 : 0);
  static constexpr int BUF = lds_pad(N - 1) + 1;  // LDS elements of one exchange buffer
  static constexpr int radix(int p) { return p < NFULL ? 8 : (1 << REM); }
  static constexpr int ns(int p) { return p == 0 ? 1 : ns(p - 1) * radix(p - 1); }
  static constexpr int tw_before(int p) {  // twiddles of the passes 1..p-1
    return p <= 1 ? 0 : tw_before(p - 1) + (8 / radix(p - 1)) * (radix(p - 1) - 1);
  }
  static constexpr int NTW = tw_before(NPASS);
};

template <typename T, int N>
struct RegFFT {
  using P = Pow2<N>;
  static constexpr int TPF = P::TPF;
  cx<T> w[P::NTW > 0 ? P::NTW : 1];

  // Loads this lane's twiddles from tab[e] = exp(-2 pi i e / N).
  __device__ __forceinline__ void init(const cx<T>* __restrict__ tab, int t) {
    init_pass<1>(tab, t);
  }

  template <int PS>
  __device__ __forceinline__ void init_pass(const cx<T>* __restrict__ tab, int t) {
    if constexpr (PS < P::NPASS) {
      constexpr int R = P::radix(PS), BPT = 8 / R, NS = P::ns(PS), OFF = P::tw_before(PS);
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int k = (t + b * TPF) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[OFF + b * (R - 1) + r - 1] = gload(tab + r * k * (N / (NS * R)));
      }
      init_pass<PS + 1>(tab, t);
    }
  }

  // Transform v in place (strided layout in and out).  `buf` is this group's exchange
  // buffer (P::BUF elements); `sync` is a barrier covering every lane of the group.
  // All lanes of the block must call this the same number of times.
  template <bool INV, typename Sync>
  __device__ __forceinline__ void run(cx<T> (&v)[8], cx<T>* buf, int t, Sync sync) const {
    pass<0, INV>(v, buf, t, sync);
  }

  template <int PS, bool INV, typename Sync>
  __device__ __forceinline__ void pass(cx<T> (&v)[8], cx<T>* buf, int t, Sync sync) const {
    if constexpr (PS < P::NPASS) {
      constexpr int R = P::radix(PS), BPT = 8 / R, NS = P::ns(PS), OFF = P::tw_before(PS);
      constexpr bool LAST = PS == P::NPASS - 1;
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        cx<T> u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b + BPT * r];
        if constexpr (PS > 0) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> ww = w[OFF + b * (R - 1) + r - 1];
            if (INV) ww.im = -ww.im;
            u[r] = cmul(u[r], ww);
          }
        }
        dft_small<T, R, INV>(u);
        if constexpr (LAST) {
#pragma unroll
          for (int r = 0; r < R; ++r) v[b + BPT * r] = u[r];
        } else {
          const int j = t + b * TPF;
          const int k = j & (NS - 1);
          const int base = (j - k) * R + k;
#pragma unroll
          for (int r = 0; r < R; ++r) buf[lds_pad(base + r * NS)] = u[r];
        }
      }
      if constexpr (!LAST) {
        sync();
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = buf[lds_pad(t + i * TPF)];
        sync();
        pass<PS + 1, INV>(v, buf, t, sync);
      }
    }
  }
};

struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

}  // namespace bttb
