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
#include <type_traits>

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

// Sizes of the register-layout kernels: N = 8 M transforms held by TPF = N/8 lanes, 8 values per
// lane (v[i] = x[t + i TPF]).  A transform's group of lanes is LANES = TPF rounded up to a power
// of two, so that a group never straddles a wave; the lanes t >= TPF of a 5-smooth size's group
// hold no values (they compute on lane 0's indices and store nothing).  BUF is one group's padded
// exchange buffer.
template <int N>
struct Len {
  static_assert(N % 8 == 0, "a multiple of 8");
  static constexpr int TPF = N / 8;
  static constexpr bool POW2 = (N & (N - 1)) == 0;
  static constexpr int LANES = TPF <= 1 ? 1 : 2 * (1 << ilog2(TPF - 1));
  static constexpr int BUF = lds_pad(N - 1) + 1;
};

// DFTs of the composite radices 6, 9, 10 and 15 used by the 5-smooth transforms, from the 2-, 3-
// and 5-point DFTs (forward exp(-2 pi i nk/R), inverse exp(+2 pi i nk/R), unscaled).  6, 10 and 15
// by the prime-factor mapping of R = R1 R2 (coprime): input n = (R2 n1 + R1 n2) mod R, R1-point
// DFTs over n1, R2-point DFTs over n2, output index the k < R with k = k1 mod R1 and k = k2 mod
// R2 (no twiddles); 9 = 3 x 3 by Cooley-Tukey: input n = 3 n1 + n2, 3-point DFTs over n1, twiddles
// exp(-+2 pi i n2 k1 / 9), 3-point DFTs over n2, output k1 + 3 k2.
__host__ __device__ constexpr int inv_mod(int a, int m) {  // a^-1 mod m (a, m coprime)
  int x = 1;
  while ((a * x) % m != 1) ++x;
  return x;
}

template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void dft_pfa(cx<T>* v) {
  constexpr int R = R1 * R2;
  // output k = (k1 E1 + k2 E2) mod R: E1 = 1 mod R1 and 0 mod R2, E2 the other way round
  constexpr int E1 = R2 * inv_mod(R2 % R1, R1), E2 = R1 * inv_mod(R1 % R2, R2);
  cx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    cx<T> a[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[(R2 * n1 + R1 * n2) % R];
    dft_small<T, R1, INV>(a);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) y[n2][k1] = a[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> b[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) b[n2] = y[n2][k1];
    dft_small<T, R2, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[(k1 * E1 + k2 * E2) % R] = b[k2];
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft9(cx<T>* v) {
  // cos and sin of 2 pi m / 9, m = 1, 2, 4
  const T c1 = T(0.766044443118978), s1 = T(0.6427876096865393);
  const T c2 = T(0.17364817766693041), s2 = T(0.984807753012208);
  const T c4 = T(-0.9396926207859083), s4 = T(0.3420201433256689);
  cx<T> y[3][3];
#pragma unroll
  for (int n2 = 0; n2 < 3; ++n2) {
    cx<T> a[3] = {v[n2], v[3 + n2], v[6 + n2]};
    dft3<T, INV>(a);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) y[n2][k1] = a[k1];
  }
  const T sg = INV ? T(1) : T(-1);  // exp(-+ i theta) = cos theta -+ i sin theta
  y[1][1] = cmul(y[1][1], cx<T>{c1, sg * s1});
  y[1][2] = cmul(y[1][2], cx<T>{c2, sg * s2});
  y[2][1] = cmul(y[2][1], cx<T>{c2, sg * s2});
  y[2][2] = cmul(y[2][2], cx<T>{c4, sg * s4});
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    cx<T> b[3] = {y[0][k1], y[1][k1], y[2][k1]};
    dft3<T, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) v[k1 + 3 * k2] = b[k2];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_any(cx<T>* v) {
  if constexpr (R == 6) dft_pfa<T, 2, 3, INV>(v);
  else if constexpr (R == 10) dft_pfa<T, 2, 5, INV>(v);
  else if constexpr (R == 15) dft_pfa<T, 3, 5, INV>(v);
  else if constexpr (R == 9) dft9<T, INV>(v);
  else dft_small<T, R, INV>(v);
}

// Pass plan of a 5-smooth length N = 8 M: radix 8 first (straight from the register layout); when
// M is even, a last pass of radix 8, 4 or 2 (the largest its power-of-two part allows), which
// also runs in registers; between them, passes through LDS over the rest of M, each of the
// largest radix among 15, 10, 9, 8, 6, 5, 4, 3, 2 that divides what remains (fewer passes, fewer
// LDS round trips).
struct MixPlan {
  int npass;
  int radix[16];
};
__host__ __device__ constexpr MixPlan mix_plan(int N) {
  MixPlan p{};
  p.npass = 0;
  p.radix[p.npass++] = 8;
  const int M = N / 8;
  int a = 0;
  for (int m = M; m % 2 == 0; m /= 2) ++a;
  const int last = a >= 3 ? 8 : a == 2 ? 4 : a == 1 ? 2 : 1;
  int rest = M / last;
  const int cand[9] = {15, 10, 9, 8, 6, 5, 4, 3, 2};
  while (rest > 1) {
    for (int i = 0; i < 9; ++i) {
      if (rest % cand[i] == 0) {
        p.radix[p.npass++] = cand[i];
        rest /= cand[i];
        break;
      }
    }
  }
  if (last > 1) p.radix[p.npass++] = last;
  return p;
}

// Transform of a 5-smooth length N = 8 M with M not a power of two, in the register layout of
// RegFFT (in and out: v[i] = x[t + i TPF], TPF = N/8 lanes).  Stockham passes as in RegFFT: pass p
// of radix R at sub-length Ns runs butterflies j in [0, N/R), reading x[j + r N/R], twiddling input r
// by w^(r k), k = j mod Ns, and writing y[(j - k) R + k + r Ns].  The first pass (radix 8, Ns = 1)
// reads the lane's own registers; the passes after it go through the group's LDS buffer, each
// lane taking the butterflies t, t + TPF, ... (radices 3 and 5 leave some lanes one butterfly
// short; radices 6, 9, 10, 15 are composite DFTs in registers); a last pass of radix 2, 4 or 8 has
// Ns = N/R and runs in registers again.  LDS indices
// are padded by one element every 8 (lds_pad), as in RegFFT, against bank conflicts.  `sync` orders
// the group's LDS accesses (a wave barrier for groups inside one wave).  Lanes with live = false
// touch no memory.  Twiddles: tab[e] = exp(-2 pi i e / N), copied once per block into LDS for the
// passes through the buffer (whose reads then overlap the data's); the last pass's are loaded once
// into registers.  init() holds a block barrier: every thread of the block calls it.
template <typename T, int N>
struct MixFFT {
  static_assert(!Len<N>::POW2, "powers of two take RegFFT");
  static constexpr int TPF = N / 8;
  static constexpr MixPlan PLAN = mix_plan(N);
  static constexpr int NP = PLAN.npass;
  static constexpr int RL = PLAN.radix[NP - 1];            // last radix
  static constexpr bool LAST_REG = RL == 2 || RL == 4 || RL == 8;
  static constexpr int BL = LAST_REG ? 8 / RL : 1;          // butterflies per lane in the last pass
  const cx<T>* tab;
  bool live = true;
  cx<T> wl[LAST_REG ? BL * (RL - 1) : 1];

  __device__ __forceinline__ void init(const cx<T>* __restrict__ t_, int t) {
    tab = t_;
    cx<T>* tl = lds_table();
    for (int i = threadIdx.x; i < N; i += blockDim.x) tl[i] = gload(tab + i);
    __syncthreads();
    if constexpr (LAST_REG) {  // last pass: k = j = t + b TPF, twiddle r k of the N-point table
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int r = 1; r < RL; ++r) wl[b * (RL - 1) + r - 1] = gload(tab + r * (t + b * TPF));
    }
  }

  template <bool INV, typename Sync>
  __device__ __forceinline__ void run(cx<T> (&v)[8], cx<T>* buf, int t, Sync sync) const {
    // pass 0: radix 8 on the lane's values x[t + r TPF] (butterfly j = t, no twiddles),
    // outputs y[8 t + r]
    dft8<T, INV>(v);
    if (live) {
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[lds_pad(8 * t + r)] = v[r];
    }
    sync();
    lds_passes<1, 8, INV>(buf, t, sync);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = buf[lds_pad(t + i * TPF)];  // (live or not: t < TPF)
    sync();
    if constexpr (LAST_REG) {
#pragma unroll
      for (int b = 0; b < BL; ++b) {
        cx<T> u[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) u[r] = v[b + BL * r];
#pragma unroll
        for (int r = 1; r < RL; ++r) {
          cx<T> w = wl[b * (RL - 1) + r - 1];
          if (INV) w.im = -w.im;
          u[r] = cmul(u[r], w);
        }
        dft_small<T, RL, INV>(u);
#pragma unroll
        for (int r = 0; r < RL; ++r) v[b + BL * r] = u[r];
      }
    }
  }

  // The block's copy of the twiddle table.
  __device__ __forceinline__ static cx<T>* lds_table() {
    __shared__ cx<T> tw_lds[N];
    return tw_lds;
  }

  // Passes PS .. (the last one excluded when it runs in registers) through the buffer.
  template <int PS, int NS, bool INV, typename Sync>
  __device__ __forceinline__ void lds_passes(cx<T>* buf, int t, Sync sync) const {
    if constexpr (PS < (LAST_REG ? NP - 1 : NP)) {
      constexpr int R = PLAN.radix[PS], NB = N / R, BPT = (NB + TPF - 1) / TPF, TWS = N / (NS * R);
      cx<T> u[BPT][R];
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int j = t + b * TPF;
        if (live && j < NB) {
          const int k = j % NS;
#pragma unroll
          for (int r = 0; r < R; ++r) u[b][r] = buf[lds_pad(j + r * NB)];
          const cx<T>* tl = lds_table();
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = tl[r * k * TWS];
            if (INV) w.im = -w.im;
            u[b][r] = cmul(u[b][r], w);
          }
          dft_any<T, R, INV>(u[b]);
        }
      }
      sync();
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int j = t + b * TPF;
        if (live && j < NB) {
          const int k = j % NS;
          const int base = (j - k) * R + k;
#pragma unroll
          for (int r = 0; r < R; ++r) buf[lds_pad(base + r * NS)] = u[b][r];
        }
      }
      sync();
      lds_passes<PS + 1, NS * R, INV>(buf, t, sync);
    }
  }
};

// The transform the kernel bodies use for size N.
template <typename T, int N>
using FFTOf = typename std::conditional<Len<N>::POW2, RegFFT<T, N>, MixFFT<T, N>>::type;

}  // namespace bttb
