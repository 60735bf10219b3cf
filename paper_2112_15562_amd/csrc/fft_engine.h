// Device FFT engine for gfx950: mixed radix (2, 3, 4, 5, 8) Stockham transforms held in
// LDS, one group of N/8 threads per length-N transform, several transforms per block.
//
// The FFT2 of Sec. 2.7.1 is computed as 1-D transforms along rows (in the row kernels)
// and along columns (in the column kernels); this header holds only the 1-D engine.
//
// Stockham pass with radix R at sub-transform length Ns (Ns = product of the radices
// already applied): butterfly j in [0, N/R) reads x[j + r N/R], r < R, multiplies input
// r by w^(r k) with k = j mod Ns and w = exp(-+2 pi i / (Ns R)), applies the R-point DFT
// and writes y[(j - k) R + k + r Ns].  After the last pass the data are in natural
// order.  Each pass reads all of a thread's inputs into registers, waits at a block
// barrier, then writes in place, so one LDS buffer of N values per transform suffices.
// With N/8 threads per transform a thread holds at most 10 values in any pass.
#pragma once
#include <hip/hip_runtime.h>

namespace bttb {

template <typename T>
struct cx {
  T re, im;
};

// Loads and stores through the global address space.  Most kernel pointers arrive through
// descriptor tables, which leaves the compiler unable to tell them from LDS pointers; it
// would then use flat instructions, which count against the LDS / scalar-load counter as
// well, so that every LDS exchange or scalar wait would also wait for them.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ __forceinline__ cx<T> gload(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  const v2 x = *(const __attribute__((address_space(1))) v2*)p;
  return cx<T>{x.x, x.y};
}
// p[i] when ok, else z, without a branch: a lane that is out of range loads p[0] (which
// exists) and discards it, so a thread's guarded loads issue back to back instead of one
// exec-masked block each, with the conversions the compiler would place inside them.
template <typename T>
__device__ __forceinline__ T gload_or(const T* p, long long i, bool ok, T z = T(0)) {
  const T x = gload(p + (ok ? i : 0));
  return ok ? x : z;
}
template <typename T>
__device__ __forceinline__ cx<T> gload_or(const cx<T>* p, long long i, bool ok) {
  const cx<T> x = gload(p + (ok ? i : 0));
  return ok ? x : cx<T>{T(0), T(0)};
}
template <typename T>
__device__ __forceinline__ void gstore(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  v2 x;
  x.x = v.re;
  x.y = v.im;
  *(__attribute__((address_space(1))) v2*)p = x;
}

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot_i(cx<T> a) {
  if (INV) return {-a.im, a.re};
  return {a.im, -a.re};
}

constexpr int kMaxPass = 12;

// Radix plan of one 1-D length (passed by value in kernel arguments).
struct FFTDesc {
  int N;
  int npass;
  int radix[kMaxPass];
};

// ---------------------------------------------------------------------------------
// Small DFTs.  Forward uses exp(-2 pi i nk/R), inverse exp(+2 pi i nk/R), unscaled.
// ---------------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  cx<T> t2 = cadd(a1, a3), t3 = rot_i<T, INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cx<T>* v) {
  const T h = T(0.5);
  const T s = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
  cx<T> t = cadd(v[1], v[2]);
  cx<T> u = csub(v[1], v[2]);
  cx<T> m = {v[0].re - h * t.re, v[0].im - h * t.im};
  cx<T> su = rot_i<T, INV>(cscale(u, s));  // -+ i s u
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, su);
  v[2] = csub(m, su);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft5(cx<T>* v) {
  const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi / 5)
  const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi / 5)
  const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi / 5)
  const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi / 5)
  cx<T> t1 = cadd(v[1], v[4]), t3 = csub(v[1], v[4]);
  cx<T> t2 = cadd(v[2], v[3]), t4 = csub(v[2], v[3]);
  cx<T> b1 = {v[0].re + c1 * t1.re + c2 * t2.re, v[0].im + c1 * t1.im + c2 * t2.im};
  cx<T> b2 = {v[0].re + c2 * t1.re + c1 * t2.re, v[0].im + c2 * t1.im + c1 * t2.im};
  cx<T> e1 = rot_i<T, INV>(cx<T>{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
  cx<T> e2 = rot_i<T, INV>(cx<T>{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(b1, e1);
  v[4] = csub(b1, e1);
  v[2] = cadd(b2, e2);
  v[3] = csub(b2, e2);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T r = T(0.70710678118654752440084436210485);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  // twiddles w^k, w = exp(-+ 2 pi i / 8), k = 1, 2, 3
  cx<T> w1, w3;
  if (INV) {
    w1 = {r * (o1.re - o1.im), r * (o1.re + o1.im)};
    w3 = {-r * (o3.re + o3.im), r * (o3.re - o3.im)};
  } else {
    w1 = {r * (o1.re + o1.im), r * (o1.im - o1.re)};
    w3 = {r * (o3.im - o3.re), -r * (o3.re + o3.im)};
  }
  cx<T> w2 = rot_i<T, INV>(o2);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1);
  v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2);
  v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3);
  v[7] = csub(e3, w3);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else dft8<T, INV>(v);
}

// One in-place Stockham pass over the transform in `buf` (N values), executed by the
// TPF = N/8 threads t = 0..TPF-1 of this transform.  tw[e] = exp(-2 pi i e / N).
// Every thread of the block must call it (it contains block barriers).
template <typename T, int R, bool INV>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int N, int Ns, const cx<T>* __restrict__ tw,
                                              int t, int TPF, bool active) {
  constexpr int BPT = (8 + R - 1) / R;  // butterflies per thread
  const int nb = N / R;
  const int tws = N / (Ns * R);
  cx<T> v[BPT][R];
  int kk[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * TPF;
    kk[b] = 0;
    if (active && j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * nb];
      const int k = j % Ns;
      kk[b] = k;
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * tws];
          if (INV) w.im = -w.im;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dft_small<T, R, INV>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * TPF;
    if (active && j < nb) {
      const int k = kk[b];
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

// Full 1-D transform of the N values in `buf` (natural order in, natural order out).
// Callers must have synchronised after writing `buf`; the function ends with a barrier.
template <typename T, bool INV>
__device__ __forceinline__ void fft_lds(cx<T>* buf, const FFTDesc& d, const cx<T>* __restrict__ tw, int t,
                                        int TPF, bool active) {
  int Ns = 1;
  for (int p = 0; p < d.npass; ++p) {
    const int R = d.radix[p];
    if (R == 8) stockham_pass<T, 8, INV>(buf, d.N, Ns, tw, t, TPF, active);
    else if (R == 4) stockham_pass<T, 4, INV>(buf, d.N, Ns, tw, t, TPF, active);
    else if (R == 2) stockham_pass<T, 2, INV>(buf, d.N, Ns, tw, t, TPF, active);
    else if (R == 5) stockham_pass<T, 5, INV>(buf, d.N, Ns, tw, t, TPF, active);
    else stockham_pass<T, 3, INV>(buf, d.N, Ns, tw, t, TPF, active);
    Ns *= R;
  }
}

}  // namespace bttb
