// Products for power-of-two transform sizes with the register-resident FFT (fft_reg.h).
//
// Same passes and intermediate layouts as the general kernels in operator.hip, with
// three differences: (1) a transform's first pass reads global memory directly and its
// last pass feeds the eigenvalue multiply, the layer accumulation and the stores from
// registers; (2) the forward column pass gives each block one column k2 and splits the
// layers over its groups, which reduce their FP64 accumulators in LDS, so one inverse
// column transform per column is written (no layer-chunk partials); (3) exchanges
// inside a transform use a wave-level barrier when the transform fits in one wave.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "fft_reg.h"

namespace bttb {

// Orders the LDS accesses of one wave: LDS requests of a wave complete in issue order,
// so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TPF>
struct GroupSync {
  __device__ __forceinline__ void operator()() const {
    if constexpr (TPF <= 64) wave_sync();
    else __syncthreads();
  }
};

template <int N>
constexpr int row_buf() {  // per-group LDS elements of the row kernels (exchange and [2][K2] staging)
  return Pow2<N>::BUF > N + 2 ? Pow2<N>::BUF : N + 2;
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

template <typename T, int N>
__global__ void __launch_bounds__(512) k_frow_r2c(FRowArgs<T> a) {
  using P = Pow2<N>;
  constexpr int TPF = P::TPF, BS = row_buf<N>(), K2 = N / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int l = blockIdx.x / a.tiles, tile = blockIdx.x - l * a.tiles;
  const int b = blockIdx.y;
  const int RT = 2 * a.fpb;
  const int r0 = tile * RT + 2 * f;
  cx<T>* buf = smem + f * BS;
  GroupSync<TPF> gsync;
  RegFFT<T, N> F;
  F.init(a.tw, t);
  const long long lofs = (long long)l * a.nrows * a.ncols;
  const T* src = a.in + b * a.in_bs + lofs;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  const bool ra = r0 < a.nrows, rb = r0 + 1 < a.nrows;
  cx<T> v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int n = t + i * TPF;
    T xa = T(0), xb = T(0);
    if (n < a.ncols) {
      const long long oa = (long long)r0 * a.ncols + n;
      if (ra) xa = sc ? src[oa] * sc[oa] : src[oa];
      if (rb) xb = sc ? src[oa + a.ncols] * sc[oa + a.ncols] : src[oa + a.ncols];
    }
    v[i] = cx<T>{xa, xb};
  }
  F.template run<false>(v, buf, t, gsync);
  // X_a[k] = (Z[k] + conj Z[N-k]) / 2,  X_b[k] = (Z[k] - conj Z[N-k]) / (2i),  k <= N/2
#pragma unroll
  for (int i = 0; i < 8; ++i) buf[lds_pad(t + i * TPF)] = v[i];
  gsync();
  const T h = T(0.5);
  cx<T> xa[5], xb[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int k = t + i * TPF;
    if (k <= N / 2) {
      const cx<T> A = v[i];
      const cx<T> C = buf[lds_pad((N - k) & (N - 1))];
      xa[i] = cx<T>{h * (A.re + C.re), h * (A.im - C.im)};
      xb[i] = cx<T>{h * (A.im + C.im), h * (C.re - A.re)};
    }
  }
  gsync();
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int k = t + i * TPF;
    if (k <= N / 2) {
      buf[k] = xa[i];
      buf[K2 + k] = xb[i];
    }
  }
  __syncthreads();
  cx<T>* dst = a.out + b * a.out_bs + (long long)l * K2 * a.ld + tile * RT;
  for (int idx = threadIdx.x; idx < K2 * RT; idx += blockDim.x) {
    const int k2 = idx / RT, rr = idx - k2 * RT;
    dst[(long long)k2 * a.ld + rr] = smem[(rr >> 1) * BS + (rr & 1) * K2 + k2];
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(512) k_frow_c2r(FRowArgs<T> a) {
  using P = Pow2<N>;
  constexpr int TPF = P::TPF, BS = row_buf<N>(), K2 = N / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int l = blockIdx.x / a.tiles, tile = blockIdx.x - l * a.tiles;
  const int b = blockIdx.y;
  const int RT = 2 * a.fpb;
  cx<T>* buf = smem + f * BS;
  GroupSync<TPF> gsync;
  RegFFT<T, N> F;
  F.init(a.tw, t);
  // here `in` is complex [nsum][L][K2][ld] and `out` real [L][nrows][ncols]
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.in) + b * a.in_bs + (long long)l * K2 * a.ld + tile * RT;
  for (int idx = threadIdx.x; idx < K2 * RT; idx += blockDim.x) {
    const int k2 = idx / RT, rr = idx - k2 * RT;
    const int row = tile * RT + rr;
    cx<T> hv{T(0), T(0)};
    if (row < a.nrows) {
      if (a.nsum == 1) {
        hv = src[(long long)k2 * a.ld + rr];
      } else {
        double hr = 0.0, hi = 0.0;
        for (int c = 0; c < a.nsum; ++c) {
          const cx<T> u = src[c * a.in_cs + (long long)k2 * a.ld + rr];
          hr += (double)u.re;
          hi += (double)u.im;
        }
        hv = cx<T>{(T)hr, (T)hi};
      }
    }
    if (k2 == 0 || k2 == K2 - 1) hv.im = T(0);  // DC and Nyquist of a real row are real
    smem[(rr >> 1) * BS + (rr & 1) * K2 + k2] = hv;
  }
  __syncthreads();
  cx<T> v[8];
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
  gsync();
  F.template run<true>(v, buf, t, gsync);
  const int r0 = tile * RT + 2 * f;
  const long long lofs = (long long)l * a.nrows * a.ncols;
  T* dst = reinterpret_cast<T*>(a.out) + b * a.out_bs + lofs;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  const bool ra = r0 < a.nrows, rb = r0 + 1 < a.nrows;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int q = t + i * TPF;
    if (q < a.ncols) {
      const long long o = (long long)r0 * a.ncols + q;
      if (ra) dst[o] = sc ? v[i].re * sc[o] : v[i].re;
      if (rb) dst[o + a.ncols] = sc ? v[i].im * sc[o + a.ncols] : v[i].im;
    }
  }
}

// ------------------------------------------------------------------------------------
// Column passes
// ------------------------------------------------------------------------------------
template <typename T>
struct FColArgs {
  const cx<T>* in;
  long long in_bs;
  const cx<T>* eig;
  cx<T>* out;
  long long out_bs;
  int L, nin, nout, ldin, ldout, K2, fpb;
  const cx<T>* tw;
};

// Forward: per column k2, sum over layers of eig_l . FFT_x(U_l column), inverse FFT_x.
template <typename T, int N>
__global__ void __launch_bounds__(512) k_fcol_fwd(FColArgs<T> a) {
  using P = Pow2<N>;
  constexpr int TPF = P::TPF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int G = a.fpb;
  const int k2 = blockIdx.x, b = blockIdx.y;
  cx<T>* buf = smem + f * P::BUF;
  GroupSync<TPF> gsync;
  RegFFT<T, N> F;
  F.init(a.tw, t);
  double ar[8], ai[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) ar[i] = ai[i] = 0.0;
  const cx<T>* src = a.in + b * a.in_bs + (long long)k2 * a.ldin;
  const cx<T>* eg = a.eig + (long long)k2 * N;
  const long long lstride_in = (long long)a.K2 * a.ldin, lstride_e = (long long)a.K2 * N;
  const int nit = (a.L + G - 1) / G;
  for (int it = 0; it < nit; ++it) {
    const int l = it * G + f;
    const bool act = l < a.L;
    cx<T> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int n = t + i * TPF;
      v[i] = (act && n < a.nin) ? src[l * lstride_in + n] : cx<T>{T(0), T(0)};
    }
    F.template run<false>(v, buf, t, gsync);
    if (act) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const cx<T> w = eg[l * lstride_e + t + i * TPF];
        const double xr = v[i].re, xi = v[i].im, wr = w.re, wi = w.im;
        ar[i] += wr * xr - wi * xi;
        ai[i] += wr * xi + wi * xr;
      }
    }
  }
  // tree reduction of the groups' accumulators (G is a power of two)
  double2* red = reinterpret_cast<double2*>(smem_raw);
  for (int half = G >> 1; half >= 1; half >>= 1) {
    __syncthreads();
    if (f >= half && f < 2 * half) {
#pragma unroll
      for (int i = 0; i < 8; ++i) red[(f - half) * N + t + i * TPF] = make_double2(ar[i], ai[i]);
    }
    __syncthreads();
    if (f < half) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double2 u = red[f * N + t + i * TPF];
        ar[i] += u.x;
        ai[i] += u.y;
      }
    }
  }
  __syncthreads();
  if (TPF > 64 || f == 0) {  // groups wider than a wave run the transform together
    cx<T> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = cx<T>{(T)ar[i], (T)ai[i]};
    F.template run<true>(v, buf, t, gsync);
    if (f == 0) {
      cx<T>* dst = a.out + b * a.out_bs + (long long)k2 * a.ldout;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = t + i * TPF;
        if (p < a.nout) dst[p] = v[i];
      }
    }
  }
}

// Transpose: per column k2, R = FFT_x(Rrow column) once, then per layer conj(eig_l) R
// and the inverse FFT_x; rows a < nout are written.
template <typename T, int N>
__global__ void __launch_bounds__(512) k_fcol_adj(FColArgs<T> a) {
  using P = Pow2<N>;
  constexpr int TPF = P::TPF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int G = a.fpb;
  const int k2 = blockIdx.x, b = blockIdx.y;
  cx<T>* buf = smem + f * P::BUF;
  GroupSync<TPF> gsync;
  RegFFT<T, N> F;
  F.init(a.tw, t);
  const cx<T>* col = a.in + b * a.in_bs + (long long)k2 * a.ldin;
  cx<T> R[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int n = t + i * TPF;
    R[i] = n < a.nin ? col[n] : cx<T>{T(0), T(0)};
  }
  F.template run<false>(R, buf, t, gsync);
  const cx<T>* eg = a.eig + (long long)k2 * N;
  cx<T>* dst = a.out + b * a.out_bs + (long long)k2 * a.ldout;
  const long long lstride_out = (long long)a.K2 * a.ldout, lstride_e = (long long)a.K2 * N;
  const int nit = (a.L + G - 1) / G;
  for (int it = 0; it < nit; ++it) {
    const int l = it * G + f;
    const bool act = l < a.L;
    cx<T> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = act ? cmulc(R[i], eg[l * lstride_e + t + i * TPF]) : cx<T>{T(0), T(0)};
    F.template run<true>(v, buf, t, gsync);
    if (act) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = t + i * TPF;
        if (p < a.nout) dst[l * lstride_out + p] = v[i];
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// Dispatch on the transform size
// ------------------------------------------------------------------------------------
#define BTTB_POW2_SWITCH(N, CALL) \
  switch (N) {                    \
    case 8: CALL(8); break;       \
    case 16: CALL(16); break;     \
    case 32: CALL(32); break;     \
    case 64: CALL(64); break;     \
    case 128: CALL(128); break;   \
    case 256: CALL(256); break;   \
    case 512: CALL(512); break;   \
    case 1024: CALL(1024); break; \
    case 2048: CALL(2048); break; \
    default: return fail(BTTB_ESIZE, "fast path: transform size is not a power of two"); \
  }

size_t fast_row_lds(int N, size_t esz, int G) {
  int bs = N + N / 8;
  if (bs < N + 2) bs = N + 2;
  return (size_t)G * bs * 2 * esz;
}

size_t fast_col_lds(int N, size_t esz, int G, bool fwd) {
  const size_t ex = (size_t)G * (N + N / 8) * 2 * esz;
  const size_t red = fwd ? (size_t)(G / 2) * N * 16 : 0;
  return ex > red ? ex : red;
}

template <typename T>
int fast_row_r2c(const T* in, long long in_bs, const T* scale, cx<T>* out, long long out_bs, int L, int nrows,
                 int ncols, int ld, int N, int G, const cx<T>* tw, int batch, hipStream_t s) {
  FRowArgs<T> a{in, in_bs, scale, out, out_bs, 0, 1, L, nrows, ncols, ld, N / 2 + 1, G, ceil_div(nrows, 2 * G), tw};
  dim3 grid(L * a.tiles, batch), block(G * (N / 8));
  const size_t sh = fast_row_lds(N, sizeof(T), G);
#define BTTB_L(NN) hipLaunchKernelGGL((k_frow_r2c<T, NN>), grid, block, sh, s, a)
  BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  BTTB_LAUNCHED("k_frow_r2c");
  return BTTB_OK;
}

template <typename T>
int fast_row_c2r(const cx<T>* in, long long in_bs, long long in_cs, int nsum, T* out, long long out_bs,
                 const T* scale, int L, int nrows, int ncols, int ld, int N, int G, const cx<T>* tw, int batch,
                 hipStream_t s) {
  FRowArgs<T> a{reinterpret_cast<const T*>(in), in_bs, scale, reinterpret_cast<cx<T>*>(out), out_bs, in_cs,
                nsum, L, nrows, ncols, ld, N / 2 + 1, G, ceil_div(nrows, 2 * G), tw};
  dim3 grid(L * a.tiles, batch), block(G * (N / 8));
  const size_t sh = fast_row_lds(N, sizeof(T), G);
#define BTTB_L(NN) hipLaunchKernelGGL((k_frow_c2r<T, NN>), grid, block, sh, s, a)
  BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  BTTB_LAUNCHED("k_frow_c2r");
  return BTTB_OK;
}

template <typename T>
int fast_col(bool fwd, const cx<T>* in, long long in_bs, const cx<T>* eig, cx<T>* out, long long out_bs, int L,
             int nin, int nout, int ldin, int ldout, int K2, int N, int G, const cx<T>* tw, int batch,
             hipStream_t s) {
  FColArgs<T> a{in, in_bs, eig, out, out_bs, L, nin, nout, ldin, ldout, K2, G, tw};
  dim3 grid(K2, batch), block(G * (N / 8));
  const size_t sh = fast_col_lds(N, sizeof(T), G, fwd);
  if (fwd) {
#define BTTB_L(NN) hipLaunchKernelGGL((k_fcol_fwd<T, NN>), grid, block, sh, s, a)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
    BTTB_LAUNCHED("k_fcol_fwd");
  } else {
#define BTTB_L(NN) hipLaunchKernelGGL((k_fcol_adj<T, NN>), grid, block, sh, s, a)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
    BTTB_LAUNCHED("k_fcol_adj");
  }
  return BTTB_OK;
}

template int fast_row_r2c<float>(const float*, long long, const float*, cx<float>*, long long, int, int, int, int,
                                 int, int, const cx<float>*, int, hipStream_t);
template int fast_row_r2c<double>(const double*, long long, const double*, cx<double>*, long long, int, int, int,
                                  int, int, int, const cx<double>*, int, hipStream_t);
template int fast_row_c2r<float>(const cx<float>*, long long, long long, int, float*, long long, const float*, int,
                                 int, int, int, int, int, const cx<float>*, int, hipStream_t);
template int fast_row_c2r<double>(const cx<double>*, long long, long long, int, double*, long long, const double*,
                                  int, int, int, int, int, int, const cx<double>*, int, hipStream_t);
template int fast_col<float>(bool, const cx<float>*, long long, const cx<float>*, cx<float>*, long long, int, int,
                             int, int, int, int, int, int, const cx<float>*, int, hipStream_t);
template int fast_col<double>(bool, const cx<double>*, long long, const cx<double>*, cx<double>*, long long, int,
                              int, int, int, int, int, int, int, const cx<double>*, int, hipStream_t);

}  // namespace bttb
