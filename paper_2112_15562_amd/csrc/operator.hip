// BTTB operator products on gfx950 (Sec. 2.7.1 of the paper).
//
// Forward, y = W_d . sum_r IFFT2(L_r . FFT2(pad(winv . x_r)))[0:sx, 0:sy]:
//   F1 k_row_r2c  : per layer row, scale by winv, zero-pad to Py, real-to-complex FFT
//                   along y (two real rows per complex transform); writes the half
//                   spectrum column-major U[l][k2][a].
//   F2 k_col_fwd  : per column k2, FFT along x of each layer's column (zero-padded to Px),
//                   multiply by the eigenvalues L_r and sum over the layers of a chunk
//                   (FP64 accumulator), inverse FFT along x; keeps rows p < sx: V[c][k2][p].
//   F3 k_row_c2r  : sums the chunk partials, complex-to-real inverse FFT along y of two
//                   rows at a time, keeps q < sy, scales by W_d.
// Transpose, z_r = winv . IFFT2(conj(L_r) . FFT2(pad(W_d . r)))[0:nx, 0:ny]:
//   T1 k_row_r2c  : as F1 on the single data array, scaled by W_d.
//   T2 k_col_adj  : per column k2, FFT along x once, then per layer conj(L_r) times it and
//                   the inverse FFT along x; keeps rows a < nx.
//   T3 k_row_c2r  : per layer row, inverse FFT along y, keeps b < ny, scales by winv.
// The 1/(Px Py) of the inverse transform is folded into the stored eigenvalues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "fft_reg.h"
#include "group.h"

namespace bttb {

// ------------------------------------------------------------------------------------
// Host helpers
// ------------------------------------------------------------------------------------
static bool smooth5(int m) {
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

int padded_size(int L) {
  int m = ceil_div(std::max(L, 1), 8);
  while (!smooth5(m)) ++m;
  return 8 * m;
}

// Relative cost of one point of a transform of size N in the register-layout kernels (products
// and groups): 1 for a power of two; for the 5-smooth sizes of the group kernels, more with every
// pass through LDS and when the last pass cannot run in registers.  The constants reproduce
// which of a 5-smooth size P and the next power of two gives the faster joint products for
// n = P / 2 at every size from 216 to 640 points (group products of both operators, FP32):
// 1.8 for one LDS pass with a register last pass, 2.1-2.5 for two.
static double transform_cost(int N) {
  if ((N & (N - 1)) == 0) return 1.0;
  const MixPlan p = mix_plan(N);
  const int last = p.radix[p.npass - 1];
  const bool reg = last == 2 || last == 4 || last == 8;
  const int lds = p.npass - 1 - (reg ? 1 : 0);
  return 1.5 + 0.3 * lds + (reg ? 0.0 : 0.4);
}

// The size of BTTB_PAD_AUTO for a circle of L points whose stations and prisms span at most n of
// them: among the next power of two >= L (at least 32) and the 5-smooth sizes in between that have
// group kernels and hold n in their first half, the one with the least N sqrt(cost(N)), i.e. the
// least estimated cost when both axes take it (N^2 points).
int auto_size(int L, int n) {
  int p2 = 32;
  while (p2 < L) p2 <<= 1;
  int best = p2;
  double best_cost = (double)p2;
  for (int N = 8 * ceil_div(L, 8); N < p2; N += 8) {  // every candidate below the power of two
    if (!mixed_size(N) || 2 * n > N) continue;
    const double c = N * std::sqrt(transform_cost(N));
    if (c < best_cost) {
      best_cost = c;
      best = N;
    }
  }
  return best;
}

FFTDesc make_fft_desc(int N) {
  FFTDesc d{};
  d.N = N;
  int n = N;
  auto push = [&](int r) { d.radix[d.npass++] = r; n /= r; };
  while (n % 8 == 0) push(8);
  while (n % 4 == 0) push(4);
  while (n % 2 == 0) push(2);
  while (n % 5 == 0) push(5);
  while (n % 3 == 0) push(3);
  return d;
}

void twiddles_fp64(int N, double* re_im) {
  // exp(-2 pi i e / N); the angle is reduced to [0, pi/4] by the octant symmetries of
  // sin and cos and evaluated in long double, so every entry is accurate to < 1 ulp.
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int e = 0; e < N; ++e) {
    // angle = 2 pi e / N = (pi/4) * (8 e / N); split 8e = q N + rem
    long long num = 8LL * e;
    long long q = num / N;
    long long rem = num - q * N;  // angle = (pi/4) (q + rem/N)
    long double f = (long double)rem / (long double)N;  // in [0, 1)
    long double c, s;
    // within the octant q, write the angle as q*pi/4 + f*pi/4
    long double a = f * pi / 4.0L;
    long double ca = cosl(a), sa = sinl(a);
    long double ca2 = cosl(pi / 4.0L - a), sa2 = sinl(pi / 4.0L - a);
    switch (q & 7) {
      case 0: c = ca; s = sa; break;
      case 1: c = sa2; s = ca2; break;
      case 2: c = -sa; s = ca; break;
      case 3: c = -ca2; s = sa2; break;
      case 4: c = -ca; s = -sa; break;
      case 5: c = -sa2; s = -ca2; break;
      case 6: c = sa; s = -ca; break;
      default: c = ca2; s = -sa2; break;
    }
    re_im[2 * e] = (double)c;
    re_im[2 * e + 1] = (double)(-s);
  }
}

// ------------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------------
template <typename T>
struct RowR2CArgs {
  const T* in;
  long long in_bs;
  const T* scale;  // nullable, [L][nrows][ncols], shared by the batch
  cx<T>* out;
  long long out_bs;
  int L, nrows, ncols, ld, K2, fpb, tiles;
  FFTDesc fd;
  const cx<T>* tw;
};

// Rows (2f, 2f+1) of the block's tile become z = x_a + i x_b; after the complex FFT,
// X_a[k] = (Z[k] + conj Z[N-k]) / 2 and X_b[k] = (Z[k] - conj Z[N-k]) / (2i), k <= N/2.
template <typename T>
__global__ void __launch_bounds__(1024) k_row_r2c(RowR2CArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int N = a.fd.N, TPF = N >> 3, stride = N + 2, K2 = a.K2;
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int l = blockIdx.x / a.tiles, tile = blockIdx.x - l * a.tiles;
  const int b = blockIdx.y;
  const int RT = 2 * a.fpb;
  const int r0 = tile * RT + 2 * f;
  cx<T>* z = smem + f * stride;
  const long long lofs = (long long)l * a.nrows * a.ncols;
  const T* src = a.in + b * a.in_bs + lofs;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  for (int n = t; n < N; n += TPF) {
    T xa = T(0), xb = T(0);
    if (n < a.ncols) {
      if (r0 < a.nrows) {
        xa = src[(long long)r0 * a.ncols + n];
        if (sc) xa *= sc[(long long)r0 * a.ncols + n];
      }
      if (r0 + 1 < a.nrows) {
        xb = src[(long long)(r0 + 1) * a.ncols + n];
        if (sc) xb *= sc[(long long)(r0 + 1) * a.ncols + n];
      }
    }
    z[n] = cx<T>{xa, xb};
  }
  __syncthreads();
  fft_lds<T, false>(z, a.fd, a.tw, t, TPF, true);
  constexpr int MU = 5;  // ceil((N/2+1) / (N/8))
  cx<T> va[MU], vb[MU];
  const T h = T(0.5);
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int k = t + u * TPF;
    if (k < K2) {
      cx<T> A = z[k];
      cx<T> C = z[k == 0 ? 0 : N - k];
      va[u] = cx<T>{h * (A.re + C.re), h * (A.im - C.im)};
      vb[u] = cx<T>{h * (A.im + C.im), h * (C.re - A.re)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int k = t + u * TPF;
    if (k < K2) {
      z[k] = va[u];
      z[K2 + k] = vb[u];
    }
  }
  __syncthreads();
  // rows beyond nrows are not stored: a tile may be taller than the padded row count ld
  cx<T>* dst = a.out + b * a.out_bs + (long long)l * K2 * a.ld + tile * RT;
  const int rows = min(RT, a.nrows - tile * RT);
  for (int idx = threadIdx.x; idx < K2 * RT; idx += blockDim.x) {
    const int k2 = idx / RT, rr = idx - k2 * RT;
    if (rr < rows) dst[(long long)k2 * a.ld + rr] = smem[(rr >> 1) * stride + (rr & 1) * K2 + k2];
  }
}

template <typename T>
struct RowC2RArgs {
  const cx<T>* in;
  long long in_bs, in_cs;
  int nsum;
  T* out;
  long long out_bs;
  const T* scale;  // nullable, [L][nrows_out][ncols_out]
  int L, nrows_out, ncols_out, ld, K2, fpb, tiles;
  FFTDesc fd;
  const cx<T>* tw;
};

// Half spectra H_a, H_b of rows (2f, 2f+1) (summed over `nsum` partials) become
// Z[k] = H_a[k] + i H_b[k] over the full circle (Hermitian extension); the inverse
// complex FFT then holds row a in its real and row b in its imaginary part.
template <typename T>
__global__ void __launch_bounds__(1024) k_row_c2r(RowC2RArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int N = a.fd.N, TPF = N >> 3, stride = N + 2, K2 = a.K2;
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int l = blockIdx.x / a.tiles, tile = blockIdx.x - l * a.tiles;
  const int b = blockIdx.y;
  const int RT = 2 * a.fpb;
  cx<T>* z = smem + f * stride;
  const cx<T>* src = a.in + b * a.in_bs + (long long)l * K2 * a.ld + tile * RT;
  for (int idx = threadIdx.x; idx < K2 * RT; idx += blockDim.x) {
    const int k2 = idx / RT, rr = idx - k2 * RT;
    const int row = tile * RT + rr;
    double hr = 0.0, hi = 0.0;
    if (row < a.nrows_out) {
      for (int c = 0; c < a.nsum; ++c) {
        cx<T> v = src[c * a.in_cs + (long long)k2 * a.ld + rr];
        hr += (double)v.re;
        hi += (double)v.im;
      }
    }
    if (k2 == 0 || k2 == K2 - 1) hi = 0.0;  // DC and Nyquist of a real row are real
    smem[(rr >> 1) * stride + (rr & 1) * K2 + k2] = cx<T>{(T)hr, (T)hi};
  }
  __syncthreads();
  constexpr int MU = 5;
  cx<T> ha[MU], hb[MU];
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int k = t + u * TPF;
    if (k < K2) {
      ha[u] = z[k];
      hb[u] = z[K2 + k];
    }
  }
  __syncthreads();
  const int half = N >> 1;
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int k = t + u * TPF;
    if (k < K2) {
      z[k] = cx<T>{ha[u].re - hb[u].im, ha[u].im + hb[u].re};
      if (k >= 1 && k < half) z[N - k] = cx<T>{ha[u].re + hb[u].im, hb[u].re - ha[u].im};
    }
  }
  __syncthreads();
  fft_lds<T, true>(z, a.fd, a.tw, t, TPF, true);
  const int r0 = tile * RT + 2 * f;
  const long long lofs = (long long)l * a.nrows_out * a.ncols_out;
  T* dst = a.out + b * a.out_bs + lofs;
  const T* sc = a.scale ? a.scale + lofs : nullptr;
  for (int q = t; q < a.ncols_out; q += TPF) {
    const cx<T> v = z[q];
    if (r0 < a.nrows_out) {
      const long long o = (long long)r0 * a.ncols_out + q;
      dst[o] = sc ? v.re * sc[o] : v.re;
    }
    if (r0 + 1 < a.nrows_out) {
      const long long o = (long long)(r0 + 1) * a.ncols_out + q;
      dst[o] = sc ? v.im * sc[o] : v.im;
    }
  }
}

template <typename T>
struct ColFwdArgs {
  const cx<T>* in;  // U [L][K2][ldin]
  long long in_bs;
  const cx<T>* eig;  // [L][K2][N], or with eig_even real [L][K2][N/2 + 1]
  cx<T>* out;        // V [chunk][K2][ldout]
  long long out_bs, out_cs;
  int L, nin, nout, ldin, ldout, K2, fpb, nchunk;
  FFTDesc fd;
  const cx<T>* tw;
  int eig_even;
};

// Eigenvalue k1 of the stored column (l, k2): complex, or from the real store of a symmetric
// operator (lambda[N - k] = lambda[k], real).
template <typename T>
__device__ __forceinline__ cx<T> eig_value(const cx<T>* eig, int even, int K2, int N, int l, int k2, int k1) {
  if (even) {
    const T* er = reinterpret_cast<const T*>(eig) + ((long long)l * K2 + k2) * (N / 2 + 1);
    return cx<T>{er[k1 <= N / 2 ? k1 : N - k1], T(0)};
  }
  return eig[((long long)l * K2 + k2) * N + k1];
}

template <typename T>
__global__ void __launch_bounds__(1024) k_col_fwd(ColFwdArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int N = a.fd.N, TPF = N >> 3, K2 = a.K2;
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int k2 = blockIdx.x * a.fpb + f;
  const bool valid = k2 < K2;
  const int c = blockIdx.y, b = blockIdx.z;
  const int l0 = (c * a.L) / a.nchunk, l1 = ((c + 1) * a.L) / a.nchunk;
  cx<T>* z = smem + f * N;
  double ar[8], ai[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) ar[i] = ai[i] = 0.0;
  const cx<T>* src = a.in + b * a.in_bs;
  for (int l = l0; l < l1; ++l) {
    const cx<T>* col = src + ((long long)l * K2 + k2) * a.ldin;
    for (int n = t; n < N; n += TPF) z[n] = (valid && n < a.nin) ? col[n] : cx<T>{T(0), T(0)};
    __syncthreads();
    fft_lds<T, false>(z, a.fd, a.tw, t, TPF, true);
    if (valid) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k1 = t + i * TPF;
        const cx<T> x = z[k1];
        const cx<T> w = eig_value(a.eig, a.eig_even, K2, N, l, k2, k1);
        const double xr = x.re, xi = x.im, wr = w.re, wi = w.im;
        ar[i] += wr * xr - wi * xi;
        ai[i] += wr * xi + wi * xr;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) z[t + i * TPF] = cx<T>{(T)ar[i], (T)ai[i]};
  __syncthreads();
  fft_lds<T, true>(z, a.fd, a.tw, t, TPF, true);
  if (valid) {
    cx<T>* dst = a.out + b * a.out_bs + c * a.out_cs + (long long)k2 * a.ldout;
    for (int p = t; p < a.ldout; p += TPF) dst[p] = p < a.nout ? z[p] : cx<T>{T(0), T(0)};
  }
}

template <typename T>
struct ColAdjArgs {
  const cx<T>* in;  // [K2][ldin]
  long long in_bs;
  const cx<T>* eig;  // as ColFwdArgs::eig
  cx<T>* out;  // [L][K2][ldout]
  long long out_bs;
  int L, nin, nout, ldin, ldout, K2, fpb, nchunk;
  FFTDesc fd;
  const cx<T>* tw;
  int eig_even;
};

template <typename T>
__global__ void __launch_bounds__(1024) k_col_adj(ColAdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int N = a.fd.N, TPF = N >> 3, K2 = a.K2;
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int k2 = blockIdx.x * a.fpb + f;
  const bool valid = k2 < K2;
  const int c = blockIdx.y, b = blockIdx.z;
  const int l0 = (c * a.L) / a.nchunk, l1 = ((c + 1) * a.L) / a.nchunk;
  cx<T>* z = smem + f * N;
  const cx<T>* col = a.in + b * a.in_bs + (long long)k2 * a.ldin;
  for (int n = t; n < N; n += TPF) z[n] = (valid && n < a.nin) ? col[n] : cx<T>{T(0), T(0)};
  __syncthreads();
  fft_lds<T, false>(z, a.fd, a.tw, t, TPF, true);
  cx<T> R[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) R[i] = z[t + i * TPF];
  __syncthreads();
  for (int l = l0; l < l1; ++l) {
    if (valid) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k1 = t + i * TPF;
        z[k1] = cmulc(R[i], eig_value(a.eig, a.eig_even, K2, N, l, k2, k1));
      }
    }
    __syncthreads();
    fft_lds<T, true>(z, a.fd, a.tw, t, TPF, true);
    if (valid) {
      cx<T>* dst = a.out + b * a.out_bs + ((long long)l * K2 + k2) * a.ldout;
      for (int p = t; p < a.ldout; p += TPF) dst[p] = p < a.nout ? z[p] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
  }
}

// Setup: kernel array -> Px x Py circle, C[r][u mod Px][v mod Py] = T[r][u+nx-1][v+ny-1].
__global__ void k_scatter(const double* __restrict__ T, double* __restrict__ C, int nz, int Lx, int Ly,
                          int nx, int ny, int Px, int Py) {
  const long long total = (long long)nz * Lx * Ly;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx % Ly);
    const long long rest = idx / Ly;
    const int i = (int)(rest % Lx);
    const int r = (int)(rest / Lx);
    int u = i - (nx - 1), v = j - (ny - 1);
    if (u < 0) u += Px;
    if (v < 0) v += Py;
    C[((long long)r * Px + u) * Py + v] = T[idx];
  }
}

// Setup: column FFT of each layer's row spectrum -> eigenvalues [L][K2][Px] * scale.
template <typename TO>
__global__ void __launch_bounds__(1024) k_col_setup(const cx<double>* in, int ldin, TO* eig, int L, int K2,
                                                    int fpb, FFTDesc fd, const cx<double>* tw, double scale) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<double>* smem = reinterpret_cast<cx<double>*>(smem_raw);
  const int N = fd.N, TPF = N >> 3;
  const int f = threadIdx.x / TPF, t = threadIdx.x - f * TPF;
  const int k2 = blockIdx.x * fpb + f;
  const bool valid = k2 < K2;
  const int l = blockIdx.y;
  cx<double>* z = smem + f * N;
  const cx<double>* col = in + ((long long)l * K2 + k2) * ldin;
  for (int n = t; n < N; n += TPF) z[n] = valid ? col[n] : cx<double>{0.0, 0.0};
  __syncthreads();
  fft_lds<double, false>(z, fd, tw, t, TPF, true);
  if (valid) {
    TO* dst = eig + 2 * ((long long)l * K2 + k2) * N;
    for (int k1 = t; k1 < N; k1 += TPF) {
      dst[2 * k1] = (TO)(z[k1].re * scale);
      dst[2 * k1 + 1] = (TO)(z[k1].im * scale);
    }
  }
}

// Symmetry test of the stored eigenvalues (complex [cols][N]): per column block, max |lambda|,
// max |Im lambda| and max |lambda[k] - lambda[N - k]|, written to part[3 col + 0..2].
template <typename T>
__global__ void __launch_bounds__(256) k_eig_symmetry(const T* eig, int N, double* part) {
  const long long col = blockIdx.x;
  const T* e = eig + 2 * col * N;
  double m[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const int km = k == 0 ? 0 : N - k;
    const double re = e[2 * k], im = e[2 * k + 1];
    const double dr = re - (double)e[2 * km], di = im - (double)e[2 * km + 1];
    m[0] = fmax(m[0], sqrt(re * re + im * im));
    m[1] = fmax(m[1], fabs(im));
    m[2] = fmax(m[2], sqrt(dr * dr + di * di));
  }
  __shared__ double sh[3][256];
  for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = m[k];
  __syncthreads();
  for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[3 * col + k] = sh[k][0];
}

// Real parts of lambda[0 .. N/2] of each column: the store of a symmetric operator.
template <typename T>
__global__ void __launch_bounds__(256) k_eig_compact(const T* eig, T* out, long long ncol, int N) {
  const int H = N / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < ncol * H;
       i += (long long)gridDim.x * blockDim.x) {
    const long long col = i / H;
    const int k = (int)(i - col * H);
    out[i] = eig[2 * (col * N + k)];
  }
}

// The complex eigenvalues [cols][N] of a real-even store.
template <typename T>
__global__ void __launch_bounds__(256) k_eig_expand(const T* er, T* out, long long ncol, int N) {
  const int H = N / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < ncol * N;
       i += (long long)gridDim.x * blockDim.x) {
    const long long col = i / N;
    const int k = (int)(i - col * N);
    out[2 * i] = er[col * H + (k <= N / 2 ? k : N - k)];
    out[2 * i + 1] = T(0);
  }
}

// A symmetric operator (kernel even in both lags, e.g. gravity with stations above the prism
// centres) has real eigenvalues, even along x: keep only Re lambda[0 .. Px/2] of each column,
// a quarter of the bytes the column passes stream.  Tested on the stored values: in FP32 to
// 1e-6 of max |lambda| (ten times the storage rounding); in FP64 to 1e-14, the transforms'
// own rounding, so that an FP64 plan changes by no more than that (the closed-form prism
// kernels are symmetric only to their evaluation noise, 1e-12 and more of max |lambda|,
// which FP64 plans keep).
template <typename T>
static int make_eig_even(Plan* P, hipStream_t s) {
  const long long ncol = (long long)P->nz * P->K2;
  const int N = P->Px;
  double* part = nullptr;
  if (hipMalloc(&part, (size_t)ncol * 3 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "bttb_setup: device allocation failed");
  }
  hipLaunchKernelGGL(k_eig_symmetry<T>, dim3((unsigned)ncol), dim3(256), 0, s, static_cast<const T*>(P->eig), N,
                     part);
  std::vector<double> h((size_t)ncol * 3);
  const bool ok = hipGetLastError() == hipSuccess &&
                  hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipStreamSynchronize(s) == hipSuccess;
  (void)hipFree(part);
  if (!ok) return fail(BTTB_EHIP, "bttb_setup: eigenvalue symmetry test");
  double mx = 0.0, mi = 0.0, ma = 0.0;
  for (long long c = 0; c < ncol; ++c) {
    mx = std::max(mx, h[3 * c]);
    mi = std::max(mi, h[3 * c + 1]);
    ma = std::max(ma, h[3 * c + 2]);
  }
  const double tol = (sizeof(T) == 8 ? 1e-14 : 1e-6) * mx;
  if (!(mx > 0.0) || mi > tol || ma > tol) return BTTB_OK;  // not symmetric: keep the complex store
  const size_t bytes = (size_t)ncol * (N / 2 + 1) * sizeof(T);
  void* er = nullptr;
  if (hipMalloc(&er, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "bttb_setup: device allocation failed");
  }
  hipLaunchKernelGGL(k_eig_compact<T>, dim3(1024), dim3(256), 0, s, static_cast<const T*>(P->eig),
                     static_cast<T*>(er), ncol, N);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(er);
    return fail(BTTB_EHIP, "bttb_setup: eigenvalue compaction");
  }
  (void)hipFree(P->eig);
  P->eig = er;
  P->eig_bytes = bytes;
  P->eig_even = 1;
  return BTTB_OK;
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
enum { KT_FWD_ROW = 0, KT_FWD_COL, KT_FWD_INV, KT_ADJ_ROW, KT_ADJ_COL, KT_ADJ_INV };

// Event pair around one kernel launch when timing is enabled (returns the slot or -1).
static int t_begin(Plan* P, int kid, hipStream_t s) {
  if (!P->t_ev || P->t_suspend > 0 || P->t_used >= P->t_cap) return -1;
  const int k = P->t_used++;
  P->t_kid[k] = kid;
  (void)hipEventRecord(P->t_ev[2 * k], s);
  return k;
}
static void t_end(Plan* P, int k, hipStream_t s) {
  if (k >= 0) (void)hipEventRecord(P->t_ev[2 * k + 1], s);
}
template <typename T>
static int launch_row_r2c(const T* in, long long in_bs, const T* scale, cx<T>* out, long long out_bs, int L,
                          int nrows, int ncols, int ld, int K2, int fpb, const FFTDesc& fd, const cx<T>* tw,
                          int batch, hipStream_t s) {
  RowR2CArgs<T> a{in, in_bs, scale, out, out_bs, L, nrows, ncols, ld, K2, fpb, ceil_div(nrows, 2 * fpb), fd, tw};
  const int TPF = fd.N / 8;
  dim3 grid(L * a.tiles, batch);
  const size_t sh = (size_t)fpb * (fd.N + 2) * sizeof(cx<T>);
  hipLaunchKernelGGL(k_row_r2c<T>, grid, dim3(fpb * TPF), sh, s, a);
  BTTB_LAUNCHED("k_row_r2c");
  return BTTB_OK;
}

template <typename T>
static int launch_row_c2r(const cx<T>* in, long long in_bs, long long in_cs, int nsum, T* out, long long out_bs,
                          const T* scale, int L, int nrows_out, int ncols_out, int ld, int K2, int fpb,
                          const FFTDesc& fd, const cx<T>* tw, int batch, hipStream_t s) {
  RowC2RArgs<T> a{in, in_bs, in_cs, nsum, out, out_bs, scale, L, nrows_out, ncols_out, ld, K2, fpb,
                  ceil_div(nrows_out, 2 * fpb), fd, tw};
  const int TPF = fd.N / 8;
  dim3 grid(L * a.tiles, batch);
  const size_t sh = (size_t)fpb * (fd.N + 2) * sizeof(cx<T>);
  hipLaunchKernelGGL(k_row_c2r<T>, grid, dim3(fpb * TPF), sh, s, a);
  BTTB_LAUNCHED("k_row_c2r");
  return BTTB_OK;
}

// Row groups per block for the single-array row kernels (the data array, sx rows):
// narrow blocks so that its few rows still spread over many compute units.
static int small_row_groups(const Plan* P, int nrows, int batch) {
  int g = P->row_fpb;
  while (g > 1 && ceil_div(nrows, 2 * g) * batch < 256) g >>= 1;
  return g;
}

template <typename T>
int apply_impl(Plan* P, int op, int batch, const T* in, long long in_stride, T* out, long long out_stride,
               const T* winv, const T* wd, hipStream_t s, void* scratch_U, void* scratch_V) {
  const cx<T>* eig = static_cast<const cx<T>*>(P->eig);
  const cx<T>* twx = static_cast<const cx<T>*>(P->twx);
  const cx<T>* twy = static_cast<const cx<T>*>(P->twy);
  cx<T>* U = static_cast<cx<T>*>(scratch_U ? scratch_U : P->U);
  cx<T>* V = static_cast<cx<T>*>(scratch_V ? scratch_V : P->V);
  const long long U_bs = (long long)P->nz * P->K2 * P->ldx;
  const long long V_cs = (long long)P->K2 * P->lds;
  const long long V_fcs = (long long)P->lds * P->ldk;  // power-of-two path: one row-major partial
  const long long V_bs = std::max((long long)P->nchunk_max * V_cs, (long long)P->nchunk_max * V_fcs);
  const int TPFx = P->Px / 8;
  // One stage: its kernel launch, bracketed by timing events when timing is on.
  auto stage = [&](int kid, auto&& launch) -> int {
    const int tk = t_begin(P, kid, s);
    const int n = tk >= 0 ? P->t_repeat : 1;
    for (int i = 0; i < n; ++i) {
      const int rc = launch();
      if (rc) return rc;
    }
    t_end(P, tk, s);
    return BTTB_OK;
  };
  for (int b0 = 0; b0 < batch; b0 += P->max_batch) {
    const int nb = std::min(P->max_batch, batch - b0);
    const T* x = in + b0 * in_stride;
    T* y = out + b0 * out_stride;
    int rc;
    if (P->fast) {
      const int gs = small_row_groups(P, P->sx, nb);
      if (op == BTTB_OP_FORWARD) {
        rc = stage(KT_FWD_ROW, [&]() -> int {
          return fast_row_r2c<T>(false, x, in_stride, winv, U, U_bs, P->nz, P->nx, P->ny, P->ldx, P->Py,
                                 P->row_fpb, twy, nb, s);
        });
        if (rc) return rc;
        rc = stage(KT_FWD_COL, [&]() -> int {
          return fast_col<T>(true, U, U_bs, eig, P->eig_even, V, V_bs, V_fcs, P->nz, P->nx, P->sx, P->ldx, P->ldk, P->K2, P->Px,
                             P->col_fpb, P->nchunk, twx, nb, s);
        });
        if (rc) return rc;
        rc = stage(KT_FWD_INV, [&]() -> int {
          return fast_row_c2r<T>(true, V, V_bs, V_fcs, P->nchunk, y, out_stride, wd, 1, P->sx, P->sy, P->ldk,
                                 P->Py, gs, twy, nb, s);
        });
        if (rc) return rc;
      } else {
        rc = stage(KT_ADJ_ROW, [&]() -> int {
          return fast_row_r2c<T>(true, x, in_stride, wd, V, V_bs, 1, P->sx, P->sy, P->ldk, P->Py, gs, twy, nb, s);
        });
        if (rc) return rc;
        rc = stage(KT_ADJ_COL, [&]() -> int {
          return fast_col<T>(false, V, V_bs, eig, P->eig_even, U, U_bs, 0, P->nz, P->sx, P->nx, P->ldk, P->ldx, P->K2, P->Px,
                             P->col_fpb, P->nchunk, twx, nb, s);
        });
        if (rc) return rc;
        rc = stage(KT_ADJ_INV, [&]() -> int {
          return fast_row_c2r<T>(false, U, U_bs, 0, 1, y, out_stride, winv, P->nz, P->nx, P->ny, P->ldx, P->Py,
                                 P->row_fpb, twy, nb, s);
        });
        if (rc) return rc;
      }
      continue;
    }
    if (op == BTTB_OP_FORWARD) {
      rc = stage(KT_FWD_ROW, [&]() -> int {
        return launch_row_r2c<T>(x, in_stride, winv, U, U_bs, P->nz, P->nx, P->ny, P->ldx, P->K2, P->row_fpb,
                                 P->fy, twy, nb, s);
      });
      if (rc) return rc;
      rc = stage(KT_FWD_COL, [&]() -> int {
        ColFwdArgs<T> a{U, U_bs, eig, V, V_bs, V_cs, P->nz, P->nx, P->sx, P->ldx, P->lds, P->K2, P->col_fpb,
                        P->nchunk, P->fx, twx, P->eig_even};
        dim3 grid(ceil_div(P->K2, P->col_fpb), P->nchunk, nb);
        hipLaunchKernelGGL(k_col_fwd<T>, grid, dim3(P->col_fpb * TPFx),
                           (size_t)P->col_fpb * P->Px * sizeof(cx<T>), s, a);
        BTTB_LAUNCHED("k_col_fwd");
        return BTTB_OK;
      });
      if (rc) return rc;
      rc = stage(KT_FWD_INV, [&]() -> int {
        return launch_row_c2r<T>(V, V_bs, V_cs, P->nchunk, y, out_stride, wd, 1, P->sx, P->sy, P->lds, P->K2,
                                 P->row_fpb, P->fy, twy, nb, s);
      });
      if (rc) return rc;
    } else {
      rc = stage(KT_ADJ_ROW, [&]() -> int {
        return launch_row_r2c<T>(x, in_stride, wd, V, V_bs, 1, P->sx, P->sy, P->lds, P->K2, P->row_fpb, P->fy,
                                 twy, nb, s);
      });
      if (rc) return rc;
      rc = stage(KT_ADJ_COL, [&]() -> int {
        ColAdjArgs<T> a{V, V_bs, eig, U, U_bs, P->nz, P->sx, P->nx, P->lds, P->ldx, P->K2, P->col_fpb,
                        P->nchunk, P->fx, twx, P->eig_even};
        dim3 grid(ceil_div(P->K2, P->col_fpb), P->nchunk, nb);
        hipLaunchKernelGGL(k_col_adj<T>, grid, dim3(P->col_fpb * TPFx),
                           (size_t)P->col_fpb * P->Px * sizeof(cx<T>), s, a);
        BTTB_LAUNCHED("k_col_adj");
        return BTTB_OK;
      });
      if (rc) return rc;
      rc = stage(KT_ADJ_INV, [&]() -> int {
        return launch_row_c2r<T>(U, U_bs, 0, 1, y, out_stride, winv, P->nz, P->nx, P->ny, P->ldx, P->K2,
                                 P->row_fpb, P->fy, twy, nb, s);
      });
      if (rc) return rc;
    }
  }
  return BTTB_OK;
}

template int apply_impl<float>(Plan*, int, int, const float*, long long, float*, long long, const float*,
                               const float*, hipStream_t, void*, void*);
template int apply_impl<double>(Plan*, int, int, const double*, long long, double*, long long, const double*,
                                const double*, hipStream_t, void*, void*);

size_t apply_scratch_bytes(const Plan* P, int batch) {
  const size_t elem = P->precision == BTTB_F64 ? 16 : 8;
  const size_t U_bs = (size_t)P->nz * P->K2 * P->ldx;
  const size_t V_one = std::max((size_t)P->K2 * P->lds, (size_t)P->lds * P->ldk);
  // batch members beyond the first start one full (nchunk_max) slot apart; the last holds nchunk
  return elem * ((size_t)(batch - 1) * (U_bs + (size_t)P->nchunk_max * V_one) + U_bs + (size_t)P->nchunk * V_one);
}

// ------------------------------------------------------------------------------------
// Launch shapes
// ------------------------------------------------------------------------------------
static constexpr size_t kMaxLds = 65536;

static bool row_fpb_ok(const Plan* P, int fpb) {
  if (fpb < 1 || fpb > 8 || (fpb & (fpb - 1))) return false;
  const size_t elem = P->precision == BTTB_F64 ? 16 : 8;
  if (P->fast) return fast_row_lds(P->Py, elem / 2, fpb) <= kMaxLds && fpb * (P->Py / 8) <= 512;
  if ((size_t)fpb * (P->Py + 2) * elem > kMaxLds) return false;
  return fpb * (P->Py / 8) <= 1024;
}

static bool col_fpb_ok(const Plan* P, int fpb) {
  if (fpb < 1) return false;
  const size_t elem = P->precision == BTTB_F64 ? 16 : 8;
  if (P->fast)
    return !(fpb & (fpb - 1)) && fast_col_lds(P->Px, elem / 2, fpb, true) <= kMaxLds &&
           fpb * (P->Px / 8) <= (P->precision == BTTB_F64 ? 256 : 512) && (P->Px <= 512 || fpb == 1);
  if ((size_t)fpb * P->Px * elem > kMaxLds) return false;
  return fpb * (P->Px / 8) <= 1024;
}

static void default_launch(Plan* P) {
  if (P->fast) {
    int rf = 8;
    while (rf > 1 && (!row_fpb_ok(P, rf) || rf * (P->Py / 8) > 512)) rf >>= 1;
    P->row_fpb = rf;
    // column jobs = Py/2; enough layer chunks for >= 256 blocks, up to 8 groups per block
    const int jobs = P->Py / 2;
    int nc = 1;
    while (jobs * nc * P->max_batch < 256 && nc * 2 <= std::min(P->nz, P->nchunk_max)) nc *= 2;
    P->nchunk = nc;
    int cf = 8;
    while (cf > 1 && (!col_fpb_ok(P, cf) || cf * nc > P->nz)) cf >>= 1;
    P->col_fpb = cf;
    return;
  }
  int rf = 8;
  while (rf > 1 && (!row_fpb_ok(P, rf) || rf * (P->Py / 8) > 512)) rf >>= 1;
  P->row_fpb = rf;
  int cf = std::max(1, 256 / (P->Px / 8));
  while (cf > 1 && !col_fpb_ok(P, cf)) --cf;
  P->col_fpb = cf;
  const int blocks = ceil_div(P->K2, cf) * P->max_batch;
  int nc = ceil_div(512, blocks);
  P->nchunk = std::max(1, std::min(std::min(nc, P->nz), P->nchunk_max));
}

}  // namespace bttb

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------
using namespace bttb;

extern "C" int bttb_setup(const double* kernels, int sx, int sy, int nx, int ny, int nz, int precision,
                          int max_batch, void* stream, bttb_plan* out) {
  if (!out) return fail(BTTB_EINVAL, "bttb_setup: out is NULL");
  *out = nullptr;
  if (!kernels || !aligned(kernels, 8)) return fail(BTTB_EINVAL, "bttb_setup: kernels NULL or misaligned");
  if (sx < 1 || sy < 1 || nx < 1 || ny < 1 || nz < 1 || max_batch < 1)
    return fail(BTTB_EINVAL, "bttb_setup: sizes must be >= 1");
  const bool pad_pow2 = (precision & BTTB_PAD_POW2) != 0;
  const bool pad_auto = (precision & BTTB_PAD_AUTO) != 0;
  const bool eig_full = (precision & BTTB_EIG_FULL) != 0;
  precision &= ~(BTTB_PAD_POW2 | BTTB_PAD_AUTO | BTTB_EIG_FULL);
  if (pad_pow2 && pad_auto) return fail(BTTB_EINVAL, "bttb_setup: BTTB_PAD_POW2 and BTTB_PAD_AUTO exclude each other");
  if (precision != BTTB_F64 && precision != BTTB_F32) return fail(BTTB_EINVAL, "bttb_setup: bad precision");
  const long long Lx = (long long)sx + nx - 1, Ly = (long long)sy + ny - 1;
  if (Lx > BTTB_MAX_TRANSFORM || Ly > BTTB_MAX_TRANSFORM)
    return fail(BTTB_ESIZE, "bttb_setup: sx+nx-1 or sy+ny-1 exceeds the maximum transform size");
  auto pow2_size = [](long long L) {
    int v = 32;
    while (v < L) v <<= 1;
    return v;
  };
  const int Px = pad_pow2 ? pow2_size(Lx) : pad_auto ? auto_size((int)Lx, std::max(sx, nx)) : padded_size((int)Lx);
  const int Py = pad_pow2 ? pow2_size(Ly) : pad_auto ? auto_size((int)Ly, std::max(sy, ny)) : padded_size((int)Ly);
  if (Px > BTTB_MAX_TRANSFORM || Py > BTTB_MAX_TRANSFORM)
    return fail(BTTB_ESIZE, "bttb_setup: padded transform size exceeds the maximum");
  hipStream_t s = static_cast<hipStream_t>(stream);

  Plan* P = new (std::nothrow) Plan{};
  if (!P) return fail(BTTB_ENOMEM, "bttb_setup: host allocation failed");
  P->sx = sx; P->sy = sy; P->nx = nx; P->ny = ny; P->nz = nz;
  P->Px = Px; P->Py = Py; P->K2 = Py / 2 + 1;
  P->ldx = round_up(nx, 16);
  P->lds = round_up(sx, 16);
  P->ldk = round_up(Py / 2 + 1, 8);
  P->precision = precision;
  P->max_batch = max_batch;
  P->nchunk_max = std::min(nz, 16);
  P->fx = make_fft_desc(Px);
  P->fy = make_fft_desc(Py);
  P->fast = !(Px & (Px - 1)) && !(Py & (Py - 1));
  default_launch(P);
  const size_t elem = precision == BTTB_F64 ? 16 : 8;  // complex element
  P->eig_bytes = (size_t)nz * P->K2 * Px * elem;
  const size_t Ub = (size_t)max_batch * nz * P->K2 * P->ldx * elem;
  const size_t Vb =
      (size_t)max_batch * P->nchunk_max * std::max((size_t)P->K2 * P->lds, (size_t)P->lds * P->ldk) * elem;
  P->scratch_bytes = Ub + Vb;

  auto cleanup = [&](int rc) {
    dfree(P->eig); dfree(P->twx); dfree(P->twy); dfree(P->U); dfree(P->V);
    delete P;
    return rc;
  };
  if (hipMalloc(&P->eig, P->eig_bytes) != hipSuccess || hipMalloc(&P->twx, Px * elem) != hipSuccess ||
      hipMalloc(&P->twy, Py * elem) != hipSuccess || hipMalloc(&P->U, Ub) != hipSuccess ||
      hipMalloc(&P->V, Vb) != hipSuccess) {
    (void)hipGetLastError();
    return cleanup(fail(BTTB_ENOMEM, "bttb_setup: device allocation failed"));
  }
  // twiddles: FP64 tables for the setup transform; the plan's own in its type
  std::vector<double> tx(2 * Px), ty(2 * Py);
  twiddles_fp64(Px, tx.data());
  twiddles_fp64(Py, ty.data());
  void *twx64 = nullptr, *twy64 = nullptr, *C = nullptr, *W = nullptr;
  auto cleanup_tmp = [&]() { dfree(twx64); dfree(twy64); dfree(C); dfree(W); };
  int rc = BTTB_OK;
  do {
    if (hipMalloc(&twx64, Px * 16) != hipSuccess || hipMalloc(&twy64, Py * 16) != hipSuccess) {
      rc = fail(BTTB_ENOMEM, "bttb_setup: device allocation failed"); break;
    }
    if (hipMemcpy(twx64, tx.data(), Px * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(twy64, ty.data(), Py * 16, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(BTTB_EHIP, "bttb_setup: twiddle upload failed"); break;
    }
    if (precision == BTTB_F64) {
      if (hipMemcpy(P->twx, tx.data(), Px * 16, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(P->twy, ty.data(), Py * 16, hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(BTTB_EHIP, "bttb_setup: twiddle upload failed"); break;
      }
    } else {
      std::vector<float> fx(2 * Px), fy(2 * Py);
      for (int i = 0; i < 2 * Px; ++i) fx[i] = (float)tx[i];
      for (int i = 0; i < 2 * Py; ++i) fy[i] = (float)ty[i];
      if (hipMemcpy(P->twx, fx.data(), Px * 8, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(P->twy, fy.data(), Py * 8, hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(BTTB_EHIP, "bttb_setup: twiddle upload failed"); break;
      }
    }
    const int K2 = P->K2;
    const int ldP = round_up(Px, 16);
    const size_t Cb = (size_t)nz * Px * Py * 8;
    const size_t Wb = (size_t)nz * K2 * ldP * 16;
    if (hipMalloc(&C, Cb) != hipSuccess || hipMalloc(&W, Wb) != hipSuccess) {
      rc = fail(BTTB_ENOMEM, "bttb_setup: device allocation failed"); break;
    }
    if (hipMemsetAsync(C, 0, Cb, s) != hipSuccess) { rc = fail(BTTB_EHIP, "bttb_setup: memset"); break; }
    const long long total = (long long)nz * Lx * Ly;
    const int blocks = (int)std::min<long long>(ceil_div((int)std::min<long long>(total, 1LL << 30), 256), 65535);
    hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, kernels, static_cast<double*>(C), nz, (int)Lx,
                       (int)Ly, nx, ny, Px, Py);
    if (hipGetLastError() != hipSuccess) { rc = fail(BTTB_EHIP, "bttb_setup: k_scatter launch"); break; }
    // row transform of all Px rows of each layer's circle (FP64)
    int rf = 8;
    while (rf > 1 && ((size_t)rf * (Py + 2) * 16 > kMaxLds || rf * (Py / 8) > 512)) rf >>= 1;
    rc = launch_row_r2c<double>(static_cast<const double*>(C), 0, nullptr, static_cast<cx<double>*>(W), 0, nz, Px,
                                Py, ldP, K2, rf, P->fy, static_cast<const cx<double>*>(twy64), 1, s);
    if (rc) break;
    int cf = std::max(1, 256 / (Px / 8));
    while (cf > 1 && (size_t)cf * Px * 16 > kMaxLds) --cf;
    dim3 grid(ceil_div(K2, cf), nz);
    const double scale = 1.0 / ((double)Px * (double)Py);
    if (precision == BTTB_F64)
      hipLaunchKernelGGL(k_col_setup<double>, grid, dim3(cf * (Px / 8)), (size_t)cf * Px * 16, s,
                         static_cast<const cx<double>*>(W), ldP, static_cast<double*>(P->eig), nz, K2, cf, P->fx,
                         static_cast<const cx<double>*>(twx64), scale);
    else
      hipLaunchKernelGGL(k_col_setup<float>, grid, dim3(cf * (Px / 8)), (size_t)cf * Px * 16, s,
                         static_cast<const cx<double>*>(W), ldP, static_cast<float*>(P->eig), nz, K2, cf, P->fx,
                         static_cast<const cx<double>*>(twx64), scale);
    if (hipGetLastError() != hipSuccess) { rc = fail(BTTB_EHIP, "bttb_setup: k_col_setup launch"); break; }
    if (hipStreamSynchronize(s) != hipSuccess) { rc = fail(BTTB_EHIP, "bttb_setup: synchronize"); break; }
    if (!eig_full) rc = precision == BTTB_F64 ? make_eig_even<double>(P, s) : make_eig_even<float>(P, s);
  } while (false);
  cleanup_tmp();
  if (rc != BTTB_OK) return cleanup(rc);
  *out = reinterpret_cast<bttb_plan>(P);
  return BTTB_OK;
}

static inline Plan* as_plan(bttb_plan p) { return reinterpret_cast<Plan*>(p); }

extern "C" int bttb_apply(bttb_plan plan, int op, int batch, const void* in, long long in_stride, void* out,
                          long long out_stride, const void* winv, const void* wd, void* stream) {
  Plan* P = as_plan(plan);
  if (!P) return fail(BTTB_EINVAL, "bttb_apply: plan is NULL");
  if (op != BTTB_OP_FORWARD && op != BTTB_OP_ADJOINT) return fail(BTTB_EINVAL, "bttb_apply: bad op");
  if (batch < 1) return fail(BTTB_EINVAL, "bttb_apply: batch must be >= 1");
  const size_t es = P->precision == BTTB_F64 ? 8 : 4;
  if (!in || !out || !aligned(in, es) || !aligned(out, es) || (winv && !aligned(winv, es)) ||
      (wd && !aligned(wd, es)))
    return fail(BTTB_EINVAL, "bttb_apply: NULL or misaligned vector");
  const long long nmod = (long long)P->nx * P->ny * P->nz, ndat = (long long)P->sx * P->sy;
  const long long nin = op == BTTB_OP_FORWARD ? nmod : ndat, nout = op == BTTB_OP_FORWARD ? ndat : nmod;
  if (batch > 1 && (in_stride < nin || out_stride < nout))
    return fail(BTTB_EINVAL, "bttb_apply: batch stride smaller than one member");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (P->precision == BTTB_F64)
    return apply_impl<double>(P, op, batch, static_cast<const double*>(in), in_stride, static_cast<double*>(out),
                              out_stride, static_cast<const double*>(winv), static_cast<const double*>(wd), s);
  return apply_impl<float>(P, op, batch, static_cast<const float*>(in), in_stride, static_cast<float*>(out),
                           out_stride, static_cast<const float*>(winv), static_cast<const float*>(wd), s);
}

extern "C" int bttb_matvec(bttb_plan plan, const void* x, void* y, void* stream) {
  return bttb_apply(plan, BTTB_OP_FORWARD, 1, x, 0, y, 0, nullptr, nullptr, stream);
}

extern "C" int bttb_rmatvec(bttb_plan plan, const void* r, void* z, void* stream) {
  return bttb_apply(plan, BTTB_OP_ADJOINT, 1, r, 0, z, 0, nullptr, nullptr, stream);
}

extern "C" int bttb_set_launch(bttb_plan plan, int col_fpb, int row_fpb, int layer_chunks) {
  Plan* P = as_plan(plan);
  if (!P) return fail(BTTB_EINVAL, "bttb_set_launch: plan is NULL");
  if (col_fpb > 0 && !col_fpb_ok(P, col_fpb)) return fail(BTTB_EINVAL, "bttb_set_launch: column FFTs per block");
  if (row_fpb > 0 && !row_fpb_ok(P, row_fpb)) return fail(BTTB_EINVAL, "bttb_set_launch: row FFTs per block");
  if (layer_chunks > 0 && layer_chunks > std::min(P->nchunk_max, P->nz))
    return fail(BTTB_EINVAL, "bttb_set_launch: layer chunks out of range");
  if (col_fpb > 0) P->col_fpb = col_fpb;
  if (row_fpb > 0) P->row_fpb = row_fpb;
  if (layer_chunks > 0) P->nchunk = layer_chunks;
  return BTTB_OK;
}

extern "C" int bttb_plan_info(bttb_plan plan, bttb_plan_desc* out) {
  Plan* P = as_plan(plan);
  if (!P || !out) return fail(BTTB_EINVAL, "bttb_plan_info: NULL argument");
  out->sx = P->sx; out->sy = P->sy; out->nx = P->nx; out->ny = P->ny; out->nz = P->nz;
  out->Px = P->Px; out->Py = P->Py; out->precision = P->precision; out->max_batch = P->max_batch;
  out->eig_bytes = P->eig_bytes; out->scratch_bytes = P->scratch_bytes;
  out->col_fft_per_block = P->col_fpb; out->row_fft_per_block = P->row_fpb; out->layer_chunks = P->nchunk;
  out->eig_real_even = P->eig_even;
  return BTTB_OK;
}

extern "C" int bttb_plan_eigenvalues(bttb_plan plan, void* out, void* stream) {
  Plan* P = as_plan(plan);
  if (!P || !out) return fail(BTTB_EINVAL, "bttb_plan_eigenvalues: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!P->eig_even) {
    BTTB_HIP(hipMemcpyAsync(out, P->eig, P->eig_bytes, hipMemcpyDeviceToDevice, s));
    return BTTB_OK;
  }
  const long long ncol = (long long)P->nz * P->K2;
  if (P->precision == BTTB_F64)
    hipLaunchKernelGGL(k_eig_expand<double>, dim3(1024), dim3(256), 0, s, static_cast<const double*>(P->eig),
                       static_cast<double*>(out), ncol, P->Px);
  else
    hipLaunchKernelGGL(k_eig_expand<float>, dim3(1024), dim3(256), 0, s, static_cast<const float*>(P->eig),
                       static_cast<float*>(out), ncol, P->Px);
  BTTB_LAUNCHED("k_eig_expand");
  return BTTB_OK;
}

static void timing_free(Plan* P) {
  if (P->t_ev) {
    for (int i = 0; i < 2 * P->t_cap; ++i)
      if (P->t_ev[i]) (void)hipEventDestroy(P->t_ev[i]);
    delete[] P->t_ev;
    delete[] P->t_kid;
  }
  P->t_ev = nullptr;
  P->t_kid = nullptr;
  P->t_cap = P->t_used = 0;
}

extern "C" int bttb_timing_enable(bttb_plan plan, int max_launches, int repeat) {
  Plan* P = as_plan(plan);
  if (!P || max_launches < 0 || repeat < 1 || repeat > 1000)
    return fail(BTTB_EINVAL, "bttb_timing_enable: bad argument");
  timing_free(P);
  P->t_repeat = repeat;
  if (max_launches == 0) return BTTB_OK;
  P->t_ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches]();
  P->t_kid = new (std::nothrow) int[max_launches];
  if (!P->t_ev || !P->t_kid) {
    delete[] P->t_ev;
    delete[] P->t_kid;
    P->t_ev = nullptr;
    P->t_kid = nullptr;
    return fail(BTTB_ENOMEM, "bttb_timing_enable: host allocation failed");
  }
  P->t_cap = max_launches;
  for (int i = 0; i < 2 * max_launches; ++i) {
    if (hipEventCreate(&P->t_ev[i]) != hipSuccess) {
      timing_free(P);
      return fail(BTTB_EHIP, "bttb_timing_enable: hipEventCreate");
    }
  }
  return BTTB_OK;
}

extern "C" int bttb_timing_read(bttb_plan plan, double* total_ms, int* count) {
  Plan* P = as_plan(plan);
  if (!P || !total_ms || !count) return fail(BTTB_EINVAL, "bttb_timing_read: NULL argument");
  for (int k = 0; k < BTTB_NKERNELS; ++k) {
    total_ms[k] = 0.0;
    count[k] = 0;
  }
  for (int i = 0; i < P->t_used; ++i) {
    BTTB_HIP(hipEventSynchronize(P->t_ev[2 * i + 1]));
    float ms = 0.0f;
    BTTB_HIP(hipEventElapsedTime(&ms, P->t_ev[2 * i], P->t_ev[2 * i + 1]));
    total_ms[P->t_kid[i]] += ms;
    count[P->t_kid[i]] += P->t_repeat;
  }
  P->t_used = 0;
  return BTTB_OK;
}

extern "C" int bttb_destroy(bttb_plan plan) {
  Plan* P = as_plan(plan);
  if (!P) return BTTB_OK;
  timing_free(P);
  dfree(P->eig); dfree(P->twx); dfree(P->twy); dfree(P->U); dfree(P->V);
  delete P;
  return BTTB_OK;
}
