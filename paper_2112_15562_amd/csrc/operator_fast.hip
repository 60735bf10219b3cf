// Products for power-of-two transform sizes with the register-resident FFT (fft_reg.h):
// the launchers of the one-plan kernels whose bodies are in fast_kernels.h.
//
// Same passes and intermediate layouts as the general kernels in operator.hip, with three
// differences: (1) a transform's first pass reads global memory directly and its last pass
// feeds the eigenvalue multiply, the layer accumulation and the stores from registers;
// (2) the forward column pass gives each block one column job and splits the layers of its
// layer chunk over the block's groups, which reduce their accumulators in LDS before one
// inverse column transform per chunk; (3) exchanges inside a transform use a wave-level
// barrier when the transform fits in one wave.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "fast_kernels.h"

namespace bttb {

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
  const size_t ex = (size_t)G * (N + N / 8) * 2 * esz + (fwd ? 0 : (size_t)N * 2 * esz);
  const size_t red = fwd ? (size_t)(G / 2) * N * 16 : 0;
  return ex > red ? ex : red;
}

template <typename T>
int fast_row_r2c(bool rowout, const T* in, long long in_bs, const T* scale, cx<T>* out, long long out_bs, int L,
                 int nrows, int ncols, int ld, int N, int G, const cx<T>* tw, int batch, hipStream_t s) {
  FRowArgs<T> a{in, in_bs, scale, out, out_bs, 0, 1, L, nrows, ncols, ld, N / 2 + 1, G, ceil_div(nrows, 2 * G), tw};
  dim3 grid(L * a.tiles, batch), block(G * (N / 8));
  const size_t sh = fast_row_lds(N, sizeof(T), G);
  const Fuse<T> f0{};
  const bool half = 2 * ncols <= N;  // the upper half of each row is zero padding
  if (rowout) {
#define BTTB_L(NN)                                                                           \
  if (half) hipLaunchKernelGGL((k_frow_r2c<T, NN, true, FUSE_NONE, true>), grid, block, sh, s, a, f0); \
  else hipLaunchKernelGGL((k_frow_r2c<T, NN, true, FUSE_NONE, false>), grid, block, sh, s, a, f0)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  } else {
#define BTTB_L(NN)                                                                            \
  if (half) hipLaunchKernelGGL((k_frow_r2c<T, NN, false, FUSE_NONE, true>), grid, block, sh, s, a, f0); \
  else hipLaunchKernelGGL((k_frow_r2c<T, NN, false, FUSE_NONE, false>), grid, block, sh, s, a, f0)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  }
  BTTB_LAUNCHED("k_frow_r2c");
  return BTTB_OK;
}

template <typename T>
int fast_row_c2r(bool rowin, const cx<T>* in, long long in_bs, long long in_cs, int nsum, T* out, long long out_bs,
                 const T* scale, int L, int nrows, int ncols, int ld, int N, int G, const cx<T>* tw, int batch,
                 hipStream_t s) {
  FRowArgs<T> a{reinterpret_cast<const T*>(in), in_bs, scale, reinterpret_cast<cx<T>*>(out), out_bs, in_cs,
                nsum, L, nrows, ncols, ld, N / 2 + 1, G, ceil_div(nrows, 2 * G), tw};
  dim3 grid(L * a.tiles, batch), block(G * (N / 8));
  const size_t sh = fast_row_lds(N, sizeof(T), G);
  const Fuse<T> f0{};
  if (!rowin && nsum != 1) return fail(BTTB_EINVAL, "fast_row_c2r: column-major input takes no partial sums");
  const bool half = 2 * ncols <= N;  // the upper half of each output row is not stored
  if (rowin) {
#define BTTB_L(NN)                                                                           \
  if (half) hipLaunchKernelGGL((k_frow_c2r<T, NN, true, FUSE_NONE, true>), grid, block, sh, s, a, f0); \
  else hipLaunchKernelGGL((k_frow_c2r<T, NN, true, FUSE_NONE, false>), grid, block, sh, s, a, f0)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  } else {
#define BTTB_L(NN)                                                                            \
  if (half) hipLaunchKernelGGL((k_frow_c2r<T, NN, false, FUSE_NONE, true>), grid, block, sh, s, a, f0); \
  else hipLaunchKernelGGL((k_frow_c2r<T, NN, false, FUSE_NONE, false>), grid, block, sh, s, a, f0)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
  }
  BTTB_LAUNCHED("k_frow_c2r");
  return BTTB_OK;
}

template <typename T>
int fast_col(bool fwd, const cx<T>* in, long long in_bs, const cx<T>* eig, int eig_even, cx<T>* out, long long out_bs,
             long long out_cs, int L, int nin, int nout, int ldin, int ldout, int K2, int N, int G, int nchunk,
             const cx<T>* tw, int batch, hipStream_t s) {
  FColArgs<T> a{in, in_bs, eig, out, out_bs, out_cs, L, nin, nout, ldin, ldout, K2, G, nchunk, tw, eig_even};
  dim3 grid(K2, nchunk, batch), block(G * (N / 8));
  const size_t sh = fast_col_lds(N, sizeof(T), G, fwd);
  const bool half = 2 * nin <= N && 2 * nout <= N;  // zero-padded inputs, unstored outputs
  if (fwd) {
#define BTTB_L(NN)                                                                       \
  if (half) hipLaunchKernelGGL((k_fcol_fwd<T, NN, true>), grid, block, sh, s, a); \
  else hipLaunchKernelGGL((k_fcol_fwd<T, NN, false>), grid, block, sh, s, a)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
    BTTB_LAUNCHED("k_fcol_fwd");
  } else {
#define BTTB_L(NN)                                                                       \
  if (half) hipLaunchKernelGGL((k_fcol_adj<T, NN, true>), grid, block, sh, s, a); \
  else hipLaunchKernelGGL((k_fcol_adj<T, NN, false>), grid, block, sh, s, a)
    BTTB_POW2_SWITCH(N, BTTB_L)
#undef BTTB_L
    BTTB_LAUNCHED("k_fcol_adj");
  }
  return BTTB_OK;
}

template int fast_row_r2c<float>(bool, const float*, long long, const float*, cx<float>*, long long, int, int, int, int,
                                 int, int, const cx<float>*, int, hipStream_t);
template int fast_row_r2c<double>(bool, const double*, long long, const double*, cx<double>*, long long, int, int, int,
                                  int, int, int, const cx<double>*, int, hipStream_t);
template int fast_row_c2r<float>(bool, const cx<float>*, long long, long long, int, float*, long long, const float*, int,
                                 int, int, int, int, int, const cx<float>*, int, hipStream_t);
template int fast_row_c2r<double>(bool, const cx<double>*, long long, long long, int, double*, long long, const double*,
                                  int, int, int, int, int, int, const cx<double>*, int, hipStream_t);
template int fast_col<float>(bool, const cx<float>*, long long, const cx<float>*, int, cx<float>*, long long, long long,
                             int, int, int, int, int, int, int, int, int, const cx<float>*, int, hipStream_t);
template int fast_col<double>(bool, const cx<double>*, long long, const cx<double>*, int, cx<double>*, long long,
                              long long, int, int, int, int, int, int, int, int, int, const cx<double>*, int,
                              hipStream_t);

}  // namespace bttb
