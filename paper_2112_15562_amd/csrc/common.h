// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "bttb.h"
#include "fft_engine.h"

namespace bttb {

// Copy of a descriptor that stays constant for a launch (a table entry written by the host
// before it), at an address that is the same for the whole block: through the constant
// address space the compiler reads it with scalar loads once, into scalar registers,
// instead of one vector load per field at each use (whose waits would also wait for every
// load issued before them).
template <typename S>
__device__ __forceinline__ S launch_const(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "descriptor of whole words");
  S out;
#if __HIP_DEVICE_COMPILE__
  using W = const __attribute__((address_space(4))) unsigned int;
  W* src = (W*)p;
  unsigned int* dst = reinterpret_cast<unsigned int*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(S) / 4); ++k) dst[k] = src[k];
#else
  out = *p;  // (the host pass only parses device code)
#endif
  return out;
}

// A value that is the same in every lane, kept in a scalar register.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Records `msg` as the calling thread's last error and returns `status`.
int fail(int status, const std::string& msg);
// Maps a HIP error to BTTB_EHIP with a message naming `what`.
int hip_fail(hipError_t e, const char* what);

#define BTTB_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::bttb::hip_fail(e_, #call); \
  } while (0)

#define BTTB_LAUNCHED(what)                              \
  do {                                                   \
    hipError_t e_ = hipGetLastError();                   \
    if (e_ != hipSuccess) return ::bttb::hip_fail(e_, what); \
  } while (0)

inline void dfree(void* p) {
  if (p) (void)hipFree(p);
}
inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return ceil_div(a, b) * b; }

// Radix plan for a 1-D length N (a 5-smooth multiple of 8).
FFTDesc make_fft_desc(int N);
// Smallest 5-smooth multiple of 8 that is >= L.
int padded_size(int L);
// BTTB_PAD_AUTO's size for a circle of L points spanning at most n of them (operator.hip).
int auto_size(int L, int n);
// Host table exp(-2 pi i e / N), e < N, in FP64 (argument reduced by octant symmetry).
void twiddles_fp64(int N, double* re_im);

// One operator plan (Sec. 2.7.1): eigenvalues of every layer's BCCB embedding plus
// the scratch for one product of up to max_batch vectors.
struct Plan {
  int sx, sy, nx, ny, nz;
  int Px, Py, K2;   // K2 = Py/2 + 1 (half spectrum along y)
  int ldx, lds;     // padded row counts of the column-major intermediates (multiples of 16)
  int ldk;          // padded K2: row stride of the row-major data-array spectra (power-of-two path)
  int precision;
  int max_batch;
  // launch shape
  int col_fpb;      // column FFTs per block
  int row_fpb;      // row-pair FFTs per block
  int nchunk;       // layer chunks of the forward column pass (general path)
  int nchunk_max;
  bool fast;        // both transform sizes are powers of two: register-resident kernels
  FFTDesc fx, fy;
  void* eig;        // complex [nz][K2][Px] of the plan's type, scaled by 1/(Px Py); with
                    // eig_even: real [nz][K2][Px/2 + 1]
  int eig_even;     // the operator is symmetric: its eigenvalues are real and even along x
  void* twx;        // complex [Px] of the plan's type
  void* twy;        // complex [Py]
  void* U;          // complex [max_batch][nz][K2][ldx]
  void* V;          // complex [max_batch][nchunk_max][K2][lds]
  size_t eig_bytes, scratch_bytes;
  // optional per-kernel event timing
  int t_cap, t_used;
  int t_repeat;      // launches of each timed kernel between its two events
  int t_suspend;     // > 0 while kernels are being captured into a graph
  hipEvent_t* t_ev;  // [2 * t_cap]
  int* t_kid;        // [t_cap]
};

// Power-of-two path (operator_fast.hip).
size_t fast_row_lds(int N, size_t esz, int G);
size_t fast_col_lds(int N, size_t esz, int G, bool fwd);
template <typename T>
int fast_row_r2c(bool rowout, const T* in, long long in_bs, const T* scale, cx<T>* out, long long out_bs, int L, int nrows,
                 int ncols, int ld, int N, int G, const cx<T>* tw, int batch, hipStream_t s);
template <typename T>
int fast_row_c2r(bool rowin, const cx<T>* in, long long in_bs, long long in_cs, int nsum, T* out, long long out_bs,
                 const T* scale, int L, int nrows, int ncols, int ld, int N, int G, const cx<T>* tw, int batch,
                 hipStream_t s);
template <typename T>
int fast_col(bool fwd, const cx<T>* in, long long in_bs, const cx<T>* eig, int eig_even, cx<T>* out, long long out_bs,
             long long out_cs, int L, int nin, int nout, int ldin, int ldout, int K2, int N, int G, int nchunk,
             const cx<T>* tw, int batch, hipStream_t s);

// The products of one plan (bttb_apply).  scratch_U, scratch_V: where the row spectra and the
// data-side spectra go, or NULL for the plan's own scratch (apply_scratch_bytes: the bytes a
// call with `batch` members needs, U first and V right after it, at batch-stride offsets).
template <typename T>
int apply_impl(Plan* P, int op, int batch, const T* in, long long in_stride, T* out, long long out_stride,
               const T* winv, const T* wd, hipStream_t s, void* scratch_U = nullptr, void* scratch_V = nullptr);
size_t apply_scratch_bytes(const Plan* P, int batch);

}  // namespace bttb
