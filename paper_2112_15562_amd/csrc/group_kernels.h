// Kernels of the group products (group.hip): one launch per stage over the members of one
// transform size, each block finding its member in the launch's prefix table and running the
// register-layout kernel body of that size.  In a header so that the power-of-two sizes
// (group.hip) and the 5-smooth ones (group_mixed.hip) are compiled in separate units.
#pragma once
#include <hip/hip_runtime.h>

#include "fast_kernels.h"
#include "group.h"

namespace bttb {

template <typename T, int MODE>
__device__ __forceinline__ Fuse<T> member_fuse(const GLaunch<T>& g, int i) {
  if constexpr (MODE != FUSE_NONE) return launch_const(g.fz + i);
  return Fuse<T>{};
}

// Row transform R2C of transform size N.  ROWOUT = false: model rows into U (forward, first
// stage); ROWOUT = true: data rows into V (transpose, first stage).
template <typename T, int N, bool ROWOUT, int MODE, bool HALF>
__global__ void __launch_bounds__(512, (row_waves<T, N, MODE, HALF>())) k_grow_r2c(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int k = uniform(group_member(g.start, g.count, blockIdx.x));
  const int i = uniform(g.idx[k]);
  const GMember<T> M = launch_const(g.mem + i);
  const int local = blockIdx.x - g.start[k], nb = g.start[k + 1] - g.start[k];
  const int G = g.bt / Len<N>::LANES;  // transforms per block
  const T* in = launch_const(g.in + i);
  FRowArgs<T> a;
  if constexpr (!ROWOUT) {
    a = FRowArgs<T>{in, 0, g.winv ? launch_const(g.winv + i) : nullptr, M.U, 0, 0, 1, M.nz, M.nx, M.ny, M.ldx, M.K2, G,
                    (M.nx + 2 * G - 1) / (2 * G), M.twy};
  } else {
    a = FRowArgs<T>{in, 0, g.wd ? launch_const(g.wd + i) : nullptr, M.V, 0, 0, 1, 1, M.sx, M.sy, M.ldk, M.K2, G,
                    (M.sx + 2 * G - 1) / (2 * G), M.twy};
  }
  const Fuse<T> fz = member_fuse<T, MODE>(g, i);
  frow_r2c_body<T, N, ROWOUT, MODE, HALF>(a, fz, local, 0, local, nb, smem_raw);
}

// Inverse row transform C2R of size N.  ROWIN = true: data rows from V (forward, last
// stage, sums the layer-chunk partials); ROWIN = false: model rows from U (transpose, last).
template <typename T, int N, bool ROWIN, int MODE, bool HALF>
__global__ void __launch_bounds__(512, (c2r_waves<T, N, ROWIN, MODE, HALF>())) k_grow_c2r(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int k = uniform(group_member(g.start, g.count, blockIdx.x));
  const int i = uniform(g.idx[k]);
  const GMember<T> M = launch_const(g.mem + i);
  const int local = blockIdx.x - g.start[k], nb = g.start[k + 1] - g.start[k];
  const int G = g.bt / Len<N>::LANES;
  T* out = launch_const(g.out + i);
  FRowArgs<T> a;
  if constexpr (ROWIN) {
    a = FRowArgs<T>{reinterpret_cast<const T*>(M.V), 0, g.wd ? launch_const(g.wd + i) : nullptr, reinterpret_cast<cx<T>*>(out), 0,
                    M.V_fcs, M.nchunk, 1, M.sx, M.sy, M.ldk, M.K2, G, (M.sx + 2 * G - 1) / (2 * G), M.twy};
  } else {
    a = FRowArgs<T>{reinterpret_cast<const T*>(M.U), 0, g.winv ? launch_const(g.winv + i) : nullptr,
                    reinterpret_cast<cx<T>*>(out), 0, 0, 1, M.nz, M.nx, M.ny, M.ldx, M.K2, G,
                    (M.nx + 2 * G - 1) / (2 * G), M.twy};
  }
  const Fuse<T> fz = member_fuse<T, MODE>(g, i);
  frow_c2r_body<T, N, ROWIN, MODE, HALF>(a, fz, local, 0, local, nb, smem_raw);
}

// Column pass of size N: forward (eigenvalue multiply and layer sum into V partials) or
// transpose (conjugate eigenvalue multiply per layer into U).
template <typename T, int N, bool FWD, bool HALF>
__global__ void __launch_bounds__(col_threads(sizeof(T))) k_gcol(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int k = uniform(group_member(g.start, g.count, blockIdx.x));
  const int i = uniform(g.idx[k]);
  const GMember<T> M = launch_const(g.mem + i);
  const int local = blockIdx.x - g.start[k];
  const int jobs = M.K2;
  const int c = local / jobs, job = local - c * jobs;
  const int G = g.bt / Len<N>::LANES;
  if constexpr (FWD) {
    const FColArgs<T> a{M.U, 0, M.eig, M.V, 0, M.V_fcs, M.nz, M.nx, M.sx, M.ldx, M.ldk, M.K2, G, M.nchunk, M.twx,
                        M.eig_even};
    fcol_fwd_body<T, N, HALF>(a, job, c, 0, smem_raw);
  } else {
    const FColArgs<T> a{M.V, 0, M.eig, M.U, 0, 0, M.nz, M.sx, M.nx, M.ldk, M.ldx, M.K2, G, M.nchunk, M.twx,
                        M.eig_even};
    fcol_adj_body<T, N, HALF>(a, job, c, 0, smem_raw);
  }
}

// The kernel of stage st at transform size N (in the CG step's fused form when fused).
template <typename T, int N, bool H>
static auto stage_kernel_h(int st, bool fused) -> void (*)(GLaunch<T>) {
  switch (st) {
    case GS_F1: return fused ? k_grow_r2c<T, N, false, FUSE_DIR, H> : k_grow_r2c<T, N, false, FUSE_NONE, H>;
    case GS_F2: return k_gcol<T, N, true, H>;
    case GS_F3: return fused ? k_grow_c2r<T, N, true, FUSE_QQ, H> : k_grow_c2r<T, N, true, FUSE_NONE, H>;
    case GS_T1: return k_grow_r2c<T, N, true, FUSE_NONE, H>;
    case GS_T2: return k_gcol<T, N, false, H>;
    default: return fused ? k_grow_c2r<T, N, false, FUSE_GRAD, H> : k_grow_c2r<T, N, false, FUSE_NONE, H>;
  }
}
template <typename T, int N>
static auto stage_kernel(int st, bool fused, bool half) -> void (*)(GLaunch<T>) {
  return half ? stage_kernel_h<T, N, true>(st, fused) : stage_kernel_h<T, N, false>(st, fused);
}

}  // namespace bttb
