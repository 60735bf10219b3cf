// Group products: the forward or transpose products of many plans (members: the gravity
// and magnetic operators of many inversions, of uneven sizes) in one launch per stage.
//
// Each stage (row transform, column pass, inverse row transform; Sec. 2.7.1) is one
// launch over the concatenated blocks of all members.  A block finds its member in the
// launch's prefix table of first blocks, builds that member's stage arguments from the
// member table, and runs the register-FFT body for the member's transform size; every
// member uses its own plan's eigenvalues and scratch.  All blocks of a launch have the
// same thread count, so a member of transform size N runs (threads / (N / 8)) FFTs per
// block.  The per-call vectors come from device arrays of pointers, so a group product
// can be captured in a HIP graph and replayed with new data in the same buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "common.h"
#include "fast_kernels.h"
#include "group.h"

namespace bttb {

__device__ __forceinline__ int group_member(const int* start, int count, int blk) {
  int i = 0;
  while (i + 1 < count && blk >= start[i + 1]) ++i;
  return i;
}

// Sizes a group kernel is compiled for.
#define BTTB_GROUP_SWITCH(N, CALL) \
  switch (N) {                     \
    case 32: CALL(32); break;      \
    case 64: CALL(64); break;      \
    case 128: CALL(128); break;    \
    case 256: CALL(256); break;    \
    case 512: CALL(512); break;    \
    case 1024: CALL(1024); break;  \
    case 2048: CALL(2048); break;  \
    default: break;                \
  }

template <typename T>
__device__ __forceinline__ Fuse<T> member_fuse(const GLaunch<T>& g, int i) {
  if (g.fz) return g.fz[i];
  return Fuse<T>{};
}

// Row transform R2C.  ROWOUT = false: model rows into U (forward, first stage);
// ROWOUT = true: data rows into V (transpose, first stage).
template <typename T, bool ROWOUT, int MODE>
__global__ void __launch_bounds__(512) k_grow_r2c(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = group_member(g.start, g.count, blockIdx.x);
  const GMember<T>& M = g.mem[i];
  const int local = blockIdx.x - g.start[i], nb = g.start[i + 1] - g.start[i];
  const int G = g.bt / (M.Py / 8);
  const T* in = g.in[i];
  FRowArgs<T> a;
  if constexpr (!ROWOUT) {
    a = FRowArgs<T>{in, 0, g.winv ? g.winv[i] : nullptr, M.U, 0, 0, 1, M.nz, M.nx, M.ny, M.ldx, M.K2, G,
                    (M.nx + 2 * G - 1) / (2 * G), M.twy};
  } else {
    a = FRowArgs<T>{in, 0, g.wd ? g.wd[i] : nullptr, M.V, 0, 0, 1, 1, M.sx, M.sy, M.ldk, M.K2, G,
                    (M.sx + 2 * G - 1) / (2 * G), M.twy};
  }
  const Fuse<T> fz = member_fuse(g, i);
#define BTTB_B(NN) frow_r2c_body<T, NN, ROWOUT, MODE>(a, fz, local, 0, local, nb, smem_raw)
  BTTB_GROUP_SWITCH(M.Py, BTTB_B)
#undef BTTB_B
}

// Inverse row transform C2R.  ROWIN = true: data rows from V (forward, last stage, sums
// the layer-chunk partials); ROWIN = false: model rows from U (transpose, last stage).
template <typename T, bool ROWIN, int MODE>
__global__ void __launch_bounds__(512) k_grow_c2r(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = group_member(g.start, g.count, blockIdx.x);
  const GMember<T>& M = g.mem[i];
  const int local = blockIdx.x - g.start[i], nb = g.start[i + 1] - g.start[i];
  const int G = g.bt / (M.Py / 8);
  T* out = g.out[i];
  FRowArgs<T> a;
  if constexpr (ROWIN) {
    a = FRowArgs<T>{reinterpret_cast<const T*>(M.V), 0, g.wd ? g.wd[i] : nullptr, reinterpret_cast<cx<T>*>(out), 0,
                    M.V_fcs, M.nchunk, 1, M.sx, M.sy, M.ldk, M.K2, G, (M.sx + 2 * G - 1) / (2 * G), M.twy};
  } else {
    a = FRowArgs<T>{reinterpret_cast<const T*>(M.U), 0, g.winv ? g.winv[i] : nullptr,
                    reinterpret_cast<cx<T>*>(out), 0, 0, 1, M.nz, M.nx, M.ny, M.ldx, M.K2, G,
                    (M.nx + 2 * G - 1) / (2 * G), M.twy};
  }
  const Fuse<T> fz = member_fuse(g, i);
#define BTTB_B(NN) frow_c2r_body<T, NN, ROWIN, MODE>(a, fz, local, 0, local, nb, smem_raw)
  BTTB_GROUP_SWITCH(M.Py, BTTB_B)
#undef BTTB_B
}

// Column pass: forward (eigenvalue multiply and layer sum into V partials) or transpose
// (conjugate eigenvalue multiply per layer into U).
template <typename T, bool FWD>
__global__ void __launch_bounds__(col_threads(sizeof(T))) k_gcol(GLaunch<T> g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = group_member(g.start, g.count, blockIdx.x);
  const GMember<T>& M = g.mem[i];
  const int local = blockIdx.x - g.start[i];
  const int jobs = M.K2 - 1;
  const int c = local / jobs, job = local - c * jobs;
  const int G = g.bt / (M.Px / 8);
  FColArgs<T> a;
  if constexpr (FWD) {
    a = FColArgs<T>{M.U, 0, M.eig, M.V, 0, M.V_fcs, M.nz, M.nx, M.sx, M.ldx, M.ldk, M.K2, G, M.nchunk, M.twx};
  } else {
    a = FColArgs<T>{M.V, 0, M.eig, M.U, 0, 0, M.nz, M.sx, M.nx, M.ldk, M.ldx, M.K2, G, M.nchunk, M.twx};
  }
  if constexpr (FWD) {
#define BTTB_B(NN) fcol_fwd_body<T, NN>(a, job, c, 0, smem_raw)
    BTTB_GROUP_SWITCH(M.Px, BTTB_B)
#undef BTTB_B
  } else {
#define BTTB_B(NN) fcol_adj_body<T, NN>(a, job, c, 0, smem_raw)
    BTTB_GROUP_SWITCH(M.Px, BTTB_B)
#undef BTTB_B
  }
}

// ------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static int stage_threads(const Group* g, int st) {
  switch (st) {
    case GS_F1: case GS_T3: return g->bt_rm;
    case GS_F3: case GS_T1: return g->bt_rd;
    default: return g->bt_c;
  }
}

// Block counts and LDS of every stage for the current launch shape.
static int layout(Group* g) {
  const size_t esz = g->precision == BTTB_F64 ? 8 : 4;
  for (int st = 0; st < GS_COUNT; ++st) {
    g->start[st][0] = 0;
    g->lds[st] = 0;
  }
  for (int i = 0; i < g->count; ++i) {
    const Plan* P = g->P[i];
    const int tr = P->Py / 8, tc = P->Px / 8;
    const int Grm = g->bt_rm / tr, Grd = g->bt_rd / tr, Gc = g->bt_c / tc;
    if (Grm < 1 || Grd < 1 || Gc < 1) return fail(BTTB_EINVAL, "group: threads per block below one transform");
    const int nch = std::min(g->nchunk, std::min(P->nz, P->nchunk_max));
    g->nch[i] = nch;
    const long long b[GS_COUNT] = {
        (long long)P->nz * ceil_div(P->nx, 2 * Grm),  // F1
        (long long)(P->K2 - 1) * nch,                 // F2
        (long long)ceil_div(P->sx, 2 * Grd),          // F3
        (long long)ceil_div(P->sx, 2 * Grd),          // T1
        (long long)(P->K2 - 1) * nch,                 // T2
        (long long)P->nz * ceil_div(P->nx, 2 * Grm),  // T3
    };
    const size_t l[GS_COUNT] = {
        fast_row_lds(P->Py, esz, Grm), fast_col_lds(P->Px, esz, Gc, true), fast_row_lds(P->Py, esz, Grd),
        fast_row_lds(P->Py, esz, Grd), fast_col_lds(P->Px, esz, Gc, false), fast_row_lds(P->Py, esz, Grm)};
    for (int st = 0; st < GS_COUNT; ++st) {
      const long long nx = g->start[st][i] + b[st];
      if (nx > (1LL << 30)) return fail(BTTB_ESIZE, "group: too many blocks");
      g->start[st][i + 1] = (int)nx;
      g->lds[st] = std::max(g->lds[st], l[st]);
    }
  }
  for (int st = 0; st < GS_COUNT; ++st)
    if (g->lds[st] > 160 * 1024) return fail(BTTB_EINVAL, "group: launch shape needs more LDS than a CU has");
  return BTTB_OK;
}

template <typename T>
static int upload_members(Group* g, hipStream_t s) {
  GMember<T> h[GMAX];
  for (int i = 0; i < g->count; ++i) {
    const Plan* P = g->P[i];
    h[i] = GMember<T>{P->Px, P->Py, P->K2, P->sx, P->sy, P->nx, P->ny, P->nz, P->ldx, P->ldk, g->nch[i],
                      static_cast<const cx<T>*>(P->eig), static_cast<const cx<T>*>(P->twx),
                      static_cast<const cx<T>*>(P->twy), static_cast<cx<T>*>(P->U), static_cast<cx<T>*>(P->V),
                      (long long)P->lds * P->ldk};
  }
  BTTB_HIP(hipMemcpyAsync(g->mem, h, sizeof(GMember<T>) * g->count, hipMemcpyHostToDevice, s));
  BTTB_HIP(hipStreamSynchronize(s));
  return BTTB_OK;
}

static int check_threads(const Group* g, int rm, int rd, int c) {
  const int cmax = g->precision == BTTB_F64 ? 256 : 512;
  if (!pow2(rm) || !pow2(rd) || !pow2(c) || rm > 512 || rd > 512 || c > cmax)
    return fail(BTTB_EINVAL, "group: threads per block must be powers of two <= 512 (columns: <= 256 in FP64)");
  for (int i = 0; i < g->count; ++i) {
    const Plan* P = g->P[i];
    if (rm < P->Py / 8 || rd < P->Py / 8 || c < P->Px / 8)
      return fail(BTTB_EINVAL, "group: threads per block below a member's transform (N / 8)");
  }
  return BTTB_OK;
}

template <typename T>
static GLaunch<T> launch_of(const Group* g, int st, const Fuse<T>* fz, const void* const* in, void* const* out,
                            const void* const* winv, const void* const* wd) {
  GLaunch<T> L{};
  L.mem = static_cast<const GMember<T>*>(g->mem);
  L.fz = fz;
  L.in = reinterpret_cast<const T* const*>(in);
  L.out = reinterpret_cast<T* const*>(out);
  L.winv = reinterpret_cast<const T* const*>(winv);
  L.wd = reinterpret_cast<const T* const*>(wd);
  L.bt = stage_threads(g, st);
  L.count = g->count;
  for (int i = 0; i <= g->count; ++i) L.start[i] = g->start[st][i];
  return L;
}

template <typename T>
int group_apply_impl(const Group* g, int op, const void* const* in, void* const* out, const void* const* winv,
                     const void* const* wd, const Fuse<T>* fz, hipStream_t s) {
  auto run = [&](int st, auto kernel) -> int {
    const GLaunch<T> L = launch_of<T>(g, st, fz, in, out, winv, wd);
    const int nb = g->start[st][g->count];
    if (nb == 0) return BTTB_OK;
    hipLaunchKernelGGL(kernel, dim3(nb), dim3(L.bt), g->lds[st], s, L);
    BTTB_LAUNCHED("group stage");
    return BTTB_OK;
  };
  int rc;
  if (op == BTTB_OP_FORWARD) {
    if (fz) {
      rc = run(GS_F1, k_grow_r2c<T, false, FUSE_DIR>);
      if (!rc) rc = run(GS_F2, k_gcol<T, true>);
      if (!rc) rc = run(GS_F3, k_grow_c2r<T, true, FUSE_QQ>);
    } else {
      rc = run(GS_F1, k_grow_r2c<T, false, FUSE_NONE>);
      if (!rc) rc = run(GS_F2, k_gcol<T, true>);
      if (!rc) rc = run(GS_F3, k_grow_c2r<T, true, FUSE_NONE>);
    }
  } else {
    rc = run(GS_T1, k_grow_r2c<T, true, FUSE_NONE>);
    if (!rc) rc = run(GS_T2, k_gcol<T, false>);
    if (!rc) rc = fz ? run(GS_T3, k_grow_c2r<T, false, FUSE_GRAD>) : run(GS_T3, k_grow_c2r<T, false, FUSE_NONE>);
  }
  return rc;
}

template int group_apply_impl<float>(const Group*, int, const void* const*, void* const*, const void* const*,
                                     const void* const*, const Fuse<float>*, hipStream_t);
template int group_apply_impl<double>(const Group*, int, const void* const*, void* const*, const void* const*,
                                      const void* const*, const Fuse<double>*, hipStream_t);

int group_set_launch(Group* g, int rm, int rd, int c, int nchunk, hipStream_t s) {
  const int orm = g->bt_rm, ord = g->bt_rd, oc = g->bt_c, onc = g->nchunk;
  const int nrm = rm > 0 ? rm : orm, nrd = rd > 0 ? rd : ord, ncc = c > 0 ? c : oc;
  int rc = check_threads(g, nrm, nrd, ncc);
  if (rc) return rc;
  g->bt_rm = nrm;
  g->bt_rd = nrd;
  g->bt_c = ncc;
  if (nchunk > 0) g->nchunk = nchunk;
  rc = layout(g);
  if (!rc) rc = g->precision == BTTB_F64 ? upload_members<double>(g, s) : upload_members<float>(g, s);
  if (rc) {  // restore the previous shape
    g->bt_rm = orm; g->bt_rd = ord; g->bt_c = oc; g->nchunk = onc;
    (void)layout(g);
    (void)(g->precision == BTTB_F64 ? upload_members<double>(g, s) : upload_members<float>(g, s));
  }
  return rc;
}

// Largest transforms of the members decide the default shape: one FFT per 64 lanes or more.
static void default_shape(Group* g) {
  int tr = 1, tc = 1;
  for (int i = 0; i < g->count; ++i) {
    tr = std::max(tr, g->P[i]->Py / 8);
    tc = std::max(tc, g->P[i]->Px / 8);
  }
  g->bt_rm = std::max(256, tr);
  g->bt_rd = std::max(64, tr);
  g->bt_c = std::max(g->precision == BTTB_F64 ? 128 : 256, tc);
  g->nchunk = 1;
}

int group_create(const bttb_plan* plans, int count, void* stream, Group** out) {
  *out = nullptr;
  if (count < 1 || count > GMAX) return fail(BTTB_EINVAL, "bttb_group_create: count must be in [1, 64]");
  Group* g = new (std::nothrow) Group{};
  if (!g) return fail(BTTB_ENOMEM, "bttb_group_create: host allocation failed");
  g->count = count;
  for (int i = 0; i < count; ++i) {
    Plan* P = reinterpret_cast<Plan*>(plans[i]);
    if (!P) {
      delete g;
      return fail(BTTB_EINVAL, "bttb_group_create: NULL plan");
    }
    if (!P->fast || P->Px < 32 || P->Py < 32) {
      delete g;
      return fail(BTTB_ESTATE, "bttb_group_create: members need power-of-two transforms of at least 32 "
                               "(bttb_setup with BTTB_PAD_POW2)");
    }
    if (i > 0 && P->precision != g->P[0]->precision) {
      delete g;
      return fail(BTTB_ESTATE, "bttb_group_create: members differ in precision");
    }
    g->P[i] = P;
  }
  g->precision = g->P[0]->precision;
  default_shape(g);
  const size_t msz = g->precision == BTTB_F64 ? sizeof(GMember<double>) : sizeof(GMember<float>);
  if (hipMalloc(&g->mem, msz * count) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return fail(BTTB_ENOMEM, "bttb_group_create: device allocation failed");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = layout(g);
  if (!rc) rc = g->precision == BTTB_F64 ? upload_members<double>(g, s) : upload_members<float>(g, s);
  if (rc) {
    group_destroy(g);
    return rc;
  }
  *out = g;
  return BTTB_OK;
}

void group_destroy(Group* g) {
  if (!g) return;
  dfree(g->mem);
  delete g;
}

}  // namespace bttb

using namespace bttb;

extern "C" int bttb_group_create(const bttb_plan* plans, int count, void* stream, bttb_group* out) {
  if (!plans || !out) return fail(BTTB_EINVAL, "bttb_group_create: NULL argument");
  Group* g = nullptr;
  const int rc = group_create(plans, count, stream, &g);
  *out = reinterpret_cast<bttb_group>(g);
  return rc;
}

extern "C" int bttb_group_apply(bttb_group gg, int op, const void* const* in, void* const* out,
                                const void* const* winv, const void* const* wd, void* stream) {
  const Group* g = reinterpret_cast<const Group*>(gg);
  if (!g || !in || !out) return fail(BTTB_EINVAL, "bttb_group_apply: NULL argument");
  if (op != BTTB_OP_FORWARD && op != BTTB_OP_ADJOINT) return fail(BTTB_EINVAL, "bttb_group_apply: bad op");
  if (!aligned(in, 8) || !aligned(out, 8) || !aligned(winv, 8) || !aligned(wd, 8))
    return fail(BTTB_EINVAL, "bttb_group_apply: misaligned pointer array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return g->precision == BTTB_F64 ? group_apply_impl<double>(g, op, in, out, winv, wd, nullptr, s)
                                  : group_apply_impl<float>(g, op, in, out, winv, wd, nullptr, s);
}

extern "C" int bttb_group_set_launch(bttb_group gg, int model_row_threads, int data_row_threads, int col_threads,
                                     int layer_chunks, void* stream) {
  Group* g = reinterpret_cast<Group*>(gg);
  if (!g) return fail(BTTB_EINVAL, "bttb_group_set_launch: NULL group");
  return group_set_launch(g, model_row_threads, data_row_threads, col_threads, layer_chunks,
                          static_cast<hipStream_t>(stream));
}

extern "C" int bttb_group_info(bttb_group gg, bttb_group_desc* out) {
  const Group* g = reinterpret_cast<const Group*>(gg);
  if (!g || !out) return fail(BTTB_EINVAL, "bttb_group_info: NULL argument");
  out->count = g->count;
  out->precision = g->precision;
  out->model_row_threads = g->bt_rm;
  out->data_row_threads = g->bt_rd;
  out->col_threads = g->bt_c;
  out->layer_chunks = g->nchunk;
  for (int st = 0; st < GS_COUNT; ++st) out->blocks[st] = g->start[st][g->count];
  return BTTB_OK;
}

extern "C" int bttb_group_destroy(bttb_group gg) {
  group_destroy(reinterpret_cast<Group*>(gg));
  return BTTB_OK;
}
