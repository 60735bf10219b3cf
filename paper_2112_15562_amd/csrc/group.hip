// Group products: the forward or transpose products of many plans (members: the gravity
// and magnetic operators of many inversions, of uneven sizes) in one launch per stage.
//
// Each stage (row transform, column pass, inverse row transform; Sec. 2.7.1) runs over the
// concatenated blocks of all members.  A block finds its member in the
// launch's prefix table of first blocks, builds that member's stage arguments from the
// member table, and runs the register-FFT body; every member uses its own plan's
// eigenvalues and scratch.  A stage is one launch per transform size present (so each
// kernel is compiled for one size and keeps that size's register budget).  All blocks of a
// stage have the same thread count, so a member of transform size N runs
// (threads / L) FFTs per block, L = N / 8 rounded up to a power of two.  The per-call vectors come from device arrays of pointers, so a group product
// can be captured in a HIP graph and replayed with new data in the same buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "common.h"
#include "group_kernels.h"

namespace bttb {


// ------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
// Lanes of one transform of size N in the group kernels: N / 8 rounded up to a power of two.
static int lanes(int N) {
  int l = 1;
  while (l < N / 8) l *= 2;
  return l;
}

static int stage_threads(const Group* g, int st) {
  switch (st) {
    case GS_F1: case GS_T3: return g->bt_rm;
    case GS_F3: case GS_T1: return g->bt_rd;
    default: return g->bt_c;
  }
}

// Block counts and LDS of every stage for the current launch shape; each stage is split into
// one launch per transform size present (rows: Py, columns: Px).
static int layout(Group* g) {
  const size_t esz = g->precision == BTTB_F64 ? 8 : 4;
  for (int st = 0; st < GS_COUNT; ++st) {
    g->ncls[st] = 0;
    g->blocks[st] = 0;
  }
  for (int i = 0; i < g->count; ++i) {
    const Plan* P = g->P[i];
    const int tr = lanes(P->Py), tc = lanes(P->Px);
    const int Grm = g->bt_rm / tr, Grd = g->bt_rd / tr, Gc = g->bt_c / tc;
    if (Grm < 1 || Grd < 1 || Gc < 1) return fail(BTTB_EINVAL, "group: threads per block below one transform");
    const int nch = std::min(g->nchunk, std::min(P->nz, P->nchunk_max));
    g->nch[i] = nch;
    const long long b[GS_COUNT] = {
        (long long)P->nz * ceil_div(P->nx, 2 * Grm),  // F1
        (long long)P->K2 * nch,                       // F2
        (long long)ceil_div(P->sx, 2 * Grd),          // F3
        (long long)ceil_div(P->sx, 2 * Grd),          // T1
        (long long)P->K2 * nch,                       // T2
        (long long)P->nz * ceil_div(P->nx, 2 * Grm),  // T3
    };
    const size_t l[GS_COUNT] = {
        fast_row_lds(P->Py, esz, Grm), fast_col_lds(P->Px, esz, Gc, true), fast_row_lds(P->Py, esz, Grd),
        fast_row_lds(P->Py, esz, Grd), fast_col_lds(P->Px, esz, Gc, false), fast_row_lds(P->Py, esz, Grm)};
    // half forms: the rows (model ny, data sy) or the columns (nx and sx) fill at most half
    // the transform
    const int half[GS_COUNT] = {2 * P->ny <= P->Py, 2 * P->nx <= P->Px && 2 * P->sx <= P->Px, 2 * P->sy <= P->Py,
                                2 * P->sy <= P->Py, 2 * P->nx <= P->Px && 2 * P->sx <= P->Px, 2 * P->ny <= P->Py};
    for (int st = 0; st < GS_COUNT; ++st) {
      const int N = (st == GS_F2 || st == GS_T2) ? P->Px : P->Py;
      int c = 0;
      while (c < g->ncls[st] && (g->cls[st][c].N != N || g->cls[st][c].half != half[st])) ++c;
      GClass& C = g->cls[st][c];
      if (c == g->ncls[st]) {
        if (c == GSIZES) return fail(BTTB_EINVAL, "group: too many transform sizes");
        g->ncls[st] += 1;
        C.N = N;
        C.half = half[st];
        C.count = 0;
        C.start[0] = 0;
        C.lds = 0;
      }
      const long long nb = C.start[C.count] + b[st];
      if (nb > (1LL << 30)) return fail(BTTB_ESIZE, "group: too many blocks");
      C.idx[C.count] = i;
      C.start[C.count + 1] = (int)nb;
      C.count += 1;
      C.lds = std::max(C.lds, l[st]);
      // (a 5-smooth size's kernels also hold its twiddle table in static LDS)
      const size_t stat = (pow2(C.N) ? 0 : (size_t)C.N * 2 * esz) + 2048;
      if (C.lds + stat > 160 * 1024) return fail(BTTB_EINVAL, "group: launch shape needs more LDS than a CU has");
      g->blocks[st] += (int)b[st];
    }
  }
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
                      (long long)P->lds * P->ldk, P->eig_even, 0};
  }
  BTTB_HIP(hipMemcpyAsync(g->mem, h, sizeof(GMember<T>) * g->count, hipMemcpyHostToDevice, s));
  BTTB_HIP(hipStreamSynchronize(s));
  return BTTB_OK;
}

static int check_threads(const Group* g, int rm, int rd, int c) {  // (powers of two >= N/8 of every member)
  const int cmax = g->precision == BTTB_F64 ? 256 : 512;
  if (!pow2(rm) || !pow2(rd) || !pow2(c) || rm > 512 || rd > 512 || c > cmax)
    return fail(BTTB_EINVAL, "group: threads per block must be powers of two <= 512 (columns: <= 256 in FP64)");
  for (int i = 0; i < g->count; ++i) {
    const Plan* P = g->P[i];
    if (rm < lanes(P->Py) || rd < lanes(P->Py) || c < lanes(P->Px))
      return fail(BTTB_EINVAL, "group: threads per block below a member's transform (N / 8 rounded up to a power of two)");
  }
  return BTTB_OK;
}

template <typename T>
static GLaunch<T> launch_of(const Group* g, int st, const GClass& C, const Fuse<T>* fz, const void* const* in,
                            void* const* out, const void* const* winv, const void* const* wd) {
  GLaunch<T> L{};
  L.mem = static_cast<const GMember<T>*>(g->mem);
  L.fz = fz;
  L.in = reinterpret_cast<const T* const*>(in);
  L.out = reinterpret_cast<T* const*>(out);
  L.winv = reinterpret_cast<const T* const*>(winv);
  L.wd = reinterpret_cast<const T* const*>(wd);
  L.bt = stage_threads(g, st);
  L.count = C.count;
  for (int i = 0; i < C.count; ++i) L.idx[i] = C.idx[i];
  for (int i = 0; i <= C.count; ++i) L.start[i] = C.start[i];
  return L;
}

#define BTTB_GROUP_SIZES(N, CALL) \
  switch (N) {                    \
    case 32: CALL(32); break;     \
    case 64: CALL(64); break;     \
    case 128: CALL(128); break;   \
    case 256: CALL(256); break;   \
    case 512: CALL(512); break;   \
    case 1024: CALL(1024); break; \
    case 2048: CALL(2048); break; \
    default: return fail(BTTB_ESIZE, "group: transform size out of range"); \
  }

template <typename T>
int group_apply_impl(const Group* g_, int op, const void* const* in, void* const* out, const void* const* winv,
                     const void* const* wd, const Fuse<T>* fz, hipStream_t s, int skip_first,
                     const Fuse<T>* fz_rep) {
  Group* g = const_cast<Group*>(g_);  // timing state only
  auto run = [&](int st) -> int {
    if (g->blocks[st] == 0) return BTTB_OK;
    int tk = -1;
    if (g->t_ev && g->t_suspend == 0 && g->t_used < g->t_cap) {
      tk = g->t_used++;
      g->t_kid[tk] = st;
      (void)hipEventRecord(g->t_ev[2 * tk], s);
    }
    // Repeats of a timed stage: a plain stage reads one buffer and writes another, so its
    // repeats change nothing; a fused stage's repeats (all but the last launch) use fz_rep,
    // which sends the in-place direction update to scratch.  A fused stage without fz_rep
    // runs once.
    const int reps = tk >= 0 && (fz == nullptr || fz_rep != nullptr) ? g->t_repeat : 1;
    for (int r = 0; r < reps; ++r) {
      const Fuse<T>* fzr = r + 1 < reps && fz != nullptr ? fz_rep : fz;
      for (int c = 0; c < g->ncls[st]; ++c) {
        const GClass& C = g->cls[st][c];
        const GLaunch<T> L = launch_of<T>(g, st, C, fzr, in, out, winv, wd);
        void (*kern)(GLaunch<T>) = nullptr;
        if (pow2(C.N)) {
#define BTTB_K(NN) kern = stage_kernel<T, NN>(st, fz != nullptr, C.half != 0)
          BTTB_GROUP_SIZES(C.N, BTTB_K)
#undef BTTB_K
        } else {
          kern = stage_kernel_mixed<T>(C.N, st, fz != nullptr, C.half != 0);
        }
        if (!kern) return fail(BTTB_ESIZE, "group: no kernel for this transform size and form");
        hipLaunchKernelGGL(kern, dim3(C.start[C.count]), dim3(L.bt), C.lds, s, L);
        BTTB_LAUNCHED("group stage");
      }
    }
    if (tk >= 0) {
      (void)hipEventRecord(g->t_ev[2 * tk + 1], s);
      g->t_nrep[tk] = reps;
    }
    return BTTB_OK;
  };
  int rc = BTTB_OK;
  if (op == BTTB_OP_FORWARD) {
    if (!skip_first) rc = run(GS_F1);
    if (!rc) rc = run(GS_F2);
    if (!rc) rc = run(GS_F3);
  } else {
    if (!skip_first) rc = run(GS_T1);
    if (!rc) rc = run(GS_T2);
    if (!rc) rc = run(GS_T3);
  }
  return rc;
}

template <typename T>
int group_stage_launch(const Group* g, int st, int bt, const Fuse<T>* fz, const void* const* in, void* const* out,
                       const void* const* winv, const void* const* wd, GLaunch<T>* L, int* blocks, int* N,
                       int* half, size_t* lds) {
  if (g->ncls[st] != 1) return BTTB_ESTATE;  // several transform sizes or half forms
  const GClass& C0 = g->cls[st][0];
  const int tr = lanes(C0.N);
  if (bt > 512 || bt < tr || bt % tr) return BTTB_ESTATE;  // the row kernels' block sizes (check_threads)
  const int G = bt / tr;
  const size_t esz = g->precision == BTTB_F64 ? 8 : 4;
  GClass C{};
  C.N = C0.N;
  C.half = C0.half;
  C.count = C0.count;
  C.start[0] = 0;
  if (st == GS_F2 || st == GS_T2) return BTTB_ESTATE;  // row stages only
  for (int k = 0; k < C0.count; ++k) {
    const Plan* P = g->P[C0.idx[k]];
    const int rows = (st == GS_F1 || st == GS_T3) ? P->nz * ceil_div(P->nx, 2 * G) : ceil_div(P->sx, 2 * G);
    C.idx[k] = C0.idx[k];
    C.start[k + 1] = C.start[k] + rows;
  }
  C.lds = fast_row_lds(C.N, esz, G);
  *L = launch_of<T>(g, st, C, fz, in, out, winv, wd);
  L->bt = bt;
  *blocks = C.start[C.count];
  *N = C.N;
  *half = C.half;
  *lds = C.lds;
  return BTTB_OK;
}

template int group_stage_launch<float>(const Group*, int, int, const Fuse<float>*, const void* const*, void* const*,
                                       const void* const*, const void* const*, GLaunch<float>*, int*, int*, int*,
                                       size_t*);
template int group_stage_launch<double>(const Group*, int, int, const Fuse<double>*, const void* const*,
                                        void* const*, const void* const*, const void* const*, GLaunch<double>*, int*,
                                        int*, int*, size_t*);

template int group_apply_impl<float>(const Group*, int, const void* const*, void* const*, const void* const*,
                                     const void* const*, const Fuse<float>*, hipStream_t, int, const Fuse<float>*);
template int group_apply_impl<double>(const Group*, int, const void* const*, void* const*, const void* const*,
                                      const void* const*, const Fuse<double>*, hipStream_t, int,
                                      const Fuse<double>*);

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

// A plan can join a group when each transform size is a power of two from 32 to 2048 (the
// register FFT), or a 5-smooth size with group kernels (mixed_size) whose rows and columns (model
// and data side) fill at most half of it.
bool group_member_ok(const Plan* P) {
  auto size_ok = [](int N, bool half) { return pow2(N) ? (N >= 32 && N <= 2048) : (mixed_size(N) && half); };
  return size_ok(P->Px, 2 * P->nx <= P->Px && 2 * P->sx <= P->Px) &&
         size_ok(P->Py, 2 * P->ny <= P->Py && 2 * P->sy <= P->Py);
}

// Largest transforms of the members decide the default shape: one FFT per 64 lanes or more.
static void default_shape(Group* g) {
  int tr = 1, tc = 1;
  for (int i = 0; i < g->count; ++i) {
    tr = std::max(tr, lanes(g->P[i]->Py));
    tc = std::max(tc, lanes(g->P[i]->Px));
  }
  g->bt_rm = std::max(512, tr);  // 16-row tiles: whole 128-byte segments in the transposed stores
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
    if (!group_member_ok(P)) {
      delete g;
      return fail(BTTB_ESTATE, "bttb_group_create: a member's transform sizes must be powers of two from 32 "
                               "(bttb_setup with BTTB_PAD_POW2), or 5-smooth sizes up to 640 whose rows and "
                               "columns fill at most half of them");
    }
    if (i > 0 && P->precision != g->P[0]->precision) {
      delete g;
      return fail(BTTB_ESTATE, "bttb_group_create: members differ in precision");
    }
    for (int j = 0; j < i; ++j) {
      if (g->P[j] == P) {  // a member's intermediates live in its plan: two uses would share them
        delete g;
        return fail(BTTB_EINVAL, "bttb_group_create: a plan appears twice");
      }
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

static void group_timing_free(Group* g) {
  if (g->t_ev) {
    for (int i = 0; i < 2 * g->t_cap; ++i)
      if (g->t_ev[i]) (void)hipEventDestroy(g->t_ev[i]);
  }
  delete[] g->t_ev;
  delete[] g->t_kid;
  delete[] g->t_nrep;
  g->t_ev = nullptr;
  g->t_kid = nullptr;
  g->t_nrep = nullptr;
  g->t_cap = g->t_used = 0;
}

void group_destroy(Group* g) {
  if (!g) return;
  group_timing_free(g);
  dfree(g->mem);
  delete g;
}

int group_timing_enable(Group* g, int max_launches, int repeat) {
  if (max_launches < 0 || repeat < 1 || repeat > 1000) return fail(BTTB_EINVAL, "group timing: bad argument");
  group_timing_free(g);
  g->t_repeat = repeat;
  if (max_launches == 0) return BTTB_OK;
  g->t_ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches]();
  g->t_kid = new (std::nothrow) int[max_launches];
  g->t_nrep = new (std::nothrow) int[max_launches];
  if (!g->t_ev || !g->t_kid || !g->t_nrep) {
    group_timing_free(g);
    return fail(BTTB_ENOMEM, "group timing: host allocation failed");
  }
  g->t_cap = max_launches;
  for (int i = 0; i < 2 * max_launches; ++i) {
    if (hipEventCreate(&g->t_ev[i]) != hipSuccess) {
      group_timing_free(g);
      return fail(BTTB_EHIP, "group timing: hipEventCreate");
    }
  }
  return BTTB_OK;
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
  for (int st = 0; st < GS_COUNT; ++st) out->blocks[st] = g->blocks[st];
  return BTTB_OK;
}

extern "C" int bttb_group_timing_enable(bttb_group gg, int max_launches, int repeat) {
  Group* g = reinterpret_cast<Group*>(gg);
  if (!g) return fail(BTTB_EINVAL, "bttb_group_timing_enable: NULL group");
  return group_timing_enable(g, max_launches, repeat);
}

extern "C" int bttb_group_timing_read(bttb_group gg, double* total_ms, int* count) {
  Group* g = reinterpret_cast<Group*>(gg);
  if (!g || !total_ms || !count) return fail(BTTB_EINVAL, "bttb_group_timing_read: NULL argument");
  for (int k = 0; k < BTTB_NKERNELS; ++k) {
    total_ms[k] = 0.0;
    count[k] = 0;
  }
  for (int i = 0; i < g->t_used; ++i) {
    BTTB_HIP(hipEventSynchronize(g->t_ev[2 * i + 1]));
    float ms = 0.0f;
    BTTB_HIP(hipEventElapsedTime(&ms, g->t_ev[2 * i], g->t_ev[2 * i + 1]));
    total_ms[g->t_kid[i]] += ms;
    count[g->t_kid[i]] += g->t_nrep[i];
  }
  g->t_used = 0;
  return BTTB_OK;
}

extern "C" int bttb_group_timing_list(bttb_group gg, int cap, int* kernel_id, double* ms, int* n) {
  Group* g = reinterpret_cast<Group*>(gg);
  if (!g || !kernel_id || !ms || !n || cap < 0) return fail(BTTB_EINVAL, "bttb_group_timing_list: bad argument");
  int k = 0;
  for (int i = 0; i < g->t_used; ++i) {
    BTTB_HIP(hipEventSynchronize(g->t_ev[2 * i + 1]));
    float t = 0.0f;
    BTTB_HIP(hipEventElapsedTime(&t, g->t_ev[2 * i], g->t_ev[2 * i + 1]));
    if (k < cap) {
      kernel_id[k] = g->t_kid[i];
      ms[k] = (double)t / g->t_nrep[i];
      ++k;
    }
  }
  g->t_used = 0;
  *n = k;
  return BTTB_OK;
}

extern "C" int bttb_group_destroy(bttb_group gg) {
  group_destroy(reinterpret_cast<Group*>(gg));
  return BTTB_OK;
}
