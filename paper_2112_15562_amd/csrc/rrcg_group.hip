// Joint RRCG over many inversions at once (Sec. 2.4 eqs. RRCG:1-8, Sec. 2.5-2.6, Sec. 2.8).
//
// Every inversion keeps its own state, scalars and parameters, exactly as the one-inversion
// solver (rrcg.hip), but each phase of a step is one launch over all of them: the products
// of all gravity and magnetic operators go through a product group (group.hip) with the CG
// pieces fused into their row transforms (gradient, direction, ||q||^2), and each
// elementwise kernel runs over the concatenated blocks of all inversions, a block finding
// its inversion in a prefix table.  The step's phases are captured once into HIP graphs.
// Inversions of uneven sizes therefore share every launch: the small ones ride along
// with the large ones instead of each leaving most of the GPU idle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "common.h"
#include "fast_kernels.h"
#include "group.h"
#include "rrcg_fuse.h"
#include "rrcg_kernels.h"

namespace bttb {

constexpr int GINV_MAX = GMAX / 2;  // inversions per group (two operators each)

// One inversion as the elementwise kernels see it (device table).
template <typename T>
struct GInv {
  long long n, nd;
  T* m[2];
  T* p[2];
  T* rt[2];
  T* l[2];
  T* w[2];
  T* wi[2];
  T* qv[2];
  const T* dobs[2];
  const T* wd[2];
  const T* wdepth[2];
  const T* whard[2];
  const T* mapr[2];
  T* mprev[2];  // previous-iterate anchor: the model at the start of the last CG step (else NULL)
  double lo[2], hi[2], q[2], amin[2], lam[2], eps2;
  int coupled, p_norm, gram_w;
  double* sc;
  double* pb;
  int* pbn;
  int pbs;
};

struct GStart {  // first elementwise block of each inversion
  int count;
  int start[GINV_MAX + 1];
};

__device__ __forceinline__ int inversion_of(const GStart& st, int blk) {
  int i = 0;
  while (i + 1 < st.count && blk >= st.start[i + 1]) ++i;
  return i;
}

template <typename T>
__global__ void __launch_bounds__(eb_threads(sizeof(T))) k_gweights(const GInv<T>* inv, GStart st) {
  const int i = uniform(inversion_of(st, blockIdx.x));
  const GInv<T> v = launch_const(inv + i);
  const int local = blockIdx.x - st.start[i], nb = st.start[i + 1] - st.start[i];
  weights_body<T>(v.n, v.m[0], v.m[1], v.mapr[0], v.mapr[1], v.wdepth[0], v.wdepth[1], v.whard[0], v.whard[1],
                  v.eps2, v.p_norm, v.gram_w, v.w[0], v.w[1], v.wi[0], v.wi[1], v.sc, Red{v.pb, v.pbn, v.pbs},
                  local, nb);
}

template <typename T>
__global__ void __launch_bounds__(eb_threads(sizeof(T))) k_gupdate(const GInv<T>* inv, GStart st) {
  const int i = uniform(inversion_of(st, blockIdx.x));
  const GInv<T> v = launch_const(inv + i);
  const int local = blockIdx.x - st.start[i], nb = st.start[i + 1] - st.start[i];
  update_body<T>(v.n, v.nd, v.m[0], v.m[1], v.p[0], v.p[1], v.w[0], v.w[1], v.rt[0], v.rt[1], v.qv[0], v.qv[1],
                 v.sc, v.lam[0], v.lam[1], v.coupled, v.gram_w, v.mprev[0], v.mprev[1], Red{v.pb, v.pbn, v.pbs},
                 local, nb);
}

// The update of a CG step that another step follows, in one launch: the next step's first
// transform (the data rows of W_d r~) with the residual update r~ <- r~ - s q in its prologue,
// in the first nt1 blocks (whose lead blocks record the step length), and the model update with
// its Gramian partials in the elementwise blocks after them.
template <typename T, int N, bool HALF>
__global__ void __launch_bounds__(eb_threads(sizeof(T))) k_gupdate_t1(const GInv<T>* inv, GStart st, GLaunch<T> g,
                                                                     int nt1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if ((int)blockIdx.x < nt1) {
    const int k = uniform(group_member(g.start, g.count, blockIdx.x));
    const int i = uniform(g.idx[k]);
    const GMember<T> M = launch_const(g.mem + i);
    const int local = blockIdx.x - g.start[k], nb = g.start[k + 1] - g.start[k];
    const int G = g.bt / (N / 8);
    const FRowArgs<T> a{launch_const(g.in + i), 0, g.wd ? launch_const(g.wd + i) : nullptr, M.V, 0, 0, 1, 1, M.sx,
                        M.sy, M.ldk, M.K2, G, (M.sx + 2 * G - 1) / (2 * G), M.twy};
    const Fuse<T> fz = launch_const(g.fz + i);
    frow_r2c_body<T, N, true, FUSE_RUPD, HALF>(a, fz, local, 0, local, nb, smem_raw);
    return;
  }
  const int b = blockIdx.x - nt1;
  const int i = uniform(inversion_of(st, b));
  const GInv<T> v = launch_const(inv + i);
  const int local = b - st.start[i], nb = st.start[i + 1] - st.start[i];
  update_body<T>(v.n, 0, v.m[0], v.m[1], v.p[0], v.p[1], v.w[0], v.w[1], v.rt[0], v.rt[1], v.qv[0], v.qv[1], v.sc,
                 v.lam[0], v.lam[1], v.coupled, v.gram_w, v.mprev[0], v.mprev[1], Red{v.pb, v.pbn, v.pbs}, local,
                 nb, false);
}

template <typename T>
__global__ void __launch_bounds__(eb_threads(sizeof(T))) k_gclip(const GInv<T>* inv, GStart st, int advance) {
  const int i = uniform(inversion_of(st, blockIdx.x));
  const GInv<T> v = launch_const(inv + i);
  const int local = blockIdx.x - st.start[i], nb = st.start[i + 1] - st.start[i];
  if (advance)
    clip_body<T>(v.n, v.m[0], v.m[1], v.lo[0], v.hi[0], v.lo[1], v.hi[1], Red{v.pb, v.pbn, v.pbs}, local, nb);
  else  // Gramian partials only
    clip_body<T>(v.n, v.m[0], v.m[1], -HUGE_VAL, HUGE_VAL, -HUGE_VAL, HUGE_VAL, Red{v.pb, v.pbn, v.pbs}, local, nb);
}

template <typename T>
__global__ void __launch_bounds__(eb_threads(sizeof(T))) k_gresid(const GInv<T>* inv, GStart st) {
  const int i = uniform(inversion_of(st, blockIdx.x));
  const GInv<T> v = launch_const(inv + i);
  const int local = blockIdx.x - st.start[i], nb = st.start[i + 1] - st.start[i];
  resid_body<T>(v.nd, v.rt[0], v.rt[1], v.dobs[0], v.dobs[1], v.wd[0], v.wd[1], Red{v.pb, v.pbn, v.pbs}, local, nb);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_gfin_outer(const GInv<T>* inv, int advance) {  // one block per inversion
  const GInv<T> v = launch_const(inv + blockIdx.x);
  fin_outer_body(v.sc, Red{v.pb, v.pbn, v.pbs}, v.q[0], v.q[1], v.amin[0], v.amin[1], advance, 0, 1);
}

// ------------------------------------------------------------------------------------
struct RrcgGroup {
  int count, precision, use_graph;
  Group* grp;             // products of the 2 count operators: member 2 i + d = data set d of inversion i
  void* inv;              // dev GInv<T>[count]
  GStart est;             // elementwise blocks
  void** ptrs;            // dev pointer arrays, PA_COUNT x (2 count)
  void* fz[4];            // dev Fuse<T>[2 count]: [0] plain step, [1] restart step; [2], [3] the same
                          // for timing repeats (new direction into a scratch vector, no recording)
  double* sc;             // [count][S_COUNT]
  double* pb;             // partials of all inversions
  int* pbn;               // [count][PB_NSLOT]
  void* vec[GINV_MAX][8];  // owned: l0, l1, w0, w1, wi0, wi1, qv (both data sets), timing scratch
                           // (both data sets)
  void* mprev[GINV_MAX][2];  // caller-owned, previous-iterate anchor only
  long long n[GINV_MAX], nd[GINV_MAX];
  double alpha0[GINV_MAX][2];
  hipStream_t cap;
  // whole outer steps captured as one graph each, per number of CG steps (most recent last)
  int n_graphs;
  int graph_inner[4];
  hipGraphExec_t graph[4];
  int fuse_t1;  // the next step's first transform rides with the update (one transform size)
};

// Device pointer arrays (one entry per member) of the group products.
enum { PA_RT = 0, PA_L, PA_WI, PA_WD, PA_P, PA_QV, PA_M, PA_COUNT };

static const void* const* pa(const RrcgGroup* h, int k) {
  return reinterpret_cast<const void* const*>(h->ptrs + (size_t)k * 2 * h->count);
}

template <typename T>
static int g_outer(RrcgGroup* h, hipStream_t s, int advance) {
  const GInv<T>* inv = static_cast<const GInv<T>*>(h->inv);
  const int nb = h->est.start[h->count];
  hipLaunchKernelGGL(k_gclip<T>, dim3(nb), dim3(eb_threads(sizeof(T))), 0, s, inv, h->est, advance);
  BTTB_LAUNCHED("k_gclip");
  int rc = group_apply_impl<T>(h->grp, BTTB_OP_FORWARD, pa(h, PA_M), const_cast<void* const*>(pa(h, PA_RT)),
                               nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gresid<T>, dim3(nb), dim3(eb_threads(sizeof(T))), 0, s, inv, h->est);
  BTTB_LAUNCHED("k_gresid");
  hipLaunchKernelGGL(k_gfin_outer<T>, dim3(h->count), dim3(RB), 0, s, inv, advance);
  BTTB_LAUNCHED("k_gfin_outer");
  return BTTB_OK;
}

template <typename T>
static int g_weights(RrcgGroup* h, hipStream_t s) {
  hipLaunchKernelGGL(k_gweights<T>, dim3(h->est.start[h->count]), dim3(eb_threads(sizeof(T))), 0, s,
                     static_cast<const GInv<T>*>(h->inv), h->est);
  BTTB_LAUNCHED("k_gweights");
  return BTTB_OK;
}

#define RRCG_GROUP_SIZES(N, CALL) \
  switch (N) {                    \
    case 32: CALL(32); break;     \
    case 64: CALL(64); break;     \
    case 128: CALL(128); break;   \
    case 256: CALL(256); break;   \
    case 512: CALL(512); break;   \
    case 1024: CALL(1024); break; \
    case 2048: CALL(2048); break; \
    default: return fail(BTTB_ESIZE, "rrcg_group: transform size out of range"); \
  }

// CG step j of n_inner (RRCG:4-7): the transpose products with the gradient fused in, the
// forward products with the direction and ||q||^2 fused in, and the update.  When the group's
// data rows share one transform size, the update of every step but the last also carries the
// next step's first transform (with the residual update), which that step then skips.
template <typename T>
static int g_inner(RrcgGroup* h, int j, int n_inner, hipStream_t s) {
  const Fuse<T>* fz = static_cast<const Fuse<T>*>(h->fz[j == 0 ? 1 : 0]);
  const Fuse<T>* fz_rep = static_cast<const Fuse<T>*>(h->fz[j == 0 ? 3 : 2]);  // timing repeats only
  const bool t1_done = h->fuse_t1 && j > 0, fuse_next = h->fuse_t1 && j + 1 < n_inner;
  int rc = group_apply_impl<T>(h->grp, BTTB_OP_ADJOINT, pa(h, PA_RT), const_cast<void* const*>(pa(h, PA_L)),
                               pa(h, PA_WI), pa(h, PA_WD), fz, s, t1_done ? 1 : 0, fz_rep);
  if (rc) return rc;
  rc = group_apply_impl<T>(h->grp, BTTB_OP_FORWARD, pa(h, PA_P), const_cast<void* const*>(pa(h, PA_QV)),
                           pa(h, PA_WI), pa(h, PA_WD), fz, s, 0, fz_rep);
  if (rc) return rc;
  const GInv<T>* inv = static_cast<const GInv<T>*>(h->inv);
  if (!fuse_next) {
    hipLaunchKernelGGL(k_gupdate<T>, dim3(h->est.start[h->count]), dim3(eb_threads(sizeof(T))), 0, s, inv, h->est);
    BTTB_LAUNCHED("k_gupdate");
    return BTTB_OK;
  }
  GLaunch<T> L{};
  int nt1 = 0, N = 0, half = 0;
  size_t lds = 0;
  rc = group_stage_launch<T>(h->grp, GS_T1, eb_threads(sizeof(T)), fz, pa(h, PA_RT), nullptr, nullptr,
                             pa(h, PA_WD), &L, &nt1, &N, &half, &lds);
  if (rc) return fail(rc, "rrcg_group: fused update launch");
  const dim3 grid(nt1 + h->est.start[h->count]);
#define RRCG_K(NN)                                                                                    \
  if (half) hipLaunchKernelGGL((k_gupdate_t1<T, NN, true>), grid, dim3(eb_threads(sizeof(T))), lds, s, inv, \
                               h->est, L, nt1);                                                       \
  else hipLaunchKernelGGL((k_gupdate_t1<T, NN, false>), grid, dim3(eb_threads(sizeof(T))), lds, s, inv, h->est, L, nt1)
  RRCG_GROUP_SIZES(N, RRCG_K)
#undef RRCG_K
  BTTB_LAUNCHED("k_gupdate_t1");
  return BTTB_OK;
}

template <typename Fn>
static int g_capture(RrcgGroup* h, Fn fn, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  int rc = BTTB_OK;
  hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "rrcg_group: hipStreamBeginCapture");
  h->grp->t_suspend += 1;  // no timing events inside graphs
  rc = fn(h->cap);
  h->grp->t_suspend -= 1;
  e = hipStreamEndCapture(h->cap, &g);
  if (rc == BTTB_OK && e != hipSuccess) rc = hip_fail(e, "rrcg_group: hipStreamEndCapture");
  if (rc == BTTB_OK) {
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_fail(e, "rrcg_group: hipGraphInstantiate");
  }
  if (g) (void)hipGraphDestroy(g);
  return rc;
}

static void g_drop_graphs(RrcgGroup* h) {
  for (int k = 0; k < h->n_graphs; ++k)
    if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
  h->n_graphs = 0;
}

// The graph of a whole outer step with n_inner CG steps, captured on first use (or by
// rrcg_group_prepare) and kept for the four most recent step lengths.
template <typename T>
static int g_step_graph(RrcgGroup* h, int n_inner, hipGraphExec_t* out) {
  for (int k = 0; k < h->n_graphs; ++k)
    if (h->graph_inner[k] == n_inner) {
      *out = h->graph[k];
      return BTTB_OK;
    }
  if (h->n_graphs == 4) {  // forget the oldest
    (void)hipGraphExecDestroy(h->graph[0]);
    for (int k = 1; k < 4; ++k) {
      h->graph[k - 1] = h->graph[k];
      h->graph_inner[k - 1] = h->graph_inner[k];
    }
    h->n_graphs = 3;
  }
  hipGraphExec_t e = nullptr;
  const int rc = g_capture(h, [&](hipStream_t s) {
    int r = g_weights<T>(h, s);
    for (int j = 0; j < n_inner && !r; ++j) r = g_inner<T>(h, j, n_inner, s);
    return r ? r : g_outer<T>(h, s, 1);
  }, &e);
  if (rc) return rc;
  h->graph[h->n_graphs] = e;
  h->graph_inner[h->n_graphs] = n_inner;
  h->n_graphs += 1;
  *out = e;
  return BTTB_OK;
}

template <typename T>
static int g_step(RrcgGroup* h, int n_inner, hipStream_t s) {
  if (h->use_graph) {
    hipGraphExec_t e = nullptr;
    const int rc = g_step_graph<T>(h, n_inner, &e);
    if (rc) return rc;
    BTTB_HIP(hipGraphLaunch(e, s));
    return BTTB_OK;
  }
  int rc = g_weights<T>(h, s);
  for (int j = 0; j < n_inner && !rc; ++j) rc = g_inner<T>(h, j, n_inner, s);
  return rc ? rc : g_outer<T>(h, s, 1);
}

static void g_free(RrcgGroup* h) {
  if (!h) return;
  g_drop_graphs(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->grp) group_destroy(h->grp);
  for (int i = 0; i < h->count; ++i)
    for (void* v : h->vec[i]) dfree(v);
  dfree(h->inv);
  dfree(h->ptrs);
  for (void* f : h->fz) dfree(f);
  dfree(h->sc);
  dfree(h->pb);
  dfree(h->pbn);
  delete h;
}

static int check_desc(const rrcg_desc* d, size_t es) {
  Plan* P0 = reinterpret_cast<Plan*>(d->plan[0]);
  Plan* P1 = reinterpret_cast<Plan*>(d->plan[1]);
  if (!P0 || !P1) return fail(BTTB_EINVAL, "rrcg_group_create: NULL plan");
  if (P0->sx != P1->sx || P0->sy != P1->sy || P0->nx != P1->nx || P0->ny != P1->ny || P0->nz != P1->nz ||
      P0->precision != P1->precision)
    return fail(BTTB_ESTATE, "rrcg_group_create: the two plans of an inversion differ in grid or precision");
  for (int i = 0; i < 2; ++i) {
    if (!d->m[i] || !d->p[i] || !d->resid[i] || !d->dobs[i] || !d->wd[i] || !d->wdepth[i])
      return fail(BTTB_EINVAL, "rrcg_group_create: NULL vector");
    const void* vs[8] = {d->m[i], d->p[i], d->resid[i], d->dobs[i], d->wd[i], d->wdepth[i], d->whard[i],
                         d->mapr[i]};
    for (const void* v : vs)
      if (v && !aligned(v, es)) return fail(BTTB_EINVAL, "rrcg_group_create: misaligned vector");
    if (!(d->lo[i] <= d->hi[i])) return fail(BTTB_EINVAL, "rrcg_group_create: lo > hi");
    if (!(d->alpha0[i] >= 0) || !(d->q[i] > 0) || !(d->lambda[i] >= 0) || !(d->alpha_min[i] >= 0))
      return fail(BTTB_EINVAL, "rrcg_group_create: alpha0, alpha_min, lambda must be >= 0 and q > 0");
  }
  if (!(d->eps2 > 0)) return fail(BTTB_EINVAL, "rrcg_group_create: eps2 must be > 0");
  if (d->p_norm != 1 && d->p_norm != 2) return fail(BTTB_EINVAL, "rrcg_group_create: p_norm must be 1 or 2");
  if (d->anchor != BTTB_ANCHOR_APR && d->anchor != BTTB_ANCHOR_PREV)
    return fail(BTTB_EINVAL, "rrcg_group_create: anchor must be BTTB_ANCHOR_APR or BTTB_ANCHOR_PREV");
  if (d->anchor == BTTB_ANCHOR_PREV) {
    for (int i = 0; i < 2; ++i)
      if (!d->mprev[i] || !aligned(d->mprev[i], es))
        return fail(BTTB_EINVAL, "rrcg_group_create: the previous-iterate anchor needs aligned mprev vectors");
  }
  return BTTB_OK;
}

template <typename T>
static int g_tables(RrcgGroup* h, const rrcg_desc* descs, hipStream_t s) {
  const int n2 = 2 * h->count;
  GInv<T> inv[GINV_MAX];
  Fuse<T> fz[4][GMAX];
  const void* ptr[PA_COUNT][GMAX];
  long long pb_off = 0;
  std::vector<long long> offs(h->count);
  for (int i = 0; i < h->count; ++i) {
    const Plan* P = reinterpret_cast<const Plan*>(descs[i].plan[0]);
    const long long rows_blocks = (long long)P->nz * ((P->nx + 1) / 2);
    offs[i] = pb_off;
    const int pbs = (int)std::max<long long>(RGRID, std::max<long long>(rows_blocks, (P->sx + 1) / 2));
    inv[i].pbs = pbs;
    pb_off += (long long)PB_NSLOT * pbs;
  }
  if (hipMalloc((void**)&h->pb, (size_t)pb_off * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "rrcg_group_create: device allocation failed");
  }
  for (int i = 0; i < h->count; ++i) {
    const rrcg_desc& d = descs[i];
    GInv<T>& v = inv[i];
    v.n = h->n[i];
    v.nd = h->nd[i];
    T* qv = static_cast<T*>(h->vec[i][6]);
    T* pscratch = static_cast<T*>(h->vec[i][7]);
    const bool prev = d.anchor == BTTB_ANCHOR_PREV;
    for (int k = 0; k < 2; ++k) {
      v.m[k] = static_cast<T*>(d.m[k]);
      v.p[k] = static_cast<T*>(d.p[k]);
      v.rt[k] = static_cast<T*>(d.resid[k]);
      v.l[k] = static_cast<T*>(h->vec[i][k]);
      v.w[k] = static_cast<T*>(h->vec[i][2 + k]);
      v.wi[k] = static_cast<T*>(h->vec[i][4 + k]);
      v.qv[k] = qv + k * h->nd[i];
      v.dobs[k] = static_cast<const T*>(d.dobs[k]);
      v.wd[k] = static_cast<const T*>(d.wd[k]);
      v.wdepth[k] = static_cast<const T*>(d.wdepth[k]);
      v.whard[k] = static_cast<const T*>(d.whard[k]);
      v.mapr[k] = static_cast<const T*>(d.mapr[k]);
      v.mprev[k] = prev ? static_cast<T*>(d.mprev[k]) : nullptr;
      v.lo[k] = d.lo[k];
      v.hi[k] = d.hi[k];
      v.q[k] = d.q[k];
      v.amin[k] = d.alpha_min[k];
      v.lam[k] = d.lambda[k];
    }
    v.eps2 = d.eps2;
    v.coupled = d.coupled ? 1 : 0;
    v.p_norm = d.p_norm;
    v.gram_w = d.gramian_weighted ? 1 : 0;
    v.sc = h->sc + (size_t)i * S_COUNT;
    v.pb = h->pb + offs[i];
    v.pbn = h->pbn + (size_t)i * PB_NSLOT;
    for (int k = 0; k < 2; ++k) {
      const int mi = 2 * i + k;
      ptr[PA_RT][mi] = v.rt[k];
      ptr[PA_L][mi] = v.l[k];
      ptr[PA_WI][mi] = v.wi[k];
      ptr[PA_WD][mi] = v.wd[k];
      ptr[PA_P][mi] = v.p[k];
      ptr[PA_QV][mi] = v.qv[k];
      ptr[PA_M][mi] = v.m[k];
      for (int r = 0; r < 4; ++r) {
        Fuse<T>& f = fz[r][mi];
        const bool rep = r >= 2;  // a timing repeat: same reads, the new direction into scratch
        f = Fuse<T>{};
        f.self = k;
        f.lead = k == 0 && !rep;
        f.restart = (r & 1) == 1 && d.restart ? 1 : 0;
        f.coupled = v.coupled;
        f.gram_w = v.gram_w;
        f.lam[0] = d.lambda[0];
        f.lam[1] = d.lambda[1];
        f.l = v.l[k];
        f.p = v.p[k];
        f.pout = rep ? pscratch + k * h->n[i] : v.p[k];
        f.m[0] = v.m[0];
        f.m[1] = v.m[1];
        f.w[0] = v.w[0];
        f.w[1] = v.w[1];
        f.ma = prev ? v.mprev[k] : v.mapr[k];  // the anchor of RRCG:4 in the original space
        f.r = v.rt[k];
        f.q = v.qv[k];
        f.sc = v.sc;
        f.pb = v.pb;
        f.pbn = v.pbn;
        f.pbs = v.pbs;
      }
    }
  }
  {  // In FP32 the update carries the next step's first transform when the data rows share one
     // transform size.  (The FP64 fused kernel needs 110 registers: with the transform's blocks
     // added, a large inversion's update would no longer fit the CUs in one round.)
    GLaunch<T> L{};
    int nt1 = 0, N = 0, half = 0;
    size_t lds = 0;
    // (power-of-two data rows only: the fused kernel is not compiled for the 5-smooth sizes)
    h->fuse_t1 = sizeof(T) == 4 && group_stage_launch<T>(h->grp, GS_T1, eb_threads(sizeof(T)), nullptr, nullptr,
                                                         nullptr, nullptr, nullptr, &L, &nt1, &N, &half,
                                                         &lds) == BTTB_OK && (N & (N - 1)) == 0;
  }
  BTTB_HIP(hipMemcpyAsync(h->inv, inv, sizeof(GInv<T>) * h->count, hipMemcpyHostToDevice, s));
  for (int r = 0; r < 4; ++r)
    BTTB_HIP(hipMemcpyAsync(h->fz[r], fz[r], sizeof(Fuse<T>) * n2, hipMemcpyHostToDevice, s));
  for (int k = 0; k < PA_COUNT; ++k)
    BTTB_HIP(hipMemcpyAsync(h->ptrs + (size_t)k * n2, ptr[k], sizeof(void*) * n2, hipMemcpyHostToDevice, s));
  // scalars: alpha = alpha0, chi^2 threshold, everything else zero
  std::vector<double> sc((size_t)h->count * S_COUNT, 0.0);
  for (int i = 0; i < h->count; ++i) {
    sc[(size_t)i * S_COUNT + S_ALPHA] = descs[i].alpha0[0];
    sc[(size_t)i * S_COUNT + S_ALPHA + 1] = descs[i].alpha0[1];
    sc[(size_t)i * S_COUNT + S_THR] = (double)h->nd[i] + std::sqrt(2.0 * (double)h->nd[i]);
  }
  BTTB_HIP(hipMemcpyAsync(h->sc, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  BTTB_HIP(hipMemsetAsync(h->pbn, 0, (size_t)h->count * PB_NSLOT * sizeof(int), s));
  BTTB_HIP(hipStreamSynchronize(s));
  return BTTB_OK;
}

static void elementwise_blocks(RrcgGroup* h) {
  const int eb = eb_threads(h->precision == BTTB_F64 ? 8 : 4);
  h->est.count = h->count;
  h->est.start[0] = 0;
  for (int i = 0; i < h->count; ++i) {
    const long long top = std::max(h->n[i], h->nd[i]);
    const long long nb = std::min<long long>(RGRID, std::max<long long>(1, ceil_div((int)std::min<long long>(
                                                                                top, 1LL << 30), eb * EW_UNROLL)));
    h->est.start[i + 1] = h->est.start[i] + (int)nb;
  }
}

}  // namespace bttb

using namespace bttb;

extern "C" int rrcg_group_create(const rrcg_desc* descs, int count, void* stream, rrcg_group* out) {
  if (!descs || !out) return fail(BTTB_EINVAL, "rrcg_group_create: NULL argument");
  *out = nullptr;
  if (count < 1 || count > GINV_MAX) return fail(BTTB_EINVAL, "rrcg_group_create: count must be in [1, 32]");
  const Plan* P00 = reinterpret_cast<const Plan*>(descs[0].plan[0]);
  if (!P00) return fail(BTTB_EINVAL, "rrcg_group_create: NULL plan");
  const int precision = P00->precision;
  const size_t es = precision == BTTB_F64 ? 8 : 4;
  for (int i = 0; i < count; ++i) {
    int rc = check_desc(&descs[i], es);
    if (rc) return rc;
    if (reinterpret_cast<const Plan*>(descs[i].plan[0])->precision != precision)
      return fail(BTTB_ESTATE, "rrcg_group_create: inversions differ in precision");
  }
  RrcgGroup* h = new (std::nothrow) RrcgGroup{};
  if (!h) return fail(BTTB_ENOMEM, "rrcg_group_create: host allocation failed");
  h->count = count;
  h->precision = precision;
  h->use_graph = descs[0].use_graph ? 1 : 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bttb_plan plans[GMAX];
  for (int i = 0; i < count; ++i) {
    plans[2 * i] = descs[i].plan[0];
    plans[2 * i + 1] = descs[i].plan[1];
    const Plan* P = reinterpret_cast<const Plan*>(descs[i].plan[0]);
    h->n[i] = (long long)P->nx * P->ny * P->nz;
    h->nd[i] = (long long)P->sx * P->sy;
  }
  int rc = group_create(plans, 2 * count, stream, &h->grp);
  if (rc) {
    h->grp = nullptr;
    g_free(h);
    return rc;
  }
  bool ok = true;
  for (int i = 0; i < count && ok; ++i) {
    const size_t nb = (size_t)h->n[i] * es;
    for (int k = 0; k < 6 && ok; ++k) ok = hipMalloc(&h->vec[i][k], nb) == hipSuccess;
    ok = ok && hipMalloc(&h->vec[i][6], 2 * (size_t)h->nd[i] * es) == hipSuccess;
    ok = ok && hipMalloc(&h->vec[i][7], 2 * nb) == hipSuccess;
    for (int k = 0; k < 2; ++k) h->mprev[i][k] = descs[i].anchor == BTTB_ANCHOR_PREV ? descs[i].mprev[k] : nullptr;
  }
  const size_t fzb = (precision == BTTB_F64 ? sizeof(Fuse<double>) : sizeof(Fuse<float>)) * 2 * count;
  const size_t invb = (precision == BTTB_F64 ? sizeof(GInv<double>) : sizeof(GInv<float>)) * count;
  for (int r = 0; r < 4 && ok; ++r) ok = hipMalloc(&h->fz[r], fzb) == hipSuccess;
  ok = ok && hipMalloc(&h->inv, invb) == hipSuccess &&
       hipMalloc((void**)&h->ptrs, sizeof(void*) * PA_COUNT * 2 * count) == hipSuccess &&
       hipMalloc((void**)&h->sc, sizeof(double) * S_COUNT * count) == hipSuccess &&
       hipMalloc((void**)&h->pbn, sizeof(int) * PB_NSLOT * count) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    g_free(h);
    return fail(BTTB_ENOMEM, "rrcg_group_create: device allocation failed");
  }
  elementwise_blocks(h);
  rc = precision == BTTB_F64 ? g_tables<double>(h, descs, s) : g_tables<float>(h, descs, s);
  if (!rc) rc = precision == BTTB_F64 ? g_outer<double>(h, s, 0) : g_outer<float>(h, s, 0);
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(BTTB_EHIP, "rrcg_group_create: synchronize");
  if (!rc && h->use_graph) {
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
      rc = fail(BTTB_EHIP, "rrcg_group_create: capture stream");
    else
      h->n_graphs = 0;  // step graphs are captured on first use per step length
  }
  if (rc) {
    g_free(h);
    return rc;
  }
  *out = reinterpret_cast<rrcg_group>(h);
  return BTTB_OK;
}

extern "C" int rrcg_group_step(rrcg_group hh, int n_inner, void* stream) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_group_step: NULL handle");
  if (n_inner < 1) return fail(BTTB_EINVAL, "rrcg_group_step: n_inner must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->precision == BTTB_F64 ? g_step<double>(h, n_inner, s) : g_step<float>(h, n_inner, s);
}

extern "C" int rrcg_group_prepare(rrcg_group hh, int n_inner) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_group_prepare: NULL handle");
  if (n_inner < 1) return fail(BTTB_EINVAL, "rrcg_group_prepare: n_inner must be >= 1");
  if (!h->use_graph) return BTTB_OK;
  hipGraphExec_t e = nullptr;
  return h->precision == BTTB_F64 ? g_step_graph<double>(h, n_inner, &e) : g_step_graph<float>(h, n_inner, &e);
}

extern "C" int rrcg_group_refresh(rrcg_group hh, void* stream) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_group_refresh: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->precision == BTTB_F64 ? g_outer<double>(h, s, 0) : g_outer<float>(h, s, 0);
}

extern "C" int rrcg_group_set_launch(rrcg_group hh, int model_row_threads, int data_row_threads, int col_threads,
                                     int layer_chunks, void* stream) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_group_set_launch: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  BTTB_HIP(hipStreamSynchronize(s));
  int rc = group_set_launch(h->grp, model_row_threads, data_row_threads, col_threads, layer_chunks, s);
  if (!rc) g_drop_graphs(h);  // recaptured with the new shape on next use
  return rc;
}

// Launch shape of the solver's products chosen by timing `reps` CG steps (the fused forms the
// solve runs) per candidate, one coordinate at a time, twice round.  The steps advance the
// iterate, so the solver state (models, directions, residuals, scalars, partials) is saved
// first and restored afterwards: the solve continues exactly as without tuning.
template <typename T>
static int g_autotune(RrcgGroup* h, int reps, hipStream_t s, bttb_tune_result* out) {
  const size_t es = sizeof(T);
  struct Seg {
    void* p;
    size_t bytes;
  };
  std::vector<Seg> segs;
  long long pb_doubles = 0;
  for (int i = 0; i < h->count; ++i) {
    const Plan* P = h->grp->P[2 * i];
    pb_doubles += (long long)PB_NSLOT * std::max<long long>(
        RGRID, std::max<long long>((long long)P->nz * ((P->nx + 1) / 2), (P->sx + 1) / 2));
  }
  segs.push_back({h->sc, sizeof(double) * S_COUNT * h->count});
  segs.push_back({h->pb, sizeof(double) * (size_t)pb_doubles});
  segs.push_back({h->pbn, sizeof(int) * PB_NSLOT * h->count});
  std::vector<const void*> st(PA_COUNT * 2 * h->count);
  BTTB_HIP(hipMemcpy(st.data(), h->ptrs, sizeof(void*) * st.size(), hipMemcpyDeviceToHost));
  for (int mi = 0; mi < 2 * h->count; ++mi) {
    const int i = mi / 2;
    segs.push_back({const_cast<void*>(st[(size_t)PA_M * 2 * h->count + mi]), (size_t)h->n[i] * es});
    segs.push_back({const_cast<void*>(st[(size_t)PA_P * 2 * h->count + mi]), (size_t)h->n[i] * es});
    segs.push_back({const_cast<void*>(st[(size_t)PA_RT * 2 * h->count + mi]), (size_t)h->nd[i] * es});
    if (h->mprev[i][mi % 2]) segs.push_back({h->mprev[i][mi % 2], (size_t)h->n[i] * es});
  }
  size_t total = 0;
  for (const Seg& g : segs) total += (g.bytes + 255) & ~(size_t)255;
  void* save = nullptr;
  if (hipMalloc(&save, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "rrcg_group_autotune: save buffer allocation failed");
  }
  auto copy = [&](bool to_save) -> int {
    size_t off = 0;
    for (const Seg& g : segs) {
      char* b = static_cast<char*>(save) + off;
      BTTB_HIP(hipMemcpyAsync(to_save ? (void*)b : g.p, to_save ? g.p : (void*)b, g.bytes,
                              hipMemcpyDeviceToDevice, s));
      off += (g.bytes + 255) & ~(size_t)255;
    }
    return BTTB_OK;
  };
  hipEvent_t ea = nullptr, eb = nullptr;
  int rc = copy(true);
  if (!rc && (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess))
    rc = fail(BTTB_EHIP, "rrcg_group_autotune: hipEventCreate");
  Group* g = h->grp;
  int cur[4] = {g->bt_rm, g->bt_rd, g->bt_c, g->nchunk};
  float best = -1.0f;
  int tried = 0;
  // a candidate runs as the solve does: one CG step (a middle one: its first transform done by
  // the previous update, its update carrying the next one's) captured as a graph and replayed;
  // the best of two rounds of `reps` replays
  auto measure = [&](float* ms) -> int {
    int r = g_weights<T>(h, s);  // valid weights for the timed steps
    if (r) return r;
    hipGraphExec_t e = nullptr;
    if (h->use_graph) {
      r = g_capture(h, [&](hipStream_t cs) { return g_inner<T>(h, 1, 3, cs); }, &e);
      if (r) return r;
    }
    auto one = [&]() -> int {
      if (e) {
        BTTB_HIP(hipGraphLaunch(e, s));
        return BTTB_OK;
      }
      return g_inner<T>(h, 1, 3, s);
    };
    float bestm = -1.0f;
    r = one();  // warm-up
    for (int round = 0; round < 2 && !r; ++round) {
      if (hipEventRecord(ea, s) != hipSuccess) r = fail(BTTB_EHIP, "rrcg_group_autotune: event");
      for (int k = 0; k < reps && !r; ++k) r = one();
      if (!r && hipEventRecord(eb, s) != hipSuccess) r = fail(BTTB_EHIP, "rrcg_group_autotune: event");
      float m = 0.0f;
      if (!r && (hipEventSynchronize(eb) != hipSuccess || hipEventElapsedTime(&m, ea, eb) != hipSuccess))
        r = fail(BTTB_EHIP, "rrcg_group_autotune: event timing");
      if (!r && (bestm < 0.0f || m < bestm)) bestm = m;
    }
    if (e) (void)hipGraphExecDestroy(e);
    *ms = bestm;
    return r;
  };
  if (!rc) rc = measure(&best);
  if (!rc) ++tried;
  const int cmax = h->precision == BTTB_F64 ? 256 : 512;
  const int cand[4][4] = {{128, 256, 512, 0}, {64, 128, 256, 0}, {128, 256, cmax, 0}, {1, 2, 4, 0}};
  for (int round = 0; round < 2 && !rc; ++round) {
    for (int coord = 0; coord < 4 && !rc; ++coord) {
      for (int ci = 0; cand[coord][ci] && !rc; ++ci) {
        int trial[4] = {cur[0], cur[1], cur[2], cur[3]};
        trial[coord] = cand[coord][ci];
        if (trial[coord] == cur[coord]) continue;
        if (group_set_launch(g, trial[0], trial[1], trial[2], trial[3], s) != BTTB_OK) continue;
        float ms = 0.0f;
        rc = measure(&ms);
        if (rc) break;
        ++tried;
        if (ms < best) {
          best = ms;
          for (int k = 0; k < 4; ++k) cur[k] = trial[k];
        }
      }
      if (!rc) rc = group_set_launch(g, cur[0], cur[1], cur[2], cur[3], s);
    }
  }
  const int rc2 = copy(false);  // restore the solver state in any case
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(BTTB_EHIP, "rrcg_group_autotune: synchronize");
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  dfree(save);
  if (!rc) rc = rc2;
  if (!rc && out) {
    out->us_per_pair = 1e3 * (double)best / reps / (2.0 * h->count);
    for (int k = 0; k < 4; ++k) out->shape[k] = cur[k];
    out->tried = tried;
  }
  return rc;
}

extern "C" int rrcg_group_autotune(rrcg_group hh, int reps, void* stream, bttb_tune_result* out) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_group_autotune: NULL handle");
  if (reps < 1 || reps > 1000) return fail(BTTB_EINVAL, "rrcg_group_autotune: reps must be in [1, 1000]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  BTTB_HIP(hipStreamSynchronize(s));
  int rc = h->precision == BTTB_F64 ? g_autotune<double>(h, reps, s, out) : g_autotune<float>(h, reps, s, out);
  if (!rc) g_drop_graphs(h);  // recaptured with the new shape on next use
  return rc;
}

extern "C" int rrcg_group_products(rrcg_group hh, bttb_group* out) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h || !out) return fail(BTTB_EINVAL, "rrcg_group_products: NULL argument");
  *out = reinterpret_cast<bttb_group>(h->grp);
  return BTTB_OK;
}

static int g_scalars_io(RrcgGroup* h, int index, double* sc, bool write, hipStream_t s) {
  if (index < 0 || index >= h->count) return fail(BTTB_EINVAL, "rrcg_group scalars: index out of range");
  double* dev = h->sc + (size_t)index * S_COUNT;
  if (write)
    BTTB_HIP(hipMemcpyAsync(dev, sc, S_COUNT * sizeof(double), hipMemcpyHostToDevice, s));
  else
    BTTB_HIP(hipMemcpyAsync(sc, dev, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  BTTB_HIP(hipStreamSynchronize(s));
  return BTTB_OK;
}

extern "C" int rrcg_group_read_scalars(rrcg_group hh, int index, rrcg_scalars* out, void* stream) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h || !out) return fail(BTTB_EINVAL, "rrcg_group_read_scalars: NULL argument");
  double sc[S_COUNT];
  int rc = g_scalars_io(h, index, sc, false, static_cast<hipStream_t>(stream));
  if (rc) return rc;
  for (int i = 0; i < 2; ++i) {
    out->alpha[i] = sc[S_ALPHA + i];
    out->L_prev[i] = sc[S_LPREV + i];
    out->phi[i] = sc[S_PHI + i];
    out->beta[i] = sc[S_BETA + i];
    out->step[i] = sc[S_STEP + i];
    out->frozen[i] = sc[S_FROZEN + i] != 0.0;
  }
  out->threshold = sc[S_THR];
  out->gramian = sc[S_GRAM];
  out->k = (int)sc[S_K];
  out->converged = sc[S_CONV] != 0.0;
  out->nonfinite = sc[S_NONFIN] != 0.0;
  out->similarity = sc[S_SIM];
  return BTTB_OK;
}

extern "C" int rrcg_group_write_scalars(rrcg_group hh, int index, const rrcg_scalars* in, void* stream) {
  RrcgGroup* h = reinterpret_cast<RrcgGroup*>(hh);
  if (!h || !in) return fail(BTTB_EINVAL, "rrcg_group_write_scalars: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double sc[S_COUNT];
  int rc = g_scalars_io(h, index, sc, false, s);
  if (rc) return rc;
  for (int i = 0; i < 2; ++i) {
    sc[S_ALPHA + i] = in->alpha[i];
    sc[S_LPREV + i] = in->L_prev[i];
    sc[S_PHI + i] = in->phi[i];
    sc[S_BETA + i] = in->beta[i];
    sc[S_STEP + i] = in->step[i];
    sc[S_FROZEN + i] = in->frozen[i] ? 1.0 : 0.0;
  }
  sc[S_GRAM] = in->gramian;
  sc[S_K] = (double)in->k;
  sc[S_CONV] = in->converged ? 1.0 : 0.0;
  sc[S_NONFIN] = in->nonfinite ? 1.0 : 0.0;
  return g_scalars_io(h, index, sc, true, s);
}

extern "C" int rrcg_group_destroy(rrcg_group hh) {
  g_free(reinterpret_cast<RrcgGroup*>(hh));
  return BTTB_OK;
}
