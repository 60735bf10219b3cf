// Joint RRCG on the GPU (Sec. 2.4 eqs. RRCG:1-8, Sec. 2.5 bounds, Sec. 2.6 chi^2 test,
// Sec. 2.8 alpha schedule with fixed Lagrange parameters).
//
// State per data set i: the model m (original space), the search direction p (weighted
// space), the current weights w = W_depth W_hard W_L1 and winv = 1/w, the weighted
// residual r~ = W_d (A m - d), and the scalars (FP64, device resident).  One outer step:
//   w, winv from m (eq. WL, eq. W), Gramian scalars                       k_weights
//   repeat n_inner times:
//     l = A~^T r~ + alpha (w m - w a) + lambda l_G                        transpose product
//         a = m_apr, or m_prev (the model at the start of the last CG step)
//         l_G on m (RRCG:2-3) or on m~ = w m (steepestascenta/b)          (+ k_grad)
//     beta = sum ||l||^2 / sum ||l_prev||^2 (0 at a restart)
//     p = l + beta p,  q = A~ p                                            forward product
//     s = sum (p,l) / sum (||q||^2 + (alpha + lambda) ||p||^2)             (+ k_dir, k_sumsq2)
//     m <- m - s p / w   (m~ <- m~ - s p, RRCG:7-8);  r~ <- r~ - s q;
//     Gramian scalars of the new m                                         k_update
//   m <- clip(m, lo, hi)                                                  k_clip
//   r~ = W_d (A m - d), Phi = ||r~||^2, chi^2 test, alpha <- max(q alpha, alpha_min)
//   unless frozen                                                         k_resid
// On plans that can join a product group (power-of-two transforms, or 5-smooth ones whose rows
// and columns fill at most half of them) the step runs as a one-inversion group solver, with the
// gradient, direction and ||q||^2 computed inside the products' row transforms; otherwise by the
// bracketed elementwise kernels.  Dot
// products are accumulated in FP64 per block and summed in a fixed order by the last
// block to finish, so results are bitwise repeatable; no scalar leaves the device
// during a step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"
#include "group.h"
#include "rrcg_fuse.h"
#include "rrcg_kernels.h"

namespace bttb {

struct Rrcg {
  Plan* P[2];
  int precision;
  long long n, nd;
  const void* dobs[2];
  const void* wd[2];
  const void* wdepth[2];
  const void* whard[2];
  const void* mapr[2];
  double lo[2], hi[2], alpha0[2], q[2], amin[2], lam[2], eps2;
  int coupled, restart, p_norm, gram_w;
  int anchor;      // bttb_anchor
  void* mprev[2];  // caller-owned, BTTB_ANCHOR_PREV only
  rrcg_group grp;  // plans that can join a product group: the step runs as a one-inversion group solver
  void* m[2];      // caller-owned
  void* p[2];      // caller-owned
  void* rt[2];     // caller-owned
  void* l[2];
  void* w[2];
  void* winv[2];
  void* qv[2];
  double* sc;      // [S_COUNT]
  double* pb;      // [PB_NSLOT][pbs] partial sums
  int* pbn;        // [PB_NSLOT]
  int pbs;
  // HIP graphs of the step's phases (captured once at creation on a private stream)
  int use_graph;
  hipStream_t cap;
  hipGraphExec_t g_weights, g_inner_restart, g_inner, g_outer;
};

template <typename T>
__global__ void __launch_bounds__(RB) k_weights(long long n, const T* m0, const T* m1, const T* ma0, const T* ma1,
                                                const T* wz0, const T* wz1, const T* wh0, const T* wh1, double eps2,
                                                int p_norm, int gram_w, T* w0, T* w1, T* wi0, T* wi1, double* sc,
                                                Red rd) {
  weights_body<T>(n, m0, m1, ma0, ma1, wz0, wz1, wh0, wh1, eps2, p_norm, gram_w, w0, w1, wi0, wi1, sc, rd,
                  blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_grad(long long n, T* l0, T* l1, const T* m0, const T* m1, const T* w0,
                                             const T* w1, const T* ma0, const T* ma1, double* sc, double lam0,
                                             double lam1, int gram_w, Red rd) {
  grad_body<T>(n, l0, l1, m0, m1, w0, w1, ma0, ma1, sc, lam0, lam1, gram_w, rd, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_dir(long long n, const T* l0, const T* l1, T* p0, T* p1, double* sc,
                                            int restart_now, int coupled, Red rd) {
  dir_body<T>(n, l0, l1, p0, p1, sc, restart_now, coupled, rd, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_sumsq2(long long n, const T* a0, const T* a1, Red rd) {
  sumsq2_body<T>(n, a0, a1, rd, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_update(long long n, long long nd, T* m0, T* m1, const T* p0, const T* p1,
                                               const T* w0, const T* w1, T* r0, T* r1, const T* q0, const T* q1,
                                               double* sc, double lam0, double lam1, int coupled, int gram_w,
                                               T* mp0, T* mp1, Red rd) {
  update_body<T>(n, nd, m0, m1, p0, p1, w0, w1, r0, r1, q0, q1, sc, lam0, lam1, coupled, gram_w, mp0, mp1, rd,
                 blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_clip(long long n, T* m0, T* m1, double lo0, double hi0, double lo1,
                                             double hi1, Red rd) {
  clip_body<T>(n, m0, m1, lo0, hi0, lo1, hi1, rd, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_resid(long long nd, T* r0, T* r1, const T* d0, const T* d1, const T* wd0,
                                              const T* wd1, Red rd) {
  resid_body<T>(nd, r0, r1, d0, d1, wd0, wd1, rd, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(RB) k_fin_outer(double* sc, Red rd, double q0, double q1, double amin0,
                                                  double amin1, int advance) {
  fin_outer_body(sc, rd, q0, q1, amin0, amin1, advance, 0, 1);
}

static Red red_of(const Rrcg* h) { return Red{h->pb, h->pbn, h->pbs}; }

// ------------------------------------------------------------------------------------
template <typename T>
static int outer_update(Rrcg* h, hipStream_t s, int advance) {
  T** m = reinterpret_cast<T**>(h->m);
  T** rt = reinterpret_cast<T**>(h->rt);
  const Red rd = red_of(h);
  if (advance) {
    hipLaunchKernelGGL(k_clip<T>, dim3(RGRID), dim3(RB), 0, s, h->n, m[0], m[1], h->lo[0], h->hi[0], h->lo[1],
                       h->hi[1], rd);
  } else {
    // Gramian partials only (no projection): clip to +-inf
    hipLaunchKernelGGL(k_clip<T>, dim3(RGRID), dim3(RB), 0, s, h->n, m[0], m[1], -HUGE_VAL, HUGE_VAL, -HUGE_VAL,
                       HUGE_VAL, rd);
  }
  BTTB_LAUNCHED("k_clip");
  for (int i = 0; i < 2; ++i) {
    int rc = apply_impl<T>(h->P[i], BTTB_OP_FORWARD, 1, m[i], 0, rt[i], 0, nullptr, nullptr, s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_resid<T>, dim3(RGRID), dim3(RB), 0, s, h->nd, rt[0], rt[1],
                     static_cast<const T*>(h->dobs[0]), static_cast<const T*>(h->dobs[1]),
                     static_cast<const T*>(h->wd[0]), static_cast<const T*>(h->wd[1]), rd);
  BTTB_LAUNCHED("k_resid");
  hipLaunchKernelGGL(k_fin_outer, dim3(1), dim3(RB), 0, s, h->sc, rd, h->q[0], h->q[1], h->amin[0], h->amin[1],
                     advance);
  BTTB_LAUNCHED("k_fin_outer");
  return BTTB_OK;
}

// Phase 1 of an outer step: w, winv from m and the Gramian scalars.
template <typename T>
static int phase_weights(Rrcg* h, hipStream_t s) {
  T** m = reinterpret_cast<T**>(h->m);
  T** w = reinterpret_cast<T**>(h->w);
  T** wi = reinterpret_cast<T**>(h->winv);
  hipLaunchKernelGGL(k_weights<T>, dim3(RGRID), dim3(RB), 0, s, h->n, m[0], m[1],
                     static_cast<const T*>(h->mapr[0]), static_cast<const T*>(h->mapr[1]),
                     static_cast<const T*>(h->wdepth[0]), static_cast<const T*>(h->wdepth[1]),
                     static_cast<const T*>(h->whard[0]), static_cast<const T*>(h->whard[1]), h->eps2, h->p_norm,
                     h->gram_w, w[0], w[1], wi[0], wi[1], h->sc, red_of(h));
  BTTB_LAUNCHED("k_weights");
  return BTTB_OK;
}

// One CG step (RRCG:2-7) at the outer step's W and alpha; restart_now sets beta = 0.
// (Plans that can join a product group do not come here: their solver is a one-inversion group solver, whose
// products carry the gradient, direction and step-length sums in their row transforms.)
template <typename T>
static int phase_inner(Rrcg* h, int restart_now, hipStream_t s) {
  T** m = reinterpret_cast<T**>(h->m);
  T** p = reinterpret_cast<T**>(h->p);
  T** l = reinterpret_cast<T**>(h->l);
  T** w = reinterpret_cast<T**>(h->w);
  T** wi = reinterpret_cast<T**>(h->winv);
  T** rt = reinterpret_cast<T**>(h->rt);
  T** qv = reinterpret_cast<T**>(h->qv);
  // the regulariser's anchor (original space): m_apr, or the model at the start of the last CG step
  T** mp = reinterpret_cast<T**>(h->mprev);
  const T* ma0 = h->anchor == BTTB_ANCHOR_PREV ? mp[0] : static_cast<const T*>(h->mapr[0]);
  const T* ma1 = h->anchor == BTTB_ANCHOR_PREV ? mp[1] : static_cast<const T*>(h->mapr[1]);
  T* mpw0 = h->anchor == BTTB_ANCHOR_PREV ? mp[0] : nullptr;
  T* mpw1 = h->anchor == BTTB_ANCHOR_PREV ? mp[1] : nullptr;
  const Red rd = red_of(h);
  {
    for (int i = 0; i < 2; ++i) {
      int rc = apply_impl<T>(h->P[i], BTTB_OP_ADJOINT, 1, rt[i], 0, l[i], 0, wi[i],
                             static_cast<const T*>(h->wd[i]), s);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_grad<T>, dim3(RGRID), dim3(RB), 0, s, h->n, l[0], l[1], m[0], m[1], w[0], w[1], ma0, ma1,
                       h->sc, h->lam[0], h->lam[1], h->gram_w, rd);
    BTTB_LAUNCHED("k_grad");
    hipLaunchKernelGGL(k_dir<T>, dim3(RGRID), dim3(RB), 0, s, h->n, l[0], l[1], p[0], p[1], h->sc, restart_now,
                       h->coupled, rd);
    BTTB_LAUNCHED("k_dir");
    for (int i = 0; i < 2; ++i) {
      int rc = apply_impl<T>(h->P[i], BTTB_OP_FORWARD, 1, p[i], 0, qv[i], 0, wi[i],
                             static_cast<const T*>(h->wd[i]), s);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_sumsq2<T>, dim3(RGRID), dim3(RB), 0, s, h->nd, qv[0], qv[1], rd);
    BTTB_LAUNCHED("k_sumsq2");
  }
  hipLaunchKernelGGL(k_update<T>, dim3(RGRID), dim3(RB), 0, s, h->n, h->nd, m[0], m[1], p[0], p[1], w[0], w[1],
                     rt[0], rt[1], qv[0], qv[1], h->sc, h->lam[0], h->lam[1], h->coupled, h->gram_w, mpw0, mpw1,
                     rd);
  BTTB_LAUNCHED("k_update");
  return BTTB_OK;
}

template <typename T>
static int step_impl(Rrcg* h, int n_inner, hipStream_t s) {
  if (h->use_graph) {
    BTTB_HIP(hipGraphLaunch(h->g_weights, s));
    for (int j = 0; j < n_inner; ++j)
      BTTB_HIP(hipGraphLaunch((j == 0 && h->restart) ? h->g_inner_restart : h->g_inner, s));
    BTTB_HIP(hipGraphLaunch(h->g_outer, s));
    return BTTB_OK;
  }
  int rc = phase_weights<T>(h, s);
  for (int j = 0; j < n_inner && rc == BTTB_OK; ++j) rc = phase_inner<T>(h, (j == 0 && h->restart) ? 1 : 0, s);
  return rc == BTTB_OK ? outer_update<T>(h, s, 1) : rc;
}

// Captures one phase on the private stream into an executable graph.
template <typename Fn>
static int capture(Rrcg* h, Fn fn, hipGraphExec_t* out) {
  for (int i = 0; i < 2; ++i) h->P[i]->t_suspend += 1;  // no timing events inside graphs
  int rc = BTTB_OK;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    rc = hip_fail(e, "rrcg: hipStreamBeginCapture");
  } else {
    rc = fn(h->cap);
    e = hipStreamEndCapture(h->cap, &g);
    if (rc == BTTB_OK && e != hipSuccess) rc = hip_fail(e, "rrcg: hipStreamEndCapture");
    if (rc == BTTB_OK) {
      e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = hip_fail(e, "rrcg: hipGraphInstantiate");
    }
    if (g) (void)hipGraphDestroy(g);
  }
  for (int i = 0; i < 2; ++i) h->P[i]->t_suspend -= 1;
  return rc;
}

template <typename T>
static int build_graphs(Rrcg* h) {
  int rc = capture(h, [&](hipStream_t s) { return phase_weights<T>(h, s); }, &h->g_weights);
  if (rc == BTTB_OK) rc = capture(h, [&](hipStream_t s) { return phase_inner<T>(h, 1, s); }, &h->g_inner_restart);
  if (rc == BTTB_OK) rc = capture(h, [&](hipStream_t s) { return phase_inner<T>(h, 0, s); }, &h->g_inner);
  if (rc == BTTB_OK) rc = capture(h, [&](hipStream_t s) { return outer_update<T>(h, s, 1); }, &h->g_outer);
  return rc;
}

static void free_rrcg(Rrcg* h) {
  if (h->grp) {
    (void)rrcg_group_destroy(h->grp);
    delete h;
    return;
  }
  for (hipGraphExec_t g : {h->g_weights, h->g_inner_restart, h->g_inner, h->g_outer})
    if (g) (void)hipGraphExecDestroy(g);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  for (int i = 0; i < 2; ++i) {
    dfree(h->l[i]); dfree(h->w[i]); dfree(h->winv[i]); dfree(h->qv[i]);
  }
  dfree(h->sc);
  dfree(h->pb);
  dfree(h->pbn);
  delete h;
}

}  // namespace bttb

using namespace bttb;

extern "C" int rrcg_create(const rrcg_desc* d, void* stream, rrcg_handle* out) {
  if (!d || !out) return fail(BTTB_EINVAL, "rrcg_create: NULL argument");
  *out = nullptr;
  Plan* P0 = reinterpret_cast<Plan*>(d->plan[0]);
  Plan* P1 = reinterpret_cast<Plan*>(d->plan[1]);
  if (!P0 || !P1) return fail(BTTB_EINVAL, "rrcg_create: NULL plan");
  if (P0->sx != P1->sx || P0->sy != P1->sy || P0->nx != P1->nx || P0->ny != P1->ny || P0->nz != P1->nz ||
      P0->precision != P1->precision)
    return fail(BTTB_ESTATE, "rrcg_create: the two plans differ in grid or precision");
  const size_t es = P0->precision == BTTB_F64 ? 8 : 4;
  for (int i = 0; i < 2; ++i) {
    if (!d->m[i] || !d->p[i] || !d->resid[i] || !d->dobs[i] || !d->wd[i] || !d->wdepth[i])
      return fail(BTTB_EINVAL, "rrcg_create: NULL vector");
    const void* vs[8] = {d->m[i], d->p[i], d->resid[i], d->dobs[i], d->wd[i], d->wdepth[i], d->whard[i],
                         d->mapr[i]};
    for (const void* v : vs)
      if (v && !aligned(v, es)) return fail(BTTB_EINVAL, "rrcg_create: misaligned vector");
    if (!(d->lo[i] <= d->hi[i])) return fail(BTTB_EINVAL, "rrcg_create: lo > hi");
    if (!(d->alpha0[i] >= 0) || !(d->q[i] > 0) || !(d->lambda[i] >= 0) || !(d->alpha_min[i] >= 0))
      return fail(BTTB_EINVAL, "rrcg_create: alpha0, alpha_min, lambda must be >= 0 and q > 0");
  }
  if (!(d->eps2 > 0)) return fail(BTTB_EINVAL, "rrcg_create: eps2 must be > 0");
  if (d->p_norm != 1 && d->p_norm != 2) return fail(BTTB_EINVAL, "rrcg_create: p_norm must be 1 or 2");
  if (d->anchor != BTTB_ANCHOR_APR && d->anchor != BTTB_ANCHOR_PREV)
    return fail(BTTB_EINVAL, "rrcg_create: anchor must be BTTB_ANCHOR_APR or BTTB_ANCHOR_PREV");
  if (d->anchor == BTTB_ANCHOR_PREV) {
    for (int i = 0; i < 2; ++i)
      if (!d->mprev[i] || !aligned(d->mprev[i], es))
        return fail(BTTB_EINVAL, "rrcg_create: the previous-iterate anchor needs aligned mprev vectors");
  }
  Rrcg* h = new (std::nothrow) Rrcg{};
  if (!h) return fail(BTTB_ENOMEM, "rrcg_create: host allocation failed");
  if (group_member_ok(P0) && group_member_ok(P1)) {
    // both operators' products in one launch per stage, the CG pieces fused into them
    const int rc = rrcg_group_create(d, 1, stream, &h->grp);
    if (rc != BTTB_OK) {
      delete h;
      return rc;
    }
    *out = reinterpret_cast<rrcg_handle>(h);
    return BTTB_OK;
  }
  h->P[0] = P0;
  h->P[1] = P1;
  h->precision = P0->precision;
  h->n = (long long)P0->nx * P0->ny * P0->nz;
  h->nd = (long long)P0->sx * P0->sy;
  for (int i = 0; i < 2; ++i) {
    h->m[i] = d->m[i]; h->p[i] = d->p[i]; h->rt[i] = d->resid[i];
    h->dobs[i] = d->dobs[i]; h->wd[i] = d->wd[i]; h->wdepth[i] = d->wdepth[i];
    h->whard[i] = d->whard[i]; h->mapr[i] = d->mapr[i];
    h->lo[i] = d->lo[i]; h->hi[i] = d->hi[i]; h->alpha0[i] = d->alpha0[i]; h->q[i] = d->q[i];
    h->amin[i] = d->alpha_min[i]; h->lam[i] = d->lambda[i];
    h->mprev[i] = d->anchor == BTTB_ANCHOR_PREV ? d->mprev[i] : nullptr;
  }
  h->anchor = d->anchor;
  h->eps2 = d->eps2;
  h->coupled = d->coupled ? 1 : 0;
  h->restart = d->restart ? 1 : 0;
  h->p_norm = d->p_norm;
  h->gram_w = d->gramian_weighted ? 1 : 0;
  h->use_graph = d->use_graph ? 1 : 0;
  const size_t nb = (size_t)h->n * es, db = (size_t)h->nd * es;
  bool ok = true;
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipMalloc(&h->l[i], nb) == hipSuccess && hipMalloc(&h->w[i], nb) == hipSuccess &&
         hipMalloc(&h->winv[i], nb) == hipSuccess && hipMalloc(&h->qv[i], db) == hipSuccess;
  }
  // partials per slot: the elementwise grid, or the most blocks a fused row transform can
  // have (one row pair per block)
  const long long rows_blocks = (long long)P0->nz * ((P0->nx + 1) / 2);
  h->pbs = (int)std::max<long long>(RGRID, std::max<long long>(rows_blocks, (P0->sx + 1) / 2));
  ok = ok && hipMalloc((void**)&h->sc, S_COUNT * sizeof(double)) == hipSuccess &&
       hipMalloc((void**)&h->pb, (size_t)PB_NSLOT * h->pbs * sizeof(double)) == hipSuccess &&
       hipMalloc((void**)&h->pbn, PB_NSLOT * sizeof(int)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_rrcg(h);
    return fail(BTTB_ENOMEM, "rrcg_create: device allocation failed");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = BTTB_OK;
  double sc[S_COUNT] = {0};
  sc[S_ALPHA] = d->alpha0[0];
  sc[S_ALPHA + 1] = d->alpha0[1];
  sc[S_THR] = (double)h->nd + std::sqrt(2.0 * (double)h->nd);
  if (rc == BTTB_OK && hipMemcpyAsync(h->sc, sc, sizeof(sc), hipMemcpyHostToDevice, s) != hipSuccess)
    rc = fail(BTTB_EHIP, "rrcg_create: scalar upload");
  if (rc == BTTB_OK && hipMemsetAsync(h->pbn, 0, PB_NSLOT * sizeof(int), s) != hipSuccess)
    rc = fail(BTTB_EHIP, "rrcg_create: partial counts reset");
  if (rc == BTTB_OK)
    rc = h->precision == BTTB_F64 ? outer_update<double>(h, s, 0) : outer_update<float>(h, s, 0);
  if (rc == BTTB_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(BTTB_EHIP, "rrcg_create: synchronize");
  if (rc == BTTB_OK && h->use_graph) {
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
      rc = fail(BTTB_EHIP, "rrcg_create: capture stream");
    else
      rc = h->precision == BTTB_F64 ? build_graphs<double>(h) : build_graphs<float>(h);
  }
  if (rc != BTTB_OK) {
    free_rrcg(h);
    return rc;
  }
  *out = reinterpret_cast<rrcg_handle>(h);
  return BTTB_OK;
}

extern "C" int rrcg_step(rrcg_handle hh, int n_inner, void* stream) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_step: NULL handle");
  if (n_inner < 1) return fail(BTTB_EINVAL, "rrcg_step: n_inner must be >= 1");
  if (h->grp) return rrcg_group_step(h->grp, n_inner, stream);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->precision == BTTB_F64 ? step_impl<double>(h, n_inner, s) : step_impl<float>(h, n_inner, s);
}

extern "C" int rrcg_refresh(rrcg_handle hh, void* stream) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_refresh: NULL handle");
  if (h->grp) return rrcg_group_refresh(h->grp, stream);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->precision == BTTB_F64 ? outer_update<double>(h, s, 0) : outer_update<float>(h, s, 0);
}

extern "C" int rrcg_read_scalars(rrcg_handle hh, rrcg_scalars* out, void* stream) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h || !out) return fail(BTTB_EINVAL, "rrcg_read_scalars: NULL argument");
  if (h->grp) return rrcg_group_read_scalars(h->grp, 0, out, stream);
  double sc[S_COUNT];
  hipStream_t s = static_cast<hipStream_t>(stream);
  BTTB_HIP(hipMemcpyAsync(sc, h->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
  BTTB_HIP(hipStreamSynchronize(s));
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

extern "C" int rrcg_write_scalars(rrcg_handle hh, const rrcg_scalars* in, void* stream) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h || !in) return fail(BTTB_EINVAL, "rrcg_write_scalars: NULL argument");
  if (h->grp) return rrcg_group_write_scalars(h->grp, 0, in, stream);
  double sc[S_COUNT];
  hipStream_t s = static_cast<hipStream_t>(stream);
  BTTB_HIP(hipMemcpyAsync(sc, h->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
  BTTB_HIP(hipStreamSynchronize(s));
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
  BTTB_HIP(hipMemcpyAsync(h->sc, sc, sizeof(sc), hipMemcpyHostToDevice, s));
  BTTB_HIP(hipStreamSynchronize(s));
  return BTTB_OK;
}

extern "C" int rrcg_prepare(rrcg_handle hh, int n_inner) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_prepare: NULL handle");
  if (n_inner < 1) return fail(BTTB_EINVAL, "rrcg_prepare: n_inner must be >= 1");
  return h->grp ? rrcg_group_prepare(h->grp, n_inner) : BTTB_OK;
}

extern "C" int rrcg_autotune(rrcg_handle hh, int reps, void* stream, bttb_tune_result* out) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h) return fail(BTTB_EINVAL, "rrcg_autotune: NULL handle");
  if (!h->grp) return fail(BTTB_ESTATE, "rrcg_autotune: the plans cannot join a product group (tune them with "
                                        "bttb_autotune before creating the solver)");
  return rrcg_group_autotune(h->grp, reps, stream, out);
}

extern "C" int rrcg_products(rrcg_handle hh, bttb_group* out) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (!h || !out) return fail(BTTB_EINVAL, "rrcg_products: NULL argument");
  *out = nullptr;
  if (!h->grp) return fail(BTTB_ESTATE, "rrcg_products: the plans cannot join a product group");
  return rrcg_group_products(h->grp, out);
}

extern "C" int rrcg_destroy(rrcg_handle hh) {
  Rrcg* h = reinterpret_cast<Rrcg*>(hh);
  if (h) free_rrcg(h);
  return BTTB_OK;
}
