// Launch-shape autotuner for plans and groups.
//
// The arithmetic of an output element does not depend on the launch shape (FFTs per
// block, threads per block, layer chunks of the forward column pass), only the work split
// does, so the shape can be chosen by measurement.  Each candidate runs a forward and a
// transpose product `reps` times on scratch vectors between two HIP events on the
// caller's stream; the fastest is kept.  Plans sweep every valid combination; groups,
// whose shapes have four coordinates, are tuned one coordinate at a time (twice round).
// The scratch vectors are allocated for the call and freed before it returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "group.h"

namespace bttb {

namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct Scratch {
  void* p = nullptr;
  ~Scratch() { dfree(p); }
};

// Elapsed milliseconds of fn() enqueued reps times on s (after one untimed call).
template <typename Fn>
int time_reps(hipStream_t s, int reps, Events& ev, Fn fn, float* ms) {
  int rc = fn();
  if (rc) return rc;
  BTTB_HIP(hipEventRecord(ev.a, s));
  for (int r = 0; r < reps && !rc; ++r) rc = fn();
  if (rc) return rc;
  BTTB_HIP(hipEventRecord(ev.b, s));
  BTTB_HIP(hipEventSynchronize(ev.b));
  BTTB_HIP(hipEventElapsedTime(ms, ev.a, ev.b));
  return BTTB_OK;
}

}  // namespace

template <typename T>
static int plan_pair(Plan* P, const T* x, T* y, const T* r, T* z, hipStream_t s) {
  int rc = apply_impl<T>(P, BTTB_OP_FORWARD, 1, x, 0, y, 0, nullptr, nullptr, s);
  return rc ? rc : apply_impl<T>(P, BTTB_OP_ADJOINT, 1, r, 0, z, 0, nullptr, nullptr, s);
}

int plan_autotune(Plan* P, int reps, hipStream_t s, bttb_tune_result* out) {
  const size_t es = P->precision == BTTB_F64 ? 8 : 4;
  const size_t n = (size_t)P->nx * P->ny * P->nz, nd = (size_t)P->sx * P->sy;
  Scratch buf;
  if (hipMalloc(&buf.p, 2 * (n + nd) * es) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "bttb_autotune: scratch allocation failed");
  }
  BTTB_HIP(hipMemsetAsync(buf.p, 0, 2 * (n + nd) * es, s));
  char* b = static_cast<char*>(buf.p);
  void *x = b, *z = b + n * es, *y = b + 2 * n * es, *r = b + (2 * n + nd) * es;
  Events ev;
  BTTB_HIP(hipEventCreate(&ev.a));
  BTTB_HIP(hipEventCreate(&ev.b));
  const int c0 = P->col_fpb, r0 = P->row_fpb, k0 = P->nchunk;
  float best = -1.0f;
  int bc = c0, br = r0, bk = k0, tried = 0;
  const int vals[5] = {1, 2, 4, 8, 16};
  for (int ci = 0; ci < 4; ++ci)
    for (int ri = 0; ri < 4; ++ri)
      for (int ki = 0; ki < 5; ++ki) {
        const int c = vals[ci], rr = vals[ri], k = vals[ki];
        if (bttb_set_launch(reinterpret_cast<bttb_plan>(P), c, rr, k) != BTTB_OK) continue;
        float ms = 0.0f;
        int rc = time_reps(s, reps, ev, [&]() -> int {
          return P->precision == BTTB_F64
                     ? plan_pair<double>(P, (const double*)x, (double*)y, (const double*)r, (double*)z, s)
                     : plan_pair<float>(P, (const float*)x, (float*)y, (const float*)r, (float*)z, s);
        }, &ms);
        if (rc) {
          P->col_fpb = c0; P->row_fpb = r0; P->nchunk = k0;
          return rc;
        }
        ++tried;
        if (best < 0.0f || ms < best) {
          best = ms; bc = c; br = rr; bk = k;
        }
      }
  P->col_fpb = bc;
  P->row_fpb = br;
  P->nchunk = bk;
  if (out) {
    out->us_per_pair = best < 0.0f ? 0.0 : 1e3 * (double)best / reps;
    out->shape[0] = bc; out->shape[1] = br; out->shape[2] = bk; out->shape[3] = 0;
    out->tried = tried;
  }
  return BTTB_OK;
}

int group_autotune(Group* g, int reps, hipStream_t s, bttb_tune_result* out) {
  const size_t es = g->precision == BTTB_F64 ? 8 : 4;
  const int m = g->count;
  std::vector<size_t> off(m + 1, 0);
  for (int i = 0; i < m; ++i) {
    const Plan* P = g->P[i];
    off[i + 1] = off[i] + 2 * ((size_t)P->nx * P->ny * P->nz + (size_t)P->sx * P->sy);
  }
  Scratch buf, tab;
  if (hipMalloc(&buf.p, off[m] * es) != hipSuccess || hipMalloc(&tab.p, 4 * m * sizeof(void*)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BTTB_ENOMEM, "bttb_group_autotune: scratch allocation failed");
  }
  BTTB_HIP(hipMemsetAsync(buf.p, 0, off[m] * es, s));
  std::vector<void*> h(4 * m);  // x, y, r, z per member
  for (int i = 0; i < m; ++i) {
    const Plan* P = g->P[i];
    const size_t n = (size_t)P->nx * P->ny * P->nz, nd = (size_t)P->sx * P->sy;
    char* b = static_cast<char*>(buf.p) + off[i] * es;
    h[i] = b;                             // x: model
    h[m + i] = b + n * es;                // y: data
    h[2 * m + i] = b + (n + nd) * es;     // r: data
    h[3 * m + i] = b + (n + 2 * nd) * es; // z: model
  }
  BTTB_HIP(hipMemcpyAsync(tab.p, h.data(), 4 * m * sizeof(void*), hipMemcpyHostToDevice, s));
  void** t = static_cast<void**>(tab.p);
  Events ev;
  BTTB_HIP(hipEventCreate(&ev.a));
  BTTB_HIP(hipEventCreate(&ev.b));
  auto pair = [&]() -> int {
    int rc = g->precision == BTTB_F64
                 ? group_apply_impl<double>(g, BTTB_OP_FORWARD, t, t + m, nullptr, nullptr, nullptr, s)
                 : group_apply_impl<float>(g, BTTB_OP_FORWARD, t, t + m, nullptr, nullptr, nullptr, s);
    if (rc) return rc;
    return g->precision == BTTB_F64
               ? group_apply_impl<double>(g, BTTB_OP_ADJOINT, t + 2 * m, t + 3 * m, nullptr, nullptr, nullptr, s)
               : group_apply_impl<float>(g, BTTB_OP_ADJOINT, t + 2 * m, t + 3 * m, nullptr, nullptr, nullptr, s);
  };
  int cur[4] = {g->bt_rm, g->bt_rd, g->bt_c, g->nchunk};
  float best = -1.0f;
  int rc = time_reps(s, reps, ev, pair, &best);
  if (rc) return rc;
  int tried = 1;
  const int cand[4][5] = {{64, 128, 256, 512, 0}, {64, 128, 256, 512, 0}, {64, 128, 256, 512, 0}, {1, 2, 4, 8, 0}};
  for (int round = 0; round < 2; ++round) {
    for (int coord = 3; coord >= 0; --coord) {
      for (int ci = 0; cand[coord][ci]; ++ci) {
        int trial[4] = {cur[0], cur[1], cur[2], cur[3]};
        trial[coord] = cand[coord][ci];
        if (trial[coord] == cur[coord]) continue;
        if (group_set_launch(g, trial[0], trial[1], trial[2], trial[3], s) != BTTB_OK) continue;
        float ms = 0.0f;
        rc = time_reps(s, reps, ev, pair, &ms);
        if (rc) {
          (void)group_set_launch(g, cur[0], cur[1], cur[2], cur[3], s);
          return rc;
        }
        ++tried;
        if (ms < best) {
          best = ms;
          for (int k = 0; k < 4; ++k) cur[k] = trial[k];
        }
      }
      rc = group_set_launch(g, cur[0], cur[1], cur[2], cur[3], s);
      if (rc) return rc;
    }
  }
  if (out) {
    out->us_per_pair = 1e3 * (double)best / reps;
    for (int k = 0; k < 4; ++k) out->shape[k] = cur[k];
    out->tried = tried;
  }
  return BTTB_OK;
}

}  // namespace bttb

using namespace bttb;

extern "C" int bttb_autotune(bttb_plan plan, int reps, void* stream, bttb_tune_result* out) {
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (!P) return fail(BTTB_EINVAL, "bttb_autotune: NULL plan");
  if (reps < 1 || reps > 1000) return fail(BTTB_EINVAL, "bttb_autotune: reps must be in [1, 1000]");
  return plan_autotune(P, reps, static_cast<hipStream_t>(stream), out);
}

extern "C" int bttb_group_autotune(bttb_group gg, int reps, void* stream, bttb_tune_result* out) {
  Group* g = reinterpret_cast<Group*>(gg);
  if (!g) return fail(BTTB_EINVAL, "bttb_group_autotune: NULL group");
  if (reps < 1 || reps > 1000) return fail(BTTB_EINVAL, "bttb_group_autotune: reps must be in [1, 1000]");
  return group_autotune(g, reps, static_cast<hipStream_t>(stream), out);
}
