// Group products (group.hip): host and kernel-side descriptions of a group of plans.
#pragma once
#include "common.h"
#include "rrcg_fuse.h"

namespace bttb {

constexpr int GMAX = 64;  // members per group

// Stages of the products: forward row / column / inverse row, transpose likewise.
enum { GS_F1 = 0, GS_F2, GS_F3, GS_T1, GS_T2, GS_T3, GS_COUNT };

// One member as the kernels see it (device table, written at creation and on a launch
// shape change).
template <typename T>
struct GMember {
  int Px, Py, K2, sx, sy, nx, ny, nz, ldx, ldk, nchunk;
  const cx<T>* eig;
  const cx<T>* twx;
  const cx<T>* twy;
  cx<T>* U;
  cx<T>* V;
  long long V_fcs;  // elements between layer-chunk partials of the data spectrum
  int eig_even;     // eigenvalues stored real and even along x
  int pad_;
};

// Arguments of one group launch (by value): the members of one transform size.
template <typename T>
struct GLaunch {
  const GMember<T>* mem;
  const Fuse<T>* fz;     // per member: the CG step's fused forms, or NULL
  const T* const* in;    // dev arrays of one pointer per member
  T* const* out;
  const T* const* winv;  // nullable arrays; entries nullable
  const T* const* wd;
  int bt;                // threads per block
  int count;             // members in this launch
  int idx[GMAX];         // their indices in the group
  int start[GMAX + 1];   // first block of each; start[count] = blocks of the launch
};

// The members of one stage that share a transform size and its half form (one launch).
struct GClass {
  int N, half, count;
  int idx[GMAX];
  int start[GMAX + 1];
  size_t lds;
};

constexpr int GSIZES = 14;  // transform sizes 32 .. 2048, each in the half form or not

struct Group {
  int count, precision;
  Plan* P[GMAX];
  void* mem;  // dev GMember<T>[count]
  int bt_rm, bt_rd, bt_c;  // threads per block: model rows (F1, T3), data rows (F3, T1), columns
  int nchunk;              // layer chunks requested for the forward column pass
  int nch[GMAX];           // per member, bounded by its plan
  int blocks[GS_COUNT];              // blocks of each stage over all its launches
  GClass cls[GS_COUNT][GSIZES];      // per stage: one launch per transform size present
  int ncls[GS_COUNT];
  // optional per-launch event timing (as for plans)
  int t_cap, t_used, t_repeat;
  int t_suspend;  // > 0 while launches are being captured into a graph
  hipEvent_t* t_ev;
  int* t_kid;
  int* t_nrep;  // launches between the two events of each timed stage
};

// The member of a launch that block blk belongs to (start: first block of each member).
__device__ __forceinline__ int group_member(const int* start, int count, int blk) {
  int i = 0;
  while (i + 1 < count && blk >= start[i + 1]) ++i;
  return i;
}

// A stage kernel of the group products.
template <typename T>
using StageKernel = void (*)(GLaunch<T>);
// The stage kernel of a 5-smooth size that is not a power of two (half forms only; group_mixed.h),
// or NULL when there is none for (N, half).
template <typename T>
StageKernel<T> stage_kernel_mixed(int N, int st, bool fused, bool half);
// N is one of those sizes.
bool mixed_size(int N);
// The plan's transform sizes have group kernels: powers of two from 32 to 2048, or 5-smooth sizes
// with group kernels whose rows and columns fill at most half of them.
bool group_member_ok(const Plan* P);

int group_create(const bttb_plan* plans, int count, void* stream, Group** out);
void group_destroy(Group* g);
int group_set_launch(Group* g, int rm, int rd, int c, int nchunk, hipStream_t s);
int group_autotune(Group* g, int reps, hipStream_t s, bttb_tune_result* out);
// skip_first: leave out the first stage (its work done elsewhere).  fz_rep: the fused forms'
// table for the timing repeats (all but the last launch of a timed stage): the same reads,
// with every in-place result sent to scratch, so that the repeats leave the state as one
// launch does.  Without it a fused product is launched once even while timing repeats are on.
template <typename T>
int group_apply_impl(const Group* g, int op, const void* const* in, void* const* out, const void* const* winv,
                     const void* const* wd, const Fuse<T>* fz, hipStream_t s, int skip_first = 0,
                     const Fuse<T>* fz_rep = nullptr);
// One launch of stage st over all members at bt threads per block, when the members share one
// transform size and half form: *L, its blocks, the transform size, the half form and the LDS.
// BTTB_ESTATE when they do not.
template <typename T>
int group_stage_launch(const Group* g, int st, int bt, const Fuse<T>* fz, const void* const* in, void* const* out,
                       const void* const* winv, const void* const* wd, GLaunch<T>* L, int* blocks, int* N,
                       int* half, size_t* lds);

}  // namespace bttb
