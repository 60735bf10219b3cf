// bttb_apply_noalloc: the products of one plan (bttb_apply with batch 1) with the row spectra and
// the data-side spectra in a fixed device array of this library instead of the plan's scratch,
// for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array; every GPU the library runs on holds its own copy (at
// its own address) until the process ends.  Host code never passes the array's name to a kernel
// or a copy: in host code that name is only a stand-in for the symbol.  The device address is
// looked up once per device with hipGetSymbolAddress, on the first call made with that device
// current, and kept here.  Every call on one GPU shares that GPU's array: calls that overlap on
// one GPU (different streams, or different threads) race.  Nothing in the array needs to start
// at zero: each stage of a product writes all that the next stage reads.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace bttb {

constexpr size_t kStaticScratchBytes = size_t(32) << 20;  // BTTB_NOALLOC_MAX_SCRATCH in bttb.h
static_assert(kStaticScratchBytes == (size_t)BTTB_NOALLOC_MAX_SCRATCH, "header and library agree");

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices];  // device address of `scratch` on each device, once looked up
}  // namespace

// The address of this device's copy of `scratch` (the current device), looked up on first use.
static int scratch_address(void** out) {
  int dev = -1;
  BTTB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BTTB_ESTATE, "bttb_apply_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "bttb_apply_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return fail(BTTB_EHIP, "bttb_apply_noalloc: hipGetSymbolAddress returned NULL");
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return BTTB_OK;
}

}  // namespace bttb

using namespace bttb;

extern "C" int bttb_apply_noalloc(bttb_plan plan, int op, const void* in, void* out, const void* winv,
                                  const void* wd, void* stream) {
  Plan* P = reinterpret_cast<Plan*>(plan);
  if (!P) return fail(BTTB_EINVAL, "bttb_apply_noalloc: plan is NULL");
  if (op != BTTB_OP_FORWARD && op != BTTB_OP_ADJOINT) return fail(BTTB_EINVAL, "bttb_apply_noalloc: bad op");
  const size_t es = P->precision == BTTB_F64 ? 8 : 4;
  if (!in || !out || !aligned(in, es) || !aligned(out, es) || (winv && !aligned(winv, es)) ||
      (wd && !aligned(wd, es)))
    return fail(BTTB_EINVAL, "bttb_apply_noalloc: NULL or misaligned vector");
  // U (the row spectra) first, V (the data-side spectra) from the next 256-byte boundary
  const size_t elem = 2 * es;
  const size_t u_bytes = (size_t)P->nz * P->K2 * P->ldx * elem;
  const size_t v_off = (u_bytes + 255) & ~(size_t)255;
  const size_t need = v_off + (apply_scratch_bytes(P, 1) - u_bytes);
  if (need > kStaticScratchBytes)
    return fail(BTTB_ESIZE, "bttb_apply_noalloc: the plan's products need " + std::to_string(need) +
                                " bytes of scratch, more than the fixed " + std::to_string(kStaticScratchBytes) +
                                " (use bttb_apply)");
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc) return rc;
  void* U = base;
  void* V = static_cast<unsigned char*>(base) + v_off;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (P->precision == BTTB_F64)
    return apply_impl<double>(P, op, 1, static_cast<const double*>(in), 0, static_cast<double*>(out), 0,
                              static_cast<const double*>(winv), static_cast<const double*>(wd), s, U, V);
  return apply_impl<float>(P, op, 1, static_cast<const float*>(in), 0, static_cast<float*>(out), 0,
                           static_cast<const float*>(winv), static_cast<const float*>(wd), s, U, V);
}
