// Kernel arrays T_(r) of eq. (d=gm) evaluated on the GPU in FP64 (Sec. 2.1, Sec. 2.7.1).
//
// Entry (r, i, j) is the response at station index p over prism index a with p - a =
// i-(nx-1) (and q - b = j-(ny-1)) from a unit-property prism of layer r; the station sits
// above prism column p + ox, so it is u = i-(nx-1)+ox cells from the prism in x (and
// v = j-(ny-1)+oy in y).  With the station at the prism-grid centre positions, the
// prism's corners relative to the station are
//   X in {(-u-1/2) dx, (-u+1/2) dx},  Y in {(-v-1/2) dy, (-v+1/2) dy},
//   Z in {top + r dz + h, top + (r+1) dz + h}   (z down, station at height h),
// and each closed form is a signed sum over the 8 corners with sign (-1)^(i+j+k)
// (i, j, k = 1 lower, 2 upper):
//   vertical gravity (mGal per g/cc):
//     C_G sum s [ Z atan(XY/(ZR)) - X ln(Y+R) - Y ln(X+R) ],  C_G = G * 1e3 * 1e5
//   total-field anomaly for induced magnetisation (nT per SI):
//     (F / 4 pi) f^T H f, f = (cos I sin D, cos I cos D, sin I) (East, North, Down), with
//     H_xx = -sum s atan(YZ/(XR)), H_yy = -sum s atan(XZ/(YR)), H_zz = -sum s atan(XY/(ZR)),
//     H_xy = sum s ln(Z+R), H_xz = sum s ln(Y+R), H_yz = sum s ln(X+R).
// ln(a+R) with a < 0 is evaluated as ln((b^2+c^2)/(R-a)) to avoid cancellation.
// X and Y are never 0 (half-integer cell offsets) and Z >= h > 0.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"

namespace bttb {

__device__ __forceinline__ double ln_plus_r(double a, double b, double c, double R) {
  return a >= 0.0 ? log(a + R) : log((b * b + c * c) / (R - a));
}

__global__ void k_prism(int kind, bttb_geometry g, double* __restrict__ out, double fx, double fy, double fz) {
  const int Lx = g.sx + g.nx - 1, Ly = g.sy + g.ny - 1;
  const long long total = (long long)g.nz * Lx * Ly;
  const double CG = 6.6743e-11 * 1.0e3 * 1.0e5;
  const double PI = 3.14159265358979323846;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx % Ly);
    const long long rest = idx / Ly;
    const int i = (int)(rest % Lx);
    const int r = (int)(rest / Lx);
    const double u = (double)(i - (g.nx - 1) + g.ox), v = (double)(j - (g.ny - 1) + g.oy);
    const double xs[2] = {(-u - 0.5) * g.dx, (-u + 0.5) * g.dx};
    const double ys[2] = {(-v - 0.5) * g.dy, (-v + 0.5) * g.dy};
    const double zs[2] = {g.top + r * g.dz + g.height, g.top + (r + 1) * g.dz + g.height};
    double acc = 0.0;
    double hxx = 0.0, hyy = 0.0, hzz = 0.0, hxy = 0.0, hxz = 0.0, hyz = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const double s = ((a + b + c) & 1) ? 1.0 : -1.0;  // (-1)^(i+j+k), 1-based
          const double X = xs[a], Y = ys[b], Z = zs[c];
          const double R = sqrt(X * X + Y * Y + Z * Z);
          if (kind == BTTB_GRAVITY) {
            acc += s * (Z * atan(X * Y / (Z * R)) - X * ln_plus_r(Y, X, Z, R) - Y * ln_plus_r(X, Y, Z, R));
          } else {
            hxx -= s * atan(Y * Z / (X * R));
            hyy -= s * atan(X * Z / (Y * R));
            hzz -= s * atan(X * Y / (Z * R));
            hxy += s * ln_plus_r(Z, X, Y, R);
            hxz += s * ln_plus_r(Y, X, Z, R);
            hyz += s * ln_plus_r(X, Y, Z, R);
          }
        }
    double val;
    if (kind == BTTB_GRAVITY) {
      val = CG * acc;
    } else {
      const double q = fx * fx * hxx + fy * fy * hyy + fz * fz * hzz + 2.0 * fx * fy * hxy + 2.0 * fx * fz * hxz +
                       2.0 * fy * fz * hyz;
      val = g.field_nt / (4.0 * PI) * q;
    }
    out[idx] = val;
  }
}

}  // namespace bttb

using namespace bttb;

extern "C" int bttb_prism_kernels(int kind, const bttb_geometry* g, double* out, void* stream) {
  if (!g || !out || !aligned(out, 8)) return fail(BTTB_EINVAL, "bttb_prism_kernels: NULL or misaligned argument");
  if (kind != BTTB_GRAVITY && kind != BTTB_MAGNETIC) return fail(BTTB_EINVAL, "bttb_prism_kernels: bad kind");
  if (g->sx < 1 || g->sy < 1 || g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(BTTB_EINVAL, "bttb_prism_kernels: sizes must be >= 1");
  if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !(g->height > 0) || !(g->top >= 0))
    return fail(BTTB_EINVAL, "bttb_prism_kernels: cell sizes and height must be > 0, top >= 0");
  const double d2r = 3.14159265358979323846 / 180.0;
  const double I = g->incl_deg * d2r, D = g->decl_deg * d2r;
  const double fx = cos(I) * sin(D), fy = cos(I) * cos(D), fz = sin(I);
  const long long total = (long long)g->nz * (g->sx + g->nx - 1) * (g->sy + g->ny - 1);
  const long long want = (total + 255) / 256;
  const int blocks = (int)(want < 65535 ? want : 65535);
  hipLaunchKernelGGL(k_prism, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), kind, *g, out, fx, fy,
                     fz);
  BTTB_LAUNCHED("k_prism");
  return BTTB_OK;
}
