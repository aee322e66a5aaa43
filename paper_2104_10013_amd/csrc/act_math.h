// sin and cos of the general activation rule, for device and host.
//
// Quadrant q = rint(2y/pi), reduced argument r = y - q pi/2 with pi/2 split in
// three parts (Cody and Waite): the first part has 8 significant bits, so
// q times it is exact for |q| < 2^16, and with the fused multiply-adds every
// step rounds once.  Then the minimax polynomials of the Cephes
// single-precision sinf / cosf on [-pi/4, pi/4].  Absolute error about 2e-7
// for |y| up to 1e5; beyond that bound the reduction loses accuracy (network
// pre-activations stay far below it).
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define DDP_HD __host__ __device__ __forceinline__
#else
#define DDP_HD inline
#endif

namespace ddp {

constexpr float kSinCosMaxArg = 1e5f;

DDP_HD void sin_cos(float y, float& sn, float& cs) {
  const float q = rintf(y * 0.636619772367581343f);
  float r = fmaf(-q, 1.5703125f, y);
  r = fmaf(-q, 4.837512969970703125e-4f, r);
  r = fmaf(-q, 7.54978995489188216e-8f, r);
  const float r2 = r * r;
  const float ps = fmaf(fmaf(-1.9515295891e-4f, r2, 8.3321608736e-3f), r2, -1.6666654611e-1f);
  const float s0 = fmaf(ps * r2, r, r);
  const float pc = fmaf(fmaf(2.443315711809948e-5f, r2, -1.388731625493765e-3f), r2, 4.166664568298827e-2f);
  const float c0 = fmaf(pc * r2, r2, fmaf(-0.5f, r2, 1.f));
  const int iq = (int)q & 3;
  const float a = (iq & 1) ? c0 : s0, b = (iq & 1) ? s0 : c0;
  sn = (iq & 2) ? -a : a;
  cs = ((iq + 1) & 2) ? -b : b;
}

}  // namespace ddp
