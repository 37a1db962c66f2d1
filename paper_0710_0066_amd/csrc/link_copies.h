// The reduced link copies the hop kernels read, written per link from its nine FP64
// entries: two-row FP64, FP32 and FP16 copies and the three-row FP16 copy of the
// LDS-staged FP16 hop (layouts in layout.hip). The copy kernel (layout.hip) and the link
// update (force.hip) share this writer, so that an update keeps the copies in step without
// reading the FP64 links again.
#pragma once
#include "internal.h"

namespace sap {

struct LinkCopies {
  double2* U64c;
  float2* U32;
  __half2* U16;   // two-row copy (48*Vhp entries), then the three-row copy (72*Vhp)
};
__device__ __forceinline__ void write_link_copies(const LinkCopies& lc, long long Vhp, int p, long long j, int mu,
                                                  const double2 e[9]) {
  typedef unsigned u4w __attribute__((ext_vector_type(4)));
  typedef unsigned u2w __attribute__((ext_vector_type(2)));
  typedef float f4w __attribute__((ext_vector_type(4)));
  const long long tile = j / TILE, lane = j % TILE;
  auto h = [](double2 v) { return __builtin_bit_cast(unsigned, __floats2half2_rn((float)v.x, (float)v.y)); };
#pragma unroll
  for (int k = 0; k < 6; ++k) lc.U64c[p * 24 * Vhp + tiled(j, 6 * mu + k, 24)] = e[k];
  float2* u32 = lc.U32 + p * 24 * Vhp + tile * 24 * TILE + 6 * mu * TILE + 2 * lane;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    *(f4w*)(u32 + 2 * k * TILE) = f4w{(float)e[2 * k].x, (float)e[2 * k].y, (float)e[2 * k + 1].x, (float)e[2 * k + 1].y};
  __half2* u2 = lc.U16 + p * 24 * Vhp + tile * 24 * TILE + 6 * mu * TILE;
  *(u4w*)(u2 + 4 * lane) = u4w{h(e[0]), h(e[1]), h(e[2]), h(e[3])};
  *(u2w*)(u2 + 4 * TILE + 2 * lane) = u2w{h(e[4]), h(e[5])};
  __half2* u3 = lc.U16 + 48 * Vhp + p * 36 * Vhp + tile * 36 * TILE + 9 * mu * TILE;
  *(u4w*)(u3 + 4 * lane) = u4w{h(e[0]), h(e[1]), h(e[2]), h(e[3])};
  *(u4w*)(u3 + 4 * TILE + 4 * lane) = u4w{h(e[4]), h(e[5]), h(e[6]), h(e[7])};
  *(unsigned*)(u3 + 8 * TILE + lane) = h(e[8]);
}

}  // namespace sap
