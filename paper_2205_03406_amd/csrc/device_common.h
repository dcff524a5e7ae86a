// Device helpers shared by the HIP sources of libhm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {
namespace dev {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Philox4x32-10 (Salmon et al., SC'11): per round, the two 32x32->64-bit
// products of words 0 and 2 with the round multipliers are mixed with words
// 1 and 3 and the key; the key advances by the two Weyl constants.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t mA = 0xD2511F53u, mB = 0xCD9E8D57u;
  const uint32_t wA = 0x9E3779B9u, wB = 0xBB67AE85u;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = mA * c.x, hi0 = __umulhi(mA, c.x);
    const uint32_t lo1 = mB * c.z, hi1 = __umulhi(mB, c.z);
    U4 n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
    k0 += wA;
    k1 += wB;
  }
  return c;
}

// 53 random bits from (hi word, top 21 bits of lo word), centred in (0, 1).
__device__ __forceinline__ double unit53(uint32_t a, uint32_t b) {
  const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
  return __dadd_rn(__dmul_rn((double)m, 0x1p-53), 0x1p-54);
}

// Two standard normals from one Philox draw (Box-Muller).
__device__ __forceinline__ void normal_pair(U4 r, double &z0, double &z1) {
  const double u1 = unit53(r.x, r.y);
  const double u2 = unit53(r.z, r.w);
  const double rad = sqrt(-2.0 * log(u1));
  const double th = __dmul_rn(6.283185307179586, u2);
  double s, c;
  sincos(th, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// The work item of this workgroup in a 1-D grid of nitems x ntiles
// workgroups.  The dispatcher sends linear workgroup ids round robin to the
// 8 XCDs, each with its own L2; the ids are remapped so that the workgroups
// of one XCD take a contiguous run of (tile, item) pairs, items fastest:
// neighbouring items of one column tile (row chunks of one box, segments
// and pair groups of one column box) then share that XCD's L2.
__device__ __forceinline__ void xcd_item_tile(int64_t nitems, int64_t ntiles, int64_t &item,
                                              int64_t &tile) {
  const int64_t G = nitems * ntiles, b = blockIdx.x;
  const int64_t q = G / 8, r = G % 8, x = b % 8;
  const int64_t L = x * q + (x < r ? x : r) + b / 8;
  tile = L / nitems;
  item = L % nitems;
}

}  // namespace dev
}  // namespace hm
