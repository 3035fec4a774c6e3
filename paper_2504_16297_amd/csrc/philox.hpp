// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the
// published description: each of the 10 rounds multiplies counter words 0 and
// 2 by two fixed 64-bit constants, mixes the 128-bit products with the other
// counter words and the key, and the key advances by two Weyl increments
// between rounds.  Usable on host and device.
//
// Stream convention shared by every random draw of the method: the j-th
// 64-bit word of the stream keyed (k0, k1) is word j % 4 of the block with
// counter (j / 4 + 1, 0, 0, 0); a uniform is (word >> 11) * 2^-53 in [0, 1).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define PTSBE_HD __host__ __device__ __forceinline__
#else
#define PTSBE_HD inline
#endif

namespace ptsbe {

struct U64x4 {
  uint64_t v[4];
};

PTSBE_HD void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  *lo = a * b;
  *hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  *lo = (uint64_t)p;
  *hi = (uint64_t)(p >> 64);
#endif
}

PTSBE_HD U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                             uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 out;
  out.v[0] = c0;
  out.v[1] = c1;
  out.v[2] = c2;
  out.v[3] = c3;
  return out;
}

// Word j of the stream keyed (k0, k1).
PTSBE_HD uint64_t philox_word(uint64_t k0, uint64_t k1, uint64_t j) {
  U64x4 b = philox4x64_10(j / 4 + 1, 0, 0, 0, k0, k1);
  return b.v[j & 3];
}

PTSBE_HD double word_to_uniform(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

PTSBE_HD uint64_t stream_key1(uint32_t stream, uint32_t cfg, uint64_t i) {
  return ((uint64_t)stream << 56) | ((uint64_t)(cfg & 0xff) << 48) | (i & 0xffffffffffffull);
}

}  // namespace ptsbe
