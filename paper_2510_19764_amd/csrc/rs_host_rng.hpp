// Host side of the counter-based generator (Philox4x64-10, Salmon et al.,
// SC'11) for the host parts of connectivity updates: the same keys and
// counters give the same draws as the device's draw_u32.
#pragma once
#include <stdint.h>

namespace rs {

inline uint64_t host_mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

inline uint32_t host_draw_u32(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1, uint64_t c2,
                              uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t k0 = seed, k1 = (uint64_t)tag | ((uint64_t)proj << 8);
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = host_mulhi64(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = host_mulhi64(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return (uint32_t)(c0 >> 32);
}

inline uint32_t host_below(uint32_t u, uint32_t n) { return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32); }

}  // namespace rs
