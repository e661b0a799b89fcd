/*
 * Philox4xW-10 counter-based generator, written from its published
 * definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): each of the 10 rounds multiplies counter words 0 and 2
 * by fixed odd constants, swaps the halves and XORs the high product halves
 * with counter words 1 and 3 and the round key; the key is bumped by the
 * Weyl constants between rounds.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle). One body serves both
 * word sizes, so the 4x64 instance, which numpy ships, pins the structure
 * the 4x32 instance used by the simulation shares.
 */
#include <stdint.h>

static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

#define DEFINE_PHILOX4(W, T, M0, M1, W0, W1)                                   \
  void ora_philox4x##W##_10(const T ctr[4], const T key[2], T out[4]) {       \
    T c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];                      \
    T k0 = key[0], k1 = key[1];                                                \
    for (int round = 0; round < 10; round++) {                                 \
      if (round > 0) {                                                         \
        k0 = (T)(k0 + (W0));                                                   \
        k1 = (T)(k1 + (W1));                                                   \
      }                                                                        \
      T hi0, lo0, hi1, lo1;                                                    \
      mulhilo##W((T)(M0), c0, &hi0, &lo0);                                     \
      mulhilo##W((T)(M1), c2, &hi1, &lo1);                                     \
      T n0 = hi1 ^ c1 ^ k0;                                                    \
      T n1 = lo1;                                                              \
      T n2 = hi0 ^ c3 ^ k1;                                                    \
      T n3 = lo0;                                                              \
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;                                      \
    }                                                                          \
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                        \
  }

/* Multipliers and Weyl increments from the SC'11 paper. The Weyl increments
 * are the leading bits of the golden ratio's fractional part and of
 * sqrt(3) - 1, which a test recomputes. */
DEFINE_PHILOX4(32, uint32_t, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
DEFINE_PHILOX4(64, uint64_t, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
               0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)
