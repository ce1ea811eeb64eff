// Reference Philox4x32-10 values from rocRAND's host-side engine, used only
// by the oracle's RNG pin test.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on
// stdin and prints the four output words for each.  rocRAND's engine starts
// at counter (0, 0, subsequence lo, subsequence hi) under key = seed and
// advances word 0/1 by one per four outputs, so counter (c0,c1,c2,c3) is
// reached with subsequence = c2 | c3<<32 and offset = 4 * (c0 | c1<<32).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
