// Host-only reference words from rocRAND's Philox4x32-10 (a library routine),
// used to pin the oracle's Philox implementation.  Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal uint32) and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds() is a protected member: expose it through a derived class.
struct engine : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  engine eng;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr{c0, c1, c2, c3};
    uint2 key{k0, k1};
    uint4 r = eng.block(ctr, key);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
