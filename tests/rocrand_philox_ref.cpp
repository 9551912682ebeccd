// Independent Philox4x32-10 outputs from the rocRAND engine (host side of its
// header-only device engine), used only to pin the oracle's generator.
// usage: rocrand_philox_ref n c0 c1 c2 c3 seed  -> n lines "w0 w1 w2 w3"
// for counters (c0 + i, c1, c2, c3), i < n, and 64-bit key `seed`.
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char** argv) {
  if (argc != 7) return 2;
  unsigned long long n = strtoull(argv[1], nullptr, 0);
  unsigned int c0 = (unsigned int)strtoul(argv[2], nullptr, 0);
  unsigned int c1 = (unsigned int)strtoul(argv[3], nullptr, 0);
  unsigned int c2 = (unsigned int)strtoul(argv[4], nullptr, 0);
  unsigned int c3 = (unsigned int)strtoul(argv[5], nullptr, 0);
  unsigned long long seed = strtoull(argv[6], nullptr, 0);
  for (unsigned long long i = 0; i < n; ++i) {
    unsigned int x = c0 + (unsigned int)i;
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)x | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, sub, off);
    unsigned int w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
