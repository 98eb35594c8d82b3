// Host-only cross-check program: prints Philox4x32-10 blocks computed by the
// open-source rocRAND engine header for counters read from stdin
// ("c0 c1 c2 c3 k0 k1" in hex per line).  Used by the tests only.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct exposed_engine : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
  unsigned c0, c1, c2, c3, k0, k1;
  exposed_engine eng;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr = {c0, c1, c2, c3};
    uint2 key = {k0, k1};
    uint4 o = eng.block(ctr, key);
    std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
