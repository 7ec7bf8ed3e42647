// Host program: Philox4x32-10 blocks from rocRAND's public engine class, used
// as an independent implementation to pin the oracle's generator.
// Reads lines "k h_lo h_hi tag key_lo key_hi" on stdin, prints four words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Engine : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Engine eng;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr{c0, c1, c2, c3};
    uint2 key{k0, k1};
    uint4 r = eng.ten_rounds(ctr, key);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
