// Prints rocRAND's Philox4x32-10 block for counters read from stdin ("seed x ind gen tag" per
// line). Built by the oracle tests on the CPU; rocRAND is an independent implementation of the
// generator, so agreement pins the oracle's own Philox.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // reads lines: seed x ind gen tag ; prints 4 words
  unsigned long long seed; unsigned x, ind, gen, tag;
  while (scanf("%llu %u %u %u %u", &seed, &x, &ind, &gen, &tag) == 5) {
    rocrand_state_philox4x32_10 st;
    unsigned long long sub = (unsigned long long)gen | ((unsigned long long)tag << 32);
    unsigned long long off = 4ull * ((unsigned long long)x | ((unsigned long long)ind << 32));
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
