// Test helper: prints raw 32-bit outputs of rocRAND's Philox4x32-10 engine on
// the host, as an implementation independent of the oracle's.
// Usage: probe seed subsequence offset count
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  if (argc != 5) return 2;
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long sub = strtoull(argv[2], 0, 0);
  unsigned long long off = strtoull(argv[3], 0, 0);
  long n = atol(argv[4]);
  rocrand_device::philox4x32_10_engine e(seed, sub, off);
  for (long i = 0; i < n; i++) printf("%u\n", e());
  return 0;
}
