// Host build of the FP32 -> fp8 E4M3 conversion used for the low plane of the BF16-refined
// form: prints "<float bits hex> <code hex>" for every input bit pattern given on stdin.
#include <cstdint>
#include <cstdio>

#include "common.h"

int main() {
  unsigned int bits;
  while (std::scanf("%x", &bits) == 1) {
    const float x = __builtin_bit_cast(float, (uint32_t)bits);
    std::printf("%08x %02x\n", bits, et::f32_to_e4m3(x));
  }
  return 0;
}
