// Host probe of the bfloat16 helpers of the FP32 multigrid levels: reads
// FP32 bit patterns (hex, one per line) and prints, per value, the rounded
// bfloat16 bits and the value they stand for.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "rh_internal.h"

int main() {
  unsigned u;
  while (std::scanf("%x", &u) == 1) {
    float f;
    std::memcpy(&f, &u, sizeof f);
    const uint16_t h = rh::bf16_round(f);
    const float back = rh::bf16_value(h);
    uint32_t ub;
    std::memcpy(&ub, &back, sizeof ub);
    std::printf("%04x %08x\n", (unsigned)h, (unsigned)ub);
  }
  return 0;
}
