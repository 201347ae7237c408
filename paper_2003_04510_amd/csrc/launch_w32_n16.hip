// Stage kernels on 32-bit words at N = 2^16 (default tiles).
#include "launch.hpp"

namespace he {

void launch_w32_n16(int stage, const Common& c, const Batch& b, hipStream_t st) {
  launch_stage_n<uint32_t, 8, 8, 2048, 1024>(stage, c, b, st);
}

}  // namespace he
