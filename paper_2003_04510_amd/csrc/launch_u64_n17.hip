// Stage kernels on 64-bit words at N = 2^17 (default tiles).
#include "launch.hpp"

namespace he {

void launch_u64_n17(int stage, const Common& c, const Batch& b, hipStream_t st) {
  launch_stage_n<u64, 8, 9>(stage, c, b, st);
}

}  // namespace he
