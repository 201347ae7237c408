// Stage kernels on 64-bit words at N = 2^12 .. 2^15 (default tiles).
#include "launch.hpp"

namespace he {

void launch_u64_small(u32 log_n, int stage, const Common& c, const Batch& b, hipStream_t st) {
  switch (log_n) {
    case 12: launch_stage_n<u64, 6, 6>(stage, c, b, st); break;
    case 13: launch_stage_n<u64, 6, 7>(stage, c, b, st); break;
    case 14: launch_stage_n<u64, 7, 7>(stage, c, b, st); break;
    case 15: launch_stage_n<u64, 7, 8>(stage, c, b, st); break;
  }
}

}  // namespace he
