// Stage kernels on 64-bit words at N = 2^16 with 2048-element cols tiles
// (the default, and a batch schedule choice).
#include "launch.hpp"

namespace he {

void launch_u64_n16(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t) {
  if (t.logr == 4) {
    launch_u64_n16_r16(stage, c, b, st, t);
    return;
  }
  if (t.epw_c != 2048) {
    launch_u64_n16_c4096(stage, c, b, st, t);
    return;
  }
  t.epw_b == 1024 ? launch_stage_n<u64, 8, 8, 2048, 1024>(stage, c, b, st)
                  : launch_stage_n<u64, 8, 8, 2048, 2048>(stage, c, b, st);
}

}  // namespace he
