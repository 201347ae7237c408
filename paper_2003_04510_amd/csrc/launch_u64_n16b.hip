// Stage kernels on 64-bit words at N = 2^16 with 4096-element cols tiles (a
// batch schedule choice).
#include "launch.hpp"

namespace he {

void launch_u64_n16_c4096(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t) {
  t.epw_b == 1024 ? launch_stage_n<u64, 8, 8, 4096, 1024>(stage, c, b, st)
                  : launch_stage_n<u64, 8, 8, 4096, 2048>(stage, c, b, st);
}

}  // namespace he
