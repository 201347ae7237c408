// Stage kernels on 64-bit words at N = 2^16 with radix-16 register rounds
// in both NTT passes (a batch schedule choice), every tile pair.
#include "launch.hpp"

namespace he {

void launch_u64_n16_r16(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t) {
  constexpr int C2 = tile_code(2048, 4), C4 = tile_code(4096, 4), B1 = tile_code(1024, 4), B2 = tile_code(2048, 4);
  if (t.epw_c == 2048)
    t.epw_b == 1024 ? launch_stage_n<u64, 8, 8, C2, B1>(stage, c, b, st) : launch_stage_n<u64, 8, 8, C2, B2>(stage, c, b, st);
  else
    t.epw_b == 1024 ? launch_stage_n<u64, 8, 8, C4, B1>(stage, c, b, st) : launch_stage_n<u64, 8, 8, C4, B2>(stage, c, b, st);
}

}  // namespace he
