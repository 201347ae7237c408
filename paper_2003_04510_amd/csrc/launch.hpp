// Stage-kernel launchers, shared by the translation units that instantiate
// the stage kernels: each unit instantiates one group (word type, ring
// degree, tiles) so that the groups compile in parallel and every kernel
// instantiation lives in exactly one unit.
#pragma once
#include <hip/hip_runtime.h>

#include "fused.hpp"

namespace he {

inline unsigned pad8(u32 n) { return (n + 7u) & ~7u; }


template <class W, int LOGS, int EPW>
void launch_tensor(const Common& c, const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL((k_tensor_intt<W, LOGS, EPW>), dim3(pad8(b.nitems)), dim3(pass_threads(LOGS, EPW)), 0, st, c, b);
}
template <class W, bool FWD, int LOGS, int EPW, int ST>
void launch_lcols(const Common& c, const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL((k_list_cols<W, FWD, LOGS, EPW, ST>), dim3(pad8(b.nitems)), dim3(pass_threads(LOGS, EPW)), 0, st,
                     c, b);
}

template <class W, bool FWD, int LOGS, int EPW, int ST>
void launch_lblocks(const Common& c, const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL((k_list_blocks<W, FWD, LOGS, EPW, ST>), dim3(pad8(b.nitems)), dim3(pass_threads(LOGS, EPW)), 0,
                     st, c, b);
}

template <class W, bool MD, int NS>
void launch_conv_ns(const Common& c, const Batch& b, hipStream_t st) {
  // 32-bit words hold primes below 2^30: only the general reduction
  constexpr bool WIDE = sizeof(W) == 8;
  if (WIDE && c.bigq) hipLaunchKernelGGL((k_conv<W, MD, NS, WIDE>), dim3(pad8(b.nitems)), dim3(CONV_THREADS), 0, st, c, b);
  else hipLaunchKernelGGL((k_conv<W, MD, NS, false>), dim3(pad8(b.nitems)), dim3(CONV_THREADS), 0, st, c, b);
}
template <class W, bool MD>
void launch_conv(int bucket, const Common& c, const Batch& b, hipStream_t st) {
  switch (bucket) {
    case 4: launch_conv_ns<W, MD, 4>(c, b, st); break;
    case 8: launch_conv_ns<W, MD, 8>(c, b, st); break;
    case 12: launch_conv_ns<W, MD, 12>(c, b, st); break;
    case 15: launch_conv_ns<W, MD, 15>(c, b, st); break;
    case 24: launch_conv_ns<W, MD, 24>(c, b, st); break;
    default: launch_conv_ns<W, MD, 32>(c, b, st); break;
  }
}

// n1 = log_n / 2 (cols passes), n2 = log_n - n1 (blocks passes); EC / EB:
// workgroup tiles of the cols / blocks passes; W: the stored word type.
template <class W, int N1, int N2, int EC = EPW_C, int EB = EPW_B>
void launch_stage_n(int stage, const Common& c, const Batch& b, hipStream_t st) {
  const dim3 g(pad8(b.nitems));
  switch (stage) {
    case ST_TENSOR: launch_tensor<W, N2, EB>(c, b, st); break;
    case ST_Y_ICOLS: launch_lcols<W, false, N1, EC, ST_Y_ICOLS>(c, b, st); break;
    case ST_MU_CONV: launch_conv<W, false>(conv_bucket((c.L + c.dnum - 1) / c.dnum), c, b, st); break;
    case ST_DT_NCOLS: launch_lcols<W, true, N1, EC, ST_DT_NCOLS>(c, b, st); break;
    case ST_DT_NBLOCKS: launch_lblocks<W, true, N2, EB, ST_DT_NBLOCKS>(c, b, st); break;
    case ST_IP:
      if (b.pairs) hipLaunchKernelGGL((k_ip<W, false, N2>), g, dim3(IP_THREADS), 0, st, c, b);
      else hipLaunchKernelGGL((k_ip<W, true, N2>), g, dim3(IP_THREADS), 0, st, c, b);
      break;
    case ST_BLOCKS_IP: hipLaunchKernelGGL((k_blocks_ip<W, N2>), g, dim3(64 * IP_WAVES), 0, st, c, b); break;
    case ST_KS_ICOLS: launch_lcols<W, false, N1, EC, ST_KS_ICOLS>(c, b, st); break;
    case ST_MD_CONV: launch_conv<W, true>(conv_bucket(c.K), c, b, st); break;
    case ST_Z_NCOLS: hipLaunchKernelGGL((k_zcols_lift<W, N1, EC>), g, dim3(pass_threads(N1, EC)), 0, st, c, b); break;
    case ST_COMBINE: hipLaunchKernelGGL((k_ntt_combine<W, N2, EB>), g, dim3(pass_threads(N2, EB)), 0, st, c, b); break;
    case ST_LIFT: hipLaunchKernelGGL((k_lift_ntt_cols<W, N1, EC>), g, dim3(pass_threads(N1, EC)), 0, st, c, b); break;
    case ST_RESCALE: hipLaunchKernelGGL((k_ntt_rescale<W, N2, EB>), g, dim3(pass_threads(N2, EB)), 0, st, c, b); break;
    case ST_Y_IBLOCKS: launch_lblocks<W, false, N2, EB, ST_Y_IBLOCKS>(c, b, st); break;
  }
}


// One per translation unit (launch_*.hip).
void launch_u64_small(u32 log_n, int stage, const Common& c, const Batch& b, hipStream_t st);  // N = 2^12..2^15
void launch_u64_n16(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t);
void launch_u64_n16_c4096(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t);
void launch_u64_n16_r16(int stage, const Common& c, const Batch& b, hipStream_t st, TileCfg t);
void launch_u64_n17(int stage, const Common& c, const Batch& b, hipStream_t st);
// 32-bit words
void launch_w32_small(u32 log_n, int stage, const Common& c, const Batch& b, hipStream_t st);  // N = 2^12..2^15
void launch_w32_n16(int stage, const Common& c, const Batch& b, hipStream_t st);

}  // namespace he
