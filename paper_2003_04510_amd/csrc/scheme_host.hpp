// C ABI of the steps around HE Mul on the device: encoding (Sec. III-A) and
// HE Add (Sec. III-B).  Included by he_lib.hip after its own C ABI.
#include "encode.hpp"

extern "C" {

he_status he_encode(he_ctx* c, const double* d_z, uint32_t n, double scale, int64_t* d_m, void* ws,
                    size_t ws_bytes, he_stream stream) {
  if (!c || !d_m || !ws || (n && !d_z)) return fail(HE_EINVAL, "he_encode: null pointer");
  if (n > c->N / 2) return fail(HE_EINVAL, "he_encode: %u slots exceed N/2", n);
  if (!(scale > 0.0)) return fail(HE_EINVAL, "he_encode: scale must be positive");
  if (ws_bytes < 16 * c->N) return fail(HE_ENOMEM, "he_encode: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N;
  enc::cplx* V = (enc::cplx*)ws;
  const u32 T = enc::THREADS;
  hipLaunchKernelGGL(enc::k_enc_scatter, dim3((u32)ceil_div(N / 2, T)), dim3(T), 0, st, d_z, n, scale, V, c->log_n);
  for (u32 s = 1; s <= c->log_n; ++s)
    hipLaunchKernelGGL(enc::k_fft_stage, dim3((u32)ceil_div(N / 2, T)), dim3(T), 0, st, V, s, c->log_n);
  hipLaunchKernelGGL(enc::k_enc_finish, dim3((u32)ceil_div(N, T)), dim3(T), 0, st, (const enc::cplx*)V, d_m,
                     c->log_n);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

he_status he_add(he_ctx* c, uint32_t level, const uint64_t* d_ct1, const uint64_t* d_ct2, uint64_t* d_out,
                 he_stream stream) {
  if (!c || !d_ct1 || !d_ct2 || !d_out) return fail(HE_EINVAL, "he_add: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_add: level %u not in [1, L]", level);
  HIP_TRY(hipSetDevice(c->device));
  const u64 tot = 2ull * level * c->N;
  hipLaunchKernelGGL(enc::k_he_add, dim3((u32)ceil_div(tot, enc::THREADS)), dim3(enc::THREADS), 0,
                     (hipStream_t)stream, d_ct1, d_ct2, d_out, c->mods, level, c->log_n);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

}  // extern "C"
