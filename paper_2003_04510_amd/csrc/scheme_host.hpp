// C ABI of the steps around HE Mul on the device: encoding (Sec. III-A),
// HE Add (Sec. III-B) and rotation (an automorphism followed by the key
// switching of HE Mul).  Included by he_lib.hip after its own C ABI.
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
    hipLaunchKernelGGL(enc::k_fft_stage, dim3((u32)ceil_div(N / 2, T)), dim3(T), 0, st, V, s, c->log_n, -1.0);
  hipLaunchKernelGGL(enc::k_enc_finish, dim3((u32)ceil_div(N, T)), dim3(T), 0, st, (const enc::cplx*)V, d_m,
                     c->log_n);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

he_status he_decode(he_ctx* c, uint32_t level, const uint64_t* d_m, double scale, uint32_t n, double* d_z,
                    void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_decode")) return r_;
  if (!c || !d_m || !ws || (n && !d_z)) return fail(HE_EINVAL, "he_decode: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_decode: level %u not in [1, L]", level);
  if (n > c->N / 2) return fail(HE_EINVAL, "he_decode: %u slots exceed N/2", n);
  if (!(scale > 0.0)) return fail(HE_EINVAL, "he_decode: scale must be positive");
  const u64 N = c->N, tabs = (u64)level * level * 8 + (u64)level * 8;
  if (ws_bytes < 16 * N + tabs + 256) return fail(HE_ENOMEM, "he_decode: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // mixed-radix tables: [W_j]_{q_i} (j < i), [W_i^-1]_{q_i}, W_i as doubles
  std::vector<u64> wmod((size_t)level * level, 0);
  std::vector<double> wd(level);
  double w = 1.0;
  for (u32 i = 0; i < level; ++i) {
    const u64 qi = c->mod[i];
    u64 W = 1 % qi;
    for (u32 j = 0; j < i; ++j) {
      wmod[(size_t)i * level + j] = W;  // [W_j]_{q_i}
      W = mulmod(W, c->mod[j] % qi, qi);
    }
    wmod[(size_t)i * level + i] = invmod(W, qi);
    wd[i] = w;
    w *= (double)qi;
  }
  enc::cplx* V = (enc::cplx*)ws;
  u64* tw = (u64*)((uint8_t*)ws + 16 * N);
  double* td = (double*)(tw + (u64)level * level);
  he_status r;
  if ((r = upload_sync(tw, wmod.data(), wmod.size() * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(td, wd.data(), wd.size() * 8, st)) != HE_OK) return r;
  enc::DecArgs a{d_m, c->mods, tw, td, V, level, c->log_n};
  const u32 T = enc::THREADS;
  hipLaunchKernelGGL(enc::k_dec_crt, dim3((u32)ceil_div(N, T)), dim3(T), 0, st, a);
  for (u32 s = 1; s <= c->log_n; ++s)
    hipLaunchKernelGGL(enc::k_fft_stage, dim3((u32)ceil_div(N / 2, T)), dim3(T), 0, st, V, s, c->log_n, 1.0);
  if (n)
    hipLaunchKernelGGL(enc::k_dec_gather, dim3((u32)ceil_div(n, T)), dim3(T), 0, st, (const enc::cplx*)V, n, scale,
                       d_z, c->log_n);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

he_status he_add(he_ctx* c, uint32_t level, const uint64_t* d_ct1, const uint64_t* d_ct2, uint64_t* d_out,
                 he_stream stream) {
  if (he_status r_ = need_w64(c, "he_add")) return r_;
  if (!c || !d_ct1 || !d_ct2 || !d_out) return fail(HE_EINVAL, "he_add: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_add: level %u not in [1, L]", level);
  HIP_TRY(hipSetDevice(c->device));
  const u64 tot = 2ull * level * c->N;
  hipLaunchKernelGGL(enc::k_he_add, dim3((u32)ceil_div(tot, enc::THREADS)), dim3(enc::THREADS), 0,
                     (hipStream_t)stream, d_ct1, d_ct2, d_out, c->mods, level, c->log_n);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

namespace {
// g = 5^r mod 2N (r taken modulo N/2, the order of 5).
u64 galois_element(u64 N, int64_t r) {
  const int64_t h = (int64_t)(N / 2);
  u64 e = (u64)(((r % h) + h) % h), g = 1, b = 5;
  const u64 m = 2 * N - 1;
  while (e) {
    if (e & 1) g = (g * b) & m;
    b = (b * b) & m;
    e >>= 1;
  }
  return g;
}
}  // namespace

he_status he_keygen_rot(he_ctx* c, const int64_t* s, int32_t rot, const int64_t* e_rk, const uint64_t* a_rk,
                        uint64_t* d_rk, void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_keygen_rot")) return r_;
  if (!c || !s || !e_rk || !a_rk || !d_rk || !ws) return fail(HE_EINVAL, "he_keygen_rot: null pointer");
  if (ws_bytes < keygen_ws_limbs(c) * c->N * 8) return fail(HE_ENOMEM, "he_keygen_rot: workspace too small");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const u64 N = c->N, g = galois_element(N, rot);
  const u32 L = c->L, nm = L + c->K;
  // -sigma_g(s), a small signed polynomial: s_k X^k -> -s_k X^(kg mod 2N), X^N = -1
  std::vector<int64_t> sg(N);
  for (u64 k = 0; k < N; ++k) {
    const u64 ex = (k * g) & (2 * N - 1);
    if (ex < N) sg[ex] = -s[k];
    else sg[ex - N] = s[k];
  }
  u64* w = (u64*)ws;
  u64* S = w;  w += (u64)nm * N;
  u64* S2 = w; w += (u64)nm * N;
  u64* E = w;  w += (u64)nm * N;
  int64_t* sv = (int64_t*)w;             // [N]
  int64_t* gv = sv + N;                  // [N]
  int64_t* eev = gv + N;                 // [dnum][N]
  he_status r;
  if ((r = upload_sync(sv, s, N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(gv, sg.data(), N * 8, st)) != HE_OK) return r;
  if ((r = upload_sync(eev, e_rk, (u64)c->dnum * N * 8, st)) != HE_OK) return r;
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, sv, S, c->iota, c->mods,
                     nm, c->log_n);
  ntt_launch(c, true, S, S, N, N, 0, 0, c->iota, nullptr, nm, 1, st);
  hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, gv, S2, c->iota, c->mods,
                     nm, c->log_n);
  ntt_launch(c, true, S2, S2, N, N, 0, 0, c->iota, nullptr, nm, 1, st);
  for (u32 j = 0; j < c->dnum; ++j) {
    u64* bj = d_rk + (u64)j * 2 * nm * N;
    u64* aj = bj + (u64)nm * N;
    if ((r = upload_sync(aj, a_rk + (u64)j * nm * N, (u64)nm * N * 8, st)) != HE_OK) return r;
    hipLaunchKernelGGL(k_small_to_limbs, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, eev + (u64)j * N, E,
                       c->iota, c->mods, nm, c->log_n);
    ntt_launch(c, true, E, E, N, N, 0, 0, c->iota, nullptr, nm, 1, st);
    const u32 dlo = j * c->alpha, dhi = std::min(L, (j + 1) * c->alpha);
    hipLaunchKernelGGL(k_evk_b, ew_grid((u64)nm * N), dim3(EW_THREADS), 0, st, aj, S, S2, E, bj, c->pmod,
                       c->mods, nm, dlo, dhi, c->log_n);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return HE_OK;
}

he_status he_rotate(he_ctx* c, uint32_t level, const uint64_t* d_ct, const uint64_t* d_rk, int32_t rot,
                    uint64_t* d_out, void* ws, size_t ws_bytes, he_stream stream) {
  if (he_status r_ = need_w64(c, "he_rotate")) return r_;
  if (!c || !d_ct || !d_rk || !d_out || !ws) return fail(HE_EINVAL, "he_rotate: null pointer");
  if (level < 1 || level > c->L) return fail(HE_ELEVEL, "he_rotate: level %u not in [1, L]", level);
  if (ws_bytes < mul_ws_limbs(c, level) * c->N * 8) return fail(HE_ENOMEM, "he_rotate: workspace too small");
  const u64 N = c->N, ct_bytes = 2ull * level * N * 8;
  if ((const uint8_t*)d_out < (const uint8_t*)d_ct + ct_bytes && (const uint8_t*)d_ct < (const uint8_t*)d_out + ct_bytes)
    return fail(HE_EINVAL, "he_rotate: output aliases the input");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const LevelPlan& P = c->lv[level];
  PairDesc pd{};
  pd.ct1 = d_ct; pd.ct2 = d_ct; pd.out = nullptr; pd.r = nullptr; pd.plan = P.plan; pd.level = level;
  pd.rs = 0;
  pd.wrl = 1;
  pair_layout(c, level, ws, pd);
  pd.rl = d_out;  // holds (sigma(b), 0), then receives the rotated ciphertext
  const u64 g = galois_element(N, rot);
  const u64 tot = (u64)level * N;
  timed(c, "automorphism", (double)tot * 2, (double)tot * 4 * 8, st, [&] {
    hipLaunchKernelGGL(k_automorphism, dim3((u32)ceil_div(tot, 256)), dim3(256), 0, st, d_ct, d_out, pd.d2, g,
                       level, c->log_n);
  });
  const Common cm = make_common(c, d_rk);
  const TileCfg tc = default_tiles(c->log_n);
  auto run = [&](int s) {
    Batch b{};
    b.one = pd;
    b.npairs = 1;
    b.nitems = stage_items(s, c->log_n, level, c->K, c->alpha, P.beta, P.dt_limbs, false, true, tc);
    double ops = 0, bytes = 0;
    if (c->timing) stage_work(c, s, level, false, ops, bytes, true);
    launch_stage(c, s, cm, b, ops, bytes, st, tc);
  };
  run(ST_Y_IBLOCKS);
  for (int s = ST_Y_ICOLS; s < ST_COUNT; ++s) run(s);
  HIP_TRY(hipGetLastError());
  return HE_OK;
}

}  // extern "C"
