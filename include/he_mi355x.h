/*
 * he_mi355x.h -- C ABI of the MI355X (gfx950) full-RNS CKKS HE Mul library.
 *
 * Method: "HEAAN Demystified" (arXiv 2003.04510).  HE Mul = region 1 tensor
 * product of two ciphertexts, region 2 key switching with the evaluation key,
 * then rescale (Fig. 2, Sec. III-B; rescale by division, Sec. III-A), in the
 * full-RNS form the paper names in Table XI: NTT/iNTT (Algorithms 3-4) plus
 * mod up / mod down (fast base conversion, the Discussion section).
 *
 * Conventions (all functions):
 *   - N = 2^log_n.  Moduli are indexed 0..L-1 for q_0..q_{L-1} and L..L+K-1
 *     for the special primes p_0..p_{K-1}.  All primes are = 1 (mod 2N),
 *     distinct, and below 2^60.
 *   - A polynomial is uint64 [limbs][N], limb-major; every stored residue is
 *     canonical, in [0, modulus).
 *   - A ciphertext at level l (l = number of q-limbs present) is
 *     uint64 [2][l][N]: poly 0 = b (the paper's bx), poly 1 = a (ax), in NTT
 *     (evaluation) form, bit-reversed slot order.  Decryption: b - a*s.
 *   - The evaluation key is uint64 [dnum][2][L+K][N] in NTT form, digit j
 *     covering q_{j*alpha} .. q_{(j+1)*alpha-1}, alpha = ceil(L/dnum).
 *   - Pointers named d_* are DEVICE pointers owned by the caller (the
 *     library never frees them).  Host pointers are read before the call
 *     returns.  Work is enqueued asynchronously on `stream` (0 = the null
 *     stream); results are ready once the stream reaches that point.
 *   - `ws` is a caller-owned device workspace of at least the size returned
 *     by the matching *_workspace_bytes query; its contents on entry are
 *     ignored and on exit undefined.
 *   - Every function returns an he_status; on failure he_last_error()
 *     returns a thread-local message.  Argument errors are detected before
 *     any work is enqueued.  Device faults surface as HE_EDEVICE, possibly
 *     from a later call.
 */
#ifndef HE_MI355X_H
#define HE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum he_status {
  HE_OK = 0,
  HE_EINVAL = -1,        /* null pointer, bad size, unsupported parameter */
  HE_ELEVEL = -2,        /* level out of range or mismatched */
  HE_ENOMEM = -3,        /* workspace too small or device allocation failed */
  HE_EDEVICE = -4,       /* a HIP call failed */
  HE_EUNSUPPORTED = -5,  /* parameter combination not implemented */
  HE_EBUSY = -6          /* a bounded queue is full: retry after progress */
} he_status;

typedef struct he_ctx he_ctx;
typedef void* he_stream; /* a hipStream_t */

/* Primes for the RNS bases (Table III/VI of the paper give the prime-size
 * ranges; the choice "largest primes below 2^bits that are 1 mod 2N,
 * scanning downward" is this library's).  Writes `count` primes to `out`
 * (host), skipping any listed in `exclude` (host, may be NULL if
 * nexclude = 0).  HE_EINVAL if bits is not in [20, 61] or too few primes
 * exist. */
he_status he_gen_primes(uint32_t log_n, uint32_t bits, uint32_t count, const uint64_t* exclude,
                        uint32_t nexclude, uint64_t* out);

/* Create a context: moduli q (host, [L]) and p (host, [K]), dnum key-switch
 * digits.  Builds twiddle tables (powers of the smallest primitive 2N-th root
 * in bit-reversed order, with Shoup companions, Algorithms 2-3; for primes
 * below 2^50 also the two factors that the NTT's later stages multiply
 * together instead) and all base-conversion constants on device `device`.  The tables go to
 * d_tables, device memory of at least he_ctx_device_bytes(...) bytes that
 * the caller owns and keeps valid until he_ctx_destroy (HE_ENOMEM if
 * tables_bytes is smaller); with d_tables = NULL the context allocates them
 * itself and frees them in he_ctx_destroy.  Constraints: 12 <= log_n <= 17,
 * 1 <= dnum <= min(L, 64) (HE_EINVAL otherwise), digit size ceil(L/dnum)
 * <= 32 and K <= 32 (HE_EUNSUPPORTED above), L <= 64, K special primes
 * whose product exceeds every digit's product.  Synchronous (the tables are
 * uploaded before return). */
he_status he_ctx_create(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                        const uint64_t* p, int device, void* d_tables, size_t tables_bytes, he_ctx** out);
/* Device bytes of the tables he_ctx_create builds for these parameters (0 if
 * they are invalid); he_ctx_table_bytes: the same for an existing context. */
size_t he_ctx_device_bytes(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                           const uint64_t* p);
size_t he_ctx_table_bytes(const he_ctx* ctx);
void he_ctx_destroy(he_ctx* ctx);

/* 32-bit words: the paper's GPU choice of word size (Table VI, GPU column:
 * primes below 2^30, residues in 32-bit words; Sec. V-C).  A context made by
 * he_ctx_create_w32 (same arguments as he_ctx_create; every prime must be
 * below 2^31, HE_EINVAL otherwise; 12 <= log_n <= 16, HE_EUNSUPPORTED
 * above) stores every residue as a uint32_t:
 * ciphertexts are uint32 [2][level][N], the evaluation key uint32
 * [dnum][2][L+K][N], and he_ct_bytes / he_evk_bytes / he_workspace_bytes
 * count 4-byte words.  Such a context runs he_mul32 only; the other entry
 * points return HE_EUNSUPPORTED for it.  With every prime below 2^30 the
 * NTT butterflies run in 32-bit integer arithmetic (Shoup's product with a
 * 2^32-scaled companion on the 32-bit multipliers), else in exact FP64.
 * he_ctx_word_bytes: 8 or 4. */
he_status he_ctx_create_w32(uint32_t log_n, uint32_t L, uint32_t K, uint32_t dnum, const uint64_t* q,
                            const uint64_t* p, int device, void* d_tables, size_t tables_bytes, he_ctx** out);
uint32_t he_ctx_word_bytes(const he_ctx* ctx);

/* Sizes in bytes. */
size_t he_ct_bytes(const he_ctx* ctx, uint32_t level);      /* 2*level*N*8 */
size_t he_evk_bytes(const he_ctx* ctx);                     /* dnum*2*(L+K)*N*8 */
size_t he_pk_bytes(const he_ctx* ctx);                      /* 2*L*N*8 */
size_t he_workspace_bytes(const he_ctx* ctx, uint32_t level); /* for he_mul/he_rescale/keygen/... */

/* Key generation (Sec. III-A: pk from sk; evk encrypts a multiple of sk^2,
 * Fig. 2).  Random draws are inputs (host): s [N] ternary secret, e_pk [N],
 * e_evk [dnum][N] small signed errors, a_pk [L][N] and a_evk [dnum][L+K][N]
 * uniform residues (already NTT form, row i uniform mod modulus i).
 * Writes d_pk = (a*s + e, a) over q_0..q_{L-1} and, per digit j,
 * d_evk_j = (a_j*s + e_j + G_j*s^2, a_j) over all L+K moduli, where
 * G_j = [P]_{q_i} for q_i in digit j and 0 elsewhere (P = prod p_k).
 * Synchronous with respect to the host arrays (they are copied before
 * return). */
he_status he_keygen(he_ctx* ctx, const int64_t* s, const int64_t* e_pk, const uint64_t* a_pk,
                    const int64_t* e_evk, const uint64_t* a_evk, uint64_t* d_pk, uint64_t* d_evk,
                    void* ws, size_t ws_bytes, he_stream stream);

/* Public-key encryption at `level` (Sec. III-A): ct = (v*pk0 + e0 + m,
 * v*pk1 + e1).  m, v, e0, e1: host signed coefficient vectors [N]
 * (m = the encoded plaintext).  d_ct: [2][level][N]. */
he_status he_encrypt(he_ctx* ctx, uint32_t level, const int64_t* m, const int64_t* v,
                     const int64_t* e0, const int64_t* e1, const uint64_t* d_pk, uint64_t* d_ct,
                     void* ws, size_t ws_bytes, he_stream stream);

/* Encoding (Sec. III-A): n <= N/2 complex slots d_z [n][2] (re, im
 * doubles, device) times `scale`, placed at the roots zeta^(5^j) of
 * X^N + 1 (zeta = exp(i pi / N)) with their conjugates, to the integer
 * coefficients d_m [N] (int64, device) of the polynomial taking those
 * values, each rounded to nearest (ties to even); slots j >= n are zero.
 * ws: 16 N bytes (HE_ENOMEM if smaller).  Enqueued on `stream`. */
he_status he_encode(he_ctx* ctx, const double* d_z, uint32_t n, double scale, int64_t* d_m, void* ws,
                    size_t ws_bytes, he_stream stream);

/* Decoding (Sec. III-A), the inverse of he_encode: d_m [level][N] residues
 * of a plaintext in coefficient form (as he_decrypt writes them) -> n <= N/2
 * complex slots d_z [n][2] (doubles) = m(zeta^(5^j)) / scale, with m the
 * centred integer polynomial (mixed-radix reconstruction from the residues,
 * exact, then converted to double).  ws: 16 N + 8 level (level + 1) + 256
 * bytes.  Enqueued on `stream` (the small reconstruction tables are
 * uploaded synchronously). */
he_status he_decode(he_ctx* ctx, uint32_t level, const uint64_t* d_m, double scale, uint32_t n, double* d_z,
                    void* ws, size_t ws_bytes, he_stream stream);

/* HE Add (Sec. III-B): d_out = d_ct1 + d_ct2 limb by limb, all
 * [2][level][N] (d_out may alias an input).  Enqueued on `stream`. */
he_status he_add(he_ctx* ctx, uint32_t level, const uint64_t* d_ct1, const uint64_t* d_ct2, uint64_t* d_out,
                 he_stream stream);

/* Rotation by `rot` slots (slot j of the result holds slot j + rot): the
 * automorphism X -> X^g, g = 5^rot mod 2N, of both polynomials, then the
 * key switching of HE Mul (ModUp, inner product, ModDown) of sigma_g(a)
 * back to sk with the rotation key of `rot`.  d_ct, d_out: [2][level][N]
 * NTT form; d_out must not overlap d_ct (HE_EINVAL).  ws: he_workspace_bytes
 * (level) bytes.  Enqueued on `stream`. */
he_status he_rotate(he_ctx* ctx, uint32_t level, const uint64_t* d_ct, const uint64_t* d_rk, int32_t rot,
                    uint64_t* d_out, void* ws, size_t ws_bytes, he_stream stream);

/* Rotation key of `rot` (layout and gadget of the evaluation key,
 * [dnum][2][L+K][N]): b_j = a_j sk + e_j - G_j sigma_g(sk), so that key
 * switching sigma_g(a) returns a pair decrypting to -sigma_g(a) sigma_g(sk).
 * s: host [N]; e_rk: host [dnum][N]; a_rk: host [dnum][L+K][N] uniform
 * residues (NTT form).  Synchronizes `stream`. */
he_status he_keygen_rot(he_ctx* ctx, const int64_t* s, int32_t rot, const int64_t* e_rk, const uint64_t* a_rk,
                        uint64_t* d_rk, void* ws, size_t ws_bytes, he_stream stream);

/* Decryption to RNS coefficients (Sec. III-A: t = bx - ax*sk): writes
 * d_m [level][N], coefficient form, limb i modulo q_i.  s: host [N]. */
he_status he_decrypt(he_ctx* ctx, uint32_t level, const uint64_t* d_ct, const int64_t* s,
                     uint64_t* d_m, void* ws, size_t ws_bytes, he_stream stream);

/* HE Mul (Fig. 2): tensor product, key switching with evk (INTT, ModUp,
 * NTT, inner product, INTT, ModDown), then optionally rescale by the last
 * prime q_{level-1}.  d_ct1, d_ct2: [2][level][N].  d_relin: [2][level][N]
 * output after key switching (may be NULL).  d_out: [2][level-1][N] output
 * after rescale (may be NULL; requires level >= 2).  At least one output.
 * Outputs must not alias inputs.  HE_ELEVEL if level is 0 or > L. */
he_status he_mul(he_ctx* ctx, uint32_t level, const uint64_t* d_ct1, const uint64_t* d_ct2,
                 const uint64_t* d_evk, uint64_t* d_relin, uint64_t* d_out, void* ws,
                 size_t ws_bytes, he_stream stream);

/* HE Mul without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same computation, arguments and errors as he_mul, but the
 * workspace is a scratch array of HE_NOALLOC_SCRATCH_BYTES (64 MiB) that the
 * library holds per GPU until the process ends; the call allocates nothing.
 * HE_ENOMEM when he_mul_noalloc_bytes(ctx, level) exceeds it (it fits every
 * level at N <= 2^15 with L <= 12, and N = 2^16 up to level 8 with K = 8).
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on the same GPU (different streams, host threads) race and must not be
 * issued; calls ordered on one stream are safe.  The scratch's contents on
 * entry are ignored. */
#define HE_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t he_mul_noalloc_bytes(const he_ctx* ctx, uint32_t level);
he_status he_mul_noalloc(he_ctx* ctx, uint32_t level, const uint64_t* d_ct1, const uint64_t* d_ct2,
                         const uint64_t* d_evk, uint64_t* d_relin, uint64_t* d_out, he_stream stream);

/* HE Mul of a 32-bit-word context (he_ctx_create_w32): the computation,
 * arguments, outputs and errors of he_mul on uint32 words; the results are
 * the same residues he_mul gives for the same primes on 64-bit words.
 * HE_EUNSUPPORTED for a 64-bit-word context. */
he_status he_mul32(he_ctx* ctx, uint32_t level, const uint32_t* d_ct1, const uint32_t* d_ct2, const uint32_t* d_evk,
                   uint32_t* d_relin, uint32_t* d_out, void* ws, size_t ws_bytes, he_stream stream);

/* Batched HE Mul: many independent products (each with its own level) of
 * one context executed as one sequence of stage kernels, each kernel
 * covering the work of every pair (the batch analogue of he_mul; the
 * paper's GPU mapping spreads one function's independent work over the
 * whole device, Sec. V-C).  Item i: level, operands ct1, ct2
 * [2][level][N], outputs relin [2][level][N] (may be NULL) and out
 * [2][level-1][N] (may be NULL, needs level >= 2); at least one output.
 * Outputs must not alias inputs or each other's buffers.
 *
 * he_batch_workspace_bytes: workspace for the items (0 if a level is out of
 * range).  he_batch_create: validates the items, lays out the workspace
 * `ws` (device, caller-owned, must stay valid for the batch's lifetime) and
 * uploads descriptors (device memory owned by the batch).  he_mul_batch:
 * enqueues the batched HE Mul on `stream`; with use_graph != 0 the kernel
 * sequence is captured once into a HIP graph (re-captured if evk changes)
 * and replayed as a single launch.  The buffers named at creation are read
 * and written at execution time, so new operand values may be written into
 * them between calls.  he_batch_destroy frees the batch (not the buffers). */
typedef struct he_batch he_batch;
typedef struct he_batch_item {
  uint32_t level;
  const uint64_t* ct1;
  const uint64_t* ct2;
  uint64_t* relin;
  uint64_t* out;
} he_batch_item;
size_t he_batch_workspace_bytes(const he_ctx* ctx, const he_batch_item* items, uint32_t n);
he_status he_batch_create(he_ctx* ctx, const he_batch_item* items, uint32_t n, void* ws, size_t ws_bytes,
                          he_batch** out);
he_status he_mul_batch(he_ctx* ctx, he_batch* batch, const uint64_t* d_evk, int use_graph, he_stream stream);
/* As he_batch_create, but the descriptors go to caller-provided device
 * memory d_desc (at least he_batch_desc_bytes(n) bytes) through an
 * asynchronous copy on `stream` (no device allocation, no host
 * synchronization); the batch must then run on that same stream, and
 * d_desc must not be reused until the batch's work has finished. */
size_t he_batch_desc_bytes(uint32_t n);
he_status he_batch_create_async(he_ctx* ctx, const he_batch_item* items, uint32_t n, void* ws, size_t ws_bytes,
                                void* d_desc, size_t desc_bytes, he_stream stream, he_batch** out);
void he_batch_destroy(he_batch* batch);

/* Batch schedule (no paper passage: an implementation choice of how the
 * batch's work is laid on the device).  cols_tile / blocks_tile: elements
 * per workgroup of the NTT "cols" / "blocks" passes (defaults 4096 / 2048,
 * at N = 2^16 4096 / 1024; there any of cols 2048 / 4096 with blocks
 * 1024 / 2048).  chunks (1..8, at most the pair count):
 * the pairs are split into that many contiguous groups of about equal total
 * level; their stage sequences alternate between the batch's stream and a
 * side stream the batch owns, so stages of different groups overlap; a
 * captured graph keeps that structure.  Results are identical under every
 * schedule.  ip_fused (0..4): for the pairs of at least ip_fused key-switching
 * digits (0: none), run the mod-up NTT blocks pass, the evk inner product and
 * the special limbs' INTT blocks pass as one fused pass (less HBM traffic,
 * longer dependency chains per workgroup) instead of the separate launches;
 * it runs one digit per wavefront of a 4-wave workgroup, so dnum <= 4, and
 * pairs of fewer digits leave waves idle in its NTT phase.
 * radix: the register radix of the NTT passes' butterfly rounds (the paper
 * sweeps the NTT radix, Table IX): 0 or the default (8 for the 256-point
 * sub-transforms at N = 2^16) or, at N = 2^16, 16 (two radix-16 rounds, one
 * LDS exchange fewer, half the waves).
 *
 * he_batch_set_sched: validates (HE_EUNSUPPORTED for tiles not available at
 * this ring degree or the fused pass with dnum > 4, HE_EINVAL for a bad
 * chunk count), re-uploads the item
 * offsets on `stream` and waits for it, drops a captured graph.
 * he_batch_get_sched: the current schedule.
 * he_batch_autotune: runs the batch (overwriting its outputs with the same
 * values) as a graph `reps` times under each candidate schedule -- every
 * available tile pair and radix with one chunk, then the best of those with
 * the fused inner product for the pairs of at least 1, 2, 3 digits
 * (dnum <= 4), then the best so far with 2 and 4 chunks --
 * times each with HIP events on `stream`, and installs the
 * fastest; *best and *best_ms (may be NULL) receive it and its time per
 * replay.  Synchronizes `stream`. */
typedef struct he_batch_sched {
  uint32_t cols_tile;
  uint32_t blocks_tile;
  uint32_t chunks;
  uint32_t ip_fused;
  uint32_t radix;  /* register radix of the NTT passes: 0 = the default (reported as its value), 16 at N = 2^16 */
} he_batch_sched;
he_status he_batch_set_sched(he_batch* batch, const he_batch_sched* sched, he_stream stream);
he_status he_batch_get_sched(const he_batch* batch, he_batch_sched* sched);
he_status he_batch_autotune(he_ctx* ctx, he_batch* batch, const uint64_t* d_evk, uint32_t reps, he_stream stream,
                            he_batch_sched* best, double* best_ms);

/* Batch groups: batches of different contexts (ring sizes, levels, keys) on
 * one device run as one unit, each batch's stage kernels on a stream of its
 * own (batch 0 on `stream`, the others on streams the group owns, forked
 * from and joined back to `stream` by events), so the rings overlap on the
 * device; with use_graph != 0 the whole group is captured once into one HIP
 * graph (recaptured when an evaluation key pointer changes) and replayed as
 * a single launch.  d_evks[i] is batch i's evaluation key.  Every batch
 * must run in one chunk (HE_EUNSUPPORTED at creation otherwise: the group
 * already runs the rings side by side), and a batch whose schedule changed
 * after the group was made is refused (HE_EUNSUPPORTED): make a new group.
 * The batches must outlive the group; destroying the group does not
 * destroy them.  (No paper passage: an implementation choice of
 * how independent HE Muls share the device, as the paper's GPU mapping
 * spreads independent work over the device, Sec. V-C.) */
typedef struct he_batch_group he_batch_group;
he_status he_batch_group_create(he_batch* const* batches, uint32_t n, he_batch_group** out);
he_status he_mul_batch_group(he_batch_group* group, const uint64_t* const* d_evks, int use_graph, he_stream stream);
void he_batch_group_destroy(he_batch_group* group);

/* Serving: a request loop with continuous batching (host side, native).
 * he_server_add_ring registers a context with its resident evk and a
 * caller-owned device arena d_arena of arena_bytes (256-byte aligned; its
 * first he_server_arena_min_bytes(cfg) bytes hold batch descriptors, the
 * rest request workspaces).  Admission by HBM footprint: a ring counts its
 * context tables (he_ctx_table_bytes), its evk (he_evk_bytes) and its arena,
 * and the rings together must stay within cfg->hbm_budget (HE_ENOMEM);
 * a request runs only when its workspace fits the free part of its ring's
 * arena.  he_server_submit queues one HE Mul with rescale (level >= 2) on
 * operands ct1, ct2 [2][level][N] into out [2][level-1][N] (device buffers
 * owned by the caller, untouched until the request completes); the arrival
 * time is taken at submission; HE_EBUSY when the ring already holds
 * cfg->max_queue queued requests (0 = unbounded).
 * The server runs on streams of its own that do not wait for any caller
 * stream: ct1 and ct2 must hold their final values when submitted (for
 * example, the caller synchronized the stream that wrote them), and the
 * caller keeps all three buffers alive until poll returns the request.
 * he_server_progress never blocks: it retires batches whose work finished
 * and, per ring, admits queued requests in arrival order while their
 * workspace fits the arena and at most max_batch per batch, launching each
 * group as one batched HE Mul on the ring's stream while at most
 * max_inflight batches of that ring are in flight.  While a batch of the
 * ring is in flight, a group smaller than max_batch is held back until its
 * oldest request has waited hold_us microseconds (0: no hold), so that
 * arrivals coalesce into fuller batches.  he_server_poll returns completed
 * request ids with their latency (seconds from submission to the moment
 * progress observed completion).  Errors are he_status codes; a failed
 * launch leaves the request queue untouched.  The server never allocates
 * device memory. */
typedef struct he_server he_server;
typedef struct he_server_cfg {
  size_t hbm_budget;     /* bytes of tables + evks + arenas over all rings */
  uint32_t max_batch;    /* requests per batch */
  uint32_t max_inflight; /* batches in flight per ring */
  uint32_t max_queue;    /* queued requests per ring before HE_EBUSY (0 = no limit) */
  uint32_t hold_us;      /* coalescing hold while the ring is busy (0 = none) */
} he_server_cfg;
he_status he_server_create(const he_server_cfg* cfg, he_server** out);
size_t he_server_arena_min_bytes(const he_server_cfg* cfg);
he_status he_server_add_ring(he_server* srv, he_ctx* ctx, const uint64_t* d_evk, void* d_arena, size_t arena_bytes,
                             uint32_t* ring_id);
he_status he_server_submit(he_server* srv, uint32_t ring, uint64_t id, uint32_t level, const uint64_t* d_ct1,
                           const uint64_t* d_ct2, uint64_t* d_out);
he_status he_server_progress(he_server* srv, uint32_t* launched);
he_status he_server_poll(he_server* srv, uint64_t* ids, double* latency_s, uint32_t max, uint32_t* n);
he_status he_server_stats(const he_server* srv, uint64_t* queued, uint64_t* inflight, uint64_t* batches,
                          uint64_t* completed);
void he_server_destroy(he_server* srv);

/* Rescale (Sec. III-A, division by the last prime, rounded to nearest):
 * d_in [2][level][N] -> d_out [2][level-1][N].  level >= 2.  d_out and the
 * workspace must not overlap d_in or each other (HE_EINVAL): the kernels
 * read input limbs while other workgroups write output limbs. */
he_status he_rescale(he_ctx* ctx, uint32_t level, const uint64_t* d_in, uint64_t* d_out, void* ws,
                     size_t ws_bytes, he_stream stream);

/* Ciphertext descriptors.  A ciphertext carries its level and its scale
 * (Sec. III-A: a message m is encrypted as the integer polynomial of
 * m * scale; a product has scale a.scale * b.scale, and rescaling by the
 * dropped prime q_{level-1} divides the scale by that prime).  `data` is
 * device memory [2][level][N] owned by the caller; the scale is metadata
 * computed in double precision. */
typedef struct he_ct {
  uint64_t* data;
  uint32_t level;
  double scale;
} he_ct;

/* Import raw residues: host [2][level][N] (every residue of limb i below
 * q_i, HE_EINVAL otherwise) into ct->data (device, preset by the caller);
 * sets ct->level and ct->scale.  Synchronizes `stream`. */
he_status he_ct_import(he_ctx* ctx, const uint64_t* host, uint32_t level, double scale, he_ct* ct,
                       he_stream stream);
/* Export ct's residues to host [2][ct->level][N].  Synchronizes `stream`. */
he_status he_ct_export(he_ctx* ctx, const he_ct* ct, uint64_t* host, he_stream stream);
/* he_mul on descriptors: a->level must equal b->level (HE_ELEVEL; the paper
 * multiplies ciphertexts under the same modulus).  relin and out (either may
 * be NULL, not both) name caller-owned data; on success relin gets level
 * a->level and scale a->scale * b->scale, out level a->level - 1 and that
 * scale divided by q_{level-1}.  Errors and workspace as he_mul. */
he_status he_mul_ct(he_ctx* ctx, const uint64_t* d_evk, const he_ct* a, const he_ct* b, he_ct* relin, he_ct* out,
                    void* ws, size_t ws_bytes, he_stream stream);
/* he_rescale on descriptors: out gets level in->level - 1 and scale
 * in->scale / q_{in->level - 1}. */
he_status he_rescale_ct(he_ctx* ctx, const he_ct* in, he_ct* out, void* ws, size_t ws_bytes, he_stream stream);

/* Negacyclic NTT (Algorithm 3) or its inverse of `nlimbs` limbs in place:
 * limb r is taken modulo modulus index first_mod + r.  Output order is
 * bit-reversed (forward) / natural (inverse). */
he_status he_ntt(he_ctx* ctx, uint64_t* d_data, uint32_t nlimbs, uint32_t first_mod, int inverse,
                 he_stream stream);

/* Parameters of a context (any pointer may be NULL). */
he_status he_ctx_info(const he_ctx* ctx, uint32_t* log_n, uint32_t* L, uint32_t* K, uint32_t* dnum,
                      uint64_t* moduli /* [L+K] or NULL */);

/* Diagnostics: per-kernel timing.  While enabled, every kernel the library
 * launches (or only those whose kind equals `only`, when non-NULL and
 * non-empty) is bracketed by two HIP events on its stream, together with the
 * kernel's algorithmic work: `ops` (butterflies for NTT passes, 64x64-bit
 * multiply-accumulates for base conversion and the inner product, modular
 * products for element-wise kernels) and `bytes` (limbs read + written x 8N,
 * tables excluded).  he_timing_read -- after the streams involved are
 * synchronized -- aggregates the recorded launches per kernel kind into
 * `out` (up to `max` entries), sets *n to the number of kinds, and clears
 * the record. */
typedef struct he_kernel_stat {
  char name[48];
  uint32_t launches;
  double ms;
  double ops;
  double bytes;
} he_kernel_stat;
he_status he_timing_enable(he_ctx* ctx, int enable, const char* only);
he_status he_timing_read(he_ctx* ctx, he_kernel_stat* out, uint32_t max, uint32_t* n);

/* ---------------------------------------------------------------------------
 * The paper's own (non-RNS) HE Mul: HEAAN with power-of-two moduli
 * (Sec. II-III, Fig. 2).  A ciphertext at level q = 2^logq is (bx, ax), two
 * polynomials of N big-integer coefficients in [0, q); the evaluation key is
 * (evk.bx, evk.ax) modulo Q^2 (Q = 2^logQ).  HE Mul runs five polynomial
 * products through RNS: region 1 (ax1+bx1)(ax2+bx2), ax1 ax2, bx1 bx2 modulo
 * q over np1 primes; region 2 ax1 ax2 times evk.bx and evk.ax over np2
 * primes, shifted right by log Q with rounding (round half up); then
 *   ax3 = ks_ax + axbx - axax - bxbx,  bx3 = ks_bx + bxbx   (mod q)
 * and optionally the rescale round(c3 / 2^logp) (Sec. II-A).  Each product
 * is CRT (Sec. IV-A, matrix form), NTT, element-wise product, inverse NTT
 * and iCRT (Algorithm 6, matrix form).
 *
 * Layout: a big-integer polynomial is [W][N] little-endian uint64 words,
 * W = ceil(logQ / 64) (words above logq zero); a ciphertext is [2][W][N]
 * (bx, ax).  The evaluation key is [2][W2][N], W2 = ceil(2 logQ / 64).
 * All pointers named d_* are device memory the caller owns. */
typedef struct he_big_ctx he_big_ctx;

/* Context for ring degree 2^log_n (12..17) and log Q in [64, 1216]: picks
 * the region primes (60-bit, 1 mod 2N; np1 of them cover 2 log Q + log N + 3
 * bits, np2 cover 3 log Q + log N + 3 bits) and uploads NTT, CRT and iCRT
 * tables to `device`.  HE_EUNSUPPORTED outside those ranges. */
he_status he_big_ctx_create(uint32_t log_n, uint32_t logQ, int device, he_big_ctx** out);
void he_big_ctx_destroy(he_big_ctx* ctx);
/* np1, np2, words per coefficient W, and the np2 primes (any may be NULL). */
he_status he_big_info(const he_big_ctx* ctx, uint32_t* np1, uint32_t* np2, uint32_t* words, uint64_t* primes);
size_t he_big_ct_bytes(const he_big_ctx* ctx);        /* 2*W*N*8 */
size_t he_big_evk_bytes(const he_big_ctx* ctx);       /* 2*W2*N*8 */
size_t he_big_evk_ntt_bytes(const he_big_ctx* ctx);   /* 2*np2*N*8 */
size_t he_big_workspace_bytes(const he_big_ctx* ctx); /* for he_big_mul */

/* One-time key preparation (the key's CRT and NTT, Fig. 2 region 2):
 * d_evk [2][W2][N] (coefficients below Q^2) -> d_evk_ntt [2][np2][N], the NTT
 * form over the np2 primes.  Enqueued on `stream`. */
he_status he_big_evk_prepare(he_big_ctx* ctx, const uint64_t* d_evk, uint64_t* d_evk_ntt, he_stream stream);

/* HE Mul at level q = 2^logq (1 <= logq <= log Q): d_ct1, d_ct2 [2][W][N]
 * with coefficients below 2^logq; d_evk_ntt from he_big_evk_prepare.  Writes
 * c3 to d_out [2][W][N], or, when logp > 0, the rescaled c3 at level
 * 2^(logq - logp) (logp < logq, logp <= 63).  d_out must not overlap the
 * inputs (HE_EINVAL).  ws: he_big_workspace_bytes bytes (HE_ENOMEM if
 * smaller).  Enqueued on `stream`; asynchronous. */
he_status he_big_mul(he_big_ctx* ctx, uint32_t logq, const uint64_t* d_ct1, const uint64_t* d_ct2,
                     const uint64_t* d_evk_ntt, uint64_t* d_out, uint32_t logp, void* ws, size_t ws_bytes,
                     he_stream stream);

/* Per-kernel timing of the big-integer path (as he_timing_*): kinds
 * big_crt, ntt_cols / ntt_blocks (NTT), intt_blocks / intt_cols (iNTT),
 * big_icrt, big_pointwise and big_finish (element-wise work). */
he_status he_big_timing_enable(he_big_ctx* ctx, int enable);
he_status he_big_timing_read(he_big_ctx* ctx, he_kernel_stat* out, uint32_t max, uint32_t* n);

/* Diagnostics: measured issue rates of the vector ALU instructions the HE
 * Mul is made of, in lane-operations per second over the whole device
 * `device`: rates[0] v_mad_u64_u32 (32x32+64-bit multiply-add, the 64-bit
 * modular products' building block), rates[1] v_mul_hi_u32, rates[2]
 * v_mul_lo_u32, rates[3] v_fma_f64 (the FP64 butterflies), rates[4] a
 * full-rate 32-bit integer instruction (v_lshl_add_u32).  Each kind runs
 * `blocks` workgroups of 256 threads, 8 independent chains of `iters`
 * instructions per thread; the best of 4 timed launches counts.  The
 * measured peaks the per-stage VALU fractions are taken against.
 * Allocates and frees a small sink buffer; synchronizes `stream`. */
he_status he_valu_peaks(int device, uint32_t blocks, uint32_t iters, double* rates, he_stream stream);

const char* he_status_str(he_status s);
const char* he_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
