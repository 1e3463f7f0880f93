/*
 * secpe.h -- C ABI of the MI355X (gfx950) encrypted-Argmax library.
 *
 * Paper: "SecPE: Secure Prompt Ensembling for Private and Robust Large
 * Language Models", arXiv 2502.00847.
 *
 * The library evaluates the paper's private voting step (Sec. 3.1, step 3)
 * under RNS-CKKS (Sec. 2.2): the server sums the encrypted per-prompt scores
 * and turns the sum y* into an encrypted one-hot vector z with
 * z_i = Sign(y_i - y_max) + 1 (Sec. 3.2, Eq. 2), y_max from Algorithm 1's
 * QuickMax, Sign = f^{d_f}(g^{d_g}(x)) (Eq. 4), Max from Eq. 6 and inputs
 * normalised by Eq. 5.  The client encrypts (step 1) and decrypts (step 4).
 *
 * Memory.  Every buffer passed as 'void* ..._dev' is device memory owned by
 * the caller, sized with the secpe_*_bytes queries.  The library owns only its
 * opaque context: parameter tables on the device, a descriptor arena and a
 * small client scratch buffer, all released by secpe_ctx_destroy.
 *
 * Layouts.  A residue is an exact integer held in an IEEE binary64 (all primes
 * are below 2^51).  A polynomial limb is N residues; a ciphertext buffer is
 * [2][n_q][N] doubles (polynomial c0, then c1, each with room for all n_q chain
 * limbs), stored in the NTT domain; limbs above the ciphertext's level are
 * unused.  The secret key is [n_q + n_p][N] (NTT domain).  A switching key is
 * [dnum][2][n_q + n_p][N] (NTT domain), dnum = ceil(n_q / n_p).
 *
 * Errors.  Functions return SECPE_OK (0) or a negative code; secpe_last_error
 * returns a thread-local message.  Argument errors are reported before any
 * work is queued.  Work is asynchronous on the context's stream unless stated;
 * device faults surface at the next synchronising call (secpe_sync and the
 * functions that return host data).
 */
#ifndef SECPE_H
#define SECPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SECPE_OK = 0,
  SECPE_EINVAL = -1,   /* bad argument or parameter set */
  SECPE_ENOMEM = -2,   /* workspace or device allocation too small / failed */
  SECPE_ENOLEVEL = -3, /* the modulus chain is exhausted and neither a key owner nor bootstrapping can refresh */
  SECPE_ENOKEY = -4,   /* no switching key for a needed rotation */
  SECPE_EDEVICE = -5   /* a HIP call failed */
};

/* CKKS parameters (Sec. 2.2; Sec. 4.1 gives N = 2^16).
   n_q chain primes = 1 mod 2N nearest 2^q_bits (alternately the next below
   and the next above), n_p special primes: the largest = 1 mod 2N below 2^p_bits.
   Key switching is hybrid with digits of alpha = n_p consecutive chain primes.
   Scale 2^log_scale.  Sign = f^df(g^dg(x)).  min_level: lowest level a
   ciphertext may reach (decryption needs two limbs, so 1).  refresh_level:
   level at which the refresh stand-in for bootstrapping re-encrypts (the
   paper's bootstrapping leaves K = 14 levels, Sec. 4.1); 0 = the top level. */
typedef struct secpe_params {
  int log_n, n_q, q_bits, n_p, p_bits, log_scale, dg, df, min_level, refresh_level;
} secpe_params;

/* A ciphertext: device buffer (layout above), its level and its scale. */
typedef struct secpe_ct {
  void* data;
  int level;
  double scale;
} secpe_ct;

typedef struct secpe_ctx secpe_ctx;

const char* secpe_last_error(void);
/* A fixed description of a status code (never NULL). */
const char* secpe_strerror(int code);

/* Create a context on HIP device 'device', issuing work on 'stream' (a
   hipStream_t; NULL = the null stream).  Builds primes and device tables. */
int secpe_ctx_create(const secpe_params* params, int device, void* stream, secpe_ctx** out);
void secpe_ctx_destroy(secpe_ctx* ctx);

/* Moduli: n_q chain primes then n_p special primes.  Returns the count; writes
   at most 'cap' values. */
int secpe_primes(const secpe_ctx* ctx, uint64_t* out, int cap);
int secpe_slots(const secpe_ctx* ctx);
size_t secpe_ct_bytes(const secpe_ctx* ctx);
size_t secpe_sk_bytes(const secpe_ctx* ctx);
size_t secpe_key_bytes(const secpe_ctx* ctx);

/* Galois element 5^step mod 2N of RotL(step) (Sec. 2.2, RotL / RotR). */
uint64_t secpe_galois_elt(const secpe_ctx* ctx, int64_t step);

/* Rotation amounts Algorithm 1 needs for every K <= k_max, C <= c_max: the
   prompt sum C'*2^i, RotR(C') = RotL(slots - C') and QuickMax 2^i.  Returns
   the count; writes at most 'cap'. */
int secpe_argmax_steps(const secpe_ctx* ctx, int k_max, int c_max, int64_t* out, int cap);

/* Key generation (client).  Samples the ternary secret from 'seed' into
   sk_dev, then 1 + n_steps switching keys into evk_dev: key 0 relinearises
   s^2 -> s, key 1+i rotates by steps[i] (sigma_g(s) -> s).  The context
   records which key serves which Galois element; evk_dev must stay alive while
   the context evaluates.  Synchronous. */
int secpe_keygen(secpe_ctx* ctx, uint64_t seed, const int64_t* steps, int n_steps, void* sk_dev, void* evk_dev);

/* Let dst evaluate with the switching keys src holds (no copy: the device
   buffers given to src's secpe_keygen must outlive both).  Only public
   switching keys are shared; no context ever holds a secret.  Both contexts
   need the same parameters on the same device; each keeps its own stream, so
   one user's requests can run on several streams at once (one server per
   context).  Bootstrapping keys are not shared. */
int secpe_keys_share(secpe_ctx* dst, const secpe_ctx* src);

/* ---- the key owner (Sec. 3.1: only the user holds the secret key; the
   server evaluates without it).  The paper refreshes exhausted ciphertexts by
   bootstrapping (Sec. 2.2; Sec. 4.1), which needs no secret.  Without
   bootstrapping, this library can instead refresh on the key owner's behalf:
   decrypt, lift the message exactly and re-encrypt with fresh randomness (an
   interactive stand-in in which the key owner takes part in the evaluation).
   A key owner handle names the secret for that purpose.  It is passed to
   each evaluation that may refresh and is never stored by a context; an
   evaluation given NULL (and not bootstrapping) stops with SECPE_ENOLEVEL at
   its first refresh point, before any work is queued.  The handle refers to
   sk_dev (caller-owned, it must outlive every evaluation given the handle)
   and to the context's parameters and device; it holds no device memory. ---- */
typedef struct secpe_key_owner secpe_key_owner;
int secpe_key_owner_create(const secpe_ctx* ctx, const void* sk_dev, secpe_key_owner** out);
void secpe_key_owner_destroy(secpe_key_owner* owner);

/* Client encryption of a K x C block of logits (row k = prompt k) at the top
   level with scale 2^log_scale.  Slot k*C' + c holds logits[k*C + c],
   C' = next power of two >= C (Sec. 3.2, Eq. 1).  out->data is caller memory
   of secpe_ct_bytes; level and scale are written. */
int secpe_encrypt(secpe_ctx* ctx, const void* sk_dev, const double* logits, int K, int C, uint64_t seed, secpe_ct* out);

/* Client encryption of an integer plaintext polynomial m[N] (coefficients). */
int secpe_encrypt_coeffs(secpe_ctx* ctx, const void* sk_dev, const int64_t* m, double scale, uint64_t seed, secpe_ct* out);

/* Client decryption: z_j for slots j < nslots (FP64) and the index of the
   largest (lowest on ties).  Synchronous. */
int secpe_decrypt(secpe_ctx* ctx, const void* sk_dev, const secpe_ct* ct, int nslots, double* z_out, int* argmax_out);

/* Decrypted integer message m[N] (centred, from limbs 0 and 1). Synchronous. */
int secpe_decrypt_coeffs(secpe_ctx* ctx, const void* sk_dev, const secpe_ct* ct, int64_t* m_out);

/* Workspace bytes for one evaluation of n queries with the given shapes. */
size_t secpe_workspace_bytes(secpe_ctx* ctx, int n, const int* K, const int* C);

/* The encrypted Argmax (Algorithm 1) of one query: prompt sum by doubling
   (Sec. 3.2, "applies to all associative operations"), normalisation with the
   public bounds d_min, d_max (Eq. 5), duplication, QuickMax with Eq. 6, then
   Sign(y - y_max) + 1 (Eq. 2).  'in' is read only.  owner: the key owner
   for the refresh stand-in, or NULL (then SECPE_ENOLEVEL where a refresh is
   needed, unless bootstrapping refreshes); refresh_seed keys the randomness
   of the refresh.  Asynchronous. */
int secpe_eval_argmax(secpe_ctx* ctx, const secpe_key_owner* owner, const secpe_ct* in, int K, int C, double d_min,
                      double d_max, uint64_t refresh_seed, void* ws_dev, size_t ws_bytes, secpe_ct* out);

/* Many queries of uneven (K, C) at once: every step of every query is issued
   in batched kernels (one launch per step kind for all queries at it).
   flags: SECPE_GRAPH captures the launches in a hipGraph and replays it on
   later calls with identical arguments (key owner included); keygen, key
   sharing, bootstrapping set-up and the autotuner discard captured graphs.
   Results are bit-identical to one query at a time.  Asynchronous. */
#define SECPE_GRAPH 1
int secpe_eval_argmax_batch(secpe_ctx* ctx, const secpe_key_owner* owner, int n, const secpe_ct* in, const int* K,
                            const int* C, const double* d_min, const double* d_max, const uint64_t* refresh_seed,
                            void* ws_dev, size_t ws_bytes, secpe_ct* out, int flags);

/* ---- the Argmax for callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc.  The evaluation of secpe_eval_argmax (same kernels, bit-identical
   results) with its workspace and descriptor arena in a device-global scratch
   array of SECPE_NOALLOC_SCRATCH_BYTES on each GPU (held from the library's
   load to the end of the process; its address is looked up once per device
   by secpe_ctx_create) and its descriptors staged through the context's
   pinned buffer of SECPE_NOALLOC_BLOB_BYTES (allocated by secpe_ctx_create).
   The call allocates nothing; an evaluation whose workspace and descriptors
   exceed the scratch, or whose descriptors exceed the staging buffer, fails
   with SECPE_ENOMEM before any work is queued (a config-2 query at N = 2^16
   needs 401 MiB and fits).  Every call on a GPU uses that GPU's one array: calls that overlap
   on one GPU (on other streams or other contexts) race, and the caller must
   order them; consecutive calls on one stream are ordered by the stream.
   Nothing in the scratch needs to start at zero: an evaluation reads only
   words it has written.  in, out and the key owner are as in
   secpe_eval_argmax.  Asynchronous. ---- */
#define SECPE_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
#define SECPE_NOALLOC_BLOB_BYTES ((size_t)8 << 20)
int secpe_eval_argmax_noalloc(secpe_ctx* ctx, const secpe_key_owner* owner, const secpe_ct* in, int K, int C,
                              double d_min, double d_max, uint64_t refresh_seed, secpe_ct* out);

/* ---- slot-packed Argmax (Sec. 3.2: N/(2n) Argmax inputs share one
   ciphertext).  A group of queries of shapes (K_b, C_b) is laid out in
   blocks of B = max(K'C', 2C') slots, K' and C' the largest padded shape of
   the group: query b at slot b*B + k*C' + c.  Every block runs Algorithm 1
   with the group's K', C' (padded classes get the normalised minimum 0, so
   they never win) and Eq. 5 with its own bounds; one evaluation serves the
   whole group. ---- */
/* Writes {K', C', B} to out3; returns the number of blocks a ciphertext holds
   (or a negative error). */
int secpe_packed_shape(secpe_ctx* ctx, int n, const int* K, const int* C, int* out3);
/* Client encryption of n queries in one ciphertext; logits: the K_b x C_b
   blocks concatenated (row k = prompt k). */
int secpe_encrypt_packed(secpe_ctx* ctx, const void* sk_dev, int n, const double* logits, const int* K, const int* C,
                         uint64_t seed, secpe_ct* out);
/* Workspace bytes for one evaluation of n packed ciphertexts; n_blocks[i]
   queries in ciphertext i, their K and C concatenated. */
size_t secpe_packed_workspace_bytes(secpe_ctx* ctx, int n, const int* n_blocks, const int* K, const int* C);
/* Evaluate n packed ciphertexts (batched like secpe_eval_argmax_batch); the
   per-block K, C, d_min, d_max are concatenated over the ciphertexts; one
   refresh seed per ciphertext.  Decrypt block b of a result with
   secpe_decrypt over nslots = n_blocks * B and read slots [b*B, b*B + C_b).
   Asynchronous. */
int secpe_eval_argmax_packed(secpe_ctx* ctx, const secpe_key_owner* owner, int n, const secpe_ct* in,
                             const int* n_blocks, const int* K, const int* C, const double* d_min, const double* d_max,
                             const uint64_t* refresh_seed, void* ws_dev, size_t ws_bytes, secpe_ct* out);

/* ---- the comparison path the paper measures against (Phoenix, Sec. 3.2):
   after the prompt sum and Eq. 5, every class is compared with each of the
   other C-1 (s = sum_i Sign(y - RotL(y, i)), y duplicated at offset C), and
   z = (Sign((s - (C-2)) / (2C-3)) + 1) / 2.  C Signs and C rotations against
   Algorithm 1's log C' + 1.  The comparisons run in the same launches.
   Needs the rotation keys of secpe_phoenix_steps; 2 <= C < 512. ---- */
int secpe_phoenix_steps(const secpe_ctx* ctx, int k_max, int C, int64_t* out, int cap);
size_t secpe_phoenix_workspace_bytes(secpe_ctx* ctx, int K, int C);
int secpe_eval_argmax_phoenix(secpe_ctx* ctx, const secpe_key_owner* owner, const secpe_ct* in, int K, int C,
                              double d_min, double d_max, uint64_t refresh_seed, void* ws_dev, size_t ws_bytes,
                              secpe_ct* out);

/* ---- Bootstrapping (Sec. 2.2; Sec. 4.1: the paper refreshes by
   bootstrapping, K = 14 of L = 35 levels, and gives no further steps).  The
   pipeline: one constant product takes the level-1 input to level 0 at scale
   T_b = q_0 2^-ratio; ModRaise lifts the centred level-0 residues to every
   chain prime (declared scale q_0); CoeffToSlot (groups of merged radix-2
   stages of the special FFT, each one level, baby-step giant-step diagonals);
   a conjugation splits real and imaginary parts; EvalMod on both (Chebyshev
   interpolant of cos(2 pi (x - 1/4) / 2^r) on |x| <= K + 1, then r double
   angles); recombination; SlotToCoeff with 2^ratio / (2 pi) folded in.  The
   output carries scale 2^log_scale at level
     n_q - 1 - (2 groups + log2(deg + 1) + 1 + r).
   Inputs need |slot value| <= 1 (the sine is read as its argument).

   The sparse-slot bootstrap (sparse_slots = n > 0) keeps slots [0, n) only,
   for ciphertexts whose other slots are never read again (the single-query
   Argmax reads slots [0, 2C') after Eq. 5): the mask of slots [0, n) takes
   the place of the scale-down constant; a trace at level 0 (sum of RotL by
   n, 2n, ..., N/4) makes the message n-periodic; after ModRaise the trace
   again; the n-slot special FFT as CoeffToSlot, its last group writing
   [w, 0] with period 2n; [re, im] = (w + conj w) + RotR(-i (w - conj w), n)
   so that ONE EvalMod serves both parts; the n-slot SlotToCoeff of
   re + i im.  Same depth and output level as the full pipeline; the
   output repeats slots [0, n) with period n. ---- */
typedef struct secpe_boot_params {
  int secret_h;   /* > 0: sparse secret, coefficient nonzero w.p. h / N (0: uniform ternary) */
  int K;          /* EvalMod range |t / q_0| <= K + 1 (bound on the ModRaise overflow) */
  int r;          /* double angles */
  int deg;        /* Chebyshev degree, 2^k - 1 */
  int ratio;      /* log2(q_0 / T_b) */
  int groups;     /* levels (merged stage groups) of each linear transform */
  int refresh;    /* 1: every refresh of an evaluation is a bootstrap */
  int sparse_slots; /* 0, or n: a power of two, 2n <= N/2, log2 n >= groups.
                       Evaluations whose refresh reads at most n slots
                       afterwards bootstrap sparsely. */
  int pack_min;   /* 0, or k >= 2 (needs sparse_slots): when at least k such
                     ciphertexts refresh together they are packed, n slots
                     each, into shared full-slot bootstraps
                     (secpe_bootstrap_packed) instead */
} secpe_boot_params;
/* the step value secpe_keygen takes as the conjugation key (X -> X^(2N-1)) */
#define SECPE_STEP_CONJUGATE INT64_MIN
/* Set the parameters; call before secpe_keygen (the secret uses secret_h).
   K <= 0 leaves bootstrapping off (secret_h still applies).  Writes the
   output level; returns SECPE_EINVAL when the chain is too short. */
int secpe_set_boot(secpe_ctx* ctx, const secpe_boot_params* bp, int* out_level);
/* Rotation steps one bootstrap uses (SECPE_STEP_CONJUGATE included); count
   returned, at most cap written. */
int secpe_boot_steps(const secpe_ctx* ctx, int64_t* out, int cap);
/* Device bytes of the precomputed linear-transform plaintexts. */
size_t secpe_boot_key_bytes(secpe_ctx* ctx);
/* Encode every group's diagonals (pre-rotated for the giant steps, at the
   plaintext scale each group's input needs) into buf_dev, which must stay
   alive while the context bootstraps.  After secpe_keygen.  Synchronous. */
int secpe_boot_setup(secpe_ctx* ctx, void* buf_dev, size_t bytes);
/* Bootstrap n ciphertexts (level >= 1) into the caller's buffers; the
   workspace size needs secpe_boot_setup first (0 and an error otherwise), as
   do the workspace sizes of evaluations that refresh by bootstrapping. */
size_t secpe_bootstrap_workspace_bytes(secpe_ctx* ctx, int n);
int secpe_bootstrap(secpe_ctx* ctx, int n, const secpe_ct* in, void* ws_dev, size_t ws_bytes, secpe_ct* out);
/* The sparse-slot bootstrap of n ciphertexts (sparse_slots set, else
   SECPE_EINVAL): slots [0, sparse_slots) of each input, repeated with that
   period over the N/2 slots of the output.  Same workspace size. */
int secpe_bootstrap_sparse(secpe_ctx* ctx, int n, const secpe_ct* in, void* ws_dev, size_t ws_bytes,
                           secpe_ct* out);
/* The window-packed bootstrap of n ciphertexts that are read only on slots
   [0, W) afterwards (W = sparse_slots; SECPE_EINVAL without it).  A design of
   this library, not of the paper (which bootstraps each ciphertext): in
   groups of m <= N/2W, taken in order, each input is masked to [0, W) at the
   scale-down, the group is packed by rotations into one ciphertext holding
   input j's window at slots [jW, jW + W), that ciphertext takes the
   full-slot bootstrap, and output j is it rotated left by jW: input j's
   slots [0, W) at [0, W), the windows of the inputs after it (cyclically
   within the group) beyond.  Every rotation is by a power-of-two multiple of
   W, the sparse-slot bootstrap's own steps.  Same level, scale and
   workspace size as secpe_bootstrap; in[i] and out[i] are the caller's. */
int secpe_bootstrap_packed(secpe_ctx* ctx, int n, const secpe_ct* in, void* ws_dev, size_t ws_bytes,
                           secpe_ct* out);
/* Single steps, for parity checks: step 0 ModRaise (level-0 input), 1
   CoeffToSlot, 2 SlotToCoeff, 3 EvalMod, 4 slots times i, 5 slots times -i,
   6 the sparse-slot CoeffToSlot, 7 the sparse-slot SlotToCoeff.
   ws sized by secpe_bootstrap_workspace_bytes(ctx, 1). */
int secpe_op_boot_step(secpe_ctx* ctx, int step, const secpe_ct* a, void* ws_dev, size_t ws_bytes, secpe_ct* out);

/* Autotuner for the batched path.  Times the batch given (same arguments
   as secpe_eval_argmax_batch, no graph) under candidate schedules and keeps
   the fastest in the context for later calls.  A candidate index is a set of
   knob bits:
     bit 0: output limbs per workgroup of the fused ModUp, 2 (set) or 4;
     bit 1: NTT passes issued in job groups of 128 MiB (set) or all jobs at once;
     bit 2: forward NTT column pass, two tiles per workgroup (set: the second
            tile's loads in flight while the first transforms) or one;
     bit 3: inverse NTT column pass, two tiles per workgroup (set) or one;
     bit 4: forward NTT row pass (with its fused epilogues), two tiles per
            workgroup (set) or one;
     bit 5: output limbs per workgroup of the fused ModDown conversion, 2 (set)
            or 4.
   (Bits 0 and 5 apply to launches of at least two workgroups per CU; a
   smaller launch, such as one query's, takes one limb per workgroup.)
   (The two-tile variants exist for N = 2^16; elsewhere bits 2-4 change nothing.)
   Search: candidate 0, then each knob flipped in turn from the best so far
   and kept when the batch is faster (coordinate descent; 1 + 6 candidates
   timed, each the faster of two runs).  Writes the chosen candidate to
   *chosen and, for i < cap, the milliseconds of candidate i to ms[i] (0 for
   candidates not timed).  Synchronous.  Returns 0 or an error. */
#define SECPE_AUTOTUNE_KNOBS 6
/* Set a schedule (candidate index as above) without timing, e.g. one a
   previous secpe_autotune chose.  Every schedule gives the same bits. */
int secpe_set_schedule(secpe_ctx* ctx, int candidate);
#define SECPE_AUTOTUNE_CANDIDATES 64
int secpe_autotune(secpe_ctx* ctx, const secpe_key_owner* owner, int n, const secpe_ct* in, const int* K,
                   const int* C, const double* d_min, const double* d_max, const uint64_t* refresh_seed,
                   void* ws_dev, size_t ws_bytes, secpe_ct* out, int* chosen, double* ms, int cap);

/* Operation counts of the last evaluation: [sign, rotate, relin, key_switch,
   refresh, poly, max, kernel launches]. */
int secpe_counters(const secpe_ctx* ctx, int64_t* out8);

/* Coefficient-domain canonical residues of a ciphertext, [2][level+1][N]
   uint64 on the host (the format parity checks compare).  Synchronous. */
int secpe_ct_export(secpe_ctx* ctx, const secpe_ct* ct, uint64_t* host_out);
/* Inverse of export: host [2][level+1][N] coefficient residues -> out. */
int secpe_ct_import(secpe_ctx* ctx, const uint64_t* host_in, int level, double scale, secpe_ct* out);

/* Switching key limb in the coefficient domain (key index as in keygen,
   digit < dnum, which 0 = b / 1 = a, prime index < n_q + n_p).  Synchronous. */
int secpe_key_export(secpe_ctx* ctx, const void* evk_dev, int key, int digit, int which, int prime, uint64_t* host_out);
/* Secret key in the coefficient domain as small integers. Synchronous. */
int secpe_sk_export(secpe_ctx* ctx, const void* sk_dev, int64_t* host_out);

/* Wait for all queued work. */
int secpe_sync(secpe_ctx* ctx);

/* ---- serving: continuous batching ---- */
/* A server keeps evaluation state for many in-flight Argmax requests in one
   workspace (caller-owned device memory).  Requests are submitted at any time;
   each call to secpe_server_step admits pending requests while the estimated
   workspace of the admitted set fits (and at most max_active run), then
   runs one round of Algorithm 1 over every admitted request, waits for the
   GPU and returns the requests that completed.  In a round the step kinds
   (prompt sum, normalisation, duplication, Max pre-step, Sign polynomial,
   Max post-step, final pre-step, final post-step) run in that order, the
   steps of one kind for all requests in the same kernel launches, and a
   request takes at most one step of each kind.  When that round holds
   little work (few requests active), further rounds join the same
   submission until a request completes or about 96 key-switches are
   queued.  A request's result is bit-identical to evaluating it alone.
   The input ciphertext must stay valid until its request completes;
   out_data receives z (secpe_ct_bytes).  owner (or NULL) refreshes as in
   secpe_eval_argmax for every request of the server. */
typedef struct secpe_server secpe_server;
int secpe_server_create(secpe_ctx* ctx, const secpe_key_owner* owner, void* ws_dev, size_t ws_bytes, int max_active,
                        secpe_server** out);
void secpe_server_destroy(secpe_server* srv);
/* Estimated workspace one request of shape (K, C) holds while active. */
size_t secpe_server_request_bytes(secpe_ctx* ctx, int K, int C);
int secpe_server_submit(secpe_server* srv, const secpe_ct* in, int K, int C, double d_min, double d_max,
                        uint64_t refresh_seed, void* out_data, uint64_t* ticket);
/* One submission of one or more rounds.  Writes up to 'cap' completed
   tickets with the level and scale of their results (completions beyond
   'cap' are kept and reported first by the next call); n_active / n_pending
   report the queue after the submission. */
int secpe_server_step(secpe_server* srv, int cap, int* n_done, uint64_t* tickets, int* levels, double* scales,
                      int* n_active, int* n_pending);
/* secpe_server_step in two halves, so that the host can keep several servers
   busy at once (one per tenant, each on its own context and stream: launch
   every server, then collect every server).  secpe_server_launch admits and
   queues the submission without waiting (nothing to run is not an error);
   calling it again before secpe_server_collect fails with SECPE_EINVAL.
   secpe_server_collect waits for the server's stream and reports as
   secpe_server_step does (n_done = 0 when nothing was launched). */
int secpe_server_launch(secpe_server* srv);
/* 1 when secpe_server_collect would not wait (the launched submission has
   finished, or nothing is launched), 0 while it runs, negative on a device
   error.  Lets the host relaunch each server as soon as its own work ends. */
int secpe_server_ready(secpe_server* srv);
int secpe_server_collect(secpe_server* srv, int cap, int* n_done, uint64_t* tickets, int* levels, double* scales,
                         int* n_active, int* n_pending);

/* ---- measurement ---- */
/* Event profiler: while enabled, every launch of the given kind is bracketed
   by HIP events on the context's stream (eager launches only; graph replays
   are not bracketed).  secpe_profile_end synchronises and returns the number
   of launches, their summed duration in ms and the units they processed:
   limb transforms for the NTT kinds (one limb transform reads and writes N
   residues), limbs for the others.  Kinds: */
enum {
  SECPE_PROF_NTT_FWD = 0, SECPE_PROF_NTT_INV = 1, SECPE_PROF_EW = 2, SECPE_PROF_MODUP = 3,
  SECPE_PROF_MODDOWN = 4, SECPE_PROF_INNER = 5, SECPE_PROF_AUTO = 6,
  /* 7 is reserved (the rescale's spread of the top limb runs fused into the forward NTT) */
  SECPE_PROF_SPREAD = 7,
  /* one kernel of the two-pass forward NTT (N > 2^12): the column pass, the row pass;
     the forward NTT carries the fused rescale / ModDown / relinearise-and-rescale
     combines in its row pass */
  SECPE_PROF_NTT_FWD_COL = 8, SECPE_PROF_NTT_FWD_ROW = 9,
  /* the segments of an evaluation: events at the start and end of every
     command list and at the start and end of every refresh stand-in, so the
     intervals alternate computation and refresh (secpe_profile_segments) */
  SECPE_PROF_SEGMENTS = 10
};
int secpe_profile_begin(secpe_ctx* ctx, int kind);
/* units_shared: the same count with data that several jobs of one launch
   read counted once (the key limbs of the key-switch inner product, read by
   every job that switches with the same key); equal to units for the other
   kinds. */
int secpe_profile_end(secpe_ctx* ctx, int64_t* launches, double* total_ms, int64_t* units, int64_t* units_shared);
/* After a SECPE_PROF_SEGMENTS profile: the milliseconds between consecutive
   events in order (count returned, at most cap written). */
int secpe_profile_segments(const secpe_ctx* ctx, double* ms, int cap);

/* The algorithmic HBM bytes of the last evaluation's key switches: for each
   key switch at l+1 limbs, (l+1) limbs read and 2 (l+1) written, and for
   each launch each distinct key's 2 dnum_l (l+1+alpha) limbs once, however
   many jobs share it (the hybrid key switch of Sec. 2.2 touches no less). */
int secpe_keyswitch_traffic(const secpe_ctx* ctx, int64_t* alg_bytes);

/* Batched negacyclic NTT (Sec. 2.2 ring) in place over limbs 0..level of both
   polynomials of n ciphertexts, one launch per direction: inverse != 0 maps
   the NTT domain to coefficients.  Asynchronous. */
int secpe_ntt_cts(secpe_ctx* ctx, const secpe_ct* cts, int n, int inverse);

/* Batched rotations out[i] = RotL(in[i], steps[i]) (Sec. 2.2), each a Galois
   automorphism and a hybrid key switch with the key registered for its step.
   ws sized by secpe_rotate_workspace_bytes.  Asynchronous. */
size_t secpe_rotate_workspace_bytes(secpe_ctx* ctx, int n);
int secpe_rotate_batch(secpe_ctx* ctx, int n, const secpe_ct* in, const int64_t* steps, void* ws, size_t ws_bytes,
                       secpe_ct* out);

/* ---- primitive operations (parity checks of single steps); ws sized by
   secpe_op_workspace_bytes; outputs are caller buffers; asynchronous. ---- */
size_t secpe_op_workspace_bytes(secpe_ctx* ctx);
int secpe_op_add(secpe_ctx* ctx, const secpe_ct* a, const secpe_ct* b, secpe_ct* out);
int secpe_op_sub(secpe_ctx* ctx, const secpe_ct* a, const secpe_ct* b, secpe_ct* out);
int secpe_op_add_const(secpe_ctx* ctx, const secpe_ct* a, double v, secpe_ct* out);
int secpe_op_mul_const(secpe_ctx* ctx, const secpe_ct* a, double v, double target, void* ws, size_t ws_bytes, secpe_ct* out);
/* K_a a + K_b b (b may be NULL) with integer constants K = llround(v T q_l / s)
   when rescale != 0 (then one rescale), K = llround(v T / s) when rescale == 0
   (level kept); the result carries scale T exactly.  Sec. 2.2 operations;
   used for the constant terms of the Sign polynomials (Sec. 4.3). */
int secpe_op_lincomb(secpe_ctx* ctx, const secpe_ct* a, double va, const secpe_ct* b, double vb, double target,
                     int rescale, void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_mul_plain(secpe_ctx* ctx, const secpe_ct* a, const double* v, int nslots, double target, void* ws,
                       size_t ws_bytes, secpe_ct* out);
int secpe_op_rescale(secpe_ctx* ctx, const secpe_ct* a, void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_mul_relin(secpe_ctx* ctx, const secpe_ct* a, const secpe_ct* b, void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_mul_relin_rescale(secpe_ctx* ctx, const secpe_ct* a, const secpe_ct* b, void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_rotate(secpe_ctx* ctx, const secpe_ct* a, int64_t step, void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_refresh(secpe_ctx* ctx, const secpe_key_owner* owner, const secpe_ct* a, uint64_t seed, uint64_t index,
                     void* ws, size_t ws_bytes, secpe_ct* out);
int secpe_op_eval_odd9(secpe_ctx* ctx, const secpe_ct* a, const double* coef5, double gain, double target, void* ws,
                       size_t ws_bytes, secpe_ct* out);
/* hybrid key switch of d (host, coefficient domain, [level+1][N]) with key
   'key'; u0, u1 written to the host in the same format.  Synchronous. */
int secpe_op_key_switch(secpe_ctx* ctx, int key, const uint64_t* d_host, int level, void* ws, size_t ws_bytes,
                        uint64_t* u0_host, uint64_t* u1_host);
/* forward then inverse NTT of limb data (host, [n][N] residues of prime
   'prime'), for the NTT checks; out_fwd may be NULL.  Synchronous. */
int secpe_op_ntt(secpe_ctx* ctx, int prime, const uint64_t* in_host, int n, uint64_t* out_fwd, uint64_t* out_roundtrip);
/* negacyclic product of two limbs mod prime 'prime' through the NTT. Synchronous. */
int secpe_op_ring_mul(secpe_ctx* ctx, int prime, const uint64_t* a_host, const uint64_t* b_host, uint64_t* out_host);
/* encoder: m[N] for real slot values z[nslots] at 'scale'. Synchronous. */
int secpe_op_encode(secpe_ctx* ctx, const double* z, int nslots, double scale, int64_t* m_out);

#ifdef __cplusplus
}
#endif
#endif /* SECPE_H */
