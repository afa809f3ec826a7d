/*
 * ckks_lt.h - C interface of the MI355X (gfx950) library for homomorphic
 * plaintext-matrix x encrypted-vector linear transformations (HE-LT) in
 * RNS-CKKS, by the triple-hoisted baby-step giant-step algorithm
 * (Akherati & Zhang, arXiv 2605.17222, Algorithm 2 and eq. (6)) and by the
 * plain BSGS algorithm it is compared with (eq. (5), Table I), the
 * double-hoisted BSGS (Algorithm 1) and the diagonal method.  Around it:
 * ragged batches in lockstep, a continuous-batching server, plaintext
 * encoding on the device (also on the fly inside an LT, for dense matrices),
 * one call per step of the path, the operation-count model with a split
 * autotuner, the paper's off-chip traffic model, and kernel timing.
 *
 * Every call takes plain pointers and sizes.  Pointers documented as "device"
 * point to GPU memory on the device that was current when the parameter set
 * was created; "host" pointers are read before the call returns.  Calls that
 * take a `stream` (a hipStream_t; NULL = the default stream) only enqueue
 * work and return without waiting: the caller keeps every buffer alive and
 * unmodified until the stream has completed.  No call throws; errors are
 * negative return codes, described by ckks_strerror().
 *
 * Data layout (fixed conventions, also followed by the test oracle):
 *  - A limb is the N residues of one polynomial modulo one prime, stored as N
 *    little-endian uint64 words, canonical in [0, q) (the [.]_q of eq. (3)).
 *  - A polynomial over several primes is its limbs back to back: [limbs][N].
 *  - Limbs are in NTT form, bit-reversed order (Section V, layout of
 *    eq. (8)): word p of a limb holds sum_k a_k psi^((2 br(p)+1) k) mod q, with
 *    br = bit reversal over log2 N bits and psi the primitive 2N-th root of
 *    unity of that prime (see ckks_params_desc.psi).
 *  - PQ-basis polynomials list the special primes first:
 *    [p_0 .. p_{alpha-1}, q_0 .. q_l] (eq. (4) indexes q_j as limb j+alpha).
 *    Truncating to a lower level keeps a prefix of that layout.
 *  - Rotation r uses the Galois element g_r = 5^(r mod N/2) mod 2N
 *    (Section II-A, eq. (2)); slots move toward slot 0.
 */
#ifndef CKKS_LT_H
#define CKKS_LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define CKKS_OK 0
#define CKKS_E_INVALID_ARG -1  /* null pointer, bad size, level or split      */
#define CKKS_E_UNSUPPORTED -2  /* missing rotation key, unsupported shape     */
#define CKKS_E_WORKSPACE -3    /* workspace smaller than ckks_*_workspace_size */
#define CKKS_E_DEVICE -4       /* a HIP runtime call failed                   */
#define CKKS_E_NOMEM -5        /* device allocation failed                    */
#define CKKS_E_TIMEOUT -6      /* server: request waited past its queue limit */
#define CKKS_E_CANCELLED -7    /* server: request cancelled before it started */

/* Server request states that are not yet a result (see ckks_server_poll). */
#define CKKS_PENDING 1         /* queued, not yet admitted                    */
#define CKKS_RUNNING 2         /* admitted; its batch is on the device        */

/* Text for an error code (static storage). */
const char* ckks_strerror(int code);

/* ---- parameter sets ---------------------------------------------------- */
/*
 * RNS-CKKS parameters (Section II-A): ring Z[X]/(X^N + 1), ciphertext modulus
 * Q = q_0 ... q_L, special modulus P = p_0 ... p_{alpha-1} for the
 * generalized key switching of Fig. 1.  A digit is a group of alpha
 * consecutive q primes, so there are dnum = beta = ceil((L+1)/alpha) digits
 * at the top level (the paper's Set-C has L+1 = 32, alpha = 12, beta = 3).
 */
typedef struct {
  int log_n;            /* log2 N, 12 <= log_n <= 16                         */
  int n_q;              /* L + 1                                             */
  const uint64_t* q;    /* host [n_q]: q_0 .. q_L                            */
  int n_p;              /* alpha                                             */
  const uint64_t* p;    /* host [n_p]: p_0 .. p_{alpha-1}                    */
  int dnum;             /* digits at the top level; must equal ceil(n_q/n_p) */
  const uint64_t* psi;  /* host [n_p + n_q] (P first) primitive 2N-th roots,
                           or NULL: then psi = g^((q-1)/2N) for the smallest
                           quadratic non-residue g >= 2 of each prime        */
} ckks_params_desc;

typedef struct ckks_params ckks_params;  /* opaque, immutable once created */

/*
 * Validates the primes (prime, distinct, = 1 mod 2N, < 2^61, and for every
 * basis conversion the sum of the source primes below 2^64) and builds the
 * twiddle and RNS-constant tables in device memory on the current device.
 * The library owns *out (free it with ckks_params_destroy).  It may be used
 * from several streams at once.  Returns CKKS_OK or a negative code.
 */
int ckks_params_create(const ckks_params_desc* desc, ckks_params** out);
void ckks_params_destroy(ckks_params* params);

/* N, L and alpha of a parameter set (any pointer may be NULL). */
void ckks_params_info(const ckks_params* params, int* log_n, int* n_q, int* n_p);

/* ---- ciphertexts, plaintext diagonals, rotation keys --------------------- */
typedef struct {
  int level;     /* l: the ciphertext has l+1 limbs per polynomial           */
  double scale;  /* CKKS scale, tracked only                                 */
  uint64_t* c0;  /* device [l+1][N], NTT form                                */
  uint64_t* c1;  /* device [l+1][N], NTT form                                */
} ckks_ct;

/*
 * The diagonals of the LT matrix as NTT-form plaintexts (Section II-B).
 * Index t = n1 n2 k + n1 j + i (TH-BSGS), n1 j + i (BSGS) or t (diagonal
 * method) holds the cyclic diagonal at offset s (t - c) mod N/2, with
 * s = stride and c = centre: plain Algorithm 2 is s = 1, c = 0 (offset t);
 * other values serve sparse matrices whose diagonals form an arithmetic
 * progression, negative offsets included (e.g. the factors of a DFT).  The
 * rotations are s i (baby / inner), s n1 j (middle) and the giant step
 * G_k = s (B k - c), B = n1 n2 (TH-BSGS) or n1 (BSGS); a block whose G_k is
 * 0 mod N/2 is added without rotation (Algorithm 2's k = 0 block).
 * Plaintext t must already carry its block's giant-step pre-rotation:
 *   TH-BSGS : f^_t = phi_{-G_k}(f_t), PQ basis [alpha + L + 1][N]
 *   BSGS    : f^_t = phi_{-G_j}(f_t), Q basis  [L + 1][N]
 *   naive   : f_t,                    Q basis  [L + 1][N]
 * A NULL pointer is an all-zero diagonal and is skipped exactly.  The
 * progression must not repeat an offset: n1 n2 n3 (or n_diag) indices at
 * most N/2 / gcd(s, N/2).
 *
 * On-the-fly plaintexts: with pt = NULL and slots set, slots[t] is the
 * diagonal itself as N/2 complex slot values (device [N/2][2] doubles, re and
 * im; NULL = absent) and the library encodes the plaintext above
 * (f^_t = encode(rot(diag_t, -G)) for TH-, DH- and plain BSGS, encode(diag_t)
 * for the diagonal method) with scale pt_scale at the ciphertext's level and
 * basis (as ckks_encode does) right before the multiply-accumulate that
 * consumes it, so no plaintext outlives its use: a dense n = N/2 matrix
 * needs N/2 slot vectors (16 B per slot) instead of n resident plaintexts of
 * alpha + l + 1 limbs.  The workspace then also holds the plaintexts of one
 * multiply-accumulate launch (up to 128 of alpha + l + 1 limbs).  Setting
 * both pt and slots is an error.
 */
typedef struct {
  int n1, n2, n3;                /* split; n3 = 1 for BSGS; ignored by naive */
  int n_diag;                    /* entries in pt                            */
  const uint64_t* const* pt;     /* host [n_diag] of device pointers          */
  double pt_scale;               /* scale the plaintexts were encoded with   */
  int stride;                    /* s; 0 reads as 1                          */
  int centre;                    /* c                                        */
  const double* const* slots;    /* host [n_diag] of device pointers or NULL */
  int pt_packed;                 /* pt are packed (ckks_pack), TH-/DH-BSGS  */
} ckks_lt_diags;

/*
 * Pre-rotated switching keys swk~_r = phi_{-r}(swk_r) (Algorithm 2, input
 * list).  Key r is [beta_max][2][alpha + L + 1][N] words with
 * beta_max = ceil((L+1)/alpha); polynomial 0 of digit b multiplies the digit
 * and is added to c0, polynomial 1 forms the new c1.  Keys are generated at
 * the top level and truncated by prefix for lower levels.
 */
typedef struct {
  int count;
  const int32_t* rot;          /* host [count]: r (taken mod N/2)           */
  const uint64_t* const* key;  /* host [count] of device pointers           */
  int packed;                  /* keys are packed (ckks_pack of the
                                  beta_max * 2 polynomials of each key)     */
} ckks_rotkeys;

/*
 * Packed storage of resident operands.  Keys and plaintexts are read once
 * per use from HBM and dominate the bytes of the HBM-bound kernels; a limb
 * of a prime below 2^40 holds values of at most 40 bits, so it is stored in
 * 5N bytes instead of 8N: runs of 256 coefficients, each run its 256 32-bit
 * low words (little-endian) followed by its 256 high bytes (1280 bytes per
 * run); limbs of larger primes stay N 64-bit words.  A packed polynomial is
 * the alpha + L + 1 limbs of the full PQ basis back to back (lower levels
 * read a prefix); ckks_packed_poly_bytes gives its size.  ckks_pack converts
 * count full PQ polynomials in (device [count][alpha+L+1][N] words, canonical)
 * into out (device, count * packed bytes), on `stream`; in and out must not
 * overlap.  A key is packed as its beta_max * 2 polynomials (count =
 * 2 beta_max), a TH-BSGS plaintext as one.  The packed and unpacked forms
 * give bit-identical LT results.  ckks_pack returns CKKS_E_INVALID_ARG for a
 * null params, count outside 0..65535, a null buffer with count > 0, or
 * overlapping buffers, CKKS_E_DEVICE if the launch fails, and CKKS_OK
 * otherwise (count 0 does nothing); the caller owns both buffers, and the
 * result is ready when `stream` reaches the launch.
 */
int ckks_packed_poly_bytes(const ckks_params* params, size_t* bytes);
int ckks_pack(const ckks_params* params, int count, const uint64_t* in, void* out, void* stream);

/* ---- the linear transformation ----------------------------------------- */
#define CKKS_LT_NAIVE 0    /* diagonal method: sum_d Rot(ct, d) f_d           */
#define CKKS_LT_BSGS 1     /* plain BSGS, eq. (5), one Decompose per rotation */
#define CKKS_LT_TH_BSGS 2  /* triple-hoisted BSGS, Algorithm 2                */
#define CKKS_LT_DH_BSGS 3  /* double-hoisted BSGS, Algorithm 1: baby steps n1,
                              giant steps n2 (exactly TH-BSGS with n1' = 1,
                              n2' = n1, n3' = n2; plaintexts pre-rotated by
                              phi_{-n1 j}, PQ basis)                       */

/* Workspace bytes ckks_lt_eval needs for this level, split and algorithm. */
int ckks_lt_workspace_size(const ckks_params* params, int level, const ckks_lt_diags* diags, int algo,
                           size_t* bytes);

/*
 * out = LT(in): enqueues the whole transformation on `stream`.
 *   TH-BSGS follows Algorithm 2 (the final line is one ModDown by P q_l,
 *   i.e. ModDown and rescale combined); BSGS and the diagonal method rotate
 *   with Rot(ct, r) = (phi_r(c0 + x), phi_r(y)), (x, y) =
 *   ModDown(<Decompose(c1), swk~_r>), and end with the rescale of eq. (1).
 * in->level = l >= 1; out must have level l-1 buffers (l limbs) and must not
 * alias in.  out->level and out->scale are set (scale = in.scale *
 * pt_scale / q_l).  ws: device workspace of ws_bytes >= ckks_lt_workspace_size.
 * Errors: CKKS_E_INVALID_ARG (nulls, level < 1, n_diag larger than the split,
 * aliasing), CKKS_E_UNSUPPORTED (a needed rotation key is missing),
 * CKKS_E_WORKSPACE, CKKS_E_DEVICE.
 */
int ckks_lt_eval(const ckks_params* params, const ckks_ct* in, const ckks_lt_diags* diags,
                 const ckks_rotkeys* keys, int algo, ckks_ct* out, void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * LT as ckks_lt_eval, with its workspace taken from a scratch array of
 * CKKS_LT_NOALLOC_MAX_WS bytes that the library holds on each device it runs
 * on (made when the library's code is loaded there, kept until the process
 * ends).  The call allocates no device memory and frees none; the caller
 * still passes the inputs, keys, plaintexts and outputs.  An LT whose
 * workspace (ckks_lt_workspace_size) exceeds CKKS_LT_NOALLOC_MAX_WS is
 * refused with CKKS_E_WORKSPACE before anything is enqueued.  Every call on
 * one device uses that device's one scratch array, which keeps the previous
 * call's contents (the LT reads no workspace word it has not written):
 * calls whose work overlaps on one device race, so the caller orders them
 * (one stream, or events between streams).  Other arguments, results and
 * errors as ckks_lt_eval.
 */
#define CKKS_LT_NOALLOC_MAX_WS ((size_t)64 << 20)

int ckks_lt_eval_noalloc(const ckks_params* params, const ckks_ct* in, const ckks_lt_diags* diags,
                         const ckks_rotkeys* keys, int algo, ckks_ct* out, void* stream);

/* ---- plaintext encoding on the device ------------------------------------- */
/*
 * Encoding (Section II-A): the plaintext of a vector z of N/2 complex slots
 * is the integer polynomial m = round(scale * sigma^-1(z)), where slot t is
 * m(zeta^(5^t)), zeta = e^(i pi / N); rounding is half away from zero.  The
 * library computes it with one length-N/2 complex FFT in FP64 per vector,
 * reduces m into the primes first_prime .. first_prime + n_limbs - 1 of the
 * PQ chain (P first: TH-BSGS plaintexts at level l are primes 0 .. alpha + l,
 * BSGS plaintexts primes alpha .. alpha + l) and returns NTT form.  Item i
 * encodes rot(z, rot): slot t takes z[(t + rot) mod N/2], so the giant-step
 * pre-rotation phi_{-G}(f) of Algorithm 2 is rot = -G.
 *   slots: device [N/2][2] doubles (re, im), read only
 *   out:   device [n_limbs][N] words, written
 *   coef:  device [N] int64 or NULL: receives m
 * |scale * sigma^-1(z)| must stay below 2^62 (coefficients beyond are
 * clamped).  FP64 rounding decides m: a coefficient within a few ulp of a
 * half-integer may round either way relative to another FFT.
 * Errors: CKKS_E_INVALID_ARG (nulls, scale not positive and finite, prime
 * range outside the chain), CKKS_E_WORKSPACE, CKKS_E_DEVICE.  Enqueues on
 * stream and returns.
 */
typedef struct {
  const double* slots;
  int32_t rot;
  uint64_t* out;
  int64_t* coef;
} ckks_encode_item;

/* Workspace bytes ckks_encode needs for count items (at most two limbs per
 * item, for at most 32 items). */
int ckks_encode_workspace_size(const ckks_params* params, int count, size_t* bytes);

int ckks_encode(const ckks_params* params, int count, const ckks_encode_item* items, double scale, int first_prime,
                int n_limbs, void* ws, size_t ws_bytes, void* stream);

/* ---- ragged batches --------------------------------------------------------- */
/*
 * One LT of a batch: its own ciphertext, diagonals (split and plaintexts),
 * rotation keys (the same ckks_rotkeys may serve many items) and output.
 * status receives the item's result code.
 */
typedef struct {
  ckks_ct in;
  ckks_lt_diags diags;
  const ckks_rotkeys* keys;
  ckks_ct out;
  int status;
} ckks_lt_item;

/* Workspace bytes ckks_lt_eval_batch needs for these items (buffers unread). */
int ckks_lt_batch_workspace_size(const ckks_params* params, int count, const ckks_lt_item* items, int algo,
                                 size_t* bytes);

/*
 * Evaluates count LTs of one parameter set whose levels, splits and diagonal
 * counts may all differ.  For CKKS_LT_TH_BSGS the items run in lockstep:
 * every line of Algorithm 2 is issued for all items at once (Decompose and
 * ModDown of all items share launches; key-switch launches group the digit
 * sets of every item that uses a key, so each key is read once per launch,
 * whatever the items' levels).  Other algorithms run the items one after the
 * other.  Results are bit-identical to evaluating each item alone.  Items
 * whose arguments are invalid, or whose key set lacks a rotation their split,
 * stride or centre needs, get that error as their status and are skipped;
 * the other items still run.  Outputs that overlap inputs or each other fail
 * every item with CKKS_E_INVALID_ARG before anything runs.  Returns the
 * first error, or CKKS_OK.  Same stream and ownership rules as ckks_lt_eval.
 */
int ckks_lt_eval_batch(const ckks_params* params, int count, ckks_lt_item* items, int algo, void* ws,
                       size_t ws_bytes, void* stream);

/* ---- continuous-batching server ------------------------------------------ */
/*
 * A server evaluates TH-BSGS LT requests (Algorithm 2) for callers that
 * submit them one at a time.  A worker thread owned by the server admits
 * queued requests, oldest first, into batches evaluated with
 * ckks_lt_eval_batch, each batch on one of max_inflight streams of its own:
 * a request that arrives while other batches run is admitted as soon as a
 * stream is free and its workspace fits in the server's arena.  The arena
 * is one device allocation of hbm_budget_bytes made at creation; it holds the
 * workspaces of the batches in flight (ciphertexts, plaintexts, keys and
 * outputs stay in the caller's device memory).  Requests are admitted in
 * arrival order: a request whose workspace does not fit yet waits (those
 * behind it wait too), a request whose workspace alone exceeds the budget is
 * refused at submission.  Results are bit-identical to evaluating the request
 * alone with ckks_lt_eval.
 *
 * backend CKKS_SERVER_DEVICE runs on the device current at creation.
 * CKKS_SERVER_SIMULATED does no device work and allocates nothing: a batch of
 * b requests "runs" for simulated_service_s * (1 + (b-1)/4) seconds and
 * request workspaces are the sim_ws_bytes the caller states; it exists to
 * exercise admission and batching on hosts without a device.
 */
#define CKKS_SERVER_DEVICE 0
#define CKKS_SERVER_SIMULATED 1

typedef struct {
  int backend;              /* CKKS_SERVER_DEVICE or CKKS_SERVER_SIMULATED      */
  size_t hbm_budget_bytes;  /* workspace arena bytes                           */
  int max_batch;            /* requests per batch, >= 1                        */
  int max_inflight;         /* batches on the device at once, 1 .. 16          */
  double queue_timeout_s;   /* a request still queued after this long fails
                               with CKKS_E_TIMEOUT; <= 0: no limit            */
  double simulated_service_s;
} ckks_server_cfg;

typedef struct ckks_server ckks_server;  /* opaque */

/* One LT request: the fields of a ckks_lt_item plus the ring it runs on. */
typedef struct {
  int ring;               /* id from ckks_server_add_ring                      */
  ckks_ct in;             /* device; complete before submission                */
  ckks_lt_diags diags;    /* TH-BSGS split; pt (or slots) array copied at submission */
  ckks_ct out;            /* device; written when the request completes        */
  size_t sim_ws_bytes;    /* simulated backend only: the request's workspace   */
} ckks_request;

/*
 * Creates a server (and its worker thread).  Errors: CKKS_E_INVALID_ARG,
 * CKKS_E_NOMEM (arena allocation), CKKS_E_DEVICE.
 */
int ckks_server_create(const ckks_server_cfg* cfg, ckks_server** out);

/*
 * Registers a ring: a parameter set and its resident rotation keys (the
 * rot array and the key pointer array are copied; the key buffers are the
 * caller's and stay alive and unmodified until ckks_server_destroy).  params
 * may be NULL for the simulated backend.  Writes the ring id.
 */
int ckks_server_add_ring(ckks_server* server, const ckks_params* params, const ckks_rotkeys* keys, int* ring_id);

/*
 * Queues a request and returns at once (never waits for the device).  The
 * caller keeps the request's buffers alive until it has finished.  Errors:
 * CKKS_E_INVALID_ARG (unknown ring, bad level or split), CKKS_E_WORKSPACE
 * (the request's workspace exceeds the budget).
 */
int ckks_server_submit(ckks_server* server, const ckks_request* request, uint64_t* id);

/*
 * Request state: CKKS_PENDING, CKKS_RUNNING, or its result (CKKS_OK or a
 * negative code; then out holds the LT and *latency_s, if not NULL, the
 * seconds from submission to completion, else -1).
 */
int ckks_server_poll(ckks_server* server, uint64_t id, int* status, double* latency_s);

/*
 * The output ciphertext of a finished request, with its level and scale set
 * (level l-1, scale = in.scale * pt_scale / q_l).  Returns the request's
 * error code if it failed, CKKS_E_INVALID_ARG if it has not finished.
 */
int ckks_server_result(ckks_server* server, uint64_t id, ckks_ct* out);

/* Cancels a request that is still queued (CKKS_E_INVALID_ARG otherwise). */
int ckks_server_cancel(ckks_server* server, uint64_t id);

/* Blocks until nothing is queued or in flight. */
int ckks_server_wait_all(ckks_server* server);

typedef struct {
  long completed;          /* requests finished with CKKS_OK                  */
  long failed;             /* finished with an error, timed out or cancelled  */
  long rejected;           /* refused at submission                           */
  long queued, inflight;   /* requests waiting / running now                  */
  long batches;            /* batches launched                                */
  long max_batch;          /* largest batch launched                          */
  long max_inflight;       /* most batches in flight at once                  */
  size_t arena_in_use;     /* arena bytes held by batches in flight           */
  size_t arena_peak;       /* most arena bytes held at once                   */
  double p50_s, p99_s;     /* latency percentiles of completed requests       */
  double mean_s;
  double span_s;           /* first submission to last completion             */
} ckks_server_stat;

int ckks_server_stats(ckks_server* server, ckks_server_stat* stat);

/* Drains queued and running requests, stops the worker, frees the arena. */
void ckks_server_destroy(ckks_server* server);

/* ---- the steps of the path, one call each (for tests and composition) ---- */
/*
 * Negacyclic NTT (forward != 0) or inverse NTT of n_limbs limbs whose primes
 * are the consecutive PQ indices first_prime .. first_prime + n_limbs - 1
 * (0 .. alpha-1 are p_i, alpha + j is q_j).  in/out: device [n_limbs][N];
 * in == out is allowed.  The inverse includes the factor N^-1.
 */
int ckks_op_ntt(const ckks_params* params, int forward, int first_prime, int n_limbs, const uint64_t* in,
                uint64_t* out, void* stream);

/*
 * Decompose (Fig. 1; eq. (3)): x is a level-l Q-basis polynomial (device
 * [l+1][N], NTT form); digits receives device [beta_l][alpha+l+1][N]
 * (beta_l = ceil((l+1)/alpha)): digit b holds the group q_{alpha b} ..
 * q_{min(alpha b + alpha - 1, l)} unchanged and its ModUp (basis conversion
 * of the coefficient-domain group) in every other PQ limb.
 * ws: device workspace >= ckks_op_workspace_size(params, l).
 */
int ckks_op_decompose(const ckks_params* params, int level, const uint64_t* x, uint64_t* digits, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * ModDown (eq. (4)): x device [alpha+l+1][N] -> out device [l+1][N],
 * out_j = P^-1 (x_{alpha+j} - BConv(x_P))_j mod q_j.
 * If rescale != 0: ModDown by P q_l (ModDown and rescale combined, final
 * line of Algorithm 2): out device [l][N].
 */
int ckks_op_moddown(const ckks_params* params, int level, int rescale, const uint64_t* x, uint64_t* out,
                    void* ws, size_t ws_bytes, void* stream);

/* Rescale (eq. (1)): x device [l+1][N] -> out device [l][N]. */
int ckks_op_rescale(const ckks_params* params, int level, const uint64_t* x, uint64_t* out, void* ws,
                    size_t ws_bytes, void* stream);

/* Workspace bytes for the ckks_op_* calls at this level. */
int ckks_op_workspace_size(const ckks_params* params, int level, size_t* bytes);

/*
 * Hoisted key-switch inner product with the automorphism applied on write
 * (Algorithm 2, lines 4-5):  for the K = alpha+l+1 PQ limbs,
 *   (x, y) = (sum_b d_b key_{b,0}, sum_b d_b key_{b,1}),
 *   out_a = phi_r(add + x),  out_b = phi_r(y).
 * digits: device [beta_l][K][N]; key: device [beta_max][2][alpha+L+1][N];
 * add: device [K][N] or NULL (treated as zero); out_a, out_b: device [K][N].
 */
int ckks_op_keyswitch(const ckks_params* params, int level, const uint64_t* digits, const uint64_t* key,
                      int32_t rot, const uint64_t* add, uint64_t* out_a, uint64_t* out_b, void* stream);

/* NTT-domain automorphism phi_r (eq. (7)) of n_limbs limbs: out[p] = in[pi_r(p)]. */
int ckks_op_automorph(const ckks_params* params, int32_t rot, int n_limbs, const uint64_t* in, uint64_t* out,
                      void* stream);

/* ---- complexity model and split autotuner (host only, no device) ------------ */
/* Operation counts and bytes of one LT (Table I; counts of Section III). */
typedef struct {
  double modmul;      /* modular multiplications (Table II's counting)          */
  double ntt_limbs;   /* limb NTTs and inverse NTTs                             */
  double decompose;   /* Decompose operations                                   */
  double moddown;     /* ModDown operations (the final one counted per polynomial) */
  double keyswitch;   /* key-switch inner products                              */
  int keys;           /* distinct switching keys                                */
  double key_bytes;   /* switching-key storage, words of word_bits bits         */
  double pt_bytes;    /* plaintext storage (all n1 n2 n3 diagonals)              */
} ckks_lt_cost;

/*
 * Cost of an LT with ring 2^log_n, ciphertext level `level`, alpha special
 * primes and split (n1, n2, n3) (n3 ignored unless TH-BSGS; BSGS and DH-BSGS
 * use n1 baby and n2 giant steps).  word_bits sizes the byte counts (64 for
 * this library's uint64 words, 54 for the paper's Table II).
 */
int ckks_lt_cost_model(int log_n, int level, int alpha, int algo, int n1, int n2, int n3, int word_bits,
                 ckks_lt_cost* out);

/* Device rates the predictor uses (NULL: values fitted on MI355X). */
typedef struct {
  double ntt_limb_s;        /* seconds per limb NTT (both passes) at N = 2^16   */
  double bconv_product_s;   /* seconds per basis-conversion product            */
  double hbm_bytes_per_s;   /* achieved bandwidth of the HBM-bound kernels     */
  double layer_s;           /* latency per active hoisting layer (a chain of
                               dependent launches)                            */
} ckks_lt_rates;

/*
 * Predicted device seconds of one LT with this split and n_diag present
 * diagonals: the operation counts of ckks_lt_cost_model priced with `rates`,
 * plus the words the key-switch and MAC kernels move as this library
 * schedules one LT (TH-BSGS with at most 4 accumulators, or 8 whose terms
 * fit one fused launch: the middle key
 * switch fused with the multiply-accumulate, the rotation products never
 * stored).  DH-BSGS (n1, n2) is priced as TH-BSGS (1, n1, n2).  The rates
 * can be refitted on a device with `python -m paper_2605_17222_amd.calibrate`.
 */
int ckks_lt_predict(int log_n, int level, int alpha, int algo, int n1, int n2, int n3, int n_diag,
                    const ckks_lt_rates* rates, double* seconds);

/*
 * Chooses the split for a banded LT with diagonal offsets 0 .. n_diag-1 that
 * minimises ckks_lt_predict, among splits with n1 n2 n3 in [n_diag, 2 n_diag)
 * (padding with absent diagonals) needing at most max_keys switching keys
 * (max_keys <= 0: no limit).  Writes the split and the predicted seconds.
 */
int ckks_lt_autotune(int log_n, int level, int alpha, int algo, int n_diag, int max_keys, const ckks_lt_rates* rates,
                     int* n1, int* n2, int* n3, double* predicted_s);

/*
 * The paper's off-chip traffic model of its memory-optimized TH-BSGS data
 * path (Table III, off-chip columns), for its phases 1-6 with the on-chip
 * parallelism parameters of Table VII: m1, l1 (phase 1), m2, l2 (phase 2:
 * m2 ModDown results share the Decompose NTT twiddles), m3 keys and m4 digit
 * sets of l3 limbs on chip (phase 3), m5 (phase 4), m6 (phase 5).  Counts are
 * in limbs; a ratio of rounds such as (n1'-1)/m2 is rounded up (a phase runs
 * whole rounds).  n_diag is the LT dimension n of phase 4's matrix reads.
 * It describes the FPGA design's schedule, not this library's (whose words
 * ckks_lt_predict prices); it is here to reproduce the paper's traffic
 * figures (with Table VII's parameters the totals come within 0.3% of
 * Table VIII's off-chip column for Set-A/B/C).
 */
typedef struct {
  int m1, l1, m2, l2, m3, m4, l3, m5, l4, m6, l5;
} ckks_th_parallelism;

typedef struct {
  double phase_limbs[6];  /* off-chip limbs of phases 1..6                     */
  double twiddle_limbs;   /* per column of Table III, summed over the phases  */
  double matrix_limbs;
  double key_limbs;
  double read_limbs;
  double write_limbs;
  double total_limbs;
  double total_bytes;     /* total_limbs * N * word_bits / 8                   */
} ckks_th_traffic;

int ckks_th_traffic_model(int log_n, int level, int alpha, int n1, int n2, int n3, int n_diag, int word_bits,
                          const ckks_th_parallelism* par, ckks_th_traffic* out);

/* ---- kernel timing (benchmarks) ---------------------------------------- */
/* Kernel identifiers: the forward NTT column / row passes, the inverse NTT
 * row / column passes, basis conversion, key-switch inner product (several
 * digit sets and keys, automorphism on write), plaintext multiply-accumulate,
 * the automorphism gather, the gather form of the key switch that adds
 * every outer rotation into the accumulator, plaintext encoding, and the
 * middle key switch fused with the multiply-accumulate (Algorithm 2, lines
 * 8-14, used for every TH-BSGS item with at most 4 accumulators, or 8 whose
 * terms fit one launch; keys and plaintexts plain or packed, plaintexts
 * resident or encoded on the fly). */
#define CKKS_KERNEL_NTT_FWD_COL 0
#define CKKS_KERNEL_NTT_FWD_ROW 1
#define CKKS_KERNEL_NTT_INV_ROW 2
#define CKKS_KERNEL_NTT_INV_COL 3
#define CKKS_KERNEL_BCONV 4
#define CKKS_KERNEL_KEYSWITCH 5
#define CKKS_KERNEL_PTMAC 6
#define CKKS_KERNEL_AUTOMORPH 7
#define CKKS_KERNEL_KEYSWITCH_GATHER 8
#define CKKS_KERNEL_ENCODE_FFT 9  /* plaintext encoding: the two FFT passes  */
#define CKKS_KERNEL_KSMAC 10
#define CKKS_KERNEL_COUNT 11

/*
 * Process-wide: for every kernel k with bit (1 << k) set in mask, each later
 * launch is bracketed by two HIP events recorded on the stream it is launched
 * on.  Passing 0 stops recording.  Every call discards earlier records.
 */
int ckks_profile_enable(int mask);

/*
 * Waits for the recorded events of `kernel` and returns the number of
 * recorded launches, their summed duration in milliseconds and their summed
 * algorithmic bytes (compulsory reads and writes of the launch: each input
 * and output word once).
 */
int ckks_profile_read(int kernel, int* launches, double* total_ms, double* total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* CKKS_LT_H */
