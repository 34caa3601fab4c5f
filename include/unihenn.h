/*
 * unihenn.h -- C ABI of the MI355X (gfx950) library for UniHENN's
 * im2col-free encrypted CNN inference (UniHENN, arXiv 2402.03060).
 *
 * The library evaluates, on one GPU, the server side of the method: CKKS
 * rotations (Galois automorphism + RNS key switching over negacyclic NTTs),
 * plaintext x ciphertext multiply-accumulate with rescale, the square
 * activation, and the convolution (Algorithm 1), average pooling
 * (Section IV-C), flatten (Section IV-E) and fully connected (Algorithm 2)
 * layers on the flattened slot vector (Section III-A).
 *
 * Conventions
 *   Ring      R = Z[X]/(X^N + 1), N = 2^log_n, N/2 real slots (Section II-B).
 *   Moduli    data primes q_0..q_L and one special prime P used only inside
 *             key switching.  A ciphertext "at n_limbs" lives mod q_0..q_{n-1}.
 *   Layout    every polynomial is n_limbs rows of N uint64 words, limb-major;
 *             a ciphertext batch is [batch][2][n_limbs][N].  Device ciphertexts
 *             are in NTT (evaluation) form; residues are canonical in [0, q_i).
 *   Slots     slot k <-> evaluation point psi^(5^k mod 2N).  Rot(ct, r) is the
 *             LEFT rotation by r of Section II-B; negative r rotates right; r is
 *             taken mod N/2 and r = 0 is a copy without key switching.
 *   Memory    the caller owns every buffer it passes (device pointers unless a
 *             parameter says "host").  The library owns only unihenn_ctx and
 *             unihenn_net objects, released by their destroy calls.
 *   Streams   `stream` is a hipStream_t (NULL = default stream).  Every call
 *             is asynchronous on it unless stated otherwise; a call that
 *             returns an error enqueued nothing.
 *   Errors    0 on success, a negative UNIHENN_E* code otherwise;
 *             unihenn_last_error() returns a thread-local message.  Device
 *             faults surface at the caller's next synchronisation.
 */
#ifndef UNIHENN_H
#define UNIHENN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UNIHENN_OK = 0,
    UNIHENN_EINVAL = -1,  /* bad argument or shape */
    UNIHENN_ELEVEL = -2,  /* not enough limbs left / level mismatch */
    UNIHENN_ESCALE = -3,  /* terms of one sum at different scales */
    UNIHENN_ENOKEY = -4,  /* no switching key bound for a needed rotation */
    UNIHENN_ESLOTS = -5,  /* packed samples do not fit the slots */
    UNIHENN_ENOMEM = -6,  /* device allocation failed */
    UNIHENN_EDEVICE = -7  /* HIP runtime error */
};

typedef struct unihenn_ctx unihenn_ctx;
typedef struct unihenn_net unihenn_net;

/* A batch of ciphertexts on the device: [batch][2][n_limbs][N] uint64, NTT
 * form.  `scale` is the CKKS scale of every ciphertext in the batch. */
typedef struct {
    uint64_t* data;
    uint32_t n_limbs;
    uint32_t batch;
    double scale;
} unihenn_ct;

/* A switching key on the device as produced by unihenn_import_evk:
 * [n_data][2][n_data+1][N] uint64 (digit, component, basis q_0..q_L then P),
 * NTT form, residues multiplied by 2^64 mod q. */
typedef struct {
    const uint64_t* data;
    uint32_t n_data;
} unihenn_evk;

const char* unihenn_last_error(void);

/* ---------------------------------------------------------------- context */
/* Ring and modulus chain.  prime_bits[0..n_data-1] are the data-prime sizes,
 * special_bits the size of P; each prime is the largest unused p < 2^b with
 * p = 1 mod 2N and bit length b, in the order given (the paper fixes only
 * N, the scale and the depth: Table of parameters, Section V).  `scale` is
 * the encoding scale Delta.  Allocates the NTT tables on the current device.
 * Errors: EINVAL (log_n outside 4..16, bits outside log_n+2..61, more than
 * 23 primes), ENOMEM, EDEVICE. */
int unihenn_ctx_create(uint32_t log_n, const uint32_t* prime_bits, uint32_t n_data, uint32_t special_bits,
                       double scale, unihenn_ctx** out);
int unihenn_ctx_destroy(unihenn_ctx* ctx);
/* out (host): n_data + 1 primes, q_0..q_{L} then P. */
int unihenn_ctx_primes(const unihenn_ctx* ctx, uint64_t* out);

/* ------------------------------------------------------------- transforms */
/* In-place negacyclic NTT / inverse NTT of n_polys polynomials, each n_limbs
 * rows mod q_0..q_{n_limbs-1}: data is [n_polys][n_limbs][N].  unihenn_to_ntt
 * takes coefficients in [0, q_i) (the import of a ciphertext made by a
 * client); unihenn_from_ntt returns canonical coefficients (export).
 * Errors: EINVAL (n_limbs outside 1..n_data). */
int unihenn_to_ntt(const unihenn_ctx* ctx, uint64_t* data, uint32_t n_limbs, uint32_t n_polys, void* stream);
int unihenn_from_ntt(const unihenn_ctx* ctx, uint64_t* data, uint32_t n_limbs, uint32_t n_polys, void* stream);
/* Out-of-place import / export of ciphertexts (Section II-B: the client
 * encrypts and decrypts, the server evaluates; here in NTT form).
 * unihenn_import_ct copies coeff ([dst->batch][2][dst->n_limbs][N]
 * coefficients in [0, q_i), device or host memory) into dst->data and
 * transforms it there; unihenn_export_ct writes the canonical coefficients
 * of src into coeff (device memory, same layout).  coeff may equal the
 * ciphertext's data (in place).  The caller owns every buffer.
 * Errors: EINVAL (null pointers, n_limbs outside 1..n_data, batch 0). */
int unihenn_import_ct(const unihenn_ctx* ctx, const uint64_t* coeff, unihenn_ct* dst, void* stream);
int unihenn_export_ct(const unihenn_ctx* ctx, const unihenn_ct* src, uint64_t* coeff, void* stream);

/* Import a switching key given in coefficient form, layout
 * [n_data][2][n_data+1][N] with evk_j = (-a_j s + e_j + [i = j] P t, a_j)
 * over q_0..q_L, P (hybrid key switching, one digit per data prime); writes
 * the device form used by the key-switching kernels to `out` (same shape;
 * may alias `coeff`).  Errors: EINVAL (n_data differs from the context). */
int unihenn_import_evk(const unihenn_ctx* ctx, const uint64_t* coeff, uint32_t n_data, uint64_t* out,
                       void* stream);

/* ------------------------------------------------------------- plaintexts */
/* Encode real slot values z_0..z_{n_slots-1} (host array; missing slots are
 * zero) at `scale` into a plaintext of n_limbs rows (Section II-B, III-A):
 *   m_j = round( scale * (2/N) sum_k z_k cos(pi (5^k mod 2N) j / N) ),
 * rounded half away from zero from the value computed in double-double
 * arithmetic, reduced mod each q_i, then NTT.  mont != 0 stores residues
 * times 2^64 mod q (the form unihenn_mul_plain_acc multiplies by);
 * mont == 0 the plain form unihenn_add_plain adds.  pt: device
 * [n_limbs][N].  Synchronous with respect to the host array.
 * Errors: EINVAL (n_slots > N/2, |m_j| >= 2^52 before reduction). */
int unihenn_encode(const unihenn_ctx* ctx, const double* slots, uint32_t n_slots, double scale, uint32_t n_limbs,
                   int mont, uint64_t* pt, void* stream);
/* Plaintext from given coefficients (device [n_limbs][N], residues in
 * [0, q_i)): NTT, and the Montgomery factor when mont != 0.  pt may alias
 * coeff. */
int unihenn_import_pt(const unihenn_ctx* ctx, const uint64_t* coeff, uint32_t n_limbs, int mont, uint64_t* pt,
                      void* stream);
/* Coefficients of a plaintext made by unihenn_encode (same `mont`) into
 * coeff_out (device [n_limbs][N]). */
int unihenn_export_pt(const unihenn_ctx* ctx, const uint64_t* pt, uint32_t n_limbs, int mont, uint64_t* coeff_out,
                      void* stream);

/* ------------------------------------------------------------- primitives */
/* Bytes of workspace unihenn_rotate / _rotate_hoisted / _rescale /
 * _square_relin need for a batch at n_limbs. */
size_t unihenn_ks_workspace_size(const unihenn_ctx* ctx, uint32_t n_limbs, uint32_t batch);

/* Rot(ct, steps) (Section II-B) for every ciphertext of the batch:
 * (tau_g(c0) + KS_0(tau_g(c1)), KS_1(tau_g(c1))), g = 5^steps mod 2N, with
 * the hybrid key switch: digits centered([c]_{q_j}), inner product with the
 * key over q_0..q_l, P, then exact rounding division by P.  `gk` must be the
 * rotation key of `steps` (mod N/2).  out may not alias in.
 * Errors: EINVAL, ELEVEL (key made for fewer limbs), ENOKEY (gk NULL and
 * steps != 0). */
int unihenn_rotate(const unihenn_ctx* ctx, const unihenn_ct* in, int32_t steps, const unihenn_evk* gk,
                   unihenn_ct* out, void* ws, size_t ws_bytes, void* stream);
/* unihenn_rotate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same rotation, bit for bit, with its key-switching workspace in a
 * fixed 64 MiB device array of the library instead of a caller buffer.  The
 * caller still passes the input, key and output.  It allocates nothing and
 * calls no allocating routine.  Each GPU holds its own copy of the array from
 * the library's load until the process ends; the first call on a device
 * looks up its address (the context's device must be current).  Every call
 * on one GPU shares that array, so calls that overlap on one GPU (on
 * different streams or threads) race; calls on one stream are ordered.
 * Errors: as unihenn_rotate, and EINVAL when the workspace the rotation needs
 * (unihenn_ks_workspace_size(ctx, n_limbs, batch)) exceeds 64 MiB, or when
 * another device than the context's is current. */
int unihenn_rotate_noalloc(const unihenn_ctx* ctx, const unihenn_ct* in, int32_t steps, const unihenn_evk* gk,
                           unihenn_ct* out, void* stream);
/* n_steps rotations of the same ciphertexts sharing one digit decomposition
 * (hoisting).  Bit-identical to n_steps calls of unihenn_rotate.  gks[i] and
 * outs[i] belong to steps[i] (host arrays of descriptors). */
int unihenn_rotate_hoisted(const unihenn_ctx* ctx, const unihenn_ct* in, const int32_t* steps, uint32_t n_steps,
                           const unihenn_evk* gks, unihenn_ct* outs, void* ws, size_t ws_bytes, void* stream);
/* acc <- [acc +] sum_t pts[t] (*) cts[t] (Mul(P) and Add(C), Section II-B;
 * the inner sum of Algorithm 1).  cts (host array of n_terms descriptors)
 * must share batch, n_limbs and scale; pts (host array of device pointers)
 * are Montgomery-form plaintexts of n_limbs rows.  overwrite != 0 ignores the
 * previous contents of acc.  acc->scale becomes cts.scale * Delta.
 * Errors: EINVAL, ELEVEL (limb mismatch), ESCALE (scale mismatch). */
int unihenn_mul_plain_acc(const unihenn_ctx* ctx, const unihenn_ct* cts, const uint64_t* const* pts,
                          uint32_t n_terms, int overwrite, unihenn_ct* acc, void* stream);
/* Drop the last prime q_l: c'_i = (c_i - centered([c]_{q_l})) q_l^-1 mod q_i,
 * the exact rounding division by q_l; out has n_limbs - 1 limbs and scale
 * in.scale / q_l.  Errors: ELEVEL (n_limbs < 2). */
int unihenn_rescale(const unihenn_ctx* ctx, const unihenn_ct* in, unihenn_ct* out, void* ws, size_t ws_bytes,
                    void* stream);
/* Mul(C) of Section II-B followed by relinearisation with the key of s^2:
 * the tensor (a0 b0, a0 b1 + a1 b0, a1 b1) with the last part key-switched
 * into the first two.  b may hold more limbs than a (its first a->n_limbs
 * are used: b dropped to a's level); out has a's limbs and scale
 * a.scale * b.scale, no rescale.  out may alias neither operand.  Errors:
 * ELEVEL (b has fewer limbs), EINVAL (batch sizes differ), ENOKEY. */
int unihenn_mul_relin(const unihenn_ctx* ctx, const unihenn_ct* a, const unihenn_ct* b, const unihenn_evk* rlk,
                      unihenn_ct* out, void* ws, size_t ws_bytes, void* stream);
/* Mul(C) of a ciphertext with itself followed by relinearisation with the
 * key of s^2 (the square activation, Section IV-F): out = (c0^2 + KS_0(c1^2),
 * 2 c0 c1 + KS_1(c1^2)), scale in.scale^2, no rescale. */
int unihenn_square_relin(const unihenn_ctx* ctx, const unihenn_ct* in, const unihenn_evk* rlk, unihenn_ct* out,
                         void* ws, size_t ws_bytes, void* stream);
/* Add(C) and Add(P) of Section II-B (out may alias a).  add_plain takes a
 * plain-form plaintext (unihenn_encode with mont = 0) at the same scale. */
int unihenn_add(const unihenn_ctx* ctx, const unihenn_ct* a, const unihenn_ct* b, unihenn_ct* out, void* stream);
int unihenn_add_plain(const unihenn_ctx* ctx, const unihenn_ct* a, const uint64_t* pt, unihenn_ct* out,
                      void* stream);
/* Drop-Level as Section IV-A states it: the input (n_limbs = l + 1) is
 * multiplied by n_ones encryptions of all-ones vectors, each product
 * relinearised (unihenn_mul_relin) and rescaled (unihenn_rescale), so out
 * has n_limbs - n_ones limbs.  ones[k] (host array of descriptors) must
 * share the input's batch and hold at least n_limbs - k limbs (it is used
 * dropped to its product's level).  out->scale = in.scale * prod_k
 * ones[k].scale / q_(n_limbs-1-k); all-ones vectors encrypted at scale
 * q_(n_limbs-1-k) keep the input scale exactly.  ws: at least
 * unihenn_drop_level_workspace_size(n_limbs, batch) bytes.  out may alias
 * no operand.  Errors: ELEVEL (n_ones outside 1 .. n_limbs - 1, short
 * operands), EINVAL, ENOKEY. */
size_t unihenn_drop_level_workspace_size(const unihenn_ctx* ctx, uint32_t n_limbs, uint32_t batch);
int unihenn_drop_level(const unihenn_ctx* ctx, const unihenn_ct* in, const unihenn_ct* ones, uint32_t n_ones,
                       const unihenn_evk* rlk, unihenn_ct* out, void* ws, size_t ws_bytes, void* stream);
/* Drop-Level (Section IV-A) read as discarding the top limbs: copy the first
 * n_limbs_out limbs of each polynomial into out; exact and free (the
 * network's input reduction). */
int unihenn_mod_drop(const unihenn_ctx* ctx, const unihenn_ct* in, uint32_t n_limbs_out, unihenn_ct* out,
                     void* stream);

/* ---------------------------------------------------------------- network */
enum {
    UNIHENN_LAYER_CONV = 1,     /* Algorithm 1: ch_in, ch_out, k, s; dims 1 = 1 x k kernel  */
    UNIHENN_LAYER_SQUARE = 2,   /* x^2 activation                                         */
    UNIHENN_LAYER_AVGPOOL = 3,  /* Section IV-C: k = c (kernel and stride)                 */
    UNIHENN_LAYER_FLATTEN = 4,  /* Section IV-E                                            */
    UNIHENN_LAYER_FC = 5,       /* Algorithm 2: ch_in = DAT_in, ch_out = DAT_out            */
    UNIHENN_LAYER_RELU_APPROX = 6 /* Section V-A: f(x) = a + b x + c x^2; weights (or NULL for
                                   * the paper's 0.375373, 0.5, 0.117071) holds (a, b, c)   */
};

typedef struct {
    int32_t kind;
    uint32_t ch_in, ch_out, k, s, dims;
    const double* weights;  /* host; conv [ch_out][ch_in][kh][k], fc [ch_out][ch_in] */
    const double* bias;     /* host; [ch_out] */
    uint32_t pad;           /* conv: zero padding on each side (1D: of the width), Section VI;
                             * reads land in the input's lead and row-pitch margin */
} unihenn_layer;

/* Input tensor (C, H, W) flattened row-major into the slots (Section III-A);
 * `samples` inputs per ciphertext at slot stride `stride` (Section III-B);
 * stride is ignored for one sample.  Padding space (Section VI): each sample
 * starts with `lead` zero slots and its rows sit at pitch `pitch` (0: w;
 * the columns past w are zero), so channel c's row y starts at
 * b * stride + lead + (c h + y) pitch.  A convolution of padding P reading
 * at interval I needs pitch - (map width) >= P and lead >= I (P pitch + P);
 * its input map must be zero off its valid slots (the input, a convolution
 * or activation output; not a pooled map) with one ciphertext per channel
 * (or one channel); net_create fails with EINVAL otherwise. */
typedef struct {
    uint32_t c, h, w;
    uint32_t samples;
    uint32_t stride;
    uint32_t pitch;
    uint32_t lead;
} unihenn_input;

/* Plan a network and encode its plaintexts on the device: the rotation
 * amounts of Algorithms 1 and 2, pooling and flatten, the structured kernel
 * vectors (weights on the valid output slots), masks and FC diagonals.  The
 * input ciphertext is first reduced to depth + 1 limbs.  Allocates the
 * plaintexts and a workspace for batches up to max_batch ciphertexts.
 * Errors: EINVAL (bad shapes, K < S: Theorem 1), ESLOTS (a sample's
 * footprint exceeds its stride or the slots, Section VI), ELEVEL (depth + 1 >
 * n_data), ENOMEM. */
int unihenn_net_create(const unihenn_ctx* ctx, const unihenn_input* input, const unihenn_layer* layers,
                       uint32_t n_layers, uint32_t max_batch, unihenn_net** out);

/* Plan options of unihenn_net_create_ex (or-ed).
 *   UNIHENN_PLAN_LAZY_MODDOWN  deferred ModDown, an evaluator variant of this
 *     library (the paper's evaluator rounds after every key switch): a
 *     rotation keeps its key-switch output over {q_0..q_l, P} as
 *     (P tau(c0) + U_0, U_1) (hybrid key switching with one special prime
 *     P, Section II-B's Rot); the multiply-accumulate sums of Algorithms 1
 *     and 2, the pooling sums of Section IV-C and the flatten sums of
 *     Section IV-E run over that basis (plaintexts carry their residue mod
 *     P), and one ModDown per sum replaces one per rotation.  A rotation by
 *     0 passes its input through; a rotation source, a plaintext addition,
 *     a product and the network outputs take the ModDown first.  Results
 *     differ from the default plan in their last bits (each sum is rounded
 *     once instead of once per term); the decrypted outputs meet the same
 *     bounds.
 *   UNIHENN_PLAN_FC_DOUBLING  Algorithm 2's closing sum of
 *     ceil(DAT_in / DAT_out) rotated copies by doubling, another variant of
 *     this library: S_1 = x, S_2m = S_m + Rot(S_m, m DAT_out), then one
 *     rotation per further set bit of the copy count, floor(log2 reps) +
 *     popcount(reps) - 1 rotations instead of reps - 1 (fewer rotation keys
 *     too).  The same sum slot by slot; results differ in their last bits.
 *   UNIHENN_PLAN_CHANNEL_CTS  a multi-channel input arrives as c ciphertexts,
 *     channel i's (h, w) plane at offset 0 of ciphertext i (sample b at
 *     b * stride; Section III-A lays out one channel per plane), so inputs
 *     whose c h w exceeds a sample's slots fit; the sample footprint counts
 *     h w for the input.  unihenn_eval_network then reads c input
 *     descriptors.
 */
enum { UNIHENN_PLAN_LAZY_MODDOWN = 1, UNIHENN_PLAN_FC_DOUBLING = 2, UNIHENN_PLAN_CHANNEL_CTS = 4 };
/* unihenn_net_create with plan options (plan_flags, 0 = the default plan).
 * Errors: as unihenn_net_create, and EINVAL for an unknown flag. */
int unihenn_net_create_ex(const unihenn_ctx* ctx, const unihenn_input* input, const unihenn_layer* layers,
                          uint32_t n_layers, uint32_t max_batch, uint32_t plan_flags, unihenn_net** out);
int unihenn_net_destroy(unihenn_net* net);
/* depth, number of distinct rotation keys, number of output ciphertexts,
 * and the number of limbs the input is reduced to. */
int unihenn_net_info(const unihenn_net* net, uint32_t* depth, uint32_t* n_rotations, uint32_t* n_outputs,
                     uint32_t* input_limbs);
/* The rotation amounts (in [1, N/2)) whose keys the evaluation needs;
 * steps (host) must hold unihenn_net_info's n_rotations entries. */
int unihenn_net_rotations(const unihenn_net* net, int32_t* steps);
/* Input ciphertexts per evaluation: 1, or c with UNIHENN_PLAN_CHANNEL_CTS. */
int unihenn_net_inputs(const unihenn_net* net, uint32_t* n_inputs);
/* Bind keys: gks[i] is the rotation key of steps[i]; rlk the key of s^2.
 * The descriptors are copied; the key memory must outlive the net's use.
 * Errors: ENOKEY if a needed rotation is missing. */
int unihenn_net_bind_keys(unihenn_net* net, const int32_t* steps, const unihenn_evk* gks, uint32_t n,
                          const unihenn_evk* rlk);

enum { UNIHENN_EVAL_PLAIN = 0, UNIHENN_EVAL_HOISTED = 1, UNIHENN_EVAL_GRAPH = 2 };
/* PLAIN: each rotation does its own key switch, layer by layer.  HOISTED:
 * rotations of one ciphertext share the digit decomposition; results are
 * bit-identical.  GRAPH may be or-ed into either: unihenn_eval_network then
 * records its launches once into a HIP graph (per batch size and buffer
 * set, up to 16 per net) on an idle stream of the net's own, and replays it
 * on the caller's stream.  Replacing or dropping a graph synchronizes the
 * device.  While kernel timing (unihenn_stats_enable) is on, launches are
 * issued directly. */
int unihenn_net_set_mode(unihenn_net* net, int mode);

/* One convolution layer (Algorithm 1) of the net, layer index `layer`:
 * in[i] is the ciphertext holding input channel i (or one ciphertext with
 * all channels for a multi-channel input); out[o] receives output channel o
 * (buffers of [batch][2][n_limbs-1][N]).  interval_out (host) receives
 * I_out = I_in * S.  Uses the net's workspace; not concurrent with other
 * calls on the same net. */
int unihenn_conv(const unihenn_ctx* ctx, unihenn_net* net, uint32_t layer, const unihenn_ct* in, uint32_t n_in,
                 unihenn_ct* out, uint32_t* interval_out, void* stream);

/* Whole network: in is a batch of input ciphertexts (at >= depth+1 limbs,
 * scale Delta), or unihenn_net_inputs' count of such descriptors (one per
 * input channel, equal batch, limbs and scale); out (host array of
 * n_outputs descriptors) receives the output ciphertexts at 1 limb (buffers
 * [batch][2][1][N]).  Uses the net's workspace.  Errors: ENOKEY (keys not
 * bound), ELEVEL, EINVAL (batch > max_batch, inputs that differ). */
int unihenn_eval_network(const unihenn_ctx* ctx, unihenn_net* net, const unihenn_ct* in, unihenn_ct* out,
                         void* stream);

/* Layer stages, for continuous batching of a stream of requests (the
 * multi-request service of Fig. 1): stage k is layer k of the plan (stage 0
 * also reduces the inputs to the network's level).  unihenn_eval_stage runs
 * one stage on the ciphertexts in batch slots [slot, slot + batch) of the
 * net's own registers (slot + batch <= max_batch): stage 0 reads `in`
 * (unihenn_net_inputs' count of descriptors of `batch` ciphertexts, as for
 * unihenn_eval_network), the last stage writes `out` (n_outputs descriptors
 * of `batch` ciphertexts at 1 limb); other stages ignore both (may be NULL).
 * A group of slots must run stages 0, 1, ..., n_stages - 1 in order; groups
 * on disjoint slots may interleave their stages in any order, because each
 * launch touches only its own slots, so requests that arrive while others
 * are in flight join at the next layer boundary.  Results equal those of
 * unihenn_eval_network bit for bit.  The stages of a net share its
 * workspace: issue all of them on one stream.  With UNIHENN_EVAL_GRAPH in the
 * net's mode each (stage, slot range, buffer set) is captured into a HIP
 * graph once (up to 256 per net) and replayed on the caller's stream.
 * Errors: EINVAL
 * (stage or slots out of range, missing inputs or outputs), ELEVEL, ESCALE,
 * ENOKEY, EDEVICE. */
int unihenn_net_stages(const unihenn_net* net, uint32_t* n_stages);
int unihenn_eval_stage(const unihenn_ctx* ctx, unihenn_net* net, uint32_t stage, uint32_t slot, uint32_t batch,
                       const unihenn_ct* in, unihenn_ct* out, void* stream);
/* Device memory of a net: fixed_bytes of encoded plaintexts, and
 * per_slot_bytes for each of its max_batch batch slots (registers and the
 * slot's share of the workspace), for admission by HBM footprint. */
int unihenn_net_memory(const unihenn_net* net, size_t* fixed_bytes, size_t* per_slot_bytes);
/* Device workspace a net uses for an evaluation of `batch` ciphertexts.  The
 * net allocates it at unihenn_net_create, laid out for max_batch ciphertexts
 * (so that captured graphs and the layer stages of every slot range keep one
 * address), and grows it when the tuner picks larger rotation groups; bytes
 * (host) receives its current size, the same for every batch up to
 * max_batch.  Errors: EINVAL (batch outside 1..max_batch, a net of another
 * context). */
int unihenn_workspace_size(const unihenn_ctx* ctx, const unihenn_net* net, uint32_t batch, size_t* bytes);

/* Slots of the network output: for sample b and output value v,
 * positions[b * n_values + v] is (output ciphertext index << 32) | slot.
 * n_values (host) receives the number of values per sample. */
int unihenn_net_output_slots(const unihenn_net* net, uint64_t* positions, uint32_t* n_values);

/* ------------------------------------------------------------ autotuning */
/* Launch parameters of the batched evaluator.  Every setting computes the
 * same results bit for bit; only speed changes.
 *   ntt_split     stages in the NTT column pass (the row pass does the rest)
 *   ntt_tile_log  LDS tile of the radix-8 NTT passes: 11 or 12 (2^t words)
 *   mac_min_wg    workgroups a multi-output MAC launch aims for (it trades
 *                 outputs per thread against parallelism)
 *   ks_min_wg     workgroups a key-switch inner product aims for (it splits
 *                 the batch to reach it)
 *   ks_group      rotations per grouped key-switch launch set, 1..64 (net
 *                 only)
 *   ks_order      workgroup order of the grouped inner product: 0 batch
 *                 chunks fastest (keys re-read from cache), 1 rotations
 *                 fastest (digits re-read from cache), 2 (plain rotations;
 *                 others take 0) one workgroup per output row that runs the
 *                 row pass of the digits' forward NTT in LDS and accumulates
 *                 its outputs, so the transformed digits never reach memory
 *                 (launches below 384 workgroups, or the value of the
 *                 environment variable UNIHENN_KS_FUSE_MIN_WG when the
 *                 context was created, stay unfused)
 *   ntt_ms, net_ms  timings of the chosen setting (filled by autotune) */
typedef struct {
    int32_t ntt_split;
    int32_t ntt_tile_log;
    int32_t mac_min_wg;
    int32_t ks_min_wg;
    int32_t ks_group;
    int32_t ks_order;
    double ntt_ms;
    double net_ms;
} unihenn_tuning;
/* Time candidate settings on the device and keep the fastest: first the NTT
 * split and tile on a forward + inverse transform of a batch of rows sized
 * from `batch`; then, when net is non-NULL and its keys are bound, one
 * coordinate at a time (NTT split and tile, group size with each workgroup
 * order, the two workgroup targets) on whole evaluations of `batch` ciphertexts in the net's mode
 * (graph replay included when set).  With a non-NULL cache_path the result
 * is looked up in, and then written to, a JSON file keyed by device, ring,
 * batch, a fingerprint of the net's plan and its mode (set the mode first);
 * a hit applies the stored setting without timing.  The chosen setting is
 * applied to ctx (and net) and returned in *out (may be NULL).  Allocates
 * scratch buffers, may grow the net's workspace and drops its captured
 * graphs; must not run concurrently with other calls on ctx or net.
 * Synchronous. */
int unihenn_autotune(unihenn_ctx* ctx, unihenn_net* net, uint32_t batch, const char* cache_path,
                     unihenn_tuning* out, void* stream);
/* Current setting of ctx (and net, when non-NULL; ks_group is 0 without). */
int unihenn_tuning_get(const unihenn_ctx* ctx, const unihenn_net* net, unihenn_tuning* out);
/* Apply a setting; fields <= 0 keep their current value.  Drops the net's
 * captured graphs.  Errors: EINVAL (split outside 1..log_n-1, tile not 11 or
 * 12, group above the library limit), ENOMEM. */
int unihenn_tuning_set(unihenn_ctx* ctx, unihenn_net* net, const unihenn_tuning* t);

/* ---------------------------------------------------------------- client */
/* A client for benchmarks and examples (the paper's client encrypts and
 * decrypts, Section III; Fig. 1).  Randomness: a counter-based hash of
 * (seed, stream, index); a research generator, not a cryptographic one.
 * sk: device [n_data + 1][N], NTT form over q_0..q_L, P. */
int unihenn_keygen_secret(const unihenn_ctx* ctx, uint64_t seed, uint64_t* sk, void* stream);
/* Switching key for Rot(., steps) (steps != 0) or, with relin != 0, for s^2;
 * written in the unihenn_import_evk device form ([n_data][2][n_data+1][N]). */
int unihenn_gen_switch_key(const unihenn_ctx* ctx, const uint64_t* sk, uint64_t seed, int32_t steps, int relin,
                           uint64_t* out, void* stream);
/* Encrypt plain-form plaintexts under the secret key: ct = (-a s + e + m, a)
 * for each of ct->batch plaintexts pts[b] ([n_limbs][N], mont = 0). */
int unihenn_encrypt_sk(const unihenn_ctx* ctx, const uint64_t* sk, const uint64_t* pts, uint64_t seed,
                       unihenn_ct* ct, void* stream);
/* Decrypt and decode selected slots: values[b * n_slots + i] (host) is slot
 * slot_index[i] of ciphertext b.  Decodes from limb q_0 alone, which is exact
 * while |scale * value| stays below q_0 / 2.  Synchronous. */
int unihenn_decrypt_slots(const unihenn_ctx* ctx, const uint64_t* sk, const unihenn_ct* ct,
                          const uint32_t* slot_index, uint32_t n_slots, double* values, void* stream);

/* ------------------------------------------------------------ measurement */
/* Per-kernel-family launch timing with HIP events recorded on the launch
 * stream around each launch (adds a little overhead while on).  KS_INNER
 * counts the separate key-switch inner products (and relinearisation);
 * KS_ROWFUSED counts the inner products fused with ModUp's row pass (one
 * kernel, k_ntt_r8_ksrow). */
enum {
    UNIHENN_KF_NTT_FWD_COL = 0, UNIHENN_KF_NTT_FWD_ROW, UNIHENN_KF_NTT_INV_ROW, UNIHENN_KF_NTT_INV_COL,
    UNIHENN_KF_MODUP, UNIHENN_KF_KS_INNER, UNIHENN_KF_MODDOWN, UNIHENN_KF_RESCALE, UNIHENN_KF_MAC, UNIHENN_KF_AUTO,
    UNIHENN_KF_TENSOR, UNIHENN_KF_ADD, UNIHENN_KF_ENCODE, UNIHENN_KF_OTHER, UNIHENN_KF_KS_ROWFUSED,
    UNIHENN_KF_COUNT
};
int unihenn_stats_enable(int on);
int unihenn_stats_reset(void);
/* Synchronises the device, then reports launches, total milliseconds,
 * algorithmic bytes (inputs read once + outputs written once) and algorithmic
 * operations (NTT butterflies; 0 for other families) of a family.  Each NTT
 * pass is its own family, one kernel dispatch per launch. */
int unihenn_stats_get(int family, uint64_t* launches, double* total_ms, double* bytes, double* ops);
const char* unihenn_kernel_family_name(int family);

#ifdef __cplusplus
}
#endif
#endif
