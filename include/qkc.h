/*
 * qkc.h -- C ABI of the batched arithmetic-circuit (AC) evaluation library
 * for MI355X (gfx950).
 *
 * The method: a noisy variational circuit is compiled once, on the host, into
 * an arithmetic circuit -- a DAG of sum and product nodes whose leaves are
 * indicators of output-qubit and noise-event values and weights (gate entries
 * depending on the variational angles theta, Kraus entries depending on the
 * noise strengths) (Huang et al., ASPLOS'21, Sec. 3.2).  It is then queried
 * many times with new parameters and evidence (Sec. 3, "repeated simulation
 * with different parameters"):
 *
 *   - amplitude of an evidence assignment: one upward pass (Sec. 3.3.1);
 *   - derivatives of the root with respect to every node: one downward pass
 *     (Sec. 3.3.2), which gives the Gibbs transition weights over assignments
 *     one variable away and, by the chain rule, gradients in theta (Sec. 5
 *     lists gradients among the queries);
 *   - samples of output bit strings by Gibbs sampling over outputs and noise
 *     events (Sec. 3.3.2).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array pointers passed to ac_eval_batch / ac_grad_batch / ac_sample
 *   are DEVICE pointers on the graph's device, owned by the caller, and must
 *   stay valid until the work enqueued on `stream` completes.  `stream` is a
 *   hipStream_t (NULL = the null stream).  Calls are asynchronous: AC_OK means
 *   the work was enqueued.
 * - complex64 data is interleaved float pairs (re, im); complex128 is
 *   interleaved double pairs.  The dtype selects the arithmetic of the DAG
 *   passes; weights are always computed in FP64 and rounded, and |f|^2,
 *   Gibbs weights and gradient reductions are always FP64.
 * - theta is float64 [P][n_angles], row-major.  noise is float64 [n_noise]
 *   or NULL for the strengths stored in the blob.
 * - evidence is uint64 [B][n_words]: every evidence variable (output qubits
 *   q0..q(n-1), then the noise events in circuit order) owns a field of
 *   ceil(log2(dom)) bits at the bit offset the blob records, LSB first; a
 *   field never straddles two words.  A noise event's value is the index of
 *   its Kraus operator (depolarizing: 0=I 1=X 2=Y 3=Z).  Field values >= dom
 *   evaluate as "no indicator true" (amplitude 0).
 * - param_of is int32 [B]: the parameter set (row of theta) of each batch
 *   element.  Values outside [0, P) are not checked on the device and are
 *   undefined behaviour; the Python binding validates them.
 * - Every call takes a caller-allocated device workspace; the library never
 *   allocates per call.  ac_workspace_size() bytes run the call at full
 *   width (every workgroup the device holds at once).  A smaller workspace
 *   runs fewer workgroups at once -- as many per-workgroup regions as fit
 *   after the fixed part, at least one -- with the same results, which
 *   leaves the rest of the device to work on other streams; below one region
 *   the call fails with AC_ERR_INVALID_ARG (the LDS-resident sampler has no
 *   regions and always needs the full size).
 * - Errors: a non-AC_OK status is returned before anything is enqueued for
 *   invalid arguments; AC_ERR_DEVICE reports a failed launch.  ac_last_error()
 *   returns a thread-local description of the last failure.  No C++
 *   exception crosses this interface.
 * - A graph handle is immutable after ac_load, so it may be used from several
 *   host threads and streams at once, each call with its own workspace.
 */
#ifndef QKC_H
#define QKC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AC_OK = 0,
    AC_ERR_INVALID_ARG = 1,
    AC_ERR_FORMAT = 2,
    AC_ERR_OOM = 3,
    AC_ERR_DEVICE = 4,
    AC_ERR_UNSUPPORTED = 5
} ac_status;

typedef enum { AC_C64 = 0, AC_C128 = 1 } ac_dtype;

/* Workspace kinds for ac_workspace_size. */
typedef enum { AC_OP_EVAL = 0, AC_OP_GRAD = 1, AC_OP_SAMPLE = 2, AC_OP_MPE = 3 } ac_op;

/* Loss forms for ac_grad_batch (the cotangent g_b of the root value f_b). */
typedef enum {
    AC_GRAD_COTANGENT = 0, /* g_b given in `cotangent` (complex, dtype)        */
    AC_GRAD_PROB = 1,      /* L = sum_b w_b |f_b|^2        -> g_b = 2 w_b f_b   */
    AC_GRAD_LOGPROB = 2    /* L = sum_b w_b log |f_b|^2    -> g_b = 2 w_b f_b / |f_b|^2 */
} ac_grad_mode;

typedef struct ac_graph ac_graph;

typedef struct {
    int32_t n_qubits;
    int32_t n_vars;            /* evidence variables: outputs + noise events   */
    int32_t n_words;           /* uint64 words per evidence assignment         */
    int32_t n_angles;          /* K: columns of theta                          */
    int32_t n_noise;           /* entries of the noise-strength vector          */
    int32_t n_slots;           /* weight leaves                                  */
    int32_t n_angle_slots;     /* weight leaves that depend on theta            */
    int32_t n_internal;        /* sum and product nodes                          */
    int64_t n_edges;           /* child references of internal nodes             */
    int32_t n_levels;          /* longest leaf-to-root path (in internal nodes) */
    int32_t max_level_width;
    int32_t n_indicator_leaves;/* sum over variables of their domain sizes       */
    int32_t root;              /* internal index of the root                     */
    int32_t device;
    int64_t n_prod_flops;      /* real flops of one upward pass (complex ops)  */
    int32_t n_selectors;       /* selector leaves                               */
    /* The sum-of-products plan the streaming sampler and the upward pass run
       on (every product whose only parent is a sum folded into that sum; see
       ac_load).  Zero when the graph has no such plan.  The row counts give
       the plan's bytes per element: upward pass s*(n_super + n_super_node_factors),
       downward pass s*(n_super + n_super_down_reads), leaf derivatives
       s*(n_super_leaf_reads + n_indicator_leaves), s = 8 (c64) or 16 (c128). */
    int32_t n_super;           /* super-nodes (one row each per element)        */
    int32_t n_super_levels;
    int32_t max_live;          /* most super-nodes alive at once in the upward pass
                                  (from a node's level to its last reader's level):
                                  the rows per element an amplitude call keeps;
                                  n_internal when there is no plan             */
    int32_t max_siblings;      /* most siblings (other factors of the term) of one
                                  occurrence of a super-node, indicator or selector
                                  in the plan, 0..3; at most 2 lets the streaming
                                  sampler take larger occurrence groups          */
    int64_t n_super_node_factors; /* factors that are super-nodes (rows read upward) */
    int64_t n_super_down_reads;   /* per occurrence of a super-node as a factor: the
                                     parent's adjoint row and each super-node sibling */
    int64_t n_super_leaf_reads;   /* the same for indicator and selector occurrences */
} ac_info_t;

/*
 * Parse and validate a serialised AC (the blob written by the host compiler)
 * and copy it to `device`.  The caller keeps ownership of `blob` and may free
 * it on return; the library owns the device copy until ac_free.
 *
 * Blob layout (little endian; every array starts on an 8-byte boundary
 * unless marked "packed", which follows the previous array directly):
 *   header   8-byte magic "QKCAC\0\0\1", then 14 uint32: version(=2), flags,
 *            n_qubits, n_vars, n_words, n_angles, n_noise, n_slots,
 *            n_angle_slots, n_internal, n_edges, n_levels, root, n_selectors
 *   uint8    var_dom[n_vars]; uint8 var_kind[n_vars] (packed; 0 output,
 *            1 depolarizing, 2 amplitude damping, 3 phase damping)
 *   uint32   var_offset[n_vars]         bit offset of each evidence field
 *   float64  noise_default[n_noise]
 *   slot     [n_slots] of 32 bytes (packed) {u8 base, u8 coef, u16 0, i32 index,
 *            f64 scale, f64 re, f64 im}; value = coef * base where
 *            coef in {1, -1, i, -i} and base is one of: const (re + i im),
 *            cos(scale*theta[index]/2), sin(..), exp(-i scale theta[index]/2),
 *            exp(+i ..), sqrt(1 - noise[index]), sqrt(noise[index]/3),
 *            sqrt(noise[index]).  The first n_angle_slots depend on theta.
 *   selector [n_selectors] of 5 uint32 (packed) {variable v, slot[4]}: the leaf
 *            sum_u lambda_{v=u} * W[slot[u]] (slot 0xFFFFFFFF: zero), i.e. the
 *            weight of v's current value; v is a noise event with at most 4
 *            values and the slots do not depend on theta.  It is the
 *            compiled form of a channel's Kraus entry (Sec. 3.1: the event's
 *            table holds the Kraus amplitudes).
 *   uint8    op[n_internal] (packed)    0 = sum, 1 = product
 *   uint32   row_ptr[n_internal + 1]    CSR over child references
 *   uint32   col[n_edges]               child reference: bits 31..30 tag,
 *            tag 0 = internal node index (bits 29..0),
 *            tag 1 = indicator, variable in bits 23..0, value in bits 29..24,
 *            tag 2 = weight slot index (bits 29..0),
 *            tag 3 = selector index (bits 29..0)
 *   uint32   level_ptr[n_levels + 1]    nodes are sorted by level; level l
 *            holds [level_ptr[l-1], level_ptr[l]) and every internal child
 *            of a node lies on a lower level.
 * Returns AC_ERR_FORMAT for any inconsistency, AC_ERR_OOM if device memory
 * runs out, AC_ERR_DEVICE for other HIP failures.
 */
ac_status ac_load(const void *blob, size_t nbytes, int device, ac_graph **out);

/* Release the device copy and the handle.  NULL is accepted. */
ac_status ac_free(ac_graph *g);

/* Sizes needed to shape the caller's tensors. */
ac_status ac_info(const ac_graph *g, ac_info_t *info);

/* Thread-local text of the last error ("" if none). */
const char *ac_last_error(void);

/*
 * Bytes of device workspace needed by one call of kind `op` with `batch`
 * elements (for AC_OP_SAMPLE: batch = P * chains_per_param).  Returns 0 for
 * invalid arguments.  The size depends on the device's compute-unit count.
 */
size_t ac_workspace_size(const ac_graph *g, ac_dtype dtype, int64_t batch, int op);

/*
 * Bytes of workspace for the same call run on a share of the device: at most
 * ceil(share * W) workgroups at once, W being the workgroups the full-size
 * workspace runs (share in (0, 1]; results are the same, the call takes
 * longer and leaves the rest of the device to other streams).  Equal to
 * ac_workspace_size when the call has no per-workgroup regions or runs one
 * workgroup.  Returns 0 for invalid arguments.
 */
size_t ac_workspace_size_share(const ac_graph *g, ac_dtype dtype, int64_t batch, int op, double share);

/* Sampler kernels, as reported by ac_sample_shape. */
typedef enum { AC_SAMPLER_STREAM = 0, AC_SAMPLER_LDS = 1, AC_SAMPLER_GLOBAL = 2 } ac_sampler_kind;

/*
 * Which Gibbs-sampler kernel ac_sample runs for `chains` chains
 * (P * chains_per_param) in `dtype` on this graph's device, and how many
 * chains it advances at once (the rest wait for a free slot), so a scheduler
 * can estimate a call's device time before making it.  Host-only; writes
 * *kind (an ac_sampler_kind) and *concurrent.  AC_ERR_INVALID_ARG for a null
 * graph or output, a bad dtype or chains < 1.
 */
ac_status ac_sample_shape(const ac_graph *g, ac_dtype dtype, int64_t chains, int32_t *kind, int64_t *concurrent);

/*
 * Upward pass (Sec. 3.3.1) for a batch: amp_out[b] = f(evidence[b]; theta[param_of[b]], noise)
 * for b in [0, B).  prob_out (optional, may be NULL) receives |amp|^2 in
 * FP64.  amp_out is complex64 or complex128 [B] as selected by dtype.
 * B = 0 enqueues nothing and returns AC_OK.  param_of lives on the device and
 * is not checked on the host: an entry outside [0, P) reads no parameters and
 * yields a NaN amplitude (and, in ac_grad_batch, NaN raw derivatives and no
 * gradient contribution).
 */
ac_status ac_eval_batch(const ac_graph *g, ac_dtype dtype,
                        const double *theta, int32_t P, const double *noise,
                        const int32_t *param_of, const uint64_t *evidence, int64_t B,
                        void *amp_out, double *prob_out,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * Allocation-free upward pass, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as ac_eval_batch
 * (bit for bit the same amplitudes and probabilities), without the
 * workspace: the fixed weights and the per-workgroup node rows live in a
 * library-owned device array of AC_STATIC_SCRATCH_BYTES on each GPU, whose
 * address ac_load resolves once per device and which the device holds until
 * the process ends.  The call allocates nothing (no hipMalloc or allocating
 * library routine) and launches as many workgroups as the array holds node
 * rows for.  Returns AC_ERR_UNSUPPORTED, before enqueuing anything, when the
 * fixed weights (16 bytes per slot) plus one 64-element tile's node rows
 * (n_internal * 64 * 8 bytes in complex64, * 16 in complex128), each rounded
 * up to 256 bytes, exceed AC_STATIC_SCRATCH_BYTES.  Every call on a GPU
 * shares that GPU's array and leaves its last contents there (nothing in it
 * needs clearing: each call writes what it reads), so calls that overlap in
 * time on one GPU race: serialise them (one stream, or events).
 */
#define AC_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
ac_status ac_eval_batch_static(const ac_graph *g, ac_dtype dtype,
                               const double *theta, int32_t P, const double *noise,
                               const int32_t *param_of, const uint64_t *evidence, int64_t B,
                               void *amp_out, double *prob_out, void *stream);

/*
 * Upward + downward pass and chain rule (Sec. 3.3.2 downward pass; Sec. 5
 * gradients).  With g_b the cotangent of f_b chosen by `mode`:
 *
 *   grad_theta[p][j] = sum over b with param_of[b] = p of Re(g_b * conj(df_b/dtheta_j))
 *
 * which is dL/dtheta for a real loss L of the complex f_b when g_b =
 * dL/dRe f_b + i dL/dIm f_b.  grad_theta (float64 [P][n_angles]) is
 * overwritten; the sum runs in FP64 in a fixed order (bitwise reproducible).
 * weight (float64 [B]) is required for AC_GRAD_PROB / AC_GRAD_LOGPROB;
 * cotangent (complex, dtype, [B]) for AC_GRAD_COTANGENT.  Under LOGPROB an
 * element with f_b = 0 contributes 0.
 * Optional outputs (NULL to skip): amp_out [B] (dtype), dfdtheta_out [B][n_angles]
 * complex (dtype) = df_b/dtheta_j, dind_out [B][n_indicator_leaves] complex
 * (dtype) = df_b/dlambda_{v=u} (variables in order, values within), which by
 * multilinearity equals the amplitude of evidence b with v set to u.
 */
ac_status ac_grad_batch(const ac_graph *g, ac_dtype dtype,
                        const double *theta, int32_t P, const double *noise,
                        const int32_t *param_of, const uint64_t *evidence, int64_t B,
                        int mode, const void *cotangent, const double *weight,
                        double *grad_theta, void *amp_out, void *dfdtheta_out,
                        void *dind_out, void *ws, size_t ws_bytes, void *stream);

/*
 * Gibbs sampling (Sec. 3.3.2) of assignments s = (x, k) with weight
 * |f(s)|^2, whose x-marginal is the output distribution rho_xx.
 * Single-site systematic scan over the evidence variables in order; variable
 * v takes value u with probability |df/dlambda_{v=u}|^2 / sum_u' |..|^2, the
 * derivatives coming from one downward pass, which stays valid until the
 * first change, so one pass serves every variable up to and including the
 * first one that changes.  Zero total weight keeps the current value; the
 * inverse CDF takes the smallest u with r * sum(w) < w_0 + ... + w_u.
 *
 * Randomness: r = (mix(seed ^ mix(chain ^ mix((sweep << 20) ^ var))) >> 11) * 2^-53
 * with mix(z) the SplitMix64 finaliser of z + 0x9E3779B97F4A7C15 (Steele, Lea
 * and Flood, OOPSLA 2014); chain = chain_offset + p * chains_per_param + c;
 * the sweeps of a call are numbered first_sweep, first_sweep + 1, ...  A
 * call over parameter sets p0 .. p0 + P - 1 of a larger request (theta from
 * row p0, chain_offset = p0 * chains_per_param), or over chains c0 ..
 * c0 + C - 1 of one parameter set p (P = 1, chains_per_param = C,
 * chain_offset = p * chains_per_param_of_the_request + c0), draws exactly
 * the chains of the whole request.  Initial state:
 * init_states[chain] (all n_words words: outputs and noise events) if
 * init_states is given, else output bit q = [r(seed, chain, 0xFFFFFFFF, q) < 1/2]
 * and every noise event 0.  Chain c of parameter set p runs burn_in +
 * samples_per_chain * thin sweeps and records its state after sweep burn_in +
 * (j + 1) * thin of the call as sample j.  Results are deterministic for fixed
 * inputs and independent of other work.
 *
 * Conditional sampling: with first_var > 0 the scan visits only variables
 * first_var .. n_vars - 1 and variables 0 .. first_var - 1 keep their start
 * values, so the chains sample the conditional law of the remaining
 * variables; with first_var = n_qubits and init_states holding an observed
 * outcome x, the noise events follow P(k | x), proportional to |f(x, k)|^2
 * (which error events explain an observed outcome).
 *
 * Resuming chains: a call started from the last recorded state of each chain
 * (states_out of sample samples_per_chain - 1) with first_sweep advanced by
 * the previous call's sweeps and the same seed continues exactly the chains of
 * one longer call; the caller owns those states, so they can stay resident in
 * device memory between the optimiser's iterations.
 *
 * Outputs, with S = chains_per_param * samples_per_chain and sample index
 * c * samples_per_chain + j:
 *   samples    uint64 [P][S][ceil(n_qubits/64)]  output bits (required)
 *   states_out uint64 [P][S][n_words]            full evidence words (optional)
 *   cost_out   float64 [P][S]  MaxCut cost of the sample over cost_edges (optional;
 *              NaN if an edge names a qubit outside [0, n_qubits))
 *   rounds_out int64 [P * chains_per_param] downward passes each chain used (optional)
 * cost_edges is a device int32 [n_cost_edges][2] array (NULL if n_cost_edges = 0);
 * init_states is a device uint64 [P * chains_per_param][n_words] array or NULL.
 * Any bit pattern is a valid state (ac_load accepts only power-of-two domains).
 * Requires n_qubits <= 64, seed < 2^64, first_sweep + sweeps per chain < 2^32 - 1,
 * n_vars < 2^20, first_var < n_vars, reserved 0.
 */
typedef struct {
    int32_t chains_per_param;
    int32_t samples_per_chain;
    int32_t burn_in_sweeps;
    int32_t thin_sweeps;
    uint64_t seed;
    int32_t n_cost_edges;
    int32_t reserved;
    const int32_t *cost_edges;
    const uint64_t *init_states;
    uint32_t first_sweep;
    uint32_t first_var;
    uint64_t chain_offset;   /* RNG chain number of chain 0 (see above); <= 2^62 */
} ac_sample_cfg;

ac_status ac_sample(const ac_graph *g, ac_dtype dtype,
                    const double *theta, int32_t P, const double *noise,
                    const ac_sample_cfg *cfg,
                    uint64_t *samples, uint64_t *states_out, double *cost_out,
                    int64_t *rounds_out,
                    void *ws, size_t ws_bytes, void *stream);

/*
 * Most probable explanation of observed outcomes (Huang et al., ASPLOS'21,
 * Sec. 5: which noise events best explain an outcome; the maximum is taken
 * over real error probabilities, not amplitudes).  For each element b, with
 * the outputs x_b from evidence[b] (its noise-event fields are ignored) and
 * angles theta[param_of[b]]:
 *   prob_out[b] = max_k |f(x_b, k)|^2 = P(x_b, k*)   float64 [B]
 *   mpe_out[b]  = evidence words of (x_b, k*)        uint64 [B][n_words]
 * computed by max-product over the noise events: nodes with an event
 * indicator below them hold the largest |value|^2 over those events
 * (products multiply, sums keep their largest branch), the rest complex
 * values; a top-down pass reads k* off the largest branches (the first in
 * child order on ties, so k* is one of the maximisers).  Exact when every
 * sum with an event below it decides one evidence variable and a product's
 * children share no event -- an AC compiled with the events explicit and
 * decided first (the search-based compiler's MPE mode); ac_load checks the
 * decisions and this call returns AC_ERR_UNSUPPORTED for other ACs (with
 * selector leaves, for one).  complex128 only; noise as in ac_eval_batch.
 * Workspace: ac_workspace_size(g, AC_C128, B, AC_OP_MPE).  Pointers are
 * device pointers owned by the caller; param_of values outside [0, P) give
 * NaN.
 */
ac_status ac_mpe_batch(const ac_graph *g, const double *theta, int32_t P, const double *noise,
                       const int32_t *param_of, const uint64_t *evidence, int64_t B, double *prob_out,
                       uint64_t *mpe_out, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QKC_H */
