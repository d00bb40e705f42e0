/*
 * qkc_cpu.h -- a plain CPU evaluator of the same arithmetic circuits
 * (libqkc_cpu.so, host only): the baseline the GPU library is timed against.
 *
 * It reads the blob that ac_load reads (layout in qkc.h) and evaluates the
 * AC directly, node by node in the blob's level order, in complex128 with
 * one thread per batch element or chain (OpenMP):
 *
 *   - upward pass (Huang et al., ASPLOS'21, Sec. 3.3.1): sum and product
 *     nodes over their children, leaves from the evidence (indicators), the
 *     angles and the noise strengths (weights);
 *   - downward pass (Sec. 3.3.2): d root / d node for every node, products
 *     through prefix and suffix products of the other children (no
 *     division), giving d root / d lambda_{v=u} for every variable value;
 *   - Gibbs sampling (Sec. 3.3.2) with the rules and the counter-based
 *     random numbers documented for ac_sample: systematic scan, one downward
 *     pass serving every visit up to and including the first change.
 *
 * It shares no code with the GPU library: its own blob reader, weights and
 * passes.  All pointers are host pointers owned by the caller.  Functions
 * return 0 on success, nonzero on error with qkc_cpu_last_error() set
 * (thread-local).
 */
#ifndef QKC_CPU_H
#define QKC_CPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qkc_cpu qkc_cpu;

/* Parse a blob (see ac_load); the caller may free it on return. */
int qkc_cpu_load(const void *blob, size_t nbytes, qkc_cpu **out);
void qkc_cpu_free(qkc_cpu *ac);
const char *qkc_cpu_last_error(void);

/* Sizes: internal nodes, child references, evidence variables, evidence
 * words, angles, output qubits (any pointer may be NULL). */
int qkc_cpu_info(const qkc_cpu *ac, int32_t *n_internal, int64_t *n_edges, int32_t *n_vars,
                 int32_t *n_words, int32_t *n_angles, int32_t *n_qubits);

/* Upward pass: amp_out[2b], amp_out[2b+1] = re, im of
 * f(evidence[b]; theta[param_of[b]], noise) for b in [0, B); theta float64
 * [P][n_angles]; noise NULL for the blob's strengths; evidence uint64
 * [B][n_words]; threads <= 0 for the OpenMP default. */
int qkc_cpu_eval(const qkc_cpu *ac, const double *theta, int32_t P, const double *noise,
                 const int32_t *param_of, const uint64_t *evidence, int64_t B, double *amp_out,
                 int threads);

/* Gibbs chains as ac_sample runs them (chain = p * chains_per_param + c,
 * seeded start, burn_in + samples_per_chain * thin sweeps, sample j after
 * sweep burn_in + (j + 1) * thin): samples_out uint64 [P][S] output bits
 * (n_qubits <= 64), states_out uint64 [P][S][n_words] or NULL, rounds_out
 * int64 [P * chains_per_param] downward passes per chain or NULL. */
int qkc_cpu_sample(const qkc_cpu *ac, const double *theta, int32_t P, const double *noise,
                   int32_t chains_per_param, int32_t samples_per_chain, int32_t burn_in, int32_t thin,
                   uint64_t seed, uint64_t *samples_out, uint64_t *states_out, int64_t *rounds_out,
                   int threads);

#ifdef __cplusplus
}
#endif

#endif /* QKC_CPU_H */
