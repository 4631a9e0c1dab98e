/*
 * paraqaoa.h -- C ABI of libparaqaoa, the MI355X (gfx950) hot path of
 * ParaQAOA (arXiv 2603.26232): batched depth-p QAOA state-vector simulation
 * of the subgraphs produced by the divide-and-conquer partition, the cut
 * expectation, top-k bitstring extraction, integer cut evaluation of merged
 * full-graph assignments and the merge itself.
 *
 * Conventions (all entry points):
 *   - A subgraph with n vertices is simulated on n qubits; amplitude index z
 *     has bit j = local vertex j (local order = increasing global index), and
 *     bit value 1 puts the vertex in S (the bitstring picture of Sec. 2.4).
 *   - H_C = diag(C(z)) with C(z) = sum over edges of w_uv [z_u != z_v] (the
 *     Max-Cut objective of Sec. 2.1); H_M = sum_j X_j; U_C = e^{-i gamma H_C},
 *     U_M = e^{-i beta H_M}; |psi> = U_M(b_p)U_C(g_p)...U_M(b_1)U_C(g_1)|+>^n
 *     (the QAOA ansatz of Sec. 2.2).
 *   - Angles, <C> and gradients are IEEE double; amplitudes are complex64
 *     on the device; cut values are int64.
 *   - Pointers named d_* are device pointers (HBM); h_* / plain pointers
 *     named in "host" comments are host pointers. The caller owns every
 *     buffer, device and host; the library never frees caller memory.
 *   - Every call that takes a stream only enqueues work on it and never
 *     synchronises the device. qaoa_batch_create and qaoa_merge_beam copy
 *     the host arrays they need into one of four pinned staging buffers
 *     owned by the library (used in turn, kept until the process ends,
 *     grown as needed) and enqueue the upload on `stream`; the host arrays
 *     may be reused on return. A call waits only if the upload made four
 *     calls earlier has not yet left its staging buffer. Outputs are valid once the caller synchronises the
 *     stream. A handle must not be used by two host threads at once.
 *   - Errors are reported as status codes only; nothing aborts or throws.
 *     All arguments are checked before any work is enqueued; on an error
 *     no work is enqueued and qaoa_last_error() holds a message
 *     (thread-local, valid until the next call on the same thread).
 *   - For identical inputs on the same device and build, every output is
 *     bit-identical (fixed-order reductions, no floating-point atomics).
 */
#ifndef PARAQAOA_H
#define PARAQAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QAOA_OK = 0,
    QAOA_ERR_INVALID_ARG = 1,          /* NULL where a pointer is required, bad id, ... */
    QAOA_ERR_OUT_OF_RANGE = 2,         /* n > 30, p > 32, k > 64, W too large, ... */
    QAOA_ERR_WORKSPACE_TOO_SMALL = 3,  /* workspace smaller than *_workspace_bytes */
    QAOA_ERR_HIP = 4,                  /* a HIP runtime call failed (text in last_error) */
    QAOA_ERR_STATE = 5,                /* call order violated (e.g. top-k before apply) */
    QAOA_ERR_NOT_SUPPORTED = 6         /* e.g. a subgraph's weight sum above 2047 */
} qaoa_status_t;

/* Opaque handle: host metadata plus views into the caller's workspace. */
typedef struct qaoa_batch_s* qaoa_batch_t;

/* A hipStream_t passed as an untyped pointer; NULL means the null stream. */
typedef void* qaoa_stream_t;

#define QAOA_MAX_QUBITS 30
#define QAOA_MAX_DEPTH 32
#define QAOA_MAX_K 64
#define QAOA_MAX_WEIGHT_SUM 2047 /* per subgraph: sum of its edge weights */
#define QAOA_MAX_BEAM 8192

/* create flags */
#define QAOA_FLAG_GRADIENT 0x1u /* reserve the adjoint state; enables qaoa_expectation_grad */
#define QAOA_FLAG_TOPK_RAW 0x2u /* top-k over all z; default: only z with bit 0 clear */
/* Do not simulate subgraphs without edges: their state is e^{-i n sum beta}|+>^n,
 * so <C> = 0, the gradient is 0 and every bitstring is equally likely (top-k =
 * the k smallest candidate indices, probability 2^-n). Their states are not
 * stored (qaoa_state_offset reports QAOA_ERR_STATE for them). */
#define QAOA_FLAG_SKIP_EDGELESS 0x4u
/* Precision modes of the mixer (Sec. 2.2: U_M(beta) = prod_j e^{-i beta X_j}).
 * For subgraphs with more than 13 qubits, the rotation of five of the qubits
 * in the first qubit group (local qubits 0..3 and 9) runs as one dense
 * 32 x 32 complex block on the matrix cores instead of the vector units:
 *   MFMA_F32    FP32 matrix products (32x32x2);
 *   MFMA_BF16X3 BF16 matrix products (32x32x16) on hi/lo splits of both
 *               operands (x = hi + lo), keeping hi*hi + hi*lo + lo*hi;
 *   MFMA_BF16X4 as BF16X3, with the block matrix split in three BF16 terms
 *               (hi + mid + lo) and the products hi*hi + hi*lo + mid*hi +
 *               lo*hi, which keeps the block unitary to FP32 rounding.
 * Accumulation is FP32; all other steps are unchanged (FP32 amplitudes). At
 * most one mode may be set (QAOA_ERR_INVALID_ARG otherwise); none can be
 * combined with QAOA_FLAG_GRADIENT (QAOA_ERR_NOT_SUPPORTED). Subgraphs of at
 * most 13 qubits keep the vector path. */
#define QAOA_FLAG_MIXER_MFMA_F32 0x8u
#define QAOA_FLAG_MIXER_MFMA_BF16X3 0x10u
#define QAOA_FLAG_MIXER_MFMA_BF16X4 0x20u
/* Gradient memory of a QAOA_FLAG_GRADIENT batch (results agree to rounding):
 *   QAOA_FLAG_GRADIENT_CHECKPOINTS keeps the state after every HBM pass of
 *     the forward sweep (for subgraphs of more than 13 qubits: max_p (G - 1)
 *     stored states, G = the subgraph's qubit groups; with the default group
 *     split 2 for 14..20 qubits, 3 for 21..28, 4 above), so that the adjoint
 *     sweep reads psi where it needs it and writes only lambda;
 *   QAOA_FLAG_GRADIENT_INPLACE keeps one psi, which the adjoint sweep
 *     rebuilds by undoing each pass (less memory, 8 more bytes per stored
 *     amplitude in each middle backward pass);
 *   neither: checkpoints, unless the batch's states and cut tables fit the
 *     256 MB Infinity Cache in place (224 MiB or less) but not with
 *     checkpoints; then in place.
 * Setting both is QAOA_ERR_INVALID_ARG. qaoa_gradient_checkpoints tells which
 * a batch uses. */
#define QAOA_FLAG_GRADIENT_INPLACE 0x40u
#define QAOA_FLAG_GRADIENT_CHECKPOINTS 0x80u
/* Run the qubit-group classes of a ragged batch concurrently (Sec. 3.3: the
 * subgraph solvers are independent). The tiles of all subgraphs with the same
 * qubit-group layout form a class, and each class runs its own sequence of
 * HBM passes; by default the classes run one after another on the caller's
 * stream. With this flag, qaoa_apply_layers, qaoa_expectation_grad and
 * qaoa_optimize keep the class of the largest subgraphs on the caller's
 * stream and give the other classes and the small-subgraph kernel to three
 * side streams of the library, forked from and joined back to the caller's
 * stream with events within each call (each Adam step of qaoa_optimize), so
 * that the smaller classes fill the device while the largest one runs.
 * Results are bit-identical to the default. The side streams and events are
 * created once per device (default priority) by the first qaoa_batch_create
 * with this flag, with that device current, and are kept until the process
 * ends; batches on one device share them, and their enqueues are serialised
 * by a lock. The calls stay capturable into a HIP graph. */
#define QAOA_FLAG_CONCURRENT_CLASSES 0x100u

/* Workspace size for a batch (paper Sec. 3.3: the subgraphs {G[V_i]} that
 * Alg. 1 produces, each solved by its own QAOA instance).
 *   B              number of subgraphs (>= 1)
 *   num_qubits     host [B], each in 1..30
 *   edge_offsets   host [B+1], subgraph b owns edges [off[b], off[b+1])
 *   edge_w         host [off[B]] edge weights (>= 0), or NULL for unit weights
 *   max_p          largest depth that will be applied (1..32)
 *   max_k          largest k that qaoa_topk will be asked for (1..64)
 *   flags          QAOA_FLAG_*
 *   out_bytes      receives the byte count (the workspace must be 256-byte aligned) */
qaoa_status_t qaoa_workspace_bytes(int32_t B, const int32_t* num_qubits, const int64_t* edge_offsets,
                                   const int32_t* edge_w, int32_t max_p, int32_t max_k, uint32_t flags,
                                   size_t* out_bytes);

/* Build a batch: validates the subgraphs, lays out states, cut tables, phase
 * tables and partial sums in the caller's workspace, copies the edge lists to
 * the device and builds every subgraph's integer cut table C(z) (1 byte per
 * entry when the subgraph's weight sum is at most 255, else 2).
 *   edge_u, edge_v host [off[B]] local vertex ids in [0, n_b), u != v
 *   edge_w         host weights >= 0 or NULL (unit); per-subgraph sum <= 2047
 *   d_workspace    device buffer of at least qaoa_workspace_bytes bytes,
 *                  256-byte aligned; it must outlive the handle
 *   stream         the upload of the metadata and the table build are
 *                  enqueued on it (after its earlier work); the host arrays
 *                  are copied to pinned staging memory before the call
 *                  returns, so they may be reused at once
 *   out            receives the handle (free it with qaoa_batch_destroy) */
qaoa_status_t qaoa_batch_create(int32_t B, const int32_t* num_qubits, const int64_t* edge_offsets,
                                const int32_t* edge_u, const int32_t* edge_v, const int32_t* edge_w,
                                int32_t max_p, int32_t max_k, uint32_t flags, void* d_workspace,
                                size_t workspace_bytes, qaoa_stream_t stream, qaoa_batch_t* out);

/* Free the host metadata of a handle. NULL is accepted. Caller memory is
 * untouched; work already enqueued for the handle keeps running (it reads
 * only the workspace), so a new batch may be created on the same workspace
 * and stream right away. */
qaoa_status_t qaoa_batch_destroy(qaoa_batch_t h);

/* The QAOA ansatz (Sec. 2.2): reset every subgraph's state to |+>^n and apply
 * p layers U_M(beta_l) U_C(gamma_l), l = 1..p.
 *   p          1..max_p
 *   d_gamma    device double [B*p], row-major (subgraph b, layer l)
 *   d_beta     device double [B*p], same layout
 * Also leaves the per-tile partial sums of <C> for qaoa_expectation. */
qaoa_status_t qaoa_apply_layers(qaoa_batch_t h, int32_t p, const double* d_gamma, const double* d_beta,
                                qaoa_stream_t stream);

/* The QAOA objective <psi|H_C|psi> = sum_z |psi(z)|^2 C(z) (Sec. 2.2) of the
 * state left by the last qaoa_apply_layers (or qaoa_expectation_grad).
 *   d_out      device double [B]
 * QAOA_ERR_STATE if neither has run since creation. */
qaoa_status_t qaoa_expectation(qaoa_batch_t h, double* d_out, qaoa_stream_t stream);

/* Selective Distribution Exploration (Sec. 3.3.2): for every subgraph the k
 * bitstrings with the largest probability pi(z) = |psi(z)|^2 of the state
 * left by the last qaoa_apply_layers, ordered by pi descending, ties by z
 * ascending. Default mode considers only z with bit 0 clear (pi(z) =
 * pi(~z) exactly, so this keeps one member of each complement pair and the
 * merge adds the complements); QAOA_FLAG_TOPK_RAW considers all z.
 *   k          1..max_k
 *   d_idx      device uint32 [B*k]; rows with fewer candidates than k are
 *              padded with 0xFFFFFFFF
 *   d_prob     device float [B*k]; padding rows hold -1
 * QAOA_ERR_STATE unless qaoa_apply_layers ran after the last
 * qaoa_expectation_grad (which consumes the state). */
qaoa_status_t qaoa_topk(qaoa_batch_t h, int32_t k, uint32_t* d_idx, float* d_prob, qaoa_stream_t stream);

/* Exact gradient of every subgraph's <C> with respect to its angles, by the
 * adjoint sweep (derivative of e^{-i theta H} is -i H e^{-i theta H}), for the
 * angle optimisation that Sec. 2.2 describes. Needs QAOA_FLAG_GRADIENT.
 *   d_gamma, d_beta   device double [B*p] (as in qaoa_apply_layers)
 *   d_E               device double [B]   receives <C>
 *   d_dgamma, d_dbeta device double [B*p] receive dE/dgamma, dE/dbeta
 * The state is consumed (call qaoa_apply_layers before qaoa_topk). */
qaoa_status_t qaoa_expectation_grad(qaoa_batch_t h, int32_t p, const double* d_gamma, const double* d_beta,
                                    double* d_E, double* d_dgamma, double* d_dbeta, qaoa_stream_t stream);

/* One Adam step (Kingma and Ba 2015) in FP64 on a flat parameter vector,
 * used for the angle optimisation of Sec. 2.2 (maximise = 1) and for the
 * angle-predictor's training (maximise = 0).
 *   count      number of parameters (>= 1)
 *   d_theta    device double [count], updated in place
 *   d_grad     device double [count]
 *   d_m, d_v   device double [count], moment estimates (start at zero)
 *   d_step     device int32 [1], steps taken so far; incremented by the call
 *   lr, beta1, beta2, eps  the usual Adam constants */
qaoa_status_t qaoa_adam_step(int32_t count, double* d_theta, const double* d_grad, double* d_m, double* d_v,
                             int32_t* d_step, double lr, double beta1, double beta2, double eps,
                             int32_t maximise, qaoa_stream_t stream);

/* `iters` steps of the angle optimisation of Sec. 2.2, all on the device:
 * each step evaluates every subgraph's <C> and its exact gradient at theta
 * (as qaoa_expectation_grad) and takes one FP64 Adam ascent step on the
 * angles (as qaoa_adam_step with count = 2*B*p, maximise = 1). Per step, the
 * gradient's reduction, the Adam update and the preparation of the next
 * step's rotation and phase tables run as one kernel; the results are
 * bit-identical to the two separate calls per step. Needs QAOA_FLAG_GRADIENT.
 *   p          1..max_p
 *   iters      >= 0 (0: nothing is enqueued)
 *   d_theta    device double [2*B*p], [gamma (row b = subgraph b, B*p) |
 *              beta (B*p)], updated in place
 *   d_m, d_v   device double [2*B*p], Adam moments (start at zero)
 *   d_step     device int32 [1], Adam steps taken so far; +iters on completion
 *   lr, beta1, beta2, eps  the Adam constants (as qaoa_adam_step)
 *   d_E        device double [B] receiving <C> at the angles each step
 *              starts from (the last step's remains), or NULL
 * The state is consumed (call qaoa_apply_layers before qaoa_topk). Calls on
 * one batch must not overlap (they share the batch's states and partial
 * sums). d_step is read by every step of the call and advanced once, after
 * its last step. */
qaoa_status_t qaoa_optimize(qaoa_batch_t h, int32_t p, int32_t iters, double* d_theta, double* d_m, double* d_v,
                            int32_t* d_step, double lr, double beta1, double beta2, double eps, double* d_E,
                            qaoa_stream_t stream);

/* CutVal (Sec. 2.1) of num_assign full-graph assignments, as the merge of
 * Alg. 2 evaluates each concatenated bitstring over all edges of G.
 *   d_u, d_v   device int32 [num_edges] vertex ids
 *   d_w        device int32 [num_edges] weights, or NULL for unit weights
 *   d_assign   device uint32 [num_assign][ceil(num_vertices/32)], vertex t is
 *              word t/32, bit t%32
 *   d_cut      device int64 [num_assign]; -1 if any edge id lies outside
 *              [0, num_vertices) */
qaoa_status_t maxcut_eval(int32_t num_vertices, int64_t num_edges, const int32_t* d_u, const int32_t* d_v,
                          const int32_t* d_w, int64_t num_assign, const uint32_t* d_assign, int64_t* d_cut,
                          qaoa_stream_t stream);

/* Workspace size for qaoa_merge_beam (device bytes, 256-byte aligned). */
qaoa_status_t qaoa_merge_workspace_bytes(int32_t num_vertices, int32_t M, int64_t num_edges, int32_t K,
                                         int32_t W, size_t* out_bytes);

/* Level-Aware Merge (Sec. 3.4, Alg. 2) of the per-subgraph candidates into a
 * full-graph assignment, as a level-wise beam of width W.
 * Candidate set of subgraph i is B_i = {b_j, ~b_j} over the top-k bitstrings
 * b_j; a path picks a member of B_1 and then, at each later level, the member
 * of each pair whose bit for the vertex shared with the previous subgraph
 * agrees with the path (2 K^M full paths). Paths are ordered as the
 * depth-first traversal of Alg. 2 visits them (level 1 lists b_1, ~b_1, b_2,
 * ~b_2, ...; later levels list by j). After each level the W paths with the
 * largest cut over the edges whose endpoints are both assigned survive, ties
 * broken by path order; the result is the best full path by (cut, path
 * order). With W >= 2 K^(M-1) nothing is pruned and the result equals the
 * exhaustive traversal of Alg. 2 (strict '>' keeps the first maximum).
 *   num_vertices     |V|
 *   M, h_start, h_size  host [M]: the chain partition; range i is
 *                    [h_start[i], h_start[i] + h_size[i]), h_start[0] = 0,
 *                    h_start[i] = h_start[i-1] + h_size[i-1] - 1, the last
 *                    range ends at |V|; sizes 2..32 (1 allowed when M = 1)
 *   num_edges, h_u, h_v, h_w  host full-graph edge list (ids in [0, |V|),
 *                    u != v), weights >= 0 or NULL for unit weights
 *   K, d_cand        device uint32 [M*K]: row i holds b_j of subgraph i in
 *                    local bit order (bit t = vertex h_start[i] + t); the
 *                    entries after the first 0xFFFFFFFF of a row are ignored
 *   W                beam width, 1..8192
 *   d_workspace      device, >= qaoa_merge_workspace_bytes, 256-byte aligned
 *   d_best_assign    device uint32 [ceil(|V|/32)], the winning assignment
 *                    (vertex t = word t/32, bit t%32; bit 1 = side S)
 *   d_best_cut       device int64 [1], its cut value; -1 (and a zero
 *                    assignment) if some row has no candidate
 * The host arrays are copied to pinned staging memory before the call
 * returns; the upload and the merge kernels are enqueued on `stream`. */
qaoa_status_t qaoa_merge_beam(int32_t num_vertices, int32_t M, const int32_t* h_start, const int32_t* h_size,
                              int64_t num_edges, const int32_t* h_u, const int32_t* h_v, const int32_t* h_w,
                              int32_t K, const uint32_t* d_cand, int32_t W, void* d_workspace,
                              size_t workspace_bytes, uint32_t* d_best_assign, int64_t* d_best_cut,
                              qaoa_stream_t stream);

/* Angle predictor for a learned warm start of the angle optimisation (not a
 * step of the paper; Sec. 2.2 notes that initialisation affects solution
 * quality and iteration count). A multilayer perceptron in -> hidden ->
 * hidden -> out, ReLU hidden layers, linear output. Parameters are one flat
 * FP64 array, row-major: W1[hidden][in], b1[hidden], W2[hidden][hidden],
 * b2[hidden], W3[out][hidden], b3[out] (qaoa_mlp_num_params gives its
 * length). Arithmetic is FP32 with FP64 gradient sums; limits in <= 64,
 * hidden <= 256, out <= 64.
 *   qaoa_mlp_forward:  d_x float [batch][in] -> d_y float [batch][out];
 *                      d_act float [batch][2*hidden] keeps both hidden
 *                      activations for the backward pass
 *   qaoa_mlp_backward: loss = mean over batch and outputs of (y - t)^2 into
 *                      d_loss double [1], its gradient into d_grad double
 *                      [num_params]; d_y/d_act from the forward call on the
 *                      same parameters and inputs; d_scratch device bytes of
 *                      at least qaoa_mlp_scratch_bytes */
qaoa_status_t qaoa_mlp_num_params(int32_t in_dim, int32_t hidden, int32_t out_dim, int64_t* out);
qaoa_status_t qaoa_mlp_scratch_bytes(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim, size_t* out);
qaoa_status_t qaoa_mlp_forward(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim, const double* d_params,
                               const float* d_x, float* d_y, float* d_act, qaoa_stream_t stream);
qaoa_status_t qaoa_mlp_backward(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                const double* d_params, const float* d_x, const float* d_y, const float* d_act,
                                const float* d_target, void* d_scratch, size_t scratch_bytes, double* d_grad,
                                double* d_loss, qaoa_stream_t stream);

/* Learned warm start, step 1: the predictor's outputs as starting angles.
 * y[b][o] holds the standardised output o of subgraph b (o < p: gamma_{o+1},
 * o >= p: beta_{o-p+1}); the angle is y * sd[o] + mu[o], computed in FP32
 * (product, then sum, each rounded) and widened to FP64.
 *   d_y        device float [B][2p] (qaoa_mlp_forward's output, out = 2p)
 *   d_mu, d_sd device float [2p], the target standardisation of training
 *   d_theta    device double [2*B*p] receiving [gamma (B*p) | beta (B*p)] in
 *              the layout of qaoa_optimize
 * QAOA_ERR_OUT_OF_RANGE for p outside 1..32. */
qaoa_status_t qaoa_warm_angles(int32_t B, int32_t p, const float* d_y, const float* d_mu, const float* d_sd,
                               double* d_theta, qaoa_stream_t stream);

/* Learned warm start, step 2: the plain method's start stays the fallback.
 * For every subgraph b, if d_E_alt[b] > d_E[b] (the alternative start has the
 * larger <C>, Sec. 2.2's objective), its angles replace row b of d_theta
 * (gamma and beta) and d_E[b] becomes d_E_alt[b]; otherwise row b is kept.
 *   d_E_alt, d_E           device double [B]
 *   d_theta_alt, d_theta   device double [2*B*p], layout of qaoa_optimize */
qaoa_status_t qaoa_keep_better(int32_t B, int32_t p, const double* d_E_alt, const double* d_theta_alt, double* d_E,
                               double* d_theta, qaoa_stream_t stream);

/* qaoa_mlp_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * allocation): the same kernels and results, with the scratch taken from a
 * buffer the library holds in device memory (8 MiB per device, kept until
 * the process ends) instead of a caller's d_scratch. The call allocates
 * nothing: no device, host or pinned memory and no events.
 *   Arguments as qaoa_mlp_backward, without d_scratch / scratch_bytes.
 *   QAOA_ERR_OUT_OF_RANGE if qaoa_mlp_scratch_bytes(batch, in_dim, hidden,
 *   out_dim) exceeds 8 MiB (e.g. batch > 8000 at in 18, hidden 128, out 6).
 * Every call on a device shares that device's buffer (each call overwrites
 * the part it uses before reading it; nothing needs to start at zero), so
 * calls that overlap on one device race: issue them on one stream, or order
 * them. The first call on a device looks up the buffer's address there. */
qaoa_status_t qaoa_mlp_backward_noalloc(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                        const double* d_params, const float* d_x, const float* d_y,
                                        const float* d_act, const float* d_target, double* d_grad, double* d_loss,
                                        qaoa_stream_t stream);

/* *out = 1 if the batch keeps forward checkpoints for its gradient (see
 * QAOA_FLAG_GRADIENT_CHECKPOINTS), else 0. */
qaoa_status_t qaoa_gradient_checkpoints(qaoa_batch_t h, int32_t* out);

/* Where subgraph b's state lives: the byte offset, inside the workspace, of
 * its stored amplitudes. The ansatz state is invariant under flipping every
 * bit (H_C, H_M and |+>^n all commute with X on every qubit, Sec. 2.2), so
 * only the 2^(n-1) amplitudes phi(z) = sqrt(2) psi(z), z < 2^(n-1), are stored
 * (complex64, interleaved real, imaginary); psi(z) = phi(z) / sqrt(2) and
 * psi(z) = psi(z XOR (2^n - 1)) for the upper half. After qaoa_apply_layers
 * they hold |psi>; after qaoa_expectation_grad an intermediate of the adjoint
 * sweep. For inspection and tests. */
qaoa_status_t qaoa_state_offset(qaoa_batch_t h, int32_t b, size_t* out_offset);

/* Tuning of the strided qubit groups (process-wide, read when a batch is
 * created). Subgraphs with n > 13 qubits are simulated in group 0 (qubits
 * 0..10 and the top qubit, 4096-amplitude tiles) and strided groups of at most
 * 8 of the qubits 11..n-2, one HBM pass per group and layer (Sec. 2.2's mixer
 * is a product over qubits, so any grouping gives the same state).
 * sizes[0..count) are the strided group sizes in qubit order for subgraphs
 * with n qubits (each 1..8, at most 3 groups, adding up to n - 12); count = 0
 * restores the default (fewest groups, sizes as even as possible). Batches
 * created earlier keep their layout. QAOA_ERR_OUT_OF_RANGE for n outside
 * 14..30, count > 3 or a size outside 1..8; QAOA_ERR_INVALID_ARG if the sizes
 * do not add up to n - 12. */
qaoa_status_t qaoa_tune_group_split(int32_t n, int32_t count, const int32_t* sizes);

/* Text of a status code (static storage). */
const char* qaoa_status_string(qaoa_status_t s);

/* Detail of the last error on this thread ("" if none). */
const char* qaoa_last_error(void);

/* Kernel timing for measurement: while enabled, the library brackets every
 * launch of its kernels with HIP events on the launch stream and adds up the
 * launch's algorithmic HBM bytes (each state read and written once per pass
 * where the pass needs it, plus the 1- or 2-byte cut table where the pass needs
 * C(z)). qaoa_profile_read
 * waits for those events and returns, for the named kernel, the number of
 * launches, their summed duration in milliseconds and their summed
 * algorithmic bytes since the last qaoa_profile_enable(1). Names: the tile
 * passes by direction, kind and qubit group, "fwd_{first,single,mid,last}_gG"
 * and "bwd_{fused,single,mid,last,single_nopsi,mid_nopsi}_gG" (G = 0..3), and
 * "small", "cut_tables", "angle_prep", "reduce", "topk", "maxcut", "adam",
 * "merge", "mlp_forward", "mlp_backward", "warm_angles", "keep_better". Not for use while another thread
 * launches. */
qaoa_status_t qaoa_profile_enable(int32_t on);
/* Restrict the timing to one kernel name (NULL or "" = all). Each timed launch
 * adds two event records to its stream; timing only the kernel of interest
 * keeps that cost off the others. */
qaoa_status_t qaoa_profile_select(const char* kernel);
qaoa_status_t qaoa_profile_read(const char* kernel, int64_t* launches, double* total_ms, double* algo_bytes);

#ifdef __cplusplus
}
#endif

#endif /* PARAQAOA_H */
