/*
 * dvq.h -- D-VQLS hot path on AMD Instinct MI355X (gfx950): C ABI.
 *
 * The library computes, for the Variational Quantum Linear Solver with a
 * Pauli (linear-combination-of-unitaries) encoding of the matrix
 * (arXiv 2604.14435):
 *   - the FWHT-based Pauli decomposition of a real matrix A with magnitude
 *     pruning (Section II-B, Eq. (5); Algorithm 1 Steps 1-2);
 *   - every Hadamard-test circuit of one cost evaluation, simulated as an
 *     ideal (n+1)-qubit state vector, for a batch of parameter vectors
 *     (Section II-A, Section II-C, Eq. (4));
 *   - the cost from those terms (Eq. (1) global; Section II-C stage iii
 *     local), its gradient by the parameter-shift rule or by an adjoint sweep
 *     over the ansatz, a gradient-descent step and the solution fidelity
 *     (Section III-A);
 *   - a small bfloat16 MLP (forward, backward, AdamW) that predicts initial
 *     angles from a system descriptor.
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless the name ends in _host.  The caller
 *     owns every buffer; the library never allocates memory for the caller
 *     and frees nothing.  Calls that need scratch memory take an explicit
 *     workspace pointer and size, with a *_workspace_bytes query.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call enqueues its work on `stream` and returns without waiting, except
 *     calls with *_host outputs, which synchronise `stream` before returning.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and return DVQ_EINVAL / DVQ_EUNSUPPORTED / DVQ_ECAPACITY; nothing is
 *     written to device memory in that case.  A failing HIP call returns
 *     DVQ_EDEVICE.  dvq_last_error() gives a one-line description of the
 *     last failure on the calling thread.
 *   - Qubit q is bit q of a basis index.  In the (n+1)-qubit circuits the
 *     ancilla is bit n.
 *   - A Pauli string is a pair of n-bit masks (x, z) and denotes
 *     P = i^{popcount(x & z)} X^x Z^z, i.e. the tensor product of I, X, Z, Y
 *     for the bit pairs (0,0), (1,0), (0,1), (1,1).  Its flat index is
 *     x * 2^n + z.
 *   - Complex numbers are {double re, im} pairs (dvq_c128).
 *   - Ansatz V(theta) (Section II-C; Section III-A): `layers` layers; layer l
 *     applies RY(theta[l*n + q]) on every qubit q, then an entangling ladder
 *     on (q, q+1), q = 0..n-2, of CZ gates or of CNOTs (control q, target
 *     q+1).  RY(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]].  theta is
 *     always float64, P = n * layers values per row.
 *   - State preparation U_b, U_b|0> = |b>: DVQ_B_PLUS means b = |+>^n and
 *     U_b = H^n; DVQ_B_VECTOR means a real unit vector b (float64, length
 *     2^n) and U_b = s (I - 2 w w^T / w^T w), w = e_0 - s b,
 *     s = -1 if b_0 > 0 else +1.
 *
 * Thread safety: every call is re-entrant; calls on different streams may
 * run concurrently.
 */
#ifndef DVQ_H
#define DVQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* dvq_stream; /* hipStream_t */

typedef int32_t dvq_status;
enum {
    DVQ_OK = 0,
    DVQ_EINVAL = -1,       /* bad argument (null pointer, size out of range, ...) */
    DVQ_ECAPACITY = -2,    /* output capacity or workspace too small            */
    DVQ_ENOMEM = -3,       /* reserved                                           */
    DVQ_EDEVICE = -4,      /* a HIP runtime call failed                          */
    DVQ_EUNSUPPORTED = -5, /* valid request this build does not implement        */
    DVQ_ENONFINITE = -6    /* a host-visible result is NaN or infinite           */
};

typedef struct { uint32_t x, z; } dvq_pauli;
typedef struct { double re, im; } dvq_c128;

enum { DVQ_COST_GLOBAL = 0, DVQ_COST_LOCAL = 1 };
enum { DVQ_ENT_CZ_LADDER = 0, DVQ_ENT_CNOT_LADDER = 1 };
enum { DVQ_F64 = 0, DVQ_F32 = 1 };
enum { DVQ_B_PLUS = 0, DVQ_B_VECTOR = 1 };
enum { DVQ_EXEC_LITERAL = 0, DVQ_EXEC_GENERIC = 1, DVQ_EXEC_SHARED = 2 };

typedef struct {
    int32_t n;         /* system qubits, 1..12 (circuits use n + 1 qubits)  */
    int32_t layers;    /* ansatz depth d >= 1                                */
    int32_t entangler; /* DVQ_ENT_CZ_LADDER or DVQ_ENT_CNOT_LADDER          */
} dvq_ansatz;

/* ------------------------------------------------------------------ misc */

const char* dvq_status_string(dvq_status s);
/* Description of the last non-OK status returned on this thread. */
const char* dvq_last_error(void);
const char* dvq_version(void);

/* --------------------------------------------------- Pauli decomposition */

/* Scratch bytes needed by dvq_pauli_decompose / _dense for n qubits. */
size_t dvq_decompose_workspace_bytes(int32_t n);

/*
 * All 4^n Pauli coefficients of a real N x N matrix, N = 2^n
 * (Section II-B, Eq. (5): c = Tr(P^dagger A) / N), by one Walsh-Hadamard
 * transform per x-mask.
 *   A          [N*N] float64, row-major, read only.
 *   n          1..12.
 *   coeffs_all [N*N] output, coefficient of string (x, z) at x*N + z.
 * Returns DVQ_EINVAL for bad n / null pointers, DVQ_ECAPACITY when
 * workspace_bytes < dvq_decompose_workspace_bytes(n).
 */
dvq_status dvq_pauli_decompose_dense(const double* A, int32_t n, dvq_c128* coeffs_all,
                                     void* workspace, size_t workspace_bytes, dvq_stream stream);

/*
 * Decompose A and keep the pruned term list (Algorithm 1 Steps 1-2).
 *   top_L <= 0: threshold mode, keep every string with |c| > tau (strict,
 *               |c| = hypot(re, im) in float64; tau >= 0, finite).
 *   top_L  > 0: keep the top_L strings by the ranking key (ties included in
 *               the key, so the set is unique).
 * Kept terms are written ordered by the ranking key: |c| descending, then
 * flat index ascending.
 *   coeffs   [capacity] output coefficients.
 *   strings  [capacity] output masks.
 *   capacity >= the number of kept terms, else DVQ_ECAPACITY (L_out_host is
 *            still written; at most the first `capacity` entries of
 *            coeffs/strings are written, their content is then
 *            unspecified).  At most 65536 kept terms are sorted
 *            (DVQ_ECAPACITY beyond).
 *   L_out_host     number of kept terms.
 *   frob_err_host  relative Frobenius error of the pruned sum,
 *                  sqrt(N * sum over dropped |c|^2) / ||A||_F (may be NULL).
 * The selection runs on the device without host round trips; the call
 * synchronises `stream` once at the end (host outputs).
 */
dvq_status dvq_pauli_decompose(const double* A, int32_t n, double tau, int64_t top_L,
                               dvq_c128* coeffs, dvq_pauli* strings, int64_t capacity,
                               int64_t* L_out_host, double* frob_err_host,
                               void* workspace, size_t workspace_bytes, dvq_stream stream);

/* Scratch bytes needed by dvq_pauli_decompose_batch for B matrices. */
size_t dvq_decompose_batch_workspace_bytes(int32_t n, int32_t B);

/*
 * dvq_pauli_decompose in top-L mode for B matrices of one size (a family of
 * systems, e.g. the training set of the warm start): Algorithm 1 Steps 1-2
 * for each.  The matrices are processed one after another on `stream`, all
 * enqueued before a single synchronisation.
 *   A        [B][N][N] float64, row-major, device.
 *   top_L    terms kept per matrix, 1 <= top_L <= min(4^n, 65536).
 *   coeffs   [B][top_L], strings [B][top_L] (device): matrix b's terms,
 *            ordered by the ranking key as in dvq_pauli_decompose.
 *   frob_err_host [B] relative Frobenius error per matrix (host).
 *   workspace >= dvq_decompose_batch_workspace_bytes(n, B) bytes, device.
 * Errors: DVQ_EINVAL for bad arguments, DVQ_ECAPACITY for a short
 * workspace, DVQ_EDEVICE if a device-side check fails (the message names
 * the matrix).
 */
dvq_status dvq_pauli_decompose_batch(const double* A, int32_t n, int32_t B, int64_t top_L,
                                     dvq_c128* coeffs, dvq_pauli* strings, double* frob_err_host,
                                     void* workspace, size_t workspace_bytes, dvq_stream stream);

/*
 * Dense operator of a term list: out[r][c] = sum_l c_l P_l[r][c] (Eq. (3)),
 * complex128 [2^n][2^n] row-major (e.g. the pruned matrix A_tilde).
 *   coeffs [L], strings [L] as written by dvq_pauli_decompose; n 1..14.
 */
dvq_status dvq_pauli_sum_dense(const dvq_c128* coeffs, const dvq_pauli* strings, int32_t L,
                               int32_t n, dvq_c128* out, dvq_stream stream);

/* ----------------------------------------------- Hadamard-test circuits */

/* Number of circuits one cost evaluation simulates for one theta row:
 * local 2(n+1)L^2, global 2(L^2 + L) (Section II-B after Eq. (4)). */
int64_t dvq_circuit_count(int32_t n, int32_t L, int32_t cost_kind);

/*
 * Simulate every Hadamard-test circuit of one cost evaluation for each of B
 * parameter rows and write the measured terms (Section II-A, II-C, Eq. (4)):
 *   beta_lm    = <x|A_l^dagger A_m|x>                       [B][L][L]
 *   local:  delta^j_lm = <x|A_l^dagger U_b Z_j U_b^dagger A_m|x>, other = [B][n][L][L]
 *   global: gamma_l    = <b|A_l|x>,                               other = [B][L]
 * with |x> = V(theta_row)|0>.  Each complex term takes two circuits: the
 * real part is <Z_ancilla> of H, controlled-U, H; the imaginary part adds
 * S^dagger on the ancilla before the final H.  One circuit = one (n+1)-qubit
 * state vector evolved gate by gate.
 *   theta     [B][P] float64, P = n * layers.
 *   precision DVQ_F64 (complex128 state) or DVQ_F32 (complex64 state;
 *             angles, terms and all outputs stay float64).
 *   strings   [L] masks, each mask < 2^n.  L >= 1.
 *   b         [2^n] float64 unit vector for DVQ_B_VECTOR, ignored for PLUS.
 *   exec      DVQ_EXEC_LITERAL: the production kernels (one wavefront per
 *             circuit, amplitudes in registers) where available, else the
 *             generic kernel; DVQ_EXEC_GENERIC: always the generic kernel
 *             (one workgroup per circuit, amplitudes in LDS, one pass per
 *             gate); DVQ_EXEC_SHARED: the prefix common to every circuit
 *             of a row (ancilla H and V(theta)) is simulated once per
 *             wavefront and each circuit's own gates (controlled strings,
 *             X_j, S^dagger, H, measurement) are applied to a copy of that
 *             state -- the same results; shapes without a shared kernel fall
 *             back to the generic kernel.
 *             The register-resident (literal and shared) kernels exist for
 *             the local cost at n = 10, 11 (F32) and n = 10 (F64), with
 *             either ladder and either b kind (a general b applies
 *             U_b Z_j U_b^dagger through its Householder form), and run
 *             the beta circuits of the global cost at the same shapes (its
 *             gamma circuits, with a controlled V(theta), run on the
 *             generic kernel); every other shape runs the generic kernel.
 * Limits: n <= 12 (F64) / 13 (F32); B * circuits < 2^31.
 */
dvq_status dvq_vqls_terms(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                          int32_t precision, const dvq_pauli* strings, int32_t L,
                          int32_t b_kind, const double* b, int32_t cost_kind, int32_t exec,
                          dvq_c128* beta, dvq_c128* other, dvq_stream stream);

/*
 * Several right-hand sides with the same A and angles: beta_lm involves
 * neither b nor U_b (Section II-C), so its 2 L^2 circuits per row run once,
 * and only the b-dependent circuits (delta for the local cost, gamma for the
 * global cost) run once per right-hand side -- the amortisation over
 * right-hand sides sharing A that the paper's conclusion points to, carried
 * from the decomposition to the circuits.
 *   b      [R][2^n] float64 unit vectors (device), one per right-hand side
 *          (as DVQ_B_VECTOR in dvq_vqls_terms).  1 <= R <= 65536.
 *   beta   [B][L][L] output, written once.
 *   other  [R][B][n][L][L] (local) or [R][B][L] (global) output: block r
 *          holds what dvq_vqls_terms writes for b_r.
 * Every other argument as in dvq_vqls_terms; the values equal those of R
 * separate dvq_vqls_terms calls with b_kind = DVQ_B_VECTOR (the same kernels
 * compute every circuit).  Errors: DVQ_EINVAL for R outside 1..65536, a NULL
 * b, or any argument dvq_vqls_terms rejects; nothing is launched then.
 */
dvq_status dvq_vqls_terms_rhs(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                              int32_t precision, const dvq_pauli* strings, int32_t L, int32_t R,
                              const double* b, int32_t cost_kind, int32_t exec, dvq_c128* beta,
                              dvq_c128* other, dvq_stream stream);

/*
 * Cost from the terms (float64): Psi = sum_lm conj(c_l) c_m beta_lm;
 *   local:  E = sum_j sum_lm conj(c_l) c_m delta^j_lm,
 *           C = 1/2 - 1/2 Re[E / (n Psi)]  (Section II-C stage iii);
 *   global: G = |sum_l c_l gamma_l|^2, C = 1 - G / Psi  (Eq. (1)).
 *   coeffs [L]; beta, other as written by dvq_vqls_terms for B rows.
 *   C      [B] output.
 *   parts  [B][2] output (E or G, Psi) as complex values, may be NULL.
 * Sums run in a fixed order, so results are bit-reproducible.
 */
dvq_status dvq_vqls_cost(const dvq_c128* coeffs, int32_t L, int32_t n, int32_t cost_kind,
                         const dvq_c128* beta, const dvq_c128* other, int32_t B,
                         double* C, dvq_c128* parts, dvq_stream stream);

/* ------------------------------------------------------------- gradients */

/* Scratch bytes for dvq_vqls_grad_shift. */
size_t dvq_grad_shift_workspace_bytes(const dvq_ansatz* ansatz, int32_t L, int32_t cost_kind);

/*
 * Plain path: cost and exact gradient by the parameter-shift rule, the
 * gradient that Algorithm 1 Step 4 hands to the classical optimizer (the
 * paper's L-BFGS-B of Section III; the paper does not name its gradient
 * method, and the shift rule is exact for RY gates).  The 2P + 1 rows
 * theta, theta +/- (pi/2) e_k go through dvq_vqls_terms and the
 * aggregation (Section II-C stages ii-iii); the shift rule is applied to
 * the expectation values Psi and E (or G), then the quotient rule gives
 * dC/dtheta.
 *   theta [P], C [1], grad [P] (float64, device).
 */
dvq_status dvq_vqls_grad_shift(const dvq_ansatz* ansatz, const double* theta, int32_t precision,
                               const dvq_c128* coeffs, const dvq_pauli* strings, int32_t L,
                               int32_t b_kind, const double* b, int32_t cost_kind,
                               double* C, double* grad, void* workspace, size_t workspace_bytes,
                               dvq_stream stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same cost and
 * gradient as dvq_vqls_grad_shift, bit for bit, with no workspace argument.
 * Its scratch is one file-scope device array of
 * dvq_grad_shift_noalloc_max_bytes() bytes (32 MiB) per GPU, held from the
 * library's first use on that GPU until the process ends; the call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * The 2P + 1 shifted rows are evaluated in chunks of as many rows as fit
 * the array.
 *   Arguments as in dvq_vqls_grad_shift, on the device of `stream`.
 * Errors: everything dvq_vqls_grad_shift rejects; DVQ_ECAPACITY when the
 * 2P + 1 angle rows with their parts plus the terms of one row
 * ((L^2 + n L^2) complex128 local, (L^2 + L) global) exceed the array.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (different streams, or host
 * threads) race and must be ordered by the caller.
 */
size_t dvq_grad_shift_noalloc_max_bytes(void);
dvq_status dvq_vqls_grad_shift_noalloc(const dvq_ansatz* ansatz, const double* theta,
                                       int32_t precision, const dvq_c128* coeffs,
                                       const dvq_pauli* strings, int32_t L, int32_t b_kind,
                                       const double* b, int32_t cost_kind, double* C,
                                       double* grad, dvq_stream stream);

/*
 * Fast path: cost and gradient by an adjoint sweep over the ansatz, the
 * same cost (Eq. (1) global, Section II-C stage iii local) and the same
 * gradient as dvq_vqls_grad_shift for the optimizer of Algorithm 1 Step 4,
 * computed on one 2^n state instead of 2P + 1 evaluations.  The
 * state |x> = V(theta)|0> is built gate by gate, lambda = M |x> with
 *   M = dC/dE * A^dagger U_b (sum_j Z_j) U_b^dagger A + dC/dPsi * A^dagger A  (local),
 *   M = dC/dG * A^dagger |b><b| A + dC/dPsi * A^dagger A                     (global),
 * A = sum_l c_l P_l, and the gates are then undone in reverse order on both
 * vectors (no stored intermediate states); each RY contributes
 * dC/dtheta_k = Re <K_q x_k | lambda_k>, K = [[0, -1], [1, 0]].
 *   theta  [B][P].
 *   coeffs [L] and strings [L] shared by all rows (per_row_system = 0), or
 *          [B][L] each (per_row_system = 1: row r uses system r).
 *   C [B], grad [B][P] float64 outputs.
 * One workgroup per row; n <= 12 (F32) / 11 (F64): three LDS-resident
 * vectors of 2^n amplitudes per row must fit the 160 KB of a CU, so F64 at
 * n = 12 returns DVQ_EUNSUPPORTED.  Rows at n = 10, 11 (F32) and n = 10
 * (F64), with either ladder, run as four wavefronts each, every wavefront
 * holding both vectors in registers (the Pauli sums and the gradients split
 * between them); other shapes use the LDS vectors, 512 threads per row.
 */
dvq_status dvq_vqls_grad_adjoint(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                                 int32_t precision, const dvq_c128* coeffs,
                                 const dvq_pauli* strings, int32_t L, int32_t per_row_system,
                                 int32_t b_kind, const double* b, int32_t cost_kind,
                                 double* C, double* grad, dvq_stream stream);

/* theta[i] -= lr * grad[i] for i < count: a gradient-descent update of
 * the angles, the classical update of Algorithm 1 Step 4 (the paper's own
 * optimizer, L-BFGS-B of Section III, runs on the host over the same cost
 * and gradient). */
dvq_status dvq_gd_step(double* theta, const double* grad, int64_t count, double lr,
                       dvq_stream stream);

/* F[r] = |<target|V(theta_r)|0>|^2 in float64 for B rows (Section III-A);
 * target [2^n] is a unit vector. */
dvq_status dvq_fidelity(const dvq_ansatz* ansatz, const double* theta, int32_t B,
                        const dvq_c128* target, double* F, dvq_stream stream);

/* ----------------------------------------------------- warm-start MLP */

typedef struct {
    int32_t d_in;   /* input features, 1..64                     */
    int32_t hidden; /* hidden width, multiple of 32, 32..512      */
    int32_t d_out;  /* outputs (angles), 1..512                   */
} dvq_mlp_shape;

/* Number of float32 parameters, packed W1[h][d_in], b1[h], W2[h][h], b2[h],
 * W3[d_out][h], b3[d_out] (row-major). */
int64_t dvq_mlp_param_count(const dvq_mlp_shape* shape);
size_t dvq_mlp_workspace_bytes(const dvq_mlp_shape* shape, int32_t batch);

/*
 * y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for `batch` rows.  Every GEMM
 * operand is rounded to bfloat16 and accumulated in float32 on the matrix
 * cores.  H1, H2 [batch][hidden] receive the float32 hidden activations
 * (needed by the backward pass), Y [batch][d_out].
 */
dvq_status dvq_mlp_forward(const dvq_mlp_shape* shape, const float* params, const float* X,
                           int32_t batch, float* H1, float* H2, float* Y, dvq_stream stream);

/* Wrap-safe angle loss l = mean(1 - cos(Y - T)) over count values;
 * dY = sin(Y - T) / count; loss [1] float64 (may be NULL). */
dvq_status dvq_mlp_loss_grad(const float* Y, const float* T, int64_t count, float* dY,
                             double* loss, dvq_stream stream);

/* Parameter gradients dparams (same packing as params) of the loss whose
 * output gradient is dY; X, H1, H2 as saved by dvq_mlp_forward. */
dvq_status dvq_mlp_backward(const dvq_mlp_shape* shape, const float* params, const float* X,
                            const float* H1, const float* H2, const float* dY, int32_t batch,
                            float* dparams, void* workspace, size_t workspace_bytes,
                            dvq_stream stream);

/* One AdamW step on float32 master weights (t >= 1 counts steps). */
dvq_status dvq_adamw_step(float* params, const float* grads, float* m, float* v, int64_t count,
                          int32_t t, float lr, float beta1, float beta2, float eps,
                          float weight_decay, dvq_stream stream);

/*
 * Fused forms of the warm-start network (hidden 64, 128 or 256, d_in <= 32,
 * d_out <= 128; DVQ_EUNSUPPORTED otherwise).  The same arithmetic as
 * dvq_mlp_forward / _loss_grad / _backward / dvq_adamw_step (bfloat16 GEMM
 * operands, float32 accumulation, bias gradients on the unrounded float32
 * values), computed per chunk of 32 batch rows with the chunk's
 * activations kept on chip.
 *
 * Input standardisation: with feat_mean and feat_inv_std (both [d_in],
 * device, or both NULL), x is replaced by (x - mean) * inv_std before the
 * first layer.
 */

/* Column mean and 1 / standard deviation (n - 1 denominator, standard
 * deviation at least 1e-12) of X [rows][d] float32; sums in float64. */
dvq_status dvq_feature_stats(const float* X, int32_t rows, int32_t d, float* mean, float* inv_std,
                             dvq_stream stream);

/* Y [batch][d_out] = the network on X [batch][d_in], one launch. */
dvq_status dvq_mlp_predict(const dvq_mlp_shape* shape, const float* params, const float* X, int32_t batch,
                           const float* feat_mean, const float* feat_inv_std, float* Y, dvq_stream stream);

/* Scratch bytes for dvq_mlp_train_step: one partial gradient and one loss
 * sum per chunk of 32 rows, and the bfloat16 copies of the weights. */
size_t dvq_mlp_train_workspace_bytes(const dvq_mlp_shape* shape, int32_t batch);

/*
 * One training step on a minibatch: the rows rows[0..batch-1] of
 * X [x_rows][d_in] and of the target angles T [x_rows][d_out] (rows = NULL:
 * rows 0..batch-1, batch <= x_rows); an index outside 0..x_rows-1
 * contributes no loss and no gradient (the mean still divides by
 * batch * d_out),
 * loss mean(1 - cos(Y - T)), its gradient, and one AdamW step
 * (t >= 1 counts steps) on params, m, v in place.
 *   grads [param_count] receives the gradient (may be NULL).
 *   loss  [1] float64 receives the minibatch loss before the step (may be NULL).
 * Three launches: the weights rounded to bfloat16 into the workspace (in
 * the layouts the products read), the chunks' forward and backward passes,
 * then the chunk-ordered sum of their gradients with the AdamW update.
 */
dvq_status dvq_mlp_train_step(const dvq_mlp_shape* shape, float* params, float* m, float* v, int32_t t,
                              float lr, float beta1, float beta2, float eps, float weight_decay,
                              const float* X, const float* T, int32_t x_rows, const int32_t* rows,
                              int32_t batch, const float* feat_mean, const float* feat_inv_std, float* grads,
                              double* loss, void* workspace, size_t workspace_bytes, dvq_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* DVQ_H */
