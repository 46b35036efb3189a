/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector library libsv.so.
 *
 * The library applies quantum gates to dense complex64 state vectors held in
 * GPU memory, reduces them to Pauli expectation values in FP64, computes
 * adjoint gradients by un-applying gates, and runs batches of uneven-size
 * circuits in one launch. Everything runs in hand-written HIP kernels.
 *
 * Conventions (all entry points):
 *   - Qubit q is bit q of the amplitude index (qubit 0 = least significant).
 *     The paper's tensor view (Sec. 4.1.1) holds one tensor dimension per
 *     qubit; in a flat row-major vector that dimension is one index bit.
 *   - A state row is 2^n complex64 amplitudes, (re, im) interleaved as two
 *     floats: the paper's layout with real/imaginary parts as the last tensor
 *     dimension (Sec. 4.2, Fig. 1). A state holds `batch` rows back to back
 *     (the batch dimension of Sec. 4.2).
 *   - A gate is (M, Q) (Sec. 4.1.1): a 2^k x 2^k matrix M and an ordered
 *     target list Q. Q[0] is the most significant bit of M's row/column index
 *     (MoveDim moves Q to the front in order; Alg. 1). Matrices are passed
 *     from the host as complex128, row-major, (re, im) interleaved doubles.
 *     Controls: the gate acts only on amplitudes whose control bits are all 1.
 *   - Pauli strings use masks: bit q of x_mask is set for X or Y on qubit q,
 *     bit q of z_mask for Z or Y (Y = iXZ).
 *   - Every entry point returns sv_status and never throws or aborts across
 *     the ABI. Arguments are validated before any GPU work is queued, so a
 *     validation error leaves the state unchanged. sv_last_error() gives a
 *     readable detail of the last failure on the calling thread.
 *   - Host arrays passed in are read (and, where needed, copied) before the
 *     call returns; the caller may free them at once. Gate calls are
 *     asynchronous on the state's stream; calls that return host results
 *     synchronise that stream.
 *   - A state is not thread-safe: calls on one state must not overlap.
 *   - SV_ERR_HIP is sticky: once a HIP runtime call fails during a call on
 *     a state, the state's contents are undefined and every later call on
 *     it returns SV_ERR_HIP (with the first failure's detail) until sv_free,
 *     which still releases it. sv_state_failed reports the flag.
 *   - Calls that synchronise the stream (host results, copies) return
 *     SV_ERR_CAPTURE without queueing anything while the state's stream is
 *     capturing a graph.
 */
#ifndef LIBSV_SV_H_
#define LIBSV_SV_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sv_status {
    SV_OK = 0,
    SV_ERR_INVALID_ARGUMENT = 1,   /* null pointer, bad size or mode */
    SV_ERR_QUBIT_OUT_OF_RANGE = 2, /* a target/control is < 0 or >= n */
    SV_ERR_QUBIT_OVERLAP = 3,      /* a qubit is named twice among targets/controls */
    SV_ERR_UNSUPPORTED = 4,        /* k or control count beyond what the kernels take */
    SV_ERR_OUT_OF_MEMORY = 5,      /* a device allocation failed */
    SV_ERR_HIP = 6,                /* a HIP runtime call failed; state contents undefined */
    SV_ERR_CAPTURE = 7,            /* a synchronising call while the stream is capturing */
    SV_ERR_NOT_UNITARY = 8         /* SV_FLAG_CHECK_UNITARY and ||M M^* - I||_max > 1e-6 */
} sv_status;

/* Flags for sv_apply_gate. */
#define SV_FLAG_ADJOINT 1u        /* apply M^* instead of M (un-apply, Sec. 4.4) */
#define SV_FLAG_CHECK_UNITARY 2u  /* reject non-unitary M (unitarity is otherwise the caller's duty, Sec. 3) */

/* Limits of the kernels. */
#define SV_MAX_QUBITS 34          /* 2^34 complex64 = 128 GiB per row */
#define SV_MAX_GATE_TARGETS 2     /* sv_apply_gate / sv_run: k <= 2 */
#define SV_MAX_FUSED_TARGETS 6    /* sv_apply_fused: k <= 6 */
#define SV_MAX_CONTROLS 3

typedef struct sv_state_s* sv_state;

/* --------------------------------------------------------------- states */

/* Create a state of `batch` rows of n_qubits each (Sec. 2.2.1: 2^n complex
 * amplitudes per state; Sec. 4.2: batch dimension first).
 *   device_buffer: NULL -> the library allocates batch * 2^n * 8 bytes of
 *     device memory (256-byte aligned) and frees it in sv_free; otherwise a
 *     caller-owned device buffer of at least that size (e.g. a torch complex64
 *     tensor), 16-byte aligned, which must outlive the state.
 *   stream: a hipStream_t every kernel of this state is queued on (NULL =
 *     the default stream).
 * The contents are not initialised; call sv_reset. Errors:
 * SV_ERR_INVALID_ARGUMENT (n_qubits outside [1, SV_MAX_QUBITS], batch < 1,
 * out == NULL), SV_ERR_OUT_OF_MEMORY, SV_ERR_HIP. */
sv_status sv_alloc(int n_qubits, int batch, void* device_buffer, void* stream, sv_state* out);

/* Release the state and everything the library allocated for it (its own
 * amplitude buffer, the adjoint buffer, reduction scratch). Waits for the
 * state's stream. NULL is accepted. */
sv_status sv_free(sv_state s);

/* Device pointer of row 0 (rows follow at a stride of 2^n amplitudes). */
sv_status sv_device_ptr(sv_state s, void** out);

/* *failed := 1 if an earlier call on s failed with SV_ERR_HIP (the state
 * is then unusable), else 0. */
sv_status sv_state_failed(sv_state s, int* failed);

/* Testing hook for the sticky-error path (no GPU work): the next call on s
 * that validates the state fails with SV_ERR_HIP before queueing anything,
 * exactly as if a HIP runtime call inside it had failed; from then on the
 * state is failed. */
sv_status sv_inject_hip_error(sv_state s);

/* Every row := e_idx (the basis state |idx>; idx = 0 gives |0..0>, the start
 * state of a circuit). Asynchronous. SV_ERR_INVALID_ARGUMENT if idx >= 2^n. */
sv_status sv_reset(sv_state s, uint64_t idx);

/* Copy all rows between the state and host memory (complex64, batch * 2^n *
 * 8 bytes). to_host = 1: device -> host, then the stream is synchronised;
 * to_host = 0: host -> device, synchronised before return. */
sv_status sv_copy_state(sv_state s, void* host, int to_host);

/* ---------------------------------------------------------------- gates */

/* psi <- (M on targets, controlled by controls) psi on every row (Alg. 1 /
 * Alg. 2 of Sec. 4.1.1; both give this result).
 *   targets[n_targets], 1 <= n_targets <= SV_MAX_GATE_TARGETS, ordered.
 *   controls[n_controls], 0 <= n_controls <= SV_MAX_CONTROLS (may be NULL if 0).
 *   matrix: host complex128, row-major 2^k x 2^k, interleaved (re, im).
 *   matrix_batch_stride: 0 = one matrix for all rows; otherwise row r uses
 *     matrix + 2 * r * matrix_batch_stride doubles (per-row gates, e.g. an
 *     angle-encoded input that differs per batch row).
 *   flags: SV_FLAG_ADJOINT, SV_FLAG_CHECK_UNITARY.
 * The matrix is rounded to complex64 for the kernel. Diagonal, permutation
 * and dense matrices take different kernels; the result is the same.
 * Errors: SV_ERR_QUBIT_OUT_OF_RANGE, SV_ERR_QUBIT_OVERLAP, SV_ERR_UNSUPPORTED
 * (k or control count too large), SV_ERR_NOT_UNITARY, SV_ERR_HIP. */
sv_status sv_apply_gate(sv_state s, const int* targets, int n_targets, const int* controls,
                        int n_controls, const double* matrix, int64_t matrix_batch_stride,
                        unsigned flags);

/* Named gate kinds for circuits (sv_op.kind). Rotations are
 * R_P(theta) = exp(-i theta P / 2) (the Pauli rotations of Sec. 3);
 * U3(theta, phi, lambda) = [[c, -e^{i lambda} s], [e^{i phi} s,
 * e^{i(phi+lambda)} c]] with c = cos(theta/2), s = sin(theta/2);
 * P(lambda) = diag(1, e^{i lambda}); RXX/RYY/RZZ = exp(-i theta P(x)P / 2).
 * CNOT is SV_X with one control, CZ is SV_Z with one control. */
typedef enum sv_kind {
    SV_H = 1, SV_X = 2, SV_Y = 3, SV_Z = 4, SV_S = 5, SV_SDG = 6, SV_T = 7, SV_TDG = 8,
    SV_SX = 9, SV_RX = 10, SV_RY = 11, SV_RZ = 12, SV_P = 13, SV_U3 = 14, SV_SWAP = 15,
    SV_RXX = 16, SV_RYY = 17, SV_RZZ = 18, SV_MATRIX = 19
} sv_kind;

/* One gate of a circuit. Unused array slots are ignored. */
typedef struct sv_op {
    int32_t kind;                 /* sv_kind */
    int32_t n_targets;            /* 1 or 2 (must match the kind; SV_MATRIX: 1..2) */
    int32_t targets[2];
    int32_t n_controls;           /* 0..SV_MAX_CONTROLS */
    int32_t controls[SV_MAX_CONTROLS];
    int32_t param[3];             /* indices into the params vector, -1 = unused */
    const double* matrix;         /* SV_MATRIX only: host complex128 2^k x 2^k */
} sv_op;

/* Apply a gate list in order (each op as sv_apply_gate would).
 *   params: host doubles; row r of the batch reads
 *     params[r * params_batch_stride + op.param[j]] (stride 0 = shared).
 *   n_params: length of one row of params (indices are checked against it).
 * Validates every op before queuing any. Errors as sv_apply_gate. */
sv_status sv_run(sv_state s, const sv_op* ops, int n_ops, const double* params,
                 int64_t params_batch_stride, int n_params);

/* ---------------------------------------------------------- fused blocks */

/* A fused gate block: one 2^k x 2^k complex128 matrix on k <= 5 ordered
 * targets (Alg. 1 with |Q| = k), the product of several gates. */
typedef struct sv_block {
    int32_t k;
    int32_t targets[SV_MAX_FUSED_TARGETS];
    const double* matrix;         /* host complex128, row-major 2^k x 2^k */
} sv_block;

/* Arithmetic of sv_apply_fused. */
#define SV_FUSED_FP32_MFMA 0      /* FP32 MFMA products, FP32 accumulation */
#define SV_FUSED_BF16X3 1         /* split BF16 (hi + lo) MFMA, 3 products, FP32 accumulation */
#define SV_FUSED_VALU 2           /* FP32 vector FMAs (no matrix cores) */

/* Apply the blocks in order to every row. Each block is one sweep over the
 * state: the 2^k amplitudes that differ only in the target bits form a
 * column, and the block computes Y = M X over all 2^(n-k) columns (Alg. 1
 * with |Q| = k).
 *   k <= 5: every mode; the matrix-core modes pad the block to five qubits
 *     (M (x) I on the lowest free qubits) and need n >= 10; SV_FUSED_VALU
 *     takes k <= 5 as given.
 *   k = 6: SV_FUSED_BF16X3 only, every target >= 6, 12 <= n <= 32.
 * The block matrices are copied to device memory held by the state (the
 * call returns once the host data is consumed).
 * Errors: SV_ERR_INVALID_ARGUMENT (bad mode, k outside 1..6, n < 10 for the
 * matrix-core modes), SV_ERR_UNSUPPORTED (a six-qubit block outside its
 * conditions), SV_ERR_QUBIT_*, SV_ERR_HIP. */
sv_status sv_apply_fused(sv_state s, const sv_block* blocks, int n_blocks, int mode);

/* sv_apply_fused with a matrix per batch row (Alg. 1 per row, e.g. a fused
 * input encoding whose angles differ between rows): each block's matrix
 * points to batch consecutive 2^k x 2^k complex128 matrices, row r's at
 * matrix + r * 2 * 4^k doubles; row r of the state is swept with its own.
 * The blocks take the same target lists on every row.
 * Matrix-core modes only (SV_FUSED_FP32_MFMA, SV_FUSED_BF16X3), k <= 5,
 * n >= 10. Errors: as sv_apply_fused, plus SV_ERR_UNSUPPORTED for
 * SV_FUSED_VALU or k = 6. */
sv_status sv_apply_fused_rows(sv_state s, const sv_block* blocks, int n_blocks, int mode);

/* Host-only fusion planner (no GPU work): group the gates of a circuit, in
 * order, into blocks of at most max_k qubits (controls count as qubits) and
 * multiply each block's gates into one complex128 matrix. Gates on disjoint
 * qubits may move past each other; no gate moves past one it shares a qubit
 * with, so the block sequence equals the circuit. Several planners run (an
 * open-block grouping and frontier growth with three tie-breaking rules) and
 * the plan with the fewest blocks is returned. With max_k = 6, blocks of six
 * qubits stay off qubits 0..5 (the condition of sv_apply_fused's six-qubit
 * form); a block touching one of them holds at most five.
 *   out_blocks[max_blocks]: block descriptors; their matrix pointers point
 *     into out_matrices.
 *   out_matrices: room for max_blocks * 4^max_k complex128 (2 doubles each).
 *   *n_blocks_out: number of blocks written.
 * Errors: SV_ERR_INVALID_ARGUMENT (max_k outside 1..6, too little room). */
sv_status sv_fuse_plan(int n_qubits, const sv_op* ops, int n_ops, const double* params,
                       int n_params, int max_k, sv_block* out_blocks, int max_blocks,
                       double* out_matrices, int* n_blocks_out);

/* --------------------------------------------------------- expectations */

/* A Pauli term coeff * P with P given by its masks. */
typedef struct sv_pauli_term {
    uint64_t x_mask;
    uint64_t z_mask;
    double coeff;
} sv_pauli_term;

/* out[r * n_terms + t] = coeff_t * <psi_r| P_t |psi_r> (Sec. 2.2.1: Z-basis
 * measurement statistics; general Pauli strings), accumulated in FP64 in a
 * fixed order (bitwise reproducible run to run). out is host memory; the
 * stream is synchronised. Errors: SV_ERR_INVALID_ARGUMENT (mask bits >= n,
 * n_terms < 1), SV_ERR_CAPTURE, SV_ERR_HIP. */
sv_status sv_expval_pauli(sv_state s, const sv_pauli_term* terms, int n_terms, double* out);

/* All single-qubit Z expectations in one sweep (the paper's measure_allZ,
 * Appendix A): out[r * (n + 1) + i] = <Z_i> for i < n and out[r * (n + 1) + n]
 * = ||psi_r||^2. <sum_i Z_i> is the sum of the first n. FP64, fixed order;
 * host output, stream synchronised. */
sv_status sv_expval_z_all(sv_state s, double* out);

/* sv_expval_z_all without any allocation, for callers that cannot allocate
 * device memory mid-run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same kernels, same fixed summation
 * order, so the values are bitwise those of sv_expval_z_all.
 *   dev_out: caller-owned device memory of batch * (n + 1) doubles, 8-byte
 *     aligned; same layout as sv_expval_z_all's out.
 * The partial sums live in one fixed device buffer of the library, 2^20
 * doubles (8 MiB) per GPU, held until the process ends. A call needs
 * batch * (n + 1) of them for n <= 14 and batch * 2^(n - 14) * 15 above, so
 * n = 30 fits at batch 1 and n = 28 up to batch 4; larger shapes return
 * SV_ERR_UNSUPPORTED before anything is queued. The call is asynchronous on the state's stream (no host
 * synchronisation, no hipMalloc, hipFree or memset; every partial is written
 * before it is read, so nothing needs clearing). All calls on one GPU share
 * that buffer: calls that may overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller. Errors:
 * SV_ERR_INVALID_ARGUMENT (NULL or misaligned dev_out), SV_ERR_UNSUPPORTED,
 * SV_ERR_HIP. */
sv_status sv_expval_z_all_noalloc(sv_state s, double* dev_out);

/* ------------------------------------------------------------- adjoint */

/* Gradient of L_r = <psi_r| O |psi_r>, O = sum_t coeff_t P_t, with respect
 * to every parameter, for a state that holds the output of sv_run(ops,
 * params) on every row. Instead of storing intermediate states, each gate's
 * input is recomputed from its output as x = U^* y (Sec. 4.4):
 *     lam <- O psi;  for l = L..1: psi <- U_l^* psi;
 *     g[p] += 2 Re <lam| dU_l/dtheta_p |psi>;  lam <- U_l^* lam.
 * The inner products are FP64.
 *   grad_out: host [batch][n_params]; loss_out: host [batch] (may be NULL);
 *   drift_out: host [batch] (may be NULL) = || psi_recomputed - e_0 ||, the
 *     distance of the recovered start state from |0..0> (meaningful when the
 *     forward pass started there).
 *   lambda_buffer: NULL -> the library allocates (once, cached in the state)
 *     a second buffer of the state's size; otherwise caller-owned device
 *     memory of batch * 2^n * 8 bytes.
 * On return the state holds the recomputed start state. Errors as sv_run,
 * plus SV_ERR_CAPTURE; SV_ERR_UNSUPPORTED for SV_MATRIX ops carrying params. */
sv_status sv_adjoint_grad(sv_state s, const sv_op* ops, int n_ops, const double* params,
                          int64_t params_batch_stride, int n_params,
                          const sv_pauli_term* obs, int n_obs, void* lambda_buffer,
                          double* grad_out, double* loss_out, double* drift_out);

/* sv_adjoint_grad with a loss whose observable weights differ per row:
 * L_r = sum_t coeff_rows[r * n_obs + t] <P_t>_r (the terms' own coeff fields
 * are ignored). This is the backward of any function of the rows' Pauli
 * expectations: with coeff_rows = dF/d<P_t>_r it returns dF/dtheta (e.g.
 * the rows' <Z_i> feeding a loss in PyTorch). coeff_rows: host doubles
 * [batch][n_obs], not NULL. Outputs and errors as sv_adjoint_grad (loss_out
 * receives L_r). */
sv_status sv_adjoint_grad_weighted(sv_state s, const sv_op* ops, int n_ops, const double* params,
                                   int64_t params_batch_stride, int n_params,
                                   const sv_pauli_term* obs, int n_obs, const double* coeff_rows,
                                   void* lambda_buffer, double* grad_out, double* loss_out,
                                   double* drift_out);

/* The same backward with the gates grouped into blocks of at most
 * block_qubits (3, 4 or 5) qubits by the fusion planner: one sweep per block
 * loads the 2^block_qubits amplitudes of psi and lambda that differ only in
 * the block's qubits, and un-applies the block's gates one by one in
 * registers, adding each derivative term on the way (the per-gate recursion
 * above, gate by gate, in far fewer sweeps). Derivatives of Pauli rotations
 * (RX, RY, RZ, RXX, RYY, RZZ, with or without controls) are Im <lam|P|psi> / 2
 * with pairwise products in FP32 and the accumulation in FP64; the others
 * use G = dU/dtheta U^* in FP64 as above.
 *   coeff_rows: NULL (the terms' coeff) or per-row weights as in
 *     sv_adjoint_grad_weighted.
 * Outputs and errors as sv_adjoint_grad, plus SV_ERR_INVALID_ARGUMENT for a
 * block width outside 3..5 or n below it, and SV_ERR_UNSUPPORTED for
 * SV_MATRIX ops on more than two targets. */
sv_status sv_adjoint_grad_blocked(sv_state s, const sv_op* ops, int n_ops, const double* params,
                                  int64_t params_batch_stride, int n_params,
                                  const sv_pauli_term* obs, int n_obs, const double* coeff_rows,
                                  int block_qubits, void* lambda_buffer, double* grad_out,
                                  double* loss_out, double* drift_out);

/* ----------------------------------------------------------------- shots */

/* Exact shot sampling (Sec. 4.3.1). Draw n_shots basis indices from row
 * `row`, each with probability p_b = |psi_b|^2 / T, T = sum_c |psi_c|^2:
 *   out[s] = the smallest b with CDF(b) > t_s, CDF(b) = sum_{c <= b} |psi_c|^2,
 *   t_s = u_s * T, clamped to the largest double below T
 * (inverse-CDF sampling; the counts of the returned indices over all shots
 * are one draw of the multinomial M(n_shots, p)).
 *   dev_uniforms: device doubles [n_shots] in [0, 1): the random numbers of
 *     the draws, from the caller's generator (read only).
 *   dev_out: device int64 [n_shots], written; -1 for every shot of a state
 *     of zero norm.
 * The running sums are FP64 in a fixed blocking and order (deterministic);
 * they differ from an exact sum by rounding only, so a u_s within ~1e-15
 * (relative) of a CDF step may select the neighbouring index. Work: one read
 * sweep over the row plus one read of each 4096-amplitude block that holds a
 * shot. Scratch device memory (about 12 B per 4096 amplitudes + 16 B per
 * shot) is kept in the state. Asynchronous on the state's stream.
 * Errors: SV_ERR_INVALID_ARGUMENT (row out of range, n_shots outside
 * 0..2^31-1, NULL pointers), SV_ERR_OUT_OF_MEMORY, SV_ERR_HIP. */
sv_status sv_sample_exact(sv_state s, int row, const double* dev_uniforms, int64_t n_shots,
                          int64_t* dev_out);

/* Shot estimates of every <Z_i> from drawn indices (Sec. 4.3; the Z
 * statistics of Sec. 2.2.1 sampled): dev_est[i] = 1 - 2 c_i / S for i < n,
 * with c_i the number of indices that have bit i set and S the number of
 * indices >= 0 (a zero state's draws, -1, are left out; with none,
 * dev_est[i] = NaN). The counts are integers, so the result is exact and
 * run-to-run identical.
 *   dev_indices: device int64 [n_shots] (e.g. the output of sv_sample_exact),
 *     8-byte aligned; dev_est: device doubles [n], 8-byte aligned, written.
 * Asynchronous on the state's stream. Errors: SV_ERR_INVALID_ARGUMENT
 * (n_shots outside 0..2^31-1, NULL or misaligned pointers), SV_ERR_HIP. */
sv_status sv_sample_z_estimate(sv_state s, const int64_t* dev_indices, int64_t n_shots, double* dev_est);

/* Gaussian approximation of the shot histogram (Sec. 4.3.2), the
 * reparameterised (differentiable) draw
 *   y = shots p + sqrt(shots) D S z,
 * p = |psi|^2 / T for row `row`, D = diag(sqrt p), S = I - 2 v v^T with
 * v = (e - sqrt p) / ||e - sqrt p||, e the last basis vector (v = 0 when
 * sqrt p = e), z = (z_0, ..., z_{N-2}, 0). S is the Householder reflection
 * that maps e to sqrt p, so S z has covariance I - sqrt p sqrt p^T and y has
 * the multinomial's mean shots p and covariance shots (diag p - p p^T);
 * sum_b y_b = shots up to rounding.
 *   dev_normals: device doubles [2^n], 16-byte aligned: standard normal
 *     draws of the caller (entry 2^n - 1 is not read).
 *   shots: the number of shots n (> 0, need not be an integer).
 *   dev_y: device doubles [2^n], 16-byte aligned, written.
 * FP64 throughout; deterministic. Two sweeps (a reduction, then y).
 * Asynchronous on the state's stream.
 * Errors: SV_ERR_INVALID_ARGUMENT (row, shots <= 0, NULL or misaligned
 * pointers), SV_ERR_HIP. */
sv_status sv_sample_gaussian(sv_state s, int row, const double* dev_normals, double shots,
                             double* dev_y);

/* Gaussian shot estimate of every <Z_i> of row `row` (Sec. 4.3.2): with y
 * the histogram sv_sample_gaussian draws from the same normals,
 * est_out[i] = (1/shots) sum_b y_b (1 - 2 bit_i(b)) (host, n doubles). y is
 * not stored. Synchronous. Errors as sv_sample_gaussian. */
sv_status sv_gaussian_expval_z(sv_state s, int row, const double* dev_normals, double shots, double* est_out);

/* Backward of sv_gaussian_expval_z with the normals held fixed (the
 * reparameterisation that makes the estimate differentiable): for
 * F = sum_i upstream[i] E_i, dev_weights[b] = dF/d|psi_b|^2 (device, 2^n
 * doubles), the diagonal observable for sv_adjoint_grad_diag. Where
 * |psi_b| = 0 the term of dF/dp_b that divides by sqrt(p_b) is taken as 0
 * (the square root has no derivative there). Asynchronous on the state's
 * stream. upstream: host, n doubles. Errors as sv_sample_gaussian. */
sv_status sv_gaussian_expval_z_backward(sv_state s, int row, const double* dev_normals, double shots,
                                        const double* upstream, double* dev_weights);

/* The blocked backward on the matrix cores (Sec. 4.4's recursion regrouped
 * per block of gates on at most four qubits, taken from the last block).
 * With psi and lambda after a block and, over every column c of the 16
 * amplitudes that differ only in the block's qubits, the correlation
 * S = sum_c psi_c lambda_c^*, gate k's derivative is 2 Re Tr(X_k S) with
 * X_k = W_k (dG_k G_k^*) W_k^* (W_k the block's gates after k), and the
 * vectors before the block are U_B^* psi, U_B^* lambda. One sweep per block
 * computes S on FP64 matrix cores (the FP32 data's products exact, FP64
 * sums) and the un-apply on FP32 matrix cores; X_k and the traces are FP64
 * on the host (for blocks whose parameters differ between rows, and for
 * batches of at most four rows, the same traces as Tr(G_k S_t) with
 * S_t = W_k^* S W_k stepped down the block's gates). Rows share each block's
 * launch. Any gate kind on at most four qubits (targets and controls).
 * The state's reduction scratch grows to hold the workgroups' parts of S:
 * 4 KiB per workgroup of 16 groups of 512 amplitudes (fewer groups on small
 * states, more once a launch would pass 2^16 workgroups), at most 264 MiB.
 * Needs n >= 9 (SV_ERR_UNSUPPORTED otherwise). Arguments, outputs and errors
 * otherwise as sv_adjoint_grad_weighted (coeff_rows may be NULL). */
sv_status sv_adjoint_grad_mfma(sv_state s, const sv_op* ops, int n_ops, const double* params,
                               int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                               const double* coeff_rows, void* lambda_buffer, double* grad_out, double* loss_out,
                               double* drift_out);

/* block_qubits value of sv_adjoint_grad_diag that selects the matrix-core
 * backward of sv_adjoint_grad_mfma. */
#define SV_ADJOINT_MFMA (-1)

/* Adjoint gradient for a diagonal observable W = diag(w) given per
 * amplitude (the backward of any function of the probabilities: with
 * w_b = dF/d|psi_b|^2, dF/dtheta = 2 Re <W psi | dpsi/dtheta>, the adjoint
 * recursion of Sec. 4.4 started from lambda = W psi). Used for the
 * reparameterised shot-noise estimates of Sec. 4.3.2.
 *   dev_weights: device doubles [batch][2^n], 8-byte aligned.
 *   block_qubits: 0 = gate by gate (as sv_adjoint_grad), 3..5 = blocked (as
 *     sv_adjoint_grad_blocked, with its restrictions on ops), SV_ADJOINT_MFMA
 *     = the matrix-core backward (as sv_adjoint_grad_mfma).
 *   loss_out[r] = sum_b w_b |psi_b|^2. Other arguments, outputs and errors
 *   as sv_adjoint_grad. */
sv_status sv_adjoint_grad_diag(sv_state s, const sv_op* ops, int n_ops, const double* params,
                               int64_t params_batch_stride, int n_params, const double* dev_weights,
                               int block_qubits, void* lambda_buffer, double* grad_out, double* loss_out,
                               double* drift_out);

/* -------------------------------------------------------------- batching */

typedef struct sv_batch_plan_s* sv_batch_plan;

/* Plan a batch of independent circuits of uneven size (1 <= n_qubits[c] <=
 * 24), each started from |0..0> and measured as every <Z_i>, to be run by ONE
 * persistent kernel launch captured in a hipGraph (the batch dimension of
 * Sec. 4.2 generalised to different qubit counts).
 *   ops[c][n_ops[c]]: circuit c. Only the kinds of SV_H..SV_RZZ (no SV_MATRIX).
 *   n_params[c]: length of circuit c's parameter row.
 *   stream: the hipStream_t the graph is launched on.
 * The plan owns device arenas for the states and gate tables. Errors:
 * SV_ERR_INVALID_ARGUMENT, SV_ERR_QUBIT_*, SV_ERR_UNSUPPORTED, SV_ERR_HIP. */
sv_status sv_batch_plan_create(int n_circuits, const int* n_qubits, const sv_op* const* ops,
                               const int* n_ops, const int* n_params, void* stream,
                               sv_batch_plan* out);

/* Launch shape of a batch plan (the tile shape of the persistent kernel).
 *   tile_bits: 10..14. A tile holds 2^tile_bits complex64 amplitudes in LDS
 *     (8 KiB .. 128 KiB per workgroup); a circuit of n <= tile_bits qubits is
 *     one task run entirely in LDS, a wider one is cut into passes of tiles
 *     that go through a device arena between passes.
 *   threads: 256, 512 or 1024 threads per workgroup.
 *   reg_min_bits: 4..15. Tiles of >= 2^reg_min_bits amplitudes apply their
 *     gates as register phases (each thread holds the 16 amplitudes of four
 *     qubits and applies every gate of a phase in registers); smaller tiles
 *     make one LDS sweep per gate. 15: never.
 *   wg_per_cu: persistent workgroups per compute unit, 1..16, at most the
 *     number that are resident at once; 0: as many as are resident.
 *   phase_mode: the arithmetic of a register phase (the fusion of Sec. 4.1.1
 *     applied to the phase's four qubits):
 *     0: every gate on its own, in registers (FP32);
 *     1: a phase of >= fuse_min_gates gates is fused into one 16 x 16
 *        unitary (the gates multiplied in FP64 when the launch starts, rounded
 *        to FP32 once) applied on FP32 matrix cores;
 *     2: as 1, the product split into BF16 parts (hi*hi + hi*lo + lo*hi,
 *        FP32 accumulation; relative error ~1e-5 per phase).
 *     Fused phases need tiles of at least 2^9 amplitudes; smaller tiles and
 *     shorter phases run gate by gate.
 *   fuse_min_gates: 1..64, the fewest gates a phase needs to be fused.
 *   run_bits: 3..6 and <= tile_bits - 5. Qubits 0..run_bits-1 belong to
 *     every tile of a pass, so a tile moves between passes as contiguous runs
 *     of 2^run_bits amplitudes (64 B .. 512 B); the other tile_bits -
 *     run_bits tile qubits are chosen per pass. Fewer run bits leave more
 *     room per pass, hence fewer passes.
 * Modes 0 and 1 compute the same <Z_i> up to FP32 rounding order. */
typedef struct sv_batch_config {
    int32_t tile_bits;
    int32_t threads;
    int32_t reg_min_bits;
    int32_t wg_per_cu;
    int32_t phase_mode;
    int32_t fuse_min_gates;
    int32_t run_bits;
} sv_batch_config;

/* The configuration sv_batch_plan_create uses: {14, 512, 12, 0, 1, 3, 3}. */
sv_status sv_batch_default_config(sv_batch_config* out);

/* sv_batch_plan_create with an explicit launch shape (config NULL: the
 * default). Errors as sv_batch_plan_create; SV_ERR_INVALID_ARGUMENT for a
 * field outside its range. */
sv_status sv_batch_plan_create_ex(int n_circuits, const int* n_qubits, const sv_op* const* ops,
                                  const int* n_ops, const int* n_params,
                                  const sv_batch_config* config, void* stream, sv_batch_plan* out);

/* The plan's effective configuration (wg_per_cu resolved to the number
 * launched per CU), its persistent grid size, number of tile tasks and of
 * passes. Any output pointer may be NULL. */
sv_status sv_batch_plan_info(sv_batch_plan p, sv_batch_config* config, int* grid, int* n_tasks,
                             int* n_passes);

/* Work of a batch plan (for rooflines).
 *   fused_amp_phases: sum over fused phases of the amplitudes they update
 *     (each update is one 16 x 16 complex product share: 64 real
 *     multiply-adds per amplitude);
 *   gate_amp_updates: sum over the gates applied one by one (register or
 *     LDS sweeps) of the amplitudes each visits. */
typedef struct sv_batch_stats {
    int32_t n_tasks;
    int32_t n_passes;
    int32_t n_phases;
    int32_t n_fused_phases;
    int64_t fused_amp_phases;
    int64_t gate_amp_updates;
    int32_t max_circuit_fused_phases;   /* most fused phases any one circuit runs */
    int32_t max_circuit_gate_sweeps;    /* most gates any one circuit applies one by one */
} sv_batch_stats;

sv_status sv_batch_plan_stats(sv_batch_plan p, sv_batch_stats* out);

/* Number of doubles in the parameter block the launch reads: circuit c's
 * parameter j is at offset param_offset[c] + j. */
sv_status sv_batch_param_layout(sv_batch_plan p, int64_t* param_offsets, int64_t* total);

/* Run every circuit once: one graph launch, asynchronous on the plan's
 * stream.
 *   dev_params: device doubles laid out as sv_batch_param_layout says (read
 *     at launch time, so they may change between launches).
 *   dev_out: device doubles [n_circuits][SV_BATCH_OUT_STRIDE]: out[c][i] =
 *     <Z_i> of circuit c for i < n_qubits[c], the rest 0. */
#define SV_BATCH_OUT_STRIDE 32
sv_status sv_batch_launch(sv_batch_plan p, const double* dev_params, double* dev_out);

/* Same work as sv_batch_launch without the graph: one kernel launch per gate
 * per circuit (the plain per-gate form the batched launch is compared with). */
sv_status sv_batch_launch_pergate(sv_batch_plan p, const double* dev_params, double* dev_out);

/* Testing hook for the bounded inter-pass wait of the batched launch (no
 * effect on results otherwise). A tile of pass p > 0 of a circuit waits until
 * every tile of pass p - 1 is done, polling at most `limit` times (default
 * 2^24, far beyond any real wait); if it gives up, the circuit is marked
 * late and its outputs out[c][*] become NaN instead of a value computed from
 * an incomplete state. limit < 0: every such wait gives up at once (so a
 * test can force the late path while every kernel still ends normally).
 * Waits for the plan's stream. */
sv_status sv_batch_set_spin_limit(sv_batch_plan p, int limit);

sv_status sv_batch_plan_free(sv_batch_plan p);

/* ------------------------------------------------------------ autotuning */

/* One configuration the batch autotuner ran. */
typedef struct sv_batch_trial {
    sv_batch_config config;   /* effective configuration */
    double ms;                /* mean time of one launch (graph replay) */
    double max_dev;           /* max |out - out of the default configuration|; NaN if an output was NaN */
    double tol;               /* the bound max_dev must meet to be chosen: the sum of both
                                 configurations' rounding-error bounds on <Z_i> */
} sv_batch_trial;

/* Autotuner of the batched launch: times the batch (the same arguments as
 * sv_batch_plan_create) under a staged search over launch shapes -- tile
 * width x threads per workgroup, then the run length (run_bits), then where
 * register phases start, then workgroups per CU, then the phase arithmetic
 * (phase_mode x fuse_min_gates in {2, 3, 4, 6}) -- and returns the fastest
 * configuration whose outputs
 * agree with the default configuration's within 1e-4 (FP32 rounding order).
 *   dev_params: the device parameter block of sv_batch_param_layout (the
 *     layout does not depend on the configuration).
 *   reps: timed launches per configuration (after one warm-up launch).
 *   stream: as for the plan; timing uses HIP events on it.
 *   trials[max_trials]: may be NULL with max_trials 0; *n_trials (may be
 *     NULL) receives the number of configurations run.
 * Synchronous. Allocates and frees one output buffer and every trial's plan.
 * Errors as sv_batch_plan_create; SV_ERR_HIP when no configuration
 * reproduces the default's output. */
sv_status sv_batch_autotune(int n_circuits, const int* n_qubits, const sv_op* const* ops,
                            const int* n_ops, const int* n_params, const double* dev_params,
                            int reps, void* stream, sv_batch_config* best,
                            sv_batch_trial* trials, int max_trials, int* n_trials);

/* Autotuner of the workgroup order of the one-target dense sweep (a gate on
 * one target t >= 7 with no control, states of n >= 8 qubits; Alg. 1 with
 * |Q| = 1, the form that applies U3/RX/RY/H on those targets). Each such
 * sweep moves the state once; the two orders -- the hardware's own and
 * XCD-contiguous (each XCD a contiguous eighth of the pairs) -- touch the same
 * bytes with the same arithmetic, and which one streams faster depends on the
 * target. For every eligible target the call times one sweep of the
 * identity on s in each order (one warm-up, then three alternating timed
 * sweeps each, medians compared on s's stream) and records the faster order
 * for this device and state size; later sweeps of that target on any state
 * of n qubits on this device use it. Results of every gate are bit-identical
 * under either order. The state's values are unchanged (x*1 + y*0; a
 * negative zero may read back as +0). Without a call every target takes the
 * hardware's order.
 *   ms_out: NULL, or host float[2 n]: ms_out[2t] / ms_out[2t + 1] = median
 *           time of target t in the hardware / XCD-contiguous order (0 for
 *           targets that do not use this form).
 * Synchronous; n < 8 tunes nothing. Errors: SV_ERR_INVALID_ARGUMENT (bad
 * state), SV_ERR_CAPTURE (s's stream is capturing), SV_ERR_HIP. */
sv_status sv_sweep_order_tune(sv_state s, float* ms_out);

/* The order record that sv_sweep_order_tune writes, set or read directly
 * (to pin a known choice, or to compare orders): bit t of xcd_mask set = the
 * one-target dense sweep on target t takes the XCD-contiguous order, for
 * states of s's size on the current device. Bits of targets that do not use
 * that sweep are ignored. Host only, immediate. Errors:
 * SV_ERR_INVALID_ARGUMENT (bad state, NULL xcd_mask). */
sv_status sv_sweep_order_set(sv_state s, uint64_t xcd_mask);
sv_status sv_sweep_order_get(sv_state s, uint64_t* xcd_mask);

/* One way of applying a circuit: plain per-gate sweeps (max_k = 1, mode =
 * -1) or the fusion planner's blocks of at most max_k qubits applied with
 * sv_apply_fused in `mode`. */
typedef struct sv_fusion_choice {
    int32_t max_k;
    int32_t mode;
    int32_t n_sweeps;         /* gates (plain) or blocks: passes over the state */
    double ms;                /* time of one application of the whole circuit */
} sv_fusion_choice;

/* Autotuner of the fusion width: times the circuit (host params, the same
 * for every row) on the state s as plain sweeps, as SV_FUSED_VALU blocks of
 * max_k = 2..5, (n >= 10) as five-qubit matrix-core blocks in the modes that
 * mode_mask allows, and (12 <= n <= 32, BF16X3 allowed) as six-qubit blocks
 * (bit 1 << SV_FUSED_* of mode_mask; plain sweeps are always tried), and
 * returns the fastest. The state's contents are overwritten (reset it
 * afterwards). A width that some gate of the circuit exceeds is skipped.
 *   reps: timed applications per candidate (after one warm-up).
 * Synchronous. Errors as sv_run / sv_fuse_plan / sv_apply_fused. */
sv_status sv_fused_autotune(sv_state s, const sv_op* ops, int n_ops, const double* params,
                            int n_params, uint32_t mode_mask, int reps, sv_fusion_choice* best,
                            sv_fusion_choice* trials, int max_trials, int* n_trials);

/* ------------------------------------------------------------- utility */

/* Plain device-to-device copy kernel of `bytes` (multiple of 16, 16-byte
 * aligned pointers) on `stream`: the measured bandwidth ceiling used to scale
 * hardware byte counters. Asynchronous. */
sv_status sv_stream_copy(void* dst, const void* src, uint64_t bytes, void* stream);

/* Static description of a status code. Never NULL. */
const char* sv_status_string(sv_status st);

/* Detail text of the last failure on this thread ("" if none). Valid until
 * the next call on this thread. */
const char* sv_last_error(void);

/* Check gate arguments without a state or GPU (host only): the same checks
 * sv_apply_gate makes before queuing work. */
sv_status sv_check_gate(int n_qubits, const int* targets, int n_targets, const int* controls,
                        int n_controls);

#ifdef __cplusplus
}
#endif

#endif /* LIBSV_SV_H_ */
