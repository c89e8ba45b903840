/*
 * qsv -- MI355X (gfx950) state-vector hot path: gate application, Pauli-sum
 * expectation values and adjoint-method Jacobians, after the PennyLane
 * Lightning paper (arXiv 2403.02512).
 *
 * C ABI only: plain pointers and sizes; no C++ types, exceptions or torch
 * types cross this boundary.  Every entry point returns a qsv_status; on an
 * error qsv_last_error() (per context, or the thread's last error when no
 * context exists) gives a message.  Arguments are validated completely before
 * any device work, so a validation error leaves every buffer untouched.
 *
 * Conventions (paper Sec. 2.1.1, Alg. 1):
 *  - a state of n qubits is 2^n contiguous complex amplitudes, interleaved
 *    (re, im), FP64 for QSV_C128 and FP32 for QSV_C64;
 *  - wire w is index bit (n-1-w): wire 0 is the most significant bit;
 *  - a gate on wires (w_1..w_k) has a 2^k x 2^k row-major matrix whose index
 *    carries w_1 as its most significant bit;
 *  - Pauli masks use index bits (bit p <-> wire n-1-p); a Y letter sets the
 *    bit in both the x and the z mask.
 * Expectation values and gradients are accumulated and returned in FP64 for
 * both state precisions (paper Sec. 2: float/double templating end to end).
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSV_OK = 0,
    QSV_ERR_ARG = -1,         /* null pointer, bad size, bad option          */
    QSV_ERR_WIRE = -2,        /* wire out of range or repeated in one op     */
    QSV_ERR_DTYPE = -3,       /* precision mismatch between objects          */
    QSV_ERR_OOM = -4,         /* device or host allocation failed            */
    QSV_ERR_HIP = -5,         /* a HIP runtime call failed (state undefined) */
    QSV_ERR_UNSUPPORTED = -6, /* gate/width/feature not supported            */
    QSV_ERR_PARAM = -7        /* parameter index or matrix offset invalid    */
} qsv_status;

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_dtype;

/* Largest register the library accepts (2^34 amplitudes). */
#define QSV_MAX_QUBITS 34
/* Most wires one operation may name (extra controls + own wires). */
#define QSV_MAX_OP_WIRES 8

/* Gate identifiers (PennyLane names; paper Sec. 2.1.2 lists the gate set).
 * Own wires: 1 for the single-qubit gates, 2 for CNOT..SINGLEEXC, 3 for
 * TOFFOLI/CSWAP, 4 for DOUBLEEXC, any for MULTIRZ/UNITARY.  Angles: 1 for
 * PHASESHIFT, RX, RY, RZ, the controlled rotations, the Ising gates,
 * SINGLEEXC, DOUBLEEXC and MULTIRZ; 3 for ROT (phi, theta, omega: RZ(omega)
 * RY(theta) RZ(phi)), U3 (theta, phi, lambda) and CROT. */
typedef enum {
    QSV_GATE_PAULIX = 1, QSV_GATE_PAULIY, QSV_GATE_PAULIZ, QSV_GATE_HADAMARD,
    QSV_GATE_S, QSV_GATE_T, QSV_GATE_SX, QSV_GATE_IDENTITY,
    QSV_GATE_PHASESHIFT = 20, QSV_GATE_RX, QSV_GATE_RY, QSV_GATE_RZ, QSV_GATE_ROT, QSV_GATE_U3,
    QSV_GATE_CNOT = 40, QSV_GATE_CY, QSV_GATE_CZ, QSV_GATE_SWAP,
    QSV_GATE_CRX, QSV_GATE_CRY, QSV_GATE_CRZ, QSV_GATE_CROT, QSV_GATE_CPHASESHIFT,
    QSV_GATE_ISINGXX, QSV_GATE_ISINGYY, QSV_GATE_ISINGZZ, QSV_GATE_ISINGXY, QSV_GATE_SINGLEEXC,
    QSV_GATE_TOFFOLI = 70, QSV_GATE_CSWAP, QSV_GATE_DOUBLEEXC, QSV_GATE_MULTIRZ,
    QSV_GATE_UNITARY = 90
} qsv_gate;

/* One operation (paper Sec. 2.1.1 Listing 1: a gate, its wires, an inverse
 * flag and its angles).  wires[0..n_ctrls-1] are extra control wires whose
 * required values are the bits of ctrl_values (bit j for control j);
 * wires[n_ctrls..n_wires-1] are the gate's own wires.  Angle slot s is
 * scale[s] * params[param[s]] if param[s] >= 0, else the constant scale[s].
 * inverse != 0 applies the adjoint M^dagger.  For QSV_GATE_UNITARY the
 * 2^k x 2^k matrix (complex FP64, row-major) starts at complex element
 * matrix_offset of the call's matrices array; it is not differentiable. */
typedef struct qsv_op {
    int32_t gate;
    int32_t n_wires;
    int32_t n_ctrls;
    uint32_t ctrl_values;
    int32_t inverse;
    int32_t wires[QSV_MAX_OP_WIRES];
    int32_t param[3];
    double scale[3];
    int64_t matrix_offset;
} qsv_op;

/* A Pauli-sum observable H = sum_t coeff[t] P_t (paper Sec. 2.2: Pauli words
 * and Hamiltonians).  P_t = tensor product with X on bits x_mask[t] & ~z,
 * Z on z & ~x, Y on x & z.  Arrays are host memory owned by the caller. */
typedef struct qsv_pauli_sum {
    int64_t n_terms;
    const double *coeff;
    const uint64_t *x_mask;
    const uint64_t *z_mask;
} qsv_pauli_sum;

typedef struct qsv_ctx qsv_ctx;     /* one device + one HIP stream; not thread-safe */
typedef struct qsv_state qsv_state; /* 2^n amplitudes in device memory              */

/* ---------------------------------------------------------------- library */
const char *qsv_version(void);
const char *qsv_status_string(int status);
/* Message of the calling thread's last failure (also for ctx-less calls). */
const char *qsv_thread_last_error(void);
/* Number of visible HIP devices (0 without a GPU; never fails). */
int qsv_device_count(void);

/* ---------------------------------------------------------------- context */
/* Create a context on `device` (paper Sec. 2.2: the GPU device selects its
 * GPU at run time and manages that GPU's memory and transfers).  hip_stream: a
 * hipStream_t to issue all work on (borrowed, e.g. torch's current stream), or
 * NULL for a library-owned stream.  *out is owned by the caller and released
 * by qsv_ctx_destroy. */
qsv_status qsv_ctx_create(int device, void *hip_stream, qsv_ctx **out);
void qsv_ctx_destroy(qsv_ctx *ctx);
const char *qsv_last_error(const qsv_ctx *ctx);
/* Switch the stream later calls are issued on (borrowed). */
qsv_status qsv_ctx_set_stream(qsv_ctx *ctx, void *hip_stream);
qsv_status qsv_ctx_synchronize(qsv_ctx *ctx);

/* Tuning options (QSV_OPT_*): value semantics given per option. */
enum {
    QSV_OPT_FUSION = 1,         /* 0: one kernel per gate, 1: LDS-tiled fusion (default) */
    QSV_OPT_TILE_BITS = 2,      /* qubits per LDS tile for one-vector passes (0: default) */
    QSV_OPT_TILE_BITS_ADJ = 3,  /* qubits per LDS tile for two-vector adjoint passes      */
    QSV_OPT_LOW_BITS = 4,       /* low index bits every tile keeps for coalescing         */
    QSV_OPT_PROFILE = 5,        /* 1: time every launch with HIP events                   */
    QSV_OPT_NONTEMPORAL = 6,    /* 1: every kernel that writes the state back uses
                                   non-temporal (streaming) stores (paper Sec. 3.1); 0 default */
    QSV_OPT_LAYERS = 7,         /* 1: one-qubit runs in register groups run as layers (default) */
    QSV_OPT_TILE_WS = 10,       /* 1: group-only tile passes of >= 2^11 amplitudes run
                                   warp-specialised where two tile buffers fit the LDS (load
                                   waves fetch the next tile while compute waves run this
                                   one); 0 (default): one buffer per block, two blocks per CU */
    QSV_OPT_DENSE_MFMA = 11,    /* 1: 6-qubit dense matrices on complex128 states run on the
                                   FP64 matrix cores (16x16x4 MFMA); 0 (default): FP64 FMA   */
    /* Fault injection, for tests of the error paths only:                                     */
    QSV_OPT_TEST_ALLOC_LIMIT = 8, /* >0: a device allocation above this many bytes fails with
                                     QSV_ERR_OOM, as if the device were full; 0: no limit    */
    QSV_OPT_TEST_FAIL_LAUNCH = 9  /* k>0: the k-th kernel launch from now fails with
                                     QSV_ERR_HIP before it is issued (then the count is spent) */
};
qsv_status qsv_ctx_set_option(qsv_ctx *ctx, int option, int64_t value);
qsv_status qsv_ctx_get_option(qsv_ctx *ctx, int option, int64_t *value);
/* Device bytes currently cached as adjoint/expval workspace; release it. */
qsv_status qsv_ctx_workspace_bytes(qsv_ctx *ctx, size_t *out);
qsv_status qsv_ctx_release_workspace(qsv_ctx *ctx);

/* Per-kernel-family statistics collected while QSV_OPT_PROFILE is on:
 * launches, summed device time (ms, from HIP events on the context stream)
 * and summed algorithmic HBM bytes (the bytes the method must move, counted
 * by the host from each launch's shape).  Synchronises the context stream.
 * kind: 0 .. qsv_kernel_kinds()-1. */
int qsv_kernel_kinds(void);
const char *qsv_kernel_name(int kind);
qsv_status qsv_ctx_kernel_stats(qsv_ctx *ctx, int kind, int64_t *launches, double *ms, double *bytes);
qsv_status qsv_ctx_reset_stats(qsv_ctx *ctx);

/* ---------------------------------------------------------------- states */
/* Allocate an owned state of n_qubits (1..QSV_MAX_QUBITS) in |0..0>, resident
 * in device memory (paper Sec. 2.2: gates, observables and the adjoint method
 * work directly on the GPU-resident state vector; Sec. 2: complex64 or
 * complex128 by dtype). */
qsv_status qsv_state_create(qsv_ctx *ctx, int n_qubits, qsv_dtype dtype, qsv_state **out);
/* Wrap caller-owned device memory of 2^n amplitudes (e.g. a torch tensor's
 * storage, 16-byte aligned for C128, 8 for C64).  The library never frees it;
 * the caller keeps it alive while the state is in use. */
qsv_status qsv_state_wrap(qsv_ctx *ctx, int n_qubits, qsv_dtype dtype, void *dev_ptr, qsv_state **out);
void qsv_state_destroy(qsv_state *s);
int qsv_state_n_qubits(const qsv_state *s);
void *qsv_state_device_ptr(const qsv_state *s);
/* psi <- |basis_index> (paper Sec. 2.1.1: a computational basis state). */
qsv_status qsv_state_reset(qsv_state *s, uint64_t basis_index);
qsv_status qsv_state_copy(qsv_state *dst, const qsv_state *src);
/* Blocking copies between the state and host memory of 2^n amplitudes. */
qsv_status qsv_state_to_host(const qsv_state *s, void *host);
qsv_status qsv_state_from_host(qsv_state *s, const void *host);

/* ---------------------------------------------------------------- validation (host only) */
/* Check an op list against an n-qubit register: gate ids, wire counts, wire
 * range and distinctness, param indices < n_params, matrix offsets within
 * n_matrix_elems complex elements.  Touches no device. */
qsv_status qsv_validate_ops(int n_qubits, const qsv_op *ops, size_t n_ops, size_t n_params,
                            size_t n_matrix_elems);
qsv_status qsv_validate_obs(int n_qubits, const qsv_pauli_sum *obs, size_t n_obs);

/* Plan of a call without running it (host only, no device): the number of
 * passes over the state (HBM round trips), how many of them are LDS-tiled
 * fused passes, the number of lowered tile ops, and the algorithmic HBM
 * bytes of all passes.  adjoint = 0 plans qsv_apply; 1 plans one reverse
 * sweep of qsv_adjoint_jacobian (one observable, without lambda = H psi).
 * tile_bits / low_bits = 0 pick the defaults, fusion = 0 one pass per gate, 1 fused
 * (default), 2 fused without one-qubit layers (QSV_OPT_LAYERS = 0). */
qsv_status qsv_plan_stats(int n_qubits, qsv_dtype dtype, const qsv_op *ops, size_t n_ops, const double *params,
                          size_t n_params, const double *matrices, size_t n_matrix_elems, int adjoint,
                          int tile_bits, int low_bits, int fusion, int64_t *n_passes, int64_t *n_tile_passes,
                          int64_t *n_kernel_ops, double *alg_bytes);

/* The same plan as a JSON document (host only): every pass with its kernel
 * arguments, the lowered tile ops, the coefficient and word tables and the
 * inner-product slot -> (parameter, coefficient) map.  Writes at most cap
 * bytes (NUL-terminated) to out and the full size + 1 to *needed. */
qsv_status qsv_plan_json(int n_qubits, qsv_dtype dtype, const qsv_op *ops, size_t n_ops, const double *params,
                         size_t n_params, const double *matrices, size_t n_matrix_elems, int adjoint,
                         int tile_bits, int low_bits, int fusion, char *out, size_t cap, size_t *needed);

/* ---------------------------------------------------------------- hot path */
/* Apply ops in order (paper Sec. 2.1.1 Alg. 1 and Alg. 2; Sec. 2.1.2 gates).
 * Asynchronous on the context stream: host arrays may be reused on return.
 * Gate matrices are built on the host in FP64 and uploaded once per call. */
qsv_status qsv_apply(qsv_state *s, const qsv_op *ops, size_t n_ops, const double *params,
                     size_t n_params, const double *matrices, size_t n_matrix_elems);

/* out[o] = <psi|H_o|psi> for n_obs Pauli sums (paper Sec. 2.2).  Host output;
 * synchronises the context stream. */
qsv_status qsv_expval(qsv_state *s, const qsv_pauli_sum *obs, size_t n_obs, double *out);

/* qsv_expval without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same results as qsv_expval, with the Pauli tables,
 * per-block partials and results kept in a static device scratch of 8 MiB
 * that every device holds for the life of the process.  Observables whose
 * tables, partials and results exceed it are rejected with QSV_ERR_ARG
 * before any device work (a few hundred thousand terms fit).  Calls that
 * overlap on one device share the scratch and race: issue them in order.
 * Host output; synchronises the context stream. */
qsv_status qsv_expval_noalloc(qsv_state *s, const qsv_pauli_sum *obs, size_t n_obs, double *out);

/* Variance out[o] = <H_o^2> - <H_o>^2 = ||H_o psi||^2 - <H_o>^2 for n_obs Pauli
 * sums (paper Sec. 2.2 lists variances among the measurements).  Host output;
 * synchronises the context stream. */
qsv_status qsv_var(qsv_state *s, const qsv_pauli_sum *obs, size_t n_obs, double *out);

/* <psi|S|psi> for a sparse 2^n x 2^n matrix S in CSR form (paper Sec. 2.2:
 * SparseHamiltonian observables): row_ptr[2^n + 1] (row_ptr[0] = 0,
 * row_ptr[2^n] = nnz), col[nnz] column indices, values[2 nnz] complex FP64
 * interleaved.  out[0], out[1] = real and imaginary part (the latter is zero
 * up to rounding for Hermitian S).  Host arrays, copied once; validated
 * (monotone row_ptr, columns in range) before any device work. */
qsv_status qsv_expval_sparse(qsv_state *s, const int64_t *row_ptr, const int64_t *col, const double *values,
                             int64_t nnz, double *out);

/* Marginal probabilities of the computational-basis outcomes of n_wires wires
 * (paper Sec. 2.2: probabilities, e.g. the GHZ listing's three wires).
 * out[b] for b < 2^n_wires, the first listed wire being the most significant
 * bit of b.  1 <= n_wires <= min(n, 20), distinct wires.  FP64 sums in a fixed
 * order.  Host output; synchronises the context stream. */
qsv_status qsv_probs(qsv_state *s, const int32_t *wires, int n_wires, double *out);

/* Shot sampling by inverse transform (paper Sec. 4.3, sampling workloads):
 * with p_i = |psi_i|^2, out[k] = the basis index i at which the running sum
 * p_0 + .. + p_i first exceeds u[k] * sum_j p_j.  The uniforms u[k] in [0, 1)
 * come from the caller's generator (host array of n_samples doubles); out is
 * a host array of n_samples indices (wire 0 = most significant bit).  Only
 * indices with p_i > 0 are returned; where a u[k] lands within rounding of a
 * boundary of the running sum either neighbour may be returned.  Errors:
 * QSV_ERR_ARG for NULL arrays, u outside [0, 1) or a zero state.
 * Synchronises the context stream. */
qsv_status qsv_sample(qsv_state *s, const double *u, size_t n_samples, uint64_t *out);

/* Adjoint-method Jacobian (paper Sec. 2.1 and Sec. 3.1.1; Jones & Gacon):
 * jac[o*n_params + p] = d<psi|H_o|psi>/d params[p], where s holds the state
 * AFTER the ops.  The forward states are recomputed by un-applying the gates.
 * expval (optional, n_obs doubles) receives <H_o>.  flags: QSV_ADJ_INPLACE
 * lets the library use s as the phi buffer (s then holds the initial state on
 * return, up to rounding) so only one workspace vector is needed; otherwise s
 * is preserved and two workspace vectors are used.  Host outputs;
 * synchronises the context stream. */
#define QSV_ADJ_INPLACE 1u
qsv_status qsv_adjoint_jacobian(qsv_state *s, const qsv_op *ops, size_t n_ops, const double *params,
                                size_t n_params, const double *matrices, size_t n_matrix_elems,
                                const qsv_pauli_sum *obs, size_t n_obs, double *jac, double *expval,
                                uint32_t flags);

/* Vector-Jacobian product: grad[p] = sum_o cotangent[o] d<H_o>/d params[p]
 * with ONE adjoint sweep (lambda = sum_o cotangent[o] H_o psi). */
qsv_status qsv_adjoint_vjp(qsv_state *s, const qsv_op *ops, size_t n_ops, const double *params,
                           size_t n_params, const double *matrices, size_t n_matrix_elems,
                           const qsv_pauli_sum *obs, size_t n_obs, const double *cotangent,
                           double *grad, double *expval, uint32_t flags);

/* ---------------------------------------------------------------- batched circuits */
/* A batch of independent circuits of possibly different widths (paper Sec.
 * 4.1-4.2: batched task execution of many circuits and observables).
 * Circuit i has n_qubits[i] qubits, the ops ops[op_offsets[i] ..
 * op_offsets[i+1]) (op_offsets has n_circuits + 1 entries), n_params[i]
 * parameters, one Pauli-sum observable obs[i], and shares the matrices array
 * (for QubitUnitary ops).  Host arrays are copied; the batch owns one pooled
 * device allocation holding every circuit's state and adjoint workspace
 * (3 x 2^n amplitudes each).  Released by qsv_batch_destroy. */
typedef struct qsv_batch qsv_batch;
qsv_status qsv_batch_create(qsv_ctx *ctx, qsv_dtype dtype, size_t n_circuits, const int32_t *n_qubits,
                            const qsv_op *ops, const size_t *op_offsets, const size_t *n_params,
                            const double *matrices, size_t n_matrix_elems, const qsv_pauli_sum *obs,
                            qsv_batch **out);
void qsv_batch_destroy(qsv_batch *b);

/* Run every circuit from |0..0> with params (concatenated in circuit order):
 * expval[i] = <H_i>; if grad != NULL also the adjoint gradient of each
 * circuit, concatenated like params.  Pass s of every circuit runs in one
 * launch.  QSV_BATCH_GRAPH: capture the launch sequence in a HIP graph on the
 * first call and replay it while the batch's gate structure is unchanged (new
 * parameter values only update the uploaded coefficient table).  Host
 * outputs; synchronises the context stream. */
#define QSV_BATCH_GRAPH 1u
qsv_status qsv_batch_run(qsv_batch *b, const double *params, double *expval, double *grad, uint32_t flags);

/* ---------------------------------------------------------------- tile-width tuner */
/* Choose the LDS tile widths (QSV_OPT_TILE_BITS and QSV_OPT_TILE_BITS_ADJ) for
 * a circuit by timing it on this device (paper Sec. 4.2: batch and chunk sizes
 * chosen per workload): the forward program (reset to |0..0> + ops) for
 * every width from 2^10 amplitudes up to the LDS limit, then, if obs and
 * parameters are given, the adjoint sweep for every two-vector width from
 * 2^9 up.  At the chosen widths it then times the whole program (forward,
 * and the adjoint sweep when given) with one-qubit layers on and off
 * (QSV_OPT_LAYERS) and with the default, one fewer and one more always-local
 * low index bits (QSV_OPT_LOW_BITS).  The fastest widths are returned; all
 * four choices are set on the context, where the single-circuit entry points
 * and qsv_batch_run (which plans every circuit with the context's options)
 * use them.  The state's contents are overwritten (it ends as the circuit's
 * output state).  On error the context options are left unchanged. */
qsv_status qsv_autotune(qsv_state *s, const qsv_op *ops, size_t n_ops, const double *params, size_t n_params,
                        const double *matrices, size_t n_matrix_elems, const qsv_pauli_sum *obs, size_t n_obs,
                        int32_t *tile_bits, int32_t *tile_bits_adj);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
