/*
 * Plain FP64 CPU oracle for the state-vector hot path of the PennyLane
 * Lightning paper (arXiv 2403.02512).  TEST INFRASTRUCTURE ONLY: it exists to
 * check the GPU library, and only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * table with the GPU library.
 *
 * Conventions (paper Sec. 2.1.1, Alg. 1): a state of n qubits is 2^n complex
 * doubles; wire w is index bit (n-1-w), so wire 0 is the most significant bit.
 * A gate acting on wires (w_1..w_k) has a 2^k x 2^k matrix whose row/column
 * index j carries w_1 as its most significant bit.
 */
#ifndef QSV_ORACLE_H
#define QSV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Gate identifiers of the oracle (its own numbering). */
enum orc_gate {
    ORC_IDENTITY = 0, ORC_PAULIX, ORC_PAULIY, ORC_PAULIZ, ORC_HADAMARD, ORC_S, ORC_T, ORC_SX,
    ORC_PHASESHIFT, ORC_RX, ORC_RY, ORC_RZ, ORC_ROT, ORC_U3,
    ORC_CNOT, ORC_CY, ORC_CZ, ORC_SWAP,
    ORC_CRX, ORC_CRY, ORC_CRZ, ORC_CROT, ORC_CPHASESHIFT,
    ORC_ISINGXX, ORC_ISINGYY, ORC_ISINGZZ, ORC_ISINGXY, ORC_SINGLEEXC,
    ORC_TOFFOLI, ORC_CSWAP, ORC_DOUBLEEXC, ORC_MULTIRZ, ORC_UNITARY,
    ORC_NUM_GATES
};

/* One operation.  The first n_ctrls wires are extra control wires (required
 * values in ctrl_values, bit j for control j); the remaining wires are the
 * gate's own wires.  Angle slot s is scale[s]*params[param[s]] when
 * param[s] >= 0, otherwise the constant scale[s].  inverse applies M^dagger.
 * For ORC_UNITARY the matrix (row-major complex doubles, interleaved re/im)
 * starts at complex element matrix_offset of the matrices array. */
typedef struct {
    int32_t gate;
    int32_t n_wires;
    int32_t n_ctrls;
    uint32_t ctrl_values;
    int32_t inverse;
    int32_t wires[8];
    int32_t param[3];
    double scale[3];
    int64_t matrix_offset;
} orc_op;

/* Number of own wires of a gate (0 for the variable-width gates
 * ORC_MULTIRZ / ORC_UNITARY) and number of angles it takes. */
int orc_gate_wires(int gate);
int orc_gate_nparams(int gate);

/* Matrix of a gate on its own wires for the given angles (dim x dim, complex
 * interleaved, row-major).  k = number of own wires.  Returns 0 on success. */
int orc_gate_matrix(int gate, int k, const double *angles, int inverse, double *out);

/* Generator G (dim x dim, complex interleaved) and constant c such that the
 * one-angle gate is U(a) = exp(i c a G).  Returns 0, or -1 for gates without
 * a single generator. */
int orc_gate_generator(int gate, int k, double *out, double *c);

/* psi <- M psi for a 2^k x 2^k matrix on the given wires (plain definition). */
void orc_apply_matrix(int n, double *psi, int k, const int32_t *wires, const double *mat);

/* Apply a list of operations in order.  Returns 0, or -1 on a bad op. */
int orc_apply(int n, double *psi, const orc_op *ops, int64_t n_ops,
              const double *params, const double *matrices);

/* <a|b> with pairwise summation (deterministic for any thread count). */
void orc_inner(int n, const double *a, const double *b, double *out_re_im);

/* Expectation value of each observable.  An observable is a Pauli sum:
 * obs_nterms[o] terms; term t has coefficient coeff[t] and letters
 * paulis[t*n + w] in {'I','X','Y','Z'} for wire w (terms of all observables
 * are concatenated in order). */
int orc_expval(int n, const double *psi, int n_obs, const int32_t *obs_nterms,
               const double *coeff, const char *paulis, double *out);

/* lambda <- H psi for one Pauli sum. */
int orc_apply_pauli_sum(int n, const double *psi, int n_terms, const double *coeff,
                        const char *paulis, double *lambda);

/* Adjoint-method Jacobian jac[o*n_params + p] = d<O_o>/d params[p], given the
 * state after all operations.  psi is not modified. */
int orc_adjoint_jacobian(int n, const double *psi, const orc_op *ops, int64_t n_ops,
                         const double *params, int64_t n_params, const double *matrices,
                         int n_obs, const int32_t *obs_nterms, const double *coeff,
                         const char *paulis, double *jac);

/* Number of OpenMP threads the oracle loops use (1 without OpenMP). */
int orc_num_threads(void);

/* Shot sampling by inverse transform (Sec. 4.3, sampling workloads): with
 * p_i = |psi_i|^2 and the running sum c_i = p_0 + .. + p_i (index order,
 * sequential FP64), out[k] = the smallest i with c_i > u[k] * c_{N-1}.  The
 * uniforms u[k] in [0, 1) are inputs.  Returns -1 for a zero state. */
int orc_sample(int n, const double *psi, int64_t n_samples, const double *u, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif
