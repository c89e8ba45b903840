/*
 * Plain FP64 CPU oracle for the state-vector hot path of arXiv 2403.02512
 * (PennyLane Lightning).  TEST INFRASTRUCTURE ONLY -- never part of the
 * product path; only tests, the smoke check and the benchmark's CPU-baseline
 * leg load it.  Shares no code with the GPU library.
 *
 * Everything here is the plain definition:
 *  - gate application (Sec. 2.1.1): for every index whose target-wire bits are
 *    all zero, gather the 2^k amplitudes, multiply by the full 2^k x 2^k
 *    matrix (controlled gates use the full block matrix diag(I,..,I,V)), and
 *    scatter back.  The paper's faster index enumerations (Alg. 1 and Alg. 2)
 *    are deliberately NOT used here; the tests check them against this.
 *  - expectation values (Sec. 2.2): <psi|P|psi> with P applied to a copy of
 *    psi one Pauli letter at a time, then an inner product with pairwise
 *    summation.
 *  - adjoint Jacobian (Sec. 2.1 and Sec. 3.1.1, which cite the adjoint
 *    method of Jones & Gacon): walk the operations backwards, for every
 *    trainable angle take -2c Im<lambda|G|phi> for U = exp(i c theta G), and
 *    un-apply each operation from phi and lambda.
 *
 * Wire w is index bit n-1-w (Alg. 1, q_offset = n - q - 1).
 * Compile with -O2 -ffp-contract=off and no fast-math.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define MAXK 10 /* widest matrix the oracle builds: 2^10 x 2^10 */

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_gate_wires(int gate) {
    switch (gate) {
    case ORC_IDENTITY: case ORC_PAULIX: case ORC_PAULIY: case ORC_PAULIZ:
    case ORC_HADAMARD: case ORC_S: case ORC_T: case ORC_SX:
    case ORC_PHASESHIFT: case ORC_RX: case ORC_RY: case ORC_RZ: case ORC_ROT: case ORC_U3:
        return 1;
    case ORC_CNOT: case ORC_CY: case ORC_CZ: case ORC_SWAP:
    case ORC_CRX: case ORC_CRY: case ORC_CRZ: case ORC_CROT: case ORC_CPHASESHIFT:
    case ORC_ISINGXX: case ORC_ISINGYY: case ORC_ISINGZZ: case ORC_ISINGXY: case ORC_SINGLEEXC:
        return 2;
    case ORC_TOFFOLI: case ORC_CSWAP:
        return 3;
    case ORC_DOUBLEEXC:
        return 4;
    default:
        return 0; /* MultiRZ, QubitUnitary: any width */
    }
}

int orc_gate_nparams(int gate) {
    switch (gate) {
    case ORC_PHASESHIFT: case ORC_RX: case ORC_RY: case ORC_RZ:
    case ORC_CRX: case ORC_CRY: case ORC_CRZ: case ORC_CPHASESHIFT:
    case ORC_ISINGXX: case ORC_ISINGYY: case ORC_ISINGZZ: case ORC_ISINGXY:
    case ORC_SINGLEEXC: case ORC_DOUBLEEXC: case ORC_MULTIRZ:
        return 1;
    case ORC_ROT: case ORC_U3: case ORC_CROT:
        return 3;
    default:
        return 0;
    }
}

/* ---------------------------------------------------------------- matrices */

static void mat_identity(cplx *m, int dim) {
    memset(m, 0, sizeof(cplx) * (size_t)dim * dim);
    for (int i = 0; i < dim; ++i) m[i * dim + i] = 1.0;
}

static void mat_mul(const cplx *a, const cplx *b, cplx *out, int dim) {
    cplx *t = malloc(sizeof(cplx) * (size_t)dim * dim);
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) {
            cplx s = 0;
            for (int j = 0; j < dim; ++j) s += a[r * dim + j] * b[j * dim + c];
            t[r * dim + c] = s;
        }
    memcpy(out, t, sizeof(cplx) * (size_t)dim * dim);
    free(t);
}

static void mat_dagger(cplx *m, int dim) {
    for (int r = 0; r < dim; ++r)
        for (int c = r; c < dim; ++c) {
            cplx a = m[r * dim + c], b = m[c * dim + r];
            m[r * dim + c] = conj(b);
            m[c * dim + r] = conj(a);
        }
}

/* Single-qubit rotation exp(-i t/2 P) for P in {X,Y,Z}. */
static void rot1(char p, double t, cplx *m) {
    double c = cos(t / 2), s = sin(t / 2);
    if (p == 'X') { m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; }
    else if (p == 'Y') { m[0] = c; m[1] = -s; m[2] = s; m[3] = c; }
    else { m[0] = cexp(-I * t / 2); m[1] = 0; m[2] = 0; m[3] = cexp(I * t / 2); }
}

/* |0><0| (x) I + |1><1| (x) V for a 2x2 V. */
static void controlled2(const cplx *v, cplx *m) {
    mat_identity(m, 4);
    m[2 * 4 + 2] = v[0]; m[2 * 4 + 3] = v[1];
    m[3 * 4 + 2] = v[2]; m[3 * 4 + 3] = v[3];
}

/* Kronecker product of 2x2 matrices a (x) b. */
static void kron2(const cplx *a, const cplx *b, cplx *m) {
    for (int r1 = 0; r1 < 2; ++r1)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int r2 = 0; r2 < 2; ++r2)
                for (int c2 = 0; c2 < 2; ++c2)
                    m[(2 * r1 + r2) * 4 + (2 * c1 + c2)] = a[r1 * 2 + c1] * b[r2 * 2 + c2];
}

static const cplx PX[4] = {0, 1, 1, 0};
static const cplx PZ[4] = {1, 0, 0, -1};
static void pauli_y(cplx *m) { m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; }

int orc_gate_matrix(int gate, int k, const double *ang, int inverse, double *out_d) {
    cplx *m = (cplx *)out_d;
    int dim = 1 << k;
    double a = ang ? ang[0] : 0.0;
    cplx t2[4], u[4], v[4];
    switch (gate) {
    case ORC_IDENTITY: mat_identity(m, 2); break;
    case ORC_PAULIX: memcpy(m, PX, sizeof PX); break;
    case ORC_PAULIY: pauli_y(m); break;
    case ORC_PAULIZ: memcpy(m, PZ, sizeof PZ); break;
    case ORC_HADAMARD: { double h = 1.0 / sqrt(2.0); m[0] = h; m[1] = h; m[2] = h; m[3] = -h; } break;
    case ORC_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; break;
    case ORC_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * M_PI / 4); break;
    case ORC_SX: m[0] = 0.5 * (1 + I); m[1] = 0.5 * (1 - I); m[2] = 0.5 * (1 - I); m[3] = 0.5 * (1 + I); break;
    case ORC_PHASESHIFT: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * a); break;
    case ORC_RX: rot1('X', a, m); break;
    case ORC_RY: rot1('Y', a, m); break;
    case ORC_RZ: rot1('Z', a, m); break;
    case ORC_ROT: /* RZ(omega) RY(theta) RZ(phi) */
        rot1('Z', ang[0], u); rot1('Y', ang[1], v); mat_mul(v, u, u, 2);
        rot1('Z', ang[2], v); mat_mul(v, u, m, 2);
        break;
    case ORC_U3: {
        double th = ang[0], ph = ang[1], la = ang[2];
        m[0] = cos(th / 2); m[1] = -cexp(I * la) * sin(th / 2);
        m[2] = cexp(I * ph) * sin(th / 2); m[3] = cexp(I * (ph + la)) * cos(th / 2);
    } break;
    case ORC_CNOT: controlled2(PX, m); break;
    case ORC_CY: pauli_y(t2); controlled2(t2, m); break;
    case ORC_CZ: controlled2(PZ, m); break;
    case ORC_SWAP: memset(m, 0, sizeof(cplx) * 16); m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[15] = 1; break;
    case ORC_CRX: rot1('X', a, t2); controlled2(t2, m); break;
    case ORC_CRY: rot1('Y', a, t2); controlled2(t2, m); break;
    case ORC_CRZ: rot1('Z', a, t2); controlled2(t2, m); break;
    case ORC_CROT:
        orc_gate_matrix(ORC_ROT, 1, ang, 0, (double *)t2); controlled2(t2, m); break;
    case ORC_CPHASESHIFT: mat_identity(m, 4); m[15] = cexp(I * a); break;
    case ORC_ISINGXX: case ORC_ISINGYY: case ORC_ISINGZZ: {
        /* exp(-i a/2 P(x)P) = cos(a/2) I - i sin(a/2) P(x)P  (Eq. 1 for XX) */
        cplx p[4], pp[16];
        if (gate == ORC_ISINGXX) memcpy(p, PX, sizeof PX);
        else if (gate == ORC_ISINGYY) pauli_y(p);
        else memcpy(p, PZ, sizeof PZ);
        kron2(p, p, pp);
        for (int i = 0; i < 16; ++i) m[i] = -I * sin(a / 2) * pp[i];
        for (int i = 0; i < 4; ++i) m[i * 4 + i] += cos(a / 2);
    } break;
    case ORC_ISINGXY: /* exp(+i a/4 (XX+YY)) */
        mat_identity(m, 4);
        m[1 * 4 + 1] = cos(a / 2); m[1 * 4 + 2] = I * sin(a / 2);
        m[2 * 4 + 1] = I * sin(a / 2); m[2 * 4 + 2] = cos(a / 2);
        break;
    case ORC_SINGLEEXC: /* Givens rotation on {|01>,|10>} */
        mat_identity(m, 4);
        m[1 * 4 + 1] = cos(a / 2); m[1 * 4 + 2] = -sin(a / 2);
        m[2 * 4 + 1] = sin(a / 2); m[2 * 4 + 2] = cos(a / 2);
        break;
    case ORC_TOFFOLI: mat_identity(m, 8); m[6 * 8 + 6] = 0; m[7 * 8 + 7] = 0; m[6 * 8 + 7] = 1; m[7 * 8 + 6] = 1; break;
    case ORC_CSWAP: mat_identity(m, 8); m[5 * 8 + 5] = 0; m[6 * 8 + 6] = 0; m[5 * 8 + 6] = 1; m[6 * 8 + 5] = 1; break;
    case ORC_DOUBLEEXC: /* rotation on {|0011>,|1100>} */
        mat_identity(m, 16);
        m[3 * 16 + 3] = cos(a / 2); m[3 * 16 + 12] = -sin(a / 2);
        m[12 * 16 + 3] = sin(a / 2); m[12 * 16 + 12] = cos(a / 2);
        break;
    case ORC_MULTIRZ: /* exp(-i a/2 Z(x)..(x)Z) */
        memset(m, 0, sizeof(cplx) * (size_t)dim * dim);
        for (int j = 0; j < dim; ++j) {
            int par = __builtin_popcount((unsigned)j) & 1;
            m[j * dim + j] = cexp((par ? I : -I) * a / 2);
        }
        break;
    default:
        return -1;
    }
    if (orc_gate_wires(gate)) dim = 1 << orc_gate_wires(gate);
    if (inverse) mat_dagger(m, dim);
    return 0;
}

/* Generator G and constant c with U(a) = exp(i c a G) for one-angle gates.
 * Returns 0 on success. */
static int gate_generator(int gate, int k, cplx *g, double *c) {
    int dim = 1 << k;
    cplx p[4];
    memset(g, 0, sizeof(cplx) * (size_t)dim * dim);
    switch (gate) {
    case ORC_PHASESHIFT: g[3] = 1; *c = 1.0; return 0;
    case ORC_RX: memcpy(g, PX, sizeof PX); *c = -0.5; return 0;
    case ORC_RY: pauli_y(g); *c = -0.5; return 0;
    case ORC_RZ: memcpy(g, PZ, sizeof PZ); *c = -0.5; return 0;
    case ORC_CRX: case ORC_CRY: case ORC_CRZ:
        if (gate == ORC_CRX) memcpy(p, PX, sizeof PX);
        else if (gate == ORC_CRY) pauli_y(p);
        else memcpy(p, PZ, sizeof PZ);
        g[2 * 4 + 2] = p[0]; g[2 * 4 + 3] = p[1]; g[3 * 4 + 2] = p[2]; g[3 * 4 + 3] = p[3];
        *c = -0.5; return 0;
    case ORC_CPHASESHIFT: g[15] = 1; *c = 1.0; return 0;
    case ORC_ISINGXX: kron2(PX, PX, g); *c = -0.5; return 0;
    case ORC_ISINGYY: pauli_y(p); kron2(p, p, g); *c = -0.5; return 0;
    case ORC_ISINGZZ: kron2(PZ, PZ, g); *c = -0.5; return 0;
    case ORC_ISINGXY: {
        cplx a[16], b[16];
        kron2(PX, PX, a); pauli_y(p); kron2(p, p, b);
        for (int i = 0; i < 16; ++i) g[i] = a[i] + b[i];
        *c = 0.25; return 0;
    }
    case ORC_SINGLEEXC: g[1 * 4 + 2] = -I; g[2 * 4 + 1] = I; *c = -0.5; return 0;
    case ORC_DOUBLEEXC: g[3 * 16 + 12] = -I; g[12 * 16 + 3] = I; *c = -0.5; return 0;
    case ORC_MULTIRZ:
        for (int j = 0; j < dim; ++j) g[j * dim + j] = (__builtin_popcount((unsigned)j) & 1) ? -1.0 : 1.0;
        *c = -0.5; return 0;
    default:
        return -1;
    }
}

/* Exposed for the tests: generator matrix and its constant c. */
int orc_gate_generator(int gate, int k, double *out, double *c) {
    return gate_generator(gate, k, (cplx *)out, c);
}

/* ------------------------------------------------------- apply (plain def.) */

void orc_apply_matrix(int n, double *psi_d, int k, const int32_t *wires, const double *mat_d) {
    cplx *psi = (cplx *)psi_d;
    const cplx *mat = (const cplx *)mat_d;
    const int dim = 1 << k;
    const int64_t N = (int64_t)1 << n;
    int64_t off[1 << MAXK];
    uint64_t wmask = 0;
    for (int j = 0; j < dim; ++j) {
        int64_t o = 0;
        for (int t = 0; t < k; ++t)
            if ((j >> (k - 1 - t)) & 1) o |= (int64_t)1 << (n - 1 - wires[t]);
        off[j] = o;
    }
    for (int t = 0; t < k; ++t) wmask |= (uint64_t)1 << (n - 1 - wires[t]);
#pragma omp parallel
    {
        cplx a[1 << MAXK], b[1 << MAXK];
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            if ((uint64_t)i & wmask) continue;
            for (int j = 0; j < dim; ++j) a[j] = psi[i | off[j]];
            for (int r = 0; r < dim; ++r) {
                cplx s = 0;
                for (int j = 0; j < dim; ++j) s += mat[r * dim + j] * a[j];
                b[r] = s;
            }
            for (int j = 0; j < dim; ++j) psi[i | off[j]] = b[j];
        }
    }
}

/* Embed a k-wire matrix v under m extra controls with required values cv
 * (control 0 is the most significant) into a 2^(m+k) matrix.  The blocks
 * whose control bits differ from cv are `fill` (identity for a unitary, zero
 * for a generator). */
static void embed_controls(const cplx *v, int k, int m, uint32_t ctrl_values, int fill_identity, cplx *out) {
    int dim = 1 << (m + k), vd = 1 << k;
    uint32_t pat = 0;
    for (int j = 0; j < m; ++j) if ((ctrl_values >> j) & 1) pat |= 1u << (m - 1 - j);
    if (fill_identity) mat_identity(out, dim);
    else memset(out, 0, sizeof(cplx) * (size_t)dim * dim);
    for (int r = 0; r < vd; ++r)
        for (int c = 0; c < vd; ++c) {
            int R = (int)(pat << k) | r, C = (int)(pat << k) | c;
            out[R * dim + C] = v[r * vd + c];
        }
}

static int op_angles(const orc_op *op, const double *params, double *ang) {
    int np = orc_gate_nparams(op->gate);
    for (int s = 0; s < np; ++s)
        ang[s] = op->param[s] >= 0 ? op->scale[s] * params[op->param[s]] : op->scale[s];
    return np;
}

static int op_width(const orc_op *op) { return op->n_wires - op->n_ctrls; }

static int check_op(int n, const orc_op *op, int64_t n_params) {
    if (op->gate < 0 || op->gate >= ORC_NUM_GATES) return -1;
    if (op->n_wires < 1 || op->n_wires > 8 || op->n_ctrls < 0 || op->n_ctrls >= op->n_wires) return -1;
    int k = op_width(op), fixed = orc_gate_wires(op->gate);
    if (fixed && k != fixed) return -1;
    if (op->n_wires > MAXK) return -1;
    for (int i = 0; i < op->n_wires; ++i) {
        if (op->wires[i] < 0 || op->wires[i] >= n) return -1;
        for (int j = 0; j < i; ++j) if (op->wires[i] == op->wires[j]) return -1;
    }
    for (int s = 0; s < orc_gate_nparams(op->gate); ++s)
        if (op->param[s] >= n_params) return -1;
    return 0;
}

/* Full matrix of an op over all its wires (controls first). */
static int op_full_matrix(const orc_op *op, const double *params, const double *matrices, cplx *full) {
    int k = op_width(op), vd = 1 << k;
    double ang[3] = {0, 0, 0};
    cplx *v = malloc(sizeof(cplx) * (size_t)vd * vd);
    if (op->gate == ORC_UNITARY) {
        memcpy(v, (const cplx *)matrices + op->matrix_offset, sizeof(cplx) * (size_t)vd * vd);
        if (op->inverse) mat_dagger(v, vd);
    } else {
        op_angles(op, params, ang);
        if (orc_gate_matrix(op->gate, k, ang, op->inverse, (double *)v)) { free(v); return -1; }
    }
    embed_controls(v, k, op->n_ctrls, op->ctrl_values, 1, full);
    free(v);
    return 0;
}

int orc_apply(int n, double *psi, const orc_op *ops, int64_t n_ops, const double *params, const double *matrices) {
    for (int64_t i = 0; i < n_ops; ++i)
        if (check_op(n, &ops[i], 1LL << 40)) return -1;
    for (int64_t i = 0; i < n_ops; ++i) {
        const orc_op *op = &ops[i];
        int dim = 1 << op->n_wires;
        cplx *full = malloc(sizeof(cplx) * (size_t)dim * dim);
        if (op_full_matrix(op, params, matrices, full)) { free(full); return -1; }
        orc_apply_matrix(n, psi, op->n_wires, op->wires, (const double *)full);
        free(full);
    }
    return 0;
}

/* ------------------------------------------------------------ reductions */

static void pairwise(const cplx *a, const cplx *b, int64_t lo, int64_t hi, double *re, double *im) {
    if (hi - lo <= 8) {
        double sr = 0, si = 0;
        for (int64_t i = lo; i < hi; ++i) {
            cplx z = conj(a[i]) * b[i];
            sr += creal(z); si += cimag(z);
        }
        *re = sr; *im = si;
        return;
    }
    int64_t mid = lo + (hi - lo) / 2;
    double r1, i1, r2, i2;
    pairwise(a, b, lo, mid, &r1, &i1);
    pairwise(a, b, mid, hi, &r2, &i2);
    *re = r1 + r2; *im = i1 + i2;
}

static void pairwise_real(const double *x, int64_t lo, int64_t hi, double *out) {
    if (hi - lo <= 8) {
        double s = 0;
        for (int64_t i = lo; i < hi; ++i) s += x[i];
        *out = s;
        return;
    }
    int64_t mid = lo + (hi - lo) / 2;
    double s1, s2;
    pairwise_real(x, lo, mid, &s1);
    pairwise_real(x, mid, hi, &s2);
    *out = s1 + s2;
}

/* Pairwise sum of conj(a_i) b_i over fixed chunks, then pairwise over the
 * chunk sums: the result does not depend on the thread count. */
static void inner(int n, const cplx *a, const cplx *b, double *re, double *im) {
    const int64_t N = (int64_t)1 << n;
    const int64_t CH = 4096;
    int64_t nch = (N + CH - 1) / CH;
    double *pr = malloc(sizeof(double) * (size_t)nch), *pi = malloc(sizeof(double) * (size_t)nch);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t lo = c * CH, hi = lo + CH < N ? lo + CH : N;
        pairwise(a, b, lo, hi, &pr[c], &pi[c]);
    }
    pairwise_real(pr, 0, nch, re);
    pairwise_real(pi, 0, nch, im);
    free(pr); free(pi);
}

void orc_inner(int n, const double *a, const double *b, double *out) {
    inner(n, (const cplx *)a, (const cplx *)b, &out[0], &out[1]);
}

/* ------------------------------------------------------------ observables */

/* out <- P psi for one Pauli word, one letter at a time. */
static int apply_pauli_word(int n, const char *word, cplx *out) {
    for (int w = 0; w < n; ++w) {
        cplx m[4];
        int32_t wire = w;
        switch (word[w]) {
        case 'I': continue;
        case 'X': memcpy(m, PX, sizeof PX); break;
        case 'Y': pauli_y(m); break;
        case 'Z': memcpy(m, PZ, sizeof PZ); break;
        default: return -1;
        }
        orc_apply_matrix(n, (double *)out, 1, &wire, (const double *)m);
    }
    return 0;
}

int orc_expval(int n, const double *psi_d, int n_obs, const int32_t *obs_nterms,
               const double *coeff, const char *paulis, double *out) {
    const cplx *psi = (const cplx *)psi_d;
    const int64_t N = (int64_t)1 << n;
    cplx *tmp = malloc(sizeof(cplx) * (size_t)N);
    int64_t t0 = 0;
    for (int o = 0; o < n_obs; ++o) {
        double acc = 0;
        for (int t = 0; t < obs_nterms[o]; ++t) {
            double re, im;
            memcpy(tmp, psi, sizeof(cplx) * (size_t)N);
            if (apply_pauli_word(n, paulis + (t0 + t) * n, tmp)) { free(tmp); return -1; }
            inner(n, psi, tmp, &re, &im);
            acc += coeff[t0 + t] * re;
        }
        out[o] = acc;
        t0 += obs_nterms[o];
    }
    free(tmp);
    return 0;
}

int orc_apply_pauli_sum(int n, const double *psi_d, int n_terms, const double *coeff,
                        const char *paulis, double *lambda_d) {
    const cplx *psi = (const cplx *)psi_d;
    cplx *lam = (cplx *)lambda_d;
    const int64_t N = (int64_t)1 << n;
    cplx *tmp = malloc(sizeof(cplx) * (size_t)N);
    memset(lam, 0, sizeof(cplx) * (size_t)N);
    for (int t = 0; t < n_terms; ++t) {
        memcpy(tmp, psi, sizeof(cplx) * (size_t)N);
        if (apply_pauli_word(n, paulis + (int64_t)t * n, tmp)) { free(tmp); return -1; }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) lam[i] += coeff[t] * tmp[i];
    }
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------ adjoint */

/* A differentiable factor of an operation: U_s = exp(i c a G) on the op's own
 * wires, angle slot `slot`.  Rot = RZ(omega) RY(theta) RZ(phi) applies
 * RZ(phi) first; U3(theta,phi,lambda) = PhaseShift(phi) RY(theta)
 * PhaseShift(lambda) exactly (no global phase); CRot is the controlled Rot. */
typedef struct { int gate; int slot; } subgate;

static int decompose(int gate, subgate *sub) {
    switch (gate) {
    case ORC_ROT:
        sub[0] = (subgate){ORC_RZ, 0}; sub[1] = (subgate){ORC_RY, 1}; sub[2] = (subgate){ORC_RZ, 2};
        return 3;
    case ORC_U3:
        sub[0] = (subgate){ORC_PHASESHIFT, 2}; sub[1] = (subgate){ORC_RY, 0}; sub[2] = (subgate){ORC_PHASESHIFT, 1};
        return 3;
    case ORC_CROT:
        sub[0] = (subgate){ORC_CRZ, 0}; sub[1] = (subgate){ORC_CRY, 1}; sub[2] = (subgate){ORC_CRZ, 2};
        return 3;
    default:
        if (orc_gate_nparams(gate) == 1) { sub[0] = (subgate){gate, 0}; return 1; }
        return 0;
    }
}

int orc_adjoint_jacobian(int n, const double *psi_d, const orc_op *ops, int64_t n_ops,
                         const double *params, int64_t n_params, const double *matrices,
                         int n_obs, const int32_t *obs_nterms, const double *coeff,
                         const char *paulis, double *jac) {
    const int64_t N = (int64_t)1 << n;
    for (int64_t i = 0; i < n_ops; ++i)
        if (check_op(n, &ops[i], n_params)) return -1;
    cplx *phi = malloc(sizeof(cplx) * (size_t)N);
    cplx *lam = malloc(sizeof(cplx) * (size_t)N);
    cplx *tmp = malloc(sizeof(cplx) * (size_t)N);
    memset(jac, 0, sizeof(double) * (size_t)n_obs * (size_t)n_params);
    int64_t t0 = 0;
    for (int o = 0; o < n_obs; ++o) {
        double *row = jac + (int64_t)o * n_params;
        if (orc_apply_pauli_sum(n, psi_d, obs_nterms[o], coeff + t0, paulis + t0 * n, (double *)lam)) goto fail;
        t0 += obs_nterms[o];
        memcpy(phi, psi_d, sizeof(cplx) * (size_t)N);
        for (int64_t i = n_ops - 1; i >= 0; --i) {
            const orc_op *op = &ops[i];
            subgate sub[3];
            int ns = op->gate == ORC_UNITARY ? 0 : decompose(op->gate, sub);
            int k = op_width(op), m = op->n_ctrls, dim = 1 << op->n_wires, vd = 1 << k;
            cplx *full = malloc(sizeof(cplx) * (size_t)dim * dim);
            cplx *v = malloc(sizeof(cplx) * (size_t)vd * vd);
            if (ns == 0) {
                /* not differentiable: un-apply the whole operation */
                op_full_matrix(op, params, matrices, full);
                mat_dagger(full, dim);
                orc_apply_matrix(n, (double *)phi, op->n_wires, op->wires, (const double *)full);
                orc_apply_matrix(n, (double *)lam, op->n_wires, op->wires, (const double *)full);
            } else {
                double ang[3] = {0, 0, 0};
                op_angles(op, params, ang);
                /* The op's matrix is U_{ns-1}..U_0, or its adjoint
                 * U_0^dag..U_{ns-1}^dag when inverse; the factor applied last
                 * is un-applied first. */
                for (int q = 0; q < ns; ++q) {
                    int idx = op->inverse ? q : ns - 1 - q;
                    subgate s = sub[idx];
                    double a = ang[s.slot], c;
                    if (op->param[s.slot] >= 0) {
                        /* at this point phi = (..U_s) psi0: -2 c Im<lam|G|phi> */
                        gate_generator(s.gate, k, v, &c);
                        if (op->inverse) c = -c;
                        embed_controls(v, k, m, op->ctrl_values, 0, full);
                        memcpy(tmp, phi, sizeof(cplx) * (size_t)N);
                        orc_apply_matrix(n, (double *)tmp, op->n_wires, op->wires, (const double *)full);
                        double re, im;
                        inner(n, lam, tmp, &re, &im);
                        row[op->param[s.slot]] += op->scale[s.slot] * (-2.0 * c * im);
                    }
                    /* un-apply this factor */
                    orc_gate_matrix(s.gate, k, &a, !op->inverse, (double *)v);
                    embed_controls(v, k, m, op->ctrl_values, 1, full);
                    orc_apply_matrix(n, (double *)phi, op->n_wires, op->wires, (const double *)full);
                    orc_apply_matrix(n, (double *)lam, op->n_wires, op->wires, (const double *)full);
                }
            }
            free(full); free(v);
        }
    }
    free(phi); free(lam); free(tmp);
    return 0;
fail:
    free(phi); free(lam); free(tmp);
    return -1;
}

/* ------------------------------------------------------------------ sampling */

int orc_sample(int n, const double *psi, int64_t n_samples, const double *u, int64_t *out) {
    const int64_t N = (int64_t)1 << n;
    double *cdf = (double *)malloc((size_t)N * sizeof(double));
    if (!cdf) return -1;
    double run = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        run += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        cdf[i] = run;
    }
    if (!(run > 0.0)) {
        free(cdf);
        return -1;
    }
    for (int64_t k = 0; k < n_samples; ++k) {
        const double t = u[k] * run;
        int64_t lo = 0, hi = N - 1; /* smallest i with cdf[i] > t (cdf[N-1] = run > t) */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        out[k] = lo;
    }
    free(cdf);
    return 0;
}
