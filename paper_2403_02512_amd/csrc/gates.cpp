// Host-side gate model: every operation becomes one or more factors, each a
// small matrix on its target wires under control wires, built in FP64 on the
// host (paper Sec. 2.2: gate matrices live on the device, built once per call)
// together with the generator data the adjoint sweep needs.
//
// Gate definitions (paper Sec. 2.1.2 lists the set; Eq. 1 fixes IsingXX):
//   RX/RY/RZ(a)       exp(-i a/2 P)                 generator P,       c = -1/2
//   PhaseShift(a)     diag(1, e^{ia})                generator |1><1|,  c = 1
//   Rot(f, t, w)      RZ(w) RY(t) RZ(f)
//   U3(t, f, l)       PhaseShift(f) RY(t) PhaseShift(l)   (exact, no global phase)
//   CRX/CRY/CRZ/CRot  controlled forms (control = first own wire)
//   IsingXX/YY/ZZ(a)  exp(-i a/2 P(x)P)              generator P(x)P,   c = -1/2
//   IsingXY(a)        exp(+i a/4 (XX+YY))           generator XX+YY,   c = 1/4
//   SingleExcitation  rotation by a/2 in span{|01>,|10>}: exp(-i a/2 G), G = Y there
//   DoubleExcitation  the same in span{|0011>,|1100>}
//   MultiRZ(a)        exp(-i a/2 Z(x)..(x)Z)
// An op's derivative: U = exp(i c a G) with a = scale * params[p] gives
// d<H>/dparams[p] += scale * (-2c) Im<lambda|G|phi> at the point just after U.
#include <cmath>
#include <stdexcept>

#include "qsv_internal.h"

namespace qsv {
namespace {

using Mat = std::vector<cd>;
const cd J(0.0, 1.0);

Mat ident(int dim) {
    Mat m((size_t)dim * dim, 0.0);
    for (int i = 0; i < dim; ++i) m[(size_t)i * dim + i] = 1.0;
    return m;
}

Mat dag(const Mat& m, int dim) {
    Mat o((size_t)dim * dim);
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) o[(size_t)c * dim + r] = std::conj(m[(size_t)r * dim + c]);
    return o;
}

Mat mul(const Mat& a, const Mat& b, int dim) {
    Mat o((size_t)dim * dim, 0.0);
    for (int r = 0; r < dim; ++r)
        for (int j = 0; j < dim; ++j)
            for (int c = 0; c < dim; ++c) o[(size_t)r * dim + c] += a[(size_t)r * dim + j] * b[(size_t)j * dim + c];
    return o;
}

Mat kron(const Mat& a, int da, const Mat& b, int db) {
    const int d = da * db;
    Mat o((size_t)d * d);
    for (int r1 = 0; r1 < da; ++r1)
        for (int c1 = 0; c1 < da; ++c1)
            for (int r2 = 0; r2 < db; ++r2)
                for (int c2 = 0; c2 < db; ++c2)
                    o[(size_t)(r1 * db + r2) * d + (c1 * db + c2)] = a[(size_t)r1 * da + c1] * b[(size_t)r2 * db + c2];
    return o;
}

const Mat PX = {0.0, 1.0, 1.0, 0.0};
const Mat PY = {0.0, -J, J, 0.0};
const Mat PZ = {1.0, 0.0, 0.0, -1.0};
const Mat P1 = {0.0, 0.0, 0.0, 1.0};  // |1><1|

// exp(i c a G) for a Hermitian G with G^2 = I: cos(ca) I + i sin(ca) G
Mat exp_involution(const Mat& g, int dim, double ca) {
    Mat o = ident(dim);
    for (size_t i = 0; i < o.size(); ++i) o[i] = o[i] * std::cos(ca) + J * std::sin(ca) * g[i];
    return o;
}

// exp(i c a G) for a projector G (G^2 = G): I + (e^{ica} - 1) G
Mat exp_projector(const Mat& g, int dim, double ca) {
    Mat o = ident(dim);
    const cd f = std::exp(J * ca) - 1.0;
    for (size_t i = 0; i < o.size(); ++i) o[i] += f * g[i];
    return o;
}

// generator of a rotation in a 2-dim subspace {|u>,|v>} of a dim-dim space:
// -i|u><v| + i|v><u| (the Pauli Y of that subspace)
Mat sub_y(int dim, int u, int v) {
    Mat g((size_t)dim * dim, 0.0);
    g[(size_t)u * dim + v] = -J;
    g[(size_t)v * dim + u] = J;
    return g;
}

// exp(i c a G) for G = Y on a subspace and 0 elsewhere (G^3 = G)
Mat exp_sub(const Mat& g, int dim, double ca, int u, int v) {
    Mat o = ident(dim);
    Mat e = exp_involution(g, dim, ca);
    o[(size_t)u * dim + u] = e[(size_t)u * dim + u];
    o[(size_t)u * dim + v] = e[(size_t)u * dim + v];
    o[(size_t)v * dim + u] = e[(size_t)v * dim + u];
    o[(size_t)v * dim + v] = e[(size_t)v * dim + v];
    return o;
}

Mat zstring(int k) {
    const int dim = 1 << k;
    Mat g((size_t)dim * dim, 0.0);
    for (int j = 0; j < dim; ++j) g[(size_t)j * dim + j] = (__builtin_popcount((unsigned)j) & 1) ? -1.0 : 1.0;
    return g;
}

// One-angle rotation: matrix builder data.
struct Rot1 {
    Mat g;             // generator on the targets
    double c;          // U = exp(i c a G)
    enum { INV, PROJ, SUBY } kind;
    int u = 0, v = 0;  // SUBY subspace
};

Rot1 rotation_of(int gate, int k) {
    switch (gate) {
    case QSV_GATE_RX: case QSV_GATE_CRX: return {PX, -0.5, Rot1::INV};
    case QSV_GATE_RY: case QSV_GATE_CRY: return {PY, -0.5, Rot1::INV};
    case QSV_GATE_RZ: case QSV_GATE_CRZ: return {PZ, -0.5, Rot1::INV};
    case QSV_GATE_PHASESHIFT: case QSV_GATE_CPHASESHIFT: return {P1, 1.0, Rot1::PROJ};
    case QSV_GATE_ISINGXX: return {kron(PX, 2, PX, 2), -0.5, Rot1::INV};
    case QSV_GATE_ISINGYY: return {kron(PY, 2, PY, 2), -0.5, Rot1::INV};
    case QSV_GATE_ISINGZZ: return {kron(PZ, 2, PZ, 2), -0.5, Rot1::INV};
    case QSV_GATE_MULTIRZ: return {zstring(k), -0.5, Rot1::INV};
    case QSV_GATE_ISINGXY: {
        // XX + YY = 2 (|01><10| + |10><01|): exp(i a/4 (XX+YY)) rotates
        // span{|01>,|10>} by exp(i a/2 sigma_x); G^3 = 4G, handled as SUBY
        // with generator 2*sigma_x in the subspace
        Mat g = kron(PX, 2, PX, 2);
        Mat yy = kron(PY, 2, PY, 2);
        for (size_t i = 0; i < g.size(); ++i) g[i] += yy[i];
        return {g, 0.25, Rot1::SUBY, 1, 2};
    }
    case QSV_GATE_SINGLEEXC: return {sub_y(4, 1, 2), -0.5, Rot1::SUBY, 1, 2};
    case QSV_GATE_DOUBLEEXC: return {sub_y(16, 3, 12), -0.5, Rot1::SUBY, 3, 12};
    default: throw std::logic_error("not a one-angle rotation");
    }
}

Mat rotation_matrix(const Rot1& r, int dim, double a) {
    const double ca = r.c * a;
    if (r.kind == Rot1::INV) return exp_involution(r.g, dim, ca);
    if (r.kind == Rot1::PROJ) return exp_projector(r.g, dim, ca);
    // subspace generator with eigenvalues +-s on the subspace (s = 2 for XX+YY)
    const cd guv = r.g[(size_t)r.u * dim + r.v];
    const double s = std::abs(guv);
    Mat gn = r.g;
    for (auto& x : gn) x /= s;
    return exp_sub(gn, dim, ca * s, r.u, r.v);
}

void set_targets(Factor& f, const int* w, int k) {
    f.k = k;
    for (int i = 0; i < k; ++i) f.tw[i] = w[i];
}

void add_control(Factor& f, int wire, int value) {
    f.cw[f.nc] = wire;
    f.cv[f.nc] = value;
    ++f.nc;
}

}  // namespace

int gate_own_wires(int gate) {
    switch (gate) {
    case QSV_GATE_PAULIX: case QSV_GATE_PAULIY: case QSV_GATE_PAULIZ: case QSV_GATE_HADAMARD:
    case QSV_GATE_S: case QSV_GATE_T: case QSV_GATE_SX: case QSV_GATE_IDENTITY:
    case QSV_GATE_PHASESHIFT: case QSV_GATE_RX: case QSV_GATE_RY: case QSV_GATE_RZ:
    case QSV_GATE_ROT: case QSV_GATE_U3:
        return 1;
    case QSV_GATE_CNOT: case QSV_GATE_CY: case QSV_GATE_CZ: case QSV_GATE_SWAP:
    case QSV_GATE_CRX: case QSV_GATE_CRY: case QSV_GATE_CRZ: case QSV_GATE_CROT: case QSV_GATE_CPHASESHIFT:
    case QSV_GATE_ISINGXX: case QSV_GATE_ISINGYY: case QSV_GATE_ISINGZZ: case QSV_GATE_ISINGXY:
    case QSV_GATE_SINGLEEXC:
        return 2;
    case QSV_GATE_TOFFOLI: case QSV_GATE_CSWAP:
        return 3;
    case QSV_GATE_DOUBLEEXC:
        return 4;
    case QSV_GATE_MULTIRZ: case QSV_GATE_UNITARY:
        return 0;
    default:
        return -1;
    }
}

int gate_n_angles(int gate) {
    switch (gate) {
    case QSV_GATE_ROT: case QSV_GATE_U3: case QSV_GATE_CROT:
        return 3;
    case QSV_GATE_PHASESHIFT: case QSV_GATE_RX: case QSV_GATE_RY: case QSV_GATE_RZ:
    case QSV_GATE_CRX: case QSV_GATE_CRY: case QSV_GATE_CRZ: case QSV_GATE_CPHASESHIFT:
    case QSV_GATE_ISINGXX: case QSV_GATE_ISINGYY: case QSV_GATE_ISINGZZ: case QSV_GATE_ISINGXY:
    case QSV_GATE_SINGLEEXC: case QSV_GATE_DOUBLEEXC: case QSV_GATE_MULTIRZ:
        return 1;
    default:
        return 0;
    }
}

void op_factors(const qsv_op& op, const double* params, const double* matrices, bool decompose,
                std::vector<Factor>& out) {
    const int nc = op.n_ctrls;
    const int* own = op.wires + nc;
    const int nown = op.n_wires - nc;
    double ang[3] = {0, 0, 0};
    const int na = gate_n_angles(op.gate);
    for (int s = 0; s < na; ++s) ang[s] = op.param[s] >= 0 ? op.scale[s] * params[op.param[s]] : op.scale[s];

    Factor base;
    for (int j = 0; j < nc; ++j) add_control(base, op.wires[j], (op.ctrl_values >> j) & 1);

    // list of (matrix builder) factors in application order, before inverse
    struct Sub {
        Mat m;
        int k;
        int slot;        // angle slot differentiated, -1 none
        Mat g;           // generator
        double c = 0.0;
        bool zrot = false;
        double zangle = 0.0;
    };
    std::vector<Sub> subs;
    int k = nown;
    const int* tgt = own;
    int own_ctrl = 0;  // leading own wires that are controls

    auto rot_sub = [&](int gate, int kk, int slot, double a) {
        Rot1 r = rotation_of(gate, kk);
        Sub s;
        s.k = kk;
        s.m = rotation_matrix(r, 1 << kk, a);
        s.slot = slot;
        s.g = r.g;
        s.c = r.c;
        s.zrot = (gate == QSV_GATE_RZ || gate == QSV_GATE_ISINGZZ || gate == QSV_GATE_MULTIRZ);
        s.zangle = a;
        return s;
    };
    auto fixed_sub = [&](Mat m, int kk) {
        Sub s;
        s.k = kk;
        s.m = std::move(m);
        s.slot = -1;
        return s;
    };
    // Rot(f, t, w) = RZ(w) RY(t) RZ(f); U3(t, f, l) = PhaseShift(f) RY(t) PhaseShift(l)
    auto euler_subs = [&](int gate) {
        std::vector<Sub> v;
        if (gate == QSV_GATE_U3) {
            v.push_back(rot_sub(QSV_GATE_PHASESHIFT, 1, 2, ang[2]));
            v.push_back(rot_sub(QSV_GATE_RY, 1, 0, ang[0]));
            v.push_back(rot_sub(QSV_GATE_PHASESHIFT, 1, 1, ang[1]));
        } else {
            v.push_back(rot_sub(QSV_GATE_RZ, 1, 0, ang[0]));
            v.push_back(rot_sub(QSV_GATE_RY, 1, 1, ang[1]));
            v.push_back(rot_sub(QSV_GATE_RZ, 1, 2, ang[2]));
        }
        return v;
    };
    const double s2 = 1.0 / std::sqrt(2.0);

    switch (op.gate) {
    case QSV_GATE_PAULIX: subs.push_back(fixed_sub(PX, 1)); break;
    case QSV_GATE_PAULIY: subs.push_back(fixed_sub(PY, 1)); break;
    case QSV_GATE_PAULIZ: subs.push_back(fixed_sub(PZ, 1)); break;
    case QSV_GATE_IDENTITY: subs.push_back(fixed_sub(ident(2), 1)); break;
    case QSV_GATE_HADAMARD: subs.push_back(fixed_sub({s2, s2, s2, -s2}, 1)); break;
    case QSV_GATE_S: subs.push_back(fixed_sub({1.0, 0.0, 0.0, J}, 1)); break;
    case QSV_GATE_T: subs.push_back(fixed_sub({1.0, 0.0, 0.0, std::exp(J * (M_PI / 4))}, 1)); break;
    case QSV_GATE_SX: {
        const cd p(0.5, 0.5), m(0.5, -0.5);
        subs.push_back(fixed_sub({p, m, m, p}, 1));
    } break;
    case QSV_GATE_PHASESHIFT: case QSV_GATE_RX: case QSV_GATE_RY: case QSV_GATE_RZ:
        subs.push_back(rot_sub(op.gate, 1, 0, ang[0]));
        break;
    case QSV_GATE_ROT: case QSV_GATE_U3: subs = euler_subs(op.gate); break;
    case QSV_GATE_CNOT: own_ctrl = 1; subs.push_back(fixed_sub(PX, 1)); break;
    case QSV_GATE_CY: own_ctrl = 1; subs.push_back(fixed_sub(PY, 1)); break;
    case QSV_GATE_CZ: own_ctrl = 1; subs.push_back(fixed_sub(PZ, 1)); break;
    case QSV_GATE_SWAP: subs.push_back(fixed_sub({1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1}, 2)); break;
    case QSV_GATE_CRX: case QSV_GATE_CRY: case QSV_GATE_CRZ: case QSV_GATE_CPHASESHIFT:
        own_ctrl = 1;
        subs.push_back(rot_sub(op.gate, 1, 0, ang[0]));
        subs.back().zrot = false;
        break;
    case QSV_GATE_CROT: own_ctrl = 1; subs = euler_subs(QSV_GATE_ROT); break;
    case QSV_GATE_ISINGXX: case QSV_GATE_ISINGYY: case QSV_GATE_ISINGZZ: case QSV_GATE_ISINGXY:
    case QSV_GATE_SINGLEEXC:
        subs.push_back(rot_sub(op.gate, 2, 0, ang[0]));
        break;
    case QSV_GATE_TOFFOLI: own_ctrl = 2; subs.push_back(fixed_sub(PX, 1)); break;
    case QSV_GATE_CSWAP:
        own_ctrl = 1;
        subs.push_back(fixed_sub({1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1}, 2));
        break;
    case QSV_GATE_DOUBLEEXC: subs.push_back(rot_sub(op.gate, 4, 0, ang[0])); break;
    case QSV_GATE_MULTIRZ: subs.push_back(rot_sub(op.gate, nown, 0, ang[0])); break;
    case QSV_GATE_UNITARY: {
        const int d = 1 << nown;
        Mat m((size_t)d * d);
        const double* src = matrices + 2 * op.matrix_offset;
        for (size_t i = 0; i < m.size(); ++i) m[i] = cd(src[2 * i], src[2 * i + 1]);
        subs.push_back(fixed_sub(std::move(m), nown));
    } break;
    default:
        throw std::invalid_argument("unknown gate");
    }
    for (int j = 0; j < own_ctrl; ++j) add_control(base, own[j], 1);
    tgt = own + own_ctrl;
    k = nown - own_ctrl;

    if (!decompose && subs.size() > 1) {
        // one factor with the product matrix (applied first = rightmost)
        Mat m = subs[0].m;
        for (size_t i = 1; i < subs.size(); ++i) m = mul(subs[i].m, m, 1 << k);
        Sub s = fixed_sub(m, k);
        subs.assign(1, s);
    }
    const bool inv = op.inverse != 0;
    const int ns = (int)subs.size();
    for (int q = 0; q < ns; ++q) {
        const Sub& s = subs[inv ? ns - 1 - q : q];
        Factor f = base;
        set_targets(f, tgt, k);
        f.m = inv ? dag(s.m, 1 << k) : s.m;
        f.src_op = -1;
        if (decompose && s.slot >= 0 && op.param[s.slot] >= 0) {
            f.has_dot = true;
            f.param = op.param[s.slot];
            const double c = inv ? -s.c : s.c;
            f.coef = op.scale[s.slot] * (-2.0 * c);
            f.g = s.g;
        }
        if (s.zrot && f.nc == 0) {
            f.zrot = true;
            f.zangle = inv ? -s.zangle : s.zangle;
            if (op.param[s.slot] >= 0) {
                f.zparam = op.param[s.slot];
                f.zscale = inv ? -op.scale[s.slot] : op.scale[s.slot];
            }
        }
        out.push_back(std::move(f));
    }
}

}  // namespace qsv
