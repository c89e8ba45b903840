"""Pins of the plain CPU oracle against what the paper and the mathematics fix.

No test here compares the oracle with itself: gate matrices are checked
against the matrices the paper prints (Eq. 1, Listing 1) and against
exp(i c theta G) built from Kronecker products of Pauli matrices; gate
application against brute-force dense 2^n x 2^n operators; expectation values
against dense Pauli-word matrices and closed forms; the adjoint Jacobian
against per-slot shift rules (trigonometric interpolation) and finite
differences, which use only the forward pass.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import workloads as W
from tests import dense_ref as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_op(o, params, n):
    """Dense operator of one op built from the oracle's small gate matrix,
    with controls, inverse and wire placement done independently here."""
    k = len(o.wires) - o.n_ctrls
    ang = [o.scale[s] * params[o.param[s]] if o.param[s] >= 0 else o.scale[s] for s in range(len(o.param))]
    if o.name == "QubitUnitary":
        v = np.asarray(o.matrix)
    else:
        v = oracle.gate_matrix(o.name, ang, inverse=False, k=k)
    if o.inverse:
        v = v.conj().T
    if o.n_ctrls:
        cv = o.ctrl_values if o.ctrl_values >= 0 else (1 << o.n_ctrls) - 1
        bits = tuple((cv >> j) & 1 for j in range(o.n_ctrls))
        v = D.controlled(v, o.n_ctrls, bits)
    return D.embed(v, list(o.wires), n)


def dense_run(c):
    psi = np.zeros(1 << c.n_qubits, dtype=complex)
    psi[0] = 1
    for o in c.ops:
        psi = dense_op(o, c.params, c.n_qubits) @ psi
    return psi


# ------------------------------------------------------------ gate matrices

def _parse_eq1(phi):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "isingxx_eq1.txt")) if l.strip() and not l.startswith("#")]
    val = {"c": math.cos(phi / 2), "-is": -1j * math.sin(phi / 2), "0": 0.0}
    return np.array([[val[t] for t in r] for r in rows], dtype=complex)


@pytest.mark.parametrize("phi", [0.0, 0.37, -1.2, 2.9, 6.1])
def test_isingxx_matches_eq1(phi):
    """Sec. 2.1.2, Eq. 1: IsingXX printed entry by entry."""
    np.testing.assert_allclose(oracle.gate_matrix("IsingXX", [phi]), _parse_eq1(phi), atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("IsingXX", [phi]), D.expm(-0.5j * phi * np.kron(D.X, D.X)),
                               atol=1e-14)


def test_listing1_paulix_and_phaseshift():
    """Listing 1: PauliX swaps the pair; PhaseShift multiplies only the |1>
    amplitude by e^{i angle} (e^{-i angle} when inverse)."""
    a = np.array([0.3 + 0.1j, -0.2 + 0.7j])
    np.testing.assert_array_equal(oracle.gate_matrix("PauliX") @ a, a[::-1])
    for ang in (0.4, -2.2):
        out = oracle.gate_matrix("PhaseShift", [ang]) @ a
        assert out[0] == a[0]
        assert abs(out[1] - a[1] * np.exp(1j * ang)) < 1e-15
        out = oracle.gate_matrix("PhaseShift", [ang], inverse=True) @ a
        assert abs(out[1] - a[1] * np.exp(-1j * ang)) < 1e-15


# generator definitions G and constants c with U(t) = exp(i c t G), written
# from the gates' definitions as Pauli products
XX, YY, ZZ = np.kron(D.X, D.X), np.kron(D.Y, D.Y), np.kron(D.Z, D.Z)
_SUB01 = np.zeros((4, 4), complex); _SUB01[1, 2] = -1j; _SUB01[2, 1] = 1j
_SUB0011 = np.zeros((16, 16), complex); _SUB0011[3, 12] = -1j; _SUB0011[12, 3] = 1j
GENERATORS = {
    "RX": (D.X, -0.5), "RY": (D.Y, -0.5), "RZ": (D.Z, -0.5), "PhaseShift": (D.P1, 1.0),
    "CRX": (np.kron(D.P1, D.X), -0.5), "CRY": (np.kron(D.P1, D.Y), -0.5), "CRZ": (np.kron(D.P1, D.Z), -0.5),
    "ControlledPhaseShift": (np.kron(D.P1, D.P1), 1.0),
    "IsingXX": (XX, -0.5), "IsingYY": (YY, -0.5), "IsingZZ": (ZZ, -0.5), "IsingXY": (XX + YY, 0.25),
    "SingleExcitation": (_SUB01, -0.5), "DoubleExcitation": (_SUB0011, -0.5),
}


@pytest.mark.parametrize("name", sorted(GENERATORS))
@pytest.mark.parametrize("t", [0.0, 0.81, -2.3, 4.4])
def test_parametric_gate_is_exp_of_generator(name, t):
    g, c = GENERATORS[name]
    np.testing.assert_allclose(oracle.gate_matrix(name, [t]), D.expm(1j * c * t * g), atol=1e-14)
    og, oc = oracle.gate_generator(name)
    np.testing.assert_allclose(og, g, atol=0)
    assert oc == c
    # inverse is the adjoint, i.e. the negated angle for one-angle gates
    np.testing.assert_allclose(oracle.gate_matrix(name, [t], inverse=True), D.expm(-1j * c * t * g), atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_multirz(k):
    zs = D.kron(*([D.Z] * k))
    for t in (0.3, -1.7):
        np.testing.assert_allclose(oracle.gate_matrix("MultiRZ", [t], k=k), D.expm(-0.5j * t * zs), atol=1e-14)


def test_fixed_gates():
    s2 = 1 / math.sqrt(2)
    np.testing.assert_allclose(oracle.gate_matrix("Hadamard"), s2 * np.array([[1, 1], [1, -1]]), atol=1e-16)
    np.testing.assert_allclose(oracle.gate_matrix("PauliY"), D.Y)
    np.testing.assert_allclose(oracle.gate_matrix("PauliZ"), D.Z)
    np.testing.assert_allclose(oracle.gate_matrix("S"), np.diag([1, 1j]))
    np.testing.assert_allclose(oracle.gate_matrix("T") @ oracle.gate_matrix("T"), np.diag([1, 1j]), atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("SX") @ oracle.gate_matrix("SX"), D.X, atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("CNOT"), D.controlled(D.X, 1))
    np.testing.assert_allclose(oracle.gate_matrix("CY"), D.controlled(D.Y, 1))
    np.testing.assert_allclose(oracle.gate_matrix("CZ"), np.diag([1, 1, 1, -1]))
    swap = D.permutation_matrix(2, [1, 0])
    np.testing.assert_allclose(oracle.gate_matrix("SWAP"), swap)
    np.testing.assert_allclose(oracle.gate_matrix("Toffoli"), D.controlled(D.X, 2))
    np.testing.assert_allclose(oracle.gate_matrix("CSWAP"), D.controlled(swap, 1))


@pytest.mark.parametrize("a", [(0.3, -1.1, 2.2), (4.0, 0.5, -0.7)])
def test_rot_u3_crot_decompositions(a):
    rz = lambda t: D.expm(-0.5j * t * D.Z)
    ry = lambda t: D.expm(-0.5j * t * D.Y)
    ps = lambda t: np.diag([1, np.exp(1j * t)])
    phi, th, om = a
    rot = rz(om) @ ry(th) @ rz(phi)
    np.testing.assert_allclose(oracle.gate_matrix("Rot", a), rot, atol=1e-14)
    np.testing.assert_allclose(oracle.gate_matrix("CRot", a), D.controlled(rot, 1), atol=1e-14)
    th, ph, la = a
    u3 = oracle.gate_matrix("U3", a)
    # U3 is PhaseShift(phi) RY(theta) PhaseShift(lambda) exactly, and equals
    # RZ(phi) RY(theta) RZ(lambda) up to the global phase e^{i(phi+lambda)/2}
    np.testing.assert_allclose(u3, ps(ph) @ ry(th) @ ps(la), atol=1e-14)
    np.testing.assert_allclose(u3, np.exp(0.5j * (ph + la)) * rz(ph) @ ry(th) @ rz(la), atol=1e-14)
    np.testing.assert_allclose(oracle.gate_matrix("U3", a, inverse=True), u3.conj().T, atol=1e-15)


# ------------------------------------------------------------ application

@pytest.mark.parametrize("seed", range(12))
def test_apply_matches_dense_unitaries(seed):
    n = 2 + seed % 5
    c = W.random_circuit(n, 25, seed=100 + seed, p_ctrl=0.3)
    np.testing.assert_allclose(oracle.apply(n, c.ops, c.params), dense_run(c), atol=1e-13)


@pytest.mark.parametrize("name", sorted(W.GATE_ARITY))
def test_every_gate_every_placement(name):
    """Each gate on every ordered wire placement of a 4-qubit register."""
    import itertools
    n = 4
    k, na = W.GATE_ARITY[name]
    k = k or 3
    rng = np.random.default_rng(7)
    psi0 = W.random_state(n, 11)
    for wires in itertools.permutations(range(n), k):
        slots = [(-1, float(rng.uniform(-3, 3))) for _ in range(na)]
        mat = W.random_unitary(k, rng) if name == "QubitUnitary" else None
        o = W.op(name, wires, *slots, matrix=mat)
        out = oracle.apply(n, [o], [], psi=psi0)
        ref = dense_op(o, [], n) @ psi0
        np.testing.assert_allclose(out, ref, atol=1e-14)


def _alg1_pairs(n, q):
    """Alg. 1 index enumeration (mask_low read as 0 when q_offset = 0)."""
    off = n - q - 1
    stride = 1 << off
    mask_high = (~0 << (off + 1)) & ((1 << 64) - 1)
    mask_low = ((1 << 64) - 1) >> (64 - off) if off > 0 else 0
    return [(((2 * k) & mask_high) | (mask_low & k), (((2 * k) & mask_high) | (mask_low & k)) | stride)
            for k in range(1 << (n - 1))]


def _alg2_pairs(n, q, ctrls):
    """Alg. 2 as read: i0 = k & masks[0]; masks from the sorted offsets of
    controls and target; the shift loop runs over all n_ctrls+1 upper masks."""
    offs = sorted([n - c - 1 for c in ctrls] + [n - q - 1])
    masks = [(1 << offs[0]) - 1]
    for i in range(1, len(offs)):
        masks.append(((1 << offs[i]) - 1) & ~((1 << (offs[i - 1] + 1)) - 1))
    masks.append(~((1 << (offs[-1] + 1)) - 1) & ((1 << n) - 1))
    ctrl_strides = [1 << (n - c - 1) for c in ctrls]
    pairs = []
    for k in range(1 << (n - 1 - len(ctrls))):
        i0 = k & masks[0]
        for i in range(1, len(ctrls) + 2):
            i0 |= (k << i) & masks[i]
        for s in ctrl_strides:
            i0 |= s
        pairs.append((i0, i0 | (1 << (n - q - 1))))
    return pairs


@pytest.mark.parametrize("n", [1, 2, 5, 7])
def test_alg1_enumerates_each_pair_once(n):
    for q in range(n):
        pairs = _alg1_pairs(n, q)
        bit = 1 << (n - 1 - q)
        want = sorted((i, i | bit) for i in range(1 << n) if not i & bit)
        assert sorted(pairs) == want


@pytest.mark.parametrize("n,q,ctrls", [(5, 2, [0, 4]), (5, 0, [1]), (6, 5, [0, 2, 3]), (4, 1, [3]), (7, 3, [6, 0])])
def test_alg2_enumerates_controlled_pairs(n, q, ctrls):
    pairs = _alg2_pairs(n, q, ctrls)
    cm = sum(1 << (n - 1 - c) for c in ctrls)
    bit = 1 << (n - 1 - q)
    want = sorted((i, i | bit) for i in range(1 << n) if not i & bit and i & cm == cm)
    assert len(pairs) == 1 << (n - 1 - len(ctrls))
    assert sorted(pairs) == want


# ------------------------------------------------------------ expectation values

@pytest.mark.parametrize("seed", range(6))
def test_expval_matches_dense_pauli_sums(seed):
    n = 1 + seed
    rng = np.random.default_rng(seed)
    psi = W.random_state(n, seed)
    obs = W.random_observables(n, rng, n_obs=3, n_terms=4)
    got = oracle.expval(psi, obs)
    for o, g in zip(obs, got):
        assert abs(g - np.vdot(psi, D.pauli_sum_matrix(o) @ psi).real) < 1e-14
    lam = oracle.apply_pauli_sum(psi, obs[0])
    np.testing.assert_allclose(lam, D.pauli_sum_matrix(obs[0]) @ psi, atol=1e-14)


def _ev(n, ops, params, letters):
    psi = oracle.apply(n, ops, params)
    return oracle.expval(psi, [W.PauliSum(np.array([1.0]), [W.pauli_word(n, letters)])])[0]


@pytest.mark.parametrize("t", [0.0, 0.5, 1.9, -2.7, math.pi])
def test_closed_forms_single_qubit(t):
    rx = [W.op("RX", [0], (0, 1.0))]
    assert abs(_ev(1, rx, [t], {0: "Z"}) - math.cos(t)) < 1e-15
    assert abs(_ev(1, rx, [t], {0: "Y"}) + math.sin(t)) < 1e-15   # fixes the sign of RX
    assert abs(_ev(1, rx, [t], {0: "X"})) < 1e-15
    hp = [W.op("Hadamard", [0]), W.op("PhaseShift", [0], (0, 1.0))]
    assert abs(_ev(1, hp, [t], {0: "X"}) - math.cos(t)) < 1e-15
    assert abs(_ev(1, hp, [t], {0: "Y"}) - math.sin(t)) < 1e-15


def test_closed_form_ry_rx_and_gradient():
    a, b = 0.7, -1.3
    ops = [W.op("RX", [0], (0, 1.0)), W.op("RY", [0], (1, 1.0))]
    psi = oracle.apply(1, ops, [a, b])
    obs = [W.PauliSum(np.array([1.0]), ["Z"])]
    assert abs(oracle.expval(psi, obs)[0] - math.cos(a) * math.cos(b)) < 1e-15
    jac = oracle.adjoint_jacobian(psi, ops, [a, b], obs)
    np.testing.assert_allclose(jac[0], [-math.sin(a) * math.cos(b), -math.cos(a) * math.sin(b)], atol=1e-15)


def test_bell_state():
    ops = [W.op("Hadamard", [0]), W.op("CNOT", [0, 1])]
    for letters, want in (({0: "Z", 1: "Z"}, 1), ({0: "X", 1: "X"}, 1), ({0: "Y", 1: "Y"}, -1), ({0: "Z"}, 0)):
        assert abs(_ev(2, ops, [], letters) - want) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 5, 8, 11])
def test_ghz_closed_forms(n):
    c = W.ghz(n)
    psi = oracle.apply(n, c.ops, c.params)
    ev = lambda d: oracle.expval(psi, [W.PauliSum(np.array([1.0]), [W.pauli_word(n, d)])])[0]
    assert abs(ev({0: "Z", n - 1: "Z"}) - 1) < 1e-14
    assert abs(ev({w: "X" for w in range(n)}) - 1) < 1e-14
    assert abs(ev({w: "Y" for w in range(n)}) - math.cos(n * math.pi / 2)) < 1e-14
    if n >= 3:
        # Listing 3: probabilities on wires [0, n//2, n-1]
        rows = [l.split() for l in open(os.path.join(GOLDEN, "ghz_probs_listing3.txt")) if not l.startswith("#")]
        want = np.array([float(r[1]) for r in rows])
        p = (np.abs(psi) ** 2).reshape([2] * n)
        keep = [0, n // 2, n - 1]
        marg = p.sum(axis=tuple(w for w in range(n) if w not in keep)).reshape(-1)
        np.testing.assert_allclose(marg, want, atol=1e-15)


@pytest.mark.parametrize("g,b", [(0.3, 0.7), (1.1, -0.4), (2.5, 1.9)])
def test_qaoa_single_edge(g, b):
    """p=1 QAOA on one edge: <Z0 Z1> = sin(2 beta) sin(gamma)."""
    ops = [W.op("Hadamard", [0]), W.op("Hadamard", [1]), W.op("IsingZZ", [0, 1], (0, 1.0)),
           W.op("RX", [0], (1, 1.0)), W.op("RX", [1], (1, 1.0))]
    psi = oracle.apply(2, ops, [g, b])
    obs = [W.PauliSum(np.array([1.0]), ["ZZ"])]
    assert abs(oracle.expval(psi, obs)[0] - math.sin(2 * b) * math.sin(g)) < 1e-14
    jac = oracle.adjoint_jacobian(psi, ops, [g, b], obs)[0]
    np.testing.assert_allclose(jac, [math.sin(2 * b) * math.cos(g), 2 * math.cos(2 * b) * math.sin(g)], atol=1e-14)


def test_norm_preserved_and_mirror():
    c = W.random_circuit(6, 60, seed=5)
    psi = oracle.apply(6, c.ops, c.params)
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    mirror = [W.Op(o.name, o.wires, o.param, o.scale, not o.inverse, o.n_ctrls, o.ctrl_values, o.matrix)
              for o in reversed(c.ops)]
    back = oracle.apply(6, mirror, c.params, psi=psi)
    np.testing.assert_allclose(back, oracle.zero_state(6), atol=1e-13)


def test_inner_product_summation_accuracy():
    """|+>^n: <X..X> = 1 exactly; the oracle's pairwise sums stay within
    a few ulps at 2^20 terms, and match math.fsum."""
    n = 20
    ops = [W.op("Hadamard", [q]) for q in range(n)]
    psi = oracle.apply(n, ops, [])
    ev = oracle.expval(psi, [W.PauliSum(np.array([1.0]), ["X" * n])])[0]
    assert abs(ev - 1) < 1e-14
    rng = np.random.default_rng(0)
    a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    b = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    z = oracle.inner(a, b)
    prod = np.conj(a) * b
    assert abs(z.real - math.fsum(prod.real)) < 1e-11
    assert abs(z.imag - math.fsum(prod.imag)) < 1e-11


# ------------------------------------------------------------ adjoint Jacobian

def _with_slot(ops, i, s, angle):
    o = ops[i]
    param = list(o.param); scale = list(o.scale)
    param[s] = -1; scale[s] = angle
    out = list(ops)
    out[i] = W.Op(o.name, o.wires, tuple(param), tuple(scale), o.inverse, o.n_ctrls, o.ctrl_values, o.matrix)
    return out


def shift_rule_jacobian(c, obs):
    """Per-slot exact shift rule: each slot's angle enters f as a trigonometric
    polynomial with frequencies {1/2, 1}; five equispaced samples over the
    4 pi period fix it exactly, and its derivative at the slot's angle times
    the slot's scale is the slot's contribution."""
    n = c.n_qubits
    jac = np.zeros((len(obs), c.n_params))
    for i, o in enumerate(c.ops):
        for s, p in enumerate(o.param):
            if p < 0:
                continue
            a0 = o.scale[s] * c.params[p]
            ts = a0 + 4 * np.pi * np.arange(5) / 5
            A = np.stack([np.ones(5), np.cos(ts / 2), np.sin(ts / 2), np.cos(ts), np.sin(ts)], 1)
            f = np.stack([oracle.expval(oracle.apply(n, _with_slot(c.ops, i, s, t), c.params), obs) for t in ts])
            coef = np.linalg.solve(A, f)
            d = (-0.5 * coef[1] * np.sin(a0 / 2) + 0.5 * coef[2] * np.cos(a0 / 2)
                 - coef[3] * np.sin(a0) + coef[4] * np.cos(a0))
            jac[:, p] += o.scale[s] * d
    return jac


def fd_jacobian(c, obs, h=1e-3):
    n = c.n_qubits
    jac = np.zeros((len(obs), c.n_params))
    for p in range(c.n_params):
        def f(dt):
            q = c.params.copy(); q[p] += dt
            return oracle.expval(oracle.apply(n, c.ops, q), obs)
        jac[:, p] = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
    return jac


@pytest.mark.parametrize("seed", range(10))
def test_adjoint_matches_shift_rule(seed):
    n = 2 + seed % 4
    c = W.random_circuit(n, 18, seed=300 + seed, n_params=7, p_ctrl=0.25)
    obs = W.random_observables(n, np.random.default_rng(seed), n_obs=2, n_terms=3)
    psi = oracle.apply(n, c.ops, c.params)
    jac = oracle.adjoint_jacobian(psi, c.ops, c.params, obs)
    np.testing.assert_allclose(jac, shift_rule_jacobian(c, obs), atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_adjoint_matches_finite_differences(seed):
    n = 3
    c = W.random_circuit(n, 14, seed=400 + seed, n_params=5)
    obs = W.random_observables(n, np.random.default_rng(seed), n_obs=1, n_terms=4)
    psi = oracle.apply(n, c.ops, c.params)
    np.testing.assert_allclose(oracle.adjoint_jacobian(psi, c.ops, c.params, obs), fd_jacobian(c, obs), atol=1e-10)


def test_adjoint_config1_small():
    c = W.config1()
    psi = oracle.apply(c.n_qubits, c.ops, c.params)
    jac = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)
    rng = np.random.default_rng(0)
    for p in rng.choice(c.n_params, 6, replace=False):
        def f(dt):
            q = c.params.copy(); q[p] += dt
            return oracle.expval(oracle.apply(c.n_qubits, c.ops, q), c.observables)[0]
        ps = (f(np.pi / 2) - f(-np.pi / 2)) / 2     # RX/RY/RZ: exact two-term rule
        assert abs(jac[0, p] - ps) < 1e-13


def test_last_rz_before_diagonal_observable_has_zero_gradient():
    c = W.config5(n=6, layers=2)
    psi = oracle.apply(6, c.ops, c.params)
    jac = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)[0]
    # U3(theta, phi, lambda) = PhaseShift(phi) RY PhaseShift(lambda): the phi
    # slots of the last layer sit just before a diagonal observable
    last = [o for o in c.ops if o.name == "U3"][-6:]
    for o in last:
        assert abs(jac[o.param[1]]) < 1e-15


# ------------------------------------------------------------------ sampling (Sec. 4.3 shots)

def test_sample_basis_state_and_ghz_closed_forms():
    for b in (0, 5, 7):
        psi = oracle.zero_state(3, b)
        assert np.all(oracle.sample(psi, [0.0, 0.3, 0.999]) == b)
    g = W.ghz(3)
    psi = oracle.apply(3, g.ops, g.params)
    # p_0 = p_7 = 1/2, nothing in between: u < 1/2 -> 0, u >= 1/2 -> 7
    assert list(oracle.sample(psi, [0.0, 0.25, 0.4999999, 0.5, 0.75, 0.9999])) == [0, 0, 0, 7, 7, 7]


def test_sample_product_state_thresholds():
    """RY product state: p(i) = prod_w p_w(bit of wire w), wire 0 = msb; every
    u strictly inside [C(i-1), C(i)) maps to i (C from the closed form)."""
    th = [0.7, 2.1, 1.3]
    ops = [W.op("RY", [w], (w, 1.0)) for w in range(3)]
    psi = oracle.apply(3, ops, np.array(th))
    p1 = [math.sin(t / 2) ** 2 for t in th]
    probs = []
    for i in range(8):
        pr = 1.0
        for w in range(3):
            bit = (i >> (2 - w)) & 1
            pr *= p1[w] if bit else 1 - p1[w]
        probs.append(pr)
    C = np.cumsum(probs)
    lo = np.concatenate([[0.0], C[:-1]])
    mids = (lo + C) / 2
    assert list(oracle.sample(psi, mids)) == list(range(8))
    # just inside both ends of each interval
    eps = 1e-9
    assert list(oracle.sample(psi, lo + eps)) == list(range(8))
    assert list(oracle.sample(psi, C - eps)) == list(range(8))


def test_sample_frequencies_match_probabilities():
    c = W.random_circuit(4, 30, seed=11)
    psi = oracle.apply(4, c.ops, c.params)
    p = np.abs(psi) ** 2
    u = np.random.default_rng(0).random(40000)
    counts = np.bincount(oracle.sample(psi, u), minlength=16) / u.size
    assert np.all(np.abs(counts - p) <= 5 * np.sqrt(p * (1 - p) / u.size) + 1e-12)
