"""CPU checks of planning and lowering: the lowered device program (passes,
tile ops, register groups, Z-parity tables, inner-product slots), run by the
CPU model in program_emulator.py, against the oracle.  No GPU needed."""
import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.program_emulator import emulate_adjoint, emulate_apply

OPTS = [{}, {"tile_bits": 5, "low_bits": 2}, {"tile_bits": 4, "low_bits": 1}, {"fusion": False}, {"fusion": 2}]


@pytest.mark.parametrize("opt", range(len(OPTS)))
@pytest.mark.parametrize("n,seed", [(2, 0), (5, 1), (7, 2), (9, 3)])
def test_forward_program(n, seed, opt):
    c = W.random_circuit(n, 40, seed=500 + seed, n_params=6, p_ctrl=0.25, max_k=min(n, 4))
    psi0 = W.random_state(n, seed)
    got = emulate_apply(n, c.ops, c.params, psi0, **OPTS[opt])
    np.testing.assert_allclose(got, oracle.apply(n, c.ops, c.params, psi=psi0), atol=1e-12)


@pytest.mark.parametrize("opt", range(len(OPTS)))
@pytest.mark.parametrize("n,seed", [(2, 0), (5, 1), (7, 2), (9, 3)])
def test_adjoint_program(n, seed, opt):
    c = W.random_circuit(n, 30, seed=600 + seed, n_params=5, p_ctrl=0.25, max_k=min(n, 4))
    obs = W.random_observables(n, np.random.default_rng(seed), n_obs=1, n_terms=3)
    psi = oracle.apply(n, c.ops, c.params)
    lam = oracle.apply_pauli_sum(psi, obs[0])
    g, phi = emulate_adjoint(n, c.ops, c.params, psi, lam, **OPTS[opt])
    np.testing.assert_allclose(g, oracle.adjoint_jacobian(psi, c.ops, c.params, obs)[0], atol=1e-11)
    np.testing.assert_allclose(phi, oracle.zero_state(n), atol=1e-12)   # the sweep un-applies everything


@pytest.mark.parametrize("n", [8, 10])
def test_qaoa_program(n):
    c = W.config3(n=n)
    psi = oracle.apply(n, c.ops, c.params)
    np.testing.assert_allclose(emulate_apply(n, c.ops, c.params, oracle.zero_state(n)), psi, atol=1e-12)
    lam = oracle.apply_pauli_sum(psi, c.observables[0])
    for opts in ({}, {"tile_bits": 6, "low_bits": 2}):
        g, _ = emulate_adjoint(n, c.ops, c.params, psi, lam, **opts)
        np.testing.assert_allclose(g, oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)[0], atol=1e-11)


@pytest.mark.parametrize("opt", [{}, {"fusion": 2}])
def test_layers_with_mixed_generators(opt):
    """Layers whose inner products mix X-, Y- and dense generators (RX next
    to RY and Rot/U3 factors) keep their generator class (regression: a mixed
    layer was once encoded as having no inner products)."""
    n = 8
    c = W.random_circuit(n, 40, seed=9, n_params=6,
                         gates=["RX", "RY", "RZ", "CNOT", "IsingXX", "CRY", "Rot", "U3", "SingleExcitation"])
    obs = W.random_observables(n, np.random.default_rng(2), n_obs=2, n_terms=3)
    psi = oracle.apply(n, c.ops, c.params)
    want = oracle.adjoint_jacobian(psi, c.ops, c.params, obs)
    for o in range(2):
        g, _ = emulate_adjoint(n, c.ops, c.params, psi, oracle.apply_pauli_sum(psi, obs[o]), **opt)
        np.testing.assert_allclose(g, want[o], atol=1e-11)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("where", ["low", "high", "mixed", "controlled"])
def test_dense_kernel_lowering(k, where):
    """Dense k-qubit unitaries through the LDS-staged kernel's index
    arithmetic (targets on the lowest bits, the highest, scattered, and with
    controls on low and high bits, which must stay outside the tile)."""
    n = k + 7 if where != "controlled" else k + 9
    rng = np.random.default_rng(10 * k + len(where))
    if where == "low":
        wires, nc = [n - 1 - b for b in range(k)], 0
    elif where == "high":
        wires, nc = list(range(k))[::-1], 0
    elif where == "mixed":
        wires, nc = [int(w) for w in rng.choice(n, size=k, replace=False)], 0
    else:
        wires, nc = [n - 1, 0] + [int(w) for w in rng.choice(range(1, n - 1), size=k, replace=False)], 2
    o = W.op("QubitUnitary", wires, n_ctrls=nc, ctrl_values=2 if nc else -1, matrix=W.random_unitary(k, rng))
    psi0 = W.random_state(n, k)
    from paper_2403_02512_amd import qsv
    prog = qsv.plan_json(n, [o], [])
    assert [st["type"] for st in prog["steps"]] == ["dense"]
    got = emulate_apply(n, [o], [], psi0)
    np.testing.assert_allclose(got, oracle.apply(n, [o], [], psi=psi0), atol=1e-12)


@pytest.mark.parametrize("opts", [{}, {"tile_bits": 6, "low_bits": 2}, {"tile_bits": 5, "low_bits": 1}])
def test_u3_brickwall_adjoint_program(opts):
    """U3 layers and CNOT bricks (the 32-qubit benchmark circuit's shape): in
    the reverse sweep the phase factors of each U3 run as one-qubit matrices
    inside register layers when their wire is a tile bit, and through the
    global-index diagonal path otherwise."""
    n = 9
    c = W.config5(n=n, layers=3)
    psi = oracle.apply(n, c.ops, c.params)
    lam = oracle.apply_pauli_sum(psi, c.observables[0])
    g, phi = emulate_adjoint(n, c.ops, c.params, psi, lam, **opts)
    np.testing.assert_allclose(g, oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)[0], atol=1e-11)
    np.testing.assert_allclose(phi, oracle.zero_state(n), atol=1e-12)


@pytest.mark.parametrize("gate", ["RX", "RY"])
def test_factored_layers(gate):
    """RX / RY layers run in the factored classes (matrices divided by their
    diagonal or off-diagonal entry, the factors carried as the pass's scale
    and undone at write-back and in the slot coefficients), at angles where
    either form is the one that applies (cos(a/2) = 0 at a = pi, sin = 0 at
    a = 0), forward and adjoint."""
    from paper_2403_02512_amd import qsv
    n = 6
    angles = [0.0, np.pi, 0.3, 2.5, 4.0, 5.9]
    ops = []
    for rep in range(3):
        for q in range(n):
            ops.append(W.op(gate, [q], ((q + rep) % len(angles), 1.0)))
        ops.append(W.op("CNOT", [rep % n, (rep + 1) % n]))
    params = np.array(angles)
    obs = W.random_observables(n, np.random.default_rng(7), n_obs=1, n_terms=4)
    psi0 = W.random_state(n, 4)
    got = emulate_apply(n, ops, params, psi0, tile_bits=6, low_bits=2)
    np.testing.assert_allclose(got, oracle.apply(n, ops, params, psi=psi0), atol=1e-12)
    psi = oracle.apply(n, ops, params)
    g, phi = emulate_adjoint(n, ops, params, psi, oracle.apply_pauli_sum(psi, obs[0]), tile_bits=6, low_bits=2)
    np.testing.assert_allclose(g, oracle.adjoint_jacobian(psi, ops, params, obs)[0], atol=1e-11)
    np.testing.assert_allclose(phi, oracle.zero_state(n), atol=1e-12)
    # both factored forms occur in the lowered programs
    classes = set()
    for adj in (False, True):
        pj = qsv.plan_json(n, ops, params, adjoint=adj, tile_bits=6, low_bits=2)
        classes |= {o["cls"] for o in pj["tops"] if o["kind"] == 12}
    d, o = (8, 9) if gate == "RX" else (10, 11)
    assert d in classes and o in classes, classes


def _same_wire_runs(n=8, layers=3, seed=7):
    rng = np.random.default_rng(seed)
    ops, k = [], 0
    for _ in range(layers):
        for w in range(n):
            ops.append(W.op("RY", [w], (k, 1.0)))
            k += 1
            ops += [W.op("Hadamard", [w]), W.op("S", [w]), W.op("T", [w])]
        for w in range(0, n - 1, 2):
            ops.append(W.op("CNOT", [w, w + 1]))
    return ops, rng.uniform(-np.pi, np.pi, k)


@pytest.mark.parametrize("opts", [{}, {"tile_bits": 6, "low_bits": 2}, {"fusion": 2}])
def test_adjacent_one_qubit_matrices_merge(opts):
    """One-qubit matrices that follow each other on one position of a
    register group, with the same controls and nothing between them, are
    lowered as one matrix (their product, the earlier acting first)."""
    n = 8
    ops, params = _same_wire_runs(n)
    obs = [W.PauliSum(np.array([0.7, -0.4]), [W.pauli_word(n, {0: "Z", 5: "X"}), W.pauli_word(n, {3: "Y"})])]
    psi = oracle.apply(n, ops, params)
    np.testing.assert_allclose(emulate_apply(n, ops, params, oracle.zero_state(n), **opts), psi, atol=1e-12)
    lam = oracle.apply_pauli_sum(psi, obs[0])
    g, phi = emulate_adjoint(n, ops, params, psi, lam, **opts)
    np.testing.assert_allclose(g, oracle.adjoint_jacobian(psi, ops, params, obs)[0], atol=1e-11)
    np.testing.assert_allclose(phi, oracle.zero_state(n), atol=1e-12)
    if opts.get("fusion") == 2:
        # without layers every one-qubit gate would be its own sub-op: the
        # runs H S T of each wire become one matrix (with RY before them)
        fwd = qsv.plan_json(n, ops, params, **opts)
        n1 = sum(t["kind"] == 1 for t in fwd["tops"])
        assert n1 < sum(o.name in ("Hadamard", "S", "T") for o in ops)
