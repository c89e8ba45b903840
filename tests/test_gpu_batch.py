"""Batched circuits (qsv_batch_*): every circuit's expectation value and
adjoint gradient against the oracle, eager and through the captured HIP
graph, including replays with new parameters."""
import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import assert_rel_close, jac_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = qsv.Context(0)
    yield c
    c.close()


def _mixed_batch(seed=0):
    """Uneven widths and gate mixes: VQE-like circuits, random circuits with
    many-qubit gates and unitaries, a circuit with no gates, a 1-qubit one."""
    rng = np.random.default_rng(seed)
    cs = [W.vqe_circuit(n, rng, n_terms=12) for n in (3, 7, 12, 13)]
    for n in (5, 9, 14):
        c = W.random_circuit(n, 40, seed=seed + n)
        c.observables = [W.random_pauli_sum(n, 6, rng)]
        cs.append(c)
    cs.append(W.Circuit(4, [], np.zeros(0), [W.random_pauli_sum(4, 5, rng)], "empty"))
    cs.append(W.Circuit(1, [W.op("RX", [0], (0, 1.0)), W.op("RY", [0], (1, 0.5))], rng.uniform(0, 6, 2),
                        [W.PauliSum(np.array([0.7, -0.2]), ["Z", "X"])], "one"))
    return cs


def _oracle(c, params):
    psi = oracle.apply(c.n_qubits, c.ops, params)
    ev = oracle.expval(psi, c.observables[:1])[0]
    jac = oracle.adjoint_jacobian(psi, c.ops, params, c.observables[:1])[0] if c.n_params else np.zeros(0)
    return ev, jac


def _check(cs, params, ev, grads, dt):
    for i, c in enumerate(cs):
        want_ev, want_j = _oracle(c, params[i])
        s = float(np.sum(np.abs(c.observables[0].coeffs)))
        assert_rel_close(ev[i], want_ev, s, dt, f"expval circuit {i} ({c.name})")
        if grads is not None and c.n_params:
            bound = jac_bound(c.ops, c.n_params, c.observables[:1])[0]
            assert_rel_close(grads[i], want_j, bound, dt, f"gradient circuit {i} ({c.name})")


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(ctx, dt, graph):
    cs = _mixed_batch()
    b = qsv.Batch(ctx, cs, dt)
    rng = np.random.default_rng(1)
    for rep in range(3):   # graph: capture once, then replays with new angles
        params = [c.params if rep == 0 else rng.uniform(0, 2 * np.pi, c.n_params) for c in cs]
        ev, grads = b.run(params, grad=True, graph=graph)
        _check(cs, params, ev, grads, dt)
        ev2, none = b.run(params, grad=False, graph=graph)
        assert none is None
        _check(cs, params, ev2, None, dt)
    b.close()


def test_batch_matches_single_circuit_path(ctx):
    """The batched launches give the per-circuit entry points' results."""
    cs = W.config4(n_circuits=16, n_min=10, n_max=16, n_terms=40)
    b = qsv.Batch(ctx, cs)
    ev, grads = b.run([c.params for c in cs], graph=True)
    for i, c in enumerate(cs):
        st = qsv.State(ctx, c.n_qubits)
        qsv.apply(st, c.ops, c.params)
        jac, e1 = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
        st.close()
        s = float(np.sum(np.abs(c.observables[0].coeffs)))
        assert_rel_close(ev[i], e1[0], s, qsv.C128, "batched vs single expval")
        bound = jac_bound(c.ops, c.n_params, c.observables)[0]
        assert_rel_close(grads[i], jac[0], bound, qsv.C128, "batched vs single gradient")
    b.close()


def test_batch_rejects_bad_input(ctx):
    c = W.vqe_circuit(4, np.random.default_rng(0), n_terms=3)
    bad = W.Circuit(4, [W.op("RX", [6], (0, 1.0))], np.zeros(1), c.observables)
    with pytest.raises(qsv.QsvError):
        qsv.Batch(ctx, [c, bad])
    b = qsv.Batch(ctx, [c])
    with pytest.raises(ValueError):
        b.run([np.zeros(c.n_params + 1)])
    b.close()


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
def test_batch_many_term_groups(ctx, dt):
    """Batched circuits whose Hamiltonians have x-groups of many terms: the
    batched Pauli kernel evaluates them through the per-circuit byte tables
    (one circuit with two table groups, one with one, one with none)."""
    from tests.test_gpu_pauli import _grouped_hamiltonian
    cs = []
    for n, sizes in ((10, (42, 30, 3)), (12, (16, 5)), (8, (7, 9, 2))):
        c = W.random_circuit(n, 40, seed=n)
        c.observables = [_grouped_hamiltonian(n, sizes, seed=n)]
        cs.append(c)
    b = qsv.Batch(ctx, cs, dt)
    for graph in (False, True):
        ev, grads = b.run([c.params for c in cs], grad=True, graph=graph)
        _check(cs, [c.params for c in cs], ev, grads, dt)
    b.close()
