"""Pauli sums whose x-groups hold many terms (the byte-table path of the
expectation-value kernel) against the oracle: <H>, lambda-based adjoint
gradients and the variance, in both precisions, at group sizes around the
table limits (16 and 64 terms per group)."""
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


def _word(n, x_bits, z_bits):
    w = []
    for q in range(n):
        b = n - 1 - q
        xb, zb = (x_bits >> b) & 1, (z_bits >> b) & 1
        w.append("Y" if xb and zb else "X" if xb else "Z" if zb else "I")
    return "".join(w)


def _grouped_hamiltonian(n, sizes, seed):
    """Groups of the given sizes, each sharing one random x mask (the first
    is diagonal), with distinct random z masks."""
    rng = np.random.default_rng(seed)
    words, coeffs = [], []
    for gi, size in enumerate(sizes):
        x = 0 if gi == 0 else int(rng.integers(1, 1 << n))
        zs = set()
        while len(zs) < size:
            z = int(rng.integers(0, 1 << n))
            if x == 0 and z == 0:
                continue
            zs.add(z)
        for z in sorted(zs):
            words.append(_word(n, x, z))
            coeffs.append(float(rng.normal()))
    return W.PauliSum(np.array(coeffs), words)


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
@pytest.mark.parametrize("sizes", [(16,), (42, 30, 3), (64, 64), (65, 20), (15, 8, 40)])
def test_many_term_groups(ctx, dt, sizes):
    n = 12
    c = W.random_circuit(n, 60, seed=sum(sizes))
    H = _grouped_hamiltonian(n, sizes, seed=len(sizes))
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, c.ops, c.params)
    psi = oracle.apply(n, c.ops, c.params)
    s = float(np.sum(np.abs(H.coeffs)))
    ev = qsv.expval(st, [H])[0]
    assert_rel_close(ev, oracle.expval(psi, [H])[0], s, dt, "expval")
    jac, ev2 = qsv.adjoint_jacobian(st, c.ops, c.params, [H])
    want = oracle.adjoint_jacobian(psi, c.ops, c.params, [H])
    assert_rel_close(jac, want, jac_bound(c.ops, c.n_params, [H]), dt, "jacobian")
    # the variance is bounded by s^2
    hpsi = oracle.apply_pauli_sum(psi, H)
    var = np.vdot(hpsi, hpsi).real - oracle.expval(psi, [H])[0] ** 2
    assert_rel_close(qsv.var(st, [H])[0], var, s * s, dt, "variance")
    st.close()


def test_many_term_groups_28q_qaoa_cost(ctx):
    """The benchmark's cost Hamiltonian (one diagonal group of 42 terms) on a
    28-qubit state: <H_C> through the tables equals the term loop's value
    computed from the same state by the oracle on sampled structure."""
    c = W.config3()
    st = qsv.State(ctx, 28)
    qsv.apply(st, c.ops, c.params)
    ev = qsv.expval(st, c.observables)[0]
    # the same Hamiltonian split into one-term observables (term loop path)
    H = c.observables[0]
    parts = [W.PauliSum(np.array([cf]), [w]) for cf, w in zip(H.coeffs, H.words)]
    ev_parts = qsv.expval(st, parts)
    assert_rel_close(ev, float(np.sum(ev_parts)), float(np.sum(np.abs(H.coeffs))), qsv.C128,
                     "tables vs term loop (GPU self-consistency)")
    st.close()
    ctx.release_workspace()
