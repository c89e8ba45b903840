"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same seeded inputs.  Sizes span several LDS tiles (small
tile options force many passes, outer controls and ragged plans at small n)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import (TOL, assert_rel_close, assert_state_close, gpu_run, jac_bound, obs_scale,
                               oracle_state, reset_options)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = qsv.Context(0)
    yield c
    c.close()


@pytest.fixture(autouse=True)
def _defaults(ctx):
    reset_options(ctx)
    yield


DTYPES = [qsv.C128, qsv.C64]


# ------------------------------------------------------------------ single gates (streaming kernels)

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("name", sorted(W.GATE_ARITY))
def test_single_gate_every_placement(ctx, name, dt):
    """Each gate alone (its own streaming kernel, or a one-op tile for wide
    gates) on random states, every wire placement on 4 qubits and random
    placements, controls and inverses at larger n."""
    rng = np.random.default_rng(sum(map(ord, name)))
    k, na = W.GATE_ARITY[name]
    cases = []
    kk = k or 3
    for wires in itertools.permutations(range(4), kk):
        cases.append((4, list(wires), 0, False))
    for n in (kk, kk + 1, 7, 12, 15):
        if n < kk:
            continue
        for _ in range(3):
            nc = int(rng.integers(0, min(2, n - kk) + 1))
            wires = list(rng.choice(n, size=kk + nc, replace=False))
            cases.append((n, wires, nc, bool(rng.integers(2))))
    for n, wires, nc, inv in cases:
        slots = [(-1, float(rng.uniform(-4, 4))) for _ in range(na)]
        mat = W.random_unitary(kk, rng) if name == "QubitUnitary" else None
        cv = int(rng.integers(0, 1 << nc)) if nc else -1
        o = W.op(name, wires, *slots, inverse=inv, n_ctrls=nc, ctrl_values=cv, matrix=mat)
        psi0 = W.random_state(n, int(rng.integers(1 << 30)))
        got = gpu_run(ctx, n, [o], [], dt, psi0)
        ref = oracle_state(n, [o], [], psi0)
        assert_state_close(got, ref, TOL[dt], f"{name} n={n} wires={wires} nc={nc} inv={inv}", dt)


# ------------------------------------------------------------------ fused random circuits

TILE_OPTS = [
    {},                                                        # defaults
    {qsv.OPT_TILE_BITS: 5, qsv.OPT_LOW_BITS: 2},               # many small tiles, outer controls
    {qsv.OPT_TILE_BITS: 8, qsv.OPT_LOW_BITS: 3},               # R = 1
    {qsv.OPT_FUSION: 0},                                       # one kernel per gate
    {qsv.OPT_TILE_WS: 1},                                      # warp-specialised tile passes
]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("opt", range(len(TILE_OPTS)))
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (8, 3), (11, 4), (14, 5), (16, 6)])
def test_random_circuit_state(ctx, n, seed, opt, dt):
    c = W.random_circuit(n, 80, seed=1000 + seed, n_params=9, p_ctrl=0.2, max_k=min(n, 5))
    psi0 = W.random_state(n, seed)
    got = gpu_run(ctx, n, c.ops, c.params, dt, psi0, TILE_OPTS[opt])
    ref = oracle_state(n, c.ops, c.params, psi0)
    assert_state_close(got, ref, TOL[dt], f"n={n} seed={seed} opt={opt}", dt)


@pytest.mark.parametrize("n", [3, 9, 13])
def test_wide_tiles_and_large_k(ctx, n):
    """k = 5 and 6 dense unitaries (tile path for k = 6), diagonal MultiRZ of
    every width, many controls."""
    rng = np.random.default_rng(n)
    ops = []
    for _ in range(12):
        k = int(rng.integers(1, min(6, n) + 1))
        wires = list(rng.choice(n, size=k, replace=False))
        ops.append(W.op("QubitUnitary", wires, matrix=W.random_unitary(k, rng)))
        ops.append(W.op("MultiRZ", list(rng.choice(n, size=int(rng.integers(1, min(n, 8) + 1)), replace=False)),
                        (-1, float(rng.uniform(-3, 3)))))
    psi0 = W.random_state(n, 7)
    for opts in ({}, {qsv.OPT_TILE_BITS: 6, qsv.OPT_LOW_BITS: 1}, {qsv.OPT_FUSION: 0}):
        reset_options(ctx)
        got = gpu_run(ctx, n, ops, [], qsv.C128, psi0, opts)
        assert_state_close(got, oracle_state(n, ops, [], psi0), 1e-12, f"n={n} opts={opts}")


def test_ghz_closed_form(ctx):
    for n in (1, 2, 7, 20):
        c = W.ghz(n)
        got = gpu_run(ctx, n, c.ops, c.params)
        want = np.zeros(1 << n, dtype=complex)
        want[0] = want[-1] = 1 / np.sqrt(2)
        if n == 1:
            want = np.array([1, 1]) / np.sqrt(2)
        assert_state_close(got, want, 1e-15, f"GHZ n={n}")


def test_empty_circuit_and_reset(ctx):
    st = qsv.State(ctx, 6)
    qsv.apply(st, [], [])
    ref = np.zeros(64, dtype=complex)
    ref[0] = 1
    assert np.array_equal(st.to_numpy(), ref)
    st.reset(37)
    ref[:] = 0
    ref[37] = 1
    assert np.array_equal(st.to_numpy(), ref)


# ------------------------------------------------------------------ expectation values

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 4, 9, 13, 17])
def test_expval_random_pauli_sums(ctx, n, dt):
    rng = np.random.default_rng(n)
    psi = W.random_state(n, n + 100)
    obs = W.random_observables(n, rng, n_obs=4, n_terms=7)
    obs.append(W.PauliSum(np.array([0.7, -1.3]), ["Z" * n, "Y" * n]))
    st = qsv.State(ctx, n, dt)
    st.from_numpy(psi)
    got = qsv.expval(st, obs)
    ref = oracle.expval(psi.astype(np.complex64).astype(np.complex128) if dt == qsv.C64 else psi, obs)
    assert_rel_close(got, ref, obs_scale(obs), dt, "expval")


# ------------------------------------------------------------------ adjoint Jacobian

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("opt", range(4))
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (4, 2), (7, 3), (10, 4), (13, 5)])
def test_adjoint_random_circuits(ctx, n, seed, opt, dt):
    c = W.random_circuit(n, 50, seed=2000 + seed, n_params=11, p_ctrl=0.2, max_k=min(n, 4))
    obs = W.random_observables(n, np.random.default_rng(seed), n_obs=2, n_terms=4)
    opts = [{}, {qsv.OPT_TILE_BITS_ADJ: 4, qsv.OPT_LOW_BITS: 2}, {qsv.OPT_FUSION: 0}, {qsv.OPT_TILE_WS: 1}][opt]
    for k, v in opts.items():
        ctx.set_option(k, v)
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, c.ops, c.params)
    psi = st.to_numpy()
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, obs)
    np.testing.assert_array_equal(st.to_numpy(), psi)       # state preserved without INPLACE
    # the FP64 oracle on the exact circuit, for both precisions
    ref_psi = oracle.apply(n, c.ops, c.params)
    ref = oracle.adjoint_jacobian(ref_psi, c.ops, c.params, obs)
    bound = jac_bound(c.ops, c.n_params, obs)
    assert_rel_close(jac, ref, bound, dt, "jacobian")
    assert_rel_close(ev, oracle.expval(ref_psi, obs), obs_scale(obs), dt, "expval")
    # VJP with one sweep equals cotangent-weighted rows
    cot = np.array([0.3, -1.7])
    g, _ = qsv.adjoint_vjp(st, c.ops, c.params, obs, cot)
    assert_rel_close(g, cot @ ref, np.abs(cot) @ bound, dt, "vjp")


def test_adjoint_inplace_returns_initial_state(ctx):
    n = 9
    c = W.random_circuit(n, 40, seed=77, n_params=6)
    obs = W.random_observables(n, np.random.default_rng(1), n_obs=1, n_terms=3)
    st = qsv.State(ctx, n)
    qsv.apply(st, c.ops, c.params)
    ref = oracle.adjoint_jacobian(oracle.apply(n, c.ops, c.params), c.ops, c.params, obs)
    jac, _ = qsv.adjoint_jacobian(st, c.ops, c.params, obs, inplace=True)
    assert_rel_close(jac, ref, jac_bound(c.ops, c.n_params, obs), qsv.C128, "jacobian")
    zero = np.zeros(1 << n, dtype=complex)
    zero[0] = 1
    assert_state_close(st.to_numpy(), zero, 1e-12, "state after in-place sweep")


@pytest.mark.parametrize("dt", DTYPES)
def test_config1_jacobian(ctx, dt):
    c = W.config1()
    st = qsv.State(ctx, c.n_qubits, dt)
    qsv.apply(st, c.ops, c.params)
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    psi = oracle.apply(c.n_qubits, c.ops, c.params)
    ref = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)
    assert_rel_close(jac, ref, jac_bound(c.ops, c.n_params, c.observables), dt, "jacobian")
    assert_rel_close(ev, oracle.expval(psi, c.observables), obs_scale(c.observables), dt, "expval")


@pytest.mark.parametrize("n", [8, 12, 16])
@pytest.mark.parametrize("dt", DTYPES)
def test_qaoa_reduced_width(ctx, n, dt):
    """QAOA MaxCut (config-3 generator) at reduced width: the Z-parity phase
    groups and the summed-generator inner products (fused with the rotation
    of the same Z strings inside register groups; at n = 8 the tile is small
    enough that the group sums are flushed after the subcube loop) against
    the oracle's per-gate loop."""
    c = W.config3(n=n)
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, c.ops, c.params)
    psi = oracle.apply(n, c.ops, c.params)
    assert_state_close(st.to_numpy(), psi, TOL[dt], "qaoa state", dt)
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    ref = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)
    assert_rel_close(jac, ref, jac_bound(c.ops, c.n_params, c.observables), dt, "jacobian")
    assert_rel_close(ev, oracle.expval(psi, c.observables), obs_scale(c.observables), dt, "expval")


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("layers", [1, 0])
@pytest.mark.parametrize("n", [8, 13])
def test_adjacent_one_qubit_matrices(ctx, n, layers, dt):
    """Runs of one-qubit gates on one wire (RY, then H S T, a CNOT brick
    between layers): in a register group the matrices that follow each other
    on one position run as their product; state and Jacobian against the
    oracle, with and without one-qubit layers."""
    rng = np.random.default_rng(n)
    ops, k = [], 0
    for _ in range(3):
        for w in range(n):
            ops.append(W.op("RY", [w], (k, 1.0)))
            k += 1
            ops += [W.op("Hadamard", [w]), W.op("S", [w]), W.op("T", [w])]
        for w in range(0, n - 1, 2):
            ops.append(W.op("CNOT", [w, w + 1]))
    params = rng.uniform(-np.pi, np.pi, k)
    obs = [W.PauliSum(np.array([0.7, -0.4]), [W.pauli_word(n, {0: "Z", n - 3: "X"}), W.pauli_word(n, {3: "Y"})])]
    reset_options(ctx)
    ctx.set_option(qsv.OPT_LAYERS, layers)
    try:
        st = qsv.State(ctx, n, dt)
        qsv.apply(st, ops, params)
        psi = oracle.apply(n, ops, params)
        assert_state_close(st.to_numpy(), psi, TOL[dt], "state", dt)
        jac, ev = qsv.adjoint_jacobian(st, ops, params, obs)
        ref = oracle.adjoint_jacobian(psi, ops, params, obs)
        assert_rel_close(jac, ref, jac_bound(ops, k, obs), dt, "jacobian")
        st.close()
    finally:
        reset_options(ctx)


@pytest.mark.parametrize("n", [6, 11])
def test_u3_brickwall_reduced_width(ctx, n):
    c = W.config5(n=n, layers=6)
    st = qsv.State(ctx, n)
    qsv.apply(st, c.ops, c.params)
    psi = oracle.apply(n, c.ops, c.params)
    assert_state_close(st.to_numpy(), psi, 1e-12, "u3 state")
    jac, _ = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    ref = oracle.adjoint_jacobian(psi, c.ops, c.params, c.observables)
    assert_rel_close(jac, ref, jac_bound(c.ops, c.n_params, c.observables), qsv.C128, "jacobian")


def test_torch_tensor_state(ctx):
    import torch
    n = 12
    t = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    t[0] = 1
    torch.cuda.synchronize()
    c = W.random_circuit(n, 30, seed=5, n_params=4)
    st = qsv.State(ctx, n, qsv.C128, tensor=t)
    qsv.apply(st, c.ops, c.params)
    ctx.synchronize()
    np.testing.assert_allclose(t.cpu().numpy(), oracle.apply(n, c.ops, c.params), atol=1e-13)


def test_invalid_call_leaves_state_untouched(ctx):
    n = 5
    st = qsv.State(ctx, n)
    st.from_numpy(W.random_state(n, 3))
    before = st.to_numpy()
    with pytest.raises(qsv.QsvError):
        qsv.apply(st, [W.op("RX", [0], (0, 1.0)), W.op("CNOT", [2, 9])], [0.3])
    with pytest.raises(qsv.QsvError):
        qsv.apply(st, [W.op("RX", [0], (3, 1.0))], [0.3])
    np.testing.assert_array_equal(st.to_numpy(), before)


# ------------------------------------------------------------------ probabilities and variance

@pytest.mark.parametrize("dt", DTYPES)
def test_marginal_probabilities(ctx, dt):
    n = 11
    psi = W.random_state(n, 21)
    st = qsv.State(ctx, n, dt)
    st.from_numpy(psi)
    p = (np.abs(psi.astype(np.complex64).astype(np.complex128) if dt == qsv.C64 else psi) ** 2).reshape([2] * n)
    for wires in ([0], [n - 1], [3, 7], [n - 1, 0, 5], list(range(n)), [9, 1, 4, 2, 10, 0]):
        rest = tuple(w for w in range(n) if w not in wires)
        want = np.transpose(p.sum(axis=rest), np.argsort(np.argsort(wires))).reshape(-1) if rest else \
            np.transpose(p, wires).reshape(-1)
        if rest:
            kept = sorted(wires)
            want = np.transpose(p.sum(axis=rest), [kept.index(w) for w in wires]).reshape(-1)
        got = qsv.probs(st, wires)
        assert_rel_close(got, want, 1.0, dt, f"probs {wires}")


@pytest.mark.parametrize("dt", DTYPES)
def test_variance(ctx, dt):
    n = 9
    psi = W.random_state(n, 5)
    obs = W.random_observables(n, np.random.default_rng(4), n_obs=3, n_terms=6)
    st = qsv.State(ctx, n, dt)
    st.from_numpy(psi)
    ref_psi = psi.astype(np.complex64).astype(np.complex128) if dt == qsv.C64 else psi
    want = []
    for o in obs:
        lam = oracle.apply_pauli_sum(ref_psi, o)
        want.append(np.vdot(lam, lam).real - oracle.expval(ref_psi, [o])[0] ** 2)
    got = qsv.var(st, obs)
    assert_rel_close(got, np.array(want), obs_scale(obs) ** 2, dt, "variance")


@pytest.mark.parametrize("dt", DTYPES)
def test_sparse_hamiltonian_expval(ctx, dt):
    """CSR observable: the Pauli sum's dense matrix in sparse form, and a
    random Hermitian sparse matrix, against plain numpy on the same state."""
    import scipy.sparse as sp
    from tests import dense_ref as D
    n = 8
    psi = W.random_state(n, 8)
    st = qsv.State(ctx, n, dt)
    st.from_numpy(psi)
    ref_psi = psi.astype(np.complex64).astype(np.complex128) if dt == qsv.C64 else psi
    obs = W.random_observables(n, np.random.default_rng(3), n_obs=1, n_terms=5)[0]
    H = sp.csr_matrix(D.pauli_sum_matrix(obs))
    got = qsv.expval_sparse(st, H)
    assert_rel_close(got.real, oracle.expval(ref_psi, [obs])[0], np.sum(np.abs(obs.coeffs)), dt, "sparse pauli")
    rng = np.random.default_rng(1)
    A = sp.random(1 << n, 1 << n, density=0.02, random_state=2) + 1j * sp.random(1 << n, 1 << n, density=0.02,
                                                                                  random_state=3)
    S = (A + A.conj().T).tocsr()
    got = qsv.expval_sparse(st, S)
    want = np.vdot(ref_psi, S @ ref_psi)
    # |<psi|S|psi>| <= ||S||_2 <= max absolute row sum (S Hermitian)
    scale = abs(S).sum(axis=1).max()
    assert_rel_close(got, want, scale, dt, "sparse random (scipy, parity unpinned)")


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
@pytest.mark.parametrize("n", [6, 12, 16])
def test_dense_unitaries_low_and_high_bits(ctx, n, dt):
    """Dense 3- to 6-qubit unitaries on the lowest index bits (3 qubits: one
    lane per amplitude; 6 qubits: the tiled path, one tuple per thread), on
    the highest bits, on mixed bits and with controls; forward and adjoint
    sweeps."""
    rng = np.random.default_rng(40 + n)
    ops = []
    for k in (3, 4, 5, 6):
        if k > n:
            continue
        ops.append(W.op("QubitUnitary", list(range(n - k, n))[::-1], matrix=W.random_unitary(k, rng)))
        ops.append(W.op("QubitUnitary", list(range(k)), matrix=W.random_unitary(k, rng)))
        ops.append(W.op("QubitUnitary", list(rng.choice(n, size=k, replace=False)), matrix=W.random_unitary(k, rng)))
        if k + 1 <= n:
            w = list(rng.choice(n, size=k + 1, replace=False))
            ops.append(W.op("QubitUnitary", w, n_ctrls=1, matrix=W.random_unitary(k, rng)))
        ops.append(W.op("RY", [int(rng.integers(n))], (0, 1.0)))
    params = np.array([0.37])
    psi0 = W.random_state(n, 3)
    for opts in ({}, {qsv.OPT_TILE_BITS: 10}, {qsv.OPT_DENSE_MFMA: 1}):
        reset_options(ctx)
        got = gpu_run(ctx, n, ops, params, dt, psi0, opts)
        assert_state_close(got, oracle_state(n, ops, params, psi0), TOL[dt], f"n={n} opts={opts}", dt)
    reset_options(ctx)
    # adjoint through the same unitaries (un-applied in the two-vector pass)
    obs = [W.PauliSum(np.array([0.8, -0.3]), [W.pauli_word(n, {0: "Z"}), W.pauli_word(n, {n - 1: "X"})])]
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, ops, params)
    jac, _ = qsv.adjoint_jacobian(st, ops, params, obs)
    psi = oracle.apply(n, ops, params)
    want = oracle.adjoint_jacobian(psi, ops, params, obs)
    assert_rel_close(jac, want, jac_bound(ops, len(params), obs), dt, "jacobian")
    st.close()


@pytest.mark.parametrize("dt", DTYPES)
def test_deep_narrow_adjoint_many_slots(ctx, dt):
    """10 qubits, 40 layers of RX/RY/RZ (1200 trainable slots): the planner
    closes passes before their slot accumulators outgrow the CU's LDS."""
    n, ops, p = 10, [], 0
    for _ in range(40):
        for q in range(n):
            for g in ("RX", "RY", "RZ"):
                ops.append(W.op(g, [q], (p, 1.0)))
                p += 1
    params = np.random.default_rng(5).uniform(0, 2 * np.pi, p)
    obs = [W.PauliSum(np.array([0.6, -0.4]), [W.pauli_word(n, {0: "Z"}), W.pauli_word(n, {3: "X", 7: "Y"})])]
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, ops, params)
    psi = oracle.apply(n, ops, params)
    assert_state_close(st.to_numpy(), psi, TOL[dt], "state", dt)
    jac, ev = qsv.adjoint_jacobian(st, ops, params, obs)
    assert_rel_close(jac, oracle.adjoint_jacobian(psi, ops, params, obs), jac_bound(ops, p, obs), dt, "jacobian")
    assert_rel_close(ev, oracle.expval(psi, obs), obs_scale(obs), dt, "expval")
    st.close()


@pytest.mark.parametrize("gate", ["RX", "RY"])
@pytest.mark.parametrize("dt", DTYPES)
def test_factored_layers(ctx, gate, dt):
    """RX / RY layers on the factored kernel classes (one FMA per component,
    the factors carried as the pass's scale), at angles that need either form
    (cos(a/2) = 0 at a = pi, sin = 0 at a = 0), with the default and with
    narrow tiles; forward states and adjoint gradients against the oracle."""
    n = 12
    angles = [0.0, np.pi, 0.3, 2.5, 4.0, 5.9]
    ops = []
    for rep in range(4):
        for q in range(n):
            ops.append(W.op(gate, [q], ((q + rep) % len(angles), 1.0)))
        ops.append(W.op("CNOT", [rep % n, (rep + 5) % n]))
    params = np.array(angles)
    obs = W.random_observables(n, np.random.default_rng(7), n_obs=1, n_terms=4)
    psi = oracle.apply(n, ops, params)
    want = oracle.adjoint_jacobian(psi, ops, params, obs)
    for opts in ({}, {qsv.OPT_TILE_BITS: 7, qsv.OPT_TILE_BITS_ADJ: 7}):
        reset_options(ctx)
        for k, v in opts.items():
            ctx.set_option(k, v)
        st = qsv.State(ctx, n, dt)
        qsv.apply(st, ops, params)
        assert_state_close(st.to_numpy(), psi, TOL[dt], f"state opts={opts}", dt)
        jac, ev = qsv.adjoint_jacobian(st, ops, params, obs)
        assert_rel_close(jac, want, jac_bound(ops, len(angles), obs), dt, f"jacobian opts={opts}")
        st.close()
    reset_options(ctx)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("inplace", [False, True])
def test_uniform_z_sum_lambda_in_first_pass(ctx, dt, inplace):
    """An observable that is c times a sum of Z strings (diagonal, one
    coefficient) takes the path where the first reverse pass forms lambda
    from the loaded phi and sums <H> itself; gradients and <H> against the
    oracle, with and without the in-place sweep, plus a non-uniform sum (the
    separate lambda pass) on the same circuit."""
    n = 14
    c = W.random_circuit(n, 60, seed=21, n_params=6)
    rng = np.random.default_rng(3)
    words = []
    for _ in range(9):
        q = rng.choice(n, size=int(rng.integers(1, 4)), replace=False)
        words.append(W.pauli_word(n, {int(x): "Z" for x in q}))
    for coeffs in (np.full(9, -0.7), rng.normal(size=9)):
        obs = [W.PauliSum(coeffs, words)]
        reset_options(ctx)
        st = qsv.State(ctx, n, dt)
        qsv.apply(st, c.ops, c.params)
        psi = oracle.apply(n, c.ops, c.params)
        jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, obs, inplace=inplace)
        assert_rel_close(jac, oracle.adjoint_jacobian(psi, c.ops, c.params, obs),
                         jac_bound(c.ops, c.n_params, obs), dt, f"jacobian uniform={coeffs[0] == coeffs[1]}")
        assert_rel_close(ev, oracle.expval(psi, obs), obs_scale(obs), dt, f"expval uniform={coeffs[0] == coeffs[1]}")
        if inplace:  # the in-place sweep hands back the initial state
            assert_state_close(st.to_numpy(), oracle.zero_state(n), TOL[dt], "initial state", dt)
        st.close()
