"""Full-size GPU cases, in the launch configuration the benchmark times.

* 28-qubit QAOA (the benchmark workload) and the 20-qubit ansatz: against
  values the oracle wrote (tests/golden/make_golden.py), including sampled
  amplitudes of the 28-qubit state; complex64 error reported against them.
* 32-qubit complex128 and 33-qubit complex64 layered U3 circuits: no host
  oracle fits, so properties that hold at any size pin them: product circuits
  factorise into one-qubit oracle runs, mirror circuits return to |0..0>,
  GHZ closed forms, norm preservation, and adjoint against the GPU's own
  per-slot parameter shift (the latter is a consistency check, parity
  unpinned against the oracle).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W
from tests.gpu_helpers import jac_bound
from tests.parity_log import record

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = qsv.Context(0)
    yield c
    c.close()


def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}_oracle.json")) as f:
        return json.load(f)


def _report(tag, **kw):
    print(f"[{tag}] " + " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


def _check(case, quantity, dtype, err, tol):
    """Record the achieved error against the oracle (or the closed form), then
    assert it."""
    record(case, quantity, dtype, err, tol)
    assert err <= tol, f"{case} {quantity}: {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
def test_qaoa_28q_against_oracle(ctx, dt):
    g = _golden("config3")
    c = W.config3()
    st = qsv.State(ctx, c.n_qubits, dt)
    qsv.apply(st, c.ops, c.params)
    amps = None
    if dt == qsv.C128:
        psi = st.to_numpy()
        amps = psi[np.array(g["amp_index"])]
        del psi
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    s = float(np.sum(np.abs(c.observables[0].coeffs)))
    bound = jac_bound(c.ops, c.n_params, c.observables)[0]
    err_ev = abs(ev[0] - g["expval"][0]) / s
    err_j = np.max(np.abs(jac[0] - np.array(g["jac"][0])) / bound)
    dname = "c128" if dt == qsv.C128 else "c64"
    _report("qaoa28", dtype=dname, err_expval_rel=err_ev, err_jac_rel=float(err_j))
    tol = 1e-12 if dt == qsv.C128 else 1e-5
    _check("28q QAOA p=4 (benchmark workload)", "expval rel", dname, err_ev, tol)
    _check("28q QAOA p=4 (benchmark workload)", "jacobian rel", dname, float(err_j), tol)
    if amps is not None:
        want = np.array(g["amp_re"]) + 1j * np.array(g["amp_im"])
        # 64 sampled amplitudes of a 2^28 state: the state tolerance spread evenly over 2^20 amplitudes
        _check("28q QAOA p=4 (benchmark workload)", "sampled amplitudes abs", dname,
               float(np.max(np.abs(amps - want))), 1e-12 / math.sqrt(1 << 20))


def test_ansatz_20q_against_oracle(ctx):
    g = _golden("config2")
    c = W.config2()
    st = qsv.State(ctx, c.n_qubits)
    qsv.apply(st, c.ops, c.params)
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    s = float(np.sum(np.abs(c.observables[0].coeffs)))
    err_j = np.max(np.abs(jac[0] - np.array(g["jac"][0])) / jac_bound(c.ops, c.n_params, c.observables)[0])
    _report("hea20", err_expval_rel=abs(ev[0] - g["expval"][0]) / s, err_jac_rel=float(err_j))
    _check("20q hardware-efficient ansatz", "expval rel", "c128", abs(ev[0] - g["expval"][0]) / s, 1e-12)
    _check("20q hardware-efficient ansatz", "jacobian rel", "c128", float(err_j), 1e-12)


def _u3_product(n, layers, seed=5):
    """config-5 circuit without its CNOTs: a product of one-qubit circuits."""
    c = W.config5(seed=seed, n=n, layers=layers)
    c.ops = [o for o in c.ops if o.name == "U3"]
    return c


@pytest.mark.parametrize("n,dt", [(32, qsv.C128), (33, qsv.C64)])
def test_product_circuit_full_size(ctx, n, dt):
    """<Z_0 Z_{n-1}> = <Z_0><Z_{n-1}> and its gradient factorise into
    one-qubit oracle runs."""
    layers = 20
    c = _u3_product(n, layers)
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, c.ops, c.params)
    obs = c.observables

    def one_qubit(w):
        ops1 = [W.Op(o.name, (0,), o.param, o.scale) for o in c.ops if o.wires[0] == w]
        psi1 = oracle.apply(1, ops1, c.params)
        z = [W.PauliSum(np.array([1.0]), ["Z"])]
        return oracle.expval(psi1, z)[0], oracle.adjoint_jacobian(psi1, ops1, c.params, z)[0]

    z0, g0 = one_qubit(0)
    zl, gl = one_qubit(n - 1)
    if dt == qsv.C128:
        jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, obs)
        want = g0 * zl + gl * z0
        err_j = float(np.max(np.abs(jac[0] - want)))
        _report("product", n=n, err_expval=abs(ev[0] - z0 * zl), err_jac=err_j)
        _check(f"{n}q U3 product circuit (one-qubit oracle runs)", "expval abs", "c128", abs(ev[0] - z0 * zl), 1e-12)
        _check(f"{n}q U3 product circuit (one-qubit oracle runs)", "jacobian abs", "c128", err_j, 1e-12)
    else:
        ev = qsv.expval(st, obs)
        _report("product", n=n, dtype="c64", err_expval=abs(ev[0] - z0 * zl))
        _check(f"{n}q U3 product circuit (one-qubit oracle runs)", "expval abs", "c64", abs(ev[0] - z0 * zl), 1e-5)
    st.close()
    ctx.release_workspace()


@pytest.mark.parametrize("n,dt", [(32, qsv.C128), (33, qsv.C64)])
def test_mirror_and_ghz_full_size(ctx, n, dt):
    """C(theta)^dagger C(theta) |0> = |0>: <Z_w> = 1 on every wire, and the
    GHZ closed forms."""
    c = W.config5(n=n, layers=4)
    mirror = c.ops + [W.Op(o.name, o.wires, o.param, o.scale, not o.inverse) for o in reversed(c.ops)]
    st = qsv.State(ctx, n, dt)
    qsv.apply(st, mirror, c.params)
    allz = W.PauliSum(np.ones(n) / n, [W.pauli_word(n, {w: "Z"}) for w in range(n)])
    norm = W.PauliSum(np.array([1.0]), ["I" * n])
    ev = qsv.expval(st, [allz, norm])
    tol = 1e-12 if dt == qsv.C128 else 1e-5
    dname = "c128" if dt == qsv.C128 else "c64"
    _report("mirror", n=n, err_z=abs(ev[0] - 1), err_norm=abs(ev[1] - 1))
    _check(f"{n}q mirror circuit C^dagger C |0>", "mean <Z_w> abs", dname, abs(ev[0] - 1), tol)
    _check(f"{n}q mirror circuit C^dagger C |0>", "norm abs", dname, abs(ev[1] - 1), tol)
    st.reset(0)
    g = W.ghz(n)
    qsv.apply(st, g.ops, g.params)
    ev = qsv.expval(st, [W.PauliSum(np.array([1.0]), [W.pauli_word(n, {0: "Z", n - 1: "Z"})]),
                         W.PauliSum(np.array([1.0]), ["X" * n]),
                         W.PauliSum(np.array([1.0]), ["Y" * n])])
    want = [1.0, 1.0, math.cos(n * math.pi / 2)]
    _report("ghz", n=n, err=float(np.max(np.abs(ev - want))))
    _check(f"{n}q GHZ closed forms", "<ZZ>, <X..X>, <Y..Y> abs", dname, float(np.max(np.abs(ev - want))), tol)
    # Listing 3: probabilities on wires [0, n//2, n-1] of the GHZ state
    rows = [l.split() for l in open(os.path.join(GOLDEN, "ghz_probs_listing3.txt")) if not l.startswith("#")]
    p = qsv.probs(st, [0, n // 2, n - 1])
    _check(f"{n}q GHZ closed forms", "Listing 3 probabilities abs", dname,
           float(np.max(np.abs(p - np.array([float(r[1]) for r in rows])))), tol)
    st.close()


def test_u3_brickwall_32q_adjoint_vs_gpu_shift_rule(ctx):
    """Entangling config-5 circuit at 32 qubits: adjoint Jacobian entries
    against the GPU's own two-term shift rule on sampled slots (U3 angles
    enter with frequency 1 only).  Consistency, parity unpinned."""
    c = W.config5()
    n = c.n_qubits
    st = qsv.State(ctx, n)
    qsv.apply(st, c.ops, c.params)
    jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables)
    rng = np.random.default_rng(0)
    # parameters of the last layers: their light cones reach both observed wires
    picks = rng.choice(np.arange(c.n_params - 3 * n, c.n_params), 3, replace=False)
    for p in picks:
        vals = []
        for sh in (math.pi / 2, -math.pi / 2):
            q = c.params.copy()
            q[p] += sh
            st.reset(0)
            qsv.apply(st, c.ops, q)
            vals.append(qsv.expval(st, c.observables)[0])
        ps = 0.5 * (vals[0] - vals[1])
        _report("u3-32q", param=int(p), adjoint=float(jac[0, p]), shift=float(ps))
        _check("32q U3 brick wall: adjoint vs GPU shift rule (parity unpinned)", f"d/dparam[{p}] abs", "c128",
               abs(jac[0, p] - ps), 1e-11)
    st.close()
    ctx.release_workspace()


@pytest.mark.parametrize("n,dt", [(32, qsv.C128), (33, qsv.C64)])
def test_two_qubit_streaming_low_bits_full_size(ctx, n, dt):
    """One kernel per gate (no tile fusion): two-qubit gates of every kernel
    class with targets among the three lowest index bits (the one lane per
    amplitude kernel, whose 2^n lanes exceed one launch's thread limit and
    run grid-stride), then their inverses in reverse order: the state
    returns to |0..0>."""
    w = lambda bit: n - 1 - bit
    pairs = [(0, 1), (1, 2), (2, 0), (0, n - 1), (n - 2, 1)]
    ops = [W.op("Hadamard", [w(b)]) for b in (0, 1, 2, n - 1, n - 2)]
    k = 0
    for g in ("IsingXX", "IsingYY", "SingleExcitation", "IsingZZ", "CRX", "CNOT"):
        for a, b in pairs:
            par = () if g == "CNOT" else ((k, 1.0),)
            ops.append(W.op(g, [w(a), w(b)], *par))
            k += 1
    params = np.random.default_rng(3).uniform(-math.pi, math.pi, k)
    mirror = ops + [W.Op(o.name, o.wires, o.param, o.scale, not o.inverse) for o in reversed(ops)]
    st = qsv.State(ctx, n, dt)
    ctx.set_option(qsv.OPT_FUSION, 0)
    try:
        qsv.apply(st, mirror, params)
    finally:
        ctx.set_option(qsv.OPT_FUSION, 1)
    allz = W.PauliSum(np.ones(n) / n, [W.pauli_word(n, {x: "Z"}) for x in range(n)])
    norm = W.PauliSum(np.array([1.0]), ["I" * n])
    ev = qsv.expval(st, [allz, norm])
    tol = 1e-12 if dt == qsv.C128 else 1e-5
    dname = "c128" if dt == qsv.C128 else "c64"
    _report("gate2-low", n=n, err_z=abs(ev[0] - 1), err_norm=abs(ev[1] - 1))
    _check(f"{n}q two-qubit gates on low bits, one kernel each, mirrored", "mean <Z_w> abs", dname,
           abs(ev[0] - 1), tol)
    _check(f"{n}q two-qubit gates on low bits, one kernel each, mirrored", "norm abs", dname, abs(ev[1] - 1), tol)
    st.close()
