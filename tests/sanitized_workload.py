"""Host-side workload run under AddressSanitizer / UndefinedBehaviorSanitizer
by tests/test_sanitizers.py (in a child process with the sanitizer runtime
preloaded).  `qsv`: the library's host runtime through its host-only entry
points (validation, planning, lowering; no GPU needed).  `oracle`: the CPU
oracle on small random circuits."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2403_02512_amd import workloads as W  # noqa: E402


def run_qsv():
    from paper_2403_02512_amd import qsv
    rng = np.random.default_rng(0)
    gates = sorted(W.GATE_ARITY)
    # every gate, random placements, controls, inverses: validation + both programs
    for n in (4, 9):
        for name in gates:
            k, na = W.GATE_ARITY[name]
            kk = k or 3
            nc = int(rng.integers(0, min(2, n - kk) + 1))
            wires = list(rng.choice(n, size=kk + nc, replace=False))
            mat = W.random_unitary(kk, rng) if name == "QubitUnitary" else None
            o = W.op(name, wires, *[(0, 0.7)] * na, n_ctrls=nc, matrix=mat)
            qsv.validate_ops(n, [o], 1)
            for adj in (False, True):
                qsv.plan_json(n, [o], [0.3], adjoint=adj)
    # random circuits under several tile options and both precisions
    for n, seed in ((3, 1), (8, 2), (12, 3), (14, 4)):
        c = W.random_circuit(n, 60, seed=seed, n_params=7, p_ctrl=0.25, max_k=min(n, 6))
        for dt in (qsv.C128, qsv.C64):
            for opts in ({}, {"tile_bits": 5, "low_bits": 2}, {"tile_bits": 8}, {"fusion": False}, {"fusion": 2}):
                for adj in (False, True):
                    qsv.plan_json(n, c.ops, c.params, dtype=dt, adjoint=adj, **opts)
                    qsv.plan_stats(n, c.ops, c.params, dtype=dt, adjoint=adj, **opts)
    for c in (W.config1(), W.config3(n=14), W.config5(n=12, layers=3)):
        for adj in (False, True):
            qsv.plan_json(c.n_qubits, c.ops, c.params, adjoint=adj)
    qsv.validate_obs(6, W.random_observables(6, rng, n_obs=3, n_terms=5))
    # invalid inputs: every one must be rejected with an error, nothing else
    bad = [lambda: qsv.validate_ops(4, [W.op("RX", [7], (0, 1.0))], 1),
           lambda: qsv.validate_ops(4, [W.op("CNOT", [1, 1])], 0),
           lambda: qsv.validate_ops(4, [W.op("RX", [0], (5, 1.0))], 1),
           lambda: qsv.plan_json(40, [], []),
           lambda: qsv.validate_obs(3, [W.PauliSum(np.array([1.0]), ["XXXX"])])]
    for f in bad:
        try:
            f()
        except (qsv.QsvError, ValueError):
            continue
        raise AssertionError("invalid input accepted")
    # no device here: context creation fails cleanly
    try:
        qsv.Context(0)
        raise AssertionError("context created without a device")
    except qsv.QsvError:
        pass
    print("qsv host runtime: ok")


def run_oracle():
    import oracle
    for n, seed in ((1, 0), (3, 1), (6, 2), (9, 3)):
        c = W.random_circuit(n, 40, seed=seed, n_params=5, p_ctrl=0.3, max_k=min(n, 4))
        obs = W.random_observables(n, np.random.default_rng(seed), n_obs=2, n_terms=4)
        psi = oracle.apply(n, c.ops, c.params)
        oracle.expval(psi, obs)
        oracle.adjoint_jacobian(psi, c.ops, c.params, obs)
        oracle.sample(psi, np.random.default_rng(seed).uniform(size=50))
    print("oracle: ok")


if __name__ == "__main__":
    {"qsv": run_qsv, "oracle": run_oracle}[sys.argv[1]]()
