"""Write the oracle's values for the full-size parity cases (this script calls
only the CPU oracle and the seeded input generators).

  python tests/golden/make_golden.py [config2|config3|all]

config3: 28-qubit QAOA MaxCut (3-regular graph, p = 4): <H_C>, the 8-entry
         gradient and 64 sampled amplitudes of the final state.
config2: 20-qubit RY/RZ + CZ ansatz: <H>, the 400-entry gradient.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2403_02512_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(name, circ, sample_amps=0):
    t0 = time.time()
    n = circ.n_qubits
    psi = oracle.apply(n, circ.ops, circ.params)
    ev = oracle.expval(psi, circ.observables)
    jac = oracle.adjoint_jacobian(psi, circ.ops, circ.params, circ.observables)
    out = {"workload": circ.name, "n_qubits": n, "generator": f"workloads.{name}()",
           "expval": [float(x) for x in ev], "jac": [[float(x) for x in row] for row in jac],
           "oracle_threads": oracle.num_threads(), "oracle_seconds": round(time.time() - t0, 1)}
    if sample_amps:
        idx = np.random.default_rng(12345).integers(0, 1 << n, sample_amps)
        out["amp_index"] = [int(i) for i in idx]
        out["amp_re"] = [float(psi[i].real) for i in idx]
        out["amp_im"] = [float(psi[i].imag) for i in idx]
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {out['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("config2", "all"):
        run("config2", W.config2())
    if which in ("config3", "all"):
        run("config3", W.config3(), sample_amps=64)
