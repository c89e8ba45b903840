"""Seeded synthetic inputs: circuits, parameters and Pauli-sum observables.

This module only describes inputs (which gate on which wires with which
parameter slot, random angles, random Pauli words); it does no state-vector
arithmetic.  Both the GPU binding and the CPU oracle consume these objects.

Workload shapes follow the paper's experiments (arXiv 2403.02512):
  * layered rotation + CNOT ansatz (Sec. 4.3 StronglyEntanglingLayers-like),
  * QAOA MaxCut with IsingZZ cost layers and RX mixers (Sec. 4.1),
  * VQE-like RY + Givens-rotation (SingleExcitation) circuits with many-term
    Pauli Hamiltonians (Sec. 3.2 and Sec. 4.2),
  * single-gate sweeps over target wires at ~30 qubits (Sec. 3.1).
The paper's molecular Hamiltonians and cut-circuit fragments are not
available; the seeded generators below stand in for them.

Wire 0 is the most significant index bit (Alg. 1).  An operation's ``wires``
list holds its ``n_ctrls`` extra control wires first, then the gate's own
wires.  Angle slot s equals ``scale[s] * params[param[s]]`` when
``param[s] >= 0``, else the constant ``scale[s]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

TWO_PI = 2.0 * np.pi

# (own wires, angle slots); 0 wires = any width (MultiRZ, QubitUnitary).
GATE_ARITY = {
    "Identity": (1, 0), "PauliX": (1, 0), "PauliY": (1, 0), "PauliZ": (1, 0), "Hadamard": (1, 0),
    "S": (1, 0), "T": (1, 0), "SX": (1, 0),
    "PhaseShift": (1, 1), "RX": (1, 1), "RY": (1, 1), "RZ": (1, 1), "Rot": (1, 3), "U3": (1, 3),
    "CNOT": (2, 0), "CY": (2, 0), "CZ": (2, 0), "SWAP": (2, 0),
    "CRX": (2, 1), "CRY": (2, 1), "CRZ": (2, 1), "CRot": (2, 3), "ControlledPhaseShift": (2, 1),
    "IsingXX": (2, 1), "IsingYY": (2, 1), "IsingZZ": (2, 1), "IsingXY": (2, 1),
    "SingleExcitation": (2, 1), "Toffoli": (3, 0), "CSWAP": (3, 0), "DoubleExcitation": (4, 1),
    "MultiRZ": (0, 1), "QubitUnitary": (0, 0),
}


@dataclass
class Op:
    name: str
    wires: tuple
    param: tuple = ()
    scale: tuple = ()
    inverse: bool = False
    n_ctrls: int = 0
    ctrl_values: int = -1          # -1: every extra control must be |1>
    matrix: Optional[np.ndarray] = None


@dataclass
class PauliSum:
    coeffs: np.ndarray             # (n_terms,) float64
    words: List[str]               # n_terms strings of length n over 'IXYZ'


@dataclass
class Circuit:
    n_qubits: int
    ops: List[Op]
    params: np.ndarray
    observables: List[PauliSum] = field(default_factory=list)
    name: str = ""

    @property
    def n_params(self) -> int:
        return int(self.params.size)


def op(name, wires, *slots, inverse=False, n_ctrls=0, ctrl_values=-1, matrix=None):
    """Op with angle slots given as (param_index, scale) pairs."""
    return Op(name, tuple(int(w) for w in wires), tuple(int(p) for p, _ in slots),
              tuple(float(s) for _, s in slots), bool(inverse), int(n_ctrls), int(ctrl_values), matrix)


def pauli_word(n: int, letters: dict) -> str:
    w = ["I"] * n
    for wire, l in letters.items():
        w[wire] = l
    return "".join(w)


# ----------------------------------------------------------------- states

def random_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Normalised state with iid complex Gaussian amplitudes."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


# ----------------------------------------------------------------- configs

def config1(seed: int = 1, n: int = 10, layers: int = 4) -> Circuit:
    """Layered ansatz: per layer RX,RY,RZ on every qubit, then a CNOT ring.
    Observable <Z_0>."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, TWO_PI, layers * n * 3)
    ops, p = [], 0
    for _ in range(layers):
        for q in range(n):
            for g in ("RX", "RY", "RZ"):
                ops.append(op(g, [q], (p, 1.0)))
                p += 1
        for q in range(n):
            ops.append(op("CNOT", [q, (q + 1) % n]))
    obs = [PauliSum(np.array([1.0]), [pauli_word(n, {0: "Z"})])]
    return Circuit(n, ops, theta, obs, f"layered-rot-cnot-ring n={n}")


def config2(seed: int = 2, n: int = 20, layers: int = 10) -> Circuit:
    """Hardware-efficient ansatz: per layer RY,RZ per qubit, then CZ on an open
    chain.  Observable sum_i c_i Z_i with c_i ~ N(0,1) drawn after theta."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, TWO_PI, layers * n * 2)
    c = rng.standard_normal(n)
    ops, p = [], 0
    for _ in range(layers):
        for q in range(n):
            ops.append(op("RY", [q], (p, 1.0)))
            ops.append(op("RZ", [q], (p + 1, 1.0)))
            p += 2
        for q in range(n - 1):
            ops.append(op("CZ", [q, q + 1]))
    obs = [PauliSum(c, [pauli_word(n, {i: "Z"}) for i in range(n)])]
    return Circuit(n, ops, theta, obs, f"hea-ry-rz-cz n={n}")


def random_regular_graph(n: int, d: int, rng) -> List[tuple]:
    """Uniform simple d-regular graph by the pairing model with rejection."""
    assert n * d % 2 == 0
    while True:
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        edges = {tuple(sorted((int(a), int(b)))) for a, b in pairs}
        if len(edges) == len(pairs):
            return sorted(edges)


def config3(seed: int = 3, n: int = 28, p_layers: int = 4) -> Circuit:
    """QAOA MaxCut on a seeded random 3-regular graph: H on every qubit, then
    per layer IsingZZ(gamma_l) on every edge and RX(beta_l) on every qubit.
    params = (gamma_0..gamma_{p-1}, beta_0..beta_{p-1}); observable
    H_C = sum_edges Z_a Z_b."""
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(n, 3, rng)
    gamma = rng.uniform(0.0, TWO_PI, p_layers)
    beta = rng.uniform(0.0, TWO_PI, p_layers)
    ops = [op("Hadamard", [q]) for q in range(n)]
    for l in range(p_layers):
        for a, b in edges:
            ops.append(op("IsingZZ", [a, b], (l, 1.0)))
        for q in range(n):
            ops.append(op("RX", [q], (p_layers + l, 1.0)))
    obs = [PauliSum(np.ones(len(edges)), [pauli_word(n, {a: "Z", b: "Z"}) for a, b in edges])]
    c = Circuit(n, ops, np.concatenate([gamma, beta]), obs, f"qaoa-maxcut-3reg n={n} p={p_layers}")
    c.edges = edges
    return c


def random_pauli_sum(n: int, n_terms: int, rng, std: float = 0.1) -> PauliSum:
    """n_terms distinct non-identity Pauli words, letters iid uniform over
    IXYZ, coefficients ~ N(0, std)."""
    words, seen = [], set()
    letters = np.array(list("IXYZ"))
    while len(words) < n_terms:
        w = "".join(letters[rng.integers(0, 4, n)])
        if w == "I" * n or w in seen:
            continue
        seen.add(w)
        words.append(w)
    return PauliSum(rng.normal(0.0, std, n_terms), words)


def vqe_circuit(n: int, rng, n_terms: int = 200, layers: int = 6) -> Circuit:
    """One VQE-like circuit: per layer RY on every qubit, then SingleExcitation
    (Givens rotation) on (q, q+1) for even q in even layers and odd q in odd
    layers; a random many-term Pauli Hamiltonian."""
    ops, p = [], 0
    for l in range(layers):
        for q in range(n):
            ops.append(op("RY", [q], (p, 1.0)))
            p += 1
        for q in range(l % 2, n - 1, 2):
            ops.append(op("SingleExcitation", [q, q + 1], (p, 1.0)))
            p += 1
    theta = rng.uniform(0.0, TWO_PI, p)
    ham = random_pauli_sum(n, n_terms, rng)
    return Circuit(n, ops, theta, [ham], f"vqe-ry-givens n={n}")


def config4(seed: int = 4, n_circuits: int = 512, n_min: int = 12, n_max: int = 22,
            n_terms: int = 200) -> List[Circuit]:
    """Batch of VQE-like circuits of uneven width n ~ UniformInt[n_min, n_max]."""
    rng = np.random.default_rng(seed)
    widths = rng.integers(n_min, n_max + 1, n_circuits)
    return [vqe_circuit(int(w), rng, n_terms) for w in widths]


def config5(seed: int = 5, n: int = 32, layers: int = 20) -> Circuit:
    """Random layered circuit: per layer U3 on every qubit, then a brick-wall of
    CNOTs ((2i,2i+1) on even layers, (2i+1,2i+2) on odd layers).
    Observable Z_0 Z_{n-1}."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, TWO_PI, layers * n * 3)
    ops, p = [], 0
    for l in range(layers):
        for q in range(n):
            ops.append(op("U3", [q], (p, 1.0), (p + 1, 1.0), (p + 2, 1.0)))
            p += 3
        for q in range(l % 2, n - 1, 2):
            ops.append(op("CNOT", [q, q + 1]))
    obs = [PauliSum(np.array([1.0]), [pauli_word(n, {0: "Z", n - 1: "Z"})])]
    return Circuit(n, ops, ang, obs, f"u3-brickwall-cnot n={n}")


def ghz(n: int) -> Circuit:
    """GHZ preparation (paper Sec. 2.2 MPI listing): H on wire 0, CNOT chain."""
    ops = [op("Hadamard", [0])] + [op("CNOT", [i - 1, i]) for i in range(1, n)]
    return Circuit(n, ops, np.zeros(0), [], f"ghz n={n}")


# ----------------------------------------------------------------- random

_ONE_Q = ["PauliX", "PauliY", "PauliZ", "Hadamard", "S", "T", "SX", "PhaseShift", "RX", "RY", "RZ", "Rot", "U3"]
_TWO_Q = ["CNOT", "CY", "CZ", "SWAP", "CRX", "CRY", "CRZ", "CRot", "ControlledPhaseShift",
          "IsingXX", "IsingYY", "IsingZZ", "IsingXY", "SingleExcitation"]
_MANY_Q = ["Toffoli", "CSWAP", "DoubleExcitation", "MultiRZ", "QubitUnitary"]


def random_unitary(k: int, rng) -> np.ndarray:
    """Haar-ish random 2^k unitary (QR of a complex Gaussian matrix)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_circuit(n: int, n_ops: int, seed: int, gates: Optional[Sequence[str]] = None,
                   n_params: Optional[int] = None, p_inverse: float = 0.2, p_ctrl: float = 0.1,
                   max_k: int = 4, shared: bool = True) -> Circuit:
    """Random circuit over the whole gate set, random wires and angle slots.
    With ``shared`` several slots point at the same parameter."""
    rng = np.random.default_rng(seed)
    pool = list(gates) if gates is not None else _ONE_Q + _TWO_Q + _MANY_Q
    pool = [g for g in pool if (GATE_ARITY[g][0] or 1) <= n]
    ops = []
    slots = 0
    n_params = n_params if n_params is not None else max(1, n_ops)
    for _ in range(n_ops):
        g = pool[rng.integers(len(pool))]
        k, na = GATE_ARITY[g]
        if k == 0:
            k = int(rng.integers(1, min(max_k, n) + 1))
        n_ctrls = 0
        if rng.random() < p_ctrl and n - k >= 1:
            n_ctrls = int(rng.integers(1, min(2, n - k) + 1))
        wires = rng.choice(n, size=k + n_ctrls, replace=False)
        sl = []
        for _s in range(na):
            if rng.random() < 0.15:
                sl.append((-1, float(rng.uniform(-TWO_PI, TWO_PI))))   # constant angle
            else:
                pidx = int(rng.integers(n_params)) if shared else slots % n_params
                sl.append((pidx, float(rng.choice([1.0, -0.5, 2.0, 0.75]))))
                slots += 1
        cv = int(rng.integers(0, 1 << n_ctrls)) if n_ctrls else -1
        mat = random_unitary(k, rng) if g == "QubitUnitary" else None
        ops.append(op(g, wires, *sl, inverse=rng.random() < p_inverse, n_ctrls=n_ctrls,
                      ctrl_values=cv, matrix=mat))
    params = rng.uniform(-np.pi, np.pi, n_params)
    return Circuit(n, ops, params, [], f"random n={n} ops={n_ops} seed={seed}")


def random_observables(n: int, rng, n_obs: int = 2, n_terms: int = 5) -> List[PauliSum]:
    return [PauliSum(rng.normal(0, 1, n_terms), [random_pauli_sum(n, 1, rng).words[0] for _ in range(n_terms)])
            for _ in range(n_obs)]
