"""Host-only checks of the pass planner through qsv_plan_stats (no GPU)."""
import numpy as np
import pytest

from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W


def test_unfused_plan_is_one_pass_per_gate():
    c = W.config3(n=20)
    st = qsv.plan_stats(20, c.ops, c.params, fusion=False)
    assert st["passes"] == len(c.ops) and st["tile_passes"] == 0
    # H, RX: 2 N B each; IsingZZ: 2 N B (diagonal quads)
    assert st["alg_bytes"] == len(c.ops) * 2 * 16 * 2 ** 20


def test_qaoa_28q_fuses_into_few_passes():
    c = W.config3()
    fwd = qsv.plan_stats(28, c.ops, c.params)
    adj = qsv.plan_stats(28, c.ops, c.params, adjoint=True)
    assert fwd["passes"] <= 12 and fwd["tile_passes"] == fwd["passes"]
    assert adj["passes"] <= 12
    N = 2 ** 28
    assert fwd["alg_bytes"] == fwd["passes"] * 2 * 16 * N
    assert adj["alg_bytes"] == adj["passes"] * 4 * 16 * N


def test_small_register_is_one_tile():
    for n in (1, 3, 8, 12):
        c = W.random_circuit(n, 60, seed=n)
        st = qsv.plan_stats(n, c.ops, c.params)
        assert st["passes"] == 1


@pytest.mark.parametrize("name,k,low", [("RX", 1, True), ("IsingXX", 2, True), ("IsingXX", 2, False),
                                        ("QubitUnitary", 3, True),
                                        ("QubitUnitary", 4, False), ("QubitUnitary", 5, False),
                                        ("QubitUnitary", 4, True), ("QubitUnitary", 5, True),
                                        ("QubitUnitary", 6, False), ("QubitUnitary", 6, True)])
def test_single_gate_kernel_choice(name, k, low):
    """One pass per single gate: the pair and quad kernels for k = 1, 2 (the
    LDS-staged dense kernel measured slower for two-qubit gates, also on the
    lowest bits), the dense kernel for k = 3..6 (low or high bits)."""
    n = 20
    rng = np.random.default_rng(0)
    mat = W.random_unitary(k, rng) if name == "QubitUnitary" else None
    slots = [(0, 1.0)] if name != "QubitUnitary" else []
    wires = list(range(n - k, n))[::-1] if low else list(range(k))
    o = W.op(name, wires, *slots, matrix=mat)
    st = qsv.plan_stats(n, [o], [0.3])
    assert st["passes"] == 1 and st["tile_passes"] == 0
    kind = qsv.plan_json(n, [o], [0.3])["steps"][0]["type"]
    assert kind == {1: "gate1", 2: "gate2"}.get(k, "dense")


def test_non_commuting_gates_keep_order():
    """Two gates on a high wire separated by a gate that mixes it cannot share
    a pass with a third gate that needs a different tile bit set: the plan
    needs at least two passes once the tile cannot hold all targets."""
    n = 20
    ops = [W.op("Hadamard", [w]) for w in range(n)]
    st = qsv.plan_stats(n, ops, [], tile_bits=6, low_bits=2)
    # 20 mixing bits, at most 6 per pass (2 of them low bits shared by all)
    assert st["passes"] >= 1 + (n - 6 + 3) // 4


def test_adjoint_plan_counts_inner_products():
    c = W.config1()
    st = qsv.plan_stats(10, c.ops, c.params, adjoint=True, fusion=2)
    # 120 trainable slots + 160 un-applies in a single tile (plus group
    # headers); a Z-parity inner product and rotation of the same strings
    # share one op
    fused = sum(t["kind"] == 13 for t in qsv.plan_json(10, c.ops, c.params, adjoint=True, fusion=2)["tops"])
    assert st["passes"] == 1 and st["kernel_ops"] + fused >= 280
    # with one-qubit layers the rotations of a layer share sub-ops
    lay = qsv.plan_stats(10, c.ops, c.params, adjoint=True)
    assert lay["passes"] == 1 and lay["kernel_ops"] < st["kernel_ops"]


def test_plan_stats_validates():
    with pytest.raises(qsv.QsvError):
        qsv.plan_stats(3, [W.op("RX", [5], (0, 1.0))], [0.1])


@pytest.mark.timeout(60)
def test_wide_gate_beside_coalescing_bits_terminates():
    """A gate whose targets plus the coalescing bits exceed the tile width gets
    a pass of its own instead of an empty pass (regression: the planner used
    to loop forever)."""
    n = 8
    rng = np.random.default_rng(3)
    ops = [W.op("QubitUnitary", [0, 1, 2, 3, 4], matrix=W.random_unitary(5, rng)), W.op("RX", [7], (0, 1.0))]
    for adj in (False, True):
        st = qsv.plan_stats(n, ops, [0.2], adjoint=adj, tile_bits=5, low_bits=2)
        assert 1 <= st["passes"] <= 2


def _deep_narrow(n=10, layers=40):
    ops, p = [], 0
    for _ in range(layers):
        for q in range(n):
            for g in ("RX", "RY", "RZ"):
                ops.append(W.op(g, [q], (p, 1.0)))
                p += 1
    return ops, np.linspace(0.1, 3.0, p)


@pytest.mark.parametrize("dt", [qsv.C128, qsv.C64])
@pytest.mark.parametrize("tile_bits", [0, 8, 12, 13])
def test_tile_passes_fit_the_cu_lds(dt, tile_bits):
    """A deep narrow circuit (10 qubits, 1200 trainable slots) puts many
    inner products next to each other; every adjoint and forward tile pass
    must stay within the CU's 160 KiB of LDS (slot accumulators and phase
    tables included), at every tile width the options allow."""
    ops, params = _deep_narrow()
    for adj in (False, True):
        prog = qsv.plan_json(10, ops, params, dtype=dt, adjoint=adj, tile_bits=tile_bits)
        tiles = [st for st in prog["steps"] if st["type"] == "tile"]
        assert tiles and all(st["lds"] <= 160 * 1024 for st in tiles), max(st["lds"] for st in tiles)
        if adj:
            assert sum(st["nslots"] for st in tiles) == len(params)


TILE_WS = 4


def test_qaoa_passes_fit_two_blocks_per_cu():
    """The benchmark's tile passes are group-only, and their LDS keeps two
    blocks per CU (<= 80 KiB each)."""
    c = W.config3(n=28)
    for adj in (False, True):
        prog = qsv.plan_json(28, c.ops, c.params, adjoint=adj)
        tiles = [st for st in prog["steps"] if st["type"] == "tile"]
        assert all(not st["generic"] and not st["flags"] & TILE_WS for st in tiles)
        assert max(st["lds"] for st in tiles) <= 80 * 1024
