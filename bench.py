"""Benchmark: adjoint-Jacobian seconds per evaluation of a 28-qubit QAOA MaxCut
circuit (random 3-regular graph, p = 4, complex128) on one MI355X, with the
dominant kernel's achieved HBM bandwidth against the 8 TB/s peak.

One step = reset to |0..0>, apply the 308 gates, then one adjoint Jacobian
call (lambda = H_C psi together with <H_C>, and the reverse sweep that
un-applies every gate from phi and lambda while taking the generator inner
products).  Inputs are seeded and synthetic; the state is resident in HBM for
the whole timed region.  The timed region records HIP events around every
launch (per-kernel durations for the roofline); the same steps are timed
again without events, and forward-only steps give gates/s.  <H_C> and the
gradient are compared with the FP64 oracle's values for the same workload.

Outside the headline (skipped with --no-extras): the same workload with a
complex64 state, the 20-layer U3 brick wall at 33 qubits complex64 (forward)
and 32 qubits complex128 (forward + Jacobian), and the 512-circuit batched
VQE sweep (captured graph vs per-circuit loop).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "gate-apply HBM GB/s (% peak) + adjoint Jacobian s/eval at 28q c128 vs plain"


def cpu_baseline(circ) -> dict:
    """Time the plain FP64 oracle on a bounded sample of the same 28-qubit
    workload whose gate mix is the workload's own: one Hadamard, 6 IsingZZ
    and 4 RX of layer 0 (1 : 6 : 4, the ratio of the 28 H, 168 IsingZZ and
    112 RX of the full circuit, which is 28 copies of this mix), their wires
    spread evenly over the register (a gate's cost depends on its index-bit
    stride), run through the full pipeline (forward apply, <H>, adjoint
    Jacobian).  The oracle's cost is a fixed part (state allocation and
    initialisation, workspace) plus a cost per gate and per cost term, so
    three runs give the parts: no gates with 1 and with 4 of the 42 terms
    (fixed part and per-term cost), and the block with 2 terms.  The full
    evaluation is the fixed part, 28 blocks and 42 terms."""
    import oracle
    from paper_2403_02512_amd import workloads as W

    n = circ.n_qubits
    n_edges = len(circ.observables[0].words)
    ops = ([circ.ops[n // 2]] + [circ.ops[n + e] for e in range(0, n_edges, n_edges // 6)][:6] +
           [circ.ops[n + n_edges + q] for q in range(n // 8, n, n // 4)][:4])
    assert [o.name for o in ops] == ["Hadamard"] + ["IsingZZ"] * 6 + ["RX"] * 4
    reps = len(circ.ops) // len(ops)
    assert reps * len(ops) == len(circ.ops)
    obs = circ.observables[0]

    def run(gates, j):
        o = W.PauliSum(obs.coeffs[:j], obs.words[:j])
        t0 = time.perf_counter()
        psi = oracle.apply(n, gates, circ.params)
        oracle.expval(psi, [o])
        oracle.adjoint_jacobian(psi, gates, circ.params, [o])
        return time.perf_counter() - t0

    t_e1 = run([], 1)
    t_e4 = run([], 4)
    t_b2 = run(ops, 2)
    per_term = max(t_e4 - t_e1, 0.0) / 3
    fixed = max(t_e1 - per_term, 0.0)
    block = max(t_b2 - fixed - 2 * per_term, 0.0)
    total = fixed + reps * block + len(obs.words) * per_term
    return {"value": round(total, 2), "unit": "s/eval", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"oracle forward + <H> + adjoint Jacobian at {n} qubits on an {len(ops)}-gate block with the "
                       f"workload's gate mix (1 Hadamard, 6 IsingZZ, 4 RX, wires spread over the register; the "
                       f"{len(circ.ops)}-gate circuit is "
                       f"{reps} such blocks) with 2 of the {len(obs.words)} cost terms ({t_b2:.1f} s), and with no "
                       f"gates and 1 and 4 terms ({t_e1:.1f} s, {t_e4:.1f} s); scaled to the fixed part + {reps} "
                       f"blocks + {len(obs.words)} terms"),
            "fixed_s": round(fixed, 3), "block_s": round(block, 3), "per_term_s": round(per_term, 3)}


def micro(n: int, reps: int = 5, dtype_name: str = "c128", nontemporal: bool = False, dense_mfma: bool = False):
    """Per-kernel-class gate-apply bandwidth at n qubits: one JSON line per
    (gate, wires) case with the algorithmic GB/s of its kernel (HIP events on
    the launch stream) and the fraction of the 8 TB/s HBM peak."""
    import torch
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W

    dt = qsv.C128 if dtype_name == "c128" else qsv.C64
    dev = torch.device("cuda", 0)
    ctx = qsv.Context(0, torch.cuda.current_stream(dev).cuda_stream)
    ctx.set_option(qsv.OPT_NONTEMPORAL, int(nontemporal))
    ctx.set_option(qsv.OPT_DENSE_MFMA, int(dense_mfma))
    psi = torch.empty(1 << n, dtype=torch.complex128 if dt == qsv.C128 else torch.complex64, device=dev)
    st = qsv.State(ctx, n, dt, tensor=psi)
    st.reset(0)
    rng = np.random.default_rng(0)
    w = lambda bit: n - 1 - bit          # wire of an index bit
    cases = []
    for b in (0, 1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 20, 24, n - 1):
        cases.append((f"RX bit{b}", [W.op("RX", [w(b)], (-1, 0.3))]))
    for b in (0, n - 1):
        cases.append((f"Hadamard bit{b}", [W.op("Hadamard", [w(b)])]))
        cases.append((f"RZ bit{b}", [W.op("RZ", [w(b)], (-1, 0.3))]))
        cases.append((f"PauliX bit{b}", [W.op("PauliX", [w(b)])]))
        cases.append((f"PhaseShift bit{b}", [W.op("PhaseShift", [w(b)], (-1, 0.3))]))
    for c, t in ((n - 1, 0), (0, n - 1), (13, 14)):
        cases.append((f"CNOT ctrl{c} tgt{t}", [W.op("CNOT", [w(c), w(t)])]))
        cases.append((f"CZ bits{c},{t}", [W.op("CZ", [w(c), w(t)])]))
    cases.append(("Toffoli bits27,26->0", [W.op("Toffoli", [w(n - 1), w(n - 2), w(0)])]))
    for a, b in ((0, 1), (0, n - 1), (13, 14), (n - 2, n - 1)):
        cases.append((f"IsingXX bits{a},{b}", [W.op("IsingXX", [w(a), w(b)], (-1, 0.3))]))
        cases.append((f"IsingZZ bits{a},{b}", [W.op("IsingZZ", [w(a), w(b)], (-1, 0.3))]))
        cases.append((f"SWAP bits{a},{b}", [W.op("SWAP", [w(a), w(b)])]))
        cases.append((f"SingleExcitation bits{a},{b}", [W.op("SingleExcitation", [w(a), w(b)], (-1, 0.3))]))
    for k in (3, 4, 5, 6):
        for lo in (True, False):
            bits = list(range(k)) if lo else list(range(n - k, n))
            cases.append((f"QubitUnitary k={k} {'low' if lo else 'high'} bits",
                          [W.op("QubitUnitary", [w(b) for b in bits], matrix=W.random_unitary(k, rng))]))
    cases.append(("fused 12 RX on bits 0-3,16-23", [W.op("RX", [w(b)], (-1, 0.1 * b)) for b in
                                                    list(range(4)) + list(range(16, 24))]))
    cases.append(("fused 28 RX layer", [W.op("RX", [w(b)], (-1, 0.1 * b)) for b in range(n)]))
    q = W.config3(n=n)
    cases.append(("QAOA forward (308 gates)", q.ops))
    for name, ops in cases:
        m = qsv.MarshalledOps(ops, q.params if ops is q.ops else np.zeros(0))
        qsv.apply(st, ops, None, marshalled=m)
        torch.cuda.synchronize()
        ctx.set_option(qsv.OPT_PROFILE, 1)
        ctx.reset_stats()
        for _ in range(reps):
            qsv.apply(st, ops, None, marshalled=m)
        stats = ctx.kernel_stats()
        ctx.set_option(qsv.OPT_PROFILE, 0)
        tot_ms = sum(s["ms"] for s in stats.values()) / reps
        tot_b = sum(s["bytes"] for s in stats.values()) / reps
        kinds = {k: s["launches"] // reps for k, s in stats.items()}
        gbs = tot_b / 1e9 / (tot_ms / 1e3)
        print(json.dumps({"case": name, "n_qubits": n, "dtype": dtype_name, "nontemporal": nontemporal,
                          "dense_mfma": dense_mfma,
                          "kernels": kinds,
                          "ms": round(tot_ms, 4), "alg_GB": round(tot_b / 1e9, 3), "GB_s": round(gbs, 1),
                          "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}), flush=True)
    # reference: torch's device-to-device copy kernel of the same state size
    src = torch.empty_like(psi)
    dst = torch.empty_like(psi)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    by = 2 * psi.numel() * psi.element_size()
    print(json.dumps({"case": "torch copy_ (reference)", "ms": round(ms, 4), "alg_GB": by / 1e9,
                      "GB_s": round(by / 1e9 / (ms / 1e3), 1), "frac_of_8TBs": round(by / 1e9 / (ms / 1e3) / 8000, 4)}),
          flush=True)


def sweep_cases(n: int, rng, only_half_touch: bool = False):
    """Gate cases of the per-wire sweep at n qubits: every target wire for the
    one-qubit gates; for the two-qubit gates the pair (0, n-1), adjacent pairs
    on low, middle and high wires and 16 random pairs; dense 3- to 5-qubit
    unitaries on the lowest and highest wires.  only_half_touch: the gates that
    touch half the amplitudes (PhaseShift, CZ, CNOT, SingleExcitation) with an
    untouched or control bit among the three lowest index bits, whose cache
    lines hold both touched and untouched amplitudes."""
    from paper_2403_02512_amd import workloads as W
    w = lambda bit: n - 1 - bit          # wire of an index bit
    out = []
    if only_half_touch:
        for b in (0, 1, 2, 3, 8, n - 1):
            out.append((f"PhaseShift bit{b}", "half", [W.op("PhaseShift", [w(b)], (-1, 0.3))]))
        for c, t in ((0, 1), (0, n - 1), (n - 1, 0), (13, 14)):
            out.append((f"CNOT ctrl{c} tgt{t}", "half", [W.op("CNOT", [w(c), w(t)])]))
        for a, b in ((0, 1), (1, 2), (13, 14)):
            out.append((f"CZ bits{a},{b}", "half", [W.op("CZ", [w(a), w(b)])]))
            out.append((f"SingleExcitation bits{a},{b}", "half",
                        [W.op("SingleExcitation", [w(a), w(b)], (-1, 0.3))]))
        return out
    for g in ("RX", "Hadamard", "RZ", "PhaseShift"):
        for b in range(n):
            par = () if g == "Hadamard" else ((-1, 0.3),)
            out.append((f"{g} bit{b}", "1q", [W.op(g, [w(b)], *par)]))
    pairs = [(0, n - 1), (0, 1), (1, 2), (n // 2 - 1, n // 2), (n - 2, n - 1)]
    while len(pairs) < 21:
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        if (a, b) not in pairs:
            pairs.append((a, b))
    for g in ("CNOT", "CZ", "IsingZZ", "IsingXX", "SingleExcitation"):
        par = () if g in ("CNOT", "CZ") else ((-1, 0.3),)
        for a, b in pairs:
            out.append((f"{g} bits{a},{b}", "2q", [W.op(g, [w(a), w(b)], *par)]))
    for k in (3, 4, 5):
        for lo in (True, False):
            bits = list(range(k)) if lo else list(range(n - k, n))
            out.append((f"QubitUnitary k={k} {'low' if lo else 'high'} bits", "dense",
                        [W.op("QubitUnitary", [w(b) for b in bits], matrix=W.random_unitary(k, rng))]))
    return out


def sweep(n: int, dtype_name: str = "c128", reps: int = 3, only_half_touch: bool = False, markers: bool = False):
    """Per-wire gate sweep at n qubits on a random normalised state (seed 0):
    one JSON line per case with its kernel class, the algorithmic bytes and
    GB/s of its launch (HIP events on the launch stream, mean of reps after
    one warm-up) and the fraction of the 8 TB/s HBM peak; then one summary
    line per gate class.  markers: a small torch fill kernel runs before each
    case's timed launches, so that a counter profile's dispatches can be split
    per case."""
    import torch
    from paper_2403_02512_amd import qsv

    dt = qsv.C128 if dtype_name == "c128" else qsv.C64
    dev = torch.device("cuda", 0)
    ctx = qsv.Context(0, torch.cuda.current_stream(dev).cuda_stream)
    cdt = torch.complex128 if dt == qsv.C128 else torch.complex64
    psi = torch.empty(1 << n, dtype=cdt, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    torch.view_as_real(psi).normal_(generator=g)
    psi.div_(torch.linalg.vector_norm(psi))
    st = qsv.State(ctx, n, dt, tensor=psi)
    marker = torch.zeros(64, device=dev)
    if markers:
        # a plain copy of the state: its counter readings calibrate the
        # counters against known bytes
        cal = torch.empty_like(psi)
        cal.copy_(psi)
        torch.cuda.synchronize()
        del cal
    rng = np.random.default_rng(0)
    rows = []
    for ci, (name, cls, ops) in enumerate(sweep_cases(n, rng, only_half_touch)):
        m = qsv.MarshalledOps(ops, np.zeros(0))
        qsv.apply(st, ops, None, marshalled=m)   # warm-up (planning, first launch)
        torch.cuda.synchronize()
        if markers:
            marker.fill_(float(ci))
        ctx.set_option(qsv.OPT_PROFILE, 1)
        ctx.reset_stats()
        for _ in range(reps):
            qsv.apply(st, ops, None, marshalled=m)
        stats = ctx.kernel_stats()
        ctx.set_option(qsv.OPT_PROFILE, 0)
        tot_ms = sum(s["ms"] for s in stats.values()) / reps
        tot_b = sum(s["bytes"] for s in stats.values()) / reps
        gbs = tot_b / 1e9 / (tot_ms / 1e3)
        row = {"case": name, "class": cls, "n_qubits": n, "dtype": dtype_name,
               "kernels": {k: s["launches"] // reps for k, s in stats.items()},
               "ms": round(tot_ms, 4), "alg_GB": round(tot_b / 1e9, 3), "GB_s": round(gbs, 1),
               "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}
        rows.append(row)
        print(json.dumps(row), flush=True)
    torch.cuda.synchronize()
    gates = {}
    for r in rows:
        gates.setdefault(r["case"].split(" ")[0], []).append(r["frac_of_8TBs"])
    for gname, fr in gates.items():
        fr = sorted(fr)
        print(json.dumps({"summary": gname, "n_qubits": n, "dtype": dtype_name, "cases": len(fr),
                          "frac_min": fr[0], "frac_median": fr[len(fr) // 2], "frac_max": fr[-1]}), flush=True)
    st.close()


def micro_tile(n: int, reps: int = 5, only: str = "", layer_modes=(1, 0)):
    """Cost structure of the LDS-tiled passes at n qubits, complex128: for
    small synthetic circuits that plan into one tile pass, the forward pass
    time (one vector) and the adjoint pass time (phi and lambda, with one
    inner product per gate), per launch."""
    import torch
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W
    ctx = qsv.Context(0)
    st = qsv.State(ctx, n)
    w = lambda bit: n - 1 - bit

    def rx(bits, reps_=1):
        ops, p = [], 0
        for _ in range(reps_):
            for b in bits:
                ops.append(W.op("RX", [w(b)], (p, 1.0)))
                p += 1
        return ops, p

    cases = [("RX bits 0,1", *rx([0, 1])), ("RX bits 0-3", *rx(range(4))), ("RX bits 0-7", *rx(range(8))),
             ("RX bits 0-3,16-23", *rx(list(range(4)) + list(range(16, 24)))),
             ("RX bits 16-19", *rx(range(16, 20))), ("RX bits 0-3 x4", *rx(range(4), 4)),
             ("RX bits 0-3 x8", *rx(range(4), 8))]
    zz = [W.op("IsingZZ", [w(b), w((b + 1) % 12)], (2, 1.0)) for b in range(12)]
    cases.append(("IsingZZ ring bits 0-11 + RX bits 0,1", zz + rx([0, 1])[0], 3))
    q = W.config3(n=n)
    cases.append(("QAOA p=4 (308 gates)", q.ops, q.n_params))
    obs = [W.PauliSum(np.array([1.0]), [W.pauli_word(n, {0: "Z"})])]
    for name, ops, npar in cases:
        if only and only != name:
            continue
        params = np.linspace(0.1, 0.9, max(1, npar))
        m = qsv.MarshalledOps(ops, params)
        mo = qsv.MarshalledObs(obs)
        for layers in layer_modes:
            ctx.set_option(qsv.OPT_LAYERS, layers)
            row = {"case": name, "n_qubits": n, "layers": layers}
            for mode in ("fwd", "adj"):
                st.reset(0)
                qsv.apply(st, ops, None, marshalled=m)
                if mode == "adj":
                    qsv.adjoint_jacobian(st, ops, None, None, marshalled=m, marshalled_obs=mo)
                ctx.synchronize()
                ctx.set_option(qsv.OPT_PROFILE, 1)
                ctx.reset_stats()
                for _ in range(reps):
                    if mode == "fwd":
                        qsv.apply(st, ops, None, marshalled=m)
                    else:
                        qsv.adjoint_jacobian(st, ops, None, None, marshalled=m, marshalled_obs=mo)
                stats = ctx.kernel_stats()
                ctx.set_option(qsv.OPT_PROFILE, 0)
                k = "tile1" if mode == "fwd" else "tile2"
                s = stats.get(k)
                row[mode] = None if s is None else {"launches": s["launches"] // reps,
                                                   "ms_per_launch": round(s["ms"] / s["launches"], 4),
                                                   "GB_s": round(s["bytes"] / 1e9 / (s["ms"] / 1e3), 1)}
                if s is None:
                    row[mode + "_kernels"] = {kk: v["launches"] // reps for kk, v in stats.items()}
            print(json.dumps(row), flush=True)
    st.close()
    ctx.close()


def batch_bench(args):
    """Batched VQE sweep: every circuit's <H> and full adjoint gradient, new
    random angles each step.  Three executions of the same work: a loop over
    circuits through the single-state entry points, batched launches, and the
    batched launches replayed from a captured HIP graph."""
    import torch
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W
    ctx = qsv.Context(0)
    cs = W.config4(n_circuits=args.batch_circuits)
    rng = np.random.default_rng(7)
    sets = [[rng.uniform(0, 2 * np.pi, c.n_params) for c in cs] for _ in range(args.warmup + args.steps)]
    states = {}
    for c in cs:
        if c.n_qubits not in states:
            states[c.n_qubits] = qsv.State(ctx, c.n_qubits)
    marsh = [(qsv.MarshalledOps(c.ops, c.params), qsv.MarshalledObs(c.observables[:1])) for c in cs]

    def loop(params):
        ev = np.zeros(len(cs))
        for i, c in enumerate(cs):
            st = states[c.n_qubits]
            st.reset(0)
            m = marsh[i][0]
            m.params[:c.n_params] = params[i]
            qsv.apply(st, c.ops, marshalled=m)
            _, e = qsv.adjoint_jacobian(st, c.ops, None, None, inplace=True, marshalled=m,
                                        marshalled_obs=marsh[i][1])
            ev[i] = e[0]
        return ev

    b = qsv.Batch(ctx, cs)
    results = {}
    for mode in ("loop", "batch", "graph"):
        for w in range(args.warmup):
            (loop(sets[w]) if mode == "loop" else b.run(sets[w], graph=(mode == "graph")))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            p = sets[args.warmup + k]
            ev = loop(p) if mode == "loop" else b.run(p, graph=(mode == "graph"))[0]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        results[mode] = (dt, ev)
    # one profiled eager batch: time per kernel kind
    ctx.set_option(qsv.OPT_PROFILE, 1)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(sets[0])
    t_prof = time.perf_counter() - t0
    kstats = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                  "GB_s": round((v["bytes"] / 1e9) / (v["ms"] / 1e3), 1) if v["ms"] > 0 else None}
              for k, v in ctx.kernel_stats().items()}
    ctx.set_option(qsv.OPT_PROFILE, 0)
    ev_loop = results["loop"][1]
    for mode in ("batch", "graph"):
        assert np.allclose(results[mode][1], ev_loop, atol=1e-10), mode
    n_grad = sum(c.n_params for c in cs)
    widths = [c.n_qubits for c in cs]
    for mode, (dt, _) in results.items():
        print(json.dumps({
            "metric": "batched VQE sweep throughput", "value": round(len(cs) / dt, 2), "unit": "circuits/s",
            "gradients_per_s": round(len(cs) / dt, 2), "grad_entries_per_s": round(n_grad / dt, 1),
            "ms_per_step": round(1e3 * dt, 3), "mode": mode, "steps": args.steps, "warmup": args.warmup,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{len(cs)} VQE-like circuits (RY + Givens layers x6), {min(widths)}-"
                                   f"{max(widths)} qubits, 200-term Pauli Hamiltonians, complex128: <H> and "
                                   f"adjoint gradient per circuit", "n_params_total": n_grad},
            "speedup_vs_loop": round(results["loop"][0] / dt, 2),
            **({"kernels_eager_batch": kstats, "profiled_batch_ms": round(1e3 * t_prof, 2)} if mode == "batch"
               else {})}), flush=True)
    b.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sections outside the headline: complex64, the 32q/33q layered U3 circuits, "
                         "the batched VQE sweep")
    ap.add_argument("--fusion", type=int, default=1)
    ap.add_argument("--tile-bits", type=int, default=0, help="qubits per LDS tile, one-vector passes (0: default)")
    ap.add_argument("--tile-bits-adj", type=int, default=0, help="qubits per LDS tile, adjoint passes (0: default)")
    ap.add_argument("--low-bits", type=int, default=0, help="coalescing low bits per tile (0: default)")
    ap.add_argument("--tile-ws", type=int, default=0, help="warp-specialised tile passes (QSV_OPT_TILE_WS)")
    ap.add_argument("--micro", action="store_true", help="per-kernel-class gate-apply bandwidth sweep")
    ap.add_argument("--micro-dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--nt", action="store_true", help="micro: non-temporal stores (QSV_OPT_NONTEMPORAL)")
    ap.add_argument("--dense-mfma", action="store_true", help="micro: 6-qubit unitaries on FP64 MFMA")
    ap.add_argument("--batch", action="store_true",
                    help="batched VQE sweep (512 circuits, 12-22 qubits): per-circuit loop vs batched launches "
                         "vs captured graph, circuits/s and gradients/s")
    ap.add_argument("--batch-circuits", type=int, default=512)
    ap.add_argument("--micro-tile", action="store_true", help="tile-pass cost structure sweep")
    ap.add_argument("--sweep", action="store_true",
                    help="per-wire gate sweep at --n qubits, --micro-dtype precision (one line per case)")
    ap.add_argument("--sweep-half-touch", action="store_true",
                    help="sweep: only the half-touch gates with low untouched/control bits")
    ap.add_argument("--sweep-markers", action="store_true",
                    help="sweep: a marker kernel before each case (splits counter profiles per case)")
    ap.add_argument("--sweep-reps", type=int, default=3)
    ap.add_argument("--micro-case", default="", help="run only this micro-tile case (layers on)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy one state-sized buffer device to device (the reference kernel that "
                         "scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU state-vector "
              f"sharding is described in the design notes and not implemented here", file=sys.stderr)
        sys.exit(2)

    if args.batch:
        batch_bench(args)
        return
    if args.micro_tile:
        micro_tile(args.n, only=args.micro_case, layer_modes=(1,) if args.micro_case else (1, 0))
        return
    if args.micro:
        micro(args.n, dtype_name=args.micro_dtype, nontemporal=args.nt, dense_mfma=args.dense_mfma)
        return
    if args.sweep:
        sweep(args.n, dtype_name=args.micro_dtype, reps=args.sweep_reps, only_half_touch=args.sweep_half_touch,
              markers=args.sweep_markers)
        return

    import torch
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W

    if args.copy_calibration:
        # a plain copy of 2^n complex128 values: its FETCH_SIZE / WRITE_SIZE
        # readings calibrate the counters against known bytes
        src = torch.zeros(1 << args.n, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    circ = W.config3(n=args.n)
    n = circ.n_qubits
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    ctx = qsv.Context(0, stream)
    ctx.set_option(qsv.OPT_FUSION, args.fusion)
    ctx.set_option(qsv.OPT_TILE_BITS, args.tile_bits)
    ctx.set_option(qsv.OPT_TILE_BITS_ADJ, args.tile_bits_adj)
    ctx.set_option(qsv.OPT_LOW_BITS, args.low_bits)
    ctx.set_option(qsv.OPT_TILE_WS, args.tile_ws)
    print(f"bench: {circ.name}, complex128, {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    h = qaoa_eval(ctx, circ, qsv.C128, args.steps, args.warmup)
    d = h["dom"]
    # measured HBM bytes per launch of the dominant kernel (FETCH_SIZE +
    # WRITE_SIZE, copy-kernel calibrated), valid only for the library source
    # the counters were taken on
    from paper_2403_02512_amd.rocprof_summary import read_traffic
    tr = None
    if n == 28 and not (args.tile_bits or args.tile_bits_adj or args.low_bits) and args.fusion and not args.tile_ws:
        tr = (read_traffic(os.path.join(ROOT, "profiles", "hbm_traffic_qaoa28_c128.txt")) or {}).get(d["kind"])
    roofline = {"bound": "hbm", "kernel": d["kind"], "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": tr,
                "alg_bytes_per_launch": d["bytes_per_launch"], "avg_launch_ms": d["avg_ms"]}

    extras = {}
    if not args.no_extras:
        print("bench: complex64 state, same workload", file=sys.stderr, flush=True)
        c64 = qaoa_eval(ctx, circ, qsv.C64, args.steps, args.warmup)
        extras["c64"] = {k: c64[k] for k in ("s_per_eval", "s_per_eval_no_events", "forward_s", "gates_per_s",
                                             "adjoint_over_forward", "errors_vs_oracle", "kernels")}
        extras["c64"]["dominant_kernel_frac_of_8TBs"] = round(c64["dom"]["gbs"] / HBM_PEAK_GBS, 4)
    ctx.release_workspace()
    if not args.no_extras and n == 28:
        extras["config5"] = config5_eval(ctx)
        extras["config4_batch"] = batch_eval(ctx)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline (bounded sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(circ)

    out = {
        "metric": METRIC, "value": round(h["s_per_eval"], 6), "unit": "s/eval", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * h["s_per_eval"], 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"QAOA MaxCut 3-regular graph, {n} qubits, p=4, complex128: forward + <H_C> + "
                               f"adjoint Jacobian", "n_qubits": n, "n_gates": len(circ.ops),
                   "n_params": circ.n_params, "n_terms": len(circ.observables[0].words), "precision": "c128",
                   "fusion": bool(args.fusion), "tile_bits": args.tile_bits or "default",
                   "tile_bits_adj": args.tile_bits_adj or "default", "low_bits": args.low_bits or "default",
                   "tile_ws": bool(args.tile_ws)},
        "roofline": roofline, "cpu_baseline": cpu,
        "ms_per_step_no_events": round(1e3 * h["s_per_eval_no_events"], 3),
        "forward_ms": round(1e3 * h["forward_s"], 3), "gates_per_s": h["gates_per_s"],
        "adjoint_over_forward": h["adjoint_over_forward"],
        "errors_vs_oracle": h["errors_vs_oracle"], "kernels": h["kernels"],
        "result": {"expval": h["expval"], "jac": h["jac"]},
        **extras,
    }
    if cpu:
        out["speedup_vs_oracle"] = round(cpu["value"] / h["s_per_eval"], 1)
    print(json.dumps(out), flush=True)


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _kernel_table(stats, steps):
    return {name: {"launches_per_step": s["launches"] / steps, "ms_per_step": round(s["ms"] / steps, 4),
                   "GB_s": round((s["bytes"] / 1e9) / (s["ms"] / 1e3), 1) if s["ms"] > 0 else None}
            for name, s in stats.items()}


def qaoa_eval(ctx, circ, dtype, steps, warmup):
    """The benchmark step (reset, 308-gate forward, <H_C> and the adjoint
    Jacobian) in one precision: the timed region with HIP events on the
    library's stream around every launch (per-kernel durations for the
    roofline), the same steps without events, forward-only steps (gates/s),
    and the errors of <H_C> and the gradient against the FP64 oracle's values
    for this workload."""
    import torch
    from paper_2403_02512_amd import qsv
    n = circ.n_qubits
    tdt = torch.complex128 if dtype == qsv.C128 else torch.complex64
    psi = torch.empty(1 << n, dtype=tdt, device="cuda")
    st = qsv.State(ctx, n, dtype, tensor=psi)
    m_ops = qsv.MarshalledOps(circ.ops, circ.params)
    m_obs = qsv.MarshalledObs(circ.observables)

    def forward():
        st.reset(0)
        qsv.apply(st, circ.ops, circ.params, marshalled=m_ops)

    def step():
        forward()
        return qsv.adjoint_jacobian(st, circ.ops, circ.params, circ.observables, marshalled=m_ops,
                                    marshalled_obs=m_obs)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, r

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_option(qsv.OPT_PROFILE, 1)
    ctx.reset_stats()
    s_eval, (jac, ev) = timed(step, steps)
    stats = ctx.kernel_stats()
    ctx.set_option(qsv.OPT_PROFILE, 0)
    s_eval_ne, _ = timed(step, steps)
    s_fwd, _ = timed(forward, steps)
    dom = max(stats, key=lambda k: stats[k]["ms"])
    d = stats[dom]
    out = {"s_per_eval": s_eval, "s_per_eval_no_events": s_eval_ne, "forward_s": s_fwd,
           "gates_per_s": round(len(circ.ops) / s_fwd, 1),
           "adjoint_over_forward": round((s_eval_ne - s_fwd) / s_fwd, 3),
           "kernels": _kernel_table(stats, steps), "expval": float(ev[0]), "jac": [float(x) for x in jac[0]],
           "dom": {"kind": dom, "gbs": (d["bytes"] / 1e9) / (d["ms"] / 1e3), "bytes_per_launch": d["bytes"] / d["launches"],
                   "avg_ms": d["ms"] / d["launches"]}}
    g = _golden("config3") if n == 28 else None
    if g is not None:
        s = float(np.sum(np.abs(circ.observables[0].coeffs)))
        # reading of the tolerance: <H> relative to sum |c_t|; a gradient entry
        # relative to sum |c_t| times sum over its slots of 2 |scale|
        per_p = np.zeros(circ.n_params)
        for o in circ.ops:
            for p, sc in zip(o.param, o.scale):
                if p >= 0:
                    per_p[p] += 2 * abs(sc)
        bound = s * np.maximum(per_p, 1.0)
        out["errors_vs_oracle"] = {
            "err_expval_rel": float(abs(ev[0] - g["expval"][0]) / s),
            "err_jac_rel": float(np.max(np.abs(jac[0] - np.array(g["jac"][0])) / bound)),
            "tolerance": 1e-12 if dtype == qsv.C128 else 1e-5,
            "oracle": "tests/golden/config3_oracle.json (FP64 oracle, same seeded workload)"}
    else:
        out["errors_vs_oracle"] = None
    st.close()
    del psi
    torch.cuda.empty_cache()
    return out


def config5_eval(ctx):
    """Layered U3 + CNOT brick wall (20 layers): the 33-qubit complex64
    forward (<Z_0 Z_32>) and the 32-qubit complex128 forward and adjoint
    Jacobian (<Z_0 Z_31>, 1920 parameters; psi, phi and lambda = 192 GiB).
    One untimed run each first.  No host oracle fits these sizes: the
    full-size tests pin them by product, mirror and GHZ properties."""
    import torch
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W
    out = {}
    for n, dt in ((33, qsv.C64), (32, qsv.C128)):
        c = W.config5(n=n)
        print(f"bench: {c.name}, {'complex64 forward' if dt == qsv.C64 else 'complex128 forward + Jacobian'}",
              file=sys.stderr, flush=True)
        st = qsv.State(ctx, n, dt)
        m_ops = qsv.MarshalledOps(c.ops, c.params)
        m_obs = qsv.MarshalledObs(c.observables)
        rec = {"n_qubits": n, "dtype": "c64" if dt == qsv.C64 else "c128", "n_gates": len(c.ops),
               "n_params": c.n_params}
        for rep in range(2):
            st.reset(0)
            ctx.synchronize()
            t0 = time.perf_counter()
            qsv.apply(st, c.ops, c.params, marshalled=m_ops)
            ctx.synchronize()
            t_fwd = time.perf_counter() - t0
            if dt == qsv.C64:
                ev = qsv.expval(st, c.observables, marshalled=m_obs)
                t_jac = None
            else:
                t0 = time.perf_counter()
                jac, ev = qsv.adjoint_jacobian(st, c.ops, c.params, c.observables, inplace=True,
                                               marshalled=m_ops, marshalled_obs=m_obs)
                t_jac = time.perf_counter() - t0
        rec["forward_s"] = round(t_fwd, 4)
        rec["gates_per_s"] = round(len(c.ops) / t_fwd, 1)
        rec["expval"] = float(ev[0])
        if t_jac is not None:
            rec["adjoint_s"] = round(t_jac, 4)
            rec["jacobian_s_per_eval"] = round(t_fwd + t_jac, 4)
            rec["adjoint_over_forward"] = round(t_jac / t_fwd, 3)
        out[f"{n}q_{rec['dtype']}"] = rec
        st.close()
        ctx.release_workspace()
        torch.cuda.empty_cache()
    return out


def batch_eval(ctx, n_circuits=512, steps=3):
    """Batched VQE sweep (512 circuits, 12-22 qubits, 200-term Hamiltonians,
    complex128): <H> and the full adjoint gradient of every circuit per step,
    new angles each step; the batched launches replayed from a captured HIP
    graph against a loop over the single-circuit entry points."""
    from paper_2403_02512_amd import qsv
    from paper_2403_02512_amd import workloads as W
    print(f"bench: batched VQE sweep, {n_circuits} circuits", file=sys.stderr, flush=True)
    cs = W.config4(n_circuits=n_circuits)
    rng = np.random.default_rng(7)
    sets = [[rng.uniform(0, 2 * np.pi, c.n_params) for c in cs] for _ in range(steps + 1)]
    b = qsv.Batch(ctx, cs)
    b.run(sets[0], graph=True)
    ctx.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev, _ = b.run(sets[k + 1], graph=True)
    ctx.synchronize()
    dt_graph = (time.perf_counter() - t0) / steps
    b.close()
    states = {}
    for c in cs:
        if c.n_qubits not in states:
            states[c.n_qubits] = qsv.State(ctx, c.n_qubits)
    marsh = [(qsv.MarshalledOps(c.ops, c.params), qsv.MarshalledObs(c.observables[:1])) for c in cs]
    ev_loop = np.zeros(len(cs))
    ctx.synchronize()
    t0 = time.perf_counter()
    for i, c in enumerate(cs):
        st = states[c.n_qubits]
        st.reset(0)
        m = marsh[i][0]
        m.params[:c.n_params] = sets[steps][i]
        qsv.apply(st, c.ops, marshalled=m)
        _, e = qsv.adjoint_jacobian(st, c.ops, None, None, inplace=True, marshalled=m, marshalled_obs=marsh[i][1])
        ev_loop[i] = e[0]
    ctx.synchronize()
    dt_loop = time.perf_counter() - t0
    for st in states.values():
        st.close()
    ctx.release_workspace()
    assert np.allclose(ev, ev_loop, atol=1e-10)
    n_grad = sum(c.n_params for c in cs)
    return {"circuits": len(cs), "widths": [min(c.n_qubits for c in cs), max(c.n_qubits for c in cs)],
            "graph_circuits_per_s": round(len(cs) / dt_graph, 1), "graph_gradients_per_s": round(len(cs) / dt_graph, 1),
            "graph_grad_entries_per_s": round(n_grad / dt_graph, 1),
            "loop_circuits_per_s": round(len(cs) / dt_loop, 1), "speedup_vs_loop": round(dt_loop / dt_graph, 2),
            "note": "each circuit: <H> of a 200-term Pauli sum and its full adjoint gradient"}


if __name__ == "__main__":
    main()
