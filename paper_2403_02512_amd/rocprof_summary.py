"""Short text summaries of rocprofv3 CSV output.

  python -m paper_2403_02512_amd.rocprof_summary stats <run_kernel_stats.csv> --cmd "<command>"
      per-kernel launch count, total and average duration (markdown table)

  python -m paper_2403_02512_amd.rocprof_summary traffic <fetch counter csv> <write counter csv>
      --copy-bytes B --cmd "<commands>"
      HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch), each scaled by the factor that makes the runtime's copy
      kernel (__amd_rocclr_copyBuffer, which moves B bytes each way) read and
      write exactly B bytes; one machine-readable line per kernel, plus one
      SHA-1 over every source file of the library (kernels, planner,
      lowering, gate tables), so that a change to any of them, and with it
      possibly the launched programs, retires the counters.

  python -m paper_2403_02512_amd.rocprof_summary sweep-traffic <fetch csv> <write csv> <sweep log>
      --reps R --cmd "<commands>"
      counter bytes beside algorithmic bytes per case of a per-wire sweep
      (bench.py --sweep --sweep-markers), calibrated by a state copy

  python -m paper_2403_02512_amd.rocprof_summary counters <pmc csv>... --elements N --cmd "<commands>"
      mean SQ counter values per dispatch and kernel, instructions per amplitude

  python -m paper_2403_02512_amd.rocprof_summary sweep-table <sweep log> --cmd "<command>"
      per-wire fractions of the HBM peak from a sweep's JSON lines
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

KINDS = [("k_tile<double, true", "tile2"), ("k_tile_lamz<double", "tile2"), ("k_tile_lamz<float", "tile2_c64"),
         ("k_tile<double, false", "tile1"), ("k_tile<float, true", "tile2_c64"),
         ("k_tile<float, false", "tile1_c64"), ("k_pauli<double, true", "pauli_lambda"),
         ("k_pauli<double, false", "pauli"), ("__amd_rocclr_copyBuffer", "copy"), ("k_init", "init"),
         ("k_reduce", "reduce"), ("k_gate1", "gate1"), ("k_diag1", "diag1"), ("k_gate2", "gate2"),
         ("k_gatek", "gatek")]


def source_sha1(root: str = CSRC) -> str:
    """SHA-1 over the names and contents of every file under csrc/, in
    sorted order."""
    h = hashlib.sha1()
    for name in sorted(os.listdir(root)):
        p = os.path.join(root, name)
        if not os.path.isfile(p):
            continue
        h.update(name.encode() + b"\0")
        with open(p, "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("qsv::", "")


def kind_of(name: str) -> str:
    for pat, k in KINDS:
        if pat in name:
            return k
    return "other"


def stats(path: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"command: {cmd}", "", "| kernel | kind | calls | total ms | avg us | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {kind_of(r['Name'])} | {r['Calls']} | "
                   f"{int(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
    return vals


def traffic(fetch_csv: str, write_csv: str, copy_bytes: float, cmd: str) -> str:
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    cp = [k for k in fetch if "copyBuffer" in k]
    if not cp:
        raise SystemExit("no copy kernel in the counter data: cannot calibrate")
    # the copy runs as several dispatches, only one of which moves the data
    f_scale = copy_bytes / max(fetch[cp[0]])
    w_scale = copy_bytes / max(write[cp[0]])
    out = [f"commands: {cmd}",
           f"calibration: copy kernel moving {copy_bytes:.0f} B each way reads FETCH_SIZE "
           f"{max(fetch[cp[0]]):.0f} B and WRITE_SIZE {max(write[cp[0]]):.0f} B -> "
           f"fetch_scale={f_scale:.4f} write_scale={w_scale:.4f}",
           f"library_source_sha1={source_sha1()}", ""]
    for k in fetch:
        if k not in write or "copyBuffer" in k:
            continue
        f = sum(fetch[k]) / len(fetch[k]) * f_scale
        w = sum(write[k]) / len(write[k]) * w_scale
        out.append(f"kind={kind_of(k)} kernel={short(k).replace(' ', '')} dispatches={len(fetch[k])} "
                   f"fetch_bytes={f:.4e} write_bytes={w:.4e} traffic_bytes={f + w:.4e}")
    return "\n".join(out) + "\n"


def _dispatches(path: str, counter: str):
    """(dispatch id, kernel name, bytes) of one counter, in dispatch order."""
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
    out.sort()
    return out


def sweep_traffic(fetch_csv: str, write_csv: str, sweep_log: str, reps: int, cmd: str) -> str:
    """Counter bytes per case of a per-wire sweep run with markers: the first
    reps x (launches per apply) library dispatches after each case's marker
    (a torch fill kernel) are that case's timed launches; each counter is scaled by the factor that
    makes the state copy (the copy kernel before the first case) move exactly
    the state's bytes; beside them, the algorithmic bytes of the case."""
    import json
    cases = [json.loads(x) for x in open(sweep_log) if x.startswith('{"case"')]
    cols = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = _dispatches(path, counter)
        cp = [v for _, k, v in d if "copyBuffer" in k]
        if not cp or not cases:
            raise SystemExit("no copy kernel or no cases: cannot calibrate")
        n, dt = cases[0]["n_qubits"], cases[0]["dtype"]
        state_bytes = float(1 << n) * (16 if dt == "c128" else 8)
        scale = state_bytes / max(cp)
        per_case, cur, calibrated = [], None, False
        for _, k, v in d:
            if "copyBuffer" in k and v == max(cp):
                calibrated = True  # markers follow the calibration copy
            elif calibrated and "FillFunctor" in k:
                cur = []
                per_case.append(cur)
            elif cur is not None and "qsv::" in k:
                cur.append(v * scale)
        cols[counter] = (scale, per_case)
    fs, fc = cols["FETCH_SIZE"]
    ws, wc = cols["WRITE_SIZE"]
    out = [f"commands: {cmd}",
           f"calibration: the state copy reads and writes {state_bytes:.0f} B: fetch_scale={fs:.4f} "
           f"write_scale={ws:.4f}", f"library_source_sha1={source_sha1()}", "",
           "| case | alg GB | counter GB (fetch + write) | ratio | ms | counter GB/s |", "|---|---|---|---|---|---|"]
    for c, f, w in zip(cases, fc, wc):
        # the case's timed launches follow its marker; the next case's
        # warm-up launch comes before the next marker
        k = reps * sum(c["kernels"].values())
        fb, wb = sum(f[:k]) / reps, sum(w[:k]) / reps
        tot = (fb + wb) / 1e9
        out.append(f"| {c['case']} | {c['alg_GB']:.3f} | {tot:.3f} ({fb / 1e9:.3f} + {wb / 1e9:.3f}) | "
                   f"{tot / c['alg_GB']:.2f} | {c['ms']:.3f} | {tot / (c['ms'] / 1e3):.0f} |")
    return "\n".join(out) + "\n"


def sweep_table(sweep_log: str, cmd: str) -> str:
    """Markdown tables of a per-wire sweep (bench.py --sweep): per gate the
    fraction of the 8 TB/s HBM peak (algorithmic bytes / HIP-event time) on
    every wire or wire pair, then the per-gate summary lines."""
    import json
    rows = [json.loads(x) for x in open(sweep_log) if x.startswith('{"case"')]
    summ = [json.loads(x) for x in open(sweep_log) if x.startswith('{"summary"')]
    if not rows:
        raise SystemExit("no sweep cases in the log")
    n, dt = rows[0]["n_qubits"], rows[0]["dtype"]
    out = [f"command: {cmd}", "", f"{n} qubits, {dt}: fraction of 8 TB/s (algorithmic bytes / kernel time)", ""]
    by = collections.OrderedDict()
    for r in rows:
        g, where = r["case"].split(" ", 1)
        by.setdefault((r["class"], g), collections.OrderedDict())[where] = r
    for cls, label in (("1q", "bit"), ("2q", "bits")):
        gates = [g for (c, g) in by if c == cls]
        if not gates:
            continue
        keys = list(by[(cls, gates[0])].keys())
        out.append("| " + label + " | " + " | ".join(gates) + " |")
        out.append("|---" * (len(gates) + 1) + "|")
        for k in keys:
            cells = [f"{by[(cls, g)][k]['frac_of_8TBs']:.3f}" if k in by[(cls, g)] else "" for g in gates]
            out.append(f"| {k.replace(label, '')} | " + " | ".join(cells) + " |")
        out.append("")
    dense = [r for r in rows if r["class"] == "dense"]
    if dense:
        out += ["| dense unitary | kernel | ms | frac |", "|---|---|---|---|"]
        for r in dense:
            out.append(f"| {r['case']} | {','.join(r['kernels'])} | {r['ms']:.3f} | {r['frac_of_8TBs']:.3f} |")
        out.append("")
    out += ["| gate | cases | min | median | max |", "|---|---|---|---|---|"]
    for s_ in summ:
        out.append(f"| {s_['summary']} | {s_['cases']} | {s_['frac_min']:.3f} | {s_['frac_median']:.3f} | "
                   f"{s_['frac_max']:.3f} |")
    return "\n".join(out) + "\n"


def counters(csvs, elements: float, cmd: str) -> str:
    """Mean per dispatch of every SQ counter in the given --pmc runs, per
    kernel kind, and per-amplitude instruction counts (wave instructions x 64
    lanes / elements; elements = amplitude indices one dispatch covers)."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in csvs:
        for r in csv.DictReader(open(path)):
            vals[kind_of(r["Kernel_Name"]) + " " + short(r["Kernel_Name"]).replace(" ", "")][r["Counter_Name"]].append(
                float(r["Counter_Value"]))
    out = [f"commands: {cmd}", f"elements per dispatch: {elements:.0f}", "",
           "| kernel | counter | dispatches | mean per dispatch | x64 / elements |", "|---|---|---|---|---|"]
    for k in sorted(vals):
        if not k.startswith(("tile", "pauli", "init")):
            continue
        for cn in sorted(vals[k]):
            v = vals[k][cn]
            m = sum(v) / len(v)
            per = f"{m * 64 / elements:.2f}" if cn.startswith("SQ_INSTS") else ""
            out.append(f"| {k} | {cn} | {len(v)} | {m:.4e} | {per} |")
    return "\n".join(out) + "\n"


def read_traffic(path: str):
    """{kind: traffic bytes per dispatch} if the summary was taken on the
    current library sources, else None."""
    if not os.path.exists(path):
        return None
    tot, cnt, sha = collections.defaultdict(float), collections.defaultdict(int), None
    for line in open(path):
        if line.startswith("library_source_sha1="):
            sha = line.strip().split("=", 1)[1]
        elif line.startswith("kind="):
            # one line per kernel; a kind with several kernels (the first
            # reverse pass's form) averages over all their dispatches
            d = dict(x.split("=", 1) for x in line.split())
            k = int(d.get("dispatches", 1))
            tot[d["kind"]] += float(d["traffic_bytes"]) * k
            cnt[d["kind"]] += k
    if sha != source_sha1():
        return None
    return {k: tot[k] / cnt[k] for k in tot}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--cmd", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--cmd", required=True)
    c = sub.add_parser("sweep-traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("sweep_log")
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--cmd", required=True)
    q = sub.add_parser("counters")
    q.add_argument("csv", nargs="+")
    q.add_argument("--elements", type=float, required=True)
    q.add_argument("--cmd", required=True)
    t = sub.add_parser("sweep-table")
    t.add_argument("sweep_log")
    t.add_argument("--cmd", required=True)
    args = ap.parse_args(argv)
    if args.mode == "stats":
        sys.stdout.write(stats(args.csv, args.cmd))
    elif args.mode == "counters":
        sys.stdout.write(counters(args.csv, args.elements, args.cmd))
    elif args.mode == "sweep-table":
        sys.stdout.write(sweep_table(args.sweep_log, args.cmd))
    elif args.mode == "sweep-traffic":
        sys.stdout.write(sweep_traffic(args.fetch_csv, args.write_csv, args.sweep_log, args.reps, args.cmd))
    else:
        sys.stdout.write(traffic(args.fetch_csv, args.write_csv, args.copy_bytes, args.cmd))


if __name__ == "__main__":
    main()
