"""Summaries of rocprofv3 output for the H.V kernel.

* kernel-trace statistics (``--kernel-trace --stats --output-format csv``):
  a table of the kernels by total time;
* HBM traffic of the H.V kernel from two counter runs (``--pmc FETCH_SIZE``
  and ``--pmc WRITE_SIZE`` of ``bench.py --profile-hv``): each counter is
  scaled by what it reads for the 1 GiB device copy that the profile run does
  first, and averaged over the H.V launches that follow the copy.

Usage (after the rocprofv3 runs):
  python -m paper_2607_17429_amd.profiling --stats DIR/trace_kernel_stats.csv \\
      --fetch DIR/fetch_counter_collection.csv --write DIR/write_counter_collection.csv \\
      --workload icosidodecahedron_Hg --out profiles --cmd "<the rocprofv3 commands>"
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that decide what the H.V kernel reads: the kernel, its launch, the
# entry table format and the Lanczos driver that calls it
HV_SOURCES = ("csrc/hv_kernel.h", "csrc/hv.hip", "csrc/sector.hip", "csrc/lanczos.hip")


def hv_source_sha() -> str:
    h = hashlib.sha256()
    for rel in HV_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_stats_markdown(stats_csv: str, top: int = 14) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def lanczos_hv(trace_csv: str, first: int = 0, match: str = ""):
    """(count, avg ms, kernel name) of the H.V dispatches made by ftlm_run: those
    that the Lanczos alpha reduction follows on the same queue.  With match only
    kernels whose name contains it count.  With first > 0 only the first
    `first` such launches (in time order) of the most frequent remaining H.V
    kernel count: with the blocks of a job run in irrep order, the run of the
    roofline block when the blocks before it take other kernel shapes."""
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    by_q = {}
    for r in rows:
        by_q.setdefault(r["Queue_Id"], []).append(r)
    picked = []
    for q in by_q.values():
        for a, b in zip(q, q[1:]):
            if "k_hv<" in a["Kernel_Name"] and "k_alpha" in b["Kernel_Name"] and match in a["Kernel_Name"]:
                picked.append(a)
    if not picked:
        return 0, None, None
    if first:
        names = {}
        for r in picked:
            names[r["Kernel_Name"]] = names.get(r["Kernel_Name"], 0) + 1
        top = max(names, key=names.get)
        picked = sorted((r for r in picked if r["Kernel_Name"] == top), key=lambda r: int(r["Start_Timestamp"]))[:first]
    ms = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in picked) / len(picked) / 1e6
    return len(picked), ms, picked[0]["Kernel_Name"]


def _dispatches(path):
    return list(csv.DictReader(open(path)))


def counter_traffic(fetch_csv: str, write_csv: str, copy_bytes: int = 1 << 30, kernel_prefix: str = "void ftlm::hvk::k_hv"):
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _dispatches(path)
        copy_idx = [i for i, r in enumerate(rows) if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) > 1e5]
        if not copy_idx:
            raise RuntimeError(f"no calibration copy in {path}")
        ci = copy_idx[-1]
        copy_kib = float(rows[ci]["Counter_Value"])
        scale = copy_bytes / (copy_kib * 1024.0)
        hv = [r for r in rows[ci + 1:] if r["Kernel_Name"].startswith(kernel_prefix)]
        if not hv:
            raise RuntimeError(f"no H.V dispatch after the copy in {path}")
        kib = sum(float(r["Counter_Value"]) for r in hv) / len(hv)
        ms = sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in hv) / len(hv) / 1e6
        res[name] = dict(raw_kib_per_launch=kib, copy_raw_kib=copy_kib, scale=scale,
                         bytes_per_launch=kib * 1024.0 * scale, launches=len(hv), avg_ms_under_counters=ms,
                         kernel=hv[0]["Kernel_Name"])
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", default="profiles")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--bench-json", default=None, help="bench.py output line, for the algorithmic bytes")
    ap.add_argument("--trace", default=None, help="kernel_trace.csv of the trace run (H.V launches inside ftlm_run)")
    ap.add_argument("--first", type=int, default=0,
                    help="count only the first N in-run launches of the most frequent H.V kernel (the roofline block)")
    ap.add_argument("--hv-json", default=None,
                    help="stdout of the counter run (bench.py --profile-hv), for the gather-efficiency figures")
    ap.add_argument("--match", default="", help="count only H.V kernels whose name contains this")
    ap.add_argument("--step-cmd", default="bench.py --steps 1 --warmup 0 --no-cpu-baseline",
                    help="the bench command of the trace run, for the summary's heading")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    tr = counter_traffic(args.fetch, args.write)
    total = tr["FETCH_SIZE"]["bytes_per_launch"] + tr["WRITE_SIZE"]["bytes_per_launch"]
    balg = None
    if args.bench_json:
        bj = json.loads(open(args.bench_json).read().strip().splitlines()[-1])
        balg = bj["roofline"]["algorithmic_bytes_per_launch"]
    rec = dict(source_sha=hv_source_sha(), bytes_per_launch=total, fetch=tr["FETCH_SIZE"], write=tr["WRITE_SIZE"],
               algorithmic_bytes_per_launch=balg, command=args.cmd)
    with open(os.path.join(args.out, f"hv_traffic_{args.workload}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    md = [f"# k_hv on {args.workload}: rocprofv3 summary", "",
          "Commands (from the repository root):", "", "```", args.cmd, "```", "",
          f"## Kernel trace statistics (one bench step, `{args.step_cmd}`)", "",
          kernel_stats_markdown(args.stats), ""]
    if args.trace:
        n, ms, name = lanczos_hv(args.trace, args.first, args.match)
        if n:
            which = (f"the first {n} of the most frequent H.V kernel"
                     + (f" whose name contains `{args.match}`" if args.match else "")
                     + ", i.e. the roofline block's run" if args.first else f"{n}")
            md += [f"H.V launches inside `ftlm_run` (each followed by `k_alpha` on its queue): {which}, "
                   f"average {ms:.3f} ms (`{name[:90]}`).", ""]
            if args.bench_json:
                bj = json.loads(open(args.bench_json).read().strip().splitlines()[-1])
                md += [f"The bench line of the same run (HIP events on the launch stream): "
                       f"{bj['roofline']['avg_launch_ms']:.3f} ms per launch over {bj['roofline']['launches']} launches.", ""]
    md += [
          "## HBM traffic of one H.V launch inside `ftlm_run` (`bench.py --profile-hv`)", "",
          "| counter | raw KiB / launch | calibration (1 GiB copy) raw KiB | scale | bytes / launch |",
          "|---|---:|---:|---:|---:|"]
    for k in ("FETCH_SIZE", "WRITE_SIZE"):
        t = tr[k]
        md.append(f"| {k} | {t['raw_kib_per_launch']:.0f} | {t['copy_raw_kib']:.0f} | {t['scale']:.3f} | "
                  f"{t['bytes_per_launch'] / 1e9:.3f} GB |")
    md.append(f"| total | | | | {total / 1e9:.3f} GB |")
    if balg:
        md += ["", f"Algorithmic bytes per launch (byte model): {balg / 1e9:.3f} GB; "
                   f"measured / algorithmic = {total / balg:.3f}."]
    if args.hv_json:
        hj = None
        for line in open(args.hv_json):
            if line.startswith('{"copy_bytes"'):
                hj = json.loads(line)
        if hj:
            st = hj["stats"]
            conn, act = st["connections"], st["active_connections"]
            useful = st["gathered_rows"] * hj["nvec"] * hj["elem_bytes"]
            fetch = tr["FETCH_SIZE"]["bytes_per_launch"]
            rec["gather"] = dict(layout=hj["layout"], connections=conn, active_connections=act,
                                 useful_slice_bytes=useful, fetch_bytes_per_connection=fetch / conn,
                                 useful_bytes_per_active_connection=useful / max(act, 1),
                                 gather_efficiency=useful / fetch)
            with open(os.path.join(args.out, f"hv_traffic_{args.workload}.json"), "w") as f:
                json.dump(rec, f, indent=1)
            md += ["", f"Gather efficiency ({hj['layout']} rows, {hj['nvec']} vectors of {hj['elem_bytes']} B): "
                       f"{conn:,} connections ({act:,} with an active target) per launch; the useful X slices "
                       f"are {useful / 1e9:.3f} GB ({useful / max(act, 1):.1f} B per active connection); "
                       f"FETCH_SIZE is {fetch / conn:.1f} B per connection; useful slice bytes / fetched bytes "
                       f"= {useful / fetch:.3f}."]
    md += ["", f"Kernel source hash ({' + '.join(os.path.basename(p) for p in HV_SOURCES)}): `{rec['source_sha']}`", ""]
    with open(os.path.join(args.out, f"k_hv_{args.workload}.md"), "w") as f:
        f.write("\n".join(md))
    print(json.dumps({"traffic_bytes_per_launch": total, "algorithmic": balg}))


if __name__ == "__main__":
    main()
