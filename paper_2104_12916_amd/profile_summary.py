"""Summaries of rocprofv3 output for the profiles/ folder.

  stats    kernel-stats CSV (rocprofv3 --kernel-trace --stats -f csv) -> markdown
           table of the top kernels with the command that produced it
  traffic  FETCH_SIZE and WRITE_SIZE counter CSVs of one profile_ops run
           (rocprofv3 --pmc, one counter per run) -> per-launch HBM bytes of
           the CG-step sweeps, scaled by what the same counters read for the
           run's calibration copy of known size, stored in profiles/traffic.json
           with the hash of the kernel sources they were taken on
  mfma     counter CSV of one rocprofv3 --pmc run with MfmaUtil and MfmaFlopsF64
           (plus its kernel trace for the durations) -> markdown table of the
           FP64 matrix-core use of each kernel

Usage:
  python -m paper_2104_12916_amd.profile_summary stats CSV OUT.md --title T --cmd C [--note N] [--top 14]
  python -m paper_2104_12916_amd.profile_summary traffic --fetch F.csv --write W.csv --workload lowdof
  python -m paper_2104_12916_amd.profile_summary mfma --counters C.csv --trace T.csv OUT.md --title T --cmd C
"""
import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 256 << 20  # the calibration copy of profile_ops

# CG-step sweeps of the float64 single-QP path: tag -> kernel name prefixes (C^T p
# and M^T v are row sweeps over stored transposes, or column sweeps)
SWEEPS = {
    "C^T": ("qpg::gemv_rows_kernel<double, 1,", "qpg::gemv_cols_part_kernel<double, 1,"),
    "M": ("qpg::gemv_rows_kernel<double, 2,",),
    "M^T": ("qpg::gemv_rows_kernel<double, 3,", "qpg::gemv_cols_part_kernel<double, 3,"),
    "M1": ("qpg::k0_sym_kernel<double,",),          # one pass over M: M^T Sigma M u
    "M1red": ("qpg::k0_sym_reduce_kernel<double>",),  # sum of its per-workgroup partials
    "q": ("qpg::pcg_q_kernel<double,",),
    # the folded CG step's kernels (same matrices, with the vector update folded in)
    "C^T fold": ("qpg::fold_ct_kernel<double,",),
    "M1red fold": ("qpg::k0_sym_reduce_fold_kernel<double>",),
    "q fold": ("qpg::fold_q_kernel<double,",),
}


def kernel_src_hash():
    """Hash of the sources of the sweep kernels and of their launch-shape table
    (counters go stale when either changes)."""
    h = hashlib.sha256()
    for f in ("csrc/gemv.hip", "csrc/gemv_core.hpp", "csrc/pcg.hip", "csrc/common.hpp", "csrc/tune.hip",
              "autotune_gfx950.txt"):
        path = os.path.join(HERE, f)
        if os.path.exists(path):
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n, m1, m2, elem=8):
    """Matrix bytes one launch of each sweep must read: C is m2 x n, M = L^{-1}[:, :n]
    is the lower trapezoid of n(n+1)/2 + m1 n entries."""
    mm = n * (n + 1) // 2 + m1 * n
    return {"C^T": m2 * n * elem, "M": mm * elem, "M^T": mm * elem, "M1": mm * elem, "M1red": 0,
            "q": m2 * n * elem, "C^T fold": m2 * n * elem, "M1red fold": 0, "q fold": m2 * n * elem}


def _short(name):
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "").replace("qpg::", "").strip()


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {args.title}", "", "Command (run from the repository root on one MI355X):", "", "```", args.cmd, "```",
             ""]
    if args.note:
        lines += [args.note, ""]
    lines += [f"Total kernel time {total / 1e6:.1f} ms over {sum(int(r['Calls']) for r in rows)} dispatches.", "",
              "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:args.top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{100 * float(r['TotalDurationNs']) / total:.2f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counters(path):
    rows = list(csv.DictReader(open(path)))
    return {int(r["Dispatch_Id"]): r for r in rows}


def traffic(args):
    sys.path.insert(0, ROOT)
    import synth
    fetch, write = _counters(args.fetch), _counters(args.write)
    # calibration: the largest copyBuffer dispatch writes COPY_BYTES
    copies = [d for d, r in write.items() if "copyBuffer" in r["Kernel_Name"]]
    cal = max(copies, key=lambda d: float(write[d]["Counter_Value"]))
    w_scale = COPY_BYTES / (float(write[cal]["Counter_Value"]) * 1024)
    f_scale = COPY_BYTES / (float(fetch[cal]["Counter_Value"]) * 1024)
    w = synth.WORKLOADS[args.workload]
    alg = algorithmic_bytes(w["n"], w["m1"], w["m2"])
    path = os.path.join(ROOT, "profiles", "traffic.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    src = kernel_src_hash()
    for tag, prefixes in SWEEPS.items():
        ids = [d for d, r in fetch.items()
               if any(r["Kernel_Name"].startswith(pre) or r["Kernel_Name"].startswith("void " + pre)
                      for pre in prefixes)]
        if not ids:
            continue
        fk = sum(float(fetch[d]["Counter_Value"]) for d in ids) / len(ids)
        wk = sum(float(write[d]["Counter_Value"]) for d in ids if d in write) / len(ids)
        out[f"{args.workload}:{tag}"] = {
            "kernel": _short(fetch[ids[0]]["Kernel_Name"]), "src_hash": src, "dispatches": len(ids),
            "bytes_per_launch": int(round(fk * 1024 * f_scale + wk * 1024 * w_scale)),
            "fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1),
            "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
            "algorithmic_bytes": alg[tag],
            "note": ("rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, over profile_ops; scaled by what the counters "
                     f"read for the run's {COPY_BYTES >> 20} MiB calibration copy"),
        }
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


FP64_PEAK = 78.6e12  # dense FP64 MFMA, flop/s


def mfma(args):
    """Per kernel and grid size: dispatches, average duration, MFMA flops per dispatch
    (MfmaFlopsF64), achieved rate and its share of the FP64 peak, and MfmaUtil
    (matrix-core busy cycles over active cycles of all SIMDs)."""
    vals = {}
    names = {}
    for r in csv.DictReader(open(args.counters)):
        d = int(r["Dispatch_Id"])
        vals.setdefault(d, {})[r["Counter_Name"]] = float(r["Counter_Value"])
        names[d] = (r["Kernel_Name"], int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"])))
    dur = {}
    for r in csv.DictReader(open(args.trace)):
        dur[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    per = {}
    for d, v in vals.items():
        if "MfmaFlopsF64" not in v or v["MfmaFlopsF64"] <= 0 or d not in dur:
            continue
        k = (_short(names[d][0]), names[d][1])
        e = per.setdefault(k, {"n": 0, "t": 0.0, "fl": 0.0, "util": 0.0})
        e["n"] += 1
        e["t"] += dur[d]
        e["fl"] += v["MfmaFlopsF64"]
        e["util"] += v.get("MfmaUtil", float("nan"))
    lines = [f"# {args.title}", "", "Command (run from the repository root on one MI355X):", "", "```", args.cmd, "```",
             ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["| kernel | workgroups | dispatches | avg us | MFMA GFLOP per dispatch | TF/s | of 78.6 TF/s | MfmaUtil % |",
              "|---|---|---|---|---|---|---|---|"]
    for (k, wg), e in sorted(per.items(), key=lambda kv: -kv[1]["t"]):
        t, fl = e["t"] / e["n"], e["fl"] / e["n"]
        lines.append(f"| `{k}` | {wg} | {e['n']} | {t * 1e6:.1f} | {fl / 1e9:.3f} | {fl / t / 1e12:.1f} | "
                     f"{100 * fl / t / FP64_PEAK:.1f} % | {e['util'] / e['n']:.1f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--title", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--note", default="")
    a.add_argument("--top", type=int, default=14)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--workload", default="lowdof")
    c = sub.add_parser("mfma")
    c.add_argument("out")
    c.add_argument("--counters", required=True)
    c.add_argument("--trace", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--note", default="")
    args = ap.parse_args()
    if args.cmd_name == "stats":
        stats(args)
    elif args.cmd_name == "mfma":
        mfma(args)
    else:
        traffic(args)


if __name__ == "__main__":
    main()
