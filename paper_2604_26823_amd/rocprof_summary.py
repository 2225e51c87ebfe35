"""Short text summaries of rocprofv3 output for profiles/.

  python -m paper_2604_26823_amd.rocprof_summary stats <kernel_stats.csv> --command CMD --out F
      per-kernel calls / total / average duration from a --kernel-trace --stats run;
  python -m paper_2604_26823_amd.rocprof_summary traffic --fetch A --write B --tag fp32 \\
          --command CMD --out F
      HBM bytes per launch from two --pmc runs (FETCH_SIZE, then WRITE_SIZE), each
      scaled by what the same counter reads for the largest device copy in the run
      (a copy of known size: bench.py --copy-mib), with the digest of the sources the
      counters were taken on.

Counter inputs may be rocprofv3 CSV (<name>_counter_collection.csv) or rocpd
SQLite databases (<name>_results.db).
"""
import argparse
import collections
import csv
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

# Device kernel -> the name the library's timing report uses for it.
SCOPES = {
    "k_paint_vec_b": "cic_paint_vec",
    "k_step_b": "pm_step",
    "k_force_adjoint_b": "force_adjoint",
    "k_final_b": "final_kick",
    "k_data_paint_b": "data_paint",
    "k_data_adjoint_b": "data_adjoint",
    "k_paint_b": "cic_paint",
    "k_scatter": "sort_scatter",
    "k_scatter_ids": "sort_scatter_ids",
    "k_gather_back": "sort_gather_back",
    "k_keys": "sort_keys",
    "k_r2c_z": "fft_r2c_z",
    "k_c2r_z": "fft_c2r_z",
    "k_r2c_zy": "fft_r2c_zy",
    "k_c2r_yz": "fft_c2r_yz",
    "k_strided": "fft_y",
    "k_x_scatter": "fft_x_scatter",
    "k_x_gather": "fft_x_gather",
    "k_mu2": "lpt_mu2",
    "k_lpt_assemble": "lpt_assemble",
    "k_phi_bar": "lpt_phi_bar",
    "k_loss": "loss",
}


# Paint kernels instantiated for the deterministic mode (second template
# argument true).
DET_PAINTS = ("k_paint_b", "k_paint_vec_b", "k_data_paint_b")


def short_name(kernel):
    """'void ic::pk::k_paint_vec_t<float>(...)' -> ('k_paint_vec_t<float>', 'k_paint_vec_t');
    the deterministic-mode paints ('k_paint_b<float, true>') get a '_det' suffix."""
    k = kernel.split("(")[0].replace("void ", "").strip()
    base = k.split("<")[0].split("::")[-1]
    if base in DET_PAINTS and ", true>" in k:
        base += "_det"
    targ = ""
    if "<float" in k:
        targ = "<float>"
    elif "<double" in k:
        targ = "<double>"
    return base + targ, base


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError("none of %s in %s" % (names, list(row)))


def read_counters(path):
    """{(dispatch, kernel): {counter: value}} from a counter-collection file."""
    out = collections.defaultdict(dict)
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        rows = con.execute("select dispatch_id, kernel_name, counter_name, value "
                           "from counters_collection").fetchall()
        for d, k, c, v in rows:
            out[(int(d), k)][c] = out[(int(d), k)].get(c, 0.0) + float(v)
        return out
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            d = int(_col(row, "Dispatch_Id", "dispatch_id"))
            k = _col(row, "Kernel_Name", "kernel_name")
            c = _col(row, "Counter_Name", "counter_name")
            v = float(_col(row, "Counter_Value", "counter_value", "value"))
            out[(d, k)][c] = out[(d, k)].get(c, 0.0) + v
    return out


def per_kernel(counts, counter):
    """{kernel short name: (dispatches, mean value)} and the largest copy's value."""
    acc = collections.defaultdict(list)
    copy = 0.0
    for (_, k), cs in counts.items():
        if counter not in cs:
            continue
        name, base = short_name(k)
        if "copyBuffer" in k:
            copy = max(copy, cs[counter])
            continue
        acc[name].append(cs[counter])
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}, copy


def traffic(a):
    from paper_2604_26823_amd import build
    fetch, copy_f = per_kernel(read_counters(a.fetch), "FETCH_SIZE")
    write, copy_w = per_kernel(read_counters(a.write), "WRITE_SIZE")
    copy_kib = a.copy_mib * 1024.0
    if copy_f <= 0 or copy_w <= 0:
        raise SystemExit("no calibration copy found in the counter files")
    ff, wf = copy_kib / copy_f, copy_kib / copy_w
    lines = [
        "# HBM traffic per launch from rocprofv3 hardware counters, %s." % a.workload,
        "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) come from two --pmc runs of the same",
        "# command; each is scaled by copy bytes / counter reading of the run's %d MiB device"
        % a.copy_mib,
        "# copy (fetch_factor, write_factor). hbm_bytes_per_launch = (fetch_kib * fetch_factor",
        "# + write_kib * write_factor) * 1024, averaged over the kernel's dispatches.",
        "# commands:",
    ]
    lines += ["#   " + c for c in a.command]
    lines.append("sources_sha256 %s" % build.sources_digest())
    lines.append("copy_calibration copy_kib %.0f fetch_kib %.1f write_kib %.1f fetch_factor %.4f "
                 "write_factor %.4f" % (copy_kib, copy_f, copy_w, ff, wf))
    rows = []
    for name in set(fetch) & set(write):
        base = name.split("<")[0]
        scope = SCOPES.get(base, base)
        nd, fk = fetch[name]
        _, wk = write[name]
        rows.append((scope, name, nd, fk, wk, (fk * ff + wk * wf) * 1024.0))
    rows.sort(key=lambda r: -r[5] * r[2])
    tag = "<float>" if a.tag == "fp32" else "<double>"
    for scope, name, nd, fk, wk, b in rows:
        if not name.endswith(tag):
            continue
        lines.append("kernel %s %s dispatches %d fetch_kib %.1f write_kib %.1f "
                     "hbm_bytes_per_launch %.0f" % (scope, name, nd, fk, wk, b))
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stats(a):
    with open(a.csv, newline="") as fh:
        rows = list(csv.DictReader(fh))
    recs = []
    for r in rows:
        name, _ = short_name(_col(r, "Name", "KernelName", "Kernel_Name"))
        calls = int(float(_col(r, "Calls")))
        tot = float(_col(r, "TotalDurationNs"))
        recs.append((name, calls, tot))
    merged = collections.OrderedDict()
    for name, calls, tot in recs:
        c, t = merged.get(name, (0, 0.0))
        merged[name] = (c + calls, t + tot)
    total = sum(t for _, t in merged.values())
    lines = ["# rocprofv3 --kernel-trace --stats summary, %s." % a.workload, "# command:"]
    lines += ["#   " + c for c in a.command]
    lines.append("# %-34s %8s %12s %12s %7s" % ("kernel", "calls", "total_ms", "avg_us", "share"))
    for name, (c, t) in sorted(merged.items(), key=lambda kv: -kv[1][1])[:a.top]:
        lines.append("%-36s %8d %12.3f %12.2f %6.2f%%" % (name, c, t / 1e6, t / c / 1e3,
                                                          100.0 * t / total))
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    st = sub.add_parser("stats")
    st.add_argument("csv")
    st.add_argument("--top", type=int, default=30)
    tr = sub.add_parser("traffic")
    tr.add_argument("--fetch", required=True)
    tr.add_argument("--write", required=True)
    tr.add_argument("--tag", default="fp32", choices=["fp32", "fp64"])
    tr.add_argument("--copy-mib", type=int, default=256)
    for p in (st, tr):
        p.add_argument("--command", action="append", default=[])
        p.add_argument("--workload", default="256^3 particles on a 256^3 mesh (c3)")
        p.add_argument("--out", required=True)
    a = ap.parse_args()
    (stats if a.mode == "stats" else traffic)(a)


if __name__ == "__main__":
    main()
