"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_1910_02371_amd.rocprof_summary stats  <kernel_stats.csv> <out.md> <cmd>
  python -m paper_1910_02371_amd.rocprof_summary traffic <fetch_dir> <write_dir> \\
        <kernel> <workload> <src_hash> <copy_bytes> <out.md> <cmd>

``stats`` renders the per-kernel table of a ``--kernel-trace --stats`` run.
``ccd`` (``ccd <out.md> <cmd> <kernel_trace.csv> ...``) gives the per-mode
pass times of the timed CCD++ sweep of the bench's CCD++ leg, one column
per trace (one trace per setting).
``trace`` (``trace <kernel_trace.csv> <last_kernel> <skip> <out.md> <cmd>``)
cuts a ``--kernel-trace`` run into calls, each ending with a dispatch whose
name contains ``last_kernel``, drops the first ``skip`` calls (warm-up) and
reports per call the dispatches, the span from the first start to the last
end, the summed kernel time, the gaps between consecutive dispatches and
the dispatches and mean duration of each kernel.
``counters`` (``counters <kernel> <workload> <src_hash> <out.md> <cmd> <pmc_dir>...``)
averages every counter of ``kernel``'s dispatches over one or more ``--pmc``
runs and records derived utilisation and request-size figures in
profiles/counters.json.
``traffic`` reads two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE; KiB per
dispatch), scales each by what the same counter reads for the plain copy
kernel of ``copy_bytes`` bytes that the profiled program runs first (a copy
reads and writes exactly copy_bytes), and records the HBM bytes per launch
of ``kernel`` in profiles/traffic.json, keyed by kernel and workload and
tagged with the kernel-source hash they were measured with.
"""
import csv
import glob
import json
import os
import sys

# library profiler names -> substrings of the device kernel names
KERNEL_MATCH = {
    "tttp": ", 3, ", "mttkrp": None, "gradient": None, "gn_matvec": None, "gn_mttkrp": None,
    "gram_heavy": "k_gram_f32_heavy", "gram_light": "k_gram_f32<",
    "gram_reduce": "k_gram_reduce", "cholesky_solve": "k_solve_rows",
    "cholesky_factor": "k_solve_rows", "precond_apply": "k_apply_rows",
    "heavy_fixup": "k_heavy_fixup",
}
# (the Gauss-Newton product's MTTKRP blocks run the MTTKRP kernel)
STREAM_OP = {"tttp": 0, "mttkrp": 1, "gradient": 2, "gn_matvec": 3, "gn_mttkrp": 1,
             "newton_terms": 4}


# fused Gram + Cholesky of rows with one light task:
# k_solve_solo<traits, RP, vec, weighted, rhs, factor_only, persist, model>;
# with one heavy task:
# k_gram_solve_heavy<traits, RP, vec, weighted, rhs, factor_only, model>
SOLO_FO = {"gram_solve_light": ("k_solve_solo<", "false"),
           "gram_factor_light": ("k_solve_solo<", "true"),
           "gram_solve_heavy": ("k_gram_solve_heavy<", "false"),
           "gram_factor_heavy": ("k_gram_solve_heavy<", "true")}


def matches(kernel, name):
    if kernel in SOLO_FO:
        kname, fo = SOLO_FO[kernel]
        if kname not in name:
            return False
        args = name.split(kname, 1)[1].split(">")[0].split(",")
        return len(args) >= 6 and args[5].strip() == fo
    if kernel in STREAM_OP:
        # k_stream<traits, order, G, vec, op, chunk>: the op is the fifth argument
        if "k_stream<" not in name:
            return False
        args = name.split("k_stream<", 1)[1].split(">")[0].split(",")
        return len(args) >= 5 and args[4].strip() == str(STREAM_OP[kernel])
    return KERNEL_MATCH[kernel] in name


def stats(csv_path, out_md, cmd):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics\n", f"Command: `{cmd}`\n",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:25]:
        lines.append(f"| `{r['Name'][:100]}` | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | "
                     f"{100 * float(r['TotalDurationNs']) / tot:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(files[0])))


def _per_dispatch(rows, counter):
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Dispatch_Id"], r["Kernel_Name"])
        out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return out


def traffic(fetch_dir, write_dir, kernel, workload, src_hash, copy_bytes, out_md, cmd):
    copy_bytes = float(copy_bytes)
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = _per_dispatch(_counter_rows(d), counter)
        # the calibration fill + copy are the program's first dispatches:
        # take the runtime/torch copy kernels dispatched before the library's
        # first kernel (later copies move the tensor's own data)
        first_tt = min((int(i) for (i, n) in disp if n.startswith("tt::") or " tt::" in n),
                       default=None)
        copies = [v for (i, n), v in disp.items()
                  if (first_tt is None or int(i) < first_tt) and "tt::" not in n
                  and ("copy" in n.lower() or "elementwise_kernel" in n.lower())]
        if not copies:
            raise SystemExit(f"{counter}: no copy-kernel dispatch found")
        ref = max(copies)  # KiB read (or written) by the calibration copy
        scale = copy_bytes / (ref * 1024.0)
        ks = [v for (i, n), v in disp.items() if matches(kernel, n)]
        if not ks:
            raise SystemExit(f"{counter}: no dispatch of {kernel}")
        res[counter] = {"scale": scale, "launches": len(ks),
                        "bytes_per_launch": sum(ks) * 1024.0 * scale / len(ks)}
    total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    path = os.path.join(os.path.dirname(out_md), "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[f"{kernel}|{workload}"] = {"bytes_per_launch": total, "src_hash": src_hash,
                                  "fetch_bytes_per_launch": res["FETCH_SIZE"]["bytes_per_launch"],
                                  "write_bytes_per_launch": res["WRITE_SIZE"]["bytes_per_launch"],
                                  "fetch_scale": res["FETCH_SIZE"]["scale"],
                                  "write_scale": res["WRITE_SIZE"]["scale"],
                                  "launches": res["FETCH_SIZE"]["launches"]}
    json.dump(db, open(path, "w"), indent=1, sort_keys=True)
    lines = [f"# HBM traffic of `{kernel}` on {workload}\n", f"Command: `{cmd}`\n",
             f"Kernel source hash: {src_hash}\n",
             "| counter | copy-kernel scale | launches | bytes per launch |",
             "|---|---|---|---|"]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        r = res[c]
        lines.append(f"| {c} | {r['scale']:.4f} | {r['launches']} | {r['bytes_per_launch']:.4e} |")
    lines.append(f"\nTotal HBM bytes per launch: {total:.4e}\n")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_dispatch_all(rows):
    """{(dispatch id, kernel name): {counter: value}} of a --pmc run."""
    out = {}
    for r in rows:
        key = (r["Dispatch_Id"], r["Kernel_Name"])
        d = out.setdefault(key, {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def counters(kernel, workload, src_hash, out_md, cmd, *pmc_dirs):
    """Per-launch averages of every counter recorded for `kernel` in the
    given --pmc runs, with the derived figures used in the design notes:
      mfma_busy      MfmaUtil / 100 (matrix-core busy cycles per SIMD over
                     the dispatch's GPU-active cycles)
      valu_busy      VALUBusy / 100
      bf16_mfma_flops, f64_mfma_flops   executed matrix-core operations
                     (SQ_INSTS_VALU_MFMA_MOPS_* x 512)
      read_req_bytes 32/64/128-byte L2->fabric read requests weighted by
                     their size (TCC_EA0_RDREQ_{32B,64B,128B}), and the
                     fraction of requests of each size.
    Records the result in profiles/counters.json keyed by kernel and
    workload, tagged with the kernel-source hash."""
    acc, n_l = {}, {}
    for d in pmc_dirs:
        disp = _per_dispatch_all(_counter_rows(d))
        for (i, name), vals in disp.items():
            if not matches(kernel, name):
                continue
            for c, v in vals.items():
                acc[c] = acc.get(c, 0.0) + v
                n_l[c] = n_l.get(c, 0) + 1
    if not acc:
        raise SystemExit(f"no dispatch of {kernel}")
    avg = {c: acc[c] / n_l[c] for c in acc}
    rec = {"src_hash": src_hash, "per_launch": avg, "launches": max(n_l.values())}
    if "MfmaUtil" in avg:
        rec["mfma_busy"] = avg["MfmaUtil"] / 100.0
    if "VALUBusy" in avg:
        rec["valu_busy"] = avg["VALUBusy"] / 100.0
    for dt in ("BF16", "F64", "F32"):
        k = f"SQ_INSTS_VALU_MFMA_MOPS_{dt}"
        if k in avg:
            rec[f"{dt.lower()}_mfma_flops"] = avg[k] * 512.0
    sizes = {32: "TCC_EA0_RDREQ_32B_sum", 64: "TCC_EA0_RDREQ_64B_sum",
             128: "TCC_EA0_RDREQ_128B_sum"}
    if all(v in avg for v in sizes.values()):
        nreq = sum(avg[v] for v in sizes.values())
        rec["read_req_bytes"] = sum(b * avg[v] for b, v in sizes.items())
        rec["read_req_mix"] = {f"{b}B": (avg[v] / nreq if nreq else 0.0)
                               for b, v in sizes.items()}
        rec["read_requests"] = nreq
    path = os.path.join(os.path.dirname(out_md), "counters.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[f"{kernel}|{workload}"] = rec
    json.dump(db, open(path, "w"), indent=1, sort_keys=True)
    lines = [f"# Counters of `{kernel}` on {workload}\n", f"Command: `{cmd}`\n",
             f"Kernel source hash: {src_hash}\n", "| counter | per launch |", "|---|---|"]
    for c in sorted(avg):
        lines.append(f"| {c} | {avg[c]:.6g} |")
    lines.append("")
    for k in ("mfma_busy", "valu_busy", "bf16_mfma_flops", "f64_mfma_flops",
              "read_req_bytes", "read_requests", "read_req_mix"):
        if k in rec:
            lines.append(f"* {k}: {rec[k]}")
    open(out_md, "w").write("\n".join(lines) + "\n")


def trace(csv_path, last_kernel, skip, out_md, cmd):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    calls, cur = [], []
    for r in rows:
        cur.append(r)
        if last_kernel in r["Kernel_Name"]:
            calls.append(cur)
            cur = []
    calls = calls[int(skip):]
    if not calls:
        raise SystemExit(f"no call ends with {last_kernel}")
    t = lambda r, k: int(r[k])
    per = []
    by_name = {}
    for c in calls:
        span = t(c[-1], "End_Timestamp") - t(c[0], "Start_Timestamp")
        busy = sum(t(r, "End_Timestamp") - t(r, "Start_Timestamp") for r in c)
        gaps = sorted(t(c[i + 1], "Start_Timestamp") - t(c[i], "End_Timestamp")
                      for i in range(len(c) - 1)) or [0]
        per.append((len(c), span / 1e3, busy / 1e3, gaps[len(gaps) // 2] / 1e3))
        for r in c:
            name = r["Kernel_Name"].split("(")[0]
            n, d = by_name.get(name, (0, 0))
            by_name[name] = (n + 1, d + t(r, "End_Timestamp") - t(r, "Start_Timestamp"))
    k = len(calls)
    lines = [f"# Kernel trace: {k} calls ending with `{last_kernel}`\n", f"Command: `{cmd}`\n",
             "| call | dispatches | span us | summed kernel us | median gap us |",
             "|---|---|---|---|---|"]
    for i, (n, span, busy, gap) in enumerate(per):
        lines.append(f"| {i} | {n} | {span:.1f} | {busy:.1f} | {gap:.2f} |")
    lines += ["", "| kernel | dispatches per call | mean us |", "|---|---|---|"]
    for name, (n, d) in sorted(by_name.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{name[:90]}` | {n / k:.1f} | {d / n / 1e3:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def ccd(out_md, cmd, *csvs):
    """Per-mode pass times of the last CCD++ sweep in each kernel trace
    (one trace per setting, in the order given by `cmd`'s settings): the
    k_ccd_tasks dispatches of a sweep run column by column, modes 0, 1, 2
    in turn, so dispatch i of the sweep is mode i mod 3."""
    cols = []
    for path in csvs:
        rows = [r for r in csv.DictReader(open(path)) if "k_ccd_" in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        tasks = [r for r in rows if "k_ccd_tasks" in r["Kernel_Name"]]
        rws = [r for r in rows if "k_ccd_rows" in r["Kernel_Name"]]
        colk = [r for r in rows if "k_ccd_column" in r["Kernel_Name"]]
        # the bench's CCD++ leg runs one untimed and one timed sweep: the
        # timed one is the second half of the dispatches
        last = tasks[-(len(tasks) // 2):]
        per_mode = {}
        for i, r in enumerate(last):
            per_mode.setdefault(i % 3, []).append(dur(r))
        names = sorted({r["Kernel_Name"].split("(")[0] for r in last})
        cols.append({"mode_us": {m: sum(v) / len(v) for m, v in per_mode.items()},
                     "rows_us": sum(dur(r) for r in rws[-len(last):]) / max(1, len(last)),
                     "column_us": sum(dur(r) for r in colk[-len(last):]) / max(1, len(last)),
                     "columns": len(last) // 3, "kernels": names})
    lines = [f"# CCD++ sweep: kernel times per mode pass\n", f"Commands: `{cmd}`\n",
             "| | " + " | ".join(f"setting {i}" for i in range(len(cols))) + " |",
             "|---" * (len(cols) + 1) + "|"]
    for m in range(3):
        lines.append(f"| mode-{m} pass (k_ccd_tasks) us | " +
                     " | ".join(f"{c['mode_us'][m]:.1f}" for c in cols) + " |")
    lines.append("| per-row solves (k_ccd_rows) us | " +
                 " | ".join(f"{c['rows_us']:.1f}" for c in cols) + " |")
    lines.append("| column start (k_ccd_column) us | " +
                 " | ".join(f"{c['column_us']:.1f}" for c in cols) + " |")
    lines.append("| columns in the sweep | " + " | ".join(str(c["columns"]) for c in cols) + " |")
    lines.append("")
    for i, c in enumerate(cols):
        lines.append(f"* setting {i} pass kernels: " + ", ".join(f"`{n}`" for n in c["kernels"]))
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:])
    elif sys.argv[1] == "trace":
        trace(*sys.argv[2:7])
    elif sys.argv[1] == "ccd":
        ccd(*sys.argv[2:])
    else:
        raise SystemExit(__doc__)
