"""Summarise rocprofv3 CSV output of a benchmark run into a short markdown
table and a per-launch HBM traffic record.

Inputs are the directories rocprofv3 writes with ``--output-format csv``:

* ``--trace DIR``  from ``--kernel-trace --stats`` (``*_kernel_trace.csv``);
* ``--fetch DIR``  from ``--pmc FETCH_SIZE``;
* ``--write DIR``  from ``--pmc WRITE_SIZE``;
* ``--hit DIR``    from ``--pmc TCC_HIT_sum TCC_MISS_sum`` (optional), with
  ``GRBM_GUI_ACTIVE`` if given: the shader clock of each kernel while it ran,
  GRBM_GUI_ACTIVE (busy cycles, one count per XCD, summed over the
  device's 8 XCDs) over 8 times the dispatch durations of that run;
* ``--mfma DIR``   from ``--pmc MfmaUtil MfmaFlopsBF16 MfmaFlopsF64`` (optional):
  MfmaUtil is the share of SIMD cycles with the matrix core busy
  (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE times the SIMD count), per
  dispatch; the MfmaFlops counters count 512 flops per MFMA operation, and
  are divided by the dispatch's own duration.

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  They are scaled
by what the same counters read for a plain device copy of known size: the
largest ``__amd_rocclr_copyBuffer`` dispatch of the run (the benchmark's
``--calib-copy`` option issues a 1 GiB copy) must read and write 1 GiB.

``--traffic-json`` records, for the kernels named with ``--record``, the
scaled fetch and write bytes per launch together with the SHA-256 of the
kernel's source files (several joined with ``+``, hashed in that order as
one text), so that a reader can tell whether the figures still describe the
source as it stands.

Example (from the repository root, after the four profiling runs)::

    python -m paper_1812_07437_amd.prof_summary --trace T --fetch F --write W \\
        --hit H --out profiles/x.md --title "..." --command "..." \\
        --traffic-json profiles/traffic.json \\
        --record k_update2=paper_1812_07437_amd/csrc/k_update.hip
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os

COPY = "__amd_rocclr_copyBuffer"


def _csv(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "*" + suffix)))
    if not files:
        raise SystemExit("no %s under %s" % (suffix, d))
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _short(name, width=64):
    name = name.replace("wlc::", "")
    return name if len(name) <= width else name[:width - 3] + "..."


def kernel_times(trace_dir):
    """name -> list of durations (ms), in dispatch order."""
    out = collections.OrderedDict()
    for r in _csv(trace_dir, "_kernel_trace.csv"):
        out.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    return out


def dispatch_times(d, name):
    """kernel name -> list of dispatch durations (ms) of a counter run, in the
    order counters() lists that counter's values."""
    per = collections.OrderedDict()
    for r in _csv(d, "_counter_collection.csv"):
        if r["Counter_Name"] != name:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        per.setdefault(key, (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    out = collections.OrderedDict()
    for (k, _), v in per.items():
        out.setdefault(k, []).append(v)
    return out


def counters(d, name):
    """kernel name -> list of per-dispatch counter values (summed over the
    dimension rows rocprofv3 may emit for one dispatch)."""
    per = collections.OrderedDict()
    for r in _csv(d, "_counter_collection.csv"):
        if r["Counter_Name"] != name:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = collections.OrderedDict()
    for (k, _), v in per.items():
        out.setdefault(k, []).append(v)
    return out


def scale(vals):
    if COPY not in vals:
        return 1.0
    return 1048576.0 / max(vals[COPY])  # KiB in 1 GiB


def sha256(paths):
    h = hashlib.sha256()
    for path in paths.split("+"):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--hit")
    ap.add_argument("--mfma")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--top", type=int, default=14)
    ap.add_argument("--traffic-json")
    ap.add_argument("--record", action="append", default=[], help="KERNEL_SUBSTRING=SOURCE_FILE")
    a = ap.parse_args()

    kt = kernel_times(a.trace)
    total = sum(sum(v) for k, v in kt.items())
    order = sorted(kt, key=lambda k: -sum(kt[k]))
    lines = ["# " + a.title, "", "Command (from the repository root on the MI355X box):", "", "```", a.command, "```",
             "", "Kernel trace (`rocprofv3 --kernel-trace --stats`):", "",
             "| kernel | calls | total ms | avg ms | min ms | max ms | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for k in order[:a.top]:
        v = kt[k]
        lines.append("| `%s` | %d | %.3f | %.4f | %.4f | %.4f | %.1f |" % (
            _short(k), len(v), sum(v), sum(v) / len(v), min(v), max(v), 100.0 * sum(v) / total))
    fe = counters(a.fetch, "FETCH_SIZE") if a.fetch else {}
    wr = counters(a.write, "WRITE_SIZE") if a.write else {}
    cf, cw = scale(fe), scale(wr)
    if fe or wr:
        lines += ["", "HBM traffic per dispatch from `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (separate runs), "
                  "scaled so that the 1 GiB device copy (`%s`) reads and writes 1 GiB: fetch x%.3f, write x%.3f." %
                  (COPY, cf, cw), "",
                  "| kernel | dispatches | fetch GB/dispatch | write GB/dispatch |", "|---|---:|---:|---:|"]
        for k in order[:a.top]:
            f, w = fe.get(k), wr.get(k)
            if f is None and w is None:
                continue
            fv = sum(f) / len(f) * cf * 1024 / 1e9 if f else float("nan")
            wv = sum(w) / len(w) * cw * 1024 / 1e9 if w else float("nan")
            lines.append("| `%s` | %d | %.4f | %.4f |" % (_short(k), len(f or w), fv, wv))
    if a.hit:
        h, m = counters(a.hit, "TCC_HIT_sum"), counters(a.hit, "TCC_MISS_sum")
        gui = counters(a.hit, "GRBM_GUI_ACTIVE")
        if gui:
            gt = dispatch_times(a.hit, "GRBM_GUI_ACTIVE")
            lines += ["", "L2 hit rate and shader clock (`--pmc TCC_HIT_sum TCC_MISS_sum GRBM_GUI_ACTIVE`; the "
                      "clock is GRBM_GUI_ACTIVE, summed over the 8 XCDs, over 8 x the kernel's time in that run):",
                      "", "| kernel | hit rate | clock GHz |", "|---|---:|---:|"]
        else:
            lines += ["", "L2 hit rate (`--pmc TCC_HIT_sum TCC_MISS_sum`):", "", "| kernel | hit rate |",
                      "|---|---:|"]
        for k in order[:a.top]:
            if k in h and k in m and sum(h[k]) + sum(m[k]) > 0:
                row = "| `%s` | %.3f |" % (_short(k), sum(h[k]) / (sum(h[k]) + sum(m[k])))
                if gui:
                    dur = sum(gt.get(k, []))
                    row += " %s |" % ("%.2f" % (sum(gui[k]) / 8.0 / (dur * 1e-3) / 1e9) if k in gui and dur > 0
                                      else "-")
                lines.append(row)
    if a.mfma:
        util = counters(a.mfma, "MfmaUtil")
        fb, fd = counters(a.mfma, "MfmaFlopsBF16"), counters(a.mfma, "MfmaFlopsF64")
        mt = dispatch_times(a.mfma, "MfmaUtil")
        lines += ["", "Matrix-core activity (`--pmc MfmaUtil MfmaFlopsBF16 MfmaFlopsF64`, one run): MfmaUtil is "
                  "the share of SIMD cycles with the MFMA unit busy, averaged over dispatches weighted by "
                  "duration; the MFMA flop rates use the counted operations and each dispatch's duration in "
                  "that run.", "",
                  "| kernel | dispatches | MfmaUtil % | bf16 MFMA TFLOP/s | f64 MFMA TFLOP/s |",
                  "|---|---:|---:|---:|---:|"]
        for k in order[:a.top]:
            if k not in util:
                continue
            dur = mt.get(k, [])
            u = util[k]
            if dur and len(dur) == len(u):
                uw = sum(x * t for x, t in zip(u, dur)) / sum(dur)
                tb = sum(fb.get(k, [0.0])) / (sum(dur) * 1e-3) / 1e12
                td = sum(fd.get(k, [0.0])) / (sum(dur) * 1e-3) / 1e12
            else:
                uw, tb, td = sum(u) / len(u), float("nan"), float("nan")
            lines.append("| `%s` | %d | %.1f | %.1f | %.1f |" % (_short(k), len(u), uw, tb, td))
    # every kernel whose name is the recorded one (all template instances)
    # counts as one kernel: launches, time and bytes are summed over them
    recs = []
    for item in a.record:
        sub, src = item.split("=", 1)
        names = [k for k in kt if sub + "(" in k or sub + "<" in k]
        if not names:
            raise SystemExit("no kernel matches %s" % sub)
        launches = sum(len(kt[k]) for k in names)
        ms = sum(sum(kt[k]) for k in names)
        f = [v for k in names for v in fe.get(k, [])]
        w = [v for k in names for v in wr.get(k, [])]
        recs.append((sub, src, names, launches, ms, f, w))
    if recs:
        lines += ["", "Recorded kernels, all instances together:", "",
                  "| kernel | launches | total ms | avg ms/launch | fetch GB/launch | write GB/launch |",
                  "|---|---:|---:|---:|---:|---:|"]
        for sub, src, names, launches, ms, f, w in recs:
            lines.append("| `%s` | %d | %.3f | %.4f | %s | %s |" % (
                sub, launches, ms, ms / launches,
                "%.4f" % (sum(f) / len(f) * cf * 1024 / 1e9) if f else "-",
                "%.4f" % (sum(w) / len(w) * cw * 1024 / 1e9) if w else "-"))
    with open(a.out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))

    if a.traffic_json:
        rec = {}
        if os.path.exists(a.traffic_json):
            with open(a.traffic_json) as fi:
                rec = json.load(fi)
        for sub, src, names, launches, ms, f, w in recs:
            rec[sub] = {
                "ms_per_launch": ms / launches,
                "kernels": names,
                "source": src,
                "source_sha256": sha256(src),
                "launches": launches,
                "fetch_bytes_per_launch": sum(f) / len(f) * cf * 1024 if f else None,
                "write_bytes_per_launch": sum(w) / len(w) * cw * 1024 if w else None,
                "calibration": {"fetch": cf, "write": cw},
                "summary": a.out,
            }
        with open(a.traffic_json, "w") as fo:
            json.dump(rec, fo, indent=1, sort_keys=True)
            fo.write("\n")


if __name__ == "__main__":
    main()
