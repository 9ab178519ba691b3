"""Summaries of rocprofv3 output for the precoder's kernels.

    python -m paper_2305_13925_amd.profile_summary trace <kernel_trace.csv> --title T --cmd C
        markdown table of per-kernel dispatch durations (grouped by kernel and grid)

    python -m paper_2305_13925_amd.profile_summary traffic --fetch D --write D \
            --copy-fetch D --copy-write D --copy-bytes N --cmd C --out profiles/hbm_traffic
        HBM bytes per dispatch of the Gram, PCG and precoder kernels from a
        FETCH_SIZE pass and a WRITE_SIZE pass (each a rocprofv3 --pmc output
        directory), each scaled by what the same counter reads for a plain copy
        kernel of N bytes read and N bytes written. Writes <out>.json (read by
        bench.py; tied to the sha256 of the kernel sources) and <out>.md.

    python -m paper_2305_13925_amd.profile_summary markers <trace dir> --cmd C --out F
        host-side roctx ranges (per call and per phase) from a --marker-trace run

    python -m paper_2305_13925_amd.profile_summary busy <pmc dir> --cmd C --out profiles/mfma_busy
        matrix-core utilisation and clock of the Gram, PCG and precoder
        kernels from a pass with GRBM_GUI_ACTIVE and SQ_VALU_MFMA_BUSY_CYCLES:
        clock = GRBM_GUI_ACTIVE / XCDs / dispatch duration, MFMA busy =
        SQ_VALU_MFMA_BUSY_CYCLES / (SIMDs x GRBM_GUI_ACTIVE / XCDs), with the
        XCD and SIMD counts read from the pass's agent info.
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2305_13925_amd/csrc/gram.hip", "paper_2305_13925_amd/csrc/pcg.hip",
                  "paper_2305_13925_amd/csrc/precoder.hip", "paper_2305_13925_amd/csrc/device_util.hpp",
                  "paper_2305_13925_amd/csrc/common.hpp"]
PHASE_PREFIX = {"gram": "gram_", "solve": "pcg_", "epilogue": "precoder_", "gram64": "gram64_",
                "refine_step": "refine_step_"}


def short_name(name):
    return name.replace("jacpcg::(anonymous namespace)::", "").replace("void ", "")


def grid_of(r):
    return int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)


def trace_table(path, title, cmd):
    rows = list(csv.DictReader(open(path)))
    d = collections.defaultdict(list)
    for r in rows:
        key = (r["Kernel_Name"], grid_of(r), int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0),
               r.get("VGPR_Count"), r.get("Accum_VGPR_Count"), r.get("LDS_Block_Size"))
        d[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = [f"# {title}\n", "Command (run from the repository root on one MI355X):\n", "```", cmd, "```\n",
           "Per-dispatch durations from the kernel trace, grouped by kernel and grid size (threads). "
           "\"working\" counts the dispatches that took at least a quarter of the group's longest one and "
           "averages them: the refinement kernels are enqueued for every possible step, and a launch whose "
           "columns have all converged returns at once.\n",
           "| kernel | grid (threads) | WG | VGPR | AGPR | LDS B | dispatches | avg us | min us | max us | "
           "working | working avg us |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        name = short_name(k[0])
        if len(name) > 70:
            name = name[:70] + "..."
        work = [x for x in v if x >= max(v) / 4]
        out.append(f"| `{name}` | {k[1]} | {k[2]} | {k[3]} | {k[4]} | {k[5]} | {len(v)} | "
                   f"{sum(v) / len(v) / 1e3:.2f} | {min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} | {len(work)} | "
                   f"{sum(work) / len(work) / 1e3:.2f} |")
    return "\n".join(out) + "\n"


def counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(files[0])))


def per_dispatch(rows, counter):
    """{(kernel, grid): [value per dispatch]} of one counter (summed over its instances)."""
    acc = collections.defaultdict(float)
    meta = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[did] += float(r["Counter_Value"])
        meta[did] = (r["Kernel_Name"], grid_of(r))
    out = collections.defaultdict(list)
    for did, v in acc.items():
        out[meta[did]].append(v)
    return out


def largest(per, prefix):
    """Dispatches of the largest-grid launch of the kernel whose short name starts with prefix."""
    cands = [(k, v) for k, v in per.items() if short_name(k[0]).startswith(prefix)]
    if not cands:
        return None, []
    k, v = max(cands, key=lambda kv: (kv[0][1], len(kv[1])))
    return k, v


def traffic(a):
    kib = 1024.0
    cf = per_dispatch(counter_rows(a.copy_fetch), "FETCH_SIZE")
    cw = per_dispatch(counter_rows(a.copy_write), "WRITE_SIZE")
    copy_f = max((max(v) for v in cf.values()), default=0.0) * kib
    copy_w = max((max(v) for v in cw.values()), default=0.0) * kib
    f_scale = a.copy_bytes / copy_f
    w_scale = a.copy_bytes / copy_w
    fetch = per_dispatch(counter_rows(a.fetch), "FETCH_SIZE")
    write = per_dispatch(counter_rows(a.write), "WRITE_SIZE")
    rec = {"per_launch_bytes": {}, "fetch_bytes": {}, "write_bytes": {}, "kernels": {},
           "calibration": {"copy_bytes": a.copy_bytes, "fetch_counter_bytes": copy_f, "write_counter_bytes": copy_w,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "command": a.cmd,
           "sources": {f: hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest()
                       for f in KERNEL_SOURCES}}
    lines = ["# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n",
             "Commands (run from the repository root on one MI355X; one counter per pass):\n", "```", a.cmd, "```\n",
             f"Calibration: a plain copy of {a.copy_bytes / 2**30:.2f} GiB reads FETCH_SIZE = "
             f"{copy_f / 2**30:.3f} GiB and WRITE_SIZE = {copy_w / 2**30:.3f} GiB, so fetch counts are "
             f"scaled by {f_scale:.3f} and write counts by {w_scale:.3f}.\n",
             "| phase | kernel | grid | dispatches | fetch MB (scaled) | write MB (scaled) | total MB |",
             "|---|---|---|---|---|---|---|"]
    for phase, prefix in PHASE_PREFIX.items():
        kf, vf = largest(fetch, prefix)
        kw, vw = largest(write, prefix)
        if not vf or not vw:
            continue
        fb = sum(vf) / len(vf) * kib * f_scale
        wb = sum(vw) / len(vw) * kib * w_scale
        rec["per_launch_bytes"][phase] = fb + wb
        rec["fetch_bytes"][phase] = fb
        rec["write_bytes"][phase] = wb
        rec["kernels"][phase] = short_name(kf[0])
        lines.append(f"| {phase} | `{short_name(kf[0])[:60]}` | {kf[1]} | {len(vf)} | {fb / 1e6:.1f} | "
                     f"{wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")
    json.dump(rec, open(a.out + ".json", "w"), indent=1)
    open(a.out + ".md", "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def busy(a):
    rows = counter_rows(a.dir)
    files = glob.glob(os.path.join(a.dir, "**", "*agent_info.csv"), recursive=True)
    gpu = [r for r in csv.DictReader(open(files[0])) if int(r.get("Simd_Count") or 0) > 0][0]
    n_xcd, n_simd = int(gpu["Num_Xcc"]), int(gpu["Simd_Count"])
    disp = collections.defaultdict(dict)
    for r in rows:
        did = r.get("Dispatch_Id") or r.get("Correlation_Id")
        d = disp[did]
        d["key"] = (r["Kernel_Name"], grid_of(r))
        d["us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    per = collections.defaultdict(list)
    for d in disp.values():
        per[d["key"]].append(d)
    lines = ["# Matrix-core utilisation and clock per launch (rocprofv3 counters)\n",
             "Command (run from the repository root on one MI355X):\n", "```", a.cmd, "```\n",
             f"Device: {n_xcd} XCDs, {n_simd} SIMDs. Clock = GRBM_GUI_ACTIVE / {n_xcd} / dispatch duration. "
             f"MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / ({n_simd} x GRBM_GUI_ACTIVE / {n_xcd}). The durations are "
             "those of the counter pass, which serialises dispatches.\n",
             "| phase | kernel | grid | dispatches | avg us | clock GHz | MFMA busy |", "|---|---|---|---|---|---|---|"]
    rec = {}
    for phase, prefix in PHASE_PREFIX.items():
        k, v = largest(per, prefix)
        if not v:
            continue
        us = sum(d["us"] for d in v) / len(v)
        cyc = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in v) / len(v) / n_xcd
        mfma = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in v) / len(v)
        ghz = cyc / (us * 1e3) if us > 0 else 0.0
        frac = mfma / (n_simd * cyc) if cyc > 0 else 0.0
        rec[phase] = {"kernel": short_name(k[0]), "us": us, "clock_ghz": ghz, "mfma_busy": frac}
        lines.append(f"| {phase} | `{short_name(k[0])[:60]}` | {k[1]} | {len(v)} | {us:.1f} | {ghz:.2f} | "
                     f"{frac:.3f} |")
    # Every launch group of the library's kernels (kernel, grid), by total time.
    groups = []
    for k, v in per.items():
        name = short_name(k[0])
        if not any(name.startswith(pf) for pf in PHASE_PREFIX.values()):
            continue
        tot = sum(d["us"] for d in v)
        cyc = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in v) / n_xcd
        mfma = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in v)
        groups.append((tot, name, k[1], len(v), cyc, mfma))
    if groups:
        lines += ["", "Every launch group of the library's kernels, by total time in the counter pass:\n",
                  "| kernel | grid | dispatches | avg us | clock GHz | MFMA busy |", "|---|---|---|---|---|---|"]
        for tot, name, grid, n, cyc, mfma in sorted(groups, reverse=True):
            ghz = cyc / (tot * 1e3) if tot > 0 else 0.0
            frac = mfma / (n_simd * cyc) if cyc > 0 else 0.0
            lines.append(f"| `{name[:60]}` | {grid} | {n} | {tot / n:.1f} | {ghz:.2f} | {frac:.3f} |")
    json.dump(dict(rec, command=a.cmd), open(a.out + ".json", "w"), indent=1)
    open(a.out + ".md", "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def markers(a):
    """Host-side roctx ranges of the library (one per call and per phase
    enqueued kernel by kernel): count and mean duration per range name."""
    files = glob.glob(os.path.join(a.dir, "**", "*marker_api_trace.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no marker_api_trace.csv under {a.dir}")
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(files[0])):
        d[r["Function"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# roctx ranges of the library (host side)\n",
             "Command (run from the repository root on one MI355X):\n", "```", a.cmd, "```\n",
             "Each call of the library opens a range named for the call; when its kernels are enqueued one by one "
             "(graph capture, eager launches with per-kernel timing) each phase opens its own range inside it. "
             "A replayed graph shows only the call's range. Durations are host time spent enqueueing.\n",
             "| range | count | mean us | max us |", "|---|---|---|---|"]
    for name, v in sorted(d.items(), key=lambda kv: -len(kv[1])):
        lines.append(f"| {name} | {len(v)} | {sum(v) / len(v):.1f} | {max(v):.1f} |")
    text = "\n".join(lines) + "\n"
    if a.out:
        open(a.out, "w").write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out")
    f = sub.add_parser("traffic")
    for n in ("fetch", "write", "copy_fetch", "copy_write"):
        f.add_argument("--" + n.replace("_", "-"), dest=n, required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--cmd", required=True)
    f.add_argument("--out", required=True)
    b = sub.add_parser("busy")
    b.add_argument("dir")
    b.add_argument("--cmd", required=True)
    b.add_argument("--out", required=True)
    m = sub.add_parser("markers")
    m.add_argument("dir")
    m.add_argument("--cmd", required=True)
    m.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd_name == "busy":
        return busy(a)
    if a.cmd_name == "markers":
        return markers(a)
    if a.cmd_name == "trace":
        text = trace_table(a.csv, a.title, a.cmd)
        if a.out:
            open(a.out, "w").write(text)
        print(text)
    else:
        traffic(a)


if __name__ == "__main__":
    main()
