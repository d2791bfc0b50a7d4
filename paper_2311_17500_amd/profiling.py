"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2311_17500_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2311_17500_amd.profiling traffic <fetch_dir> <write_dir> <out.json> "<command>" [config]
    python -m paper_2311_17500_amd.profiling resources <remarks.txt> <out.txt> "<command>" [<kernel_stats.csv>]
    python -m paper_2311_17500_amd.profiling activity <dir1,dir2,...> <out.txt> "<command>"
    python -m paper_2311_17500_amd.profiling traffic-text <traffic.json> <config> <out.txt> ["<notes>"]

`stats` turns the per-kernel statistics of a `rocprofv3 --kernel-trace
--stats` run into a short text table (kernel, calls, total and average
duration).  `traffic` takes two counter runs of `bench.py --kernel-probe`
(`--pmc FETCH_SIZE` and `--pmc WRITE_SIZE`, KiB per dispatch), calibrates the
counters on the probe's 1 GiB device copy (1 GiB read, 1 GiB written) and
writes the HBM bytes per launch of each library kernel under the workload's
config number, with the hash of the kernel sources they were measured on
(entries of other configs measured on the same sources are kept).  Kernel names are reduced to the
library's short form, e.g. ``k_coef_fused<float, ...>`` -> ``coef_fused<f32>``.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

_PREC = {"double": "f64", "float": "f32", "__hip_bfloat16": "bf16"}
_FN = {"k_sweep": "gather_sweep", "k_sweep_flat": "gather_sweep", "k_sweep_dual": "sweep_dual",
       "k_gather": "gather_scalar", "k_gather_v4": "gather_v4", "k_gather_rows": "gather_rows",
       "k_dense_mode": "dense_mode_mfma", "k_dense_modeE": "dense_mode_mfma", "k_dense_modeU": "dense_mode_mfma",
       "k_dense_rows": "dense_mode_mfma", "k_coef_fused": "coef_fused", "k_coef_fused_pf": "coef_fused",
       "k_quad_fused": "quad_fused", "k_time_core": "time_core", "k_time_mix": "time_mix", "k_arrowhead": "arrowhead",
       "k_multidot": "multidot", "k_multidot_v": "multidot", "k_update_norm": "update_norm",
       "k_pointwise_ionic": "pointwise_ionic", "k_mode_max": "mode_max", "k_react_point": "react_point",
       "k_band_solve": "band_solve", "k_band_factor": "band_factor"}


def short_name(full: str) -> str:
    """Library short name of a (demangled) kernel name, else the name cut at '('."""
    m = re.search(r"\b(k_\w+)(?:<([^,>]+))?", full)
    if m:
        base = _FN.get(m.group(1), m.group(1)[2:])
        prec = _PREC.get((m.group(2) or "").strip(), "")
        if m.group(1) in ("k_quad_fused", "k_mode_max", "k_pointwise_ionic"):
            prec = "f64"
        return f"{base}<{prec}>" if prec else base
    return re.sub(r"\(anonymous namespace\)::", "", full).split("(")[0][:80]


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources (measured traffic is valid for these only)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp"):
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def stats(stats_csv: str, out_txt: str, command: str, top: int = 30) -> None:
    rows = _rows(stats_csv)
    agg = defaultdict(lambda: [0, 0.0])
    for r in rows:
        name = short_name(r.get("Name") or r.get("KernelName") or "")
        agg[name][0] += int(float(r.get("Calls", 0)))
        agg[name][1] += float(r.get("TotalDurationNs", 0.0))
    tot = sum(v[1] for v in agg.values()) or 1.0
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}",
             f"# kernels grouped by library function and storage precision", "",
             f"{'kernel':40s} {'calls':>8s} {'total ms':>10s} {'avg us':>10s} {'share':>7s}"]
    for name, (calls, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{name:40s} {calls:8d} {ns / 1e6:10.2f} {ns / max(calls, 1) / 1e3:10.2f} {100 * ns / tot:6.1f}%")
    lines.append("")
    lines.append(f"all kernels: {tot / 1e6:.2f} ms")
    with open(out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _per_kernel(counter_dir: str, counter: str):
    rows = _rows(_find(counter_dir, "counter_collection.csv"))
    per = defaultdict(list)
    for r in rows:
        if r.get("Counter_Name", counter) != counter:
            continue
        name = r.get("Kernel_Name") or r.get("KernelName") or ""
        per[name].append(float(r["Counter_Value"]))
    return per


def traffic(fetch_dir: str, write_dir: str, out_json: str, command: str, cfg: str = "2",
            copy_bytes: int = 1 << 30) -> None:
    fetch = _per_kernel(fetch_dir, "FETCH_SIZE")
    write = _per_kernel(write_dir, "WRITE_SIZE")
    # the copy: the non-library kernel (library kernels live in namespace
    # stiga) with the largest fetch, i.e. the probe's 1 GiB device copy
    cands = [n for n in fetch if "stiga" not in n and n in write]
    copy = max(cands, key=lambda n: max(fetch[n]))
    f_scale = copy_bytes / (max(fetch[copy]) * 1024.0)
    w_scale = copy_bytes / (max(write[copy]) * 1024.0)
    kern = {}
    for n in fetch:
        if n not in write or "stiga" not in n:
            continue
        s = short_name(n)
        rd = sum(fetch[n]) / len(fetch[n]) * 1024.0 * f_scale
        wr = sum(write[n]) / len(write[n]) * 1024.0 * w_scale
        k = kern.setdefault(s, {"reads": [], "writes": []})
        k["reads"].append(rd)
        k["writes"].append(wr)
    out = {}
    for s, k in kern.items():
        rd = sum(k["reads"]) / len(k["reads"])
        wr = sum(k["writes"]) / len(k["writes"])
        out[s] = {"fetch_bytes_per_launch": rd, "write_bytes_per_launch": wr, "hbm_bytes_per_launch": rd + wr}
    sha = kernel_source_hash()
    doc = {"kernel_source_sha256": sha, "configs": {}}
    try:
        with open(out_json) as fh:
            old = json.load(fh)
        if old.get("kernel_source_sha256") == sha:
            doc["configs"] = old.get("configs", {})
    except (OSError, ValueError):
        pass
    doc["configs"][str(cfg)] = {"command": command, "copy_kernel": copy[:120], "fetch_scale": f_scale,
                                "write_scale": w_scale, "kernels": out}
    with open(out_json, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)


def activity(dirs: str, out_txt: str, command: str, cus: int = 256, simds: int = 1024, xcds: int = 8) -> None:
    """Per-kernel hardware activity from one or more `rocprofv3 --pmc` runs
    (comma-separated output directories, at most 8 SQ counters and one GRBM
    counter each): counter values averaged over each kernel's dispatches and
    the usual derived ratios (VALU busy = 4 SQ_ACTIVE_INST_VALU / SIMDs /
    G, MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (CUs 4 G), with G the active
    cycles of one XCD: GRBM_GUI_ACTIVE, which sums the XCDs' GRBMs, divided by
    the XCD count; LDS bank-conflict share = SQ_LDS_BANK_CONFLICT /
    SQ_LDS_IDX_ACTIVE; instructions per wave)."""
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs.split(","):
        for r in _rows(_find(d, "counter_collection.csv")):
            name = r.get("Kernel_Name") or r.get("KernelName") or ""
            if "stiga" not in name:
                continue
            vals[short_name(name)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}

    def ratio(a, b, scale=1.0):
        return scale * a / b if (a is not None and b) else None
    lines = ["# hardware activity per kernel (rocprofv3 --pmc, values averaged over the kernel's dispatches)",
             f"# command: {command}",
             "# G = GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs' GRBMs): one XCD's active cycles",
             "# VALU%: 4 SQ_ACTIVE_INST_VALU / SIMDs / G;  MFMA%: SQ_VALU_MFMA_BUSY_CYCLES / (CUs 4 G);", "# LDS conf%: SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE;  "
             "VALU/w, MFMA/w, VMEM/w, LDS/w: instructions per wave;  wait%: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES", "",
             f"{'kernel':28s} {'waves':>8s} {'VALU%':>6s} {'MFMA%':>6s} {'LDSconf%':>8s} {'VALU/w':>8s} "
             f"{'MFMA/w':>7s} {'VMEM/w':>7s} {'LDS/w':>7s} {'wait%':>6s}"]
    for k in sorted(avg, key=lambda n: -avg[n].get("GRBM_GUI_ACTIVE", 0.0)):
        a = avg[k]
        g = a.get("GRBM_GUI_ACTIVE")
        g = g / xcds if g else g
        wv = a.get("SQ_WAVES")
        vmem = (a.get("SQ_INSTS_VMEM_RD", 0.0) + a.get("SQ_INSTS_VMEM_WR", 0.0)) if "SQ_INSTS_VMEM_RD" in a else None
        cells = [ratio(a.get("SQ_ACTIVE_INST_VALU"), g, 4.0 * 100.0 / simds) if "SQ_ACTIVE_INST_VALU" in a else None,
                 ratio(a.get("SQ_VALU_MFMA_BUSY_CYCLES"), g, 100.0 / (4 * cus)) if "SQ_VALU_MFMA_BUSY_CYCLES" in a else None,
                 ratio(a.get("SQ_LDS_BANK_CONFLICT"), a.get("SQ_LDS_IDX_ACTIVE"), 100.0) if "SQ_LDS_BANK_CONFLICT" in a else None,
                 ratio(a.get("SQ_INSTS_VALU"), wv) if "SQ_INSTS_VALU" in a else None,
                 ratio(a.get("SQ_INSTS_MFMA"), wv) if "SQ_INSTS_MFMA" in a else None,
                 ratio(vmem, wv),
                 ratio(a.get("SQ_INSTS_LDS"), wv) if "SQ_INSTS_LDS" in a else None,
                 ratio(a.get("SQ_WAIT_INST_ANY"), a.get("SQ_WAVE_CYCLES"), 100.0) if "SQ_WAIT_INST_ANY" in a else None]
        fmt = lambda v, w, p: (f"{v:{w}.{p}f}" if v is not None else f"{'-':>{w}s}")
        lines.append(f"{k[:28]:28s} {(wv or 0):8.0f} {fmt(cells[0], 6, 1)} {fmt(cells[1], 6, 1)} {fmt(cells[2], 8, 1)} "
                     f"{fmt(cells[3], 8, 0)} {fmt(cells[4], 7, 0)} {fmt(cells[5], 7, 0)} {fmt(cells[6], 7, 0)} "
                     f"{fmt(cells[7], 6, 1)}")
    lines.append("")
    lines.append("# raw averages")
    for k in sorted(avg):
        lines.append(f"{k}: " + ", ".join(f"{c}={v:.4g}" for c, v in sorted(avg[k].items())))
    with open(out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def resources(remarks_txt: str, out_txt: str, command: str, launched_csv: str = "") -> None:
    """Per-kernel register, LDS, spill and occupancy figures from the
    compiler's `-Rpass-analysis=kernel-resource-usage` remarks; with a
    rocprofv3 kernel_stats.csv, only the instantiations that run launched."""
    import subprocess
    fields = ("TotalSGPRs", "VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]", "SGPRs Spill",
              "VGPRs Spill", "LDS Size [bytes/block]")
    kern, cur = {}, None
    with open(remarks_txt) as fh:
        for line in fh:
            m = re.search(r"remark: Function Name: (\S+)", line)
            if m:
                cur = m.group(1)
                kern[cur] = {}
                continue
            m = re.search(r"remark:\s+([A-Za-z ]+(?:\[[^\]]*\])?): (\S+)", line)
            if cur and m and m.group(1).strip() in fields:
                kern[cur][m.group(1).strip()] = m.group(2)
    names = list(kern)
    try:
        dem = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True).stdout.split("\n")
    except OSError:
        dem = names
    rows = []
    for mangled, full in zip(names, dem):
        if not full.strip():
            continue
        m = re.search(r"(k_\w+)(<[^()]*>)?\(", full)
        short = (m.group(1) + (m.group(2) or "")) if m else full[:60]
        short = short.replace("__hip_bfloat16", "bf16").replace("(anonymous namespace)::", "")
        f = kern[mangled]
        rows.append((short, f.get("VGPRs", "?"), f.get("AGPRs", "?"), f.get("TotalSGPRs", "?"),
                     f.get("VGPRs Spill", "?"), f.get("SGPRs Spill", "?"), f.get("ScratchSize [bytes/lane]", "?"),
                     f.get("LDS Size [bytes/block]", "?"), f.get("Occupancy [waves/SIMD]", "?")))
    if launched_csv:
        launched = set()
        for r in _rows(launched_csv):
            m = re.search(r"(k_\w+)(<[^()]*>)?\(", r["Name"])
            if m:
                launched.add((m.group(1) + (m.group(2) or "")).replace("__hip_bfloat16", "bf16"))
        rows = [r for r in rows if r[0] in launched]
    rows.sort()
    lines = ["# compiler resource usage per kernel instantiation (gfx950)"
             + (" launched by the benchmark run" if launched_csv else ""), f"# command: {command}", "",
             f"{'kernel':78s} {'VGPR':>5s} {'AGPR':>5s} {'SGPR':>5s} {'Vspill':>6s} {'Sspill':>6s} "
             f"{'scratch':>7s} {'LDS B':>7s} {'waves/SIMD':>10s}"]
    for r in rows:
        lines.append(f"{r[0][:78]:78s} {r[1]:>5s} {r[2]:>5s} {r[3]:>5s} {r[4]:>6s} {r[5]:>6s} {r[6]:>7s} "
                     f"{r[7]:>7s} {r[8]:>10s}")
    with open(out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def traffic_text(in_json: str, cfg: str, out_txt: str, notes: str = "") -> None:
    """Text table of one workload's entry in the traffic record (read, write
    and total HBM MB per launch), sorted by total, with optional note lines."""
    with open(in_json) as fh:
        doc = json.load(fh)
    c = doc["configs"][cfg]
    lines = [f"# HBM traffic per launch from rocprofv3 counters (config {cfg} workload)",
             f"# command: {c['command']}",
             f"# calibration: the probe's 1 GiB device copy ({c['copy_kernel']}): its known bytes are FETCH_SIZE x "
             f"{c['fetch_scale']:.4f}",
             f"#              and WRITE_SIZE x {c['write_scale']:.4f}; both factors applied below",
             f"# kernel sources sha256 {doc['kernel_source_sha256']}",
             "", f"{'kernel':28s} {'read MB':>8s} {'write MB':>10s} {'total MB':>10s}"]
    rows = sorted(c["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"])
    for name, k in rows:
        lines.append(f"{name:28s} {k['fetch_bytes_per_launch'] / 1e6:8.1f} {k['write_bytes_per_launch'] / 1e6:10.1f} "
                     f"{k['hbm_bytes_per_launch'] / 1e6:10.1f}")
    if notes:
        lines += [""] + ["# " + ln for ln in notes.split("\n")]
    with open(out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if len(sys.argv) >= 5 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 5 and sys.argv[1] == "activity":
        activity(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 5 and sys.argv[1] == "resources":
        resources(sys.argv[2], sys.argv[3], sys.argv[4], *(sys.argv[5:6]))
    elif len(sys.argv) >= 5 and sys.argv[1] == "traffic-text":
        traffic_text(sys.argv[2], sys.argv[3], sys.argv[4], *(sys.argv[5:6]))
    elif len(sys.argv) >= 6 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], *(sys.argv[6:7]))
    else:
        sys.exit(__doc__)
