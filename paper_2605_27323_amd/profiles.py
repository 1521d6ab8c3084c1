"""Summaries of rocprofv3 runs of the renderer's kernels.

Reads the CSV output of rocprofv3 (a kernel trace with --stats, counter runs
with --pmc) and writes a short text summary (Markdown) and the figures the
benchmark reads back (JSON): per kernel the dispatch count and mean duration
(overall and per stream), registers, LDS and scratch, HBM bytes per dispatch
(FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads for
a device copy of known size), wave64 VALU instructions issued per CU and
cycle, L2 hit rate and the mean number of resident waves per SIMD.

    python -m paper_2605_27323_amd.profiles --name NAME --title TITLE \\
        --trace DIR --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --pmc DIR [--pmc DIR ...] --cmd "command" [--cmd ...]

writes profiles/NAME.md and profiles/NAME.json.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# kernel sources: counters taken before a change of these no longer
# describe the kernels
SOURCES = ["device.h", "wavefront.h", "wave.h", "kernels.hip", "kernels.h", "ptmi_internal.h", "adjoint.h",
           "adjoint.hip"]
N_XCD, N_CU, SIMD_PER_CU = 8, 256, 4


def source_hash():
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def short_name(name):
    """'void ptmi::k_mega<8, false, 4>(ptmi::SceneView, ...)' -> 'ptmi::k_mega<8, false, 4>'."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def _rows(d, suffix):
    out = []
    for p in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(p, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def kernel_trace(d):
    """Per kernel: calls, mean duration (us) overall and per stream, and the
    resources of its dispatches (VGPRs, SGPRs, LDS bytes, scratch bytes)."""
    stats = {}
    for r in _rows(d, "kernel_stats.csv"):
        k = short_name(r["Name"])
        stats[k] = dict(calls=int(r["Calls"]), total_ms=float(r["TotalDurationNs"]) / 1e6,
                        avg_us=float(r["AverageNs"]) / 1e3, min_us=float(r["MinNs"]) / 1e3,
                        max_us=float(r["MaxNs"]) / 1e3, percent=float(r["Percentage"]))
    per_stream = defaultdict(list)
    res = {}
    for r in _rows(d, "kernel_trace.csv"):
        k = short_name(r["Kernel_Name"])
        per_stream[(k, int(r.get("Stream_Id", 0) or 0))].append(
            (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3)
        res[k] = dict(vgpr=int(r["VGPR_Count"]), agpr=int(r.get("Accum_VGPR_Count", 0) or 0),
                      sgpr=int(r["SGPR_Count"]), lds=int(r["LDS_Block_Size"]), scratch=int(r["Scratch_Size"]))
    streams = defaultdict(dict)
    for (k, s), v in per_stream.items():
        streams[k][s] = dict(dispatches=len(v), avg_us=sum(v) / len(v))
    return stats, dict(streams), res


def counter_runs(dirs):
    """Kernel -> counter -> (sum over dispatches, dispatches), over all runs."""
    acc = defaultdict(dict)
    for d in dirs:
        sums = defaultdict(lambda: defaultdict(float))
        disp = defaultdict(lambda: defaultdict(set))
        for r in _rows(d, "counter_collection.csv"):
            k = short_name(r["Kernel_Name"])
            c = r["Counter_Name"]
            sums[k][c] += float(r["Counter_Value"])
            disp[k][c].add(r["Dispatch_Id"])
        for k in sums:
            for c in sums[k]:
                acc[k][c] = (sums[k][c], len(disp[k][c]))
    return dict(acc)


def copy_scale(d, counter, kib):
    """Ratio of the copied KiB to what `counter` reads for the copy kernel."""
    got = counter_runs([d])
    vals = [v for k, c in got.items() if "copyBuffer" in k for n, v in c.items() if n == counter]
    if not vals:
        return None, None
    tot, n = vals[0]
    per = tot / max(n, 1)
    return kib / per, per


def summarize(args):
    stats, streams, res = kernel_trace(args.trace)
    copy_kib = float(args.copy_kib)
    fscale, fper = copy_scale(args.copy_fetch, "FETCH_SIZE", copy_kib)
    wscale, wper = copy_scale(args.copy_write, "WRITE_SIZE", copy_kib)
    fetch = counter_runs([args.fetch])
    write = counter_runs([args.write])
    pmc = counter_runs(args.pmc or [])
    kernels = {}
    names = sorted(set(stats) | set(fetch) | set(pmc), key=lambda k: -stats.get(k, {}).get("total_ms", 0.0))
    for k in names:
        if k.startswith("at::") or "rocclr" in k:
            continue
        e = {}
        if k in stats:
            e.update(calls=stats[k]["calls"], avg_us=stats[k]["avg_us"], total_ms=stats[k]["total_ms"])
            e["avg_us_by_stream"] = {str(s): v["avg_us"] for s, v in sorted(streams.get(k, {}).items())}
        if k in res:
            e.update(res[k])
        if k in fetch and "FETCH_SIZE" in fetch[k]:
            tot, n = fetch[k]["FETCH_SIZE"]
            e["fetch_kib"] = tot / n
            e["counter_dispatches"] = n
        if k in write and "WRITE_SIZE" in write[k]:
            tot, n = write[k]["WRITE_SIZE"]
            e["write_kib"] = tot / n
        if "fetch_kib" in e and "write_kib" in e and fscale and wscale:
            e["hbm_bytes_per_dispatch"] = 1024.0 * (e["fetch_kib"] * fscale + e["write_kib"] * wscale)
        c = pmc.get(k, {})

        def per(name):
            return c[name][0] / c[name][1] if name in c and c[name][1] else None
        gui = per("GRBM_GUI_ACTIVE")
        wave_cycles = per("SQ_WAVE_CYCLES")
        valu = per("SQ_INSTS_VALU")
        busy = per("SQ_BUSY_CYCLES")
        if gui:
            cyc = gui / N_XCD  # GPU cycles of the dispatch (the counter sums the XCDs)
            if valu is not None:
                e["valu_per_cu_cycle"] = valu / (cyc * N_CU)
            if wave_cycles is not None:
                # SQ_WAVE_CYCLES counts resident waves every 4 cycles
                e["waves_per_simd"] = 4.0 * wave_cycles / (cyc * N_CU * SIMD_PER_CU)
        if busy is not None:
            e["sq_busy_cycles"] = busy
        for name, key in [("SQ_WAVES", "waves"), ("SQ_INSTS_VALU", "valu_insts"), ("SQ_INSTS_SALU", "salu_insts"),
                          ("SQ_INSTS_VMEM_RD", "vmem_rd_insts"), ("SQ_INSTS_LDS", "lds_insts"),
                          ("SQ_INSTS_BRANCH", "branch_insts"), ("SQ_WAVE_CYCLES", "wave_cycles")]:
            v = per(name)
            if v is not None:
                e[key] = v
        hit, miss = per("TCC_HIT_sum"), per("TCC_MISS_sum")
        if hit is not None and miss is not None and hit + miss > 0:
            e["l2_hit_rate"] = hit / (hit + miss)
        kernels[k] = e
    out = {"name": args.name, "title": args.title, "source_hash": source_hash(), "fetch_scale": fscale,
           "write_scale": wscale, "copy_kib": copy_kib, "copy_fetch_kib": fper, "copy_write_kib": wper,
           "commands": args.cmd or [], "kernels": kernels}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", args.name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(ROOT, "profiles", args.name + ".md"), "w") as f:
        f.write(markdown(out))
    return out


def _f(v, fmt="{:.2f}"):
    return "" if v is None else fmt.format(v)


def markdown(p):
    L = [f"# {p['title']}", "",
         f"Kernel sources hash ({', '.join(SOURCES)}): `{p['source_hash']}`", "",
         "Commands (on the MI355X box, run from /tmp with TMPDIR=/tmp; R = repository root):", "", "```"]
    L += p["commands"] + ["```", ""]
    L += ["Calibration with a device copy of "
          f"{p['copy_kib']:.0f} KiB (`__amd_rocclr_copyBuffer`): FETCH_SIZE reads {_f(p['copy_fetch_kib'], '{:.1f}')}"
          f" KiB (scale {_f(p['fetch_scale'], '{:.4f}')}), WRITE_SIZE {_f(p['copy_write_kib'], '{:.1f}')} KiB "
          f"(scale {_f(p['write_scale'], '{:.4f}')}).", "",
          "VGPR and SGPR are rocprofv3's VGPR_Count and SGPR_Count of the dispatch (the VGPR count is reported in "
          "units of two registers on this device: the megakernel at four waves per SIMD holds 128 VGPRs and shows 64). "
          "Waves/SIMD = 4 x SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x 1024 SIMDs): mean resident waves per SIMD "
          "over the dispatch. VALU/CU-cycle = SQ_INSTS_VALU / (GRBM_GUI_ACTIVE / 8 x 256 CUs): wave64 VALU "
          "instructions issued per CU and cycle (1.0 = the issue limit without packed FP32). L2 hit = "
          "TCC_HIT / (TCC_HIT + TCC_MISS).", "",
          "| kernel | calls | avg us | avg us by stream | VGPR | SGPR | LDS B | scratch B | FETCH KiB | WRITE KiB "
          "| HBM MB / dispatch | VALU / CU-cycle | L2 hit | waves / SIMD |",
          "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, e in p["kernels"].items():
        bys = ", ".join(f"{s}: {v:.1f}" for s, v in e.get("avg_us_by_stream", {}).items())
        L.append(f"| {k} | {e.get('calls', '')} | {_f(e.get('avg_us'), '{:.1f}')} | {bys} | {e.get('vgpr', '')} | "
                 f"{e.get('sgpr', '')} | {e.get('lds', '')} | {e.get('scratch', '')} | "
                 f"{_f(e.get('fetch_kib'), '{:.0f}')} | {_f(e.get('write_kib'), '{:.0f}')} | "
                 f"{_f(e.get('hbm_bytes_per_dispatch', None) and e['hbm_bytes_per_dispatch'] / 1e6)} | "
                 f"{_f(e.get('valu_per_cu_cycle'))} | {_f(e.get('l2_hit_rate'))} | {_f(e.get('waves_per_simd'))} |")
    L += ["", "Instruction counts per dispatch:", "",
          "| kernel | waves | VALU | SALU | VMEM rd | LDS | branch |", "|---|---|---|---|---|---|---|"]
    for k, e in p["kernels"].items():
        if "valu_insts" not in e:
            continue
        L.append(f"| {k} | {_f(e.get('waves'), '{:.3g}')} | {_f(e.get('valu_insts'), '{:.3g}')} | "
                 f"{_f(e.get('salu_insts'), '{:.3g}')} | {_f(e.get('vmem_rd_insts'), '{:.3g}')} | "
                 f"{_f(e.get('lds_insts'), '{:.3g}')} | {_f(e.get('branch_insts'), '{:.3g}')} |")
    return "\n".join(L) + "\n"


def load(name):
    """Figures of profiles/NAME.json, or None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    p = json.load(open(path))
    if p.get("source_hash") != source_hash():
        return None
    return p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-kib", default=str(1 << 20))
    ap.add_argument("--pmc", action="append")
    ap.add_argument("--cmd", action="append")
    args = ap.parse_args()
    summarize(args)


if __name__ == "__main__":
    main()
