"""Summaries of rocprofv3 output for this library's kernels.

rocprofv3 writes one CSV row per (dispatch, counter) for ``--pmc`` runs and one
row per dispatch for ``--kernel-trace``.  This module reduces them to per-kernel
means, turns the memory-side request counters into bytes per dispatch, and
writes/reads the short text summaries kept beside the benchmark.

Bytes read past L2 come either from the read requests by size,
32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B (exact; a
plain copy kernel of known size is then only a check), or from FETCH_SIZE
scaled by that copy kernel.  FETCH_SIZE counts a 128-byte read as 64 bytes on
this GPU, so the copy (all 128-byte reads) gives a factor near 2, while
instruction fetches (64-byte reads) are counted in full: for a kernel whose
reads are mostly code, the scaled FETCH_SIZE overstates its bytes.  Bytes
written come from WRITE_SIZE, which the copy reproduces exactly.

  python -m paper_2302_11719_amd.profile_summary traffic \\
      --fetch DIR --write DIR --kernel NAME [--kernel NAME ...] --copy-bytes N [--trace DIR] \\
      --out FILE --command "..."
  python -m paper_2302_11719_amd.profile_summary counters --pmc DIR [DIR ...] --trace DIR \\
      --kernel NAME [--kernel NAME ...] --out FILE --command "..."
  python -m paper_2302_11719_amd.profile_summary stats --trace DIR --out FILE --command "..."

A traffic summary carries a digest of the kernel sources; ``load_traffic``
returns None once the sources have changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNELS = ("__amd_rocclr_copyBuffer", "copyBuffer")
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak (packed FMA); 78.6e12 without packing
PEAK_HBM = 8.0e12


def kernel_sources_digest() -> str:
    """sha256 over the HIP sources (sorted by name), first 16 hex digits."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if f.endswith((".hip", ".hpp", ".h")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(kernel: str) -> str:
    """'void ns::k_fused<0, 192, 1, true>(ns::FusedArgs) [clone .kd]' -> 'k_fused<0, 192, 1, true>'
    (namespaces and the parameter list dropped)."""
    k = re.sub(r"^void\s+", "", kernel.strip())
    k = re.sub(r"\s*\[clone.*$", "", k)
    k = k.replace("(anonymous namespace)::", "")
    k = re.sub(r"^(\w+::)+", "", k)
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return k[:i]
    return k


def _csvs(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def read_counters(d: str):
    """{kernel short name: {counter: [value per dispatch]}} from a --pmc run."""
    per = defaultdict(lambda: defaultdict(dict))
    for f in _csvs(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = short_name(r["Kernel_Name"])
                disp = (f, r["Dispatch_Id"])
                c = r["Counter_Name"]
                per[k][c][disp] = per[k][c].get(disp, 0.0) + float(r["Counter_Value"])
    return {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in per.items()}


def read_trace(d: str):
    """{kernel short name: [duration ns per dispatch]} from a --kernel-trace run."""
    out = defaultdict(list)
    for f in _csvs(d, "kernel_trace.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                out[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return dict(out)


def read_stats(d: str):
    rows = []
    for f in _csvs(d, "kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _match(names, pattern):
    return [k for k in names if k == pattern or k.startswith(pattern + "<") or k.startswith(pattern + "(")]


def _mean(v):
    return sum(v) / len(v) if v else float("nan")


def _copy_factor(counters, counter, copy_bytes):
    """Known bytes / counter bytes for the plain copy kernel (largest dispatch)."""
    for k in counters:
        if any(c in k for c in COPY_KERNELS) and counter in counters[k]:
            kib = max(counters[k][counter])
            if kib > 0:
                return copy_bytes / (kib * 1024.0), kib
    return None, None


RDREQ = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))


def read_bytes(cs):
    """Bytes read past L2 per dispatch from the read requests by size, or None
    when the run did not take those counters."""
    if not all(c in cs for c, _ in RDREQ):
        return None
    cols = [cs[c] for c, _ in RDREQ]
    return [sum(n * b for n, (_, b) in zip(v, RDREQ)) for v in zip(*cols)]


def traffic_summary(fetch_dir, write_dir, kernel, copy_bytes, trace=None):
    """HBM bytes per dispatch of the kernels matching `kernel` (a name or a list
    of names); with a kernel trace, also the mean duration and GB/s.  The read
    side is exact when `fetch_dir` holds the request-size counters, else
    FETCH_SIZE scaled by the copy kernel."""
    fc, wc = read_counters(fetch_dir), read_counters(write_dir)
    tr = read_trace(trace) if trace else {}
    by_size = any(read_bytes(cs) is not None for cs in fc.values())
    if by_size:
        ff, fcopy = None, None
        for k, cs in fc.items():
            if any(c in k for c in COPY_KERNELS) and read_bytes(cs):
                fcopy = max(read_bytes(cs)) / 1024.0
                ff = copy_bytes / (fcopy * 1024.0) if fcopy > 0 else None
                break
    else:
        ff, fcopy = _copy_factor(fc, "FETCH_SIZE", copy_bytes)
    wf, wcopy = _copy_factor(wc, "WRITE_SIZE", copy_bytes)
    out = {"digest": kernel_sources_digest(), "copy_bytes": copy_bytes,
           "read_method": "request sizes" if by_size else "FETCH_SIZE x copy factor",
           "copy_fetch_kib": fcopy, "copy_write_kib": wcopy, "fetch_factor": ff, "write_factor": wf,
           "kernels": {}}
    pats = [kernel] if isinstance(kernel, str) else list(kernel)
    names = sorted({k for pat in pats for k in set(_match(fc, pat)) | set(_match(wc, pat))})
    for k in names:
        if by_size:
            fk = [b / 1024.0 for b in (read_bytes(fc.get(k, {})) or [])]
            fb = _mean(fk) * 1024.0
        else:
            fk = fc.get(k, {}).get("FETCH_SIZE", [])
            fb = _mean(fk) * 1024.0 * (ff or float("nan"))
        wk = wc.get(k, {}).get("WRITE_SIZE", [])
        wb = _mean(wk) * 1024.0 * (wf or float("nan"))
        out["kernels"][k] = {"dispatches": [len(fk), len(wk)], "fetch_kib": _mean(fk), "write_kib": _mean(wk),
                             "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
        if tr.get(k):
            dur = _mean(tr[k])
            out["kernels"][k]["duration_ns"] = dur
            out["kernels"][k]["hbm_gbps"] = (fb + wb) / dur
            out["kernels"][k]["frac_hbm_peak"] = (fb + wb) / dur / (PEAK_HBM / 1e9)
    return out


def derived(cs, simds=1024, xcds=8):
    """Derived rates of one kernel's mean counters (keys as rocprofv3 names them):
    FP32 FLOP from the VALU instruction mix (64 lanes per instruction, FMA = 2),
    its rate against the vector peaks, and VALU issue utilisation (each wave64
    VALU instruction holds its SIMD for 4 cycles; GRBM_GUI_ACTIVE counts cycles on
    every XCD)."""
    out = {}
    dur = cs.get("duration_ns", float("nan"))
    if "SQ_INSTS_VALU_FLOPS_FP32" in cs:
        fl = 64.0 * cs["SQ_INSTS_VALU_FLOPS_FP32"]
        out["fp32_flop_per_dispatch"] = fl
        out["fp32_tflops"] = fl / dur / 1e3
        out["frac_fp32_peak_packed"] = fl / dur / (PEAK_FP32 / 1e9)
        out["frac_fp32_peak_unpacked"] = 2 * fl / dur / (PEAK_FP32 / 1e9)
    if "SQC_TC_INST_REQ" in cs:
        # instruction caches fetch 64-byte lines from L2
        out["l2_instruction_request_bytes"] = 64.0 * cs["SQC_TC_INST_REQ"]
    if "TCC_MISS_sum" in cs:
        # L2 lines are 128 bytes
        out["l2_miss_line_bytes"] = 128.0 * cs["TCC_MISS_sum"]
        if "TCC_HIT_sum" in cs:
            out["l2_hit_rate"] = cs["TCC_HIT_sum"] / max(cs["TCC_HIT_sum"] + cs["TCC_MISS_sum"], 1.0)
    if "GRBM_GUI_ACTIVE" in cs:
        cyc = cs["GRBM_GUI_ACTIVE"] / xcds
        out["gui_active_ghz"] = cyc / dur
        if "SQ_INSTS_VALU" in cs:
            out["valu_issue_util"] = 4.0 * cs["SQ_INSTS_VALU"] / (simds * cyc)
        if "SQ_ACTIVE_INST_VALU" in cs:
            out["active_inst_valu_util"] = 4.0 * cs["SQ_ACTIVE_INST_VALU"] / (simds * cyc)
    return out


def _md_table(head, rows):
    s = "| " + " | ".join(head) + " |\n|" + "---|" * len(head) + "\n"
    for r in rows:
        s += "| " + " | ".join(str(x) for x in r) + " |\n"
    return s


def write_md(path, title, command, body, payload):
    with open(path, "w") as fh:
        fh.write(f"# {title}\n\nCommand (from the repository root on the GPU host):\n\n```\n{command}\n```\n\n")
        fh.write(body)
        fh.write("\n```json\n" + json.dumps(payload, indent=1, sort_keys=True) + "\n```\n")


def load_payload(path):
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    return json.loads(m.group(1)) if m else None


def load_traffic(path, kernel_prefix):
    """(bytes per launch, summary) for the first kernel matching the prefix, or
    (None, reason) when the summary is missing or the sources have changed."""
    p = load_payload(path)
    if p is None:
        return None, "no traffic summary"
    if p.get("digest") != kernel_sources_digest():
        return None, "kernel sources changed since the counters were taken"
    for k, v in p.get("kernels", {}).items():
        if k.startswith(kernel_prefix):
            return v["traffic_bytes"], p
    return None, "kernel not in summary"


def _cmd_traffic(a):
    s = traffic_summary(a.fetch, a.write, a.kernel, a.copy_bytes, a.trace)
    rows = [[k, v["dispatches"], f"{v['fetch_kib']:.1f}", f"{v['write_kib']:.1f}", f"{v['traffic_bytes']:.0f}",
             f"{v['duration_ns']:.0f}" if "duration_ns" in v else "",
             f"{v['hbm_gbps']:.2f} ({100 * v['frac_hbm_peak']:.3f} %)" if "hbm_gbps" in v else ""]
            for k, v in s["kernels"].items()]
    if s["read_method"] == "request sizes":
        how = (f"Read bytes = 32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B (TCC_EA0, summed over the L2 "
               f"channels), used as counted; the plain copy of {a.copy_bytes} bytes reads {s['copy_fetch_kib']} KiB "
               f"by the same sum (known / counted {s['fetch_factor']}, a check, not applied).  Write bytes = "
               f"WRITE_SIZE; the copy writes {s['copy_write_kib']} KiB by it (factor {s['write_factor']}, applied).")
        fcol = "read KiB/dispatch (by request size)"
    else:
        how = (f"Plain copy of {a.copy_bytes} bytes (read + write) reads FETCH_SIZE {s['copy_fetch_kib']} KiB and "
               f"WRITE_SIZE {s['copy_write_kib']} KiB; factors (known / counted) fetch {s['fetch_factor']}, "
               f"write {s['write_factor']}, applied.")
        fcol = "FETCH_SIZE KiB/dispatch"
    body = (how + f"  GB/s: bytes / mean duration from the kernel trace (fraction of {PEAK_HBM / 1e12:.0f} TB/s)."
            "\n\n" + _md_table(["kernel", "dispatches (read, write run)", fcol, "WRITE_SIZE KiB/dispatch",
                                 "HBM bytes/dispatch", "duration ns", "HBM GB/s"], rows))
    write_md(a.out, a.title or f"HBM traffic of {', '.join(a.kernel)}", a.command, body, s)


def _cmd_counters(a):
    merged = defaultdict(dict)
    for d in a.pmc:
        for k, cs in read_counters(d).items():
            for c, v in cs.items():
                merged[k][c] = v
    tr = read_trace(a.trace) if a.trace else {}
    payload = {"digest": kernel_sources_digest(), "kernels": {}}
    rows = []
    for pat in a.kernel:
        for k in _match(merged, pat):
            cs = {c: _mean(v) for c, v in merged[k].items()}
            dur = _mean(tr.get(k, [])) if tr else float("nan")
            cs["duration_ns"] = dur
            dv = derived(cs, a.simds, a.xcds)
            payload["kernels"][k] = dict(cs, derived=dv)
            for c in sorted(cs):
                rows.append([k, c, f"{cs[c]:.6g}"])
            for c in sorted(dv):
                rows.append([k, f"derived: {c}", f"{dv[c]:.4g}"])
    note = ("Derived rows: fp32_flop = 64 x SQ_INSTS_VALU_FLOPS_FP32 (the ADD + MUL + TRANS + 2 FMA "
            "instruction mix, 64 lanes each), fp32_tflops = that / duration, frac_fp32_peak_packed = of "
            f"{PEAK_FP32 / 1e12} TFLOP/s, frac_fp32_peak_unpacked = of {PEAK_FP32 / 2e12} (packed FP32 is off in "
            f"this build); cycles = GRBM_GUI_ACTIVE / {a.xcds} XCDs, gui_active_ghz = cycles / duration (the "
            "clock for long kernels; a short kernel's count also covers its dispatch, so it reads high); "
            f"valu_issue_util = 4 cycles x SQ_INSTS_VALU / ({a.simds} SIMDs x cycles), active_inst_valu_util "
            "the same with SQ_ACTIVE_INST_VALU; l2_instruction_request_bytes = 64 x SQC_TC_INST_REQ (instruction "
            "cache lines requested from L2), l2_miss_line_bytes = 128 x TCC_MISS_sum, l2_hit_rate = hits / "
            "(hits + misses).\n\n")
    write_md(a.out, a.title or "Counters", a.command,
             note + _md_table(["kernel", "counter (mean per dispatch)", "value"], rows), payload)


def _cmd_stats(a):
    rows = read_stats(a.trace)
    keep = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"]
    rows = sorted(rows, key=lambda r: -float(r.get("TotalDurationNs", 0)))[: a.top]
    body = _md_table(keep, [[short_name(r["Name"]) if c == "Name" else r.get(c, "") for c in keep] for r in rows])
    payload = {"digest": kernel_sources_digest(),
               "kernels": {short_name(r["Name"]): {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"])}
                           for r in rows}}
    write_md(a.out, a.title or "Kernel statistics", a.command, body, payload)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", action="append", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--trace")
    c = sub.add_parser("counters")
    c.add_argument("--pmc", nargs="+", required=True)
    c.add_argument("--trace")
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--xcds", type=int, default=8)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--top", type=int, default=20)
    for p in (t, c, s):
        p.add_argument("--out", required=True)
        p.add_argument("--command", required=True)
        p.add_argument("--title")
    a = ap.parse_args(argv)
    {"traffic": _cmd_traffic, "counters": _cmd_counters, "stats": _cmd_stats}[a.cmd](a)


if __name__ == "__main__":
    main()
