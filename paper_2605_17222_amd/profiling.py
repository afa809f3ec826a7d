"""rocprofv3 summaries for the benchmark: per-kernel traces and counters.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats`` and
``--pmc ...``, ``-f csv``) and writes short markdown summaries with a
machine-readable JSON block; ``bench.py`` reads the blocks back.  Every block
records a digest of the library's kernel sources: a counter figure belongs to
the kernels that were profiled, so a reader whose sources differ gets None
instead of a stale number.

Usage (after the rocprofv3 runs, paths to their output directories):

    python -m paper_2605_17222_amd.profiling trace  --dir D --out F --cmd "..."
    python -m paper_2605_17222_amd.profiling hbm    --fetch D1 --write D2 --out F --cmd "..." --cmd "..."
    python -m paper_2605_17222_amd.profiling valu   --dir D --trace D0 --out F --cmd "..."

HBM bytes of a dispatch are FETCH_SIZE and WRITE_SIZE (KiB) scaled by what
the same counters read for a device copy of known size in the same run
(the largest ``__amd_rocclr_copyBuffer`` dispatch; the benchmark's profile
mode copies 256 MiB first).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
from typing import Dict, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIBRATION_BYTES = 256 << 20  # the benchmark's profile mode copies 256 MiB first
CLOCK_HZ = 2.4e9               # MI355X peak engine clock
SIMDS = 256 * 4                # compute units x SIMDs per CU


def sources_digest() -> str:
    """SHA-256 (16 hex digits) over the kernel and host sources of the library."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if f.endswith((".hip", ".cpp", ".hpp")):
            h.update(os.path.basename(f).encode())
            h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """`void ckks::(anonymous namespace)::mac_kernel<4, false>(ckks::MacArgs, ...)` -> `mac_kernel<4, false>`."""
    n = name.strip().strip('"').replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*$", "", n)  # the argument list
    n = n.replace("void ", "").replace("ckks::", "")
    return n.strip()


def _csv(path_glob: str):
    files = sorted(glob.glob(path_glob))
    if not files:
        raise FileNotFoundError(path_glob)
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def read_trace(d: str) -> Dict[str, dict]:
    """Per kernel: calls, total and average duration (us) from the kernel trace."""
    rows = _csv(os.path.join(d, "*kernel_trace.csv"))
    agg = collections.defaultdict(list)
    for r in rows:
        agg[short_name(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: {"calls": len(v), "total_us": sum(v), "avg_us": sum(v) / len(v)} for k, v in agg.items()}


def read_counters(d: str) -> Dict[str, dict]:
    """Per kernel: dispatch count and the per-dispatch mean of every counter
    (a dispatch's value summed over the rows rocprofv3 reports for it), and
    the per-dispatch mean duration (us) of the counter run."""
    rows = _csv(os.path.join(d, "*counter_collection.csv"))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    meta = {}
    for r in rows:
        key = (short_name(r["Kernel_Name"]), r["Dispatch_Id"])
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        meta[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out = collections.defaultdict(lambda: {"dispatches": 0, "counters": collections.defaultdict(float), "us": 0.0,
                                           "max": collections.defaultdict(float)})
    for (k, _), cs in per.items():
        o = out[k]
        o["dispatches"] += 1
        for c, v in cs.items():
            o["counters"][c] += v
            o["max"][c] = max(o["max"][c], v)
    for (k, disp), us in meta.items():
        out[k]["us"] += us
    res = {}
    for k, o in out.items():
        n = o["dispatches"]
        res[k] = {"dispatches": n, "us": o["us"] / n, "counters": {c: v / n for c, v in o["counters"].items()},
                  "max": dict(o["max"])}
    return res


def _largest_copy(cnt: Dict[str, dict], counter: str) -> float:
    """The counter's value for the largest copy dispatch (per dispatch)."""
    rows = [v for k, v in cnt.items() if k.startswith(COPY_KERNEL)]
    if not rows:
        raise RuntimeError("no %s dispatch to calibrate %s" % (COPY_KERNEL, counter))
    return max(v["max"].get(counter, 0.0) for v in rows)


def read_block(path: str) -> Optional[dict]:
    """The JSON block of a summary written by this module, or None."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def current_block(path: str) -> Optional[dict]:
    """The block if it was taken from the current sources, else None."""
    b = read_block(path)
    if b is None or b.get("sources_digest") != sources_digest():
        return None
    return b


def _write(path: str, title: str, cmds, intro: str, table, block: dict, notes: str = ""):
    lines = ["# " + title, "", "Command%s (on one MI355X; the repository at /root/repo):" % ("s" if len(cmds) > 1 else ""),
             "", "```", "export TMPDIR=/tmp; cd /tmp"] + list(cmds) + ["```", ""]
    if intro:
        lines += [intro, ""]
    lines += table + [""]
    if notes:
        lines += [notes, ""]
    lines += ["Machine-readable (read by bench.py; `sources_digest` is a SHA-256 over the library's sources "
              "when the profile was taken):", "", "```json", json.dumps(block, indent=1, sort_keys=True), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def write_trace(d: str, out: str, cmd: str, title: str, intro: str = ""):
    tr = read_trace(d)
    total = sum(v["total_us"] for v in tr.values())
    table = ["| Kernel | Calls | Total ms | Avg us | % |", "|---|---|---|---|---|"]
    for k, v in sorted(tr.items(), key=lambda kv: -kv[1]["total_us"]):
        table.append("| `%s` | %d | %.3f | %.1f | %.2f |" % (k, v["calls"], v["total_us"] / 1e3, v["avg_us"],
                                                             100 * v["total_us"] / total))
    block = {"sources_digest": sources_digest(), "kernels": {k: {"calls": v["calls"], "avg_us": round(v["avg_us"], 3)}
                                                             for k, v in tr.items()}}
    _write(out, title, [cmd], intro, table, block)


def write_hbm(fetch_dir: str, write_dir: str, out: str, cmds, title: str):
    f = read_counters(fetch_dir)
    w = read_counters(write_dir)
    cal_kib = CALIBRATION_BYTES / 1024
    kf = cal_kib / _largest_copy(f, "FETCH_SIZE")
    kw = cal_kib / _largest_copy(w, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(f) & set(w)):
        if k.startswith(COPY_KERNEL):
            continue
        fk = f[k]["counters"].get("FETCH_SIZE", 0.0)
        wk = w[k]["counters"].get("WRITE_SIZE", 0.0)
        hbm = (kf * fk + kw * wk) * 1024
        us = (f[k]["us"] + w[k]["us"]) / 2
        kernels[k] = {"dispatches": f[k]["dispatches"], "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                      "hbm_bytes": round(hbm), "us_counter_run": round(us, 2)}
    table = ["| Kernel | Dispatches | FETCH_SIZE KiB/disp | WRITE_SIZE KiB/disp | HBM MB/disp | avg us (pmc run) | GB/s |",
             "|---|---|---|---|---|---|---|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["hbm_bytes"] * kv[1]["dispatches"]):
        table.append("| `%s` | %d | %.1f | %.1f | %.1f | %.1f | %.0f |" % (
            k, v["dispatches"], v["fetch_kib"], v["write_kib"], v["hbm_bytes"] / 1e6, v["us_counter_run"],
            v["hbm_bytes"] / (v["us_counter_run"] * 1e-6) / 1e9 if v["us_counter_run"] else 0))
    intro = ("Calibration: the largest `%s` dispatch of each run copies %d MiB; it reads FETCH_SIZE = %.1f KiB and "
             "WRITE_SIZE = %.1f KiB, so HBM bytes = %.3f x FETCH_SIZE + %.3f x WRITE_SIZE (KiB per dispatch).  "
             "Durations are from the counter runs (inflated by counter collection)." % (
                 COPY_KERNEL, CALIBRATION_BYTES >> 20, _largest_copy(f, "FETCH_SIZE"), _largest_copy(w, "WRITE_SIZE"),
                 kf, kw))
    block = {"sources_digest": sources_digest(), "fetch_scale": kf, "write_scale": kw, "kernels": kernels}
    _write(out, title, cmds, intro, table, block)


def write_valu(d: str, trace_dir: str, out: str, cmd: str, title: str):
    c = read_counters(d)
    tr = read_trace(trace_dir)
    kernels = {}
    for k, v in c.items():
        cs = v["counters"]
        waves = cs.get("SQ_WAVES", 0.0)
        if not waves or k.startswith(COPY_KERNEL):
            continue
        us = tr[k]["avg_us"] if k in tr else v["us"]
        insts = cs.get("SQ_INSTS_VALU", 0.0)
        kernels[k] = {
            "dispatches": v["dispatches"], "waves": round(waves), "valu_insts_per_wave": round(insts / waves, 1),
            # wave-instructions issued / (SIMDs x cycles / 4): the share of the
            # device's VALU issue slots (a 64-lane instruction occupies a SIMD
            # for at least 4 cycles) over the kernel's traced duration
            "valu_issue_frac": round(insts * 4 / (SIMDS * us * 1e-6 * CLOCK_HZ), 4) if us else None,
            "valu_active_per_wave_cycle": round(cs.get("SQ_ACTIVE_INST_VALU", 0.0) / cs["SQ_WAVE_CYCLES"], 4)
            if cs.get("SQ_WAVE_CYCLES") else None,
            "wait_per_wave_cycle": round(cs.get("SQ_WAIT_ANY", 0.0) / cs["SQ_WAVE_CYCLES"], 4)
            if cs.get("SQ_WAVE_CYCLES") else None,
            "avg_us_trace": round(us, 2),
        }
    table = ["| Kernel | Dispatches | waves/disp | VALU instr/wave | VALU issue share | VALU-active / wave cycle | "
             "waiting / wave cycle |", "|---|---|---|---|---|---|---|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_us_trace"] * kv[1]["dispatches"]):
        table.append("| `%s` | %d | %d | %.0f | %s | %s | %s |" % (
            k, v["dispatches"], v["waves"], v["valu_insts_per_wave"],
            "%.1f%%" % (100 * v["valu_issue_frac"]) if v["valu_issue_frac"] is not None else "-",
            "%.1f%%" % (100 * v["valu_active_per_wave_cycle"]) if v["valu_active_per_wave_cycle"] is not None else "-",
            "%.1f%%" % (100 * v["wait_per_wave_cycle"]) if v["wait_per_wave_cycle"] is not None else "-"))
    intro = ("VALU issue share = SQ_INSTS_VALU x 4 / (1024 SIMDs x traced kernel duration x 2.4 GHz): the share of "
             "the device's VALU issue capacity the kernel used (a 64-lane VALU instruction holds a SIMD for at least "
             "4 cycles, 64-bit integer multiplies longer, so this is a lower bound on the SIMDs' busy time).  "
             "VALU-active and waiting are SQ_ACTIVE_INST_VALU and SQ_WAIT_ANY over SQ_WAVE_CYCLES: shares of the "
             "waves' lifetimes.  Durations from the kernel trace of the same command.")
    block = {"sources_digest": sources_digest(), "kernels": kernels}
    _write(out, title, [cmd], intro, table, block)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("trace")
    a.add_argument("--dir", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("--intro", default="")
    b = sub.add_parser("hbm")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--cmd", action="append", required=True)
    b.add_argument("--title", required=True)
    c = sub.add_parser("valu")
    c.add_argument("--dir", required=True)
    c.add_argument("--trace", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", required=True)
    args = ap.parse_args()
    if args.what == "trace":
        write_trace(args.dir, args.out, args.cmd, args.title, args.intro)
    elif args.what == "hbm":
        write_hbm(args.fetch, args.write, args.out, args.cmd, args.title)
    else:
        write_valu(args.dir, args.trace, args.out, args.cmd, args.title)


if __name__ == "__main__":
    main()
