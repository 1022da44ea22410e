"""Summaries of rocprofv3 output for the library's kernels.

Two summaries are kept as short text files next to the code they describe:

* kernel statistics of a run (``rocprofv3 --kernel-trace --stats``): calls,
  total and average device time per kernel;
* HBM traffic of one kernel from two counter runs (``--pmc FETCH_SIZE`` and
  ``--pmc WRITE_SIZE``, KiB per dispatch), each scaled by what the same
  counter reads for a plain device-to-device copy of known size issued in the
  same process (``bench.py --calibrate-copy``);
* matrix-core use of a rank-k kernel from one run of shader-sequencer
  counters: the cycles the MFMA pipes were busy, summed over the chip, over
  (SIMDs x the kernel's GPU-active cycles per XCD), and the clock those
  active cycles imply over the dispatch's own time stamps.

A traffic summary records a hash of the kernel's sources and build flags;
``traffic_if_current`` returns its figure only while they are unchanged.

Command line (paths are the rocprofv3 CSV files):
  python -m paper_1910_06409_amd.profiling stats STATS_CSV --command "..." > out.txt
  python -m paper_1910_06409_amd.profiling traffic FETCH_CSV WRITE_CSV --family rankk \
      --precision fp64 --copy-bytes N --command-fetch "..." --command-write "..." > out.txt
  python -m paper_1910_06409_amd.profiling mfma COUNTER_CSV AGENT_CSV --precision fp64 \
      --workload "..." --command "..." > out.txt
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# timing family -> device symbol per precision, and the sources that define it
# (every kernel also depends on the shared headers and the build flags)
KERNELS = {
    "plane_sums": ({"fp64": "k_plane_sums", "bf16x3": "k_plane_sums_gy"}, ["k_stats.hip"]),
    "fluct_xfft": ({"fp64": "k_fluct_xfft", "bf16x3": "k_fluct_xfft"}, ["k_spectra.hip"]),
    "zfft_pack": ({"fp64": "k_zfft_pack_blk", "bf16x3": "k_zfft_rec"}, ["k_spectra.hip"]),
    "rankk": ({"fp64": "k_rankk_f64", "bf16x3": "k_rankk_bf16x3"},
              ["k_rankk.hip", "k_rankk_bf16.hip", "rankk_common.h"]),
    "rankk_rem": ({"fp64": "k_rankk_rem", "bf16x3": "k_rankk_rem"},
                  ["k_rankk.hip", "k_rankk_bf16.hip", "rankk_common.h"]),
    "fin_kz": ({"fp64": "k_fin_kz", "bf16x3": "k_fin_kz"}, ["k_final.hip"]),
    "fin_kx": ({"fp64": "k_fin_kx", "bf16x3": "k_fin_kx"}, ["k_final.hip"]),
    "fd_terms": ({"fp64": "k_fd_terms", "bf16x3": "k_fd_terms"}, ["k_final.hip"]),
}
SHARED = ["gke_internal.h", "fft_lds.h", "build.py"]
COPY_KERNEL = "copyBuffer"


def symbol(family: str, precision: str) -> str:
    return KERNELS[family][0][precision]


def source_hash(family: str) -> str:
    h = hashlib.sha256()
    for name in KERNELS[family][1] + SHARED:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_csv(path: str) -> list[dict]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    """Kernel name without its argument list and namespace."""
    base = name.split("(")[0]
    return base.replace("void ", "").replace("gke::", "")


def stats_summary(stats_csv: str, command: str) -> str:
    rows = read_csv(stats_csv)
    out = ["# rocprofv3 kernel statistics", f"# command: {command}",
           f"{'kernel':<44} {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'pct':>6}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"{_short(r['Name'])[:44]:<44} {int(r['Calls']):>7} "
                   f"{float(r['TotalDurationNs']) / 1e6:>10.3f} "
                   f"{float(r['AverageNs']) / 1e3:>10.2f} {float(r['Percentage']):>6.2f}")
    return "\n".join(out) + "\n"


def counter_values(rows: list[dict], counter: str, match: str) -> list[tuple[int, float]]:
    """(grid size, value) of every dispatch whose kernel name contains `match`."""
    vals = []
    for r in rows:
        if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
            vals.append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return vals


def copy_reading(rows: list[dict], counter: str) -> float:
    """Mean counter value of the calibration copies: the copy dispatches that
    read within 10 % of the largest reading (the calibration copy is by far the
    largest copy of the run; every copy dispatch has the same grid)."""
    vals = [v for _, v in counter_values(rows, counter, COPY_KERNEL)]
    if not vals:
        raise ValueError(f"no {COPY_KERNEL} dispatch with {counter}")
    big = [v for v in vals if v >= 0.9 * max(vals)]
    return sum(big) / len(big)


def kernel_reading(rows: list[dict], counter: str, sym: str) -> tuple[float, int]:
    vals = [v for _, v in counter_values(rows, counter, sym + "(")]
    if not vals:
        vals = [v for _, v in counter_values(rows, counter, sym)]
    if not vals:
        raise ValueError(f"no dispatch of {sym} with {counter}")
    return sum(vals) / len(vals), len(vals)


def traffic_summary(fetch_csv: str, write_csv: str, family: str, precision: str,
                    copy_bytes: int, command_fetch: str, command_write: str,
                    workload: str) -> str:
    sym = symbol(family, precision)
    fr, wr = read_csv(fetch_csv), read_csv(write_csv)
    cf, cw = copy_reading(fr, "FETCH_SIZE"), copy_reading(wr, "WRITE_SIZE")
    kf, nf = kernel_reading(fr, "FETCH_SIZE", sym)
    kw, nw = kernel_reading(wr, "WRITE_SIZE", sym)
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    fetch_b, write_b = kf * 1024.0 * ff, kw * 1024.0 * fw
    lines = [
        f"# HBM traffic of {sym} ({family}), {workload}, rank-k precision {precision}",
        f"# fetch command: {command_fetch}",
        f"# write command: {command_write}",
        f"family: {family}",
        f"precision: {precision}",
        f"kernel: {sym}",
        f"source_hash: {source_hash(family)}",
        f"copy_bytes: {copy_bytes}",
        f"copy_fetch_kib: {cf:.1f}",
        f"copy_write_kib: {cw:.1f}",
        f"fetch_factor: {ff:.4f}",
        f"write_factor: {fw:.4f}",
        f"kernel_dispatches: {nf} {nw}",
        f"kernel_fetch_kib: {kf:.1f}",
        f"kernel_write_kib: {kw:.1f}",
        f"fetch_bytes_per_launch: {fetch_b:.0f}",
        f"write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    return "\n".join(lines) + "\n"


MFMA_COUNTERS = ["SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_WAVES", "SQ_WAVE_CYCLES",
                 "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY",
                 "SQ_ACTIVE_INST_VALU"]


def gpu_agent(agent_csv: str) -> tuple[int, int]:
    """(SIMDs, XCDs) of the profiled GPU."""
    for r in read_csv(agent_csv):
        if r["Agent_Type"] == "GPU":
            return int(r["Simd_Count"]), int(r["Num_Xcc"])
    raise ValueError("no GPU agent")


def mfma_summary(counter_csv: str, agent_csv: str, precision: str, workload: str,
                 command: str) -> str:
    """Per-dispatch means of the shader-sequencer counters of the rank-k
    kernel and the fraction of cycles its matrix pipes were busy."""
    sym = symbol("rankk", precision)
    simds, xcc = gpu_agent(agent_csv)
    per = {}   # dispatch -> {counter: value}, plus its duration
    for r in read_csv(counter_csv):
        if sym + "(" not in r["Kernel_Name"] and not r["Kernel_Name"].endswith(sym):
            continue
        d = per.setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["_ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    if not per:
        raise ValueError(f"no dispatch of {sym}")
    mean = {c: sum(d[c] for d in per.values()) / len(per)
            for c in MFMA_COUNTERS + ["_ns"] if all(c in d for d in per.values())}
    active = mean["GRBM_GUI_ACTIVE"] / xcc   # GPU-active cycles of one XCD
    busy = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * active)
    lines = [
        f"# matrix-core use of {sym} (rankk), {workload}, precision {precision}",
        f"# command: {command}",
        "family: rankk",
        f"precision: {precision}",
        f"kernel: {sym}",
        f"source_hash: {source_hash('rankk')}",
        f"dispatches: {len(per)}",
        f"simds: {simds}",
        f"xcds: {xcc}",
    ]
    lines += [f"{c}: {mean[c]:.0f}" for c in MFMA_COUNTERS if c in mean]
    lines += [
        f"dispatch_ns: {mean['_ns']:.0f}",
        f"active_cycles_per_xcd: {active:.0f}",
        f"clock_ghz: {active / mean['_ns']:.3f}",
        f"mfma_busy_fraction: {busy:.4f}",
    ]
    if "SQ_WAVES" in mean:
        lines.append(f"mfma_busy_cycles_per_wave: "
                     f"{mean['SQ_VALU_MFMA_BUSY_CYCLES'] / mean['SQ_WAVES']:.0f}")
    return "\n".join(lines) + "\n"


def read_summary(path: str) -> dict:
    d = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    return d


def read_summary_if_current(path: str, family: str) -> dict | None:
    """A committed summary's fields, provided the kernel's sources still
    hash to the value it records (else None)."""
    if not os.path.exists(path):
        return None
    d = read_summary(path)
    if d.get("source_hash") != source_hash(family):
        return None
    return d


def stated_error(path: str) -> dict | None:
    """Per-term errors recorded for a workload (a committed text file:
    `T1: 1.2e-07` lines for the norm-wise error, `pw_T1: ...` lines for the
    pointwise relative error over the points where |T| > 1e-3 max|T|, a
    `source:` line naming the test that measured them and a `command:`
    comment)."""
    if not os.path.exists(path):
        return None
    terms, pw, out = {}, {}, {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                if line.startswith("# command:"):
                    out["command"] = line.split(":", 1)[1].strip()
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k.startswith("T") and k[1:].isdigit():
                terms[k] = float(v)
            elif k.startswith("pw_T") and k[4:].isdigit():
                pw[k[3:]] = float(v)
            else:
                out[k] = v
    if not terms:
        return None
    out["per_term"] = terms
    out["max"] = max(terms.values())
    if pw:
        out["pointwise_per_term"] = pw
    return out


def traffic_if_current(path: str, family: str, precision: str) -> float | None:
    """Bytes per launch from a traffic summary, or None when there is none or
    the kernel's sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    d = read_summary(path)
    if d.get("family") != family or d.get("precision") != precision:
        return None
    if d.get("source_hash") != source_hash(family):
        return None
    return float(d["traffic_bytes_per_launch"])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="rocprofv3 summaries")
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("stats_csv")
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--family", required=True, choices=sorted(KERNELS))
    t.add_argument("--precision", default="fp64", choices=["fp64", "bf16x3"])
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("counter_csv")
    m.add_argument("agent_csv")
    m.add_argument("--precision", default="fp64", choices=["fp64", "bf16x3"])
    m.add_argument("--workload", required=True)
    m.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.what == "mfma":
        sys.stdout.write(mfma_summary(a.counter_csv, a.agent_csv, a.precision, a.workload,
                                      a.command))
    elif a.what == "stats":
        sys.stdout.write(stats_summary(a.stats_csv, a.command))
    else:
        sys.stdout.write(traffic_summary(a.fetch_csv, a.write_csv, a.family, a.precision,
                                         a.copy_bytes, a.command_fetch, a.command_write,
                                         a.workload))
    return 0


if __name__ == "__main__":
    sys.exit(main())
