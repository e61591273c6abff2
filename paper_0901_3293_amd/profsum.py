"""Summarise rocprofv3 result databases (kernel trace + FETCH_SIZE/WRITE_SIZE
passes) into a short text table: per kernel, average duration, HBM bytes per
dispatch (counter KiB scaled by the reading of a plain copy of known size),
and the algorithmic bytes the kernel has to move.

usage: python -m paper_0901_3293_amd.profsum TRACE_DB [FETCH_DB WRITE_DB]
       --copy-bytes 536870912 --alg k_lb=VALUES ... --esz 4 --sites N
       [--mfma]   (convolution kernels: padded MFMA flops per dispatch from the
                   channel counts in the kernel name, TFLOP/s against 2.5 PFLOP/s)
       [--valu DB] (a pass of SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_WAVES,
                   GRBM_GUI_ACTIVE: VALU instructions per site and the time
                   their issue takes at the chip's vector rate against the
                   kernel's duration)
       [--stall DB] (a pass of SQ_WAVE_CYCLES and other SQ_ cycle counters,
                   e.g. SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_*: each
                   as a share of the cycles the waves were resident)
With the trace alone: calls, average and total duration per kernel, and the
algorithmic rate where --alg gives the kernel's values per site.
"""
from __future__ import annotations

import argparse
import re
import sqlite3
from collections import defaultdict


# Sources of the step kernels; their hash tags traffic records so that a
# record taken on other kernels is not used.
KERNEL_SOURCES = ["kernels.hip", "site.h", "sitekern.h", "tiles.h", "kernels.h"]


def kernel_source_sha():
    """sha256 (first 16 hex digits) of the step kernels' sources."""
    import hashlib
    import os

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    m = re.search(r"k_conv<(\d+), (\d+), (\d+)", name)
    if m:  # keep the channel counts and epilogue mode of the convolutions
        return f"k_conv<{m.group(1)},{m.group(2)},{m.group(3)}>"
    m = re.search(r"k_wgrad<(\d+)>", name)
    if m:  # weight gradient: 32 input channels, COP output channels
        return f"k_wgrad<32,{m.group(1)}>"
    m = re.search(r"k_phase<(?:float|double), (\d)>", name)
    if m:  # batched phase kernels: stress, LB, predictor, corrector
        return "k_phase_" + ("stress", "lb", "pred", "corr")[int(m.group(1))]
    m = re.search(r"(k_\w+|__amd_rocclr_copyBuffer)", name)
    return m.group(1) if m else name[:40]


def conv_flops(k, sites):
    """Padded multiply-adds x 2 of one dispatch of a 3x3x3 convolution (or its
    weight gradient) over `sites` sites, from the channel counts in its name."""
    m = re.match(r"k_(conv|wgrad)<(\d+),(\d+)", k)
    return 2.0 * sites * 27 * int(m.group(2)) * int(m.group(3)) if m else float("nan")


def trace(db):
    con = sqlite3.connect(db)
    d = defaultdict(list)
    for name, dur in con.execute("select name, duration from kernels"):
        d[short(name)].append(dur)
    return {k: (len(v), sum(v) / len(v) / 1e3) for k, v in d.items()}  # us


COPY = "__amd_rocclr_copyBuffer"


def counter(db, cname):
    """Value per dispatch, averaged per kernel (KiB for FETCH_SIZE and
    WRITE_SIZE).  A counter read from several hardware instances (one row
    per shader engine or XCD) is reduced per dispatch first: summed, or the
    maximum for GRBM_ (clock-type) counters.  For the runtime's copy kernel
    only the dispatches of the calibration copy (the largest ones) count."""
    con = sqlite3.connect(db)
    per = defaultdict(list)
    for name, disp, v in con.execute(
            "select name, dispatch_id, counter_value from pmc_events where counter_name = ?", (cname,)):
        per[(short(name), disp)].append(v)
    red = max if cname.startswith("GRBM_") else sum
    d = defaultdict(list)
    for (k, _), vals in per.items():
        d[k].append(red(vals))
    if COPY in d:
        top = max(d[COPY])
        if top > 0:
            d[COPY] = [v for v in d[COPY] if v > 0.5 * top]
    return {k: sum(v) / len(v) for k, v in d.items() if v}


# Vector issue rate of the chip: 256 CUs x 4 SIMDs, one 64-lane VALU
# instruction per SIMD every 4 cycles (16 lanes per cycle), at 2.4 GHz.
SIMDS = 1024
CLOCK_HZ = 2.4e9


def valu_table(t, db, sites):
    """Per kernel: VALU instructions per site (wave instructions x 64 lanes /
    sites), the issue time of those instructions at the chip's full vector
    rate (the ALU bound of the kernel), its fraction of the measured
    duration, and the waves and VALU-active cycles the counters saw."""
    cs = {c: counter(db, c) for c in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE")}
    print(f"{'kernel':12s} {'avg_us':>8s} {'waves':>9s} {'valu/site':>9s} {'alu_us':>7s} {'alu/dur':>7s} "
          f"{'gui_MHz':>8s}")
    for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if k == COPY or k not in cs["SQ_INSTS_VALU"]:
            continue
        wi = cs["SQ_INSTS_VALU"][k]
        per_site = wi * 64 / sites
        alu_us = wi * 4 / SIMDS / CLOCK_HZ * 1e6
        gui = cs["GRBM_GUI_ACTIVE"].get(k, float("nan"))
        print(f"{k:12s} {us:8.2f} {cs['SQ_WAVES'].get(k, float('nan')):9.0f} {per_site:9.1f} {alu_us:7.2f} "
              f"{alu_us / us:7.2f} {gui / us:8.0f}")


def stall_table(t, db):
    """Per kernel: every SQ_ counter of the pass (summed over the chip per
    dispatch) as a share of SQ_WAVE_CYCLES, the cycles its waves were
    resident -- the share of wave time spent waiting, or issuing a given
    kind of instruction."""
    con = sqlite3.connect(db)
    names = sorted(r[0] for r in con.execute("select distinct counter_name from pmc_events")
                   if r[0].startswith("SQ_") and r[0] != "SQ_WAVE_CYCLES")
    cyc = counter(db, "SQ_WAVE_CYCLES")
    cs = {c: counter(db, c) for c in names}
    print(f"{'kernel':12s} {'avg_us':>8s} " + " ".join(f"{c[3:]:>16s}" for c in names))
    for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if k == COPY or not cyc.get(k):
            continue
        print(f"{k:12s} {us:8.2f} " + " ".join(f"{cs[c].get(k, float('nan')) / cyc[k]:16.3f}" for c in names))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace_db")
    ap.add_argument("fetch_db", nargs="?")
    ap.add_argument("write_db", nargs="?")
    ap.add_argument("--copy-bytes", type=float, default=512 * 2 ** 20)
    ap.add_argument("--sites", type=int, required=True)
    ap.add_argument("--esz", type=int, required=True)
    ap.add_argument("--alg", nargs="*", default=[], help="kernel=values_per_site")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    ap.add_argument("--mfma", action="store_true")
    ap.add_argument("--valu", default=None, help="database of a VALU counter pass")
    ap.add_argument("--stall", default=None, help="database of a pass of SQ_ cycle counters with SQ_WAVE_CYCLES")
    ap.add_argument("--traffic-json", default=None, metavar="PREC",
                    help="also print the line 'bench-traffic: {json}' with the HBM bytes per dispatch of "
                         "every step kernel for precision PREC (fp32/fp64), tagged with the kernel sources' hash")
    a = ap.parse_args()
    alg = {k: float(v) for k, v in (x.split("=") for x in a.alg)}
    t = trace(a.trace_db)
    if a.stall:
        print(f"# {a.title}")
        stall_table(t, a.stall)
        return
    if a.valu:
        print(f"# {a.title}")
        if a.command:
            print(f"command: {a.command}")
        valu_table(t, a.valu, a.sites)
        return
    if a.fetch_db is None or a.write_db is None:
        print(f"# {a.title}")
        print(f"{'kernel':16s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'alg_MB':>8s} {'alg_GB/s':>9s}")
        for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            al = alg.get(k, float("nan")) * a.esz * a.sites / 1e6
            print(f"{k:16s} {n:6d} {us:9.2f} {n * us / 1e3:9.3f} {al:8.1f} {al / us * 1e3:9.0f}")
        return
    fe = counter(a.fetch_db, "FETCH_SIZE")
    wr = counter(a.write_db, "WRITE_SIZE")
    cname = COPY
    fscale = a.copy_bytes / (fe[cname] * 1024)
    wscale = a.copy_bytes / (wr[cname] * 1024)
    print(f"# {a.title}")
    if a.command:
        print(f"command: {a.command}")
    print(f"copy calibration: {a.copy_bytes / 2**20:.0f} MiB copy reads FETCH_SIZE {fe[cname]:.0f} KiB, "
          f"WRITE_SIZE {wr[cname]:.0f} KiB -> scale fetch x{fscale:.3f}, write x{wscale:.3f}")
    if a.mfma:
        print(f"{'kernel':18s} {'calls':>5s} {'avg_us':>9s} {'fetch_MB':>9s} {'write_MB':>9s} {'hbm_GB/s':>9s} "
              f"{'GFLOP':>8s} {'TFLOP/s':>8s} {'of_2.5P':>8s}")
        for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            if k == cname:
                continue
            f = fe.get(k, float("nan")) * 1024 * fscale / 1e6
            w = wr.get(k, float("nan")) * 1024 * wscale / 1e6
            fl = conv_flops(k, a.sites)
            print(f"{k:18s} {n:5d} {us:9.2f} {f:9.1f} {w:9.1f} {(f + w) / us * 1e3:9.0f} {fl / 1e9:8.1f} "
                  f"{fl / us / 1e6:8.1f} {fl / us / 1e6 / 2500:8.3f}")
        return
    print(f"{'kernel':12s} {'calls':>5s} {'avg_us':>9s} {'fetch_MB':>9s} {'write_MB':>9s} {'hbm_MB':>8s} "
          f"{'alg_MB':>8s} {'hbm/alg':>7s} {'alg_GB/s':>9s} {'hbm_GB/s':>9s}")
    rec = {}
    for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if k == cname:
            continue
        f = fe.get(k, float("nan")) * 1024 * fscale / 1e6
        w = wr.get(k, float("nan")) * 1024 * wscale / 1e6
        al = alg.get(k, float("nan")) * a.esz * a.sites / 1e6
        print(f"{k:12s} {n:5d} {us:9.2f} {f:9.1f} {w:9.1f} {f + w:8.1f} {al:8.1f} {(f + w) / al:7.2f} "
              f"{al / us * 1e3:9.0f} {(f + w) / us * 1e3:9.0f}")
        if k in alg and f + w == f + w:  # step kernels with counter readings
            rec[k] = round((f + w) * 1e6)
    if a.traffic_json:
        import json

        print("bench-traffic: " + json.dumps({"kernel_source_sha": kernel_source_sha(), a.traffic_json: rec}))


if __name__ == "__main__":
    main()
