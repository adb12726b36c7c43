"""Summaries of rocprofv3 output for the benchmark's kernels.

``python -m paper_1211_0582_amd.profiling stats <kernel_stats.csv | results.db> <out.txt> <command...>``
    writes the per-kernel duration table of a ``--kernel-trace --stats`` run
    (from the CSV summary, or from the rocpd database, where launches are
    grouped by kernel and grid size so that one kernel on meshes of
    different sizes gives one row per mesh).
``python -m paper_1211_0582_amd.profiling traffic <fetch_dir> <write_dir> <out.txt> <substr> <copy_bytes> <command...>``
    writes the HBM traffic per dispatch of the kernels whose name contains
    ``substr``: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two
    ``--pmc`` runs, each scaled by what the same counter reads for a plain
    copy of ``copy_bytes`` bytes in the same run.

``python -m paper_1211_0582_amd.profiling counters <dir> <out.txt> <substr> <command...>``
    writes, per kernel and launch size, the matrix-core busy fraction, the
    mean waves per SIMD, the vector-ALU issue fraction, the share of wave time
    spent waiting on outstanding instructions, LDS bank-conflict and
    texture-address (TA) busy fractions per CU, VALU / MFMA / LDS
    instructions per dispatch, and the HBM bytes from the 32-byte-granular
    EA counters, from one or more ``--pmc`` runs (SQ counters are summed over
    all SIMDs, GRBM_GUI_ACTIVE over the 8 XCDs, TA and TCP counters over the
    256 CUs).

The traffic summary records a hash of the kernel sources; ``bench.py`` only
reports the traffic while the sources still hash to that value.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def source_hash(csrc: str | None = None) -> str:
    """sha256 over the HIP/C++ sources of the library (sorted by name), with
    comments and whitespace removed: only a change of the code itself makes a
    recorded traffic figure stale."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(csrc or os.path.join(HERE, "csrc"), "*"))):
        if path.endswith((".hip", ".hpp", ".cpp")):
            h.update(os.path.basename(path).encode())
            with open(path, encoding="utf-8") as f:
                code = _COMMENT.sub(" ", f.read())
            h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def stats_summary_db(db_path: str, command: str) -> str:
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, grid_x, workgroup_x, count(*), avg(duration), min(duration), max(duration), "
                       "sum(duration) from kernels group by name, grid_x, workgroup_x order by sum(duration) desc")
    rows = list(rows)
    total = sum(r[7] for r in rows) or 1.0
    out = [f"command: {command}", "", "launches grouped by kernel and launch size (grid lanes / workgroup lanes)", "",
           f"{'kernel':64s} {'grid':>9s} {'wg':>4s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
           f"{'pct':>6s}"]
    for name, gx, wx, n, avg, mn, mx, tot in rows:
        out.append(f"{name[:64]:64s} {gx:>9d} {wx:>4d} {n:>6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} "
                   f"{100.0 * tot / total:6.2f}")
    return "\n".join(out) + "\n"


def stats_summary(csv_path: str, command: str) -> str:
    if csv_path.endswith(".db"):
        return stats_summary_db(csv_path, command)
    rows = list(csv.DictReader(open(csv_path)))
    out = [f"command: {command}", "", f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{r['Name'][:70]:70s} {r['Calls']:>6s} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def _per_kernel(rows, counter):
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return acc


def _calibration_copy(fetch_rows, write_rows, kib):
    """FETCH_SIZE and WRITE_SIZE of the calibration copy: the copy dispatch
    whose WRITE_SIZE is closest to its size (other copies of the run, e.g. of
    whole state arrays, differ in size), and the same dispatch of the FETCH
    run (both runs issue the same sequence of dispatches)."""
    def copies(rows, counter):
        return {r["Dispatch_Id"]: float(r["Counter_Value"]) for r in rows
                if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower()}
    w = copies(write_rows, "WRITE_SIZE")
    f = copies(fetch_rows, "FETCH_SIZE")
    if not w or not f:
        raise RuntimeError("no calibration copy kernel in the counter runs")
    d = min(w, key=lambda k: abs(w[k] - kib))
    if d not in f:
        raise RuntimeError("calibration copy missing from the FETCH_SIZE run")
    return f[d], w[d]


def traffic_summary(fetch_dir, write_dir, substr, copy_bytes, command):
    fetch_rows, write_rows = _counter_rows(fetch_dir), _counter_rows(write_dir)
    fetch = _per_kernel(fetch_rows, "FETCH_SIZE")
    write = _per_kernel(write_rows, "WRITE_SIZE")
    kib = copy_bytes / 1024.0
    copy_f, copy_w = _calibration_copy(fetch_rows, write_rows, kib)
    f_scale = kib / copy_f
    w_scale = kib / copy_w
    out = [f"command: {command}", f"source_sha256: {source_hash()}",
           f"calibration: copy of {copy_bytes:.0f} bytes reads FETCH_SIZE {copy_f:.1f} KiB, "
           f"WRITE_SIZE {copy_w:.1f} KiB -> scale {f_scale:.4f} / {w_scale:.4f}", ""]
    for name in sorted(fetch):
        if substr not in name:
            continue
        fv = fetch[name][1:] if len(fetch[name]) > 1 else fetch[name]
        wv = write.get(name, [0.0])
        wv = wv[1:] if len(wv) > 1 else wv
        fb = sum(fv) / len(fv) * f_scale * 1024.0
        wb = sum(wv) / len(wv) * w_scale * 1024.0
        out.append(f"kernel: {name}")
        out.append(f"  fetch_bytes_per_dispatch: {fb:.0f}")
        out.append(f"  write_bytes_per_dispatch: {wb:.0f}")
        out.append(f"  traffic_bytes_per_dispatch: {fb + wb:.0f}")
    return "\n".join(out) + "\n"


CUS = 256
SIMDS = CUS * 4   # MI355X: 256 CUs x 4 SIMDs
XCDS = 8


def counters_summary(dirs, substr, command):
    per = {}
    for d in dirs:
        for r in _counter_rows(d):
            if substr not in r["Kernel_Name"]:
                continue
            key = (r["Kernel_Name"], r.get("Grid_Size", ""))
            per.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = [f"command: {command}", f"source_sha256: {source_hash()}",
           "normalisation: SQ_* summed over all 1024 SIMDs (SQ_WAVE_CYCLES in quad-cycles), GRBM_GUI_ACTIVE summed "
           "over the 8 XCDs; HBM bytes = 32 x TCC_EA0_RDREQ_DRAM_32B_sum / TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", ""]
    for (name, grid), c in sorted(per.items()):
        m = {k: sum(v) / len(v) for k, v in c.items()}
        out.append(f"kernel: {name}  (grid {grid}, {max(len(v) for v in c.values())} dispatches)")
        gui = m.get("GRBM_GUI_ACTIVE")
        if gui:
            cyc = gui / XCDS
            if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
                out.append(f"  mfma_busy_fraction: {m['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * SIMDS):.4f}")
            if "SQ_WAVE_CYCLES" in m:
                out.append(f"  mean_waves_per_simd: {4 * m['SQ_WAVE_CYCLES'] / (cyc * SIMDS):.3f}")
            if "SQ_INSTS_VALU" in m:
                # a wave64 vector instruction occupies its SIMD for 4 cycles
                out.append(f"  valu_issue_fraction: {4 * m['SQ_INSTS_VALU'] / (cyc * SIMDS):.4f}")
            if "SQ_LDS_BANK_CONFLICT" in m:
                out.append(f"  lds_bank_conflict_fraction_per_cu: {m['SQ_LDS_BANK_CONFLICT'] / (cyc * CUS):.4f}")
            for k in ("TA_TA_BUSY_sum", "TA_BUFFER_TOTAL_CYCLES_sum", "TCP_PENDING_STALL_CYCLES_sum"):
                if k in m:
                    out.append(f"  {k[:-4].lower()}_fraction_per_cu: {m[k] / (cyc * CUS):.4f}")
            out.append(f"  kernel_cycles: {cyc:.0f}")
        if "SQ_WAIT_INST_ANY" in m and "SQ_WAVE_CYCLES" in m:
            out.append(f"  wait_inst_fraction_of_wave_time: {m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.4f}")
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_WAVES", "TCP_TCC_READ_REQ_sum"):
            if k in m:
                out.append(f"  {k.lower()}_per_dispatch: {m[k]:.0f}")
        if "TCC_EA0_RDREQ_DRAM_32B_sum" in m:
            out.append(f"  hbm_read_bytes_per_dispatch: {32 * m['TCC_EA0_RDREQ_DRAM_32B_sum']:.0f}")
        if "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum" in m:
            out.append(f"  hbm_write_bytes_per_dispatch: {32 * m['TCC_EA0_WRREQ_WRITE_DRAM_32B_sum']:.0f}")
        if "TCC_EA0_RDREQ_128B_sum" in m and m.get("TCC_EA0_RDREQ_sum"):
            out.append(f"  read_requests_128B_fraction: {m['TCC_EA0_RDREQ_128B_sum'] / m['TCC_EA0_RDREQ_sum']:.4f}")
    return "\n".join(out) + "\n"


def read_traffic(path: str, kernel_name: str):
    """Traffic per dispatch of ``kernel_name`` from a summary, or None when the
    summary is missing, lacks the kernel, or was taken on other sources."""
    if not os.path.exists(path):
        return None
    lines = open(path).read().splitlines()
    src = next((l.split(":", 1)[1].strip() for l in lines if l.startswith("source_sha256:")), None)
    if src != source_hash():
        return None
    for i, l in enumerate(lines):
        if l.startswith("kernel:") and l.split(":", 1)[1].strip() == kernel_name:
            for l2 in lines[i + 1:i + 4]:
                if "traffic_bytes_per_dispatch" in l2:
                    return float(l2.split(":")[1])
    return None


def main(argv):
    if argv[0] == "stats":
        open(argv[2], "w").write(stats_summary(argv[1], " ".join(argv[3:])))
    elif argv[0] == "traffic":
        open(argv[3], "w").write(traffic_summary(argv[1], argv[2], argv[4], float(argv[5]), " ".join(argv[6:])))
    elif argv[0] == "counters":
        open(argv[2], "w").write(counters_summary(argv[1].split(","), argv[3], " ".join(argv[4:])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
