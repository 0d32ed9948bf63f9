"""Summarise rocprofv3 result databases of the page-cipher benchmark.

Usage (from the repository root, on the databases a profiling run left):

    python -m paper_2004_09252_amd.profsum trace  <trace.db>  <out.md>  <cmd>
    python -m paper_2004_09252_amd.profsum trace-titled <title> <trace.db> \
        <out.md> <cmd>
    python -m paper_2004_09252_amd.profsum traffic <fetch.db> <write.db> \
        <out.txt> <cmd-fetch> <cmd-write>
    python -m paper_2004_09252_amd.profsum valu <valu.db> <out.txt> <cmd>
    python -m paper_2004_09252_amd.profsum host <csv-dir> <out.md> <cmd>
    python -m paper_2004_09252_amd.profsum resident <trace.db> <fetch.db> \
        <write.db> <sq.db> <pages> <out.txt> <cmd-prefix>

``trace`` writes the kernel-trace statistics (rocprofv3 --kernel-trace
--stats): per kernel and grid size, the number of dispatches and their
average, minimum and maximum duration; where fused batch launches were
traced, also the parts of one launch (descriptor copy, batch kernel and the
gaps before each).

``resident`` summarises one run of the resident-key kernel on HBM pages
(bench.py --resident-device-only): its dispatch duration, HBM bytes per page
(FETCH_SIZE and WRITE_SIZE calibrated on the copy probe of the same run),
vector instructions per page, and the share of wave cycles spent waiting.
The kernel is one dispatch for the whole engine lifetime, so the counters
include its idle polling between tickets; ``pages`` is the number of pages
the run pushed through it.

``traffic`` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) into HBM bytes
per launch of the bulk plain page kernel.  Both counters are first calibrated
on the copy probe, which reads and writes a known 1 GiB: the factor is
(known bytes) / (counter bytes) for each counter, and the kernel's traffic is
its counter bytes times that factor.  The summary records the SHA-256 of the
kernel's sources (page_cipher.hip, cipher_core.h) so that a reader
(bench.py) can tell when the kernel has changed since the counters were
taken.
"""
from __future__ import annotations

import collections
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("page_cipher.hip", "cipher_core.h")]
COPY_BYTES = 1 << 30
# ChaCha (cipher 0), 20 rounds, unroll 1, linear nonces
BULK_KERNEL = "plain_pages_kernel<0u, 20, 1, 1u>"
COPY_KERNEL = "copy_probe_kernel"
PROBE_KERNEL = "valu_probe_kernel"
N_XCD = 8   # GRBM_GUI_ACTIVE comes summed over the 8 XCDs of an MI355X


def _short(name: str) -> str:
    name = name.replace("ms::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name if len(name) <= 90 else name[:87] + "..."


def trace(db_path: str, out_path: str, cmd: str,
          title: str = "page-cipher benchmark") -> None:
    db = sqlite3.connect(db_path)
    groups = collections.defaultdict(list)
    for name, gx, wx, dur in db.execute(
            "select name, grid_x, workgroup_x, duration from kernels"):
        groups[(name, gx // max(wx, 1))].append(dur)
    lines = ["# rocprofv3 kernel trace: " + title, "",
             "Command (from the repository root, after `cd /tmp && export "
             "TMPDIR=/tmp`):", "", "    " + cmd, "",
             "Durations in microseconds; `blocks` is the grid size in "
             "256-thread workgroups.", "",
             "| kernel | blocks | calls | avg us | min us | max us |",
             "|---|---|---|---|---|---|"]
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (name, blocks), d in rows[:25]:
        lines.append("| %s | %d | %d | %.2f | %.2f | %.2f |" % (
            _short(name), blocks, len(d), sum(d) / len(d) / 1e3,
            min(d) / 1e3, max(d) / 1e3))
    # the top_kernels view reports microseconds (the kernels table, ns)
    lines += ["", "rocprofv3 --stats (all dispatches of a kernel together):",
              "", "| kernel | calls | total ms | avg us | % |",
              "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in db.execute(
            "select name, total_calls, total_duration, average, percentage "
            "from top_kernels limit 12"):
        lines.append("| %s | %d | %.2f | %.2f | %.1f |" % (
            _short(name), calls, total / 1e3, avg, pct))
    lines += _batch_launch_lines(db)
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


DESC_COPY_KERNEL = "desc_copy_kernel"
BATCH_KERNEL = "batch_pages_kernel"


def _batch_launch_lines(db) -> list:
    """Fused batch launches (descriptor copy kernel, then the batch kernel
    on the same queue): the gap from the queue's previous kernel to the
    copy, the copy, the gap from the copy to the batch kernel, and the batch
    kernel, as median / 10th / 90th percentile over the launches traced,
    per hardware queue (graph replays and direct launches may run on
    different queues)."""
    ks = list(db.execute("select name, queue_id, start, end from kernels "
                         "order by start"))
    by_q = collections.defaultdict(list)
    for k in ks:
        by_q[k[1]].append(k)
    names = ("previous kernel -> copy", "descriptor copy",
             "copy -> batch kernel", "batch kernel")
    per_q = {}
    for qid, q in sorted(by_q.items()):
        parts = collections.defaultdict(list)
        for i in range(1, len(q) - 1):
            if DESC_COPY_KERNEL in q[i][0] and BATCH_KERNEL in q[i + 1][0]:
                parts[names[0]].append(q[i][2] - q[i - 1][3])
                parts[names[1]].append(q[i][3] - q[i][2])
                parts[names[2]].append(q[i + 1][2] - q[i][3])
                parts[names[3]].append(q[i + 1][3] - q[i + 1][2])
        if parts:
            per_q[qid] = parts
    if not per_q:
        return []
    out = ["", "Fused batch launches (descriptor copy kernel, then the batch "
           "kernel, on one queue); microseconds:", "",
           "| queue | launches | part | median | p10 | p90 |",
           "|---|---|---|---|---|---|"]
    for qid, parts in per_q.items():
        n = len(parts[names[3]])
        for name in names:
            v = sorted(parts[name])
            out.append("| %s | %d | %s | %.1f | %.1f | %.1f |" % (
                qid, n, name, v[len(v) // 2] / 1e3, v[len(v) // 10] / 1e3,
                v[(9 * len(v)) // 10] / 1e3))
    return out


def _counter(db_path: str, counter: str):
    db = sqlite3.connect(db_path)
    out = collections.defaultdict(list)
    for name, val in db.execute(
            "select kernel_name, value from counters_collection "
            "where counter_name = ?", (counter,)):
        out[name].append(val)
    return out


def _pick(d, needle):
    for name, vals in d.items():
        if needle in name:
            return sum(vals) / len(vals), len(vals)
    raise KeyError(needle)


def traffic(fetch_db: str, write_db: str, out_path: str, cmd_f: str,
            cmd_w: str) -> None:
    f = _counter(fetch_db, "FETCH_SIZE")
    w = _counter(write_db, "WRITE_SIZE")
    kf, nkf = _pick(f, BULK_KERNEL)
    cf, ncf = _pick(f, COPY_KERNEL)
    kw, nkw = _pick(w, BULK_KERNEL)
    cw, ncw = _pick(w, COPY_KERNEL)
    ff = COPY_BYTES / (cf * 1024.0)
    fw = COPY_BYTES / (cw * 1024.0)
    fetch_b = kf * 1024.0 * ff
    write_b = kw * 1024.0 * fw
    algo = 2.0 * 262144 * 4096
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    digest = h.hexdigest()
    lines = [
        "# HBM traffic of the bulk plain page kernel (1 GiB pass, 262144 "
        "pages), from rocprofv3 counters",
        "# fetch command: " + cmd_f,
        "# write command: " + cmd_w,
        "# copy probe: reads and writes %d bytes per dispatch" % COPY_BYTES,
        "kernel: %s" % BULK_KERNEL,
        "fetch_size_kib_kernel: %.3f  (avg of %d dispatches)" % (kf, nkf),
        "fetch_size_kib_copy: %.3f  (avg of %d dispatches)" % (cf, ncf),
        "write_size_kib_kernel: %.3f  (avg of %d dispatches)" % (kw, nkw),
        "write_size_kib_copy: %.3f  (avg of %d dispatches)" % (cw, ncw),
        "fetch_scale: %.6f" % ff,
        "write_scale: %.6f" % fw,
        "fetch_bytes_per_launch: %.0f" % fetch_b,
        "write_bytes_per_launch: %.0f" % write_b,
        "hbm_bytes_per_launch: %.0f" % (fetch_b + write_b),
        "algorithmic_bytes_per_launch: %.0f" % algo,
        "traffic_over_algorithmic: %.5f" % ((fetch_b + write_b) / algo),
        "kernel_source_sha256: %s" % digest,
    ]
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def valu(db_path: str, out_path: str, cmd: str) -> None:
    """VALU counters of the bulk plain kernel: VALUBusy (rocprofv3's derived
    metric: SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE), vector
    instructions issued per page, and the effective shader clock
    (GRBM_GUI_ACTIVE cycles over the dispatch duration)."""
    db = sqlite3.connect(db_path)
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    probe = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, counter, value, dur in db.execute(
            "select kernel_name, counter_name, value, duration from "
            "counters_collection"):
        if BULK_KERNEL in name:
            vals[counter]["v"].append(value)
            vals[counter]["d"].append(dur)
        elif PROBE_KERNEL in name:
            probe[counter]["v"].append(value)
            probe[counter]["d"].append(dur)
    pages = 262144

    def avg(c, v=vals):
        v = v[c]["v"]
        return sum(v) / len(v) if v else float("nan")

    durs = vals["GRBM_GUI_ACTIVE"]["d"]
    dur = sum(durs) / len(durs) if durs else float("nan")
    pdurs = probe["GRBM_GUI_ACTIVE"]["d"]
    pdur = sum(pdurs) / len(pdurs) if pdurs else float("nan")
    lines = ["# VALU counters of the bulk plain page kernel (1 GiB pass, "
             "262144 pages)",
             "# command: " + cmd,
             "kernel: %s" % BULK_KERNEL,
             "dispatches: %d" % len(vals["SQ_INSTS_VALU"]["v"]),
             "VALUBusy_percent: %.2f" % avg("VALUBusy"),
             "SQ_INSTS_VALU_per_launch: %.0f" % avg("SQ_INSTS_VALU"),
             "SQ_INSTS_VALU_per_page: %.1f" % (avg("SQ_INSTS_VALU") / pages),
             "SQ_INSTS_VALU_INT32_per_page: %.1f" % (
                 avg("SQ_INSTS_VALU_INT32") / pages),
             "algorithmic_int_ops_per_page_per_lane: %d" % (992),
             "GRBM_GUI_ACTIVE_cycles_sum_over_%d_xcds: %.0f" % (
                 N_XCD, avg("GRBM_GUI_ACTIVE")),
             "dispatch_duration_us: %.2f" % (dur / 1e3),
             "effective_clock_GHz: %.3f" % (avg("GRBM_GUI_ACTIVE") / N_XCD /
                                            dur),
             "valu_instr_rate_T_lane_ops: %.2f" % (
                 avg("SQ_INSTS_VALU") * 64 / dur / 1e3),
             "valu_peak_at_effective_clock_T: %.2f" % (
                 256 * 64 * avg("GRBM_GUI_ACTIVE") / N_XCD / dur / 1e3),
             "",
             "# the VALU calibration probe (%s) in the same run: %d "
             "dispatches" % (PROBE_KERNEL, len(probe["SQ_INSTS_VALU"]["v"])),
             "probe_SQ_INSTS_VALU_per_dispatch: %.0f" % avg("SQ_INSTS_VALU",
                                                           probe),
             "probe_dispatch_duration_us: %.2f" % (pdur / 1e3),
             "probe_valu_instr_rate_T_lane_ops: %.2f" % (
                 avg("SQ_INSTS_VALU", probe) * 64 / pdur / 1e3),
             "probe_effective_clock_GHz: %.3f" % (
                 avg("GRBM_GUI_ACTIVE", probe) / N_XCD / pdur),
             "probe_VALUBusy_percent: %.2f" % avg("VALUBusy", probe)]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def host(trace_dir: str, out_path: str, cmd: str) -> None:
    """Kernel dispatches and memory copies of a host-resident run, from the
    CSV traces of rocprofv3 --kernel-trace --memory-copy-trace
    --output-format csv: per kernel (and grid) or copy direction, the count
    and the average, minimum and maximum duration."""
    import csv
    import glob
    groups = collections.defaultdict(list)
    for f in glob.glob(os.path.join(trace_dir, "**", "*_kernel_trace.csv"),
                       recursive=True):
        for r in csv.DictReader(open(f)):
            blocks = int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1)
            groups[("kernel", _short(r["Kernel_Name"]), blocks)].append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    for f in glob.glob(os.path.join(trace_dir, "**",
                                    "*_memory_copy_trace.csv"),
                       recursive=True):
        for r in csv.DictReader(open(f)):
            groups[("copy", r["Direction"].replace("MEMORY_COPY_", ""), 0)
                   ].append(int(r["End_Timestamp"]) -
                            int(r["Start_Timestamp"]))
    lines = ["# rocprofv3 kernel and memory-copy trace: host-resident pages",
             "", "Command (from the repository root, after `cd /tmp && "
             "export TMPDIR=/tmp`):", "", "    " + cmd, "",
             "Durations in microseconds; `blocks` is the grid size in "
             "256-thread workgroups (0 for copy-engine transfers).", "",
             "| kind | name | blocks | calls | avg us | min us | max us | "
             "total ms |", "|---|---|---|---|---|---|---|---|"]
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (kind, name, blocks), d in rows[:30]:
        lines.append("| %s | %s | %d | %d | %.2f | %.2f | %.2f | %.2f |" % (
            kind, name, blocks, len(d), sum(d) / len(d) / 1e3,
            min(d) / 1e3, max(d) / 1e3, sum(d) / 1e6))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


RESIDENT_KERNEL = "ms_resident_pages"


def resident(trace_db: str, fetch_db: str, write_db: str, sq_db: str,
             pages: int, out_path: str, cmd: str) -> None:
    db = sqlite3.connect(trace_db)
    rows = [r for r in db.execute(
        "select name, duration, vgpr_count, sgpr_count, lds_size, grid_x, "
        "workgroup_x from kernels") if RESIDENT_KERNEL in r[0]]
    durs = [r[1] for r in rows]
    f = _counter(fetch_db, "FETCH_SIZE")
    w = _counter(write_db, "WRITE_SIZE")
    kf, _ = _pick(f, RESIDENT_KERNEL)
    cf, _ = _pick(f, COPY_KERNEL)
    kw, _ = _pick(w, RESIDENT_KERNEL)
    cw, _ = _pick(w, COPY_KERNEL)
    fetch_b = kf * 1024.0 * COPY_BYTES / (cf * 1024.0)
    write_b = kw * 1024.0 * COPY_BYTES / (cw * 1024.0)
    sq = {c: _pick(_counter(sq_db, c), RESIDENT_KERNEL)[0]
          for c in ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_BUSY_CYCLES",
                    "SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "GRBM_GUI_ACTIVE")}
    lines = [
        "# rocprofv3 summary of the resident-key kernel on HBM pages",
        "# trace command: " + cmd,
        "# counter commands: the same with --kernel-trace --stats replaced "
        "by --pmc FETCH_SIZE, then --pmc WRITE_SIZE, then --pmc "
        "SQ_INSTS_VALU SQ_WAVES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAVE_CYCLES "
        "GRBM_GUI_ACTIVE (one run each)",
        "# one dispatch spans the engine's life, idle polling included",
        "kernel: %s" % RESIDENT_KERNEL,
        "dispatches_traced: %d" % len(durs),
        "dispatch_duration_ms: %.3f" % (
            (sum(durs) / len(durs) / 1e6) if durs else float("nan")),
        "vgprs_sgprs_lds_bytes: %s" % (
            "%d %d %d" % rows[0][2:5] if rows else "n/a"),
        "workgroups_x_threads: %s" % (
            "%d x %d" % (rows[0][5] // max(rows[0][6], 1), rows[0][6])
            if rows else "n/a"),
        "pages_processed: %d" % pages,
        "hbm_fetch_bytes_per_page: %.1f" % (fetch_b / pages),
        "hbm_write_bytes_per_page: %.1f" % (write_b / pages),
        "algorithmic_bytes_per_page: %d" % (2 * 4096),
        "valu_instructions_per_page: %.1f" % (sq["SQ_INSTS_VALU"] / pages),
        "waves: %.0f" % sq["SQ_WAVES"],
        "wave_cycles_waiting_frac: %.4f" % (sq["SQ_WAIT_ANY"] /
                                            sq["SQ_WAVE_CYCLES"]),
        "sq_busy_cycles: %.0f" % sq["SQ_BUSY_CYCLES"],
        "grbm_gui_active_cycles_per_xcd: %.0f" % (sq["GRBM_GUI_ACTIVE"] /
                                                  N_XCD),
    ]
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def main(argv):
    if len(argv) >= 9 and argv[1] == "resident":
        resident(argv[2], argv[3], argv[4], argv[5], int(argv[6]), argv[7],
                 " ".join(argv[8:]))
        return 0
    if len(argv) >= 5 and argv[1] == "host":
        host(argv[2], argv[3], " ".join(argv[4:]))
        return 0
    if len(argv) >= 5 and argv[1] == "valu":
        valu(argv[2], argv[3], " ".join(argv[4:]))
        return 0
    if len(argv) >= 6 and argv[1] == "trace-titled":
        trace(argv[3], argv[4], " ".join(argv[5:]), title=argv[2])
        return 0
    if len(argv) >= 5 and argv[1] == "trace":
        trace(argv[2], argv[3], " ".join(argv[4:]))
    elif len(argv) >= 7 and argv[1] == "traffic":
        traffic(argv[2], argv[3], argv[4], argv[5], argv[6])
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
