"""CPU checks of the measurement tooling: the bench's one-GPU contract and
constants, the committed traffic summary belonging to the current kernel
sources, and the arithmetic of the rocprofv3 summaries on a small synthetic
result database."""
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_algorithmic_constants():
    import bench
    # 20 rounds x 4 quarter rounds x 12 add/xor/rotate + 16 feed-forward
    # adds + 16 data XORs per 64-byte block
    assert bench.OPS_PER_BLOCK == 992
    assert bench.OPS_PER_PAGE == 992 * 64
    assert bench.HBM_BYTES_PER_PAGE == 8192
    assert abs(bench.MI355X_INT32_VALU_OPS - 256 * 64 * 2.4e9) < 1
    assert abs(bench.PCIE_GEN5_X16_GBPS - 63.0) < 0.1


def test_committed_traffic_summary_matches_kernel_sources():
    """bench.py reports roofline.traffic only while the counters in
    profiles/ were taken on the current kernel sources."""
    import bench
    from paper_2004_09252_amd import profsum
    t = bench.read_traffic(profsum.BULK_KERNEL)
    assert t is not None, ("kernel sources or the bulk kernel changed since "
                           "the counters")
    assert abs(t / (2 * 262144 * 4096) - 1) < 0.01


def _db(path, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (kernel_name text, "
               "counter_name text, value real, duration real)")
    db.executemany("insert into counters_collection values (?, ?, ?, ?)",
                   rows)
    db.commit()
    db.close()


def test_traffic_calibration_arithmetic(tmp_path):
    from paper_2004_09252_amd import profsum
    k = "void ms::(anonymous namespace)::" + profsum.BULK_KERNEL + "(args)"
    c = "ms::(anonymous namespace)::copy_probe_kernel(a, b, c)"
    # the fetch counter reads half of the copy's known 1 GiB, the write
    # counter all of it; the kernel moves 2 GiB (1 in, 1 out) at 1.5x
    _db(tmp_path / "f.db", [(k, "FETCH_SIZE", 1.5 * 524288, 1.0),
                            (c, "FETCH_SIZE", 524288, 1.0)])
    _db(tmp_path / "w.db", [(k, "WRITE_SIZE", 1048576, 1.0),
                            (c, "WRITE_SIZE", 1048576, 1.0)])
    out = tmp_path / "t.txt"
    profsum.traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(out),
                    "cmd f", "cmd w")
    vals = dict(l.split(":", 1) for l in out.read_text().splitlines()
                if ":" in l and not l.startswith("#"))
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    assert float(vals["fetch_bytes_per_launch"]) == pytest.approx(1.5 * 2**30)
    assert float(vals["write_bytes_per_launch"]) == pytest.approx(2**30)
    assert float(vals["traffic_over_algorithmic"]) == pytest.approx(1.25)


def test_resident_summary_arithmetic(tmp_path):
    """profsum's resident summary: bytes per page from FETCH_SIZE and
    WRITE_SIZE calibrated on the copy probe of the same run, instructions
    per page, the waiting share of wave cycles."""
    from paper_2004_09252_amd import profsum
    k = "ms_resident_pages_r20"
    c = "ms::(anonymous namespace)::copy_probe_kernel(a, b, c)"
    pages = 1000
    # FETCH_SIZE reads half of the bytes (the copy's 1 GiB reads 512 MiB)
    _db(tmp_path / "f.db", [(k, "FETCH_SIZE", pages * 4096 / 1024 / 2, 1.0),
                            (c, "FETCH_SIZE", 524288.0, 1.0)])
    _db(tmp_path / "w.db", [(k, "WRITE_SIZE", pages * 4096 / 1024, 1.0),
                            (c, "WRITE_SIZE", 1048576.0, 1.0)])
    _db(tmp_path / "s.db", [(k, "SQ_INSTS_VALU", 976.5 * pages, 1.0),
                            (k, "SQ_WAVES", 1024.0, 1.0),
                            (k, "SQ_BUSY_CYCLES", 10.0, 1.0),
                            (k, "SQ_WAIT_ANY", 1.0, 1.0),
                            (k, "SQ_WAVE_CYCLES", 4.0, 1.0),
                            (k, "GRBM_GUI_ACTIVE", 800.0, 1.0)])
    db = sqlite3.connect(tmp_path / "t.db")
    db.execute("create table kernels (name text, duration real, "
               "vgpr_count int, sgpr_count int, lds_size int, grid_x int, "
               "workgroup_x int)")
    db.execute("insert into kernels values (?, ?, ?, ?, ?, ?, ?)",
               (k, 2.5e6, 64, 96, 18432, 65536, 256))
    db.commit()
    db.close()
    out = tmp_path / "r.txt"
    profsum.resident(str(tmp_path / "t.db"), str(tmp_path / "f.db"),
                     str(tmp_path / "w.db"), str(tmp_path / "s.db"), pages,
                     str(out), "cmd")
    vals = dict(l.split(": ", 1) for l in out.read_text().splitlines()
                if ": " in l and not l.startswith("#"))
    assert float(vals["hbm_fetch_bytes_per_page"]) == pytest.approx(4096)
    assert float(vals["hbm_write_bytes_per_page"]) == pytest.approx(4096)
    assert float(vals["valu_instructions_per_page"]) == pytest.approx(976.5)
    assert float(vals["wave_cycles_waiting_frac"]) == pytest.approx(0.25)
    assert float(vals["dispatch_duration_ms"]) == pytest.approx(2.5)
    assert vals["workgroups_x_threads"] == "256 x 256"
    assert float(vals["grbm_gui_active_cycles_per_xcd"]) == pytest.approx(100)


def test_batch_launch_parts_from_a_trace():
    """profsum's breakdown of fused batch launches: per queue, each
    descriptor copy directly followed by a batch kernel gives the gap
    before the copy, the copy, the gap to the batch kernel and the batch
    kernel; a copy followed by anything else does not count, and each
    queue gets rows of its own."""
    from paper_2004_09252_amd import profsum
    db = sqlite3.connect(":memory:")
    db.execute("create table kernels (name text, queue_id int, start int, "
               "end int)")
    rows = [("plain_pages_kernel", 1, 0, 100_000)]
    t = 100_000
    for i in range(5):   # gaps 10 us, copy 4 us, 0 us, batch 400 us
        rows.append(("ms::desc_copy_kernel(a)", 1, t + 10_000, t + 14_000))
        rows.append(("void ms::batch_pages_kernel<0u, 20, 1>(x)", 1,
                     t + 14_000, t + 414_000))
        t += 414_000
    # a copy with no batch kernel after it, and a pair on another queue
    rows.append(("ms::desc_copy_kernel(a)", 1, t + 1000, t + 2000))
    rows.append(("plain_pages_kernel", 1, t + 3000, t + 4000))
    rows.append(("other", 2, 0, 1))
    rows.append(("ms::desc_copy_kernel(a)", 2, 5, 6))
    rows.append(("void ms::batch_pages_kernel<0u, 20, 1>(x)", 2, 8, 9))
    db.executemany("insert into kernels values (?, ?, ?, ?)", rows)
    lines = profsum._batch_launch_lines(db)
    rows = [l.split(" | ") for l in lines if l.startswith("| 1 ")]
    table = {r[2]: tuple(float(x.strip(" |")) for x in r[3:]) for r in rows}
    assert all(r[1] == "5" for r in rows), rows
    assert table["previous kernel -> copy"] == (10.0, 10.0, 10.0)
    assert table["descriptor copy"] == (4.0, 4.0, 4.0)
    assert table["copy -> batch kernel"] == (0.0, 0.0, 0.0)
    assert table["batch kernel"] == (400.0, 400.0, 400.0)
    # queue 2's pair is reported on its own rows
    q2 = [l for l in lines if l.startswith("| 2 | 1 | ")]
    assert len(q2) == 4, lines
