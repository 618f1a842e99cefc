"""Host logic of the NTT traffic record: counter CSVs of rocprofv3 (synthetic
here) scaled by a plain copy's counters, per limb of a transform."""
import csv
import json
import os

from paper_2606_10477_amd import traffic_record

FIELDS = ["Dispatch_Id", "Grid_Size", "Workgroup_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, r in enumerate(rows):
            w.writerow(dict(zip(FIELDS, [k + 1] + list(r))))


def test_record_from_counters(tmp_path):
    mib = 1 << 20
    # copy of 512 MiB: FETCH reads half its bytes (scale 2), WRITE all of them (scale 1)
    _write(tmp_path / "cf", [(131072, 256, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512 * 1024 / 2)])
    _write(tmp_path / "cw", [(131072, 256, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 512 * 1024)])
    # a 3-limb transform with 16 words per thread (4096 threads a limb) and a
    # 2-limb one with 4 words per thread (16384 threads a limb): each pass reads
    # and writes every limb (512 KiB), the blocks passes read 0.5 MiB of twiddles
    kib = 512
    f_rows = [(3 * 4096, 256, "gpu::k_ntt16_rows_fwd<false>(...)", "FETCH_SIZE", 3 * kib / 2),
              (3 * 4096, 256, "gpu::k_ntt16_blocks_fwd<false>(...)", "FETCH_SIZE", 3 * 2 * kib / 2),
              (2 * 16384, 1024, "void gpu::k_nttr_blocks_inv<4>(...)", "FETCH_SIZE", 2 * 2 * kib / 2),
              (2 * 16384, 1024, "void gpu::k_nttr_rows_inv<4>(...)", "FETCH_SIZE", 2 * kib / 2),
              (65536, 256, "gpu::k_add(...)", "FETCH_SIZE", 99999.0)]
    w_rows = [(g, wg, n, "WRITE_SIZE", (g // (16 * wg)) * kib) for g, wg, n, _, _ in f_rows[:4]]
    _write(tmp_path / "f", f_rows)
    _write(tmp_path / "w", w_rows)
    out = tmp_path / "rec.json"
    traffic_record.main([str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                         "--out", str(out)])
    rec = json.loads(out.read_text())
    assert rec["limbs"] == 5
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    # per limb: fetch 0.5 + 1.0 MiB, write 2 x 0.5 MiB -> 2.5 MiB = 2.5 x 16 N bytes
    assert abs(rec["fetch_bytes_per_limb"] - 1.5 * mib) < 1e-6
    assert abs(rec["write_bytes_per_limb"] - 1.0 * mib) < 1e-6
    assert abs(rec["ratio_to_algorithmic"] - 2.5) < 1e-12
    assert rec["kernels_hip_sha256"] == traffic_record.kernels_sha256()


def _write_trace(d, rows):
    """rows: (kernel name, grid x, grid y, start ns, end ns)"""
    os.makedirs(d, exist_ok=True)
    fields = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"]
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for n, gx, gy, t0, t1 in rows:
            w.writerow(dict(zip(fields, [n, gx, gy, 1, t0, t1])))


def test_counter_table_derived_figures(tmp_path):
    """Duration from the trace, HBM rate from the scaled byte counters, VALU
    busy / issue and CU busy against 256 CUs at 2.4 GHz, stall share from the
    wave-cycle counters, all per (kernel, limbs)."""
    name = "void gpu::k_nttr_rows_fwd<4, 4, false>(...)"
    g = 8 * 16384                       # 8 limbs at 4 words per thread
    _write_trace(tmp_path / "t", [(name, g, 1, 0, 10_000), (name, g, 1, 20_000, 30_000)])   # 10 us each
    _write(tmp_path / "cf", [(131072, 256, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512 * 1024 / 2)])
    _write(tmp_path / "cw", [(131072, 256, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 512 * 1024)])
    kib = 512
    _write(tmp_path / "f", [(g, 256, name, "FETCH_SIZE", 8 * kib / 2)] * 2)
    _write(tmp_path / "w", [(g, 256, name, "WRITE_SIZE", 8 * kib)] * 2)
    cyc = 2.4e3 * 10.0                  # cycles of a 10 us dispatch
    sq = [(g, 256, name, "SQ_INSTS_VALU", 0.25 * 256 * cyc), (g, 256, name, "SQ_ACTIVE_INST_VALU", 0.5 * 256 * cyc),
          (g, 256, name, "SQ_BUSY_CU_CYCLES", 0.75 * 256 * cyc), (g, 256, name, "SQ_WAVE_CYCLES", 1000.0),
          (g, 256, name, "SQ_WAIT_ANY", 400.0)]
    rows_sq = []
    for k in range(2):                  # two dispatches, ids 1..5 and 6..10
        rows_sq += sq
    os.makedirs(tmp_path / "s", exist_ok=True)
    with open(tmp_path / "s" / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, r in enumerate(rows_sq):
            w.writerow(dict(zip(FIELDS, [k // 5 + 1] + list(r))))
    fs = traffic_record._copy_scale(str(tmp_path / "cf"), 512 << 20)
    ws = traffic_record._copy_scale(str(tmp_path / "cw"), 512 << 20)
    rows = traffic_record.counter_table(str(tmp_path / "t"), [str(tmp_path / "s")], str(tmp_path / "f"),
                                        str(tmp_path / "w"), fs, ws)
    assert len(rows) == 1
    r = rows[0]
    assert r["kernel"] == "gpu::k_nttr_rows_fwd<4, 4, false>" and r["limbs"] == 8 and r["dispatches"] == 2
    assert abs(r["us"] - 10.0) < 1e-9
    assert abs(r["hbm_bytes_per_limb"] - 2 * kib * 1024) < 1e-6        # one read and one write of the limb
    assert abs(r["hbm_GBps"] - 8 * 2 * kib * 1024 / 10e-6 / 1e9) < 1e-6
    assert abs(r["valu_issue"] - 25.0) < 1e-9 and abs(r["valu_busy"] - 50.0) < 1e-9
    assert abs(r["cu_busy"] - 75.0) < 1e-9 and abs(r["wait"] - 40.0) < 1e-9
    every = traffic_record.counter_table(str(tmp_path / "t"), [str(tmp_path / "s")], str(tmp_path / "f"),
                                         str(tmp_path / "w"), fs, ws, every=True)
    assert every[0]["limbs"] == 0 and abs(every[0]["hbm_bytes"] - 8 * 2 * kib * 1024) < 1e-6
