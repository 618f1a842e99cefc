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
