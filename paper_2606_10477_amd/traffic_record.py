"""HBM traffic of the NTT kernels from rocprofv3 counter runs, stored for the
benchmark's roofline line.

Inputs: four `rocprofv3 --pmc ... --output-format csv -o run` directories:
FETCH_SIZE and WRITE_SIZE of a benchmark run, and of a plain device copy of
known size (the `copy` command below, 512 MiB).  The copy's counters against
its byte count give one scale per counter; the NTT dispatches' scaled
counters, divided by the limbs they transform, give HBM bytes per limb of one
transform (both passes).  The record carries the SHA-256 of kernels.hip: the
benchmark reports the figure only while the kernels are unchanged.

    python -m paper_2606_10477_amd.traffic_record copy [--mib 512] [--reps 5]
    python -m paper_2606_10477_amd.traffic_record record FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR [--out PATH]

The `counters` command tabulates, per NTT kernel and call size, the duration
from a kernel trace, HBM bytes and rate from the FETCH_SIZE / WRITE_SIZE runs
and the VALU, CU-occupancy and stall figures from SQ counter runs:

    python -m paper_2606_10477_amd.traffic_record counters TRACE_DIR FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR SQ_DIR...
"""
import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
RECORD = os.path.join(HERE, "ntt_traffic.json")
KERNELS = os.path.join(HERE, "csrc", "kernels.hip")
N = 1 << 16


def kernels_sha256():
    with open(KERNELS, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _rows(d):
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        return list(csv.DictReader(f))


def _copy_scale(d, nbytes):
    vals = [float(r["Counter_Value"]) for r in _rows(d) if "copyBuffer" in r["Kernel_Name"]
            and int(r["Grid_Size"]) >= 65536]
    return nbytes / (sum(vals) / len(vals) * 1024.0)


def _is_ntt16(name):
    return "k_ntt16_" in name or "k_nttr_" in name


def _words_per_thread(name):
    """Words each thread holds in an N = 2^16 transform kernel: 16 for the
    k_ntt16_* kernels, the first template argument for k_nttr_<R, S, ...>."""
    if "k_nttr_" in name:
        return int(name.split("k_nttr_", 1)[1].split("<", 1)[1].split(",")[0].split(">")[0])
    return 16


def _limbs(name, grid_size):
    """Limbs a dispatch transforms: each limb takes N / R threads."""
    return int(grid_size) * _words_per_thread(name) // N


def _first_pass(name):
    return "rows_fwd" in name or "blocks_inv" in name


def ntt_bytes(fetch_dir, write_dir, fs, ws):
    tot = {"fetch": 0.0, "write": 0.0}
    limbs = 0
    for d, key, scale in ((fetch_dir, "fetch", fs), (write_dir, "write", ws)):
        for r in _rows(d):
            name = r["Kernel_Name"]
            if not _is_ntt16(name):
                continue
            tot[key] += float(r["Counter_Value"]) * 1024.0 * scale
            if key == "fetch" and _first_pass(name):
                limbs += _limbs(name, r["Grid_Size"])
    return tot, limbs


def ntt_bytes_by_kernel(fetch_dir, write_dir, fs, ws):
    """Markdown table: per NTT kernel, dispatches, limbs and scaled bytes per
    limb fetched and written (in limbs of 8 N bytes)."""
    acc = {}
    for d, key, scale in ((fetch_dir, "fetch", fs), (write_dir, "write", ws)):
        for r in _rows(d):
            name = r["Kernel_Name"]
            if not _is_ntt16(name):
                continue
            a = acc.setdefault(_short(name), {"fetch": 0.0, "write": 0.0, "limbs": 0, "n": 0})
            a[key] += float(r["Counter_Value"]) * 1024.0 * scale
            if key == "fetch":
                a["limbs"] += _limbs(name, r["Grid_Size"])
                a["n"] += 1
    out = ["| kernel | dispatches | limbs | fetch / limb | write / limb |", "|---|---|---|---|---|"]
    for k in sorted(acc):
        a = acc[k]
        out.append(f"| `{k}` | {a['n']} | {a['limbs']} | {a['fetch'] / a['limbs'] / (8 * N):.3f} | "
                   f"{a['write'] / a['limbs'] / (8 * N):.3f} |")
    return "\n".join(out)


def copy_run(mib, reps):
    """The calibration copy: `reps` device-to-device copies of `mib` MiB."""
    import torch
    torch.cuda.set_device(0)
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": reps}), flush=True)


CU_NUM = 256
CLOCK_GHZ = 2.4


def _short(name):
    return name.split("(", 1)[0].replace("void ", "").strip()


def _dispatches(d, every=False):
    """{dispatch id: (kernel, limbs, {counter: value})} of the NTT dispatches
    of one counter run (every=True: of every kernel, limbs 0)."""
    out = {}
    for r in _rows(d):
        name = r["Kernel_Name"]
        if not (every or _is_ntt16(name)):
            continue
        k = int(r["Dispatch_Id"])
        e = out.setdefault(k, (_short(name), _limbs(name, r["Grid_Size"]) if _is_ntt16(name) and not every else 0,
                               {}))
        e[2][r["Counter_Name"]] = e[2].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _trace_durations(d, every=False):
    """{(kernel, limbs): [duration us]} of the NTT dispatches of a kernel trace
    (every=True: of every kernel, limbs 0)."""
    out = {}
    with open(os.path.join(d, "run_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            if not (every or _is_ntt16(name)):
                continue
            g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            key = (_short(name), 0 if every else _limbs(name, g))
            out.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return out


def counter_table(trace_dir, sq_dirs, fetch_dir, write_dir, fs, ws, every=False):
    """Per (kernel, limbs): mean duration from the trace, mean counters over
    the counter runs' dispatches, and the derived figures (per dispatch):
      hbm_GBps   = (FETCH_SIZE fs + WRITE_SIZE ws) KiB / duration,
      cycles     = CLOCK_GHZ * duration (the published peak clock; GRBM_GUI_ACTIVE as
                   collected is summed over counter instances and not used),
      valu_busy  = 100 SQ_ACTIVE_INST_VALU / (CU_NUM cycles): SIMD time in VALU work
                   (quad-cycles per wave, four SIMDs per CU; rocprofv3's VALUBusy formula),
      valu_issue = 100 SQ_INSTS_VALU / (CU_NUM cycles): wave instructions issued against
                   one per CU per cycle (four SIMDs, each taking four cycles for a
                   64-lane instruction on 16 lanes),
      cu_busy    = 100 SQ_BUSY_CU_CYCLES / (CU_NUM cycles) (cycles, summed over CUs),
      wait       = 100 SQ_WAIT_ANY / SQ_WAVE_CYCLES (share of wave time stalled)."""
    dur = _trace_durations(trace_dir, every)
    acc = {}
    for d in list(sq_dirs) + [fetch_dir, write_dir]:
        for name, limbs, cnt in _dispatches(d, every).values():
            a = acc.setdefault((name, limbs), {})
            for c, v in cnt.items():
                a.setdefault(c, []).append(v)
    rows = []
    for key in sorted(acc, key=lambda k: (k[1], k[0])):
        m = {c: sum(v) / len(v) for c, v in acc[key].items()}
        t = dur.get(key)
        r = {"kernel": key[0], "limbs": key[1], "dispatches": len(t) if t else 0,
             "us": sum(t) / len(t) if t else None}
        if "FETCH_SIZE" in m and "WRITE_SIZE" in m:
            b = (m["FETCH_SIZE"] * fs + m["WRITE_SIZE"] * ws) * 1024.0
            r["hbm_bytes"] = b
            if key[1]:
                r["hbm_bytes_per_limb"] = b / key[1]
            if r["us"]:
                r["hbm_GBps"] = b / r["us"] / 1e3
        if r["us"]:
            cyc = CLOCK_GHZ * 1e3 * r["us"]
            if "SQ_ACTIVE_INST_VALU" in m:
                r["valu_busy"] = 100.0 * m["SQ_ACTIVE_INST_VALU"] / (CU_NUM * cyc)
            if "SQ_INSTS_VALU" in m:
                r["valu_issue"] = 100.0 * m["SQ_INSTS_VALU"] / (CU_NUM * cyc)
            if "SQ_BUSY_CU_CYCLES" in m:
                r["cu_busy"] = 100.0 * m["SQ_BUSY_CU_CYCLES"] / (CU_NUM * cyc)
        if m.get("SQ_WAVE_CYCLES"):
            r["wait"] = 100.0 * m.get("SQ_WAIT_ANY", 0.0) / m["SQ_WAVE_CYCLES"]
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_VALU_INT64", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_FMA_F64",
                  "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS"):
            if c in m:
                r[c.replace("SQ_", "").lower() + "_per_limb"] = m[c] / (key[1] or 1)
        rows.append(r)
    return rows


def counters_markdown(rows):
    f = lambda v, p=1: "" if v is None else f"{v:.{p}f}"
    out = ["| kernel | limbs | dispatches | avg us | HBM bytes / limb (limbs) | HBM GB/s | % of 8 TB/s "
           "| VALUBusy % | VALU issue % | CU busy % | wave time waiting % | VALU instr / limb | int64 | int32 "
           "| f64 FMA | LDS instr / limb |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        hb = r.get("hbm_bytes_per_limb")
        gb = r.get("hbm_GBps")
        out.append(f"| `{r['kernel']}` | {r['limbs']} | {r['dispatches']} | {f(r['us'], 2)} | "
                   f"{f(hb / (8 * N) if hb else None, 3)} | {f(gb, 0)} | {f(gb / 80.0 if gb else None, 1)} | "
                   f"{f(r.get('valu_busy'))} | {f(r.get('valu_issue'))} | {f(r.get('cu_busy'))} | "
                   f"{f(r.get('wait'))} | {f(r.get('insts_valu_per_limb'), 0)} | "
                   f"{f(r.get('insts_valu_int64_per_limb'), 0)} | {f(r.get('insts_valu_int32_per_limb'), 0)} | "
                   f"{f(r.get('insts_valu_fma_f64_per_limb'), 0)} | {f(r.get('insts_lds_per_limb'), 0)} |")
    return "\n".join(out)


def main(argv=None):
    import sys
    argv = list(sys.argv[1:] if argv is None else argv)
    if argv and argv[0] == "counters":
        cp = argparse.ArgumentParser()
        cp.add_argument("trace_dir")
        cp.add_argument("fetch_dir")
        cp.add_argument("write_dir")
        cp.add_argument("copy_fetch_dir")
        cp.add_argument("copy_write_dir")
        cp.add_argument("sq_dirs", nargs="+")
        cp.add_argument("--copy-mib", type=int, default=512)
        cp.add_argument("--json", default=None)
        cp.add_argument("--every-kernel", action="store_true",
                        help="every kernel, grouped by name (per-dispatch figures averaged)")
        c = cp.parse_args(argv[1:])
        nb = c.copy_mib << 20
        rows = counter_table(c.trace_dir, c.sq_dirs, c.fetch_dir, c.write_dir,
                             _copy_scale(c.copy_fetch_dir, nb), _copy_scale(c.copy_write_dir, nb), c.every_kernel)
        if c.json:
            with open(c.json, "w") as f:
                json.dump(rows, f, indent=1)
        print(counters_markdown(rows))
        return
    if argv and argv[0] == "copy":
        cp = argparse.ArgumentParser()
        cp.add_argument("--mib", type=int, default=512)
        cp.add_argument("--reps", type=int, default=5)
        c = cp.parse_args(argv[1:])
        copy_run(c.mib, c.reps)
        return
    if argv and argv[0] == "record":
        argv = argv[1:]
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("copy_fetch_dir")
    ap.add_argument("copy_write_dir")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=RECORD)
    ap.add_argument("--by-kernel", action="store_true", help="also print a per-kernel table")
    a = ap.parse_args(argv)
    nbytes = a.copy_mib << 20
    fs = _copy_scale(a.copy_fetch_dir, nbytes)
    ws = _copy_scale(a.copy_write_dir, nbytes)
    tot, limbs = ntt_bytes(a.fetch_dir, a.write_dir, fs, ws)
    per_limb = (tot["fetch"] + tot["write"]) / limbs
    rec = {"kernel": "ntt (N = 2^16, both passes)", "kernels_hip_sha256": kernels_sha256(),
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4), "limbs": limbs,
           "fetch_bytes_per_limb": tot["fetch"] / limbs, "write_bytes_per_limb": tot["write"] / limbs,
           "hbm_bytes_per_limb": per_limb, "algorithmic_bytes_per_limb": 16 * N,
           "ratio_to_algorithmic": per_limb / (16 * N), "command": a.command}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
    if a.by_kernel:
        print(ntt_bytes_by_kernel(a.fetch_dir, a.write_dir, fs, ws))


if __name__ == "__main__":
    main()
