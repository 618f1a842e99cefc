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
                limbs += int(r["Grid_Size"]) // (16 * int(r["Workgroup_Size"]))
    return tot, limbs


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


def main(argv=None):
    import sys
    argv = list(sys.argv[1:] if argv is None else argv)
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


if __name__ == "__main__":
    main()
