"""Write tests/golden/fullsize_chain_p16b.json: the oracle's digests of every
step of the benchmarked workload at N = 2^16 (see fullsize_chain.py).  Calls
only the oracle (and the seeded input generator).  Takes a few minutes on one
core.

    python tests/golden/make_fullsize_golden.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

OUT = os.path.join(HERE, "fullsize_chain_p16b.json")
SOURCES = ("oracle/ckks_oracle.c", "paper_2606_10477_amd/params.json", "tests/golden/fullsize_chain.py")


def source_digest():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def main():
    from oracle import oracle as O
    from paper_2606_10477_amd import inputs
    import fullsize_chain as F
    t0 = time.time()
    o = O.Context.from_set("p16b")
    o.keygen(F.KEY_SEED, o.bts_galois())
    x = inputs.log_uniform(o.n, F.LO, F.HI, F.INPUT_SEED)
    print(f"set-up {time.time() - t0:.0f} s", flush=True)
    steps = F.run(o, x, on_step=lambda n, d: print(f"{n}: level {d['level']} ({time.time() - t0:.0f} s)", flush=True))
    rec = {"about": "oracle digests of the benchmarked workload's steps at N = 2^16 (fullsize_chain.py); "
                    "written by make_fullsize_golden.py",
           "sources_sha256": source_digest(), "steps": steps}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
