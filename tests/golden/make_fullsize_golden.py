"""Write tests/golden/fullsize_chain_<set>.json: the oracle's digests of
every step of the benchmarked workload at N = 2^16 on a bootstrapping set
(see fullsize_chain.py).  Calls only the oracle (and the seeded input
generator).  Takes several minutes on one core.

    python tests/golden/make_fullsize_golden.py [p16b|p16c]
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

SETS = ("p16b", "p16c")
SOURCES = ("oracle/ckks_oracle.c", "tests/golden/fullsize_chain.py")


def out_path(name):
    return os.path.join(HERE, f"fullsize_chain_{name}.json")


def source_digest(name):
    """SHA-256 over the oracle's source, the recipe and the set's own entry
    of the parameter file (canonical JSON: other sets do not enter)."""
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "paper_2606_10477_amd", "params.json")) as f:
        h.update(json.dumps(json.load(f)[name], sort_keys=True, separators=(",", ":")).encode())
    return h.hexdigest()


def main(name="p16b"):
    from oracle import oracle as O
    from paper_2606_10477_amd import inputs
    import fullsize_chain as F
    if name not in SETS:
        raise SystemExit(f"unknown set {name!r}; one of {SETS}")
    t0 = time.time()
    o = O.Context.from_set(name)
    o.keygen(F.KEY_SEED, o.bts_galois())
    x = inputs.log_uniform(o.n, F.LO, F.HI, F.INPUT_SEED)
    print(f"set-up {time.time() - t0:.0f} s", flush=True)
    xp = inputs.linspace_input(o.n, F.PAPER_LO, F.PAPER_HI)
    steps = F.run(o, x, x_paper=xp,
                  on_step=lambda n, d: print(f"{n}: level {d['level']} ({time.time() - t0:.0f} s)", flush=True))
    rec = {"about": f"oracle digests of the benchmarked workload's steps at N = 2^16 on set {name} "
                    "(fullsize_chain.py); written by make_fullsize_golden.py",
           "sources_sha256": source_digest(name), "steps": steps}
    out = out_path(name)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main(*sys.argv[1:2])
