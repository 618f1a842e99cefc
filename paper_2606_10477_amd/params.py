"""Named CKKS parameter sets (data in params.json next to this file).

Each set gives the ring degree, the computation levels, the special primes,
the digit size of hybrid key switching, the secret's Hamming weight and, for
a bootstrapping set, the bootstrapping levels (SlotToCoeff, EvalMod,
CoeffToSlot, their scale bits) and the EvalMod approximation.  The primes
themselves are generated from these numbers by the library (and, from the
same published rule, independently by the oracle).
"""
import json
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "params.json")


def load(name):
    """The set `name` ("p12", "p16", "p16b") as a dict."""
    with open(PATH) as f:
        sets = json.load(f)
    if name not in sets:
        raise KeyError(f"unknown parameter set {name!r}; known: {sorted(sets)}")
    return sets[name]


def set_sha256(name):
    """SHA-256 of the set's canonical JSON: the key a tuning table is valid for."""
    import hashlib
    return hashlib.sha256(json.dumps(load(name), sort_keys=True, separators=(",", ":")).encode()).hexdigest()


def context_kwargs(name):
    """Keyword arguments of ckks.Context for the set `name`."""
    s = load(name)
    kw = {k: s[k] for k in ("log_n", "max_level", "num_special", "digit_size", "hamming_weight")}
    if "bts" in s:
        kw["bts"] = tuple(s["bts"])
    return kw


def evalmod(name):
    """(K, r, degree) of the set's EvalMod, or None without bootstrapping."""
    s = load(name)
    e = s.get("evalmod")
    return None if e is None else (float(e["K"]), int(e["r"]), int(e["degree"]))
