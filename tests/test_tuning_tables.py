"""The committed tuning tables (CPU only): each is keyed to the parameter set
it was measured on, and that set is unchanged; every pick meets its MRE
target on the measured run, and no feasible row that meets the target was
measured faster than the pick by more than the timing noise the selection
works from (it selects on predicted time, so a small regret is allowed)."""
import glob
import json
import os

import pytest

from paper_2606_10477_amd import params

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_10477_amd")
TABLES = sorted(glob.glob(os.path.join(PKG, "tuning_mi355x*.json")))


def test_tables_present():
    names = {os.path.basename(p) for p in TABLES}
    assert {"tuning_mi355x.json", "tuning_mi355x_bts.json", "tuning_mi355x_bts11.json"} <= names


@pytest.mark.parametrize("path", TABLES, ids=os.path.basename)
def test_table_keyed_to_current_set(path):
    with open(path) as f:
        rep = json.load(f)
    key = rep["key"]
    assert key["params_sha256"] == params.set_sha256(key["params"]), \
        f"{os.path.basename(path)} was tuned on another version of set {key['params']}: re-tune"


@pytest.mark.parametrize("path", TABLES, ids=os.path.basename)
def test_picks_meet_targets(path):
    with open(path) as f:
        rep = json.load(f)
    rows = [r for r in rep["rows"] if r.get("ok")]
    for lvl, by_target in rep["table"].items():
        for tgt, pick in by_target.items():
            if pick is None:
                continue
            assert pick["mre"] <= float(tgt)
            meets = [r for r in rows if r["level"] == int(lvl) and r["m"] <= float(tgt)]
            assert meets
            assert pick["t_meas"] <= 1.5 * min(r["t"] for r in meets) + 1e-3
