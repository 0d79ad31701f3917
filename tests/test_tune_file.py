"""The committed plan file of the batched step's product (host logic, no GPU)."""
import math
import os

import synth

PLANS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2104_14101_amd", "tune",
                     "hp_plans.txt")


def _plans():
    out = {}
    for line in open(PLANS):
        if line.startswith("#") or not line.strip():
            continue
        prec, lg, db, kind, rows, ms, tried = line.split()
        out[(prec, int(lg), int(db))] = (kind, int(rows), float(ms))
    return out


def test_plan_lines_are_well_formed():
    for (prec, lg, db), (kind, rows, ms) in _plans().items():
        assert prec in ("fp32", "fp64") and kind in ("fused", "twopass")
        assert rows >= 16 and rows % 16 == 0 and ms > 0
        if kind == "fused":  # the fused form's width limits
            assert db <= (4 if prec == "fp64" else 8)


def test_plans_cover_the_batched_workload():
    plans = _plans()
    for sp in synth.batched_specs(64, seed=0):
        lg = math.ceil(math.log2(sp["n"]))
        db = math.ceil(sp["d"] / 256)
        for prec in ("fp32", "fp64"):
            assert (prec, lg, db) in plans, (prec, sp)
