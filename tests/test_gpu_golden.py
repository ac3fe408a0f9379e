"""GPU parity at the full sizes of the L = 64 ferromagnet (R = 10^5) and the
L = 32 +-J spin glass with two populations (R = 2 x 2.10^5), against stored
oracle digests (tests/golden/c2_c3_oracle.json, written by
tests/golden/make_c2_c3.py from the CPU oracle only).

Every step compares, per population: the digest of the spins, energies,
family labels and descendant counts (bit-exact), the digest of the record's
integer fields (bit-exact), and ln Q and A (FP64, 1e-10 relative).  The full
sizes run the first three temperature steps; R = 2000 (two populations of
2000) runs the whole schedule, through the ordered phase of the ferromagnet
(beta up to 0.6) and the spin-glass phase (beta up to 3).  The bit-packed
path runs with the launch shapes of the committed tuning cache that the
benchmark applies (for L = 64: the single-size sweep kernel on a persistent
grid).
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from golden_hash import record_digest, state_digests  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_05535_amd as pa  # noqa: E402

GOLDEN = os.path.join(HERE, "golden", "c2_c3_oracle.json")
TUNING = os.path.join(os.path.dirname(HERE), "paper_2207_05535_amd", "tuning_cache.json")
RTOL, ATOL = 1e-10, 1e-12


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


def apply_tuning_cache(ctx, L, path=TUNING):
    """Sets the cache entry's launch shape for L (threads, groups, lockstep
    calls, persistent grid, pooled sparse rounds, chunks of sweeps) and
    checks it took."""
    with open(path) as fh:
        ent = [e for e in json.load(fh)["entries"] if e["repr"] == "msc" and e["L"] == L]
    assert ent, f"no tuning entry for L={L}"
    e = ent[0]
    ctx.set_tuning(L, e["threads"], e["groups"], e["dense"])
    ctx.set_persistent(e["persistent"])
    ctx.set_pooled(e["pooled"])
    ctx.set_sweep_chunks(e.get("chunks", 1))
    got = ctx.tuning(L)
    for k in ("threads", "groups", "dense", "persistent", "pooled"):
        assert got[k] == e[k], (k, got, e)
    return e


def compare_step(ctx, ref, i, where):
    obs = ctx.obs()
    assert obs.shape[1] >= len(ref["pops"])
    for p, rp in enumerate(ref["pops"]):
        s, E, f, r = ctx.state(0, p)
        got = state_digests(s, E, f, r if i > 0 else r[:0])
        rec = obs[0, p, i]
        assert int(rec["R_i"]) == rp["R_i"], f"{where} i={i} pop {p}: R_i {rec['R_i']} != {rp['R_i']}"
        for k, v in rp["state"].items():
            assert got[k] == v, f"{where} i={i} pop {p}: {k} differs"
        assert record_digest(rec) == rp["record"], f"{where} i={i} pop {p}: integer record fields differ"
        for fld in ("lnQ", "A"):
            a, b = float(rec[fld]), rp[fld]
            assert abs(a - b) <= RTOL * max(abs(a), abs(b)) + ATOL, f"{where} i={i} pop {p}: {fld} {a} vs {b}"


CASES = ["fm_L64_R100000_steps1-3", "ea_L32_2x200000_steps1-3", "fm_L64_R2000_all_steps",
         "ea_L32_2x2000_all_steps"]


@pytest.mark.parametrize("repr_", ["int8", "msc"])
@pytest.mark.parametrize("case", CASES)
def test_full_size_and_full_schedule_parity(case, repr_):
    g = golden()[case]
    desc = g["desc"]
    steps = g["steps"]
    say(f"golden parity {case} {repr_}: L={desc['L']} R={desc['R']} steps 0..{steps[-1]['i']}")
    ctx = pa.Context([desc], repr_)
    if repr_ == "msc":
        apply_tuning_cache(ctx, desc["L"])
    compare_step(ctx, steps[0], 0, case)
    for ref in steps[1:]:
        i = ref["i"]
        ctx.step(i)
        compare_step(ctx, ref, i, f"{case} {repr_}")
    say(f"golden parity {case} {repr_}: {len(steps) - 1} steps equal")
    ctx.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", ["fm_L64_R2000_all_steps", "ea_L32_2x2000_all_steps"])
def test_full_schedule_graph_replay(case):
    """The same whole schedules replayed from the captured step graph
    (pa_run) with the benchmark's launch shapes: the records equal the
    oracle's at every temperature and the final state is the oracle's."""
    g = golden()[case]
    desc = g["desc"]
    steps = g["steps"]
    say(f"golden graph replay {case}")
    ctx = pa.Context([desc], "msc")
    apply_tuning_cache(ctx, desc["L"])
    ctx.run(1, desc["K"])
    obs = ctx.obs()
    for ref in steps:
        for p, rp in enumerate(ref["pops"]):
            rec = obs[0, p, ref["i"]]
            assert record_digest(rec) == rp["record"], f"{case} i={ref['i']} pop {p}"
            for fld in ("lnQ", "A"):
                a, b = float(rec[fld]), rp[fld]
                assert abs(a - b) <= RTOL * max(abs(a), abs(b)) + ATOL
    compare_step(ctx, steps[-1], steps[-1]["i"], f"{case} graph")
    ctx.close()
