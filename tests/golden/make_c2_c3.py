"""Writes tests/golden/c2_c3_oracle.json: digests of the oracle's state and
records, step by step, for the L = 64 ferromagnet (R = 10^5, 3 steps; R = 2000,
all 199 steps) and the L = 32 +-J spin glass with two populations
(R = 2 x 2.10^5, 3 steps; R = 2 x 2000, all 300 steps), on the seeds of the
benchmark's workloads.  It calls only the CPU oracle (Sec. II B, steps
(i)-(v)); the GPU tests compare the library's int8 and bit-packed paths with
these values.

    python tests/golden/make_c2_c3.py      # about 12 minutes on 4 cores
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

OUT = os.path.join(HERE, "c2_c3_oracle.json")


def cases():
    import workloads as W
    return {
        "fm_L64_R100000_steps1-3": (W.fm_L64_R100k(), 3),
        "ea_L32_2x200000_steps1-3": (W.ea_L32_two_pop(), 3),
        "fm_L64_R2000_all_steps": (W.fm_L64_R100k(R=2000), None),
        "ea_L32_2x2000_all_steps": (W.ea_L32_two_pop(R=2000), None),
    }


def run_case(name):
    import oracle
    from golden_hash import record_digest, state_digests
    desc, n_steps = cases()[name]
    t0 = time.time()
    orc = oracle.OracleRun(desc)
    last = desc["K"] - 1 if n_steps is None else n_steps
    steps = []

    def snap(i):
        obs = orc.obs()
        pops = []
        for p in range(orc.npop):
            s, E, f, st = orc.state(p)
            r, _, _ = orc.counts(p) if i > 0 else (E[:0], None, None)
            rec = obs[p, i]
            pops.append({"state": state_digests(s, E, f, r), "record": record_digest(rec),
                         "lnQ": float(rec["lnQ"]), "A": float(rec["A"]), "R_i": int(rec["R_i"])})
        steps.append({"i": i, "pops": pops})

    snap(0)
    for i in range(1, last + 1):
        orc.step(i)
        snap(i)
    print(f"{name}: {last} steps in {time.time() - t0:.0f} s", flush=True)
    d = dict(desc)
    return name, {"desc": d, "steps": steps}


def main():
    names = list(cases())
    with mp.Pool(min(4, len(names))) as pool:
        res = dict(pool.map(run_case, names))
    out = {"generator": "tests/golden/make_c2_c3.py (CPU oracle only)", "cases": res}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=None, separators=(",", ":"))
        fh.write("\n")
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
