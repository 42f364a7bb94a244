"""Write tests/golden/synth_sha256.json: sha256 of every generated input array
of the five workloads (database rows, queries, k; the serving schedules; the
sensor stream), with the NumPy version that produced them.  The generators'
streams are NumPy Generator methods, whose output can change between NumPy
versions; tests/test_synth_digests.py regenerates the arrays and compares.

Run from the repository root: python tests/golden/make_synth_digests.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_sha256.json")


def digests() -> dict:
    d = {}
    for name, make in (("c1", synth.c1_tiny), ("c2", synth.c2_oom_boundary), ("c3", synth.c3_hierarchy),
                       ("c5", synth.c5_sensor)):
        w = make()
        d[name] = {"N": w.N, "L": w.L, "V": w.V, "Q": w.Q, "db": synth.sha256_of(w.db),
                   "queries": synth.sha256_of(w.queries), "k": synth.sha256_of(w.k)}
    # c4: the serving schedules (arrival seconds, batch sizes, k) at the three offered loads
    for rate in (1000.0, 10000.0, 100000.0):
        for mode in ("fixed", "uniform"):
            t, b, k = synth.serving_schedule(rate, 4.0, seed=1004, k_mode=mode, k_fixed=10)
            d[f"c4_{int(rate)}_{mode}"] = {"requests": int(len(t)), "schedule": synth.sha256_of(t, b, k)}
    # c5 stream: the 1,050 steps after the 1,000-step history (seed 1005)
    st = synth.SensorStream(seed=1005)
    list(st.steps(1000))
    d["c5_stream_1050"] = {"steps": synth.sha256_of(np.stack(list(st.steps(1050))))}
    return d


if __name__ == "__main__":
    out = {"numpy": np.__version__, "digests": digests()}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(OUT)
