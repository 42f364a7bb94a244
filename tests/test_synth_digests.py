"""The seeded generators reproduce the recorded inputs of the five workloads
byte for byte (sha256 of every array; tests/golden/synth_sha256.json, written
by tests/golden/make_synth_digests.py).  NumPy's Generator streams may change
between NumPy versions, so a mismatch under another NumPy version is reported
as such."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_synth_digests  # noqa: E402


def test_generated_inputs_match_recorded_digests():
    rec = json.load(open(os.path.join(HERE, "golden", "synth_sha256.json")))
    got = make_synth_digests.digests()
    if got != rec["digests"]:
        bad = sorted(k for k in rec["digests"] if got.get(k) != rec["digests"][k])
        raise AssertionError(f"generated inputs differ from the recorded digests for {bad} "
                             f"(recorded with NumPy {rec['numpy']}, running {np.__version__})")
