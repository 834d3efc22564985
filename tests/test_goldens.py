"""Regression goldens of the generator and the oracle (CPU only).  The values
were written by tests/golden/make_goldens.py, which calls only synth and
oracle; the pins in test_oracle_pins.py are what make them trustworthy."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_goldens.json")))


def sha(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m", "large-6m"])
def test_frame_golden(name):
    g = GOLD[name]
    spec, seed = synth.FRAME_WORKLOADS[name]
    rec = synth.make_frame(spec, seed)
    assert sha(rec) == g["records_sha256"]
    res = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    assert res.num_pairs == g["num_pairs"] and res.num_tiles == g["num_tiles"]
    assert sha(res.keys) == g["keys_sha256"]
    assert sha(res.values) == g["values_sha256"]
    assert sha(res.ranges) == g["ranges_sha256"]


def test_batch_golden():
    g = GOLD["batch-8-small"]
    b = oracle.sort_batch(synth.make_batch(g["frames"], n_range=g["n_range"]))
    assert [int(x) for x in b.num_pairs] == g["num_pairs"]
    assert sha(b.keys) == g["keys_sha256"] and sha(b.values) == g["values_sha256"]
    assert sha(b.ranges) == g["ranges_sha256"]
