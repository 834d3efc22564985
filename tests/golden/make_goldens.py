"""Write oracle_goldens.json: per workload, the generator's record hash and
the oracle's M, T and output hashes.  Calls only ``synth`` and ``oracle``.
These guard against regressions; the truth is pinned by the tests in
test_oracle_pins.py, which must pass before this script is re-run.

    python tests/golden/make_goldens.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def main():
    out = {}
    for name, (spec, seed) in synth.FRAME_WORKLOADS.items():
        rec = synth.make_frame(spec, seed)
        res = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
        assert res.status == oracle.OK
        out[name] = {"seed": seed, "width": spec.width, "height": spec.height, "n": spec.n,
                     "records_sha256": sha(rec), "num_pairs": res.num_pairs,
                     "num_tiles": res.num_tiles, "keys_sha256": sha(res.keys),
                     "values_sha256": sha(res.values), "ranges_sha256": sha(res.ranges)}
        print(name, res.num_pairs, flush=True)
    frames = synth.make_batch(8, n_range=(5_000, 50_000))
    b = oracle.sort_batch(frames)
    out["batch-8-small"] = {"seed": synth.SEED_BASE + 3, "frames": 8, "n_range": [5_000, 50_000],
                            "num_pairs": [int(x) for x in b.num_pairs],
                            "keys_sha256": sha(b.keys), "values_sha256": sha(b.values),
                            "ranges_sha256": sha(b.ranges)}
    with open(os.path.join(HERE, "oracle_goldens.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
