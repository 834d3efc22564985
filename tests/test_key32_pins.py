"""The normalised-key order of the oracle against its independent pins, and
the pins against planted mistakes in copies of the oracle functions (CPU)."""
import inspect

import pytest

import key32_pins
import oracle


def test_key32_oracle_pins():
    key32_pins.run_all_key32()


MUTANTS = {
    # rounding to nearest instead of toward zero (a key can reach the next tile)
    "round_to_nearest": ("key32_normalized",
                         "    f = np.where(f.astype(np.float64) > exact, np.nextafter(f, np.float32(0)), f)  # toward zero\n",
                         ""),
    # the depth not capped below 2^10
    "no_cap": ("key32_normalized", "d = np.minimum(depth, KEY32_DEPTH_CAP).astype(np.float64)",
               "d = depth.astype(np.float64)"),
    # tile scaled by 2^9 instead of 2^10
    "tile_scale": ("key32_normalized", "exact = tile * 1024.0 + d", "exact = tile * 512.0 + d"),
    # ties broken by descending index
    "ties_descending": ("sort_frame_key32", "order = np.lexsort((r.values, k32))",
                        "order = np.lexsort((-r.values.astype(np.int64), k32))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_key32_pins_catch_mutant(name, monkeypatch):
    fn, old, new = MUTANTS[name]
    src = inspect.getsource(getattr(oracle, fn))
    assert old in src, (name, old)
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    monkeypatch.setattr(oracle, fn, ns[fn])
    with pytest.raises(AssertionError):
        key32_pins.run_all_key32()
