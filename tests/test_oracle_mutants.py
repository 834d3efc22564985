"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch every one of them (CPU only).  Each mutant is a textual edit of
oracle.cpp, built with g++ into a temporary library."""
import os

import pytest

import oracle
import pins

MUTANTS = {
    # an upper tile bound that floors instead of ceiling (drops edge tiles)
    "ceil_to_floor": ("r.x1 = clamp64(ceil_div(X + R, span), 0, tiles_x);",
                      "r.x1 = clamp64(floor_div(X + R, span), 0, tiles_x);"),
    # a closed box on the upper side (touches a tile it only reaches the edge of)
    "closed_upper": ("r.y1 = clamp64(ceil_div(Y + R, span), 0, tiles_y);",
                     "r.y1 = clamp64(ceil_div(Y + R + 1, span), 0, tiles_y);"),
    # truncating division instead of floor for negative numerators
    "trunc_div": ("if (a % b != 0 && a < 0) --q;", ""),
    # radius 0 not culled
    "no_cull": ("if (g.radius == 0) return 0;                    // culled by definition", ""),
    # tile id transposed (column-major)
    "tile_transposed": ("const uint64_t tile = static_cast<uint64_t>(ty) * tiles_x + static_cast<uint64_t>(tx);",
                        "const uint64_t tile = static_cast<uint64_t>(tx) * tiles_y + static_cast<uint64_t>(ty);"),
    # inclusive instead of exclusive scan
    "inclusive_scan": ("std::exclusive_scan(wide.begin(), wide.end(), offsets, uint64_t{0});",
                       "std::inclusive_scan(wide.begin(), wide.end(), offsets);"),
    # an unstable sort
    "unstable_sort": ("std::stable_sort(pairs.begin(), pairs.end(),", "std::sort(pairs.begin(), pairs.end(),"),
    # descending (back-to-front) order
    "descending": ("return a.key < b.key;", "return a.key > b.key;"),
    # empty tiles zero-filled instead of partition form
    "zero_fill": ("start[t] = end[t] = next;", "start[t] = end[t] = 0;"),
    # depth and tile swapped in the key
    "key_swapped": ("keys[pos] = (tile << 32) | depth_bits(G.depth);",
                    "keys[pos] = (static_cast<uint64_t>(depth_bits(G.depth)) << 32) | tile;"),
    # the y span measured with the x extent
    "wrong_axis": ("r.y0 = clamp64(floor_div(Y - R, span), 0, tiles_y);",
                   "r.y0 = clamp64(floor_div(X - R, span), 0, tiles_y);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut_src = tmp_path / "oracle_mut.cpp"
    mut_src.write_text(src.replace(old, new))
    lib_path = str(tmp_path / "liboracle_mut.so")
    oracle.build(src=str(mut_src), out=lib_path, extra=("-Wno-unused-function",))
    saved = oracle._LIB
    oracle._LIB = oracle.load(lib_path)
    try:
        with pytest.raises(AssertionError):
            pins.run_all_small()
    finally:
        oracle._LIB = saved


def test_unmutated_oracle_passes_the_same_suite():
    pins.run_all_small()
