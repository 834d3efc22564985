"""The preprocess oracle against its independent pins, and the pins against
planted mistakes in a copy of the oracle (CPU only)."""
import pytest

import oracle
import preprocess_pins

MUTANTS = {
    # no 0.3 low-pass dilation
    "no_dilation": ("      a = C[0][0] + 0.3;", "      a = C[0][0];"),
    # Jacobian not clamped
    "no_clamp": ("      const double tx = std::min(lx, std::max(-lx, t[0] / t[2])) * t[2];",
                 "      const double tx = t[0];"),
    # conic off-diagonal sign
    "conic_sign": ("      co[1] = -b / det;", "      co[1] = b / det;"),
    # floor instead of ceil for the radius
    "radius_floor": ("      rec.radius = static_cast<uint32_t>(std::ceil(r3));",
                     "      rec.radius = static_cast<uint32_t>(std::floor(r3));"),
    # no 0.1 floor under the eigenvalue gap
    "no_gap_floor": ("      const double l1 = mid + std::sqrt(std::max(0.1, mid * mid - det));",
                     "      const double l1 = mid + std::sqrt(std::max(0.0, mid * mid - det));"),
    # harmonics without the Condon-Shortley phase
    "no_cs_phase": ("      pmm *= -f * s;", "      pmm *= f * s;"),
    # sin and cos swapped for negative orders
    "sin_cos_swapped": ("      else y = std::sqrt(2.0) * K * std::sin(am * phi) * P;",
                        "      else y = std::sqrt(2.0) * K * std::cos(am * phi) * P;"),
    # every degree used whatever sh_degree says
    "degree_ignored": ("      const int nb = (static_cast<int>(cam->sh_degree) + 1) * (static_cast<int>(cam->sh_degree) + 1);",
                       "      const int nb = 16;"),
    # the near plane test inclusive the other way
    "near_open": ("    bool culled = t[2] <= cam->near_plane;", "    bool culled = t[2] < 0.0;"),
    # rounding by truncation
    "truncate_mean": ("      rec.mean_x = static_cast<int32_t>(std::nearbyint(X));   // current rounding mode: half to even",
                      "      rec.mean_x = static_cast<int32_t>(X);"),
    # projection with the principal point dropped
    "no_centre": ("      x = cam->fx * t[0] / t[2] + cam->cx;", "      x = cam->fx * t[0] / t[2];"),
}


def test_preprocess_oracle_pins():
    preprocess_pins.run_all_preprocess()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_preprocess_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut_src = tmp_path / "oracle_mut.cpp"
    mut_src.write_text(src.replace(old, new))
    lib_path = str(tmp_path / "liboracle_mut.so")
    oracle.build(src=str(mut_src), out=lib_path, extra=("-Wno-unused-function", "-Wno-unused-variable"))
    saved = oracle._LIB
    oracle._LIB = oracle.load(lib_path)
    try:
        with pytest.raises(AssertionError):
            preprocess_pins.run_all_preprocess()
    finally:
        oracle._LIB = saved
