"""The render oracle against its independent pins, and the pins against
planted mistakes in a copy of the oracle (CPU only)."""
import pytest

import oracle
import render_pins

MUTANTS = {
    # the cross term of the quadratic form without its factor 2
    "cross_term_once": ("const double q = a * dx * dx + 2.0 * b * dx * dy + cc * dy * dy;",
                        "const double q = a * dx * dx + b * dx * dy + cc * dy * dy;"),
    # sampling the pixel's corner instead of its centre (x only)
    "pixel_corner": ("const double dx = G.mean_x / 16.0 - (static_cast<double>(x) + 0.5);",
                     "const double dx = G.mean_x / 16.0 - static_cast<double>(x);"),
    # back to front
    "back_to_front": ("for (uint32_t i = start; i < end; ++i) {", "for (uint32_t i = end; i-- > start;) {"),
    # transmittance updated before the colour uses it
    "T_first": ("        for (int ch = 0; ch < 3; ++ch) c[ch] += rgb[4 * g + ch] * alpha * T;\n"
                "        T *= 1.0 - alpha;",
                "        T *= 1.0 - alpha;\n"
                "        for (int ch = 0; ch < 3; ++ch) c[ch] += rgb[4 * g + ch] * alpha * T;"),
    # no early stop
    "no_stop": ("          if (next < kMinT) break;\n", ""),
    # no alpha cap
    "no_cap": ("          alpha = std::min(kMaxAlpha, alpha);\n", ""),
    # background dropped
    "no_background": ("out_color[ch * W * H + px] = c[ch] + T * background[ch];",
                      "out_color[ch * W * H + px] = c[ch];"),
    # wrong sign in the exponent
    "exp_sign": ("std::exp(-0.5 * q)", "std::exp(0.5 * q)"),
    # faint Gaussians not skipped
    "no_faint_skip": ("          if (alpha < kMinAlpha) continue;\n", ""),
}


def test_render_oracle_pins():
    render_pins.run_all_render()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_render_pins_catch_mutant(name, tmp_path):
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
            render_pins.run_all_render()
    finally:
        oracle._LIB = saved
