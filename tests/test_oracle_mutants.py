"""Plant plausible mistakes in copies of the C oracle and check that the pins
catch every one of them (CPU only; the real oracle source is not touched)."""
import os
import subprocess

import pytest

import oracle

MUTANTS = {
    "tie_goes_down": ("if (a >= (int64_t)thr[k]) q++;", "if (a > (int64_t)thr[k]) q++;"),
    "relu_dropped": ("if (act == 1 && a < 0) a = 0;", ""),
    "bias_dropped": ("int64_t a = bias;", "int64_t a = 0;"),
    "digit_order_reversed": ("(r >> (j * b)) & digit_mask", "(r >> ((F - 1 - j) * b)) & digit_mask"),
    "weight_index_shifted": ("a += (int64_t)w[j] * x;", "a += (int64_t)w[(j + 1) % F] * x;"),
    "bit_order_reversed": ("|= (uint64_t)1 << (r % 64);", "|= (uint64_t)1 << (63 - r % 64);"),
    "plane_stride_wrong": ("planes[(uint64_t)p * W + r / 64]", "planes[(uint64_t)p + r / 64]"),
    "support_skips_top_value": ("for (uint64_t v = 1; v <= digit_mask; ++v)",
                                "for (uint64_t v = 1; v < digit_mask; ++v)"),
    "layout_ignores_o": ("acc += (uint64_t)o[i] * oracle_words_per_plane(F[i], b[i]);",
                         "acc += oracle_words_per_plane(F[i], b[i]);"),
    "one_threshold_dropped": ("const int K = (1 << o) - 1;", "const int K = (1 << o) - 2;"),
    "weight_sign_flipped": ("a += (int64_t)w[j] * x;", "a -= (int64_t)w[j] * x;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-w", "-o", so, str(msrc)])
    # A mutant may also write out of bounds, so its pins run in a child process.
    script = (
        "import sys, oracle, pins\n"
        f"lib = oracle.load({so!r})\n"
        "caught = []\n"
        "for check in pins.ALL_CHECKS:\n"
        "    try:\n"
        "        check(lib)\n"
        "    except (AssertionError, IndexError, ValueError):\n"
        "        caught.append(check.__name__)\n"
        "print('CAUGHT', caught)\n"
        "sys.exit(0 if caught else 3)\n"
    )
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([os.path.dirname(here), here]))
    r = subprocess.run(["python", "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 3, f"mutant {name} passed every pin"
    # exit 0: a pin failed as it should; any other non-zero status: the mutant
    # corrupted memory while being checked, which the pins also expose.
