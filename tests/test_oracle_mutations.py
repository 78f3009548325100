"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source
(on the CPU), rebuilds it, and checks that at least one pin test fails."""
import inspect
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "kmerco_oracle.c")

MUTATIONS = {
    "canonical picks larger hash": ("return (h < h1) ? 0 : 1;", "return (h > h1) ? 0 : 1;"),
    "j uses X": ("uint64_t j = h % L->Y;", "uint64_t j = h % L->X;"),
    "row stride X": ("*word = i * L->Y + j;", "*word = i * L->X + j;"),
    "saturate one early": ("if (value == maxv)\n            continue;",
                           "if (value + 1u == maxv)\n            continue;"),
    "complement C->C": ("case 'C': return 'G';", "case 'C': return 'C';"),
    "same seed twice": ("uint64_t lo = kco_mm3_32(bytes, 8, 2u * a - 1u);",
                        "uint64_t lo = kco_mm3_32(bytes, 8, 2u * a - 2u);"),
    "query max not min": ("if (a == 1 || value < best)", "if (a == 1 || value > best)"),
    "distinct on freq<=1": ("if (freq == 0) {", "if (freq <= 1) {"),
    "little-endian key bytes reversed": ("bytes[i] = (uint8_t)(key >> (8 * i));",
                                         "bytes[i] = (uint8_t)(key >> (56 - 8 * i));"),
    "Y is 2nd prime": ("for (int i = 0; i < 3; i++)\n        y = next_prime_after(y);",
                       "for (int i = 0; i < 2; i++)\n        y = next_prime_after(y);"),
    "mm3 rotation": ("k = rotl32(k, 15);\n        k *= c2;\n        h ^= k;\n        h = rotl32(h, 13);",
                     "k = rotl32(k, 13);\n        k *= c2;\n        h ^= k;\n        h = rotl32(h, 13);"),
    "classify >=": ("if (kco_query(L, words, distinct[i]) > tau)",
                    "if (kco_query(L, words, distinct[i]) >= tau)"),
    "last window dropped": ("for (uint64_t p = start; p + K <= end; p++) {\n            memcpy(read, reads + p, K);                 /* Read <- K-mer */",
                            "for (uint64_t p = start; p + K < end; p++) {\n            memcpy(read, reads + p, K);                 /* Read <- K-mer */"),
    "l uses alpha": ("*l = (uint32_t)(h % kco_eta(L->alpha));", "*l = (uint32_t)(h % L->alpha);"),
}
# Not listed: flipping the tie rule (h < h1 vs h <= h1).  H_1 ties only when the
# forward and reverse-complement keys are equal (even-K palindromes), where both
# choices give the same k-mer, so that mutant computes the same function.


def _pin_calls():
    """Every pin test as a zero-argument callable (parametrized ones expanded)."""
    calls = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        params = inspect.signature(fn).parameters
        marks = getattr(fn, "pytestmark", [])
        grid = [{}]
        for m in marks:
            if m.name == "parametrize":
                argnames = [a.strip() for a in m.args[0].split(",")]
                grid = [dict(g, **dict(zip(argnames, v if isinstance(v, tuple) else (v,))))
                        for g in grid for v in m.args[1]]
        for g in grid:
            kw = dict(g)
            if "oracle_lib" in params:
                kw["oracle_lib"] = oracle
            calls.append((name, fn, kw))
    return calls


@pytest.mark.parametrize("case", sorted(MUTATIONS))
def test_planted_mistake_is_caught(case, tmp_path):
    old, new = MUTATIONS[case]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {case}"
    mutated = src.replace(old, new, 1)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so),
                           str(c), "-lm"])
    saved_lib, saved_path = oracle._lib, oracle._LIB
    caught = []
    try:
        oracle._lib = None
        oracle._LIB = str(so)
        for name, fn, kw in _pin_calls():
            try:
                fn(**kw)
            except Exception:  # noqa: BLE001 - any failure counts as caught
                caught.append(name)
                break
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
    assert caught, f"no pin caught the planted mistake '{case}'"
