"""The pins must catch plausible mistakes: each case below plants one mistake
in a copy of the oracle's C source (CPU only), builds it, and runs the pin
tests against it; at least one pin has to fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "jc_union_without_minus_h": ("return H / (double)(da + dc - h);", "return H / (double)(da + dc);"),
    "sc_without_sqrt": ("return H / sqrt(A * C);", "return H / (A * C);"),
    "hp_uses_max": ("return H / (double)(da < dc ? da : dc);", "return H / (double)(da > dc ? da : dc);"),
    "lhn_sum": ("return H / (A * C);", "return H / (A + C);"),
    "aa_log10": ("1.0 / log((double)db)", "1.0 / log10((double)db)"),
    "ra_off_by_one": ("1.0 / (double)db", "1.0 / (double)(db + 1)"),
    "hub_strict": ("return deg_of(off, b) <= L;", "return deg_of(off, b) < L;"),
    "skip_rule": ("if (c == a || (mode == 0 && c < a)) continue;", "if (mode == 0 && c < a) continue;"),
    "no_first_order_clear": ("for (int64_t e = off[a]; e < off[a + 1]; e++) t->adj_a[idx[e]] = 1;", ""),
    "tie_order": ("if (x->a != y->a) return x->a < y->a;", "if (x->a != y->a) return x->a > y->a;"),
    "subset_ignores_list": ("const int64_t a = sources ? sources[i] : i;", "const int64_t a = i;"),
    "threshold_inclusive": ("if (!(s32 > s_th)) continue; /* strictly above the score threshold */",
                            "if (!(s32 >= s_th)) continue;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(text.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(mutated),
                    "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, LP_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-k", "closed_forms or hub_limit or worked or topk_matches or random_graphs"
                              " or wedge_identity or source_subset"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} was not caught:\n{r.stdout[-2000:]}"
