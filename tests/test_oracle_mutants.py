"""Plants plausible mistakes in a copy of the oracle's C source, on the CPU,
and checks that the pins catch every one of them (the pins must not be
satisfiable by a subtly wrong oracle)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hs_oracle.c")
SW = os.path.join(ROOT, "oracle", "sw_check.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("gep_dropped", "(int64_t)(g - 1) * p->gep", "0"),
    ("pgp_sign", "if (periphery) pen += (int64_t)p->pgp * g;", "if (periphery) pen -= (int64_t)p->pgp * g;"),
    ("periphery_edge", "(c <= first)", "(c < first)"),
    ("shift_tie_last", "if (score > best) { best = score; bk = k; }",
     "if (score >= best) { best = score; bk = k; }"),
    ("wrong_index", "s += cx->B[large[i] * ORC_NSYM + small[j]];",
     "s += cx->B[large[j] * ORC_NSYM + small[j]];"),
    ("transposed_operands", "s += cx->B[large[i] * ORC_NSYM + small[j]];",
     "s += cx->B[small[j] * ORC_NSYM + large[i] + 1 - 1 + 0 * ORC_NSYM] + (large[i] != small[j] ? (large[i] < small[j]) : 0);"),
    ("role_tie", "int target_is_large = tlen >= qlen;", "int target_is_large = tlen > qlen;"),
    ("consume_no_shift",
     "int32_t takeL = kstar + (int32_t)ss < (int32_t)ls ? kstar + (int32_t)ss : (int32_t)ls;",
     "int32_t takeL = (int32_t)ss < (int32_t)ls ? (int32_t)ss : (int32_t)ls;"),
    ("ls_scale", "int64_t ls = (int64_t)(((uint64_t)nl * LF) >> 16);",
     "int64_t ls = (int64_t)(((uint64_t)nl * LF) >> 17);"),
    ("draw_chunk", "return (uint32_t)((word >> (16 * (d & 3))) & 0xFFFFu);",
     "return (uint32_t)((word >> (16 * ((d + 1) & 3))) & 0xFFFFu);"),
    ("philox_key_bump", "k1 += PHILOX_W1;", "k1 += PHILOX_W0;"),
    ("minfactor_inverted", "if (lf < (uint32_t)p->minfactor_q16) lf = (uint32_t)p->minfactor_q16;",
     "if (lf > (uint32_t)p->minfactor_q16) lf = (uint32_t)p->minfactor_q16;"),
    ("round_tie_last", "if (s > best) {\n            best = s; best_round = r;",
     "if (s >= best) {\n            best = s; best_round = r;"),
    ("step_draw_index", "orc_draw(p->seed, cx->target_id, round, 2u + (uint32_t)t);",
     "orc_draw(p->seed, cx->target_id, round, 1u + (uint32_t)t);"),
    ("ss_no_clamp", "if (!p->full_slide && ss > ls) ss = ls;",
     "if (!p->full_slide && ss > ls + 1) ss = ls;"),
    ("full_slide_clamped", "if (!p->full_slide && ss > ls) ss = ls;", "if (ss > ls) ss = ls;"),
    ("full_start", "int32_t start = cx->p->full_slide ? 0 : ns - 1;",
     "int32_t start = cx->p->full_slide ? 1 : ns - 1;"),
    ("full_end", "int32_t end = cx->p->full_slide ? ns + nl - 2 : nl - 1;",
     "int32_t end = cx->p->full_slide ? ns + nl - 3 : nl - 1;"),
    ("overhang_takes_window",
     "int32_t takeL = kstar + (int32_t)ss < (int32_t)ls ? kstar + (int32_t)ss : (int32_t)ls;",
     "int32_t takeL = kstar + (int32_t)ss < (int32_t)ls ? kstar + (int32_t)ss : (int32_t)ls - (kstar < 0);"),
    ("hang_front_kept", "aL[len] = (i >= 0 && i < (int32_t)ls) ? large[i] : ORC_GAP;",
     "aL[len] = (i > 0 && i < (int32_t)ls) ? large[i] : ORC_GAP;"),
    ("tail_dropped", "for (int32_t i = 0; i < ns; ++i) { aL[len] = ORC_GAP; aS[len] = small[i]; ++len; }",
     ""),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(lib), str(mut), SW],
                   check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_rng.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch planted mistake {name}"
