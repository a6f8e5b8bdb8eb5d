"""The pins have teeth: plant one plausible mistake at a time in a copy of the
oracle (CPU only), rebuild the copy, and check that the oracle's own pin tests
(hand-worked cases, brute force, invariants) then fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lob_oracle.c")

# (name, exact text in lob_oracle.c, replacement)
MUTANTS = [
    ("best_bid_is_min", "return is_bid_side ? x->f[P] > y->f[P] : x->f[P] < y->f[P];",
     "return is_bid_side ? x->f[P] < y->f[P] : x->f[P] < y->f[P];"),
    ("later_time_first", "if (x->f[TS] != y->f[TS]) return x->f[TS] < y->f[TS];",
     "if (x->f[TS] != y->f[TS]) return x->f[TS] > y->f[TS];"),
    ("strict_overlap", "int overlap = aggressor_buys ? (P_a >= P_s) : (P_a <= P_s);",
     "int overlap = aggressor_buys ? (P_a > P_s) : (P_a <= P_s);"),
    ("no_max_in_Q_s", "int32_t Q_s_new = Q_s - Q_a > 0 ? Q_s - Q_a : 0;",
     "int32_t Q_s_new = Q_s - Q_a;"),
    ("trade_ids_swapped", "t[2] = o_s->f[OID];\n    t[3] = m[M_OID];",
     "t[2] = m[M_OID];\n    t[3] = o_s->f[OID];"),
    ("trade_time_of_standing", "t[4] = m[M_TS];", "t[4] = o_s->f[TS];"),
    ("trade_price_of_aggressor", "t[0] = P_s;", "t[0] = P_a;"),
    ("market_uses_price_field", "int32_t P_m = buys ? INT32_MAX : 0;",
     "int32_t P_m = m[M_P];"),
    ("cancel_other_side", "order_t *own = bid_side ? b->B : b->A;\n  int32_t k = -1;",
     "order_t *own = bid_side ? b->A : b->B;\n  int32_t k = -1;"),
    ("init_bound_strict", "own[i].f[OID] <= -9000", "own[i].f[OID] < -9000"),
    ("cleanup_keeps_zero", "if (b->A[i].f[Q] <= 0) set_empty(&b->A[i]);",
     "if (b->A[i].f[Q] < 0) set_empty(&b->A[i]);"),
    ("remainder_not_added", "if (rem > 0) add(b, buys, m, rem); /* R8 */", "(void)rem;"),
    ("l2_wrong_sum", "if (!is_empty(&side[i]) && side[i].f[P] == px) qsum += side[i].f[Q];",
     "if (!is_empty(&side[i]) && side[i].f[P] == px) qsum = side[i].f[Q];"),
    ("seed_ids_side_by_side", "for (int32_t l = 0; l < levels; ++l) {\n    for (int sd = 0; sd < 2; ++sd) {",
     "for (int sd = 0; sd < 2; ++sd) {\n    for (int32_t l = 0; l < levels; ++l) {"),
    ("seed_accepts_locked_book", "if (best_px[1] >= best_px[0]) ok = 0;", "if (best_px[1] > best_px[0]) ok = 0;"),
    ("seed_ids_ascending", "own[slot].f[OID] = oid--;", "own[slot].f[OID] = oid++;"),
    ("l2_sum_in_int32", "int64_t qsum = 0; /* R19 */", "int32_t qsum = 0; /* R19 */"),
    ("l2_sum_not_capped", "o[1] = qsum > INT32_MAX ? INT32_MAX : (int32_t)qsum;", "o[1] = (int32_t)qsum;"),
    ("time_ignored_at_equal_price",
     "if (x->f[TS] != y->f[TS]) return x->f[TS] < y->f[TS];\n  if (x->f[TNS] != y->f[TNS]) return x->f[TNS] < y->f[TNS];",
     ""),
    ("seed_time_not_latest", "b->seen_time = 1;\n  b->last_ts = ts;", "b->seen_time = 0;\n  b->last_ts = ts;"),
]

PIN_TESTS = ["tests/test_oracle_golden.py", "tests/test_oracle_bruteforce.py::test_random_sequences",
             "tests/test_oracle_invariants.py", "tests/test_oracle_seed.py"]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique / not found"
    mut = tmp_path / "lob_oracle.c"
    mut.write_text(src.replace(old, new))
    (tmp_path / "lob_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "lob_oracle.h")).read())
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-w",
                           str(mut), "-o", str(so)])
    env = dict(os.environ, LOB_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + PIN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pin tests:\n{r.stdout[-2000:]}"
