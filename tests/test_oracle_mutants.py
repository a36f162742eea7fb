"""The pins bite: a plausible mistake planted in a copy of the oracle (a
swapped weight, a wrong sign or index, a dropped term, a wrong constant, a
wrong branch) makes at least one of the pins that cover that part fail.  Each
mutant is one textual change of oracle/nlfem_oracle.c, built to a temporary
library; the named pin tests run in a child pytest against it
(NLFEM_ORACLE_LIB) and must end with failures (exit status 1), not pass and
not error out."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = "tests/test_oracle_pins.py::"

# (what is planted, text in the oracle, replacement, pin tests that must catch it)
MUTANTS = [
    ("outer rule weights swapped",
     "static double rule(int r, int l) { return r == l ? g_alpha : g_beta; }",
     "static double rule(int r, int l) { return r == l ? g_beta : g_alpha; }",
     [PINS + "test_outer_points_integrate_quadratics"]),
    ("sign of phi_(n,u)(p) in a_u",
     "a[u] = yv - M->c[u];",
     "a[u] = yv + M->c[u];",
     [PINS + "test_plain_symmetry_rowsums_spd"]),
    ("kernel factors of T_Omega and T_OmegaI swapped",
     "double fm = region[m] ? 1.0 : 2.0;",
     "double fm = region[m] ? 2.0 : 1.0;",
     [PINS + "test_nonlocal_operator_on_x1_squared", PINS + "test_large_horizon_closed_form"]),
    ("first spacing not subtracted",
     "lam[1] = (double)(u1 - u0) * sc;",
     "lam[1] = (double)(u1) * sc;",
     [PINS + "test_tet_sampling_is_uniform_dirichlet"]),
    ("edge crossing weights swapped",
     "e[a] = 1.0 - g->t[a][b];\n    e[b] = g->t[a][b];",
     "e[a] = g->t[a][b];\n    e[b] = 1.0 - g->t[a][b];",
     [PINS + "test_edge_points_lie_on_sphere", PINS + "test_subdivision_volumes_closed_forms_and_hull"]),
    ("Philox multiplier off by two",
     "uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;",
     "uint64_t p0 = (uint64_t)0xD2511F55u * (uint64_t)c0;",
     [PINS + "test_philox_known_answers"]),
    ("load vector weight of the wrong outer point",
     "S->rhs[free_id[u]] += (wk * rule(k, j)) * fp;",
     "S->rhs[free_id[u]] += (wk * rule(j, j)) * fp;",
     [PINS + "test_rhs_pins"]),
    ("closest-point vertex region taken on either condition",
     "if (d1 <= 0.0 && d2 <= 0.0) {",
     "if (d1 <= 0.0 || d2 <= 0.0) {",
     [PINS + "test_classification_matches_independent_distance", PINS + "test_classification_hand_cases"]),
]


@pytest.mark.parametrize("what,old,new,pins", MUTANTS, ids=[m[0].replace(" ", "_") for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, what, old, new, pins):
    with open(oracle._SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", str(lib), str(mutant), "-lm"], check=True)
    env = dict(os.environ, NLFEM_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    tail = r.stdout[-1500:]
    assert r.returncode == 1 and "failed" in tail, f"mutant survived or errored ({what}): exit {r.returncode}\n{tail}"
