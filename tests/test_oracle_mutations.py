"""Planted mistakes in copies of the oracle must fail a named pin (no GPU).

Each case copies ``oracle/frg_oracle.c`` to a temporary directory, changes one
expression (a plausible slip in the channel arrangement or the quadrature),
builds the copy and runs the pins that must catch it in a child process that
loads the copy instead of the oracle.  The unmodified oracle passes the same
pins (the control case).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "frg_oracle.c")
HDR = os.path.join(ROOT, "oracle", "frg_oracle.h")

SU2 = ["tests/test_oracle_symmetries.py::test_su2_spinful_equation_exact_momentum_closure",
       "tests/test_oracle_symmetries.py::test_su2_spinful_equation_general_geometry"]
WEIGHTS = ["tests/test_oracle_symmetries.py::test_weights_integrate_closed_forms"]
SE = ["tests/test_oracle_self_energy.py::test_tadpole_is_the_spin_sum_of_the_antisymmetrised_vertex",
      "tests/test_oracle_self_energy.py::test_hartree_shift_against_the_closed_form_density_of_states",
      "tests/test_oracle_self_energy.py::test_binned_equals_brute_force_with_a_self_energy"]
EGRID = ["tests/test_oracle_egrid.py::test_points_lie_on_their_shells",
         "tests/test_oracle_egrid.py::test_dos_nearest_neighbour_band_is_the_elliptic_integral"]

# (name, original text, planted text, pins that must fail)
CASES = [
    ("crossed ph: V(j1,b,a) for V(j1,a,b)",
     "VI(j1, a, b) * VI(b, j2, j3)", "VI(j1, b, a) * VI(b, j2, j3)", SU2),
    ("direct ph -2 term: a and b exchanged",
     "-2.0 * VI(j1, b, j3) * VI(a, j2, b)", "-2.0 * VI(j1, a, j3) * VI(b, j2, a)", SU2),
    ("fine-grid weight without the radial Jacobian r",
     "*wt = r * (R / (double)m->p.n_rad)", "*wt = (R / (double)m->p.n_rad)", WEIGHTS),
    ("energy-angle density without the radius r of r dr dtheta",
     "return r / dedr;", "return 1.0 / dedr;", EGRID),
    ("energy shells at their lower edges instead of their midpoints",
     "double E = Emin + ((double)i + 0.5) * dE", "double E = Emin + (double)i * dE", EGRID),
    ("every angle of a sector integrated, also where the ray stays below the shell energy",
     "    *c1 = a1;\n    if (e0 >= E && e1 >= E) return;", "    *c1 = a1;\n    return;", EGRID),
    ("self-energy exchange term with the legs of the wrong pair crossed",
     "(2.0 * VI(j, a, j) - VI(a, j, j))", "(2.0 * VI(j, a, j) - VI(j, a, a))", SE),
    ("self-energy direct term without its spin sum",
     "(2.0 * VI(j, a, j) - VI(a, j, j))", "(VI(j, a, j) - VI(a, j, j))", SE),
    ("self-energy left out of the second loop line",
     "xi2 = xi2 + S[b];", "xi2 = xi2;", SE),
]


def _build(tmp_path, old, new):
    src = open(SRC).read()
    n = src.count(old)
    assert n >= 1, f"mutation site not found: {old}"
    d = tmp_path / "mutant"
    d.mkdir()
    (d / "frg_oracle.c").write_text(src.replace(old, new))
    (d / "frg_oracle.h").write_text(open(HDR).read())
    lib = d / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos",
                    "-fPIC", "-shared", "-o", str(lib),
                    str(d / "frg_oracle.c"), "-lm"], check=True)
    return str(lib)


def _run_pins(pins, lib=None):
    env = dict(os.environ)
    env.pop("FRG_ORACLE_LIB", None)
    if lib:
        env["FRG_ORACLE_LIB"] = lib
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


def test_pins_pass_on_the_oracle():
    r = _run_pins(SU2 + WEIGHTS + EGRID + SE)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new,pins", CASES, ids=["crossed-swap", "direct-swap", "no-jacobian", "egrid-no-r", "egrid-edge-energies",
                              "egrid-uncovered-angles", "se-exchange-legs", "se-no-spin-sum",
                              "se-second-line"])
def test_planted_mistake_fails_its_pin(tmp_path, name, old, new, pins):
    lib = _build(tmp_path, old, new)
    r = _run_pins(pins, lib)
    print(name, "->", r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-500:])
    assert r.returncode == 1, f"{name}: pins did not fail\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout
