"""The polarization pins catch the plausible mistakes they are meant to catch.

Each case copies the oracle's sources to a temporary directory, plants one
mistake in the copy (on the CPU, never in the product), builds it, and runs
the polarization pins against it in a subprocess; they must fail.  A control
copy without a mistake must pass.  The mistakes:

- swap_sp: r_s <-> r_p and t_s <-> t_p at mirror events, consistently in the
  forward and the adjoint (Eq. 5 s/p assignment);
- conj_tir: the other evanescent branch at a totally reflecting face, which
  conjugates the reflection phase (Eq. 3 under total internal reflection);
- swap_face: r_s <-> r_p at face reflections;
- swap_exit: t_s <-> t_p at the exit face;
- pout_sign: the outgoing p axis s x k instead of k x s at mirrors.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "swap_sp": [
        ("double complex cs = reflect ? co[0] : co[2];\n    double complex cp = reflect ? co[1] : co[3];",
         "double complex cs = reflect ? co[1] : co[3];\n    double complex cp = reflect ? co[0] : co[2];"),
        ("int cs_i = t->reflect ? 0 : 2, cp_i = t->reflect ? 1 : 3;",
         "int cs_i = t->reflect ? 1 : 3, cp_i = t->reflect ? 0 : 2;"),
    ],
    "conj_tir": [("CMPLX(0.0, sqrt(st2 - na2))", "CMPLX(0.0, -sqrt(st2 - na2))")],
    "swap_face": [("r->E = apply_sp(r->E, sv, pin, pout, rs, rp, 1.0);",
                   "r->E = apply_sp(r->E, sv, pin, pout, rp, rs, 1.0);")],
    "swap_exit": [("r->E = apply_sp(r->E, sv, pin, pout, ts, tp, flux);",
                   "r->E = apply_sp(r->E, sv, pin, pout, tp, ts, flux);")],
    "pout_sign": [("vec3 pout = cross3(dnew, s);", "vec3 pout = cross3(s, dnew);")],
}


def _copy_tree(dst):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "inputs"), os.path.join(dst, "inputs"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in ("conftest.py", "numpy_ref.py", "test_oracle_polarization.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))


def _run_pins(dst):
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    subprocess.run([sys.executable, "-c", "import oracle.build as b; b.build()"], cwd=dst, env=env,
                   check=True, capture_output=True)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "tests/test_oracle_polarization.py"], cwd=dst, env=env,
                          capture_output=True, text=True, timeout=600)


def test_control_copy_passes(tmp_path):
    _copy_tree(str(tmp_path))
    r = _run_pins(str(tmp_path))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    _copy_tree(str(tmp_path))
    path = os.path.join(str(tmp_path), "oracle", "trace.c")
    src = open(path).read()
    for a, b in MUTATIONS[name]:
        assert src.count(a) == 1, (name, a)
        src = src.replace(a, b)
    open(path, "w").write(src)
    r = _run_pins(str(tmp_path))
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-2000:])
