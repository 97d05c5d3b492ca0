"""Sanitizer runs of the host code (CPU only).

* The sharp-interface theory solver of the library (threaded host code) is
  built with g++ from its source together with tests/sanitize/theory_driver.cpp,
  once under ThreadSanitizer and once under AddressSanitizer with
  UndefinedBehaviorSanitizer; the driver solves a mixed batch of columns on
  1, 4 and all threads and checks that the results agree bit for bit.
* The C oracle is built under AddressSanitizer and UndefinedBehaviorSanitizer
  and exercised from a child Python process: EOS, critical point,
  coexistence, and a few steps of every lattice with walls and periodic.
Any sanitizer report fails the test (UBSan does not recover; ASan and TSan
exit non-zero on a report).
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
THEORY = os.path.join(ROOT, "paper_2301_12869_amd", "csrc", "theory_host.cpp")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "theory_driver.cpp")
ORACLE_SRC = os.path.join(ROOT, "oracle", "tplbm_oracle.c")


def _tool(name):
    from shutil import which

    return which(name)


pytestmark = pytest.mark.skipif(_tool("g++") is None or _tool("gcc") is None, reason="needs gcc and g++")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout, r.stderr


@pytest.mark.parametrize("flags", [["-fsanitize=thread"],
                                   ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]],
                         ids=["thread", "address+undefined"])
def test_theory_solver_under_sanitizer(flags):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "theory_driver")
        rc, _, err = _run(["g++", "-std=c++17", "-O1", "-g", "-pthread", *flags, "-I", os.path.join(ROOT, "include"),
                           "-o", exe, DRIVER, THEORY])
        assert rc == 0, err
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
        rc, out, err = _run([exe], env=env)
        assert rc == 0, out + err
        assert "Sanitizer" not in err, err
        assert "identical on 1, 4 and all threads" in out


_ORACLE_SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, ROOT)
import oracle as O
import workloads as W
O._LIB = LIB
rho_c, T_c, p_c = O.critical()
P = O.make_params("D2Q9", nx=8, ny=24)
rv, rl, ps = O.coexistence(P, 0.8 * T_c)
O.spinodal(P, 0.8 * T_c)
for lattice, shape, walls, form in (("D2Q9", (24, 8), True, 1), ("D2Q9", (16, 6), False, 2),
                                    ("D1Q3", (40, 1), True, 2), ("D3Q19", (8, 6, 5), True, 1),
                                    ("D3Q19", (6, 5, 4), False, 2)):
    if lattice == "D3Q19":
        kw = dict(nx=shape[2], ny=shape[1], nz=shape[0])
    else:
        kw = dict(nx=shape[1], ny=shape[0])
    P = O.make_params(lattice, walls=walls, gravity_form=form, g=1e-4, **kw)
    rho0 = W.layered_density(shape, shape[0] // 2, rl, rv, 1e-3, seed=5)
    f = O.init_rest(P, rho0.ravel())
    T = np.full(rho0.size, 0.8 * T_c)
    O.step(P, f, T, 3)
    O.macro(P, f, T)
P = O.make_params("D2Q9", nx=7, ny=12, tau=(1.0, 0.8, 1.1, 1.0, 1.2, 0.7))
f = O.init_rest(P, W.layered_density((12, 7), 6, rl, rv, 1e-3, seed=6).ravel())
O.step(P, f, np.full(84, 0.8 * T_c), 3)
print("oracle ok")
"""


def test_oracle_under_address_and_undefined_sanitizers():
    rc, asan, _ = _run(["gcc", "-print-file-name=libasan.so"])
    if rc != 0 or not os.path.isabs(asan.strip()):
        pytest.skip("libasan not found")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liborc_tplbm_san.so")
        rc, _, err = _run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", lib, ORACLE_SRC,
                           "-lm"])
        assert rc == 0, err
        script = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + _ORACLE_SCRIPT
        # Python itself is not instrumented: the ASan runtime is preloaded and
        # its leak check (which would report the interpreter's own
        # allocations) is off
        env = dict(os.environ, LD_PRELOAD=asan.strip(), ASAN_OPTIONS="detect_leaks=0")
        rc, out, err = _run([sys.executable, "-c", script], env=env)
        assert rc == 0, out + err
        assert "oracle ok" in out
        assert "runtime error" not in err and "Sanitizer" not in err, err
