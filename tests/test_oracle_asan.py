"""The oracle's C part (oracle/mf.c) built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only, gcc) and run on small products in
every mode (one and several columns, transposed or not, row ranges, kernel
rows), in a child process with the sanitizer runtime preloaded. CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mf.c")

DRIVER = r"""
import sys
import numpy as np
sys.path.insert(0, ROOT)
import workloads as wl
from oracle import mf, nystrom as orc
dom, gam = wl.config2(n=64, m1=5)
A = 1.0 + 0.3j * np.cos(np.arange(dom.N))
geo = mf.Geometry(dom.eta, dom.etap, A, dom.n)
Aop, Cop = orc.fbie_operators(dom.eta, dom.etap, A, dom.n)
rng = np.random.default_rng(0)
worst = 0.0
for nc in (1, 3, 17):
    x = rng.normal(size=(dom.N, nc))
    for tr in (False, True):
        ya, yc = mf.fbie_ops(geo, x, trans=tr, nthreads=3)
        ra, rc = (Aop.T @ x, Cop.T @ x) if tr else (Aop @ x, Cop @ x)
        worst = max(worst, np.abs(ya - ra).max() / np.abs(ra).max(), np.abs(yc - rc).max() / np.abs(rc).max())
    ya, yc = mf.fbie_rows(geo, x, 7, dom.N - 3, nthreads=2)
K = mf.kernel_rows(geo, 3, 40, nthreads=2)
worst = max(worst, np.abs(K - orc.kernel_matrix(dom.eta, dom.etap, A, dom.n)[3:40]).max())
print("WORST", worst)
assert worst < 1e-12
"""


@pytest.mark.skipif(sys.platform != "linux", reason="gcc sanitizers on Linux")
def test_oracle_c_under_address_and_ub_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libgnk_oracle_asan.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-shared", "-fPIC", "-o", lib, SRC], check=True)
    script = tmp_path / "drive.py"
    script.write_text(f"ROOT = {ROOT!r}\n" + DRIVER)
    env = dict(os.environ)
    env["GNK_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan
    # Python's own allocations are not instrumented; report only errors in the library
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "WORST" in r.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
