"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library's OGIP reader (``ppm_ogip.cpp``, through a small driver
executable) on valid and malformed ARF/RMF files, and the FP64 oracle
(``oracle/ppm_oracle.c``, as a shared library loaded into a Python child
process with the ASan runtime preloaded) on small cases of every workload
kind.  Any sanitizer report fails the test (recovery disabled)."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from fits_mangle import malformed_rmfs, rmf_with_float_columns
from fits_writer import write_arf, write_rmf

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++ (host compilers)")


def clean(r):
    text = r.stdout + r.stderr
    return r.returncode == 0 and "Sanitizer" not in text and "runtime error" not in text


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "ogip_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "paper_2510_07764_amd", "csrc", "ppm_ogip.cpp"),
                           os.path.join(HERE, "sanitize", "ogip_driver.cpp"), "-o", exe])
    return exe


def run_driver(exe, mode, path):
    r = subprocess.run([exe, mode, path], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert clean(r), (path, r.stdout[-2000:], r.stderr[-4000:])
    line = [s for s in r.stdout.splitlines() if s.startswith("status")][-1].split()
    return int(line[1]), float(line[7])


def test_ogip_reader_valid_and_malformed_files(driver, tmp_path):
    rng = np.random.default_rng(5)
    lo = np.geomspace(0.1, 4.0, 41)[:-1]
    hi = np.geomspace(0.1, 4.0, 41)[1:]
    area = rng.uniform(100, 300, 40)
    m = np.where(rng.uniform(size=(40, 25)) < 0.3, rng.uniform(size=(40, 25)), 0.0)
    cl, ch = np.linspace(0.1, 4.0, 26)[:-1], np.linspace(0.1, 4.0, 26)[1:]
    pa = str(tmp_path / "v.arf")
    write_arf(pa, lo, hi, area)
    st, s = run_driver(driver, "arf", pa)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    assert st == 0 and s == pytest.approx(f32(area).sum() + f32(lo).sum(), rel=1e-12)
    for variable in (True, False):
        pr = str(tmp_path / f"v{int(variable)}.rmf")
        write_rmf(pr, lo, hi, m, cl, ch, variable=variable)
        st, s = run_driver(driver, "rmf", pr)
        assert st == 0 and s == pytest.approx(f32(m).sum() + f32(lo).sum(), rel=1e-12)
    valid = open(str(tmp_path / "v1.rmf"), "rb").read()
    for name, raw in malformed_rmfs(valid):
        q = str(tmp_path / (name + ".rmf"))
        with open(q, "wb") as f:
            f.write(raw)
        st, _ = run_driver(driver, "rmf", q)
        assert st != 0, name
    for vals in [(float("nan"), 1.0, 1.0), (1e30, 1.0, 1.0), (1.0, -1e30, 1.0), (1.0, 1.0, float("nan"))]:
        q = str(tmp_path / "f.rmf")
        rmf_with_float_columns(q, *vals)
        st, _ = run_driver(driver, "rmf", q)
        assert st != 0, vals


ORACLE_CASES = r'''
import os, sys, math
sys.path.insert(0, os.environ["PPM_ROOT"])
import numpy as np
import oracle, synthetic as syn
spec, p = syn.config1(n_cells=6, n_phase=8, n_energy=16)
ft, cnt, d = oracle.forward(spec, p)
data = syn.poisson_data(cnt)
ll = oracle.loglike_from_counts(cnt, data)
spec2, p2 = syn.config2(n_cells=6, n_phase=8, n_fp=64)
spec2["energy"] = syn.logspace(0.2, 3.0, 16)
syn.attach_instrument(spec2)
oracle.forward(spec2, p2)
s0, q0 = syn.config0()
oracle.forward(dict(s0, n_phase=8), q0)
for test in (1, 2):
    s3, q3 = syn.interp_test_geometry(test)
    for interp in (0, 1, 2, 3):
        oracle.forward(dict(s3, interp=interp, n_phase=4), q3)
sm, pm, mm = syn.map_config(2, "random", n_phase=8, n_energy=16)
oracle.forward_map(sm, pm, 2, mm)
assert np.all(np.isfinite(cnt)) and math.isfinite(ll)
print("oracle cases done", flush=True)
'''


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "libppm_oracle_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-fPIC", "-shared", "-fopenmp", *SAN, "-Wno-unknown-pragmas",
                           os.path.join(ROOT, "oracle", "ppm_oracle.c"), "-o", lib, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, PPM_ORACLE_LIB=lib, PPM_ROOT=ROOT, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", ORACLE_CASES], capture_output=True, text=True, timeout=600, env=env,
                       cwd=ROOT)
    assert clean(r) and "oracle cases done" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
