"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The symbolic analysis (analyze.cpp, capi_symbolic.cpp) is built with g++
-fsanitize=address,undefined together with a small driver
(sanitize/analyze_driver.cpp) and run on several patterns and option sets;
its results must equal the regular library's bit for bit, and malformed
patterns must be rejected cleanly.  The CPU oracle (oracle.c) is built the
same way and the oracle pin tests run against it in a subprocess with the
sanitizer runtimes preloaded.  Only host code is built here; no GPU code.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2007_01541_amd import Symbolic
from workloads import small_fp64, tiny

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_01541_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1"]


def runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


pytestmark = pytest.mark.skipif(runtime("libasan.so") is None or runtime("libubsan.so") is None,
                                reason="gcc sanitizer runtimes not installed")


@pytest.fixture(scope="module")
def analyze_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "analyze_driver")
    cmd = ["g++", "-std=c++17", "-pthread"] + SAN + ["-o", exe, os.path.join(ROOT, "tests", "sanitize", "analyze_driver.cpp"),
                                                      os.path.join(CSRC, "analyze.cpp"), os.path.join(CSRC, "capi_symbolic.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


def write_pattern(path, m):
    with open(path, "wb") as f:
        np.array([m["n"]], np.int32).tofile(f)
        np.array([m["colptr"][-1]], np.int64).tofile(f)
        np.asarray(m["colptr"], np.int64).tofile(f)
        np.asarray(m["rowind"], np.int32).tofile(f)
        np.ascontiguousarray(m["coords"], np.float64).tofile(f)


def read_results(path, count):
    raw = open(path, "rb").read()
    out, pos = [], 0
    for _ in range(count):
        info = np.frombuffer(raw, np.int64, 14, pos)
        pos += 14 * 8
        n, nsf, ns = int(info[0]), int(info[5]), int(info[6])
        arrs = []
        for size in (n, n, n, nsf + 1, ns + 1, ns):
            arrs.append(np.frombuffer(raw, np.int32, size, pos))
            pos += 4 * size
        out.append((info, arrs))
    assert pos == len(raw)
    return out


def expected(m):
    n = m["n"]
    rev = np.arange(n - 1, -1, -1, dtype=np.int32)
    syms = [Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"]),
            Symbolic(n, m["colptr"], m["rowind"], leaf_size=16, dense_degree_min=64),
            Symbolic(n, m["colptr"], m["rowind"], user_perm=rev),
            Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"], relax=False)]
    syms.append(Symbolic.batch(syms[:2]))
    res = []
    for s in syms:
        i, e = s.info, s.export()
        info = [i[k] for k in ("n", "nnz_lower", "nnz_l", "flops", "flops_padded", "nsuper_fund", "nsuper", "nlevels",
                               "max_front", "nsep_nodes", "npeeled", "front_elems", "nnz_l_padded", "nseg")]
        res.append((info, [e["perm"], e["parent"], e["colcount"], e["super_ptr"], e["relaxed_ptr"], e["front_order"]]))
    return res


@pytest.mark.parametrize("case", ["g4", "g5", "small"])
def test_analysis_under_sanitizers_matches_library(analyze_driver, case):
    exe, d = analyze_driver
    m = {"g4": lambda: tiny(4, 1.5, seed=3).matrix(), "g5": lambda: tiny(5, 2.0, seed=4).matrix(),
         "small": lambda: small_fp64().matrix()}[case]()
    pat, out = str(d / f"{case}.bin"), str(d / f"{case}.out")
    write_pattern(pat, m)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, pat, out], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok 0"), r.stdout + r.stderr
    got = read_results(out, 5)
    for (gi, ga), (ei, ea) in zip(got, expected(m)):
        assert list(gi) == list(ei)
        for a, b in zip(ga, ea):
            assert np.array_equal(a, b)


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    r = subprocess.run(["gcc", "-std=c99", "-shared", "-fPIC"] + SAN + ["-o", lib, os.path.join(ROOT, "oracle", "oracle.c"),
                                                                         "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=runtime("libasan.so") + ":" + runtime("libubsan.so"),
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins_lu_field.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail
