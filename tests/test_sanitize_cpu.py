"""The host layer of the library (validation, enumeration, decompose's searches, the
front end's text translation) and the oracle, built with AddressSanitizer and
UndefinedBehaviorSanitizer (every report fatal) and run on seeded fuzz cases:
random and corrupted candidate records checked against the oracle's validator,
random bytes, enumeration and argmin searches against the oracle's, and mutated
mapper texts through the parser (fuzz_host.cpp beside this file).  CPU only."""
import os
import re
import shutil
import subprocess

import pytest

import workloads  # noqa: F401  (puts the repository root on the path, like the other tests)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
CASES = 12000


@pytest.fixture(scope="module")
def fuzz_bin(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")
    d = tmp_path_factory.mktemp("sanitize")
    csrc = os.path.join(ROOT, "paper_2507_17087_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include")]
    # host-only parts of the library: no device code, so the HIP headers are only
    # needed for their host declarations
    hip = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
    jobs = [["gcc", "-std=c11"] + SAN + ["-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(d / "oracle.o")]]
    for f in ("tm_host.cpp", "tm_frontend.cpp"):
        jobs.append(["g++", "-std=c++17"] + SAN + hip + inc + ["-c", os.path.join(csrc, f), "-o", str(d / (f + ".o"))])
    jobs.append(["g++", "-std=c++17"] + SAN + inc + ["-c", os.path.join(ROOT, "tests", "fuzz_host.cpp"), "-o",
                                                     str(d / "fuzz.o")])
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for j in jobs]
    for j, p in zip(jobs, procs):
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, (" ".join(j), out)
    exe = str(d / "fuzz")
    subprocess.check_call(["g++", "-fsanitize=address,undefined", "-o", exe, str(d / "fuzz.o"),
                           str(d / "tm_host.cpp.o"), str(d / "tm_frontend.cpp.o"), str(d / "oracle.o")])
    corpus = d / "corpus.bin"
    from test_frontend_cpu import HIER, ROWS, TILES
    corpus.write_bytes(b"\0".join(s.encode() for s in (TILES, HIER, ROWS)))
    return exe, str(corpus)


def test_host_layer_and_oracle_under_sanitizers(fuzz_bin):
    exe, corpus = fuzz_bin
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([exe, "17087", str(CASES), corpus], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    line = p.stdout.strip().splitlines()[-1]
    num = {k: int(v) for k, v in re.findall(r"\b(cases|checks|mismatches|valid|translated) (\d+)", line)}
    assert num["cases"] >= 10_000 and num["mismatches"] == 0, line
    assert num["valid"] > 1000, line  # candidates deep enough to reach the oracle's evaluators
    assert num["translated"] > 50, line  # mutated mappers that still translate
