"""Host code of libpft under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds every library source with the sanitizers on its host part only (the device code is compiled as
usual), links the harness tests/host_check/main.cpp into an executable and runs it: the edge-sharing
face order on random and broken meshes, and the synchronous validation of the entry points. The build
is kept under the package's _build folder and redone when a source is newer than the executable.
"""
import os
import shutil
import subprocess

import pytest

from paper_2104_08309_amd import build as b

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(b.BUILD, "host_sanitizers")
EXE = os.path.join(OUT, "host_check")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _stale(srcs):
    return not os.path.exists(EXE) or any(os.path.getmtime(s) > os.path.getmtime(EXE) for s in srcs)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_host_code_under_sanitizers():
    hipcc = b._hipcc()
    os.makedirs(OUT, exist_ok=True)
    main = os.path.join(HERE, "host_check", "main.cpp")
    srcs = [os.path.join(b.CSRC, f) for f in b.SOURCES] + [main]
    if _stale(srcs + [os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC) if f.endswith(".h")]):
        objs = []
        procs = []
        for src in srcs:
            obj = os.path.join(OUT, os.path.splitext(os.path.basename(src))[0] + ".o")
            cmd = [hipcc, "-x", "hip"] + [f for f in b.COMMON if f != "-fPIC"] + SAN + ["-c", src, "-o", obj]
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), src))
            objs.append(obj)
        for p, src in procs:
            out, err = p.communicate()
            assert p.returncode == 0, f"compile {src}:\n{err[-3000:]}"
        cmd = [hipcc, f"--offload-arch={b.ARCH}"] + SAN + ["-o", EXE] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout
