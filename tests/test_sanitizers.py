"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built in a temporary directory and run:
  - the library's host-side assignment (KD-trees, the auction, its
    optimality certificate, heaps, exact reductions; Eq. (1), Sec. 4.3) on
    instances of up to 2300 x 2100 points and targets (the auction's searches
    on several threads), through ts_assign and
    ts_assign_auction; the HIP sources are compiled with the sanitizers on
    their host pass only;
  - the CPU oracle (diagram, full reduction, a short solve and one
    assignment step) on small random fields.
A sanitizer report makes the driver exit non-zero."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_12399_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
HOST_SAN = [f for s in SAN for f in ("-Xarch_host", s)]


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    return env


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_main")
    _run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off"] + SAN +
         ["-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "tso.cpp"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_main.cpp"), "-o", exe], str(tmp_path))
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None,
                    reason="no hipcc or g++")
def test_library_host_code_under_sanitizers(tmp_path):
    inc = os.path.join(ROOT, "include")
    dev = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"]

    def hip_obj(src):
        obj = str(tmp_path / (src.rsplit(".", 1)[0] + ".o"))
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-pthread", "-ffp-contract=off",
              "-x", "hip"] + dev + HOST_SAN + ["-I", inc, "-c", os.path.join(CSRC, src),
                                              "-o", obj], str(tmp_path))
        return obj

    with ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(hip_obj, ["sort.hip", "persistence.hip", "solver.hip", "unet.hip"]))
    host = []
    for src, out in ((os.path.join(CSRC, "api.cpp"), "api.o"),
                     (os.path.join(ROOT, "tests", "sanitize", "assign_main.cpp"), "main.o")):
        host.append(str(tmp_path / out))
        _run(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__"] + SAN +
             ["-I", "/opt/rocm/include", "-I", inc, "-c", src, "-o", host[-1]], str(tmp_path))
    exe = str(tmp_path / "assign_main")
    _run(["g++", "-pthread"] + SAN + host + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe], str(tmp_path))
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr
