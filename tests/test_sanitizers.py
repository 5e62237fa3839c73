"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The seeded graph generator (graphgen/graphgen.c) and the C oracle (oracle/pagerank_oracle.c),
  built with gcc -fsanitize=address,undefined, run on small R-MAT and Erdos-Renyi graphs through
  tests/sanitize/host_paths.c: edge draws, CSR builds, oracle solves in every norm, argument
  checks.  Leak detection is on.
* The C ABI of libprpull.so: every HIP source rebuilt with the host half instrumented (hipcc
  -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined; device code as usual), linked
  to the same driver built with -DWITH_PRPULL, which calls the entry points on their host-side
  argument paths (NULL pointers, out-of-range sizes and parameters, size queries, pr_create on a
  device that does not exist) -- no GPU is touched.
Any sanitizer report ends the driver with a non-zero status (-fno-sanitize-recover=all).
"""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_paths.c")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_generator_and_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_paths")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-fopenmp", DRIVER, os.path.join(ROOT, "oracle", "pagerank_oracle.c"),
          os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm", "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2"))
    assert "host paths ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not found")
def test_c_abi_argument_paths_under_asan_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2108_02997_amd", "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + flags + SAN_HOST + ["-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libprpull_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-o", lib] + objs)
    exe = str(tmp_path / "abi_paths")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-DWITH_PRPULL", DRIVER, "-I" + os.path.join(ROOT, "include"), "-L" + str(tmp_path), "-lprpull_san",
          "-Wl,-rpath," + str(tmp_path), "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert "host paths ok" in r.stdout
