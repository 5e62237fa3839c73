"""The C ABI library loads and exports every function include/prpull.h declares (no GPU)."""
import ctypes
import os

import pytest

torch = pytest.importorskip("torch")

from paper_2108_02997_amd import _lib  # noqa: E402


def test_library_exports_every_declared_function():
    names = _lib.header_functions()
    assert "pr_pull" in names and "pr_prepare" in names
    lib = _lib.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(_lib.SIGNATURES), "binding lacks a declared function"


def test_sizes_without_device():
    lib = _lib.load()
    assert lib.pr_workspace_bytes(1000, 8000, 0, 0) > 16000
    assert lib.pr_workspace_bytes(1000, 8000, 1, 0) > lib.pr_workspace_bytes(1000, 8000, 0, 0)
    assert lib.pr_workspace_bytes(1000, 8000, 0, 1) > lib.pr_workspace_bytes(1000, 8000, 0, 0)
    assert lib.pr_workspace_bytes(0, 8000, 0, 0) == 0
    assert lib.pr_workspace_bytes(10, 10, 5, 0) == 0
    assert lib.pr_prep_bytes(1 << 20, 16 << 20) > 16 * (1 << 14)
    assert b"gfx950" in lib.pr_version()


def test_no_context_without_device():
    lib = _lib.load()
    h = ctypes.c_void_p()
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    assert lib.pr_create(ctypes.byref(h), 0) < 0
    assert lib.pr_last_error()


def test_null_arguments_rejected_on_host():
    lib = _lib.load()
    assert lib.pr_pull(None, None, None, None, None, 10, 10, None, 0.85, 1e-6, 1, 10, 0, None, None, None, None,
                       0, None) == _lib.PR_EINVAL
    assert lib.pr_set_option(None, b"grid", 3) == _lib.PR_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_size_limits_of_the_int32_csr():
    # the largest graph the ABI takes: N = 2^31 - 2 vertices, E = 2^31 - 1 entries (int32 offsets)
    lib = _lib.load()
    n_max, e_max = (1 << 31) - 2, (1 << 31) - 1
    for prec in (0, 1, 2):
        b = lib.pr_workspace_bytes(n_max, e_max, prec, 1)
        assert b >= 2 * 8 * n_max and b < 1 << 40
        assert lib.pr_workspace_bytes(n_max + 1, e_max, prec, 1) == 0
        assert lib.pr_workspace_bytes(n_max, e_max + 1, prec, 1) == 0
    assert lib.pr_prep_bytes(n_max, e_max) > 0 and lib.pr_prep_bytes(n_max, e_max + 1) == 0
    assert lib.pr_batch_workspace_bytes(n_max, e_max, 16, 1, 1) > 0
    assert lib.pr_batch_workspace_bytes(n_max, e_max, 17, 1, 1) == 0
    assert lib.pr_batch_workspace_bytes(n_max, e_max, 4, 2, 1) == 0   # no float32-only batches
    assert lib.pr_mlp_backward_workspace_bytes(n_max) > 0 and lib.pr_mlp_backward_workspace_bytes(0) == 0


def test_every_option_key_is_documented():
    # the keys pr_set_option accepts (its string compares) and the ones the header documents
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = open(os.path.join(root, "paper_2108_02997_amd", "csrc", "api.hip")).read()
    header = open(os.path.join(root, "include", "prpull.h")).read()
    accepted = set(re.findall(r'strcmp\(key, "([a-z_0-9]+)"\)', code))
    documented = set(re.findall(r'^ \*   "([a-z_0-9]+)"', header, flags=re.M))
    assert accepted and accepted == documented, (sorted(accepted - documented), sorted(documented - accepted))


def test_struct_mirrors_match_the_header(tmp_path):
    # every ctypes mirror of a header struct has the header's size and field offsets, compiled
    # from include/prpull.h by the host C compiler
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    mirrors = [_lib.pr_result, _lib.pr_problem, _lib.pr_graph_problem, _lib.pr_tune_result]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "prpull.h"', "int main(void) {"]
    for m in mirrors:
        name = m.__name__
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in m._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([cc, "-I", os.path.join(root, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for m in mirrors:
        name = m.__name__
        assert int(got[name]) == ctypes.sizeof(m), name
        for f, _ in m._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(m, f).offset, (name, f)
