"""The C-ABI library loads and exports every function include/ipr.h declares
(no device calls: these run without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipr.h")
LIB = os.path.join(ROOT, "paper_1703_02283_amd", "libipr.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ipr_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libipr.so is not built (python -m paper_1703_02283_amd.build)")
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ipr_solve", "ipr_solve_batched", "ipr_workspace_size", "ipr_gemm",
                 "ipr_features", "ipr_mlp_forward", "ipr_mlp_train_step", "ipr_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(ipr_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_host_only_calls_work(lib):
    import paper_1703_02283_amd as ipr
    ipr.load()
    s = ipr.ipr_schedule_default()
    assert s.init == ipr.IPR_INIT_IDENTITY and s.max_iter == 100 and s.triangle == 1
    assert s.poly[0] == 1.0
    w1 = ipr.ipr_workspace_size(256, 2)
    w2 = ipr.ipr_workspace_size(512, 2)
    assert 4 * 256 * 256 * 8 <= w1 < w2
    assert ipr.ipr_workspace_size(0, 2) == 0
    assert ipr.ipr_last_error() == ""


def test_binding_signatures_match_header(lib):
    from paper_1703_02283_amd import binding
    assert set(binding._SIGS) == set(declared())


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of ipr_schedule / ipr_result have the header's field
    offsets and sizes (checked with the host compiler, no GPU)."""
    import ctypes as ct
    from paper_1703_02283_amd import binding
    lines = ["#include <cstdio>", "#include <cstddef>", '#include "ipr.h"', "int main() {"]
    for cname, cls in (("ipr_schedule", binding.IprSchedule), ("ipr_result", binding.IprResult)):
        lines.append(f'  std::printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  std::printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I",
                        os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-2000:])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True,
                               check=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, cls in (("ipr_schedule", binding.IprSchedule), ("ipr_result", binding.IprResult)):
        assert got[(cname, "size")] == ct.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
