"""The boundary used from C: `c_abi_example.c` includes only include/sdc.h
(and the HIP runtime API for device memory), is compiled as C11 with gcc and
linked against the in-tree library.  Without a GPU the build and link are
checked; with one, the program runs its own checks (exact pair counts,
C(0, 0) = 1, the FP64 self term)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2308_07487_amd")
SRC = os.path.join(ROOT, "tests", "c_abi_example.c")


def _build(out):
    if not os.path.exists(os.path.join(PKG, "libsdc.so")):
        pytest.skip("libsdc.so is not built")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", SRC,
           "-L", PKG, "-lsdc", "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{PKG}:/opt/rocm/lib", "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return out


def test_c_program_builds_against_the_header(tmp_path):
    assert os.path.exists(_build(tmp_path / "c_abi_example"))


@pytest.mark.gpu
def test_c_program_runs(tmp_path):
    exe = _build(tmp_path / "c_abi_example")
    print("[case] C ABI example", flush=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    assert "ok" in r.stdout
