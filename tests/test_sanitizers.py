"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The oracle's C source is rebuilt with gcc and the sanitizers, and its pins
  (tests/test_oracle.py) run against that build.
- The library is rebuilt with the sanitizers on its host code only (hipcc's
  -Xarch_host; the device code is unchanged), and the host tests of the
  boundary (tests/test_abi_host.py: argument validation, layout keys,
  exports) run against that build.
Each run is a subprocess with the sanitizer runtime preloaded; any report
fails it (UBSan halts on error; leak checking is off: the Python
interpreter's own allocations are not this code's)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _run(script, preload, env_extra=None):
    env = dict(os.environ)
    env.update({"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "LD_PRELOAD": preload, "OMP_NUM_THREADS": "4"})
    env.update(env_extra or {})
    r = subprocess.run([sys.executable, "-c", script], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    return r.returncode


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = tmp_path / "libsdc_oracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                           "-shared", "-fPIC", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "sdc_oracle.c"), "-o", str(lib), "-lm"])
    pre = " ".join(subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
                   for n in ("libasan.so", "libubsan.so"))
    script = ("import sys, oracle, pytest\n"
              f"oracle._LIB_PATH = {str(lib)!r}\n"
              "oracle.build = lambda force=True: oracle._LIB_PATH\n"
              "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_oracle.py']))\n")
    assert _run(script, pre) == 0


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="needs hipcc")
def test_boundary_host_code_under_sanitizers(tmp_path):
    lib = tmp_path / "libsdc_san.so"
    csrc = os.path.join(ROOT, "paper_2308_07487_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".cpp", ".hip")))
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "include"), *srcs, "-o", str(lib)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    clang = "/opt/rocm/llvm/bin/clang"
    pre = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    script = ("import sys, pytest\n"
              "from paper_2308_07487_amd import sdc\n"
              f"sdc.LIB_PATH = {str(lib)!r}\n"
              "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_abi_host.py']))\n")
    assert _run(script, pre) == 0
