"""AddressSanitizer and UndefinedBehaviorSanitizer over the host code:

* the oracle (plain C, gcc), driven through every exported function on small
  and edge-sized inputs (tests/helpers/sanitize_oracle.c);
* the library's host code (argument validation, threshold table, fast
  division; all C-ABI translation units, sanitizers on the host side only),
  driven with invalid arguments on every entry point
  (tests/helpers/sanitize_abi.c).

Both run without a GPU; any out-of-bounds access or undefined behaviour
aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPERS = os.path.join(ROOT, "tests", "helpers")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "san_oracle")
    subprocess.run([gcc, "-std=c11", "-O1", "-g", *SAN, "-ffp-contract=off",
                    os.path.join(ROOT, "oracle", "shaken_oracle.c"), os.path.join(HELPERS, "sanitize_oracle.c"),
                    "-lm", "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "sanitized oracle run ok" in res.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("HIP toolchain missing")
    from paper_1908_07341_amd import build as B
    # host-side sanitizers only: each -fsanitize= goes to the host compilation
    host_san = []
    for flag in SAN:
        host_san += ["-Xarch_host", flag]
    srcs = sorted(os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith((".cpp", ".hip")))
    objs = []
    procs = []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [hipcc, f"--offload-arch={B.ARCH}", *B.COMMON, *host_san, "-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out
    lib = str(tmp_path / "libshaken_san.so")
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *host_san, *objs, "-o", lib],
                   check=True)
    exe = str(tmp_path / "san_abi")
    subprocess.run([clang, "-std=c11", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(HELPERS, "sanitize_abi.c"), lib, f"-Wl,-rpath,{tmp_path}",
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:]
    assert "0 failure(s)" in res.stdout
