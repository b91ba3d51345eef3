"""The oracle and the host side of plan creation built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: on the hipcc lines every -fsanitize= follows
-Xarch_host) and run on small meshes of every kind; no sanitizer report, exit status 0.
Runs without a GPU: plan creation then stops at its first device call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address", "-fsanitize=undefined"]


def _run(exe, tmp):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env, cwd=tmp)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", *SAN,
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-o", exe,
                    os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "dg_oracle.c"), "-lm"],
                   check=True, capture_output=True)
    assert "oracle driver ok" in _run(exe, tmp_path)


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_plan_host_code_under_sanitizers(tmp_path):
    build = os.path.join(ROOT, "paper_2210_03523_amd", "_build")
    kernels = [os.path.join(build, f) for f in sorted(os.listdir(build))
               if f.endswith(".o") and f not in ("api.o", "tables.o")] if os.path.isdir(build) else []
    if not kernels:
        pytest.skip("kernel objects not built")
    host = []
    for s in SAN:
        host += ["-Xarch_host", s]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
             *host, "-Xarch_host", "-fno-omit-frame-pointer"]
    src = [os.path.join(ROOT, "paper_2210_03523_amd", "csrc", "api.cpp"),
           os.path.join(ROOT, "paper_2210_03523_amd", "csrc", "tables.cpp"),
           os.path.join(HERE, "plan_driver.cpp")]
    objs = []
    for f in src:
        o = str(tmp_path / (os.path.basename(f) + ".o"))
        subprocess.run(["hipcc", "-x", "hip", *flags, "-c", f, "-o", o], check=True, capture_output=True)
        objs.append(o)
    exe = str(tmp_path / "plan_driver")
    subprocess.run(["hipcc", "--offload-arch=gfx950", *host, *objs, *kernels, "-o", exe, "-lrocsolver", "-lrocblas"],
                   check=True,
                   capture_output=True)
    assert "plan driver ok" in _run(exe, tmp_path)
