"""The reference library under the sanitizers (CPU): AddressSanitizer + UndefinedBehavior-
Sanitizer with gcc and libgomp, and ThreadSanitizer with LLVM's OpenMP runtime and its
Archer tool (which tells ThreadSanitizer about OpenMP's own synchronisation).  The driver
tests/oracle_sanitize_main.c calls every entry point of oracle/rsi_oracle.c on small inputs.
A planted race in a separate probe program shows that the ThreadSanitizer set-up reports
races at all."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "oracle", "rsi_oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_main.c")]
LLVM = "/opt/rocm/llvm"


def _run(exe, env_extra, timeout=300):
    env = dict(os.environ, OMP_NUM_THREADS="4", **env_extra)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=timeout)


def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_asan")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    *SOURCES, "-lm", "-o", exe], check=True)
    r = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def _tsan_build(src_list, exe):
    clang, archer = os.path.join(LLVM, "bin", "clang"), os.path.join(LLVM, "lib", "libarcher.so")
    if not (shutil.which(clang) and os.path.exists(archer)):
        pytest.skip("LLVM clang with the Archer OpenMP tool is not installed")
    subprocess.run([clang, "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=thread",
                    *src_list, "-lm", "-o", exe, f"-Wl,-rpath,{LLVM}/lib"], check=True)
    return {"TSAN_OPTIONS": "ignore_noninstrumented_modules=1 halt_on_error=1",
            "OMP_TOOL_LIBRARIES": archer}


def test_oracle_tsan(tmp_path):
    exe = str(tmp_path / "orc_tsan")
    env = _tsan_build(SOURCES, exe)
    r = _run(exe, env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr[-2000:]


def test_tsan_setup_reports_a_planted_race(tmp_path):
    src = tmp_path / "race.c"
    src.write_text("#include <stdio.h>\n"
                   "int main(void) {\n"
                   "    double s = 0.0;\n"
                   "#pragma omp parallel for\n"
                   "    for (int i = 0; i < 100000; ++i) s += 1.0;\n"
                   "    printf(\"%g\\n\", s);\n"
                   "    return 0;\n"
                   "}\n")
    exe = str(tmp_path / "race")
    env = _tsan_build([str(src)], exe)
    r = _run(exe, env)
    assert r.returncode != 0 and "data race" in r.stderr
