"""Sanitizer tier on the CPU: the oracle and the library's host code built
with AddressSanitizer + UndefinedBehaviorSanitizer, each run under the tests
that exercise it.

* oracle/sv_oracle.c (gcc, -fsanitize=address,undefined): the oracle's pins
  (tests/test_oracle_pins.py, tests/test_oracle_shots.py) run on it; a copy
  with a planted out-of-bounds write must be caught.
* the library's host-only sources (validation, fusion planner, batch
  planner, autotuner driver, gate matrices; hipcc with the sanitizers on the
  host side only), linked with the regular device objects:
  tests/test_abi.py runs on it (argument validation, status strings, the
  fusion planner against the oracle, batch-plan validation). No GPU work.

Each run is a subprocess with the sanitizer runtime preloaded (Python itself
is not instrumented); leak checking is off (the interpreter's own
allocations are not ours).
"""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "sv_oracle.c")
CSRC = os.path.join(ROOT, "paper_2511_19291_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.timeout(600)


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def _clang_asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def _env(preload, **extra):
    env = dict(os.environ)
    prev = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = preload + (":" + prev if prev else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    env.update(extra)
    return env


def _build_oracle(src, out):
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", out, src, "-lm"], check=True)


@pytest.fixture(scope="module")
def asan_rt():
    rt = _gcc_runtime("libasan.so")
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    return rt


def test_oracle_pins_under_sanitizers(tmp_path, asan_rt):
    lib = str(tmp_path / "liboracle_san.so")
    _build_oracle(ORACLE_SRC, lib)
    env = _env(asan_rt, SV_ORACLE_LIB=lib)
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.load()._name)"], cwd=ROOT, env=env,
                           capture_output=True, text=True)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_shots.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def test_sanitizer_catches_planted_overflow(tmp_path, asan_rt):
    """The instrumented build has teeth: a copy of the oracle whose basis
    write lands one element past the end is stopped by AddressSanitizer."""
    src = open(ORACLE_SRC).read()
    good = "    psi[idx] = 1;\n"
    assert src.count(good) == 1
    bad = tmp_path / "sv_oracle_overflow.c"
    bad.write_text(src.replace(good, "    psi[N] = 1;\n    psi[idx] = 1;\n"))
    lib = str(tmp_path / "liboracle_overflow.so")
    _build_oracle(str(bad), lib)
    r = subprocess.run([sys.executable, "-c", "import oracle; oracle.basis_state(4, 0)"], cwd=ROOT,
                       env=_env(asan_rt, SV_ORACLE_LIB=lib), capture_output=True, text=True)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr and "heap-buffer-overflow" in r.stderr


def _device_objects():
    """The regular build's device objects (one per .hip file); built first
    if missing."""
    objs = sorted(glob.glob(os.path.join(ROOT, "paper_2511_19291_amd", "_build", "*.hip.o")))
    hips = glob.glob(os.path.join(CSRC, "*.hip"))
    if len(objs) != len(hips):
        from paper_2511_19291_amd.csrc import build as hb
        hb.build()
        objs = sorted(glob.glob(os.path.join(ROOT, "paper_2511_19291_amd", "_build", "*.hip.o")))
    return objs


def test_library_host_code_under_sanitizers(tmp_path):
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC) or not os.path.exists(CLANGXX):
        pytest.skip("ROCm's clang AddressSanitizer runtime or hipcc is missing")
    dev = _device_objects()
    procs, objs = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        # host code only: -Xarch_host keeps the sanitizers off any device pass
        procs.append(subprocess.Popen([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                                       "-Xarch_host", "-fsanitize=address,undefined",
                                       "-Xarch_host", "-fno-sanitize-recover=undefined",
                                       "-fno-omit-frame-pointer", "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    lib = str(tmp_path / "libsv_san.so")
    subprocess.run([CLANGXX, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libasan",
                    "-o", lib, *objs, *dev, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                   check=True)
    env = _env(rt, SV_LIB_PATH=lib)
    probe = subprocess.run([sys.executable, "-c", "from paper_2511_19291_amd import sv; print(sv.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
