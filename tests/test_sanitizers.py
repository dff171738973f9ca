"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the pool's
range allocator against a bitmap model, the FP64 oracle under a subset of its pins, and the
host side of the C ABI (parameter checks, layout planning, workspace sizes, footprints)
under the CPU tests that call it.  Each part is built with the sanitizers into a temporary
directory and run in a child process with the sanitizer runtime preloaded (Python itself
is not instrumented); any report fails the child and so the test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_07842_amd", "csrc")
ENV_SAN = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _child(cmd, env_extra, logdir, timeout=600):
    env = dict(os.environ, **ENV_SAN, **env_extra)
    # reports go to files as well: pytest in the child may hold its stderr
    logs = os.path.join(str(logdir), "reports")
    os.makedirs(logs, exist_ok=True)
    env["ASAN_OPTIONS"] += f":log_path={logs}/asan"
    env["UBSAN_OPTIONS"] += f":log_path={logs}/ubsan"
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout, cwd=ROOT)
    out = r.stdout + r.stderr
    for fn in glob.glob(os.path.join(logs, "*")):
        out += open(fn, errors="replace").read()
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_range_allocator_under_sanitizers(tmp_path):
    exe = tmp_path / "arena_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", f"-I{CSRC}",
                           os.path.join(ROOT, "tests", "native", "test_arena.cpp"), "-o", str(exe)])
    out = _child([str(exe)], {}, tmp_path)
    assert "ok" in out.split()


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    asan = _gcc_runtime("libasan.so")
    if not asan:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build(force=True, out=str(tmp_path / "libvbc_oracle_san.so"),
                       extra_flags=("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                    "-fno-sanitize-recover=all"))
    sel = ("worked_examples or virial or bond_single or bond_virial or net_force or integers or "
           "stability_bound or observables or known_shapes or subset_matches or philox or "
           "exclusions_of_a_whole or multitype_reduces or repulsion_only or no_vbc or nve_energy")
    _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-k", sel,
            os.path.join(ROOT, "tests", "test_oracle_pins.py")],
           dict(LD_PRELOAD=asan, VBC_ORACLE_LIBRARY=lib, OMP_NUM_THREADS="2"), tmp_path)


def test_c_abi_host_side_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=fast-honor-pragmas",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}"]
    # sanitizers on the host code only (each -fsanitize behind -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("vbc_kernels.hip", "vbc_api.hip"):
        o = str(tmp_path / src.replace(".hip", ".o"))
        subprocess.check_call([hipcc, *flags, *san, "-c", os.path.join(CSRC, src), "-o", o],
                              stderr=subprocess.DEVNULL)
        objs.append(o)
    lib = str(tmp_path / "libvbc_san.so")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
                           "-o", lib, *objs, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                           "-Wl,-rpath,/opt/rocm/lib"], stderr=subprocess.DEVNULL)
    _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
            os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_serve_host.py"),
            os.path.join(ROOT, "tests", "test_tune_host.py")],
           dict(LD_PRELOAD=rt[-1], VBC_LIBRARY=lib), tmp_path)
