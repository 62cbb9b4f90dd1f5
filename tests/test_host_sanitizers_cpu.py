"""Host sanitizer build (CPU): the library's host code compiled with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged) and
exercised without a GPU.

Two parts, both in a subprocess that preloads the sanitizer runtime (the
Python interpreter itself is not instrumented):
* the C-ABI checks of test_abi_cpu.py against the sanitized library: status
  strings, default settings, NULL-argument rejection, context creation
  without a GPU (an error, not a crash);
* tests/host/runtime_host_test.hip, which includes the runtime source and
  checks the view plan, the work-item tables of every order and tile size
  (each 8x8 block once, queue offsets, per-tile records) and the autotuner
  cache file, including keys longer than its line buffer.
Any sanitizer report aborts the subprocess (halt_on_error) and fails the
test with the report."""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_16144_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

BASE = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
        "-packed-fp32-ops", "-munsafe-fp-atomics", "-Wno-unused-command-line-argument", "-Wno-unused-result",
        "-Wno-unused-value", "-I", os.path.join(ROOT, "include")]
# host-only instrumentation: each sanitizer flag applies to the host pass
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
KERNEL_SOURCES = ["project.hip", "binning.hip", "radix_sort.hip", "raster.hip", "loss.hip", "decoder.hip",
                  "prune.hip"]


def _cc(args):
    r = subprocess.run([HIPCC, *args], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if not os.path.exists(HIPCC) or not ASAN_RT:
        pytest.skip("hipcc or the sanitizer runtime is not available")
    d = tmp_path_factory.mktemp("san")
    jobs = [(BASE + ["-c", os.path.join(CSRC, s), "-o", str(d / (s + ".o"))]) for s in KERNEL_SOURCES]
    jobs.append(BASE + SAN + ["-c", os.path.join(CSRC, "runtime.hip"), "-o", str(d / "runtime.o")])
    jobs.append(BASE + SAN + ["-c", os.path.join(ROOT, "tests", "host", "runtime_host_test.hip"),
                              "-o", str(d / "host_test.o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_cc, jobs))
    kern = [str(d / (s + ".o")) for s in KERNEL_SOURCES]
    lib = str(d / "liblego_raster_san.so")
    _cc(["-shared", "-fPIC", "--offload-arch=gfx950", *kern, str(d / "runtime.o"), "-o", lib])
    test_lib = str(d / "libruntime_host_test.so")
    _cc(["-shared", "-fPIC", "--offload-arch=gfx950", *kern, str(d / "host_test.o"), "-o", test_lib])
    return {"lib": lib, "test_lib": test_lib, "dir": str(d)}


def _run(code):
    env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1],
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], capture_output=True, text=True, env=env,
                       timeout=300)
    return r.returncode, r.stdout + r.stderr


def test_abi_checks_under_host_sanitizers(sanitized):
    rc, out = _run(f"""
        import ctypes as C
        lib = C.CDLL({sanitized['lib']!r})
        lib.lgs_status_string.restype = C.c_char_p
        lib.lgs_last_error.restype = C.c_char_p
        names = ["LGS_OK", "LGS_ERR_INVALID_ARG", "LGS_ERR_HIP", "LGS_ERR_CAPACITY", "LGS_ERR_UNSUPPORTED",
                 "LGS_ERR_STATE"]
        for code, name in enumerate(names):
            assert lib.lgs_status_string(code).decode() == name
        assert lib.lgs_status_string(99) is not None
        assert lib.lgs_context_create(0, None) == 1
        assert lib.lgs_forward(None, None, None, 1, None, None, None, None) == 1
        assert lib.lgs_backward(None, None, None, None, None, None) == 1
        assert lib.lgs_backward_l1(None, None, None, None, None, None, None, None) == 1
        assert lib.lgs_decoder_l1(None, 1, 1, 256, None, None, None, None, 0, C.c_float(1.0), None, None, None,
                                  None, None) == 1
        assert lib.lgs_decoder_l1_noalloc(None, 1, 1, 256, None, None, None, None, 0, C.c_float(1.0), None, None,
                                          None, None, None) == 1
        assert lib.lgs_last_error(None).decode() == "NULL context"
        h = C.c_void_p()
        assert lib.lgs_context_create(0, C.byref(h)) == 2 and not h.value   # no GPU here: an error, no crash
        print("abi checks OK")
        """)
    assert rc == 0 and "abi checks OK" in out, out[-6000:]


def test_planning_code_under_host_sanitizers(sanitized):
    cache = os.path.join(sanitized["dir"], "tune_cache.json")
    rc, out = _run(f"""
        import ctypes as C
        lib = C.CDLL({sanitized['test_lib']!r})
        n = lib.lgs_host_selftest({cache!r}.encode())
        print("failed checks:", n)
        raise SystemExit(1 if n else 0)
        """)
    assert rc == 0 and "failed checks: 0" in out, out[-6000:]
