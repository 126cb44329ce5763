"""AddressSanitizer and UndefinedBehaviorSanitizer builds (CPU only).

* The oracle, built with -fsanitize=address,undefined, runs every pin in a
  child process with the ASan runtime preloaded; any report fails it.
* The host side of the library (argument checks, plan and batch
  planning, the allocation-free entry point's size check), built with the
  same sanitizers on the host pass only, runs its validation-only paths in
  a child process.  No device code is sanitized and no GPU is touched.
"""

import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _gcc_runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                           text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _instrumented(lib):
    """The library calls the sanitizers' report hooks."""
    r = subprocess.run(["nm", "-D", lib], capture_output=True, text=True)
    return r.returncode == 0 and "__asan_report" in r.stdout and "__ubsan_handle" in r.stdout


def _run_child(code, preload, tmp):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], cwd=tmp, env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and \
        "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None or shutil.which("gcc") is None:
        pytest.skip("gcc ASan runtime not available")
    import oracle
    lib = oracle.build(out=str(tmp_path / "liboracle_san.so"),
                       extra=["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                              "-fno-sanitize-recover=undefined", "-O1"])
    assert _instrumented(lib)
    out = _run_child(f"""
        import oracle
        from tests import oracle_pins
        orc = oracle.load({lib!r})
        for pin in oracle_pins.PINS:
            if pin.__name__ == "pin_overflow_edge":
                continue   # 16.7M samples: minutes under ASan; it only sums zeros
            pin(orc)
            print("ok", pin.__name__, flush=True)
        print("ALL PINS OK")
    """, asan, str(tmp_path))
    assert "ALL PINS OK" in out


def test_host_library_validation_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    rt = subprocess.run(["/opt/rocm/lib/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True)
    asan = rt.stdout.strip()
    if rt.returncode != 0 or not os.path.exists(asan):
        pytest.skip("clang ASan runtime not available")
    src = os.path.join(ROOT, "paper_1503_06189_amd", "csrc", "xengine.hip")
    lib = str(tmp_path / "libxengine_san.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-shared-libasan",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), src, "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert _instrumented(lib)
    out = _run_child(f"""
        import ctypes
        from paper_1503_06189_amd import xengine as xe
        xe.LIB_PATH = {lib!r}
        L = xe.lib()
        vp = ctypes.c_void_p
        h = vp()
        assert L.xe_create(ctypes.byref(h), xe.XE_DEVICE_NONE, 0) == xe.XE_OK
        fake = vp(0x10000000)
        for N, F, T, B in [(1, 1, 1, 1), (256, 64, 16384, 256), (4096, 1, 40, 16),
                           (300, 3, 9001, 2**31 - 1), (0, 1, 1, 1), (16, 1, 2**24, 256)]:
            for fn in (L.xe_correlate_frame, L.xe_accumulate):
                s = fn(h, fake, None, N, F, T, B, fake, fake, None)
                assert s in (xe.XE_ERR_NO_DEVICE, xe.XE_ERR_ARG, xe.XE_ERR_OVERFLOW), s
            if N >= 1 and T < 2**24:
                xe.plan_query(N, F, T, B)
        shapes = [(64 * (1 + k % 16), 1 + k % 3, 256 * (1 + 37 * k % 250), 256) for k in range(128)]
        info = xe.batch_query(shapes, n_cu=256)
        assert info.instances + info.unaligned == 128
        assert L.xe_accumulate_noalloc(fake, None, 256, 64, 16_000_000, 256, fake, fake, None) \\
            == xe.XE_ERR_WORKSPACE
        assert L.xe_destroy(h) == xe.XE_OK
        print("HOST OK")
    """, asan, str(tmp_path))
    assert "HOST OK" in out
