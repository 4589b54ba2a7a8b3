"""CPU: the host code under sanitizers.

* The scheduler of the request server (simulated executor: manual steps with injected launch and
  device failures and cancellations; the threaded mode with concurrent submitters, cancellers and
  a poller), the planner over a sweep of sizes and the host-side argument checks -- built with
  AddressSanitizer + UndefinedBehaviorSanitizer, and the threaded scheduler with
  ThreadSanitizer (tests/native/server_driver.cpp).
* The C oracle's entry points on small images, every order and variant, with AddressSanitizer +
  UndefinedBehaviorSanitizer (tests/native/oracle_driver.c).

The library sources under test (planner, C API, server) are compiled with the sanitizers; the
kernel sources, whose host parts only enqueue launches, are linked from the regular build.
Nothing here touches a GPU.  Every sanitizer flag goes to the host compilation only
(-Xarch_host), so no device code is instrumented.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_14970_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
OUT = os.path.join(ROOT, "_build", "sanitize")
SANITIZED = ["fge_plan.cpp", "fge_api.cpp", "fge_server.cpp"]
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
TSAN = ["-Xarch_host", "-fsanitize=thread"]


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _regular_objects():
    """Objects of the regular build for the sources not under test, compiled when missing or
    older than their source."""
    from paper_2006_14970_amd import build
    objs = []
    for src in build.SOURCES:
        if src in SANITIZED:
            continue
        obj = os.path.join(build.BUILD_DIR, src + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(os.path.join(CSRC, src)):
            os.makedirs(build.BUILD_DIR, exist_ok=True)
            build._compile(build.hipcc(), src, False)
        objs.append(obj)
    return objs


def _build_driver(kind, san):
    cc = _hipcc()
    out_dir = os.path.join(OUT, kind)
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = [os.path.join(CSRC, f) for f in SANITIZED] + [os.path.join(NATIVE, "server_driver.cpp")]
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((subprocess.Popen([cc, *flags, *san, "-c", src, "-o", obj],
                                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
                      src))
    for p, src in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"compiling {src}:\n{err[-4000:]}"
    exe = os.path.join(out_dir, "server_driver")
    # the same flags at the link (as -Xarch_host pairs), less the code-generation one
    link_san = []
    for k in range(0, len(san), 2):
        if san[k + 1] != "-fno-omit-frame-pointer":
            link_san += san[k:k + 2]
    _run([cc, "--offload-arch=gfx950", *link_san, *objs, *_regular_objects(), "-o", exe])
    return exe


def test_server_and_planner_under_asan_ubsan():
    exe = _build_driver("asan", ASAN)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = _run([exe, "manual", "plan", "threaded"], env=env, timeout=600)
    assert "manual: ok" in r.stdout and "plan: ok" in r.stdout and "threaded: ok" in r.stdout


def test_threaded_scheduler_under_tsan():
    exe = _build_driver("tsan", TSAN)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = _run([exe, "threaded", "manual"], env=env, timeout=600)
    assert "threaded: ok" in r.stdout and "manual: ok" in r.stdout


def test_oracle_under_asan_ubsan():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run([cc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "fge_oracle.c"), os.path.join(NATIVE, "oracle_driver.c"),
          "-lm", "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"),
             timeout=300)
    assert "oracle: ok" in r.stdout
