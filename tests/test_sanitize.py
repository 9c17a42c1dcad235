"""The CPU oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven on the CPU (no GPU needed).

* oracle: oracle/so3_oracle.c in both builds (double, long double) under
  gcc's sanitizers, every entry point at B = 1 ... 8 (non-powers of two take
  the direct-DFT path) with a round-trip check (tests/sanitize/oracle_driver.c).
* library host code: soft_api.hip with the sanitizers on its host half only
  (the device code is not instrumented), linked with the plain kernel objects,
  driving soft_plan_check (plan tables, work lists and their checks for one,
  batched and mixed bandwidths in every precision and flag) and the argument
  checks of the entry points (tests/sanitize/plan_driver.cpp).
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def run(cmd, **kw):
    r = subprocess.run([str(c) for c in cmd], capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    objs = []
    for tag, defs in (("f64", []), ("f80", ["-DSO3O_LONG_DOUBLE"])):
        obj = tmp_path / f"so3_oracle_{tag}.o"
        run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", *san, *defs, "-c",
             os.path.join(ROOT, "oracle", "so3_oracle.c"), "-o", obj])
        objs.append(obj)
    exe = tmp_path / "oracle_driver"
    run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", *san, os.path.join(HERE, "oracle_driver.c"), *objs,
         "-lm", "-o", exe])
    r = run([exe], env=ENV, timeout=600)
    assert "ok" in r.stdout


def test_plan_host_code_under_sanitizers(tmp_path):
    from paper_1808_00896_amd import build as lib_build
    kernels = [os.path.join(lib_build.OUT_DIR, f + ".o")
               for f in sorted(os.listdir(lib_build.CSRC)) if f.endswith(".hip") and f != "soft_api.hip"]
    if not all(os.path.exists(k) for k in kernels):
        lib_build.build()
    # host sanitizers only: each -fsanitize goes to the host compilation
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    api = tmp_path / "soft_api_san.o"
    run([lib_build.HIPCC, *lib_build.CFLAGS, "-O1", "-g", *san, "-c",
         os.path.join(lib_build.CSRC, "soft_api.hip"), "-o", api])
    drv = tmp_path / "plan_driver.o"
    run([lib_build.HIPCC, f"--offload-arch={lib_build.ARCH}", "-std=c++17", "-O1", "-g", *san,
         "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "plan_driver.cpp"), "-o", drv])
    exe = tmp_path / "plan_driver"
    run([lib_build.HIPCC, f"--offload-arch={lib_build.ARCH}", *san, drv, api, *kernels, "-o", exe])
    # the HIP runtime's own allocations outlive main: leaks are not checked here
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = run([exe], env=env, timeout=300)
    assert "ok" in r.stdout
