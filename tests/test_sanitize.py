"""AddressSanitizer / UndefinedBehaviorSanitizer builds on the CPU (no GPU needed):

* the C oracle, driven over hundreds of small seeded graphs with every option combination,
  edge cases and invalid arguments (tests/sanitize/oracle_driver.c);
* the library's host code (launch plans, workspace carve-up, batch chunking, schedule and
  argument checks), built with the sanitizers on the host side only and driven through the
  size queries and argument checks of the C ABI, which never touch a device
  (tests/sanitize/plan_driver.c).

A sanitizer report aborts the driver (no recovery), so a clean exit is the pass."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, f"{os.path.basename(exe)} exit {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", *SAN, os.path.join(HERE, "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "gee_oracle.c"), "-lm", "-o", exe], check=True)
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})


def test_a_planted_out_of_bounds_write_is_caught(tmp_path):
    """The harness itself: an oracle copy whose degree loop writes one slot past the end
    must make the sanitized driver fail."""
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    text = open(os.path.join(ROOT, "oracle", "gee_oracle.c")).read()
    old = "deg[L.i[t]] += L.v[t];"
    assert old in text
    bad = tmp_path / "oracle_oob.c"
    bad.write_text(text.replace(old, "deg[L.i[t] + 1] += L.v[t];", 1))
    exe = str(tmp_path / "oracle_driver_oob")
    subprocess.run(["gcc", "-O1", "-g", *SAN, os.path.join(HERE, "oracle_driver.c"), str(bad), "-lm", "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2406_03726_amd import build as B

    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    hip = B.hipcc()
    # sanitizers on the host side only (each -fsanitize after -Xarch_host); device code as usual
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    objs = []
    procs = []
    for src in B.sources():
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([hip, "-c", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}",
                                       "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
                                       f"-I{B.INCLUDE}", f"-I{B.CSRC}", src, "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode()[-3000:]
    drv = str(tmp_path / "plan_driver.o")
    subprocess.run(["gcc", "-O1", "-g", "-c", *SAN, f"-I{B.INCLUDE}", os.path.join(HERE, "plan_driver.c"), "-o", drv],
                   check=True)
    exe = str(tmp_path / "plan_driver")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hip)))
    subprocess.run(["g++", *SAN, drv, *objs, f"-L{rocm}/lib", f"-Wl,-rpath,{rocm}/lib", "-lamdhip64", "-o", exe],
                   check=True, capture_output=True)
    # the HIP runtime keeps allocations for the process's life: leaks are not this test's subject
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
