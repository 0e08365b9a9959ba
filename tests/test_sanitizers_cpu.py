"""Host sanitizers over the CPU code: the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (every entry point, FP64 and FP32-coordinate forms,
both particle orders), the oracle's threaded walker runner under
ThreadSanitizer, and the exchange model of the cooperative sweep
(tests/spread_protocol_model.cc) under ThreadSanitizer.  All builds use gcc /
g++ on host code only; a sanitizer report makes the program exit non-zero."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")


def _build(tmp, name, flags):
    exe = str(tmp / name)
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-pthread", *flags,
           "-I" + ORACLE, os.path.join(ORACLE, "oracle.c"), DRIVER, "-o", exe, "-lm"]
    try:
        subprocess.run(cmd, check=True, capture_output=True, text=True)
    except subprocess.CalledProcessError as e:   # the toolchain lacks the runtime
        pytest.skip("sanitizer build failed: " + e.stderr[-400:])
    return exe


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
    assert "runtime error" not in out.stderr and "WARNING: ThreadSanitizer" not in out.stderr, out.stderr[-4000:]
    return out.stdout.split()


@pytest.fixture(scope="module")
def asan(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("asan"), "oracle_asan",
                  ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])


@pytest.fixture(scope="module")
def tsan(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("tsan"), "oracle_tsan", ["-fsanitize=thread"])


@pytest.mark.parametrize("n,fp32,order", [(32, 0, 0), (108, 0, 1), (108, 1, 0), (61, 1, 1)])
def test_oracle_under_address_and_ub_sanitizers(asan, n, fp32, order):
    r = _run(asan, n, fp32, order, 2)
    assert r[0] == "ok" and int(r[1]) == 12 and int(r[2]) > 0


def test_threaded_walker_runner_under_thread_sanitizer(tsan):
    r = _run(tsan, 108, 0, 0, 3)
    assert r[0] == "ok" and int(r[1]) == 12


def test_exchange_model_under_thread_sanitizer(tmp_path):
    exe = str(tmp_path / "model_tsan")
    try:
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread",
                        os.path.join(HERE, "spread_protocol_model.cc"), "-o", exe],
                       check=True, capture_output=True, text=True)
    except subprocess.CalledProcessError as e:
        pytest.skip("sanitizer build failed: " + e.stderr[-400:])
    r = _run(exe, 3, 61, 3000, 1 << 30, -1)
    assert r[0] == "ok" and int(r[1]) == 3000
    r = _run(exe, 4, 64, 2000, 20000, 123)
    assert r[0] == "gaveup" and int(r[1]) == 123 and int(r[2]) == 4
