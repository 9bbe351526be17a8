"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc) runs every entry point on seeded matrices and malformed inputs
without a report (tests/oracle_sanitize_driver.c); a planted out-of-bounds
write in a copy of the oracle is reported, which shows the sanitizers are
active in this build."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _build_and_run(tmp_path, src):
    exe = tmp_path / "osan"
    subprocess.check_call(["gcc", *FLAGS, str(src), "-o", str(exe), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_clean_under_sanitizers(tmp_path):
    r = _build_and_run(tmp_path, os.path.join(HERE, "oracle_sanitize_driver.c"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "OK"


def test_planted_overflow_is_reported(tmp_path):
    """The level pass reading one past the end of its own fill array (a
    planted mistake in a copy of the oracle) makes the sanitized driver fail."""
    root = os.path.dirname(HERE)
    src = open(os.path.join(root, "oracle", "oracle.c")).read()
    bad = src.replace("for (int32_t r = 0; r < n; ++r) level_rows[fill[lev[r]]++] = r;",
                      "for (int32_t r = 0; r < n; ++r) level_rows[fill[lev[r]]++] = r;\n"
                      "  if (fill[nlev] == 0x5eed) level_ptr[0] = 1;")
    assert bad != src
    (tmp_path / "oracle").mkdir()
    (tmp_path / "oracle" / "oracle.c").write_text(bad)
    (tmp_path / "tests").mkdir()
    drv = tmp_path / "tests" / "oracle_sanitize_driver.c"
    drv.write_text(open(os.path.join(HERE, "oracle_sanitize_driver.c")).read())
    r = _build_and_run(tmp_path, drv)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr
