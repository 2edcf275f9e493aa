"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only) runs a
small scene with every noise knob, both precisions, the neural-SDF oracle and the thermal solver
without a report (tests/oracle_sanitize_main.c)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    srcs = [os.path.join(ROOT, "tests", "oracle_sanitize_main.c")] + [
        os.path.join(ROOT, "oracle", f) for f in ("oracle.c", "nsdf.c", "thermal.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized oracle run ok" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("which,extra", [("SAN_PROX", ("oracle.c", "nsdf.c")), ("SAN_ELAST", ()), ("SAN_RAY", ())])
def test_sensor_oracles_under_address_and_undefined_sanitizers(tmp_path, which, extra):
    """The ProximityTaxel, ElastomerTaxel and raycast oracles on a small scene with an env without
    an object, an object id out of range, an empty link and a zero-radius probe
    (tests/oracle_sanitize_sensors.c), each built with both sanitizers."""
    exe = str(tmp_path / ("sensor_" + which))
    srcs = [os.path.join(ROOT, "tests", "oracle_sanitize_sensors.c")] + [os.path.join(ROOT, "oracle", f) for f in extra]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D" + which, "-o", exe] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized sensor oracle run ok" in r.stdout
