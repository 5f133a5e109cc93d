"""The CPU oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer: every entry
point over flat walls, a curved obstacle, open inlet/outlet columns, both wetting schemes, the
surface-energy rule and degenerate lattices (one fluid row, all solid, 1 x 1, a 2-column open
channel).  Any sanitizer report aborts the driver with a non-zero status."""
import subprocess

import pytest

import oracle


def test_oracle_is_clean_under_address_and_ub_sanitizers(tmp_path):
    try:
        exe = oracle.build_sanitize_check(str(tmp_path / "sanitize_check"))
    except (subprocess.CalledProcessError, FileNotFoundError) as e:
        pytest.skip(f"gcc with sanitizer runtimes is not available: {e}")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer check passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
