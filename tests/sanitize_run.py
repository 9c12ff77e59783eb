"""Runs CPU test files against sanitizer builds of the oracle and of the
library's host code (used by tests/test_sanitizers.py in a child process
started with the AddressSanitizer runtime preloaded).

    python tests/sanitize_run.py <liboracle> <libibdvm> <test file> ...
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

if __name__ == "__main__":
    import pytest

    from oracle import oracle as O
    from paper_2512_20252_amd import ibdvm as I

    O.LIB_PATH, I.LIB_PATH = sys.argv[1], sys.argv[2]
    files = [os.path.join(ROOT, f) for f in sys.argv[3:]]
    sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"] + files))
