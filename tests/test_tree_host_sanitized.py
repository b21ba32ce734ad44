"""The host tree builder's index arithmetic under the host sanitizers: the
builder (plain C++) and tests/tree_host_check.cpp are compiled with g++
-fsanitize=address,undefined and run on seeded point sets; every invariant of
the boxes and pair lists (permutation, sorted keys, children partitioning
their parent, key prefixes, list order, admissibility, completeness of the
free and image lists) must hold with no sanitizer report."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_09136_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tree_host_builder_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tree_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-I", CSRC, os.path.join(ROOT, "tests", "tree_host_check.cpp"), os.path.join(CSRC, "tree_host.cpp"),
               "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        print(r.stdout[-2000:], r.stderr[-2000:])
        assert r.returncode == 0
        assert "all tree checks passed" in r.stdout
