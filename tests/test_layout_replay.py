"""CPU replay of the batched kernel's indexing over the packed layout
(tests/cpp/layout_check.cpp): every access in bounds, every panel entry read
once, every output written once, product equal to the direct block product."""
import os
import subprocess

import pytest

from paper_2110_12165_amd.build import HOST_SOURCES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_12165_amd", "csrc")


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("replay") / "layout_check")
    srcs = [os.path.join(ROOT, "tests", "cpp", "layout_check.cpp")] + [
        os.path.join(CSRC, f) for f in HOST_SOURCES]
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC] + srcs + ["-o", out]
    subprocess.run(cmd, check=True)
    return out


@pytest.mark.parametrize("args", [
    ("64", "32", "100", "90", "0", "32", "1", "1e-6"),      # planar strike-slip, normal H
    ("48", "24", "100", "30", "1", "16", "4", "1e-6"),      # lattice 4, ragged leaves
    ("37", "23", "100", "90", "0", "20", "2", "1e-5"),
    ("150", "70", "100", "30", "1", "32", "8", "1e-6"),     # lattice 8
    ("3", "2", "100", "90", "0", "1", "1", "1e-6"),         # tiny
])
def test_replay(binary, args):
    r = subprocess.run([binary, *args], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().endswith("OK")


@pytest.fixture(scope="module")
def binary_sanitized(tmp_path_factory):
    """The same replay built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only: tree, partition, ACA, packing)."""
    out = str(tmp_path_factory.mktemp("replay_asan") / "layout_check")
    srcs = [os.path.join(ROOT, "tests", "cpp", "layout_check.cpp")] + [
        os.path.join(CSRC, f) for f in HOST_SOURCES]
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC] + srcs + ["-o", out]
    subprocess.run(cmd, check=True)
    return out


@pytest.mark.parametrize("args", [
    ("48", "24", "100", "30", "1", "16", "4", "1e-6"),
    ("37", "23", "100", "90", "0", "20", "2", "1e-5"),
    ("3", "2", "100", "90", "0", "1", "1", "1e-6"),
])
def test_replay_sanitized(binary_sanitized, args):
    r = subprocess.run([binary_sanitized, *args], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().endswith("OK")
