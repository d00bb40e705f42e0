"""The host runtime of libqkc (blob parser, derived plans, argument checks)
built with the host compiler's address and undefined-behaviour sanitizers
against host-only stand-ins for the kernels, and fuzzed with mutated blobs
(truncations, bit flips, header fields and words set to edge values, random
byte runs): every case must come back as a status -- AC_ERR_FORMAT, or the
device error of this GPU-less build when the mutation leaves a well-formed
blob -- with no sanitizer report.  Also the CPU evaluator's parser."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_2103_17226_amd.blob import to_blob
from paper_2103_17226_amd.compiler import compile_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_17226_amd", "csrc")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _blobs():
    from tests.test_zz_no_alloc import _wide_sum_graph
    circs = [W.config(2, small=True)["circuit"], W.config(1, small=True)["circuit"], W.random_circuit(7),
             W.random_circuit(11), W.qaoa_maxcut(4, W.ring_graph(4), 2, dep=0.02, ad=0.01)]
    out = [to_blob(compile_circuit(c)) for c in circs]
    out.append(to_blob(_wide_sum_graph(50)))
    from paper_2103_17226_amd.dnnf import compile_circuit_dpll
    out.append(to_blob(compile_circuit_dpll(W.random_circuit(1), mpe=True)))   # the MPE plan's checks
    return out


@pytest.fixture(scope="module")
def fuzzer(tmp_path_factory):
    if not shutil.which("g++") or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("needs g++ and the HIP host runtime")
    d = tmp_path_factory.mktemp("fuzz")
    exe = str(d / "fuzz_load")
    cmd = ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                                         "-I", CSRC, os.path.join(CSRC, "qkc_host.cpp"),
                                         os.path.join(ROOT, "tests", "fuzz", "device_stub.cpp"),
                                         os.path.join(ROOT, "tests", "fuzz", "fuzz_load.cpp"),
                                         "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return d, exe


def test_mutated_blobs_are_refused_without_sanitizer_reports(fuzzer):
    d, exe = fuzzer
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for i, blob in enumerate(_blobs()):
        path = d / f"blob{i}.bin"
        path.write_bytes(blob)
        r = subprocess.run([exe, str(path), "1500", str(100 + i)], capture_output=True, text=True, timeout=600,
                           env=env)
        report = (r.stdout + r.stderr)[-3000:]
        assert r.returncode == 0, report
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
        counts = dict(zip(r.stdout.split()[0::2], map(int, r.stdout.split()[1::2])))
        assert counts["other"] == 0 and counts["format"] > 0, r.stdout


def test_cpu_evaluator_parser_refuses_mutated_blobs():
    from paper_2103_17226_amd import cpu_eval
    rng = np.random.default_rng(3)
    blob = to_blob(compile_circuit(W.config(2, small=True)["circuit"]))
    refused = 0
    for _ in range(400):
        b = bytearray(blob)
        if rng.random() < 0.5:
            b = b[:int(rng.integers(0, len(b)))]
        else:
            for _ in range(int(rng.integers(1, 6))):
                b[int(rng.integers(0, len(b)))] ^= 1 << int(rng.integers(0, 8))
        try:
            cpu_eval.CpuAC(bytes(b)).close()
        except RuntimeError:
            refused += 1
    assert refused > 100
