"""The oracle's C part (binary128 Newell tensor, compensated direct demag sum)
built once with AddressSanitizer and UndefinedBehaviorSanitizer (no OpenMP,
so the loops run serially) and run on a small grid whose far radius puts
offsets on both sides of the near/far switch: no sanitizer report, and the
same tensor and field as the regular build to rounding."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_c_under_asan_ubsan(tmp_path):
    n, d, P = (7, 6, 4), (2.5e-9, 2.0e-9, 3e-9), 2.0
    exe = tmp_path / "oracle_san"
    srcs = [os.path.join(ROOT, "oracle", "newell_q.c"), os.path.join(ROOT, "oracle", "direct_sum.c"),
            os.path.join(HERE, "oracle_sanitize_main.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] + srcs +
                          ["-o", str(exe), "-lquadmath", "-lm"])
    m = synth.random_unit(n, 3)
    cells = np.array([[0, 0, 0], [3, 2, 1], [6, 5, 3]], dtype=np.int64)
    (tmp_path / "m.bin").write_bytes(np.ascontiguousarray(m, dtype=np.float64).tobytes())
    (tmp_path / "cells.bin").write_bytes(cells.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)] + [str(v) for v in n] + [repr(v) for v in d] + [repr(P), str(tmp_path / "m.bin"),
                        str(tmp_path / "cells.bin"), str(len(cells)), str(tmp_path / "oct.bin"),
                        str(tmp_path / "h.bin")], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    oct_san = np.frombuffer((tmp_path / "oct.bin").read_bytes(), dtype=np.float64).reshape(n + (6,))
    h_san = np.frombuffer((tmp_path / "h.bin").read_bytes(), dtype=np.float64).reshape(len(cells), 3)
    oct_ref = oracle.tensor_octant(n, d, P=P)
    assert np.max(np.abs(oct_san - oct_ref)) <= 1e-15 * np.max(np.abs(oct_ref))
    h_ref = oracle.demag_direct_at(m, 1.0, oct_ref, [tuple(c) for c in cells])
    assert np.max(np.abs(h_san - h_ref)) <= 1e-13 * np.max(np.abs(h_ref))
