"""Host side of the streaming pipeline (Sec. 4.2, Fig. 1), no GPU needed:
the batch planner exported by the library against a direct restatement of
its rule, its argument checks, and a thread-sanitised stress run of the
loader/consumer ring (tests/native/stream_engine_check.cpp)."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1906_08556_amd import ivx

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1906_08556_amd", "csrc")


def _reference_plan(off, max_utts, max_frames):
    """Consecutive utterances go into a batch until one more would exceed
    either limit."""
    U = len(off) - 1
    starts, u = [], 0
    while u < U:
        starts.append(u)
        u0 = u
        while u < U and u - u0 < max_utts and off[u + 1] - off[u0] <= max_frames:
            u += 1
    return np.array(starts + [U], dtype=np.int64)


def test_plan_matches_the_rule_on_random_lengths():
    rng = np.random.default_rng(0)
    for _ in range(300):
        U = int(rng.integers(0, 80))
        mf = int(rng.integers(1, 500))
        mu = int(rng.integers(1, 12))
        lens = rng.integers(0, mf + 1, size=U)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        np.testing.assert_array_equal(ivx.plan_batches(off, mu, mf), _reference_plan(off, mu, mf))


def test_plan_edge_cases():
    assert ivx.plan_batches(np.zeros(1, np.int64), 4, 10).tolist() == [0]
    off = np.array([0, 10, 10, 10, 20], np.int64)        # an utterance exactly at the limit
    assert ivx.plan_batches(off, 8, 10).tolist() == [0, 3, 4]
    assert ivx.plan_batches(off, 1, 10).tolist() == [0, 1, 2, 3, 4]
    with pytest.raises(ivx.IvxError):
        ivx.plan_batches(np.array([0, 5, 17], np.int64), 4, 10)  # 12 frames > 10
    with pytest.raises(ivx.IvxError):
        ivx.plan_batches(np.array([0, 5, 3], np.int64), 4, 10)   # decreasing offsets
    with pytest.raises(ivx.IvxError):
        ivx.plan_batches(np.array([1, 5], np.int64), 4, 10)      # utt_off[0] != 0
    with pytest.raises(ivx.IvxError):
        ivx.plan_batches(off, 0, 10)


def test_plan_reports_the_needed_capacity():
    lib = ivx.load()
    off = np.array([0, 3, 6, 9, 12], np.int64)
    starts = np.zeros(2, np.int64)
    nb = ctypes.c_int64()
    st = lib.ivx_plan_batches(ctypes.c_void_p(off.ctypes.data), 4, 1, 100,
                              ctypes.c_void_p(starts.ctypes.data), 2, ctypes.byref(nb))
    assert st == -1 and nb.value == 4


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_ring_stress_under_thread_sanitizer():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sec")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                        f"-I{CSRC}", os.path.join(HERE, "native", "stream_engine_check.cpp"),
                        "-o", exe], check=True, capture_output=True, timeout=240)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0
        assert "ThreadSanitizer" not in r.stderr
        assert r.stdout.startswith("OK")
