"""The record transport's host agent against CPU threads that play the GPU
waves (same request/completion structs and atomics), built with
ThreadSanitizer: data staged correctly, completions in order, injected
stragglers and failed reads handled per query, agent re-armable."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _build(tmp_path, sanitize):
    exe = tmp_path / ("agent_test_" + sanitize)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=" + sanitize,
           os.path.join(HERE, "agent_protocol_test.cpp"),
           os.path.join(ROOT, "paper_2507_10070_amd", "csrc", "agent.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    return str(exe)


def test_agent_protocol_tsan(tmp_path):
    exe = _build(tmp_path, "thread")
    r = subprocess.run([exe, "48", "3"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr


def test_agent_protocol_asan(tmp_path):
    exe = _build(tmp_path, "address")
    r = subprocess.run([exe, "64", "4"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_agent_protocol_sequence_wrap(tmp_path):
    """Lines that outlive their queries (server waves) run their request
    numbers past the wrap point; the agent follows them across it."""
    exe = _build(tmp_path, "address")
    r = subprocess.run([exe, "32", "3", "wrap"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_agent_file_async_reads(tmp_path):
    """Records in a file read with O_DIRECT through Linux asynchronous I/O:
    every staged record and completion right, faults per request."""
    exe = _build(tmp_path, "address")
    r = subprocess.run([exe, "48", "3", "file", str(tmp_path)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    print(r.stdout)


def test_agent_striped_files_tsan(tmp_path):
    """Three striped record files (record v in file v % 3), served by agent
    threads under ThreadSanitizer; every stripe serves its share."""
    exe = _build(tmp_path, "thread")
    r = subprocess.run([exe, "40", "2", "stripes", str(tmp_path)], capture_output=True,
                       text=True, timeout=300, env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr
