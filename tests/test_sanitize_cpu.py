"""The planner and the C ABI built with the host compiler under
AddressSanitizer and UndefinedBehaviorSanitizer (kernel launches replaced by
stand-ins that a host-only context never reaches), driven through planning,
plan validation, tuning changes, memory budgets (shared-area admission and
recomputation), the cost model and argument checks on small random 3-regular
graphs, the 100-vertex p = 4 workload and two amplitude networks.  Any
sanitizer report or unexpected status fails the test."""
import os
import shutil
import subprocess

import pytest

from workloads import random_regular_graph, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_15740_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _graph_line(kind, n, p, edges):
    return f"{kind} {n} {p} {len(edges)} " + " ".join(f"{a} {b}" for a, b in edges)


@pytest.mark.timeout(900)
def test_planner_and_abi_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are missing")
    srcs = [os.path.join(HERE, "abi_driver.cpp"), os.path.join(HERE, "kernel_stubs.cpp"),
            os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "api.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
    procs = [subprocess.Popen([gxx, *flags, "-c", s, "-o", str(tmp_path / (os.path.basename(s) + ".o"))],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True) for s in srcs]
    for pr in procs:
        out, _ = pr.communicate()
        assert pr.returncode == 0, out
    exe = str(tmp_path / "abi_driver")
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    link = [gxx, "-fsanitize=address,undefined", "-static-libasan", "-static-libubsan", *objs, f"-L{ROCM}/lib",
            "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-lpthread", "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [_graph_line("qaoa", n, p, random_regular_graph(n, 3, seed))
             for n, p, seed in ((8, 1, 0), (12, 2, 1), (16, 3, 2), (40, 3, 3))]
    w = workload("p4_n100")
    lines.append(_graph_line("qaoa64", w.n, w.p, w.edges))
    lines += [_graph_line("amp", n, p, random_regular_graph(n, 3, seed)) for n, p, seed in ((10, 2, 4), (16, 2, 5))]
    graphs = tmp_path / "graphs.txt"
    graphs.write_text("\n".join(lines) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(graphs)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "0 unexpected results" in r.stdout
