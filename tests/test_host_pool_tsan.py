"""The host worker pool of the library (validation and staging threads) under
ThreadSanitizer: its source, taken from lf_api.cpp as it stands, is built
for the host alone with g++ -fsanitize=thread and driven by several callers
at once, many parallel sections each (every index of a section run once,
each section's first failure the serial one).  Host code only; nothing here
touches a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
API = os.path.join(ROOT, "paper_2402_14670_amd", "csrc", "lf_api.cpp")

DRIVER = r'''
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>
namespace {
%s
}
int main() {
    std::vector<std::thread> callers;
    std::atomic<int> bad{0};
    for (int c = 0; c < 6; ++c)
        callers.emplace_back([&, c] {
            for (int rep = 0; rep < 200; ++rep) {
                const size_t n = 1000 + 37 * c + rep;
                std::vector<int> runs(n, 0);
                const size_t stop = (rep * 7919 + c) %% n;
                const size_t got = first_failure(n, size_t(1) << 21, [&](size_t i) { ++runs[i]; return i != stop; });
                if (got != stop) ++bad;
                for (size_t i = 0; i < n; ++i)
                    if (runs[i] > 1) { ++bad; break; }
            }
        });
    for (auto &t : callers) t.join();
    std::printf("bad=%%d\n", bad.load());
    return bad.load() != 0;
}
'''


def test_worker_pool_under_thread_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++ on this host")
    src = open(API).read()
    a = src.index("unsigned host_threads(size_t work)")
    b = src.index("// memcpy of several (dst, src, n) pieces")
    prog = tmp_path / "pool.cpp"
    prog.write_text(DRIVER % src[a:b])
    exe = tmp_path / "pool"
    build = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", str(prog), "-o", str(exe)],
                           capture_output=True, text=True, timeout=300)
    if build.returncode != 0 and "sanitizer" in build.stderr.lower():
        pytest.skip("ThreadSanitizer is not available to g++ here")
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66"))
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-4000:]
    assert run.returncode == 0 and "bad=0" in run.stdout, (run.returncode, run.stdout, run.stderr[-2000:])
