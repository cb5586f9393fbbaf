"""Host threads of the planner (csrc/parallel.hpp): parallel_sort gives the
order std::sort gives for a strict total order, parallel_for visits every
index once, and an exception thrown in a worker reaches the caller (the C ABI
turns it into a status instead of terminating the process).  Compiled with g++
into a temporary folder; no GPU."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2003_01836_amd", "csrc")

PROGRAM = r"""
#include "parallel.hpp"
#include <cstdio>
#include <random>
#include <stdexcept>
struct Rec { long long key; int a, b; };
int main()
{
    for (long long n : {0LL, 1LL, 1000LL, 65535LL, 65536LL, 300001LL}) {
        std::vector<Rec> v(n);
        std::mt19937_64 g(n + 7);
        for (long long i = 0; i < n; ++i)
            v[i] = Rec{static_cast<long long>(g() % 1000), static_cast<int>(g() % 50),
                       static_cast<int>(i)};
        auto cmp = [](const Rec& x, const Rec& y) {
            if (x.key != y.key) return x.key > y.key;
            return x.a != y.a ? x.a < y.a : x.b < y.b;
        };
        std::vector<Rec> w = v;
        std::sort(w.begin(), w.end(), cmp);
        bltc::parallel_sort(v.begin(), v.end(), cmp);
        for (long long i = 0; i < n; ++i)
            if (v[i].key != w[i].key || v[i].a != w[i].a || v[i].b != w[i].b) {
                std::printf("sort mismatch n=%lld i=%lld\n", n, i);
                return 1;
            }
    }
    std::vector<std::atomic<int>> seen(100000);
    bltc::parallel_for(100000, [&](int64_t i) { seen[i] += 1; });
    for (auto& s : seen)
        if (s != 1) { std::printf("parallel_for visit count\n"); return 1; }
    bool caught = false;
    try {
        bltc::parallel_for(100000, [&](int64_t i) {
            if (i == 77777) throw std::runtime_error("worker failure");
        });
    } catch (const std::runtime_error&) {
        caught = true;
    }
    if (!caught) { std::printf("exception lost\n"); return 1; }
    caught = false;
    try {
        bltc::parallel_each(5, [&](int64_t i) { if (i == 3) throw std::bad_alloc(); });
    } catch (const std::bad_alloc&) {
        caught = true;
    }
    if (!caught) { std::printf("bad_alloc lost\n"); return 1; }
    std::printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_parallel_helpers(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I" + CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
