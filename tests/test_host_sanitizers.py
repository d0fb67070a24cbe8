"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the serving scheduler (the library's own header, driven by the simulated
executor of tests/serve_sim.cpp) and the oracle, each built with g++/gcc
into a small program that exercises it; any sanitizer report fails the
test.  (GPU code is not built here: these flags apply to host code only.)"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2508_05797_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
       "-fno-sanitize-recover=all"]

SERVE_MAIN = r"""
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>
extern "C" int sim_run(uint32_t n, const double* arrival, const uint64_t* cost,
                       const uint8_t* valid, uint64_t budget, uint32_t max_batch,
                       uint32_t slots, double base, double per_byte,
                       double* latency, int8_t* outcome, double* launch_t,
                       int32_t* slot_of, int32_t* batch_of, double* done_t,
                       uint64_t* stats);
int main() {
    std::mt19937_64 rng(7);
    for (int scen = 0; scen < 24; scen++) {
        const uint32_t n = 1 + (uint32_t)(rng() % 5000);
        std::vector<double> arr(n), lat(n), lt(n), dn(n);
        std::vector<uint64_t> cost(n);
        std::vector<uint8_t> valid(n);
        std::vector<int8_t> out(n);
        std::vector<int32_t> sl(n), bt(n);
        std::exponential_distribution<double> gap(1000.0 * (1 + scen % 5));
        double t = 0;
        for (uint32_t i = 0; i < n; i++) {
            t += gap(rng);
            arr[i] = t;
            cost[i] = 1 + rng() % (1u << (10 + scen % 12));
            valid[i] = (rng() % 50) != 0;
        }
        uint64_t stats[5] = {0, 0, 0, 0, 0};
        const uint64_t budget = 1ull << (12 + scen % 14);
        const int rc = sim_run(n, arr.data(), cost.data(), valid.data(), budget,
                               1 + scen % 64, 1 + scen % 5, 1e-5, 1e-9, lat.data(),
                               out.data(), lt.data(), sl.data(), bt.data(), dn.data(),
                               stats);
        if (rc != 0) { std::printf("scenario %d: rc %d\n", scen, rc); return 1; }
    }
    std::printf("ok\n");
    return 0;
}
"""

ORACLE_MAIN = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int64_t oracle_chunk(int algo, const uint8_t* x, uint64_t n, uint64_t w,
                     uint64_t M, uint64_t* cuts, uint64_t cap);
int main(void) {
    srand(11);
    for (int it = 0; it < 400; it++) {
        const uint64_t n = (uint64_t)(rand() % (it < 100 ? 40 : 200000));
        /* exactly n bytes on the heap, so a read past the end is reported */
        uint8_t* x = (uint8_t*)malloc(n ? n : 1);
        const int kind = it % 4;
        for (uint64_t i = 0; i < n; i++)
            x[i] = kind == 0 ? (uint8_t)rand() : kind == 1 ? (uint8_t)(i / 4096)
                 : kind == 2 ? 7 : (uint8_t)(i % 251);
        const uint64_t w = 1 + (uint64_t)(rand() % 5000);
        const uint64_t M = w + 1 + (uint64_t)(rand() % 70000);
        const uint64_t cap = n + 2;                /* a chunk holds at least one byte */
        uint64_t* cuts = (uint64_t*)malloc(cap * sizeof(uint64_t));
        for (int algo = 0; algo < 4; algo++) {
            const int64_t k = oracle_chunk(algo, x, n, w, M, cuts, cap);
            if (k < 0) { printf("oracle failed: %d %lld\n", algo, (long long)k); return 1; }
            if (k > 0 && cuts[k - 1] != n) { printf("last cut\n"); return 1; }
        }
        free(cuts);
        free(x);
    }
    printf("ok\n");
    return 0;
}
"""


def build_and_run(tmp_path, name, compiler, sources, extra):
    exe = str(tmp_path / name)
    cmd = [compiler, "-O1", "-g", *SAN, *extra, *sources, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    report = r.stdout + r.stderr
    assert r.returncode == 0 and "ok" in r.stdout, report[-3000:]
    assert "runtime error" not in report and "Sanitizer" not in report, report[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_serve_scheduler_sanitized(tmp_path):
    main = tmp_path / "serve_main.cpp"
    main.write_text(SERVE_MAIN)
    build_and_run(tmp_path, "serve_san", "g++",
                  [str(main), os.path.join(HERE, "serve_sim.cpp")],
                  ["-std=c++17", "-I", CSRC])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_sanitized(tmp_path):
    main = tmp_path / "oracle_main.c"
    main.write_text(ORACLE_MAIN)
    build_and_run(tmp_path, "oracle_san", "gcc",
                  [str(main), os.path.join(ROOT, "oracle", "cdc_oracle.c")],
                  ["-std=c11"])
