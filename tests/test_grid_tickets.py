"""The grid-solve ticket pool (host logic, no GPU).  Coarsest-level solves
with software grid barriers are only safe while all their work-groups are
resident, which the library guarantees by letting at most 16 run at once per
device: a solve takes a ticket if one is free (try_acquire, falling back to
the single-work-group form otherwise) or waits for one (acquire).  Compiled
from the library's own header with g++ and driven by many threads."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_07913_amd", "csrc")

PROG = r'''
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>
#include <chrono>
#include "tickets.h"
using namespace hot;
int main() {
  // exhaustion: try_acquire succeeds exactly kGridSolves times
  {
    TicketPool p(kGridSolves);
    int got = 0;
    for (int k = 0; k < kGridSolves + 5; ++k) got += p.try_acquire() ? 1 : 0;
    if (got != kGridSolves || p.available() != 0) { std::printf("exhaust %d\n", got); return 1; }
    p.release();
    if (!p.try_acquire()) { std::printf("reuse\n"); return 2; }
  }
  // 64 threads, each taking a ticket (waiting or trying) 200 times: never more
  // than kGridSolves held at once, and every ticket comes back
  {
    TicketPool p(kGridSolves);
    std::atomic<int> held{0}, peak{0}, fallbacks{0};
    std::vector<std::thread> th;
    for (int t = 0; t < 64; ++t)
      th.emplace_back([&, t] {
        for (int k = 0; k < 200; ++k) {
          bool wait = ((t + k) % 3) == 0;
          bool ok = true;
          if (wait) p.acquire(); else ok = p.try_acquire();
          if (!ok) { fallbacks++; continue; }
          int h = ++held;
          int pk = peak.load();
          while (h > pk && !peak.compare_exchange_weak(pk, h)) {}
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          --held;
          p.release();
        }
      });
    for (auto& x : th) x.join();
    if (peak.load() > kGridSolves || peak.load() < 2) { std::printf("peak %d\n", peak.load()); return 3; }
    if (p.available() != kGridSolves) { std::printf("leak %d\n", p.available()); return 4; }
    std::printf("peak %d fallbacks %d\n", peak.load(), fallbacks.load());
  }
  return 0;
}
'''


def test_ticket_pool_bounds_concurrent_grid_solves():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        open(src, "w").write(PROG)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC, src, "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stdout
