"""The serving pool's first-fit allocator (csrc/dtw_pool.h), on the host."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_02734_amd", "csrc")

PROGRAM = r'''
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>
#include "dtw_pool.h"
using dtw::PoolAllocator;
int main() {
  PoolAllocator a(1 << 20);
  assert(a.size() == (1u << 20) && a.free_bytes() == (1u << 20));
  size_t x = a.alloc(1000), y = a.alloc(256), z = a.alloc(1);
  assert(x == 0 && y == 1024 && z == 1280);  // 256-byte granules, first fit
  assert(a.alloc((1 << 20)) == SIZE_MAX);    // too large
  assert(a.release(y) && !a.release(y));     // double release refused
  assert(a.alloc(200) == 1024);              // the hole is reused
  assert(a.release(x) && a.release(1024) && a.release(z));
  assert(a.free_bytes() == (1u << 20) && a.largest_free() == (1u << 20) && a.n_used() == 0);  // merged back
  // random alloc/free: blocks never overlap, everything merges back at the end
  std::mt19937 rng(7);
  std::vector<std::pair<size_t, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3) {
      const size_t n = 1 + rng() % 20000;
      const size_t off = a.alloc(n);
      if (off == SIZE_MAX) { assert(a.largest_free() < PoolAllocator::round_up(n)); continue; }
      assert(off % 256 == 0 && off + n <= a.size());
      for (auto& p : live) assert(off + n <= p.first || p.first + p.second <= off);
      live.push_back({off, n});
    } else {
      const size_t i = rng() % live.size();
      assert(a.release(live[i].first));
      live.erase(live.begin() + i);
    }
  }
  for (auto& p : live) assert(a.release(p.first));
  assert(a.free_bytes() == a.size() && a.largest_free() == a.size());
  std::puts("ok");
  return 0;
}
'''


def test_pool_allocator(tmp_path):
    src = tmp_path / "pool.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "pool"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-I", CSRC, str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr
