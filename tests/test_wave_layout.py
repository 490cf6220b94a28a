"""The small-piece kernel's LDS layout (kernel_types.hpp, wave_lds_layout),
checked on the host: compiled with g++ and evaluated for many piece sizes,
every array is 16-byte aligned, inside the allocation and disjoint from the
others, each wave's slice included, and the slice is as large as its arrays."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r'''
#include <cstdio>
#include <cstdint>
#include <vector>
#include <algorithm>
#include "kernel_types.hpp"
using namespace sbc;
struct R { uint64_t a, b; };
int main() {
  const int64_t sizes[] = {1, 2, 3, 7, 63, 64, 65, 127, 255, 256, 257, 1000, 4096};
  const int64_t arcs[] = {0, 1, 6, 100, 4097, 65535};
  long checked = 0;
  for (int64_t np : sizes) for (int64_t na : arcs) for (int64_t w : {1, 4, 8}) {
    const WaveLds L = wave_lds_layout(np, na, w);
    std::vector<R> r = {{L.bc, 8 * (uint64_t)np}, {L.row, 4 * (uint64_t)(np + 1)}, {L.rch, 4 * (uint64_t)np},
                        {L.idn, 4 * (uint64_t)np}, {L.col, 2 * (uint64_t)na}};
    const uint64_t in[][2] = {{L.sig, 8 * (uint64_t)np}, {L.fsu, 8 * 64}, {L.d, 4 * (uint64_t)np}, {L.scan, 4 * 64},
                              {L.fe0, 4 * 64}, {L.q, 2 * (uint64_t)np}, {L.lvl, 2 * (uint64_t)(np + 2)}};
    for (int64_t k = 0; k < w; ++k)
      for (auto& x : in) r.push_back({L.wave0 + (uint64_t)k * L.wave_bytes + x[0], x[1]});
    for (auto& x : in) if (x[0] + x[1] > L.wave_bytes) { printf("slice overflow np=%lld\n", (long long)np); return 1; }
    for (auto& x : r) {
      if (x.a % 16 != 0) { printf("misaligned np=%lld\n", (long long)np); return 1; }
      if (x.a + x.b > L.total) { printf("outside np=%lld arcs=%lld\n", (long long)np, (long long)na); return 1; }
    }
    std::sort(r.begin(), r.end(), [](const R& p, const R& q) { return p.a < q.a; });
    for (size_t i = 1; i < r.size(); ++i)
      if (r[i - 1].b > 0 && r[i - 1].a + r[i - 1].b > r[i].a) { printf("overlap np=%lld\n", (long long)np); return 1; }
    ++checked;
  }
  printf("layouts ok %ld\n", checked);
  return 0;
}
'''


def test_wave_lds_layout(tmp_path):
    src = tmp_path / "layout.cpp"
    exe = tmp_path / "layout"
    src.write_text(SRC)
    inc = os.path.join(ROOT, "paper_1209_6007_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True)
    assert r.returncode == 0 and "layouts ok" in r.stdout, r.stdout
