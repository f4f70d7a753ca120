"""Host check of the Step-3 work mapping (csrc/tile_map.hpp): for every
region shape tried, linear work index -> tile is a bijection onto the region
and stays in bounds, and the per-XCD remap of workgroup ids visits every
index once.  The header is compiled with g++ for the host."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2605_13209_amd", "csrc")

HARNESS = r'''
#include "tile_map.hpp"
#include <cstdio>
#include <vector>
using namespace chol;
static int fail(const char* what, long a, long b, long c) {
  std::printf("FAIL %s %ld %ld %ld\n", what, a, b, c); return 1;
}
int main() {
  // triangle regions
  for (long R = 1; R <= 300; R += (R < 40 ? 1 : 37)) {
    for (long S : {1L, 2L, 3L, 4L, 8L, 16L}) {
      const long G = triangle_count(R);
      std::vector<char> seen(R * R, 0);
      for (long t = 0; t < G; ++t) {
        int64_t ir, kr;
        map_triangle(t, R, S, ir, kr);
        if (ir < 0 || ir >= R || kr < 0 || kr > ir) return fail("tri-bounds", R, S, t);
        if (seen[ir * R + kr]++) return fail("tri-dup", R, S, t);
      }
    }
  }
  // a large one (N = 1024 tiles), spot-checked by sum
  {
    const long R = 1024, S = 8, G = triangle_count(R);
    long long sumi = 0, sumk = 0;
    for (long t = 0; t < G; ++t) {
      int64_t ir, kr;
      map_triangle(t, R, S, ir, kr);
      if (ir < 0 || ir >= R || kr < 0 || kr > ir) return fail("tri-big", R, S, t);
      sumi += ir; sumk += kr;
    }
    long long ei = 0, ek = 0;
    for (long i = 0; i < R; ++i) for (long k = 0; k <= i; ++k) { ei += i; ek += k; }
    if (sumi != ei || sumk != ek) return fail("tri-big-sum", R, S, 0);
  }
  // band regions
  for (long R = 1; R <= 200; R += 3) {
    for (long K = 1; K <= 8 && K <= R; ++K) {
      const long G = band_count(R, K);
      std::vector<char> seen(R * K, 0);
      for (long t = 0; t < G; ++t) {
        int64_t ir, kr;
        map_band(t, K, ir, kr);
        if (ir < 0 || ir >= R || kr < 0 || kr >= K || kr > ir) return fail("band-bounds", R, K, t);
        if (seen[ir * K + kr]++) return fail("band-dup", R, K, t);
      }
      long cnt = 0;
      for (char c : seen) cnt += c;
      if (cnt != G) return fail("band-count", R, K, cnt);
    }
  }
  // per-XCD remap: grid 8*ceil(G/8), t = (bid % 8) * G8 + bid / 8, t < G kept
  for (long G = 1; G <= 1000; ++G) {
    const long G8 = (G + 7) / 8;
    std::vector<char> seen(G, 0);
    for (long bid = 0; bid < 8 * G8; ++bid) {
      const long t = (bid % 8) * G8 + bid / 8;
      if (t >= 8 * G8) return fail("xcd-range", G, bid, t);
      if (t < G && seen[t]++) return fail("xcd-dup", G, bid, t);
    }
    for (long t = 0; t < G; ++t) if (!seen[t]) return fail("xcd-miss", G, t, 0);
  }
  std::printf("OK\n");
  return 0;
}
'''


def test_tile_map_bijection():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "h.cpp")
        exe = os.path.join(d, "h")
        open(src, "w").write(HARNESS)
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", HDR, src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
