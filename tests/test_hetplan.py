"""Host logic of the heterodyned time marginal's work split (csrc/gw_hetplan.h).

The plan cuts the edges into chunks of about equal cost; a frequency block
cut by several chunks gets one piece per chunk, summed in chunk order.  The
driver below builds plans for random block layouts (edges crowded into the
lowest blocks as for bins of equal phase change, uniform, or all in one
block) and checks, by simulating the moment kernel and the fix-up on
per-edge values, that every edge is summed exactly once, every block gets
exactly the sum of its edges, the pieces' slots are distinct, and no chunk
exceeds its share of the cost by more than a few units.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2607_28265_amd", "csrc")

DRIVER = r"""
#include "gw_hetplan.h"
#include <cmath>
#include <cstdio>
#include <random>
using namespace gw;
int main() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  int failures = 0;
  for (int trial = 0; trial < 5000; ++trial) {
    const int n_blk = 1 + (int)(rng() % 200), ne = 1 + (int)(rng() % 600), mode = (int)(rng() % 3);
    std::vector<int> cnt(n_blk, 0);
    for (int e = 0; e < ne; ++e) {
      const double u = U(rng);
      const int b = mode == 0 ? (int)(n_blk * u * u * u) : (mode == 1 ? (int)(n_blk * u) : 0);
      cnt[b < n_blk ? b : n_blk - 1]++;
    }
    std::vector<int32_t> bs(n_blk + 1, 0);
    for (int b = 0; b < n_blk; ++b) bs[b + 1] = bs[b] + cnt[b];
    const int want = 1 + (int)(rng() % 300);
    const HetTmPlan p = het_tm_plan(bs, n_blk, ne, want);
    const int nch = p.nch();
    bool ok = nch >= 1 && nch <= want && p.e0[0] == 0 && p.e0[nch] == ne;
    for (int c = 0; ok && c < nch; ++c)
      ok = p.e0[c] <= p.e0[c + 1] && p.blo[c] < p.bhi[c] && p.e0[c] >= bs[p.blo[c]];
    std::vector<double> mom(n_blk, -1.0), slot(p.nslot, -7.0);
    std::vector<int> seen(ne, 0);
    for (int c = 0; ok && c < nch; ++c) {
      int e = p.e0[c];
      for (int b = p.blo[c]; b < p.bhi[c]; ++b) {
        const int be = bs[b + 1] < p.e0[c + 1] ? bs[b + 1] : p.e0[c + 1];
        double s = 0.0;
        for (; e < be; ++e) { seen[e]++; s += std::sqrt(e + 1.0); }
        const int sl = b == p.bhi[c] - 1 ? p.slast[c] : (b == p.blo[c] ? p.sfirst[c] : -1);
        if (sl < 0) { ok = ok && mom[b] == -1.0; mom[b] = s; }
        else { ok = ok && sl < p.nslot && slot[sl] == -7.0; if (sl < p.nslot) slot[sl] = s; }
      }
      ok = ok && e == p.e0[c + 1];
    }
    for (size_t i = 0; ok && i < p.fb.size(); ++i) {
      const int b = p.fb[i];
      ok = mom[b] == -1.0;
      double s = 0.0;
      for (int k = 0; k < p.fc[i]; ++k) { ok = ok && slot[p.fs[i] + k] != -7.0; s += slot[p.fs[i] + k]; }
      mom[b] = s;
    }
    for (int e = 0; ok && e < ne; ++e) ok = seen[e] == 1;
    for (int b = 0; ok && b < n_blk; ++b) {
      double s = 0.0;
      for (int e = bs[b]; e < bs[b + 1]; ++e) s += std::sqrt(e + 1.0);
      ok = mom[b] != -1.0 && std::fabs(mom[b] - s) <= 1e-9 * (1.0 + s);
    }
    const double per = (double)(ne + n_blk) / want;
    for (int c = 0; ok && c < nch; ++c) ok = (p.e0[c + 1] - p.e0[c]) + (p.bhi[c] - p.blo[c]) <= per + 3.0;
    if (!ok) {
      if (failures < 5) std::printf("failed: ne %d n_blk %d want %d nch %d\n", ne, n_blk, want, nch);
      ++failures;
    }
  }
  std::printf("%d failures\n", failures);
  return failures != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_het_time_marginal_plan(tmp_path):
    src = tmp_path / "plan_check.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "plan_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
