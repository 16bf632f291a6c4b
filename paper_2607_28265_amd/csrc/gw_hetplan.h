// Work split of the heterodyned time marginal's edge-weight moments (host
// only).  The edges lie in n_blk frequency blocks (block b holds edges
// [bs[b], bs[b + 1])); a block's moment needs all of its edges, and a chunk
// costs one unit per edge plus one per block it emits.  Edges of equal phase
// change crowd into the lowest blocks (hundreds of edges in the first), so
// chunks are edge ranges of about equal cost that may cut a block: a block
// cut by several chunks gets one partial moment per chunk (a "piece" with a
// slot of its own), and a fix-up pass adds a block's pieces in chunk order.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace gw {

struct HetTmPlan {
  std::vector<int32_t> e0;       // [nch + 1] first edge of each chunk (nondecreasing), then n_edges
  std::vector<int32_t> blo, bhi;  // [nch] the chunk emits blocks [blo, bhi)
  std::vector<int32_t> sfirst, slast;  // [nch] piece slot of the first / last emitted block, -1 if whole
  std::vector<int32_t> fb, fs, fc;     // per cut block: block, first slot, pieces (chunk order)
  int nslot = 0;
  int nch() const { return (int)e0.size() - 1; }
};

// Chunks for at most want_nch of about (ne + n_blk) / want_nch units each;
// ne >= 1 edges, bs[0] = 0, bs[n_blk] = ne, nondecreasing.  The units are
// walked in order (block b's edges, then its end) and a chunk closes once the
// running cost reaches its share; a chunk that closes after an edge cuts
// that edge's block.
inline HetTmPlan het_tm_plan(const std::vector<int32_t>& bs, int n_blk, int ne, int want_nch) {
  HetTmPlan p;
  const int nch_max = std::max(1, want_nch);
  const double per = (double)(ne + n_blk) / nch_max;
  std::vector<int32_t> c0(n_blk), c1(n_blk), base(n_blk, -1);
  std::vector<char> mid(1, 0);  // chunk c starts inside a block
  p.e0.push_back(0);
  p.blo.push_back(0);
  double cost = 0.0;
  auto close = [&]() { return (int)p.e0.size() < nch_max && cost >= per * (double)p.e0.size(); };
  for (int b = 0; b < n_blk; ++b) {
    c0[b] = (int)p.e0.size() - 1;
    for (int e = bs[b]; e < bs[b + 1]; ++e) {
      cost += 1.0;
      if (close()) {  // the next chunk starts at edge e + 1, inside block b
        p.e0.push_back(e + 1);
        p.blo.push_back(b);
        mid.push_back(1);
      }
    }
    cost += 1.0;  // the block's moment stores
    c1[b] = (int)p.e0.size() - 1;
    if (b + 1 < n_blk && close()) {
      p.e0.push_back(bs[b + 1]);
      p.blo.push_back(b + 1);
      mid.push_back(0);
    }
  }
  p.e0.push_back(ne);
  const int nch = p.nch();
  p.bhi.resize(nch);
  for (int c = 0; c < nch; ++c) p.bhi[c] = c + 1 < nch ? p.blo[c + 1] + (mid[c + 1] ? 1 : 0) : n_blk;
  for (int b = 0; b < n_blk; ++b)
    if (c1[b] > c0[b]) {
      base[b] = p.nslot;
      p.fb.push_back(b);
      p.fs.push_back(p.nslot);
      p.fc.push_back(c1[b] - c0[b] + 1);
      p.nslot += c1[b] - c0[b] + 1;
    }
  p.sfirst.assign(nch, -1);
  p.slast.assign(nch, -1);
  for (int c = 0; c < nch; ++c) {
    const int bf = p.blo[c], bl = p.bhi[c] - 1;
    if (base[bf] >= 0) p.sfirst[c] = base[bf] + (c - c0[bf]);
    if (base[bl] >= 0) p.slast[c] = base[bl] + (c - c0[bl]);
  }
  return p;
}

}  // namespace gw
