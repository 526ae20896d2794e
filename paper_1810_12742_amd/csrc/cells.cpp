// Tables of the cell-lane solve kernel: one lane per cell, 64 cells of similar
// size per wave.  Pure C++17; no HIP.
//
// The Hines elimination (paper §2) needs only that every compartment is
// eliminated after all its children and substituted after its parent.  A
// depth-first (preorder) numbering of a cell satisfies both when the backward
// sweep runs it in reverse.  In reverse preorder the compartment eliminated
// just before p is p's first child in the order, so that child's contribution
// to p stays in registers; the other children of p finish earlier, and their
// contributions wait on a per-lane stack (all of them in one merged entry,
// since they share the target p).  Visiting last the child whose subtree needs
// the deepest stack bounds the depth by a Strahler-like number, O(log) of the
// number of tips.  The forward sweep mirrors this: x of a compartment with two
// or more children waits on the stack for its later children.
#include <algorithm>
#include <numeric>

#include "setup.hpp"

namespace hines {

namespace {

// Preorder of one cell (relative indices 0..m-1, root 0) with the deepest-
// stack child last; fills flags per relative index and returns the stack need.
int32_t cell_order(const int32_t* par, int64_t lo, int32_t m, std::vector<int32_t>& pre,
                   std::vector<uint8_t>& fl, std::vector<int32_t>& ch_off, std::vector<int32_t>& ch,
                   std::vector<int32_t>& need, std::vector<int32_t>& heavy) {
  ch_off.assign(m + 1, 0);
  for (int32_t i = 1; i < m; ++i) ch_off[par[lo + i] - lo + 1]++;
  for (int32_t i = 0; i < m; ++i) ch_off[i + 1] += ch_off[i];
  ch.resize(std::max(m - 1, 0));
  {
    std::vector<int32_t> fill(ch_off.begin(), ch_off.end() - 1);
    for (int32_t i = 1; i < m; ++i) ch[fill[par[lo + i] - lo]++] = i;  // ascending per parent
  }
  need.assign(m, 0);
  heavy.assign(m, -1);
  for (int32_t v = m - 1; v >= 0; --v) {
    int32_t b1 = -1, b2 = -1, h = -1;
    for (int32_t k = ch_off[v]; k < ch_off[v + 1]; ++k) {
      const int32_t c = ch[k], nc = need[c];
      if (nc > b1) {
        b2 = b1;
        b1 = nc;
        h = c;
      } else if (nc > b2) {
        b2 = nc;
      }
    }
    const int32_t nch = ch_off[v + 1] - ch_off[v];
    need[v] = nch == 0 ? 0 : (nch == 1 ? b1 : std::max(b1, b2 + 1));
    heavy[v] = h;
  }
  // preorder: light children in ascending index, the heavy child last
  pre.clear();
  fl.assign(m, 0);
  std::vector<int32_t> st;
  st.push_back(0);
  while (!st.empty()) {
    const int32_t v = st.back();
    st.pop_back();
    pre.push_back(v);
    const int32_t b = ch_off[v], e = ch_off[v + 1], nch = e - b;
    uint8_t f = 0;
    if (nch == 0) f |= CF_TIP;
    if (nch >= 2) f |= CF_POP;
    if (v == 0) f |= CF_ROOT;
    fl[v] |= f;
    if (nch == 0) continue;
    const int32_t h = heavy[v];
    st.push_back(h);
    // the light children, popped in ascending order
    for (int32_t k = e - 1; k >= b; --k)
      if (ch[k] != h) st.push_back(ch[k]);
    if (nch >= 2) {
      fl[h] |= CF_PUSH;
      bool first = true;
      for (int32_t k = b; k < e; ++k) {
        if (ch[k] == h) continue;
        if (first) first = false;  // the first light child carries in registers
        else fl[ch[k]] |= CF_MERGE;
      }
    }
  }
  return m > 0 ? need[0] : 0;
}

}  // namespace

Status build_cell_lanes(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                        CellLanes& out, std::string& err) {
  out = CellLanes{};
  std::vector<int64_t> order(ncells);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t c = 0; c < ncells; ++c) {
    const int64_t m = cell_offsets[c + 1] - cell_offsets[c];
    if (m > kCellMaxSize) {
      err = "cell " + std::to_string(c) + " has " + std::to_string(m) + " compartments; the cell-lane kernel takes " +
            std::to_string(kCellMaxSize) + " at most";
      return ERR_TOO_BIG;
    }
  }
  auto size_of = [&](int64_t c) { return cell_offsets[c + 1] - cell_offsets[c]; };
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return size_of(a) > size_of(b); });
  const int64_t nw = (ncells + 63) / 64;
  out.nwaves = nw;
  out.waves.resize(nw);
  out.lane_cell.assign(nw * 64, -1);
  out.base.assign(nw * 64, 0);
  int64_t chunks = 0;
  for (int64_t w = 0; w < nw; ++w) {
    const int64_t first = order[w * 64];
    const int32_t nk = (int32_t)((size_of(first) + kCellChunk - 1) / kCellChunk);
    out.waves[w] = KCellWave{chunks, nk, (int32_t)std::min<int64_t>(64, ncells - w * 64)};
    chunks += nk;
  }
  out.nchunks = chunks;
  out.pos.assign(chunks * 1024, kCellPadPos);
  out.flags.assign(chunks * 1024, (uint8_t)(CF_PAD | CF_TIP));
  std::vector<int32_t> pre, ch_off, ch, need, heavy;
  std::vector<uint8_t> fl;
  for (int64_t w = 0; w < nw; ++w) {
    const KCellWave& W = out.waves[w];
    const int64_t span = (int64_t)W.nchunk * kCellChunk;
    for (int32_t c = 0; c < W.ncell; ++c) {
      const int64_t cell = order[w * 64 + c];
      const int64_t lo = cell_offsets[cell];
      const int32_t m = (int32_t)size_of(cell);
      out.lane_cell[w * 64 + c] = (int32_t)cell;
      out.base[w * 64 + c] = lo;
      const int32_t nd = cell_order(parent, lo, m, pre, fl, ch_off, ch, need, heavy);
      if (nd > kCellStack) {
        err = "cell " + std::to_string(cell) + " needs " + std::to_string(nd) +
              " contribution stack entries; the cell-lane kernel holds " + std::to_string(kCellStack);
        return ERR_TOO_BIG;
      }
      out.max_need = std::max(out.max_need, nd);
      // backward step q: padding for q < npad, then the reverse preorder
      const int64_t npad = span - m;
      for (int64_t q = npad; q < span; ++q) {
        const int32_t v = pre[m - 1 - (q - npad)];
        const int64_t k = q / kCellChunk, e = q % kCellChunk;
        const int64_t j = ((c & 3) << 4) | e, r = c >> 2;
        out.pos[(W.chunk_off + k) * 1024 + j * 16 + r] = (uint16_t)v;
        out.flags[(W.chunk_off + k) * 1024 + c * 16 + e] = fl[v];
      }
    }
  }
  (void)n;
  out.built = true;
  return OK;
}

}  // namespace hines
