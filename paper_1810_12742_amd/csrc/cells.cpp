// Tables of the cell-lane solve kernel: one lane per cell (or per half of a
// large cell), 64 lanes of similar length per wave.  Pure C++17; no HIP.
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
//
// A cell much longer than the average is cut at one edge (v, p(v)) into the
// subtree S of v and the rest P, walked by the paired lanes c and c + 32 of
// one wave.  S starts at step 0 and ends with v; P ends with the cell root and
// visits the path from the root to p(v) first in its preorder, so p(v) comes
// late in its backward walk.  The contribution of v crosses through an LDS
// mailbox at a strictly later step, and x of p(v) crosses back in the forward
// sweep, which runs the steps in reverse.
#include <algorithm>
#include <numeric>

#include "setup.hpp"

namespace hines {

namespace {

struct CellTree {
  std::vector<int32_t> ch_off, ch;  // children CSR (relative indices, ascending)
  std::vector<int32_t> size;        // subtree sizes
};

void cell_tree(const int32_t* par, int64_t lo, int32_t m, CellTree& T) {
  T.ch_off.assign(m + 1, 0);
  for (int32_t i = 1; i < m; ++i) T.ch_off[par[lo + i] - lo + 1]++;
  for (int32_t i = 0; i < m; ++i) T.ch_off[i + 1] += T.ch_off[i];
  T.ch.resize(std::max(m - 1, 0));
  std::vector<int32_t> fill(T.ch_off.begin(), T.ch_off.end() - 1);
  for (int32_t i = 1; i < m; ++i) T.ch[fill[par[lo + i] - lo]++] = i;
  T.size.assign(m, 1);
  for (int32_t i = m - 1; i >= 1; --i) T.size[par[lo + i] - lo] += T.size[i];
}

// Walk of the subtree of `root` without the subtree of `cut` (-1: none).
// `forced[a]` (-1: none) is put first among a's children; among the others
// the child with the deepest stack need goes last (the highest index among
// equal needs: breadth-first numbered siblings are adjacent in memory, so
// the backward walk then runs down through them).  Appends the preorder to
// `pre`, sets the flags of the visited nodes in `fl` (indexed by relative
// node) and returns the stack need of the walk.
int32_t walk(const CellTree& T, int32_t root, int32_t cut, const std::vector<int32_t>& forced,
             std::vector<int32_t>& pre, std::vector<uint8_t>& fl, std::vector<int32_t>& need,
             std::vector<int32_t>& seen, std::vector<int32_t>& st) {
  // the visited set in some preorder, then the needs in reverse (children first)
  seen.clear();
  st.clear();
  st.push_back(root);
  while (!st.empty()) {
    const int32_t a = st.back();
    st.pop_back();
    seen.push_back(a);
    for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k)
      if (T.ch[k] != cut) st.push_back(T.ch[k]);
  }
  // children of a in walk order: forced child, the others ascending, the deepest-need child last
  auto ordered = [&](int32_t a, std::vector<int32_t>& out) {
    out.clear();
    int32_t h = -1, hn = -1;
    const int32_t f = forced[a];
    for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k) {
      const int32_t c = T.ch[k];
      if (c == cut || c == f) continue;
      if (need[c] >= hn) {
        hn = need[c];
        h = c;
      }
    }
    if (f >= 0) out.push_back(f);
    for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k) {
      const int32_t c = T.ch[k];
      if (c != cut && c != f && c != h) out.push_back(c);
    }
    if (h >= 0) out.push_back(h);
  };
  std::vector<int32_t> kids;
  for (size_t i = seen.size(); i-- > 0;) {
    const int32_t a = seen[i];
    ordered(a, kids);
    const int32_t nk = (int32_t)kids.size();
    int32_t nd = 0;
    if (nk == 1) {
      nd = need[kids[0]];
    } else if (nk >= 2) {
      int32_t early = 0;
      for (int32_t j = 0; j + 1 < nk; ++j) early = std::max(early, need[kids[j]]);
      nd = std::max(need[kids[nk - 1]], early + 1);
    }
    need[a] = nd;
  }
  // preorder with the chosen child orders, and the flags
  st.clear();
  st.push_back(root);
  while (!st.empty()) {
    const int32_t a = st.back();
    st.pop_back();
    pre.push_back(a);
    ordered(a, kids);
    const int32_t nk = (int32_t)kids.size();
    uint8_t f = 0;
    if (nk == 0) f |= CF_TIP;
    if (nk >= 2) f |= CF_POP;
    fl[a] |= f;
    for (int32_t j = nk - 1; j >= 0; --j) st.push_back(kids[j]);
    if (nk >= 2) {
      fl[kids[nk - 1]] |= CF_PUSH;
      for (int32_t j = 1; j + 1 < nk; ++j) fl[kids[j]] |= CF_MERGE;
    }
  }
  return need[root];
}

// One lane's work: relative positions in backward order (padding excluded),
// their flags, and whether the padding goes after the walk.
struct LaneWork {
  int64_t cell = -1;
  std::vector<int32_t> back;  // backward order
  std::vector<uint8_t> bfl;
  bool pad_after = false;
};

}  // namespace

Status build_cell_lanes(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                        CellLanes& out, std::string& err) {
  out = CellLanes{};
  auto size_of = [&](int64_t c) { return cell_offsets[c + 1] - cell_offsets[c]; };
  for (int64_t c = 0; c < ncells; ++c) {
    if (size_of(c) > kCellMaxSize) {
      err = "cell " + std::to_string(c) + " has " + std::to_string(size_of(c)) +
            " compartments; the cell-lane kernel takes " + std::to_string(kCellMaxSize) + " at most";
      return ERR_TOO_BIG;
    }
  }
  // cells longer than 0.8 times the mean are cut in two (when the pieces fit): shorter
  // lanes and more waves than wave slots, so that short waves fill in behind long ones
  const double mean = ncells ? (double)n / (double)ncells : 0.0;
  const int64_t split_above = std::max<int64_t>(4 * kCellChunk, (int64_t)(0.8 * mean));

  CellTree T;
  std::vector<int32_t> forced, need, pre, seen, st;
  std::vector<uint8_t> fl;
  std::vector<LaneWork> whole, halves;  // halves: S, P, S, P, ...
  std::vector<int64_t> pair_span;        // per pair: the shortest span that keeps the mailbox order
  auto to_back = [](const std::vector<int32_t>& pre_, const std::vector<uint8_t>& fl_, LaneWork& w) {
    w.back.assign(pre_.rbegin(), pre_.rend());
    w.bfl.resize(w.back.size());
    for (size_t i = 0; i < w.back.size(); ++i) w.bfl[i] = fl_[w.back[i]];
  };
  for (int64_t c = 0; c < ncells; ++c) {
    const int64_t lo = cell_offsets[c];
    const int32_t m = (int32_t)size_of(c);
    cell_tree(parent, lo, m, T);
    forced.assign(m, -1);
    need.assign(m, 0);
    bool done = false;
    if (m > split_above) {
      // cut vertex: subtree size closest to m / 2 from below
      int32_t v = -1;
      for (int32_t i = 1; i < m; ++i)
        if (2 * T.size[i] <= m && (v < 0 || T.size[i] > T.size[v])) v = i;
      if (v > 0 && 4 * T.size[v] >= m) {
        const int32_t pv = parent[lo + v] - (int32_t)lo;
        int32_t depth = 0;
        for (int32_t a = pv; a != 0; a = parent[lo + a] - (int32_t)lo) {
          forced[parent[lo + a] - lo] = a;
          ++depth;
        }
        LaneWork S, P;
        S.cell = P.cell = c;
        fl.assign(m, 0);
        pre.clear();
        const int32_t ns = walk(T, v, -1, forced, pre, fl, need, seen, st);
        fl[v] |= CF_MBOUT;
        to_back(pre, fl, S);
        S.pad_after = true;
        pre.clear();
        const int32_t np = walk(T, 0, v, forced, pre, fl, need, seen, st);
        fl[pv] |= CF_MBIN;
        fl[0] |= CF_ROOT;
        to_back(pre, fl, P);
        if (ns <= kCellStack && np <= kCellStack && pre.size() > (size_t)depth && pre[depth] == pv) {
          out.max_need = std::max(out.max_need, std::max(ns, np));
          pair_span.push_back(std::max<int64_t>((int64_t)P.back.size(), (int64_t)S.back.size() + depth + 1));
          halves.push_back(std::move(S));
          halves.push_back(std::move(P));
          done = true;
        }
        forced.assign(m, -1);
      }
    }
    if (!done) {
      LaneWork W;
      W.cell = c;
      fl.assign(m, 0);
      pre.clear();
      const int32_t nd = walk(T, 0, -1, forced, pre, fl, need, seen, st);
      if (nd > kCellStack) {
        err = "cell " + std::to_string(c) + " needs " + std::to_string(nd) +
              " contribution stack entries; the cell-lane kernel holds " + std::to_string(kCellStack);
        return ERR_TOO_BIG;
      }
      fl[0] |= CF_ROOT;
      out.max_need = std::max(out.max_need, nd);
      to_back(pre, fl, W);
      whole.push_back(std::move(W));
    }
  }
  // waves: 32 cut cells (lanes c and c + 32) or 64 whole cells, longest first
  struct WavePlan {
    int64_t span;
    std::vector<const LaneWork*> lanes;  // 64 entries, nullptr for empty lanes
  };
  std::vector<WavePlan> plans;
  {
    std::vector<int64_t> idx(whole.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int64_t a, int64_t b) { return whole[a].back.size() > whole[b].back.size(); });
    for (size_t w = 0; w < idx.size(); w += 64) {
      WavePlan P{0, std::vector<const LaneWork*>(64, nullptr)};
      for (size_t l = 0; l < 64 && w + l < idx.size(); ++l) {
        P.lanes[l] = &whole[idx[w + l]];
        P.span = std::max<int64_t>(P.span, (int64_t)whole[idx[w + l]].back.size());
      }
      plans.push_back(std::move(P));
    }
    std::vector<int64_t> pidx(pair_span.size());
    std::iota(pidx.begin(), pidx.end(), 0);
    std::stable_sort(pidx.begin(), pidx.end(), [&](int64_t a, int64_t b) { return pair_span[a] > pair_span[b]; });
    for (size_t w = 0; w < pidx.size(); w += 32) {
      WavePlan P{0, std::vector<const LaneWork*>(64, nullptr)};
      for (size_t l = 0; l < 32 && w + l < pidx.size(); ++l) {
        P.lanes[l] = &halves[2 * pidx[w + l]];
        P.lanes[l + 32] = &halves[2 * pidx[w + l] + 1];
        P.span = std::max(P.span, pair_span[pidx[w + l]]);
      }
      plans.push_back(std::move(P));
    }
    std::stable_sort(plans.begin(), plans.end(), [](const WavePlan& a, const WavePlan& b) { return a.span > b.span; });
  }
  const int64_t nw = (int64_t)plans.size();
  out.nwaves = nw;
  out.waves.resize(nw);
  out.lane_cell.assign(nw * 64, -1);
  out.base.assign(nw * 64, 0);
  int64_t chunks = 0;
  for (int64_t w = 0; w < nw; ++w) {
    const int32_t nk = (int32_t)((plans[w].span + kCellChunk - 1) / kCellChunk);
    int32_t nc = 0;
    for (int l = 0; l < 64; ++l) nc += plans[w].lanes[l] && !plans[w].lanes[l]->pad_after;
    out.waves[w] = KCellWave{chunks, nk, nc};
    chunks += nk;
  }
  out.nchunks = chunks;
  out.pos.assign(chunks * kCellChunkElems, kCellPadPos);
  out.flags.assign(chunks * kCellChunkElems, (uint8_t)(CF_PAD | CF_TIP));
  for (int64_t w = 0; w < nw; ++w) {
    const KCellWave& W = out.waves[w];
    const int64_t span = (int64_t)W.nchunk * kCellChunk;
    for (int c = 0; c < 64; ++c) {
      const LaneWork* L = plans[w].lanes[c];
      if (!L) continue;
      out.lane_cell[w * 64 + c] = (int32_t)L->cell;
      out.base[w * 64 + c] = cell_offsets[L->cell];
      const int64_t len = (int64_t)L->back.size();
      const int64_t q0 = L->pad_after ? 0 : span - len;
      for (int64_t t = 0; t < len; ++t) {
        const int64_t q = q0 + t;
        const int64_t k = q / kCellChunk;
        const int32_t e = (int32_t)(q % kCellChunk);
        out.pos[cell_pos_index(W.chunk_off + k, c, e)] = (uint16_t)L->back[t];
        out.flags[cell_flag_index(W.chunk_off + k, c, e)] = L->bfl[t];
      }
    }
  }
  out.built = true;
  return OK;
}

}  // namespace hines
