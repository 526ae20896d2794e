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
// A cell much longer than the average is cut at edges (v_i, p(v_i)) into
// subtrees S_i of v_i and the rest P, each walked by a lane of one wave.  All
// receivers p(v_i) lie on one path from the root, which P visits first in its
// preorder, so they come late in its backward walk.  S_i starts at step 0 and
// ends with v_i, whose contribution crosses through the LDS mailbox of S_i's
// lane at a strictly later step; P reads the mailboxes in the order its walk
// meets the receivers (a per-lane list of source lanes).  x of p(v_i) crosses
// back in the forward sweep, which runs the steps in reverse.  One cut takes
// the subtree closest to half the cell; a cell that stays much longer than
// the average is instead cut along its heavy path (the child with the most
// compartments at every step from the root), up to kCellMaxCuts subtrees.

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <new>
#include <numeric>
#include <system_error>
#include <thread>

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

// Walk of the subtree of `root` without the subtrees whose roots `excl` marks.
// `forced[a]` (-1: none) is put first among a's children; among the others
// the child with the deepest stack need goes last (the highest index among
// equal needs: breadth-first numbered siblings are adjacent in memory, so
// the backward walk then runs down through them).  Appends the preorder to
// `pre`, sets the flags of the visited nodes in `fl` (indexed by relative
// node) and returns the stack need of the walk.
int32_t walk(const CellTree& T, int32_t root, const std::vector<uint8_t>& excl, const std::vector<int32_t>& forced,
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
      if (!excl[T.ch[k]]) st.push_back(T.ch[k]);
  }
  // children of a in walk order: forced child, the others ascending, the deepest-need child last
  auto ordered = [&](int32_t a, std::vector<int32_t>& out) {
    out.clear();
    int32_t h = -1, hn = -1;
    const int32_t f = forced[a];
    for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k) {
      const int32_t c = T.ch[k];
      if (excl[c] || c == f) continue;
      if (need[c] >= hn) {
        hn = need[c];
        h = c;
      }
    }
    if (f >= 0) out.push_back(f);
    for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k) {
      const int32_t c = T.ch[k];
      if (!excl[c] && c != f && c != h) out.push_back(c);
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
                        CellLanes& out, std::string& err, int32_t cut_percent, int32_t max_cuts) {
  out = CellLanes{};
  auto size_of = [&](int64_t c) { return cell_offsets[c + 1] - cell_offsets[c]; };
  for (int64_t c = 0; c < ncells; ++c) {
    if (size_of(c) > kCellMaxSize) {
      err = "cell " + std::to_string(c) + " has " + std::to_string(size_of(c)) +
            " compartments; the cell-lane kernel takes " + std::to_string(kCellMaxSize) + " at most";
      return ERR_TOO_BIG;
    }
  }
  if (cut_percent < 1 || max_cuts < 1 || max_cuts > kCellMaxCuts) {
    err = "cell cut options out of range";
    return ERR_OPTION;
  }
  // cells longer than cut_percent of the mean (80% by default) are cut (when
  // the pieces fit): shorter lanes and more waves than wave slots, so that
  // short waves fill in behind long ones
  const double mean = ncells ? (double)n / (double)ncells : 0.0;
  const int64_t split_above = std::max<int64_t>(4 * kCellChunk, (int64_t)(0.01 * cut_percent * mean));
  // cutting a lane below the steps every wave slot of the device walks anyway
  // only adds padding: 1,024 slots (256 compute units, 4 SIMDs, one wave each
  // at this kernel's register use), 64 lanes, about 15% padding
  const int64_t slot_steps = (int64_t)(1.15 * (double)n / (64.0 * 1024.0));
  // too few cells to give every wave slot's lanes work (two lanes per cell or
  // more fit): cut every cell longer than a slot's share, whatever the mean
  const bool underfull = 2 * ncells <= 64 * 1024;
  const int64_t cut_above = underfull ? std::max<int64_t>(4 * kCellChunk, slot_steps) : split_above;
  const int64_t heavy_above = underfull ? cut_above : 2 * split_above;
  const int64_t target_floor = underfull ? cut_above : std::max(split_above, slot_steps);

  // a group: the lanes of one cell, lanes[0] whole or P, then the S_i in the
  // order P's backward walk takes their contributions
  struct Group {
    int64_t span = 0;
    std::vector<LaneWork> lanes;
  };
  std::vector<Group> groups(ncells);
  auto to_back = [](const std::vector<int32_t>& pre_, const std::vector<uint8_t>& fl_, LaneWork& w) {
    w.back.assign(pre_.rbegin(), pre_.rend());
    w.bfl.resize(w.back.size());
    for (size_t i = 0; i < w.back.size(); ++i) w.bfl[i] = fl_[w.back[i]];
  };
  // the cells are planned independently, by several threads over blocks of
  // cells; each result lands at its cell's index, so the tables do not
  // depend on the thread count
  struct RangeResult {
    int32_t max_need = 0;
    int64_t bad = -1;  // first cell whose walk needs too deep a stack
    std::string err;
  };
  auto run_range = [&](int64_t c0, int64_t c1, RangeResult& R) {
    CellTree T;
    std::vector<int32_t> forced, need, pre, seen, st, depth, path, pick;
    std::vector<uint8_t> fl, excl, onpath;
    // span of cutting off the subtrees `vs` (receivers on one root path): P
    // ends with the root and has receiver r at step span - 1 - depth(r)
    auto cut_span = [&](int32_t m, const std::vector<int32_t>& vs, int32_t lo) {
      int64_t rest = m, sp = 0;
      for (int32_t v : vs) {
        rest -= T.size[v];
        sp = std::max<int64_t>(sp, (int64_t)T.size[v] + depth[parent[lo + v] - lo] + 1);
      }
      return std::max(rest, sp);
    };
    // cut along the heavy path: for a target span t, per receiver the largest
    // off-path child that fits, largest first, until the rest fits
    auto heavy_cut = [&](int32_t m, int64_t t, std::vector<int32_t>& out) {
      std::vector<std::pair<int32_t, int32_t>> cand;  // (size, child)
      for (size_t i = 0; i + 1 < path.size(); ++i) {
        const int32_t a = path[i];
        int32_t best = -1;
        for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k) {
          const int32_t c = T.ch[k];
          if (onpath[c] || (int64_t)T.size[c] + depth[a] + 1 > t) continue;
          if (best < 0 || T.size[c] > T.size[best]) best = c;
        }
        if (best >= 0) cand.push_back({T.size[best], best});
      }
      std::sort(cand.begin(), cand.end(), [](auto x, auto y) { return x.first > y.first || (x.first == y.first && x.second < y.second); });
      out.clear();
      int64_t rest = m;
      for (auto& cs : cand) {
        if (rest <= t || (int)out.size() >= max_cuts) break;
        out.push_back(cs.second);
        rest -= cs.first;
      }
      return rest <= t;
    };
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t lo = cell_offsets[c];
      const int32_t m = (int32_t)size_of(c);
      cell_tree(parent, lo, m, T);
      forced.assign(m, -1);
      need.assign(m, 0);
      excl.assign(m, 0);
      bool done = false;
      if (m > cut_above) {
        depth.assign(m, 0);
        for (int32_t i = 1; i < m; ++i) depth[i] = depth[parent[lo + i] - lo] + 1;
        // one cut: the subtree closest to m / 2 from below (at least a quarter)
        // candidate cuts, preferred first: (subtree roots, span)
        std::vector<std::pair<std::vector<int32_t>, int64_t>> cands;
        int32_t v = -1;
        for (int32_t i = 1; i < m; ++i)
          if (2 * T.size[i] <= m && (v < 0 || T.size[i] > T.size[v])) v = i;
        int64_t span = m;
        if (v > 0 && 4 * T.size[v] >= m) {
          cands.push_back({{v}, cut_span(m, {v}, (int32_t)lo)});
          span = cands.back().second;
        }
        if (span > heavy_above) {  // still much longer than the average (or a slot's share): the heavy path
          path.assign(1, 0);
          onpath.assign(m, 0);
          onpath[0] = 1;
          for (;;) {
            const int32_t a = path.back();
            int32_t h = -1;
            for (int32_t k = T.ch_off[a]; k < T.ch_off[a + 1]; ++k)
              if (h < 0 || T.size[T.ch[k]] > T.size[h]) h = T.ch[k];
            if (h < 0) break;
            path.push_back(h);
            onpath[h] = 1;
          }
          int64_t tl = std::max<int64_t>((m + max_cuts) / (max_cuts + 1), target_floor), th = span;
          if (tl < th && heavy_cut(m, th - 1, pick)) {
            while (tl < th) {  // smallest feasible target
              const int64_t mid = (tl + th) / 2;
              if (heavy_cut(m, mid, pick)) th = mid;
              else tl = mid + 1;
            }
            heavy_cut(m, th, pick);
            if (!pick.empty() && cut_span(m, pick, (int32_t)lo) < span)
              cands.insert(cands.begin(), {pick, cut_span(m, pick, (int32_t)lo)});
          }
        }
        // the first candidate whose walks fit the stack and keep every receiver in place
        for (auto& cand : cands) {
          if (done) break;
          std::vector<int32_t> vs = cand.first;
          span = cand.second;
          // P's forced path: from the root to the deepest receiver; every receiver on it
          int32_t deep = -1;
          for (int32_t x : vs) {
            const int32_t r = parent[lo + x] - (int32_t)lo;
            if (deep < 0 || depth[r] > depth[deep]) deep = r;
          }
          for (int32_t a = deep; a != 0; a = parent[lo + a] - (int32_t)lo) forced[parent[lo + a] - lo] = a;
          // S_i in the order P's backward walk meets their receivers: deepest first
          std::sort(vs.begin(), vs.end(), [&](int32_t x, int32_t y) {
            const int32_t dx = depth[parent[lo + x] - lo], dy = depth[parent[lo + y] - lo];
            return dx > dy || (dx == dy && x < y);
          });
          Group g;
          g.lanes.resize(1 + vs.size());
          fl.assign(m, 0);
          bool ok = true;
          int32_t nd = 0;
          for (size_t i = 0; i < vs.size(); ++i) {
            pre.clear();
            nd = std::max(nd, walk(T, vs[i], excl, forced, pre, fl, need, seen, st));
            fl[vs[i]] |= CF_MBOUT;
            LaneWork& S = g.lanes[1 + i];
            S.cell = c;
            S.pad_after = true;
            to_back(pre, fl, S);
            excl[vs[i]] = 1;
          }
          pre.clear();
          nd = std::max(nd, walk(T, 0, excl, forced, pre, fl, need, seen, st));
          for (size_t i = 0; i < vs.size(); ++i) {
            const int32_t r = parent[lo + vs[i]] - (int32_t)lo;
            fl[r] |= CF_MBIN;
            ok = ok && pre.size() > (size_t)depth[r] && pre[depth[r]] == r;
            ok = ok && (i == 0 || r != parent[lo + vs[i - 1]] - (int32_t)lo);  // one take per receiver
          }
          fl[0] |= CF_ROOT;
          LaneWork& P = g.lanes[0];
          P.cell = c;
          to_back(pre, fl, P);
          if (ok && nd <= kCellStack) {
            R.max_need = std::max(R.max_need, nd);
            g.span = span;
            groups[c] = std::move(g);
            done = true;
          }
          forced.assign(m, -1);
          excl.assign(m, 0);
        }
      }
      if (!done) {
        Group g;
        g.lanes.resize(1);
        LaneWork& W = g.lanes[0];
        W.cell = c;
        fl.assign(m, 0);
        pre.clear();
        const int32_t nd = walk(T, 0, excl, forced, pre, fl, need, seen, st);
        if (nd > kCellStack) {
          R.bad = c;
          R.err = "cell " + std::to_string(c) + " needs " + std::to_string(nd) +
                  " contribution stack entries; the cell-lane kernel holds " + std::to_string(kCellStack);
          return;
        }
        fl[0] |= CF_ROOT;
        R.max_need = std::max(R.max_need, nd);
        to_back(pre, fl, W);
        g.span = (int64_t)W.back.size();
        groups[c] = std::move(g);
      }
    }
  };
  {
    constexpr int64_t kBlock = 256;
    const int64_t nblocks = (ncells + kBlock - 1) / kBlock;
    // threads: HINES_SETUP_THREADS if set, else the host's cores, at most 16
    int64_t want = std::thread::hardware_concurrency();
    if (const char* env = std::getenv("HINES_SETUP_THREADS")) want = std::atoll(env);
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({want, 16, nblocks}));
    std::atomic<int64_t> next{0};
    std::vector<RangeResult> res(nth);
    std::atomic<bool> oom{false};  // a worker ran out of memory: raised again in this thread
    auto worker = [&](int t) {
      try {
        for (;;) {
          const int64_t b = next.fetch_add(1);
          if (b >= nblocks) break;
          RangeResult r;
          run_range(b * kBlock, std::min(ncells, (b + 1) * kBlock), r);
          res[t].max_need = std::max(res[t].max_need, r.max_need);
          if (r.bad >= 0 && (res[t].bad < 0 || r.bad < res[t].bad)) {
            res[t].bad = r.bad;
            res[t].err = r.err;
          }
        }
      } catch (const std::bad_alloc&) {
        oom = true;
      }
    };
    std::vector<std::thread> pool;
    try {
      for (int t = 1; t < nth; ++t) pool.emplace_back(worker, t);
    } catch (const std::system_error&) {  // no more threads: the ones started and this one finish the work
    }
    worker(0);
    for (auto& th : pool) th.join();
    if (oom) throw std::bad_alloc();
    const RangeResult* first = nullptr;  // the lowest failing cell, whatever the thread count
    for (const RangeResult& r : res) {
      out.max_need = std::max(out.max_need, r.max_need);
      if (r.bad >= 0 && (!first || r.bad < first->bad)) first = &r;
    }
    if (first) {
      err = first->err;
      return ERR_TOO_BIG;
    }
  }
  // waves: groups of the same lane count, longest first.  A wave holds 64
  // whole cells, or 32 two-lane cells (the cut-off subtree in lane c, the rest
  // in lane c + 32), or 64 / g cells of g lanes on consecutive lanes
  struct WavePlan {
    int64_t span;
    std::vector<const LaneWork*> lanes;  // 64 entries, nullptr for empty lanes
    std::vector<uint64_t> src;           // per lane: mailbox source lanes, backward | forward order << 32
  };
  std::vector<WavePlan> plans;
  {
    std::vector<int64_t> idx(groups.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      const size_t la = groups[a].lanes.size(), lb = groups[b].lanes.size();
      return la < lb || (la == lb && groups[a].span > groups[b].span);
    });
    size_t prev = 0;
    int slot = 0, per = 0;
    for (int64_t gi : idx) {
      const Group& g = groups[gi];
      const int nl = (int)g.lanes.size();
      if ((size_t)nl != prev || slot == per) {
        plans.push_back(WavePlan{0, std::vector<const LaneWork*>(64, nullptr), std::vector<uint64_t>(64, 0)});
        prev = (size_t)nl;
        per = 64 / nl;
        slot = 0;
      }
      WavePlan& P = plans.back();
      // lane of piece i: piece-major, so that lanes of similar length are
      // adjacent and their padding fills whole memory lines of the walk
      // layout.  Pieces: the rest P in the first block, the cut-off subtrees
      // ranked by length (longest first) in the next ones; pairs split across
      // the halves (P in the upper one).
      int blk[kCellMaxCuts + 1] = {0, 1, 2, 3};
      if (nl >= 3) {
        int ord[kCellMaxCuts];
        for (int i = 1; i < nl; ++i) ord[i - 1] = i;
        std::stable_sort(ord, ord + nl - 1, [&](int a, int b) { return g.lanes[a].back.size() > g.lanes[b].back.size(); });
        for (int r = 0; r + 1 < nl; ++r) blk[ord[r]] = r + 1;
      }
      auto lane_of = [&](int i) { return nl == 2 ? (i == 0 ? slot + 32 : slot) : blk[i] * per + slot; };
      uint64_t bw = 0, fw = 0;
      for (int i = 1; i < nl; ++i) {
        bw |= (uint64_t)lane_of(i) << (6 * (i - 1));
        fw |= (uint64_t)lane_of(i) << (6 * (nl - 1 - i));
      }
      P.src[lane_of(0)] = bw | (fw << 32);
      for (int i = 0; i < nl; ++i) P.lanes[lane_of(i)] = &g.lanes[i];
      P.span = std::max(P.span, g.span);
      ++slot;
    }
    std::stable_sort(plans.begin(), plans.end(), [](const WavePlan& a, const WavePlan& b) { return a.span > b.span; });
  }
  const int64_t nw = (int64_t)plans.size();
  out.nwaves = nw;
  out.waves.resize(nw);
  out.lane_cell.assign(nw * 64, -1);
  out.base.assign(nw * 64, 0);
  out.mbsrc.assign(nw * 64, 0);
  out.range.assign(nw * 64, 0);
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
      out.mbsrc[w * 64 + c] = plans[w].src[c];
      out.base[w * 64 + c] = cell_offsets[L->cell];
      const int64_t len = (int64_t)L->back.size();
      const int64_t q0 = L->pad_after ? 0 : span - len;
      out.range[w * 64 + c] = (uint64_t)q0 | ((uint64_t)(q0 + len) << 32);
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

// ---------------------------------------------------------------------------
// Index-order cell lanes (cell_lanes 2)
// ---------------------------------------------------------------------------

namespace {

struct SeqPiece {
  std::vector<int32_t> walk;   // relative index per step in backward order, -1 for padding
  std::vector<uint16_t> code;  // per step
  int32_t slots = 0;
  bool depth_first = false;
};

// Line-aligned layout of a children-first order: padding in front of the first
// run and of every later run of at least kSeqMinRun consecutive decreasing
// indices, so that its step s holds user index g with s + g = 15 (mod 16).
void seq_layout(const std::vector<int32_t>& order, int64_t lo, std::vector<int32_t>& out) {
  out.clear();
  size_t a = 0;
  while (a < order.size()) {
    size_t b = a + 1;
    while (b < order.size() && order[b] == order[b - 1] - 1) ++b;
    if (a == 0 || b - a >= (size_t)kSeqMinRun) {
      const int64_t t = (int64_t)out.size(), g = lo + order[a];
      const int64_t pad = ((kSeqLine - 1 - t - g) % kSeqLine + kSeqLine) % kSeqLine;
      out.insert(out.end(), (size_t)pad, -1);
    }
    out.insert(out.end(), order.begin() + (ptrdiff_t)a, order.begin() + (ptrdiff_t)b);
    a = b;
  }
}

// Step codes of a laid-out walk.  root: the piece's root (0: the cell root,
// else a cut-off subtree's root, whose contribution leaves through the
// mailbox); recv[i] != 0: i receives a cut-off subtree's contribution.
// A contribution goes to the next step when that step is the parent, else into
// the parent's slot, taken at the first such child (the smallest free one) and
// released when the parent reads it.  slot_of (per relative index, all zero)
// is left all zero.  Returns the slots used, -1 if more than kSeqSlots.
int32_t seq_codes(const int32_t* parent, int64_t lo, const std::vector<int32_t>& w, int32_t root,
                  const std::vector<uint8_t>& recv, std::vector<uint16_t>& code, std::vector<uint8_t>& slot_of) {
  const size_t L = w.size();
  code.assign(L, (uint16_t)(SQ_PAD | SQ_TIP));
  auto par = [&](int32_t i) { return parent[lo + i] - (int32_t)lo; };
  uint32_t used = 0;
  int32_t top = 0;
  for (size_t t = 0; t < L; ++t) {
    const int32_t i = w[t];
    if (i < 0) continue;
    uint16_t q = 0;
    const bool carry = t > 0 && w[t - 1] >= 0 && w[t - 1] != root && par(w[t - 1]) == i;
    if (!carry) q |= SQ_TIP;
    if (slot_of[i]) {
      q |= (uint16_t)(slot_of[i] << SQ_READ_SHIFT);
      used &= ~(1u << (slot_of[i] - 1));
      slot_of[i] = 0;
    }
    if (i == 0) q |= SQ_ROOT;
    if (i == root) {
      if (root != 0) q |= SQ_MBOUT;
    } else if (!(t + 1 < L && w[t + 1] == par(i))) {
      const int32_t p = par(i);
      if (!slot_of[p]) {
        const int s = __builtin_ctz(~used) + 1;
        if (s > kSeqSlots) {
          for (int32_t j : w)
            if (j >= 0) slot_of[j] = 0;
          return -1;
        }
        used |= 1u << (s - 1);
        slot_of[p] = (uint8_t)s;
        top = std::max(top, s);
        q |= SQ_FIRST;
      }
      q |= slot_of[p];
    }
    if (recv[i]) q |= SQ_MBIN;
    code[t] = q;
  }
  return top;
}

}  // namespace

Status build_seq_lanes(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                       SeqLanes& out, std::string& err, int32_t cut_percent, int32_t max_cuts) {
  out = SeqLanes{};
  auto size_of = [&](int64_t c) { return cell_offsets[c + 1] - cell_offsets[c]; };
  for (int64_t c = 0; c < ncells; ++c) {
    if (size_of(c) > kCellMaxSize) {
      err = "cell " + std::to_string(c) + " has " + std::to_string(size_of(c)) +
            " compartments; the cell-lane kernel takes " + std::to_string(kCellMaxSize) + " at most";
      return ERR_TOO_BIG;
    }
  }
  if (cut_percent < 1 || max_cuts < 1 || max_cuts > kCellMaxCuts) {
    err = "cell cut options out of range";
    return ERR_OPTION;
  }
  // when to cut: as for the depth-first lanes (longer than cut_percent of the
  // mean cell, or than a wave slot's share when there are few cells)
  const double mean = ncells ? (double)n / (double)ncells : 0.0;
  const int64_t split_above = std::max<int64_t>(4 * kSeqLine, (int64_t)(0.01 * cut_percent * mean));
  const int64_t slot_steps = (int64_t)(1.15 * (double)n / (64.0 * 1024.0));
  const bool underfull = 2 * ncells <= 64 * 1024;
  const int64_t cut_above = underfull ? std::max<int64_t>(4 * kSeqLine, slot_steps) : split_above;

  constexpr int32_t kMaxPieces = kCellMaxCuts + 1;
  struct Group {
    int64_t span = 0;
    int32_t npiece = 0;
    SeqPiece piece[kMaxPieces];  // piece 0 holds the cell root; piece k > 0 a cut-off subtree
    int8_t nsrc[kMaxPieces] = {};
    int8_t src[kMaxPieces][kMaxPieces] = {};  // per piece: the pieces whose mailboxes it takes, in step order
  };
  std::vector<Group> groups(ncells);
  struct RangeResult {
    int32_t max_slots = 0;
    int64_t depth_first = 0;
    int64_t bad = -1;
    std::string err;
  };
  auto run_range = [&](int64_t c0, int64_t c1, RangeResult& R) {
    CellTree T;
    std::vector<int32_t> order, forced, need, pre, seen, st, szx, cnt;
    std::vector<uint8_t> fl, excl, slot_of, own, mbin;
    int64_t lo = 0;
    int32_t m = 0;
    auto par = [&](int32_t i) { return parent[lo + i] - (int32_t)lo; };
    // piece k: the index walk, or the depth-first walk when that needs too many slots
    auto make_piece = [&](int32_t k, int32_t root, int32_t recv0, SeqPiece& P) {
      order.clear();
      for (int32_t i = m - 1; i >= 0; --i)
        if (own[i] == k) order.push_back(i);
      seq_layout(order, lo, P.walk);
      P.slots = seq_codes(parent, lo, P.walk, root, mbin, P.code, slot_of);
      if (P.slots >= 0) return true;
      // a receiver's path first in preorder, so that it comes late in the backward walk
      forced.assign(m, -1);
      if (recv0 >= 0)
        for (int32_t a = recv0; a != root; a = par(a)) forced[par(a)] = a;
      need.assign(m, 0);
      fl.assign(m, 0);
      pre.clear();
      walk(T, root, excl, forced, pre, fl, need, seen, st);
      order.assign(pre.rbegin(), pre.rend());
      seq_layout(order, lo, P.walk);
      P.slots = seq_codes(parent, lo, P.walk, root, mbin, P.code, slot_of);
      P.depth_first = true;
      return P.slots >= 0;
    };
    for (int64_t c = c0; c < c1; ++c) {
      lo = cell_offsets[c];
      m = (int32_t)size_of(c);
      Group& g = groups[c];
      if (m == 0) continue;
      cell_tree(parent, lo, m, T);
      own.assign(m, 0);
      mbin.assign(m, 0);
      excl.assign(m, 0);
      slot_of.assign(m, 0);
      // pieces: repeatedly cut the longest piece while it is longer than
      // cut_above, at the subtree S of v minimising the longer lane with the
      // receiver p(v) after S's last step in the index walk (the piece's
      // steps above p(v) number cnt(p(v) + 1) - |S|; a shortfall pads the
      // front), one cut-off subtree per receiver
      int32_t np = 1;
      int32_t root[kMaxPieces] = {0}, size[kMaxPieces] = {m}, up[kMaxPieces] = {-1}, recv[kMaxPieces] = {-1};
      while (m > cut_above && np < max_cuts + 1) {
        int32_t X = 0;
        for (int32_t k = 1; k < np; ++k)
          if (size[k] > size[X]) X = k;
        if (size[X] <= cut_above) break;
        szx.assign(m, 0);
        for (int32_t i = 0; i < m; ++i) szx[i] = own[i] == X;
        for (int32_t i = m - 1; i >= 1; --i)
          if (own[i] == X && own[par(i)] == X) szx[par(i)] += szx[i];
        cnt.assign(m + 1, 0);
        for (int32_t i = m - 1; i >= 0; --i) cnt[i] = cnt[i + 1] + (own[i] == X);
        int64_t best = size[X];
        int32_t v = -1;
        for (int32_t i = 1; i < m; ++i) {
          if (own[i] != X || i == root[X] || mbin[par(i)]) continue;
          const int64_t S = szx[i];
          const int64_t above = cnt[par(i) + 1] - S;
          const int64_t len = std::max<int64_t>(S, size[X] - S + std::max<int64_t>(0, S - above));
          if (len < best) {
            best = len;
            v = i;
          }
        }
        if (v < 0) break;
        const int32_t Y = np++;
        own[v] = (uint8_t)Y;
        for (int32_t i = v + 1; i < m; ++i)
          if (own[i] == X && own[par(i)] == Y) own[i] = (uint8_t)Y;
        size[X] -= szx[v];
        size[Y] = szx[v];
        root[Y] = v;
        up[Y] = X;
        recv[Y] = par(v);
        mbin[par(v)] = 1;
        excl[v] = 1;
        for (int32_t j = 1; j < Y; ++j)  // earlier receivers inside the new piece now take there
          if (own[recv[j]] == Y) up[j] = Y;
      }
      g.npiece = np;
      bool ok = true;
      for (int32_t k = 0; k < np && ok; ++k) {
        int32_t r0 = -1;
        for (int32_t j = 1; j < np; ++j)
          if (up[j] == k && r0 < 0) r0 = recv[j];
        ok = make_piece(k, root[k], r0, g.piece[k]);
        R.max_slots = std::max(R.max_slots, g.piece[k].slots);
        R.depth_first += (int64_t)g.piece[k].depth_first;
      }
      if (!ok) {
        R.bad = c;
        R.err = "cell " + std::to_string(c) + " needs more than " + std::to_string(kSeqSlots) +
                " contribution slots in either walk order";
        return;
      }
      // mailbox order: each receiver takes its subtree's contribution at a
      // strictly later step (and sends x back at a strictly earlier forward
      // step).  Pieces deepest in the piece tree first, so that a piece's
      // sources are final when its front is padded (by whole lines)
      int32_t depth[kMaxPieces], byd[kMaxPieces];
      for (int32_t k = 0; k < np; ++k) {
        depth[k] = 0;
        for (int32_t a = k; up[a] >= 0; a = up[a]) ++depth[k];
        byd[k] = k;
      }
      std::stable_sort(byd, byd + np, [&](int32_t a, int32_t b) { return depth[a] > depth[b]; });
      for (int32_t kk = 0; kk < np; ++kk) {
        const int32_t k = byd[kk];
        SeqPiece& P = g.piece[k];
        int64_t sh = 0;
        int32_t js[kMaxPieces];
        int64_t ts[kMaxPieces];
        int32_t nj = 0;
        for (int32_t j = 1; j < np; ++j) {
          if (up[j] != k) continue;
          int64_t tr = 0;
          while (tr < (int64_t)P.walk.size() && P.walk[tr] != recv[j]) ++tr;
          if (tr == (int64_t)P.walk.size()) {
            R.bad = c;
            R.err = "cell " + std::to_string(c) + ": a receiver outside its piece";
            return;
          }
          const int64_t tv = (int64_t)g.piece[j].walk.size() - 1;
          sh = std::max<int64_t>(sh, tv + 1 - tr);
          js[nj] = j;
          ts[nj++] = tr;
        }
        if (sh > 0) {
          sh = (sh + kSeqLine - 1) / kSeqLine * kSeqLine;
          P.walk.insert(P.walk.begin(), (size_t)sh, -1);
          P.code.insert(P.code.begin(), (size_t)sh, (uint16_t)(SQ_PAD | SQ_TIP));
        }
        // takes in the order of the backward walk
        for (int32_t a = 1; a < nj; ++a)
          for (int32_t b = a; b > 0 && ts[b] < ts[b - 1]; --b) {
            std::swap(ts[b], ts[b - 1]);
            std::swap(js[b], js[b - 1]);
          }
        g.nsrc[k] = (int8_t)nj;
        for (int32_t a = 0; a < nj; ++a) g.src[k][a] = (int8_t)js[a];
      }
      g.span = 0;
      for (int32_t k = 0; k < np; ++k) g.span = std::max<int64_t>(g.span, (int64_t)g.piece[k].walk.size());
    }
  };
  {
    constexpr int64_t kBlock = 256;
    const int64_t nblocks = (ncells + kBlock - 1) / kBlock;
    int64_t want = std::thread::hardware_concurrency();
    if (const char* env = std::getenv("HINES_SETUP_THREADS")) want = std::atoll(env);
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({want, 16, nblocks}));
    std::atomic<int64_t> next{0};
    std::vector<RangeResult> res(nth);
    std::atomic<bool> oom{false};
    auto worker = [&](int t) {
      try {
        for (;;) {
          const int64_t b = next.fetch_add(1);
          if (b >= nblocks) break;
          RangeResult r;
          run_range(b * kBlock, std::min(ncells, (b + 1) * kBlock), r);
          res[t].max_slots = std::max(res[t].max_slots, r.max_slots);
          res[t].depth_first += r.depth_first;
          if (r.bad >= 0 && (res[t].bad < 0 || r.bad < res[t].bad)) {
            res[t].bad = r.bad;
            res[t].err = r.err;
          }
        }
      } catch (const std::bad_alloc&) {
        oom = true;
      }
    };
    std::vector<std::thread> pool;
    try {
      for (int t = 1; t < nth; ++t) pool.emplace_back(worker, t);
    } catch (const std::system_error&) {
    }
    worker(0);
    for (auto& th : pool) th.join();
    if (oom) throw std::bad_alloc();
    const RangeResult* first = nullptr;
    for (const RangeResult& r : res) {
      out.max_slots = std::max(out.max_slots, r.max_slots);
      out.depth_first += r.depth_first;
      if (r.bad >= 0 && (!first || r.bad < first->bad)) first = &r;
    }
    if (first) {
      err = first->err;
      return ERR_TOO_BIG;
    }
  }
  // waves: cells by span, longest first; the pieces of a cut cell on
  // adjacent lanes of one wave, piece k on lane l0 + k
  struct WavePlan {
    int64_t span = 0;
    int32_t used = 0, ncell = 0;
    int64_t cell[64];
    int32_t piece[64];
    uint64_t src[64];
  };
  std::vector<WavePlan> plans;
  {
    std::vector<int64_t> idx;
    idx.reserve(ncells);
    for (int64_t c = 0; c < ncells; ++c)
      if (groups[c].npiece) idx.push_back(c);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return groups[a].span > groups[b].span; });
    for (int64_t gi : idx) {
      const Group& g = groups[gi];
      if (plans.empty() || plans.back().used + g.npiece > 64) {
        plans.emplace_back();
        std::fill(plans.back().src, plans.back().src + 64, (uint64_t)0);
      }
      WavePlan& P = plans.back();
      const int32_t l0 = P.used;
      for (int32_t k = 0; k < g.npiece; ++k) {
        P.cell[l0 + k] = gi;
        P.piece[l0 + k] = k;
        uint64_t bw = 0, fw = 0;
        const int32_t nj = g.nsrc[k];
        for (int32_t a = 0; a < nj; ++a) {
          bw |= (uint64_t)(l0 + g.src[k][a]) << (6 * a);
          fw |= (uint64_t)(l0 + g.src[k][a]) << (6 * (nj - 1 - a));
        }
        P.src[l0 + k] = bw | (fw << 32);
      }
      P.used += g.npiece;
      P.ncell += 1;
      P.span = std::max(P.span, g.span);
    }
  }
  const int64_t nw = (int64_t)plans.size();
  out.nwaves = nw;
  out.waves.resize(nw);
  out.lane_cell.assign(nw * 64, -1);
  out.base.assign(nw * 64, 0);
  out.mbsrc.assign(nw * 64, 0);
  int64_t chunks = 0;
  for (int64_t w = 0; w < nw; ++w) {
    const int32_t nk = (int32_t)((plans[w].span + kSeqChunk - 1) / kSeqChunk);
    out.waves[w] = KCellWave{chunks, nk, plans[w].ncell};
    chunks += nk;
  }
  out.nchunks = chunks;
  out.pos.assign(chunks * kSeqChunkElems, kCellPadPos);
  out.code.assign(chunks * kSeqChunkElems, (uint16_t)(SQ_PAD | SQ_TIP));
  for (int64_t w = 0; w < nw; ++w) {
    const KCellWave& W = out.waves[w];
    for (int32_t c = 0; c < plans[w].used; ++c) {
      const int64_t cell = plans[w].cell[c];
      const SeqPiece& P = groups[cell].piece[plans[w].piece[c]];
      out.lane_cell[w * 64 + c] = (int32_t)cell;
      out.base[w * 64 + c] = cell_offsets[cell];
      out.mbsrc[w * 64 + c] = plans[w].src[c];
      for (size_t t = 0; t < P.walk.size(); ++t) {
        const int64_t k = (int64_t)t / kSeqChunk;
        const int32_t e = (int32_t)(t % kSeqChunk);
        out.pos[seq_pos_index(W.chunk_off + k, c, e)] = P.walk[t] >= 0 ? (uint16_t)P.walk[t] : kCellPadPos;
        out.code[seq_code_index(W.chunk_off + k, c, e)] = P.code[t];
      }
    }
  }
  out.built = true;
  return OK;
}

bool check_seq_lanes(const SeqLanes& Q, const int32_t* parent, int64_t n, const int64_t* cell_offsets,
                     int64_t ncells, std::string& why) {
  std::vector<uint8_t> seen(n, 0);
  const int64_t nw = Q.nwaves;
  if ((int64_t)Q.waves.size() != nw || (int64_t)Q.lane_cell.size() != 64 * nw || (int64_t)Q.base.size() != 64 * nw ||
      (int64_t)Q.mbsrc.size() != 64 * nw || (int64_t)Q.pos.size() != Q.nchunks * kSeqChunkElems ||
      (int64_t)Q.code.size() != Q.nchunks * kSeqChunkElems) {
    why = "index-order lane table sizes";
    return false;
  }
  for (int64_t w = 0; w < nw; ++w) {
    const KCellWave& W = Q.waves[w];
    const int64_t steps = (int64_t)W.nchunk * kSeqChunk;
    if (W.chunk_off < 0 || W.chunk_off + W.nchunk > Q.nchunks) {
      why = "wave " + std::to_string(w) + " outside the tables";
      return false;
    }
    int64_t mbout_step[64], mbin_step[64];
    int32_t mbout_node[64], mbin_node[64], mbin_lane[64];
    for (int c = 0; c < 64; ++c) mbout_step[c] = mbin_step[c] = -1, mbout_node[c] = mbin_node[c] = mbin_lane[c] = -1;
    for (int c = 0; c < 64; ++c) {
      const int64_t cell = Q.lane_cell[w * 64 + c];
      const uint64_t src = Q.mbsrc[w * 64 + c];
      auto fail = [&](const std::string& s) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + ": " + s;
        return false;
      };
      if (cell < 0) {
        for (int64_t t = 0; t < steps; ++t) {
          const int64_t k = t / kSeqChunk, e = t % kSeqChunk;
          if (Q.pos[seq_pos_index(W.chunk_off + k, c, (int32_t)e)] != kCellPadPos ||
              Q.code[seq_code_index(W.chunk_off + k, c, (int32_t)e)] != (SQ_PAD | SQ_TIP))
            return fail("empty lane with work");
        }
        continue;
      }
      if (cell >= ncells || Q.base[w * 64 + c] != cell_offsets[cell]) return fail("cell or base");
      const int64_t lo = cell_offsets[cell], m = cell_offsets[cell + 1] - lo;
      int32_t owner[kSeqSlots + 1];
      for (int s = 0; s <= kSeqSlots; ++s) owner[s] = -1;
      int32_t prev = -1;
      bool prev_up = false;  // the previous step's contribution goes to the next step
      uint32_t msl = (uint32_t)src;  // the backward source list, next take in the low 6 bits
      int32_t takes[6];
      int32_t ntake = 0;
      for (int64_t t = 0; t < steps; ++t) {
        const int64_t k = t / kSeqChunk, e = t % kSeqChunk;
        const uint16_t p16 = Q.pos[seq_pos_index(W.chunk_off + k, c, (int32_t)e)];
        const uint16_t q = Q.code[seq_code_index(W.chunk_off + k, c, (int32_t)e)];
        if (q & SQ_PAD) {
          if (p16 != kCellPadPos || q != (SQ_PAD | SQ_TIP)) return fail("padding code");
          if (prev_up) return fail("a contribution runs into padding");
          prev = -1;
          continue;
        }
        if (p16 == kCellPadPos || (int64_t)p16 >= m) return fail("position");
        if (((q & SQ_ROOT) != 0) != (p16 == 0)) return fail("root flag");
        const int32_t i = p16;
        if (seen[lo + i]++) return fail("compartment twice");
        const bool carry = !(q & SQ_TIP);
        if (carry != prev_up) return fail("carry flag");
        if (carry && (prev < 0 || parent[lo + prev] - lo != i)) return fail("carry from a non-child");
        const int rd = (q >> SQ_READ_SHIFT) & SQ_SLOT, dp = q & SQ_SLOT;
        if (rd) {
          if (rd > kSeqSlots || owner[rd] != i) return fail("slot read");
          owner[rd] = -1;
        }
        if (q & SQ_MBIN) {
          const int32_t from = (int32_t)(msl & 63u);
          msl >>= 6;
          if (from == c || ntake == 5 || mbin_step[from] >= 0) return fail("mailbox source");
          takes[ntake++] = from;
          mbin_step[from] = t;
          mbin_node[from] = i;
          mbin_lane[from] = c;
        }
        prev_up = false;
        if (q & SQ_MBOUT) {
          if (dp || i == 0) return fail("mailbox root");
          mbout_step[c] = t;
          mbout_node[c] = i;
        } else if (i == 0) {
          if (dp) return fail("cell root with a parent slot");
        } else if (dp) {
          const int32_t p = parent[lo + i] - (int32_t)lo;
          if (dp > kSeqSlots) return fail("slot id");
          if (q & SQ_FIRST) {
            if (owner[dp] != -1) return fail("slot taken");
            owner[dp] = p;
          } else if (owner[dp] != p) {
            return fail("slot of another parent");
          }
        } else {
          prev_up = true;
        }
        prev = i;
      }
      if (prev_up) return fail("contribution after the last step");
      uint64_t fw = 0;
      for (int32_t a = 0; a < ntake; ++a) fw |= (uint64_t)takes[a] << (6 * (ntake - 1 - a));
      if (msl != 0 || (src >> 32) != fw) return fail("mailbox source lists");
      for (int s = 1; s <= kSeqSlots; ++s)
        if (owner[s] != -1) return fail("slot never read");
    }
    // each mailbox: the receiver, the root's parent in the same cell, takes it strictly later
    for (int c = 0; c < 64; ++c) {
      if (mbout_step[c] < 0 && mbin_step[c] < 0) continue;
      const int64_t cell = Q.lane_cell[w * 64 + c];
      if (mbout_step[c] < 0 || mbin_step[c] <= mbout_step[c] || Q.lane_cell[w * 64 + mbin_lane[c]] != cell ||
          parent[cell_offsets[cell] + mbout_node[c]] - cell_offsets[cell] != mbin_node[c]) {
        why = "wave " + std::to_string(w) + " lane " + std::to_string(c) + ": mailbox order";
        return false;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (seen[i] != 1) {
      why = "compartment " + std::to_string(i) + " not walked once";
      return false;
    }
  return true;
}

}  // namespace hines

