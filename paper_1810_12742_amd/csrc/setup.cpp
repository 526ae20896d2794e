// Host-side setup of the fine-grained Hines solver (paper §4-§6).  O(N) in the
// number of compartments except for the per-(group, level) lane sorts.
//
// Rules (the paper leaves tie-breaks open; these are the ones this library
// fixes):
//  * branches: a compartment continues the branch of its parent q iff q has
//    exactly one child, the two are consecutive user indices, the step keeps
//    the branch's direction, and no user branch starts there (§2, §5);
//  * re-rooting: the tree centre, smaller user index on a tie (§6);
//  * numbering: branches breadth first, children by ascending user index of
//    their first compartment; compartments by distance to the root (§6);
//  * splitting: per level over all cells, cut at floor(level average) (§6);
//  * packing: greedy, every level's count <= group width (§4);
//  * lanes: per (group, level) by descending length, ties (cell, rank) (§4).
#include "setup.hpp"

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <numeric>

namespace hines {
namespace {

// Static chunk schedule of one group (the flow kernel).
//
// The group's branch tree is cut into heavy paths: a path starts at a branch
// that is a root or a light child and follows, at every branch end, the child
// whose elimination finishes last (as soon as possible, one compartment per
// step); a path therefore runs from a leaf up to its top branch.  One lane
// eliminates a whole path, kFlowChunk compartments per chunk step, from the
// leaf upward; the path is padded at its leaf end to a whole number of chunks
// with identity compartments (d = 1, u = 0, b = 0), which eliminate to zero
// and leave the next compartment untouched.  Inside a path the contribution
// to the next compartment stays in registers; a light path adds its top's
// contribution into its parent compartment in LDS, at least two chunk steps
// before the chunk that holds that compartment (operands are read one chunk
// step ahead).  Paths are placed latest deadline first, each on the lane where
// it can end latest, so light paths fill the gaps of the lanes.
struct SchedIn {
  int32_t len, parent, child0, nchild;
};

struct PathPlan {
  std::vector<int32_t> top_of;   // per branch: top branch of its path
  std::vector<int32_t> heavy;    // per branch: heavy child or -1
  std::vector<int32_t> below;    // per branch: compartments of its path below it (processed before it)
  std::vector<int32_t> plen;     // per path top: compartments of the path
  std::vector<int32_t> start;    // per path top: first chunk step
  std::vector<int32_t> lane;     // per path top: lane
  int32_t makespan = 0;          // chunk steps
};

static inline int32_t nchunks(int32_t len) { return (len + kFlowChunk - 1) / kFlowChunk; }

static bool schedule_paths(const std::vector<SchedIn>& br, PathPlan& pp) {
  const int32_t nb = (int32_t)br.size();
  const int32_t K = kFlowChunk;
  std::vector<int32_t> fin(nb);
  pp.heavy.assign(nb, -1);
  for (int32_t b = nb - 1; b >= 0; --b) {  // compartment-level as soon as possible: heavy children
    int32_t hf = 0, h = -1;
    for (int32_t c = br[b].child0; c < br[b].child0 + br[b].nchild; ++c)
      if (h < 0 || fin[c] > hf) {  // the child finishing last; the smallest id on ties
        hf = fin[c];
        h = c;
      }
    pp.heavy[b] = h;
    fin[b] = hf + br[b].len;
  }
  // paths: tops are roots and light children; below[b] = compartments of the
  // path under branch b (its heavy descendants)
  pp.top_of.assign(nb, -1);
  pp.below.assign(nb, 0);
  pp.plen.assign(nb, 0);
  std::vector<int32_t> tops;
  for (int32_t b = 0; b < nb; ++b) {
    const int32_t p = br[b].parent;
    if (p < 0 || pp.heavy[p] != b) {
      tops.push_back(b);
      int32_t len = 0;
      for (int32_t x = b; x >= 0; x = pp.heavy[x]) {
        pp.top_of[x] = b;
        len += br[x].len;
      }
      pp.plen[b] = len;
      int32_t acc = len;
      for (int32_t x = b; x >= 0; x = pp.heavy[x]) {
        acc -= br[x].len;
        pp.below[x] = acc;
      }
    }
  }
  // chunk index (within its parent path) of the compartment a light path attaches to:
  // the far end of its parent branch, processed right after the path part below it
  auto attach_chunk = [&](int32_t top) {
    const int32_t pb = br[top].parent;
    const int32_t q = pp.top_of[pb];
    const int32_t npad = nchunks(pp.plen[q]) * K - pp.plen[q];
    return (npad + pp.below[pb]) / K;
  };
  // as soon as possible in chunk steps (tops in descending id: light children first)
  std::vector<int32_t> pfin(nb, 0), kids_begin, kids;  // light child paths per path
  std::vector<std::vector<int32_t>> light(nb);
  for (int32_t t : tops)
    if (br[t].parent >= 0) light[pp.top_of[br[t].parent]].push_back(t);
  for (auto it = tops.rbegin(); it != tops.rend(); ++it) {
    const int32_t q = *it;
    int32_t s = 0;
    for (int32_t l : light[q]) s = std::max(s, pfin[l] + 1 - attach_chunk(l));
    pfin[q] = s + nchunks(pp.plen[q]);
  }
  int32_t F = 0, total = 0;
  for (int32_t q : tops) {
    if (br[q].parent < 0) F = std::max(F, pfin[q]);
    total += nchunks(pp.plen[q]);
  }
  pp.start.assign(nb, 0);
  pp.lane.assign(nb, 0);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> busy(kSchedLanes);
  struct Item {
    int32_t deadline, top;
  };
  std::vector<Item> work;
  for (; F <= 2 * total + 2 && F <= kMaxSteps; ++F) {
    for (auto& v : busy) v.clear();
    work.clear();
    for (int32_t q : tops)
      if (br[q].parent < 0) work.push_back({F, q});
    bool ok = true;
    while (!work.empty()) {
      size_t pick = 0;  // latest deadline first; longer path first; smaller id
      for (size_t k = 1; k < work.size(); ++k) {
        const Item &a = work[k], &bb = work[pick];
        const int32_t la = nchunks(pp.plen[a.top]), lb = nchunks(pp.plen[bb.top]);
        if (a.deadline > bb.deadline || (a.deadline == bb.deadline && la > lb) ||
            (a.deadline == bb.deadline && la == lb && a.top < bb.top))
          pick = k;
      }
      const Item it = work[pick];
      work.erase(work.begin() + (std::ptrdiff_t)pick);
      const int32_t L = nchunks(pp.plen[it.top]);
      int32_t best_end = -1, best_lane = -1;
      for (int32_t ln = 0; ln < kSchedLanes; ++ln) {
        int32_t end = it.deadline;
        const auto& iv = busy[ln];  // sorted by start
        for (int64_t k = (int64_t)iv.size() - 1; k >= 0; --k) {
          if (iv[k].first >= end) continue;    // entirely after the window end
          if (iv[k].second <= end - L) break;  // gap [iv.second, end) fits
          end = iv[k].first;                   // move the window before this interval
        }
        if (end - L >= 0 && end > best_end) {
          best_end = end;
          best_lane = ln;
        }
      }
      if (best_lane < 0) {
        ok = false;
        break;
      }
      auto& iv = busy[best_lane];
      iv.push_back({best_end - L, best_end});
      std::sort(iv.begin(), iv.end());
      pp.start[it.top] = best_end - L;
      pp.lane[it.top] = best_lane;
      for (int32_t l : light[it.top]) work.push_back({best_end - L + attach_chunk(l) - 1, l});
    }
    if (ok) {
      pp.makespan = F;
      return true;
    }
  }
  return false;
}

static inline int popc64(uint64_t m) { return __builtin_popcountll(m); }

struct Builder {
  const int32_t* parent;
  int64_t n;
  const int64_t* boff;
  int64_t nb_user;
  const int64_t* coff;
  int64_t ncells;
  Options opt;
  HostPlan& P;
  std::string& err;

  // branch records (creation order; tails of splits are appended)
  std::vector<int32_t> bfirst, bdir, blen, bparent, bcell, btail, bcl_lo, bcl_hi;
  std::vector<int32_t> clist;      // children lists (ascending first compartment)
  std::vector<int32_t> root_br;    // root branch of each cell
  std::vector<int32_t> npar;       // parent in the (re-rooted) orientation

  Builder(const int32_t* p, int64_t n_, const int64_t* bo, int64_t nb, const int64_t* co, int64_t nc,
          const Options& o, HostPlan& out, std::string& e)
      : parent(p), n(n_), boff(bo), nb_user(nb), coff(co), ncells(nc), opt(o), P(out), err(e) {}

  Status fail(Status s, const std::string& m) {
    err = m;
    return s;
  }

  Status validate() {
    if (n < 0 || ncells < 0) return fail(ERR_BAD_OFFSETS, "negative size");
    if (n > INT32_MAX) return fail(ERR_BAD_OFFSETS, "more than 2^31-1 compartments");
    if (ncells > INT32_MAX) return fail(ERR_BAD_OFFSETS, "too many cells");
    if (n > 0 && !parent) return fail(ERR_NULL, "parent is NULL");
    if (!coff) return fail(ERR_NULL, "cell_offsets is NULL");
    if (opt.group_width < 64 || opt.group_width > 1024 || opt.group_width % 64)
      return fail(ERR_OPTION, "group_width must be a multiple of 64 in [64, 1024]");
    if (opt.cell_order != 0 && opt.cell_order != 1) return fail(ERR_OPTION, "cell_order must be 0 or 1");
    if (opt.split_branches < 0 || opt.split_branches > 2) return fail(ERR_OPTION, "split_branches must be 0, 1 or 2");
    if (opt.level_balance != 0 && opt.level_balance != 1) return fail(ERR_OPTION, "level_balance must be 0 or 1");
    if (opt.max_group_unknowns < 0) return fail(ERR_OPTION, "max_group_unknowns < 0");
    if (coff[0] != 0 || coff[ncells] != n) return fail(ERR_BAD_OFFSETS, "cell_offsets must run from 0 to n");
    for (int64_t c = 0; c < ncells; ++c)
      if (coff[c + 1] <= coff[c]) return fail(ERR_BAD_OFFSETS, "cells must be non-empty and increasing");
    for (int64_t c = 0; c < ncells; ++c) {
      int64_t lo = coff[c], hi = coff[c + 1];
      if (parent[lo] != -1) return fail(ERR_BAD_PARENT, "root " + std::to_string(lo) + " must have parent -1");
      for (int64_t i = lo + 1; i < hi; ++i)
        if (!(parent[i] >= lo && parent[i] < i))
          return fail(ERR_BAD_PARENT, "parent[" + std::to_string(i) + "] out of [cell start, i)");
    }
    if (boff) {
      if (nb_user < (n > 0 ? 1 : 0)) return fail(ERR_BAD_BRANCHES, "empty branch layout");
      if (boff[0] != 0 || boff[nb_user] != n) return fail(ERR_BAD_BRANCHES, "branch_offsets must run from 0 to n");
      for (int64_t k = 0; k < nb_user; ++k) {
        if (boff[k + 1] <= boff[k]) return fail(ERR_BAD_BRANCHES, "branches must be non-empty and increasing");
        for (int64_t i = boff[k] + 1; i < boff[k + 1]; ++i)
          if (parent[i] != i - 1) return fail(ERR_BAD_BRANCHES, "parent[i] != i-1 inside a branch");
      }
      // every cell start must be a branch start (both arrays ascending)
      int64_t k = 0;
      for (int64_t c = 0; c < ncells; ++c) {
        while (k < nb_user && boff[k] < coff[c]) ++k;
        if (k >= nb_user || boff[k] != coff[c]) return fail(ERR_BAD_BRANCHES, "a branch crosses a cell start");
      }
    }
    return OK;
  }

  // Re-root every cell at its centre; fills npar and a parent-first order.
  void reroot(std::vector<int32_t>& order) {
    order.resize(n);
    int64_t maxm = 0;
    for (int64_t c = 0; c < ncells; ++c) maxm = std::max(maxm, coff[c + 1] - coff[c]);
    std::vector<int32_t> deg(maxm + 1), adj(2 * std::max<int64_t>(maxm - 1, 0)), dist(maxm), prev(maxm),
        q(maxm);
    for (int64_t c = 0; c < ncells; ++c) {
      const int32_t lo = (int32_t)coff[c];
      const int32_t m = (int32_t)(coff[c + 1] - coff[c]);
      std::fill(deg.begin(), deg.begin() + m + 1, 0);
      for (int32_t i = 1; i < m; ++i) {
        ++deg[i + 1];
        ++deg[parent[lo + i] - lo + 1];
      }
      for (int32_t i = 0; i < m; ++i) deg[i + 1] += deg[i];
      std::vector<int32_t> fillpos(deg.begin(), deg.begin() + m);
      for (int32_t i = 1; i < m; ++i) {
        int32_t p = parent[lo + i] - lo;
        adj[fillpos[i]++] = p;
        adj[fillpos[p]++] = i;
      }
      auto bfs = [&](int32_t s) -> int32_t {  // returns farthest node (smallest index on ties)
        std::fill(dist.begin(), dist.begin() + m, -1);
        int32_t head = 0, tail = 0;
        q[tail++] = s;
        dist[s] = 0;
        prev[s] = -1;
        while (head < tail) {
          int32_t v = q[head++];
          for (int32_t e = deg[v]; e < deg[v + 1]; ++e) {
            int32_t w = adj[e];
            if (dist[w] < 0) {
              dist[w] = dist[v] + 1;
              prev[w] = v;
              q[tail++] = w;
            }
          }
        }
        int32_t far = 0, best = s;
        for (int32_t v = 0; v < m; ++v)
          if (dist[v] > far || (dist[v] == far && v < best)) {
            far = dist[v];
            best = v;
          }
        return best;
      };
      int32_t a = bfs(0);
      int32_t b = bfs(a);
      int32_t D = dist[b];
      // path b -> a through prev; position k from a is node at distance k
      std::vector<int32_t> path;
      path.reserve(D + 1);
      for (int32_t v = b; v != -1; v = prev[v]) path.push_back(v);
      std::reverse(path.begin(), path.end());
      int32_t centre = std::min(path[D / 2], path[(D + 1) / 2]);
      // orientation away from the centre, breadth first
      std::fill(dist.begin(), dist.begin() + m, -1);
      int32_t head = 0, tail = 0;
      q[tail++] = centre;
      dist[centre] = 0;
      npar[lo + centre] = -1;
      while (head < tail) {
        int32_t v = q[head++];
        order[lo + head - 1] = lo + v;
        for (int32_t e = deg[v]; e < deg[v + 1]; ++e) {
          int32_t w = adj[e];
          if (dist[w] < 0) {
            dist[w] = 0;
            npar[lo + w] = lo + v;
            q[tail++] = w;
          }
        }
      }
    }
  }

  int32_t new_branch(int32_t first, int32_t par, int32_t cell) {
    int32_t id = (int32_t)bfirst.size();
    bfirst.push_back(first);
    bdir.push_back(1);
    blen.push_back(1);
    bparent.push_back(par);
    bcell.push_back(cell);
    return id;
  }

  Status run() {
    Status s = validate();
    if (s != OK) return s;
    P.n = n;
    P.ncells = ncells;
    P.opt = opt;

    // ---- orientation ----
    npar.assign(parent, parent + n);
    std::vector<int32_t> order;
    if (opt.rebalance_root) reroot(order);
    std::vector<uint8_t> nch(n, 0);
    for (int64_t i = 0; i < n; ++i)
      if (npar[i] >= 0 && nch[npar[i]] < 2) ++nch[npar[i]];
    std::vector<uint8_t> ustart;
    if (boff && !opt.rebalance_root) {
      ustart.assign(n, 0);
      for (int64_t k = 0; k < nb_user; ++k) ustart[boff[k]] = 1;
    }

    // ---- branches ----
    std::vector<int32_t> br(n);
    root_br.assign(ncells, -1);
    for (int64_t c = 0; c < ncells; ++c) {
      for (int64_t k = coff[c]; k < coff[c + 1]; ++k) {
        int32_t i = opt.rebalance_root ? order[k] : (int32_t)k;
        int32_t qn = npar[i];
        if (qn < 0) {
          br[i] = new_branch(i, -1, (int32_t)c);
          root_br[c] = br[i];
          continue;
        }
        int32_t bq = br[qn];
        bool qfirst = bfirst[bq] == qn;
        int32_t step = i - qn;
        bool cont = nch[qn] == 1 && (step == 1 || step == -1) && (qfirst || step == bdir[bq]) &&
                    !(!ustart.empty() && ustart[i]);
        if (cont) {
          if (qfirst) bdir[bq] = step;
          ++blen[bq];
          br[i] = bq;
        } else {
          br[i] = new_branch(i, bq, (int32_t)c);
        }
      }
    }
    std::vector<uint8_t>().swap(nch);
    std::vector<uint8_t>().swap(ustart);
    std::vector<int32_t>().swap(order);
    const int64_t nb0 = (int64_t)bfirst.size();
    // children lists, ascending first compartment
    bcl_lo.assign(nb0, 0);
    bcl_hi.assign(nb0, 0);
    btail.assign(nb0, -1);
    {
      std::vector<int32_t> cnt(nb0 + 1, 0);
      for (int64_t b = 0; b < nb0; ++b)
        if (bparent[b] >= 0) ++cnt[bparent[b] + 1];
      for (int64_t b = 0; b < nb0; ++b) cnt[b + 1] += cnt[b];
      for (int64_t b = 0; b < nb0; ++b) {
        bcl_lo[b] = cnt[b];
        bcl_hi[b] = cnt[b];
      }
      clist.assign(cnt[nb0], 0);
      for (int64_t i = 0; i < n; ++i) {
        int32_t b = br[i];
        if (bfirst[b] == i && bparent[b] >= 0) clist[bcl_hi[bparent[b]]++] = b;
      }
    }
    std::vector<int32_t>().swap(br);

    // packing order of the cells (§4)
    std::vector<int64_t> cells(ncells);
    std::iota(cells.begin(), cells.end(), 0);
    if (opt.cell_order == 1)
      std::stable_sort(cells.begin(), cells.end(),
                       [&](int64_t a, int64_t b) { return coff[a + 1] - coff[a] > coff[b + 1] - coff[b]; });
    const int32_t T = opt.group_width;
    const int64_t cap = opt.max_group_unknowns;

    // ---- split (level by level over all cells, or inside the groups of an
    // intermediate packing of the unsplit trees: the outlook of §8) ----
    auto split_from = [&](std::vector<int32_t> cur) {
      std::vector<int32_t> nxt;
      while (!cur.empty()) {
        int64_t S = 0;
        for (int32_t b : cur) S += blen[b];
        const int64_t m = (int64_t)cur.size();
        nxt.clear();
        for (int32_t b : cur) {
          if ((int64_t)blen[b] * m > S) {
            int32_t k = (int32_t)(S / m);
            int32_t t = (int32_t)bfirst.size();
            bfirst.push_back(bfirst[b] + bdir[b] * k);
            bdir.push_back(bdir[b]);
            blen.push_back(blen[b] - k);
            bparent.push_back(b);
            bcell.push_back(bcell[b]);
            btail.push_back(-1);
            bcl_lo.push_back(bcl_lo[b]);
            bcl_hi.push_back(bcl_hi[b]);
            for (int32_t e = bcl_lo[b]; e < bcl_hi[b]; ++e) bparent[clist[e]] = t;
            bcl_lo[b] = bcl_hi[b] = 0;
            btail[b] = t;
            blen[b] = k;
          }
          if (btail[b] >= 0)
            nxt.push_back(btail[b]);
          else
            for (int32_t e = bcl_lo[b]; e < bcl_hi[b]; ++e) nxt.push_back(clist[e]);
        }
        cur.swap(nxt);
      }
    };
    if (opt.split_branches == 1) split_from(std::vector<int32_t>(root_br.begin(), root_br.end()));
    if (opt.split_branches == 2) {
      // intermediate packing (S7 without level balancing) on the natural levels
      std::vector<int32_t> gc, lvl, nxtl, roots;
      int64_t gU = 0;
      auto natural = [&](int64_t c, std::vector<int32_t>& cnt) {
        cnt.clear();
        lvl.assign(1, root_br[c]);
        while (!lvl.empty()) {
          cnt.push_back((int32_t)lvl.size());
          nxtl.clear();
          for (int32_t b : lvl)
            for (int32_t e = bcl_lo[b]; e < bcl_hi[b]; ++e) nxtl.push_back(clist[e]);
          lvl.swap(nxtl);
        }
      };
      std::vector<int32_t> cc;
      for (int64_t c : cells) {
        natural(c, cc);
        const int64_t sz = coff[c + 1] - coff[c];
        bool fits = true;
        if (!roots.empty()) {
          for (size_t l = 0; l < cc.size() && fits; ++l)
            if ((l < gc.size() ? gc[l] : 0) + cc[l] > T) fits = false;
          if (cap && gU + sz > cap) fits = false;
        }
        if (!fits) {
          split_from(roots);
          roots.clear();
          gc.clear();
          gU = 0;
        }
        roots.push_back(root_br[c]);
        if (gc.size() < cc.size()) gc.resize(cc.size(), 0);
        for (size_t l = 0; l < cc.size(); ++l) gc[l] += cc[l];
        gU += sz;
      }
      if (!roots.empty()) split_from(roots);
    }
    const int64_t nb = (int64_t)bfirst.size();
    P.nbranches = nb;

    // ---- breadth-first numbering, levels ----
    std::vector<int32_t> gorder;  // gid -> creation id
    gorder.reserve(nb);
    std::vector<int32_t> glevel(nb), grank(nb), gfchild(nb, -1), gnchild(nb, 0), gid_of(nb);
    std::vector<int64_t> cell_br_lo(ncells + 1, 0);
    for (int64_t c = 0; c < ncells; ++c) {
      int64_t head = (int64_t)gorder.size();
      cell_br_lo[c] = head;
      gorder.push_back(root_br[c]);
      glevel[head] = 0;
      for (int64_t k = head; k < (int64_t)gorder.size(); ++k) {
        int32_t b = gorder[k];
        grank[k] = (int32_t)(k - head);
        int32_t first = (int32_t)gorder.size();
        int32_t cntc = 0;
        if (btail[b] >= 0) {
          glevel[gorder.size()] = glevel[k] + 1;
          gorder.push_back(btail[b]);
          cntc = 1;
        } else {
          for (int32_t e = bcl_lo[b]; e < bcl_hi[b]; ++e) {
            glevel[gorder.size()] = glevel[k] + 1;
            gorder.push_back(clist[e]);
            ++cntc;
          }
        }
        if (cntc) {
          gfchild[k] = first;
          gnchild[k] = cntc;
        }
      }
    }
    cell_br_lo[ncells] = (int64_t)gorder.size();
    for (int64_t k = 0; k < nb; ++k) gid_of[gorder[k]] = (int32_t)k;
    std::vector<int32_t>().swap(clist);
    std::vector<int32_t>().swap(bcl_lo);
    std::vector<int32_t>().swap(bcl_hi);
    std::vector<int32_t>().swap(btail);

    // per gid branch fields
    std::vector<int32_t> gfirst(nb), gdir(nb), glen(nb), gparent(nb), gcell(nb);
    for (int64_t k = 0; k < nb; ++k) {
      int32_t b = gorder[k];
      gfirst[k] = bfirst[b];
      gdir[k] = bdir[b];
      glen[k] = blen[b];
      gparent[k] = bparent[b] >= 0 ? gid_of[bparent[b]] : -1;
      gcell[k] = bcell[b];
    }
    for (auto* v : {&bfirst, &bdir, &blen, &bparent, &bcell, &gorder, &gid_of, &root_br})
      std::vector<int32_t>().swap(*v);
    int32_t maxlev = -1;

    // ---- node numbering and coupling sources ----
    std::vector<int32_t> node_plan(n), u_src(n);
    {
      int64_t off = 0;
      int32_t curcell = -1;
      for (int64_t k = 0; k < nb; ++k) {
        if (gcell[k] != curcell) {
          curcell = gcell[k];
          off = coff[curcell];
        }
        for (int32_t j = 0; j < glen[k]; ++j) node_plan[gfirst[k] + gdir[k] * j] = (int32_t)(off + j);
        for (int32_t j = 0; j < glen[k]; ++j) {
          int32_t i = gfirst[k] + gdir[k] * j;
          int32_t qn;
          if (j > 0)
            qn = i - gdir[k];
          else if (gparent[k] >= 0) {
            int32_t pb = gparent[k];
            qn = gfirst[pb] + gdir[pb] * (glen[pb] - 1);
          } else {
            u_src[off + j] = -1;
            continue;
          }
          u_src[off + j] = (parent[i] == qn) ? i : qn;  // flipped edge: stored at the old child
        }
        off += glen[k];
      }
    }

    // ---- packing (§4; with level balancing, the outlook of §8) ----
    // slev: the level of each branch in the level-synchronous sweeps; the
    // breadth-first depth unless packing moved its subtree down
    std::vector<int32_t> slev(glevel.begin(), glevel.end());
    std::vector<int32_t> subn(nb, 1);  // branches in each branch's subtree
    for (int64_t k = nb - 1; k >= 0; --k)
      for (int32_t j = 0; j < gnchild[k]; ++j) subn[k] += subn[gfchild[k] + j];
    std::vector<int32_t> gcnt, ccnt, trial, stk;
    auto cell_counts = [&](int64_t c, const int32_t* lv, std::vector<int32_t>& cnt) {
      cnt.clear();
      for (int64_t k = cell_br_lo[c]; k < cell_br_lo[c + 1]; ++k) {
        const int32_t l = lv[k - cell_br_lo[c]];
        if ((int32_t)cnt.size() <= l) cnt.resize(l + 1, 0);
        ++cnt[l];
      }
    };
    // the smallest level on which the cell has branches and overflows the
    // open group, or -1
    auto overflow = [&](const std::vector<int32_t>& cnt) {
      for (size_t l = 0; l < cnt.size(); ++l)
        if (cnt[l] > 0 && (l < gcnt.size() ? gcnt[l] : 0) + cnt[l] > T) return (int32_t)l;
      return (int32_t)-1;
    };
    P.group_offsets.assign(1, 0);
    P.group_cells.clear();
    P.group_cells.reserve(ncells);
    {
      int64_t gU = 0;
      for (int64_t c : cells) {
        const int64_t kb = cell_br_lo[c], nbc = cell_br_lo[c + 1] - kb;
        const int64_t sz = coff[c + 1] - coff[c];
        bool open = (int64_t)P.group_cells.size() > P.group_offsets.back();
        cell_counts(c, slev.data() + kb, ccnt);
        bool fits = true;
        if (open) {
          const bool cap_ok = !(cap && gU + sz > cap);
          fits = cap_ok && overflow(ccnt) < 0;
          if (!fits && cap_ok && opt.level_balance) {
            trial.assign(slev.begin() + kb, slev.begin() + kb + nbc);
            int64_t moves = 0;
            for (;;) {
              cell_counts(c, trial.data(), ccnt);
              const int32_t l = overflow(ccnt);
              if (l < 0) {
                fits = true;
                break;
              }
              if (l == 0 || moves >= 4 * nbc) break;
              int64_t pick = -1;  // fewest branches in the subtree, then the smallest rank
              for (int64_t r = 0; r < nbc; ++r)
                if (trial[r] == l && (pick < 0 || subn[kb + r] < subn[kb + pick])) pick = r;
              stk.assign(1, (int32_t)(kb + pick));
              while (!stk.empty()) {
                const int32_t x = stk.back();
                stk.pop_back();
                ++trial[x - kb];
                for (int32_t j = 0; j < gnchild[x]; ++j) stk.push_back(gfchild[x] + j);
              }
              ++moves;
            }
            if (fits) std::copy(trial.begin(), trial.end(), slev.begin() + kb);
            else cell_counts(c, slev.data() + kb, ccnt);
          }
        }
        if (open && !fits) {
          P.group_offsets.push_back((int64_t)P.group_cells.size());
          gcnt.clear();
          gU = 0;
        }
        P.group_cells.push_back(c);
        if (gcnt.size() < ccnt.size()) gcnt.resize(ccnt.size(), 0);
        for (size_t l = 0; l < ccnt.size(); ++l) gcnt[l] += ccnt[l];
        gU += sz;
      }
      if ((int64_t)P.group_cells.size() > P.group_offsets.back())
        P.group_offsets.push_back((int64_t)P.group_cells.size());
    }
    std::copy(slev.begin(), slev.end(), glevel.begin());
    for (int64_t k = 0; k < nb; ++k) maxlev = std::max(maxlev, glevel[k]);
    P.max_level = maxlev;
    // per cell: its branches ordered by level (stable in breadth-first order)
    // and the first entry of each level
    std::vector<int64_t> cnt_off(ncells + 1, 0);
    std::vector<int32_t> by_lev(nb);
    for (int64_t c = 0; c < ncells; ++c) {
      int32_t nl = 0;
      for (int64_t k = cell_br_lo[c]; k < cell_br_lo[c + 1]; ++k) nl = std::max(nl, glevel[k] + 1);
      cnt_off[c + 1] = cnt_off[c] + nl;
    }
    std::vector<int32_t> lvl_lo(cnt_off[ncells] + ncells, 0);  // lvl_lo[cnt_off[c] + c + l]: first entry of level l
    for (int64_t c = 0; c < ncells; ++c) {
      const int64_t base = cnt_off[c] + c, kb = cell_br_lo[c];
      const int32_t nl = (int32_t)(cnt_off[c + 1] - cnt_off[c]);
      for (int64_t k = kb; k < cell_br_lo[c + 1]; ++k) ++lvl_lo[base + glevel[k] + 1];
      for (int32_t l = 0; l < nl; ++l) lvl_lo[base + l + 1] += lvl_lo[base + l];
      std::vector<int32_t> fillp(lvl_lo.begin() + base, lvl_lo.begin() + base + nl);
      for (int64_t k = kb; k < cell_br_lo[c + 1]; ++k) by_lev[kb + fillp[glevel[k]]++] = (int32_t)k;
    }
    const int64_t ng = (int64_t)P.group_offsets.size() - 1;
    P.ngroups = ng;
    std::vector<int32_t> group_of_cell(ncells, 0);
    for (int64_t g = 0; g < ng; ++g)
      for (int64_t e = P.group_offsets[g]; e < P.group_offsets[g + 1]; ++e) group_of_cell[P.group_cells[e]] = (int32_t)g;

    // ---- lanes (§4, Fig 4.1) and kernel tables ----
    P.kgroup.assign(ng, KGroup{});
    P.kcell.assign(ncells, KCell{});
    P.kbranch.assign(nb, KBranch{});
    P.lanes.assign(nb, 0);
    P.kseg.clear();
    P.group_seg_offsets.assign(ng + 1, 0);
    std::vector<int32_t> cell_lds(ncells, 0), cell_gbr(ncells, 0);  // per cell: LDS offset, first group-local id
    int64_t lane = 0;
    std::vector<int32_t> seg;
    for (int64_t g = 0; g < ng; ++g) {
      KGroup& G = P.kgroup[g];
      G.seg_begin = (int32_t)P.kseg.size();
      G.cell_begin = (int32_t)P.group_offsets[g];
      G.ncell = (int32_t)(P.group_offsets[g + 1] - P.group_offsets[g]);
      int64_t U = 0, nbr = 0;
      int32_t gnl = 0;
      // Contiguous groups (consecutive cells) keep the user layout in LDS:
      // slot k holds user index user_base + k with user_base even, so one
      // aligned range copy stages the whole group.  Others: each cell starts
      // at an even slot.
      bool contig = true;
      for (int64_t e = P.group_offsets[g] + 1; e < P.group_offsets[g + 1]; ++e)
        if (P.group_cells[e] != P.group_cells[e - 1] + 1) contig = false;
      const int64_t c_first = P.group_cells[P.group_offsets[g]];
      const int64_t ubase = coff[c_first] & ~(int64_t)1;
      G.ws_off = -1;
      G.contig = contig ? 1 : 0;
      G.user_base = contig ? ubase : 0;
      G.user_lo = contig ? (int32_t)(coff[c_first] - ubase) : 0;
      G.user_n = 0;
      G.makespan = 0;
      U = kLdsPad + (contig ? coff[c_first] - ubase : 0);
      for (int64_t e = P.group_offsets[g]; e < P.group_offsets[g + 1]; ++e) {
        int64_t c = P.group_cells[e];
        if (!contig) U = (U + 1) & ~(int64_t)1;  // each cell starts 16-byte aligned in the LDS image
        G.user_n += (int32_t)(coff[c + 1] - coff[c]);
        cell_lds[c] = (int32_t)U;
        cell_gbr[c] = (int32_t)nbr;
        P.kcell[e] = KCell{coff[c], (int32_t)(coff[c + 1] - coff[c]), (int32_t)U};
        U += coff[c + 1] - coff[c];
        nbr += cell_br_lo[c + 1] - cell_br_lo[c];
        gnl = std::max(gnl, (int32_t)(cnt_off[c + 1] - cnt_off[c]));
      }
      U = (U + kLdsPad + 1) & ~(int64_t)1;  // back padding, even size
      G.nunk = (int32_t)std::min<int64_t>(U, INT32_MAX);
      G.nbr = (int32_t)nbr;
      G.nlev = gnl;
      G.br_begin = (int32_t)lane;
      int64_t cost = 0;
      for (int32_t l = 0; l < gnl; ++l) {
        seg.clear();
        for (int64_t e = P.group_offsets[g]; e < P.group_offsets[g + 1]; ++e) {
          int64_t c = P.group_cells[e];
          int32_t nl = (int32_t)(cnt_off[c + 1] - cnt_off[c]);
          if (l >= nl) continue;
          int64_t base = cnt_off[c] + c;
          for (int32_t r = lvl_lo[base + l]; r < lvl_lo[base + l + 1]; ++r) seg.push_back(by_lev[cell_br_lo[c] + r]);
        }
        std::sort(seg.begin(), seg.end(), [&](int32_t a, int32_t b) {
          if (glen[a] != glen[b]) return glen[a] > glen[b];
          if (gcell[a] != gcell[b]) return gcell[a] < gcell[b];
          return grank[a] < grank[b];
        });
        P.kseg.push_back((int32_t)lane);
        for (size_t t = 0; t < seg.size(); t += (size_t)T) cost += glen[seg[t]];
        for (int32_t k : seg) {
          P.lanes[lane] = k;
          const int32_t c = gcell[k];
          auto local = [&](int32_t user) { return cell_lds[c] + (int32_t)(user - coff[c]); };
          int32_t f_start = local(gfirst[k]);
          int32_t f_lendir = gdir[k] > 0 ? glen[k] : -glen[k];
          if (gdir[k] < 0) P.all_ascending = false;
          int32_t f_u0 = -1, f_pslot = -1;
          if (gparent[k] >= 0) {
            int32_t pb = gparent[k];
            int32_t plast = gfirst[pb] + gdir[pb] * (glen[pb] - 1);
            f_pslot = local(plast);
            f_u0 = local(u_src[node_plan[gfirst[k]]]);
          }
          int32_t f_self = cell_gbr[c] + grank[k];
          int32_t f_child0 = gnchild[k] ? cell_gbr[c] + grank[gfchild[k]] : 0;
          KBranch& B = P.kbranch[lane];
          if (U > kMaxGroupSlots || nbr > kMaxGroupSlots) {
            P.kernel_tables_fit = false;
            B = KBranch{};
          } else {
            B.start = (int16_t)f_start;
            B.lendir = (int16_t)f_lendir;
            B.u0 = (int16_t)f_u0;
            B.pslot = (int16_t)f_pslot;
            B.self = (int16_t)f_self;
            B.child0 = (int16_t)f_child0;
            B.nchild = (int16_t)gnchild[k];
            B.pad = 0;
          }
          ++lane;
        }
      }
      G.cost = (int32_t)std::min<int64_t>(cost, INT32_MAX);
      P.group_seg_offsets[g + 1] = (int64_t)P.kseg.size();
    }
    P.kseg.push_back((int32_t)lane);
    P.nseg = (int64_t)P.kseg.size() - 1;

    // ---- groups whose image exceeds LDS run from a global workspace ----
    P.ws_doubles = 0;
    for (int64_t g = 0; g < ng; ++g) {
      KGroup& G = P.kgroup[g];
      const LdsLayout lds{G.nunk, (G.nbr + 1) & ~1, G.nlev};
      if (lds.bytes() > kLdsLimitBytes) {
        G.ws_off = P.ws_doubles;
        P.ws_doubles += 3 * (int64_t)G.nunk;
      }
    }

    // ---- static chunk schedule and flow tables (ascending plans, LDS groups) ----
    // Every child branch must hang off the far end of its parent (always true
    // for maximal chains and splits; user layouts may attach mid-branch).
    bool tips_only = true;
    for (int64_t g = 0; g < ng && tips_only; ++g) {
      const KGroup& G = P.kgroup[g];
      std::vector<int32_t> rec_of(G.nbr, -1);
      for (int32_t r = 0; r < G.nbr; ++r) rec_of[P.kbranch[G.br_begin + r].self] = r;
      for (int32_t r = 0; r < G.nbr && tips_only; ++r) {
        const KBranch& B = P.kbranch[G.br_begin + r];
        for (int32_t c = B.child0; c < B.child0 + B.nchild; ++c)
          if (P.kbranch[G.br_begin + rec_of[c]].pslot != B.start + B.lendir - 1) tips_only = false;
      }
    }
    if (opt.scheduler && !opt.bitwise && P.all_ascending && P.kernel_tables_fit && tips_only) {
      const int32_t K = kFlowChunk;
      P.kflow.assign(ng, KFlow{});
      std::vector<SchedIn> sin;
      std::vector<int32_t> slot_elem, R, tops;
      std::vector<uint64_t> M, E;
      PathPlan pp;
      bool all_ok = true;
      int64_t steps = 0, elems = 0;
      for (int64_t g = 0; g < ng && all_ok; ++g) {
        const KGroup& G = P.kgroup[g];
        KFlow& W = P.kflow[g];
        W.step_off = steps;
        W.pos_off = elems;
        if (P.faux.size() & 1) P.faux.push_back(0);  // 4-byte aligned start of the group's push targets
        W.aux_off = (int64_t)P.faux.size();
        if (G.ws_off >= 0) continue;  // level-synchronous from the workspace (all counts 0)
        const int32_t nbg = G.nbr;
        sin.assign(nbg, SchedIn{0, -1, 0, 0});
        std::vector<int32_t> rec_of(nbg, -1);  // group-local BFS id -> record
        for (int32_t r = 0; r < nbg; ++r) {
          const KBranch& B = P.kbranch[G.br_begin + r];
          rec_of[B.self] = r;
          sin[B.self] = SchedIn{B.lendir, -1, B.child0, B.nchild};
        }
        for (int32_t b = 0; b < nbg; ++b)
          for (int32_t c = sin[b].child0; c < sin[b].child0 + sin[b].nchild; ++c) sin[c].parent = b;
        if (!schedule_paths(sin, pp)) {
          all_ok = false;
          break;
        }
        const int32_t F = pp.makespan;
        M.assign(F, 0);
        E.assign(F, 0);
        tops.clear();
        for (int32_t b = 0; b < nbg; ++b)
          if (pp.top_of[b] == b) {
            tops.push_back(b);
            const int32_t s = pp.start[b], n = nchunks(pp.plen[b]);
            for (int32_t i = 0; i < n; ++i) M[s + i] |= 1ull << pp.lane[b];
            if (sin[b].parent >= 0) E[s + n - 1] |= 1ull << pp.lane[b];
          }
        R.assign(F + 1, 0);  // lane-chunks (blocks) before chunk step t
        for (int32_t t = 0; t < F; ++t) R[t + 1] = R[t] + popc64(M[t]);
        const int32_t nent = K * R[F];
        // LDS offset (8-byte units) of sub-step j of chunk step t on lane l:
        // block (R[t] + rank of l) of kFlowBlock8 units, entry j at 3 j
        auto entry = [&](int32_t t, int32_t j, int32_t l) {
          return (R[t] + popc64(M[t] & ((1ull << l) - 1))) * kFlowBlock8 + 3 * j;
        };
        // entry of the compartment with processing index idx (pads first) of path q
        auto entry_of = [&](int32_t q, int32_t idx) {
          return entry(pp.start[q] + idx / K, idx % K, pp.lane[q]);
        };
        slot_elem.assign(G.nunk, -1);
        int32_t cum = 0;
        for (int c = 0; c < G.ncell; ++c) {
          const KCell& C = P.kcell[G.cell_begin + c];
          for (int32_t k = 0; k < C.n; ++k) slot_elem[C.lds + k] = cum + k;
          cum += C.n;
        }
        if (cum != G.user_n || (int64_t)R[F] * kFlowBlock8 + kFlowTail8 > 32767) {
          all_ok = false;
          break;
        }
        W.nstep = F;
        W.nelem = cum;
        W.nent = nent;
        W.makespan = F;
        if (flow_lds_bytes(W) > kLdsLimitBytes) {  // e.g. very long single branches: level kernel
          W = KFlow{};
          W.step_off = steps;
          W.pos_off = elems;
          W.aux_off = (int64_t)P.faux.size();
          continue;
        }
        P.fpos.resize(elems + cum);
        for (int32_t q : tops) {
          const int32_t npad = nchunks(pp.plen[q]) * K - pp.plen[q];
          for (int32_t x = q; x >= 0; x = pp.heavy[x]) {
            const KBranch& B = P.kbranch[G.br_begin + rec_of[x]];
            for (int32_t k = 0; k < sin[x].len; ++k) {
              // far end (k = len - 1) first
              const int32_t idx = npad + pp.below[x] + (sin[x].len - 1 - k);
              uint32_t p = (uint32_t)entry_of(q, idx);
              if (k == 0 && sin[x].parent < 0) p |= 0x8000u;  // the cell's root: no coupling
              P.fpos[elems + slot_elem[B.start + k]] = (uint16_t)p;
            }
          }
        }
        // push targets in (chunk step, lane) order: the far end of the parent branch
        std::vector<int32_t> end_top((int64_t)F * kSchedLanes, -1);
        for (int32_t q : tops)
          if (sin[q].parent >= 0) end_top[(int64_t)(pp.start[q] + nchunks(pp.plen[q]) - 1) * kSchedLanes + pp.lane[q]] = q;
        for (int32_t t = 0; t < F; ++t)
          for (int32_t l = 0; l < kSchedLanes; ++l) {
            const int32_t q = end_top[(int64_t)t * kSchedLanes + l];
            if (q < 0) continue;
            const int32_t pb = sin[q].parent, pq = pp.top_of[pb];
            const int32_t npad = nchunks(pp.plen[pq]) * K - pp.plen[pq];
            P.faux.push_back((int16_t)entry_of(pq, npad + pp.below[pb]));
          }
        for (int32_t t = 0; t < F; ++t) {
          P.fmask.push_back(M[t]);
          P.fmask.push_back(E[t]);
        }
        W.naux = (int32_t)((int64_t)P.faux.size() - W.aux_off);
        P.kgroup[g].makespan = F;
        steps += F;
        elems += cum;
      }
      if (all_ok) {
        P.flow = true;
      } else {  // level-synchronous kernel instead
        std::vector<KFlow>().swap(P.kflow);
        std::vector<uint64_t>().swap(P.fmask);
        std::vector<uint16_t>().swap(P.fpos);
        std::vector<int16_t>().swap(P.faux);
      }
    }
    P.seg_offsets.assign(P.kseg.begin(), P.kseg.end());

    // ---- exported tables ----
    if (opt.keep_tables) {
      P.node_plan.swap(node_plan);
      P.u_src.swap(u_src);
      P.br_cell.swap(gcell);
      P.br_level.swap(glevel);
      P.br_first.swap(gfirst);
      P.br_dir.swap(gdir);
      P.br_len.swap(glen);
      P.br_parent.swap(gparent);
      P.br_rank.swap(grank);
      P.br_group.resize(nb);
      for (int64_t k = 0; k < nb; ++k) P.br_group[k] = group_of_cell[P.br_cell[k]];
    }
    return OK;
  }
};

}  // namespace

Status build_plan(const int32_t* parent, int64_t n, const int64_t* branch_offsets, int64_t nbranches,
                  const int64_t* cell_offsets, int64_t ncells, const Options& opt, HostPlan& out,
                  std::string& err) {
  try {
    Builder b(parent, n, branch_offsets, nbranches, cell_offsets, ncells, opt, out, err);
    return b.run();
  } catch (const std::bad_alloc&) {
    err = "host allocation failed during setup";
    return ERR_OOM;
  }
}

int64_t export_table(const HostPlan& p, int32_t id, int64_t* out, int64_t capacity) {
  auto put = [&](const auto& v) -> int64_t {
    int64_t cnt = (int64_t)v.size();
    if (out) {
      if (capacity < cnt) return -1;
      for (int64_t k = 0; k < cnt; ++k) out[k] = (int64_t)v[k];
    }
    return cnt;
  };
  if (!p.opt.keep_tables && (id == T_NODE_PLAN || id == T_BRANCHES || id == T_U_SRC || id == T_FLOW_MASKS ||
                             id == T_FLOW_POS || id == T_FLOW_AUX || id == T_CELL_POS || id == T_CELL_FLAGS))
    return -1;
  switch (id) {
    case T_NODE_PLAN: return put(p.node_plan);
    case T_U_SRC: return put(p.u_src);
    case T_BRANCHES: {
      int64_t nb = p.nbranches, cnt = nb * 8;
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t k = 0; k < nb; ++k) {
          int64_t* r = out + 8 * k;
          r[0] = p.br_cell[k];
          r[1] = p.br_level[k];
          r[2] = p.br_first[k];
          r[3] = p.br_dir[k];
          r[4] = p.br_len[k];
          r[5] = p.br_parent[k];
          r[6] = p.br_group[k];
          r[7] = p.br_rank[k];
        }
      }
      return cnt;
    }
    case T_GROUP_OFFSETS: return put(p.group_offsets);
    case T_GROUP_CELLS: return put(p.group_cells);
    case T_GROUP_SEG_OFFSETS: return put(p.group_seg_offsets);
    case T_SEG_OFFSETS: return put(p.seg_offsets);
    case T_LANES: return put(p.lanes);
    case T_FLOW_GROUPS: {
      const int64_t cnt = p.flow ? 8 * (int64_t)p.kflow.size() : 0;
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t g = 0; g < cnt / 8; ++g) {
          const KFlow& w = p.kflow[g];
          int64_t* r = out + 8 * g;
          r[0] = w.step_off;
          r[1] = w.pos_off;
          r[2] = w.aux_off;
          r[3] = w.nstep;
          r[4] = w.nelem;
          r[5] = w.naux;
          r[6] = w.nent;
          r[7] = kFlowChunk;
        }
      }
      return cnt;
    }
    case T_FLOW_MASKS: return put(p.fmask);
    case T_FLOW_POS: return put(p.fpos);
    case T_FLOW_AUX: return put(p.faux);
    case T_CELL_WAVES: {
      const int64_t cnt = 3 * (int64_t)p.cl.waves.size();
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t w = 0; w < cnt / 3; ++w) {
          out[3 * w] = p.cl.waves[w].chunk_off;
          out[3 * w + 1] = p.cl.waves[w].nchunk;
          out[3 * w + 2] = p.cl.waves[w].ncell;
        }
      }
      return cnt;
    }
    case T_CELL_LANES: return put(p.cl.lane_cell);
    case T_CELL_POS: return put(p.cl.pos);
    case T_CELL_FLAGS: return put(p.cl.flags);
    case T_CELL_MBSRC: return put(p.cl.mbsrc);
    case T_CELL_RANGE: return put(p.cl.range);
    case T_SEQ_WAVES: {
      const int64_t cnt = 3 * (int64_t)p.sq.waves.size();
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t w = 0; w < cnt / 3; ++w) {
          out[3 * w] = p.sq.waves[w].chunk_off;
          out[3 * w + 1] = p.sq.waves[w].nchunk;
          out[3 * w + 2] = p.sq.waves[w].ncell;
        }
      }
      return cnt;
    }
    case T_SEQ_LANES: return put(p.sq.lane_cell);
    case T_SEQ_POS: return put(p.sq.pos);
    case T_SEQ_CODE: return put(p.sq.code);
    case T_SEQ_MBSRC: return put(p.sq.mbsrc);
    case T_RES_GROUPS: {
      constexpr int64_t kF = 16;
      const int64_t cnt = kF * (int64_t)p.res.groups.size();
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t g = 0; g < cnt / kF; ++g) {
          const KResGroup& G = p.res.groups[g];
          int64_t* r = out + kF * g;
          r[0] = G.lo;
          r[1] = G.blob;
          r[2] = G.nslot;
          r[3] = G.ndma;
          r[4] = G.first;
          r[5] = G.count;
          r[6] = G.nchunk;
          r[7] = G.blob_units;
          r[8] = G.nroot;
          r[9] = G.npath;
          r[10] = G.nlist;
          r[11] = G.rec_off;
          r[12] = G.list_off;
          r[13] = G.cls;
          r[14] = kResK;
          r[15] = G.nflip;
        }
      }
      return cnt;
    }
    case T_RES_BLOB: {
      const int64_t cnt = (int64_t)p.res.blob.size() / 2;
      if (out) {
        if (capacity < cnt) return -1;
        for (int64_t k = 0; k < cnt; ++k) {
          uint16_t v;
          std::memcpy(&v, p.res.blob.data() + 2 * k, 2);
          out[k] = v;
        }
      }
      return cnt;
    }
    default: return -1;
  }
}

}  // namespace hines
