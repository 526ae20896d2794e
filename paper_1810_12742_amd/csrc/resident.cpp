// Host tables of the LDS-resident solve (kernel k_solve_res).  Pure C++17.
//
// The elimination of paper §2 needs only that every compartment is eliminated
// after all its children.  Per group (consecutive whole cells, one wave) the
// compartments are covered by root-ward paths: from a top (a cell root or a
// "light" child) the path follows the heavy child down to a leaf, the heavy
// child of a compartment being the one whose subtree finishes last when every
// compartment runs as soon as its children are done.  A lane eliminates a
// path bottom-up in consecutive steps, kResK steps per chunk, so inside a path
// the contribution to the parent stays in registers; a light child's path adds
// its contribution into the parent's LDS entry at the end of its last chunk.
// Paths are placed as late as possible, in whole chunks: the root paths end in
// the last chunk, and every other path must end at least two chunks before
// the chunk that eliminates its top's parent (the kernel reads a chunk's
// operands while the chunk before it runs; §3's level-by-level order is
// replaced by these per-compartment deadlines).  A path goes on the lane whose
// earliest placed path starts latest.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "setup.hpp"

namespace hines {
namespace {

struct PathInfo {
  int32_t bottom, len;  // local indices; the top is the key of the path
};

struct Ready {
  int32_t deadline, nch, top;  // chunks
};
// max deadline first, then the longer path, then the smaller top
inline bool ready_less(const Ready& a, const Ready& b) {
  if (a.deadline != b.deadline) return a.deadline < b.deadline;
  if (a.nch != b.nch) return a.nch < b.nch;
  return a.top > b.top;
}

struct Placed {
  int32_t lane, c0, nch, top;
};

inline int32_t nchunks(int32_t len) { return (len + kResK - 1) / kResK; }

// Schedule the paths of one group (local numbering, parent lpar[i] < i or -1)
// on 64 lanes within NC chunks.  chunk_of[i] receives the chunk that
// eliminates compartment i.  Returns false if some path does not fit.
bool schedule_group(int32_t m, const std::vector<int32_t>& lpar, const std::vector<int32_t>& ch_off,
                    const std::vector<int32_t>& ch, const std::vector<int32_t>& heavy,
                    const std::vector<PathInfo>& path_of_top, int32_t NC, std::vector<Placed>& placed,
                    std::vector<int32_t>& chunk_of) {
  placed.clear();
  int32_t frontier[kSchedLanes];
  for (int l = 0; l < kSchedLanes; ++l) frontier[l] = NC;
  std::vector<Ready> heap;
  for (int32_t i = 0; i < m; ++i)
    if (lpar[i] < 0) heap.push_back({NC - 1, nchunks(path_of_top[i].len), i});
  std::make_heap(heap.begin(), heap.end(), ready_less);
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), ready_less);
    const Ready r = heap.back();
    heap.pop_back();
    int best = 0;
    for (int l = 1; l < kSchedLanes; ++l)
      if (frontier[l] > frontier[best]) best = l;
    const int32_t end = std::min(r.deadline, frontier[best] - 1);
    const int32_t c0 = end - r.nch + 1;
    if (c0 < 0) return false;
    frontier[best] = c0;
    placed.push_back({best, c0, r.nch, r.top});
    const PathInfo& P = path_of_top[r.top];
    const int32_t pad = r.nch * kResK - P.len;
    // step q of the path (0 = its bottom) runs in chunk c0 + (pad + q) / kResK;
    // light children of each of its compartments must end two chunks earlier
    int32_t j = P.bottom;
    for (int32_t q = 0; q < P.len; ++q) {
      const int32_t cj = c0 + (pad + q) / kResK;
      chunk_of[j] = cj;
      for (int32_t e = ch_off[j]; e < ch_off[j + 1]; ++e) {
        const int32_t c = ch[e];
        if (c == heavy[j]) continue;
        heap.push_back({cj - 2, nchunks(path_of_top[c].len), c});
        std::push_heap(heap.begin(), heap.end(), ready_less);
      }
      j = lpar[j];
    }
  }
  return true;
}

// Re-rooting at the tree centre (paper §6): the compartment of least
// eccentricity (largest hop distance to another compartment), the smaller
// index on ties.  lp: parents of one cell in local numbering (lp[0] = -1,
// lp[i] < i).  Fills path with the old root, its child toward the centre, ...,
// the centre (a single entry when the root is the centre).
void center_path(const int32_t* lp, int32_t m, std::vector<int32_t>& h, std::vector<int32_t>& up,
                 std::vector<int32_t>& b1, std::vector<int32_t>& b2, std::vector<int32_t>& path) {
  h.assign(m, 0);
  for (int32_t i = m - 1; i >= 1; --i) h[lp[i]] = std::max(h[lp[i]], h[i] + 1);
  b1.assign(m, -1);  // the two tallest children subtrees (height + 1) of each node
  b2.assign(m, -1);
  for (int32_t i = m - 1; i >= 1; --i) {
    const int32_t p = lp[i], v = h[i] + 1;
    if (v > b1[p]) {
      b2[p] = b1[p];
      b1[p] = v;
    } else if (v > b2[p]) {
      b2[p] = v;
    }
  }
  up.assign(m, 0);  // longest path that leaves i through its parent
  for (int32_t i = 1; i < m; ++i) {
    const int32_t p = lp[i];
    const int32_t other = b1[p] == h[i] + 1 ? b2[p] : b1[p];
    up[i] = std::max(up[p], std::max(other, 0)) + 1;
  }
  int32_t z = 0;
  for (int32_t i = 1; i < m; ++i)
    if (std::max(h[i], up[i]) < std::max(h[z], up[z])) z = i;
  path.clear();
  for (int32_t v = z; v >= 0; v = lp[v]) path.push_back(v);
  std::reverse(path.begin(), path.end());
}

// Smallest LDS class (most groups per CU) that holds the image.
int32_t res_class(int32_t nslot, int64_t blob_units) {
  for (int32_t k = kResClasses - 1; k >= 0; --k)
    if (nslot + 1 <= kResClassStride[k] && res_lds_bytes(k, blob_units) <= kResClassBytes[k]) return k;
  return -1;
}

}  // namespace

Status build_resident(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                      ResPlan& out, std::string& err, int32_t pack, bool reroot) {
  out = ResPlan{};
  if (pack < 1 || pack > kResMaxSlots) {
    err = "resident pack size out of range";
    return ERR_OPTION;
  }
  std::vector<int32_t> lpar, ch_off, ch, fin, heavy, fill, chunk_of, topo, roots, lp1, hh, uu, b1, b2, path;
  std::vector<std::pair<int32_t, int32_t>> flips;
  std::vector<PathInfo> path_of_top;
  std::vector<Placed> placed;
  std::vector<int32_t> lane_rec(kSchedLanes + 1), lane_list(kSchedLanes + 1);
  // One group: cells [ca, cb), re-rooted when rr.  Appends the group and its
  // blob on success; ERR_TOO_BIG (nothing appended) when the image does not
  // fit the largest LDS class.
  auto build_group = [&](int64_t ca, int64_t cb, bool rr) -> Status {
    const int64_t u0 = cell_offsets[ca], u1 = cell_offsets[cb];    const int64_t m64 = u1 - u0;
    KResGroup G{};
    G.lo = u0 & ~(int64_t)1;
    G.first = (int32_t)(u0 - G.lo);
    if (m64 + G.first + 2 > kResMaxSlots) {
      err = "a cell of " + std::to_string(m64) + " compartments exceeds the resident kernel's LDS image";
      return ERR_TOO_BIG;
    }
    const int32_t m = (int32_t)m64;
    G.count = m;
    G.nslot = (G.first + m + 1) & ~1;
    G.ndma = (int32_t)std::min<int64_t>(G.nslot, n - G.lo);
    G.nroot = (int32_t)(cb - ca);
    // local tree (re-rooted at each cell's centre on request): children
    // (ascending), finishing steps, heavy children
    lpar.assign(m, -1);
    for (int32_t i = 0; i < m; ++i) {
      const int32_t p = parent[u0 + i];
      lpar[i] = p < 0 ? -1 : (int32_t)(p - u0);
    }
    flips.clear();  // (slot whose coupling changes, slot it comes from)
    roots.clear();
    for (int64_t c = ca; c < cb; ++c) {
      const int32_t c0 = (int32_t)(cell_offsets[c] - u0), cm = (int32_t)(cell_offsets[c + 1] - cell_offsets[c]);
      int32_t z = c0;
      if (rr && cm > 2) {
        lp1.resize(cm);
        for (int32_t i = 0; i < cm; ++i) lp1[i] = i == 0 ? -1 : lpar[c0 + i] - c0;
        center_path(lp1.data(), cm, hh, uu, b1, b2, path);
        // the edges on the path from the old root to the centre turn round:
        // a_i's parent becomes a_(i+1), whose stored coupling (u of the old
        // child) is the coupling of that edge
        for (size_t k = 0; k + 1 < path.size(); ++k) {
          lpar[c0 + path[k]] = c0 + path[k + 1];
          flips.push_back({c0 + path[k] + G.first, c0 + path[k + 1] + G.first});
        }
        z = c0 + path.back();
        lpar[z] = -1;
      }
      roots.push_back(z + G.first);
    }
    ch_off.assign(m + 1, 0);
    for (int32_t i = 0; i < m; ++i)
      if (lpar[i] >= 0) ++ch_off[lpar[i] + 1];
    for (int32_t i = 0; i < m; ++i) ch_off[i + 1] += ch_off[i];
    ch.assign(std::max(ch_off[m], 1), 0);
    fill.assign(ch_off.begin(), ch_off.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      if (lpar[i] >= 0) ch[fill[lpar[i]]++] = i;
    // breadth-first order from the roots; children are finished before
    // their parents when it is taken backwards
    topo.clear();
    for (int32_t r : roots) topo.push_back(r - G.first);
    for (size_t k = 0; k < topo.size(); ++k)
      for (int32_t e = ch_off[topo[k]]; e < ch_off[topo[k] + 1]; ++e) topo.push_back(ch[e]);
    if ((int32_t)topo.size() != m) {
      err = "resident: the cells of a group do not form a forest";
      return ERR_STATE;
    }
    fin.assign(m, 0);
    heavy.assign(m, -1);
    for (int32_t k = m - 1; k >= 0; --k) {
      const int32_t i = topo[k];
      int32_t h = -1;
      for (int32_t e = ch_off[i]; e < ch_off[i + 1]; ++e)
        if (h < 0 || fin[ch[e]] > fin[h]) h = ch[e];  // last to finish; the smallest index on ties
      heavy[i] = h;
      fin[i] = h < 0 ? 0 : fin[h] + 1;
    }
    path_of_top.assign(m, PathInfo{-1, 0});
    int32_t NC = 1;
    for (int32_t i = 0; i < m; ++i) {
      if (lpar[i] >= 0 && heavy[lpar[i]] == i) continue;
      int32_t b = i, len = 1;
      while (heavy[b] >= 0) {
        b = heavy[b];
        ++len;
      }
      path_of_top[i] = {b, len};
      if (lpar[i] < 0) NC = std::max(NC, nchunks(len));
    }
    chunk_of.assign(m, -1);
    while (!schedule_group(m, lpar, ch_off, ch, heavy, path_of_top, NC, placed, chunk_of))
      NC += std::max(1, NC / 32);
    if (NC > 65535) {
      err = "resident schedule longer than 65535 chunks";
      return ERR_TOO_BIG;
    }
    G.nchunk = NC;
    G.npath = (int32_t)placed.size();
    const int32_t nrec = G.npath + kSchedLanes + 1;  // records and sentinels
    // records lane by lane in chunk order; list entries in the same order
    std::stable_sort(placed.begin(), placed.end(), [](const Placed& a, const Placed& b) {
      return a.lane != b.lane ? a.lane < b.lane : a.c0 < b.c0;
    });
    std::fill(lane_rec.begin(), lane_rec.end(), 0);
    std::fill(lane_list.begin(), lane_list.end(), 0);
    for (const Placed& p : placed) {
      ++lane_rec[p.lane + 1];
      lane_list[p.lane + 1] += p.nch;
    }
    // records: an idle sentinel before every lane's records and after the
    // last lane's, so a lane reads its next (or previous) record ahead of
    // use without a bounds test
    lane_rec[0] = 1;
    for (int l = 0; l < kSchedLanes; ++l) {
      lane_rec[l + 1] += lane_rec[l] + 1;
      lane_list[l + 1] += lane_list[l];
    }
    G.nlist = lane_list[kSchedLanes];
    if (nrec > 65535 || G.nlist > 65535) {
      err = "resident group with too many paths";
      return ERR_TOO_BIG;
    }
    const int64_t root_bytes = (2 * (int64_t)G.nroot + 15) & ~(int64_t)15;
    G.nflip = (int32_t)flips.size();
    const int64_t flip_bytes = (4 * (int64_t)G.nflip + 15) & ~(int64_t)15;
    const int64_t rec_bytes = (8 * (int64_t)nrec + 15) & ~(int64_t)15;
    // one spare entry past the last: a lane reads its next entry ahead of use
    const int64_t list_bytes = (kResEntBytes * ((int64_t)G.nlist + 1) + 15) & ~(int64_t)15;
    G.rec_off = kResLaneTab + (int32_t)(root_bytes + flip_bytes);
    G.list_off = G.rec_off + (int32_t)rec_bytes;
    const int64_t bytes = G.list_off + list_bytes;
    G.blob_units = (int32_t)(bytes / 16);
    G.cls = res_class(G.nslot, G.blob_units);
    if (G.cls < 0) {
      err = "a group of " + std::to_string(m) + " compartments exceeds LDS in the resident kernel";
      return ERR_TOO_BIG;
    }
    G.blob = (int64_t)out.blob.size() / 16;
    const size_t b0 = out.blob.size();
    out.blob.resize(b0 + bytes, 0);
    uint8_t* bp = out.blob.data() + b0;
    auto put16 = [&](int64_t off, uint16_t v) { std::memcpy(bp + off, &v, 2); };
    for (int l = 0; l <= kSchedLanes; ++l) {
      put16(2 * l, (uint16_t)lane_rec[l]);
      put16(2 * (kSchedLanes + 1) + 2 * l, (uint16_t)lane_list[l]);
    }
    for (int32_t c = 0; c < G.nroot; ++c) put16(kResLaneTab + 2 * c, (uint16_t)roots[c]);
    for (int32_t k = 0; k < G.nflip; ++k) {
      put16(kResLaneTab + root_bytes + 4 * k, (uint16_t)flips[k].first);
      put16(kResLaneTab + root_bytes + 4 * k + 2, (uint16_t)flips[k].second);
    }
    const uint16_t zero_off = (uint16_t)(8 * G.nslot);
    const KResRec idle{0xffff, 0, (uint16_t)kResNoParent, 0};
    for (int l = 0; l <= kSchedLanes; ++l) std::memcpy(bp + G.rec_off + 8 * (lane_rec[l] - 1), &idle, 8);
    int64_t le = 0;
    for (int32_t k = 0; k < G.npath; ++k) {
      const Placed& p = placed[k];
      const PathInfo& P = path_of_top[p.top];
      KResRec r;
      r.c0 = (uint16_t)p.c0;
      r.nch = (uint16_t)p.nch;
      r.par = lpar[p.top] >= 0 ? (uint16_t)(8 * (lpar[p.top] + G.first)) : (uint16_t)kResNoParent;
      r.spare = 0;
      std::memcpy(bp + G.rec_off + 8 * ((int64_t)k + p.lane + 1), &r, 8);  // k records and lane + 1 sentinels before
      // slot lists: the path's steps from its bottom up, padding first
      const int32_t pad = p.nch * kResK - P.len;
      int32_t j = P.bottom;
      for (int32_t s = 0; s < p.nch * kResK; ++s) {
        uint16_t v = zero_off;
        if (s >= pad) {
          v = (uint16_t)(8 * (j + G.first));
          j = lpar[j];
        }
        put16(G.list_off + kResEntBytes * le + 2 * (s % kResK), v);
        if (s % kResK == kResK - 1) ++le;
      }
    }
    out.max_lds = std::max<int64_t>(out.max_lds, res_lds_bytes(G.cls, G.blob_units));
    out.groups.push_back(G);
    return OK;
  };
  // groups of consecutive cells of at most `pack` compartments (a larger
  // cell alone); a group whose image does not fit LDS is built again with
  // half its cells, and a single cell that does not fit re-rooted is built
  // from its own root
  for (int64_t c = 0; c < ncells;) {
    int64_t slots = cell_offsets[c + 1] - cell_offsets[c];
    int64_t c1 = c + 1;
    while (c1 < ncells && slots + (cell_offsets[c1 + 1] - cell_offsets[c1]) <= pack) {
      slots += cell_offsets[c1 + 1] - cell_offsets[c1];
      ++c1;
    }
    bool rr = reroot;
    for (;;) {
      const Status st = build_group(c, c1, rr);
      if (st == OK) break;
      if (st != ERR_TOO_BIG) return st;
      if (c1 - c > 1) {
        c1 = c + (c1 - c) / 2;
      } else if (rr) {
        rr = false;
      } else {
        return st;
      }
    }
    c = c1;
  }
  out.built = true;
  return OK;
}

bool check_resident(const ResPlan& R, const int32_t* parent, int64_t n, std::string& why) {
  std::vector<int32_t> chunk, sub, top_end, np, cell_of;
  for (size_t g = 0; g < R.groups.size(); ++g) {
    const KResGroup& G = R.groups[g];
    const std::string gs = "resident group " + std::to_string(g);
    if (G.lo < 0 || (G.lo & 1) || G.first < 0 || G.first > 1 || G.count < 1 || G.nslot < G.first + G.count ||
        (G.nslot & 1) || G.nslot + 2 > kResMaxSlots || G.ndma < G.first + G.count || G.ndma > G.nslot ||
        G.lo + G.ndma > n || G.nchunk < 1 || G.nchunk > 65535 || G.blob < 0 || G.cls < 0 || G.cls >= kResClasses ||
        G.nslot + 1 > kResClassStride[G.cls] || res_lds_bytes(G.cls, G.blob_units) > kResClassBytes[G.cls] ||
        16 * (G.blob + G.blob_units) > (int64_t)R.blob.size() || G.rec_off < kResLaneTab ||
        (G.rec_off & 7) || (G.list_off & 7)) {
      why = gs + ": record out of range";
      return false;
    }
    const uint8_t* bp = R.blob.data() + 16 * G.blob;
    auto get16 = [&](int64_t off) {
      uint16_t v;
      std::memcpy(&v, bp + off, 2);
      return (int32_t)v;
    };
    const int32_t nrec = G.npath + kSchedLanes + 1;
    if (get16(0) != 1 || get16(2 * kSchedLanes) != nrec || get16(2 * (kSchedLanes + 1)) != 0 ||
        get16(2 * (kSchedLanes + 1) + 2 * kSchedLanes) != G.nlist || G.list_off < G.rec_off + 8 * nrec ||
        G.list_off + kResEntBytes * ((int64_t)G.nlist + 1) > 16 * (int64_t)G.blob_units) {
      why = gs + ": lane table";
      return false;
    }
    const int32_t s0 = G.first, s1 = G.first + G.count;
    chunk.assign(G.nslot, -1);
    sub.assign(G.nslot, -1);
    top_end.assign(G.nslot, -1);  // for a path top: the chunk of its contribution
    // the (re-rooted) parent slot of every compartment: the user parents with
    // the pairs of the blob turned round and the listed roots cut off
    np.assign(G.nslot, -1);
    cell_of.assign(G.nslot, -1);
    int32_t ncell = -1;
    for (int32_t s = s0; s < s1; ++s) {
      const int64_t p = parent[G.lo + s];
      if (p < 0) ++ncell;
      cell_of[s] = ncell;
      np[s] = p < 0 ? -1 : (int32_t)(p - G.lo);
    }
    const int64_t root_bytes = (2 * (int64_t)G.nroot + 15) & ~(int64_t)15;
    if (G.nflip < 0 || G.rec_off < kResLaneTab + root_bytes + 4 * (int64_t)G.nflip || ncell + 1 != G.nroot) {
      why = gs + ": root and re-rooting lists";
      return false;
    }
    for (int32_t k = 0; k < G.nflip; ++k) {
      const int32_t dst = get16(kResLaneTab + root_bytes + 4 * k), src = get16(kResLaneTab + root_bytes + 4 * k + 2);
      // src must be dst's child in the user tree: its coupling is the edge's
      if (dst < s0 || dst >= s1 || src < s0 || src >= s1 || parent[G.lo + src] != G.lo + dst) {
        why = gs + ": re-rooting pair";
        return false;
      }
      np[dst] = src;
    }
    for (int32_t c = 0; c < G.nroot; ++c) {
      const int32_t r = get16(kResLaneTab + 2 * c);
      if (r < s0 || r >= s1 || cell_of[r] != c) {
        why = gs + ": root list";
        return false;
      }
      np[r] = -1;
    }
    for (int32_t s = s0; s < s1; ++s) {  // every compartment reaches its cell's root
      int32_t v = s, hops = 0;
      while (np[v] >= 0 && hops <= G.count) {
        if (cell_of[np[v]] != cell_of[s]) {
          why = gs + ": re-rooted parent outside the cell";
          return false;
        }
        v = np[v];
        ++hops;
      }
      if (np[v] >= 0) {
        why = gs + ": re-rooted parents form a cycle";
        return false;
      }
    }
    auto sentinel = [&](int32_t k) {
      KResRec r;
      std::memcpy(&r, bp + G.rec_off + 8 * (int64_t)k, 8);
      return r.c0 == 0xffff && r.nch == 0 && r.par == kResNoParent;
    };
    for (int l = 0; l < kSchedLanes; ++l) {
      // records [a, b); sentinels at a - 1 and b
      const int32_t a = get16(2 * l), b = get16(2 * l + 2) - 1;
      const int32_t la = get16(2 * (kSchedLanes + 1) + 2 * l), lb = get16(2 * (kSchedLanes + 1) + 2 * l + 2);
      if (a < 1 || a > b || b >= nrec || la > lb || lb > G.nlist || !sentinel(a - 1) || !sentinel(b)) {
        why = gs + ": lane offsets";
        return false;
      }
      int32_t busy_until = 0, le = la;
      for (int32_t k = a; k < b; ++k) {
        KResRec r;
        std::memcpy(&r, bp + G.rec_off + 8 * k, 8);
        if (r.nch < 1 || r.c0 < busy_until || (int32_t)r.c0 + r.nch > G.nchunk || le + r.nch > lb) {
          why = gs + ": path record";
          return false;
        }
        busy_until = r.c0 + r.nch;
        // walk the path's list: padding (the zero entry) first, then a chain
        // of parents up to the top
        int32_t prev = -1;
        bool started = false;
        for (int32_t s = 0; s < r.nch * kResK; ++s) {
          const int32_t v = get16(G.list_off + kResEntBytes * (le + s / kResK) + 2 * (s % kResK));
          if (v & 7) {
            why = gs + ": list entry alignment";
            return false;
          }
          const int32_t slot = v / 8;
          if (slot == G.nslot) {
            if (started) {
              why = gs + ": padding above a path's bottom";
              return false;
            }
            continue;
          }
          if (slot < s0 || slot >= s1 || chunk[slot] >= 0) {
            why = gs + ": path walk";
            return false;
          }
          if (started) {
            if (np[prev] != slot) {
              why = gs + ": path does not follow parents";
              return false;
            }
          }
          started = true;
          chunk[slot] = r.c0 + s / kResK;
          sub[slot] = s % kResK;
          prev = slot;
        }
        if (!started || sub[prev] != kResK - 1 || chunk[prev] != busy_until - 1) {
          why = gs + ": a path top is not the last step of its last chunk";
          return false;
        }
        const int32_t want = np[prev] < 0 ? kResNoParent : 8 * np[prev];
        if (r.par != want) {
          why = gs + ": push target";
          return false;
        }
        top_end[prev] = busy_until - 1;
        le += r.nch;
      }
      if (le != lb) {
        why = gs + ": list entries of lane " + std::to_string(l);
        return false;
      }
    }
    for (int32_t s = s0; s < s1; ++s) {
      if (chunk[s] < 0) {
        why = gs + ": compartment not scheduled";
        return false;
      }
      if (np[s] < 0) continue;
      const int32_t ps = np[s];
      if (top_end[s] >= 0) {
        // a light path's top: its contribution lands two chunks before the
        // chunk that eliminates the parent (and the parent's x is written two
        // chunks before the forward sweep reads it)
        if (chunk[ps] < top_end[s] + 2) {
          why = gs + ": a light path ends too late for its parent";
          return false;
        }
      } else if (!(chunk[ps] * kResK + sub[ps] == chunk[s] * kResK + sub[s] + 1)) {
        why = gs + ": a path's next step is not its parent";
        return false;
      }
    }
  }
  return true;
}

}  // namespace hines
