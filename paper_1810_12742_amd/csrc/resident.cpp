// Host tables of the LDS-resident solve (kernel k_solve_res).  Pure C++17.
//
// The elimination of paper §2 needs only that every compartment is eliminated
// after all its children.  Per group (consecutive whole cells, one wave) the
// compartments are covered by root-ward paths: from a top (a cell root or a
// "light" child) the path follows the heavy child down to a leaf, the heavy
// child of a compartment being the one whose subtree finishes last when every
// compartment runs as soon as its children are done.  A lane eliminates a
// path bottom-up in consecutive steps, so inside a path the contribution to
// the parent stays in registers; a light child's path adds its contribution
// into the parent's LDS entry at its last step.  Paths are placed as late as
// possible: the root paths end at the last step, and every other path must end
// at least one step before the step that eliminates its top's parent (§3's
// level-by-level order is replaced by these per-compartment deadlines).  A
// path goes on the lane whose earliest placed path starts latest.
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
  int32_t deadline, len, top;
};
// max deadline first, then the longer path, then the smaller top
inline bool ready_less(const Ready& a, const Ready& b) {
  if (a.deadline != b.deadline) return a.deadline < b.deadline;
  if (a.len != b.len) return a.len < b.len;
  return a.top > b.top;
}

struct Placed {
  int32_t lane, start, len, bottom, top;
};

// Schedule the compartments [0, m) of one group (local numbering, parent
// lpar[i] < i or -1) on 64 lanes within F steps.  Returns false if some path
// does not fit.
bool schedule_group(int32_t m, const std::vector<int32_t>& lpar, const std::vector<int32_t>& ch_off,
                    const std::vector<int32_t>& ch, const std::vector<int32_t>& heavy,
                    const std::vector<PathInfo>& path_of_top, int32_t F, std::vector<Placed>& placed) {
  placed.clear();
  int32_t frontier[kSchedLanes];
  for (int l = 0; l < kSchedLanes; ++l) frontier[l] = F;
  std::vector<Ready> heap;
  for (int32_t i = 0; i < m; ++i)
    if (lpar[i] < 0) heap.push_back({F - 1, path_of_top[i].len, i});
  std::make_heap(heap.begin(), heap.end(), ready_less);
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), ready_less);
    const Ready r = heap.back();
    heap.pop_back();
    int best = 0;
    for (int l = 1; l < kSchedLanes; ++l)
      if (frontier[l] > frontier[best]) best = l;
    const int32_t end = std::min(r.deadline, frontier[best] - 1);
    const int32_t start = end - r.len + 1;
    if (start < 0) return false;
    frontier[best] = start;
    const PathInfo& P = path_of_top[r.top];
    placed.push_back({best, start, r.len, P.bottom, r.top});
    // light children of every compartment of the path: their paths must end
    // one step before the compartment's step
    int32_t j = P.bottom;
    for (int32_t k = 0; k < r.len; ++k) {
      for (int32_t e = ch_off[j]; e < ch_off[j + 1]; ++e) {
        const int32_t c = ch[e];
        if (c == heavy[j]) continue;
        heap.push_back({start + k - 1, path_of_top[c].len, c});
        std::push_heap(heap.begin(), heap.end(), ready_less);
      }
      j = lpar[j];
    }
  }
  return true;
}

}  // namespace

Status build_resident(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                      ResPlan& out, std::string& err, int32_t pack) {
  out = ResPlan{};
  if (pack < 1 || pack > kResMaxSlots) {
    err = "resident pack size out of range";
    return ERR_OPTION;
  }
  out.par.assign((size_t)n + 2, 0);
  // groups of consecutive cells
  std::vector<int64_t> gc;  // first cell of each group, then ncells
  for (int64_t c = 0; c < ncells;) {
    gc.push_back(c);
    int64_t slots = cell_offsets[c + 1] - cell_offsets[c];
    int64_t c1 = c + 1;
    while (c1 < ncells && slots + (cell_offsets[c1 + 1] - cell_offsets[c1]) <= pack) {
      slots += cell_offsets[c1 + 1] - cell_offsets[c1];
      ++c1;
    }
    c = c1;
  }
  gc.push_back(ncells);
  const int64_t ng = (int64_t)gc.size() - 1;
  std::vector<int32_t> lpar, ch_off, ch, fin, heavy, fill;
  std::vector<PathInfo> path_of_top;
  std::vector<Placed> placed;
  std::vector<int32_t> lane_count(kSchedLanes + 1);
  for (int64_t g = 0; g < ng; ++g) {
    const int64_t u0 = cell_offsets[gc[g]], u1 = cell_offsets[gc[g + 1]];
    const int32_t m = (int32_t)(u1 - u0);
    KResGroup G{};
    G.lo = u0 & ~(int64_t)1;
    G.first = (int32_t)(u0 - G.lo);
    G.count = m;
    G.nslot = (G.first + m + 1) & ~1;
    G.ndma = (int32_t)std::min<int64_t>(G.nslot, n - G.lo);
    G.nroot = (int32_t)(gc[g + 1] - gc[g]);
    if (G.nslot > kResMaxSlots) {
      err = "a cell of " + std::to_string(m) + " compartments exceeds the resident kernel's LDS image";
      return ERR_TOO_BIG;
    }
    // local tree: children (ascending), finishing steps, heavy children
    lpar.assign(m, -1);
    ch_off.assign(m + 1, 0);
    for (int32_t i = 0; i < m; ++i) {
      const int32_t p = parent[u0 + i];
      lpar[i] = p < 0 ? -1 : (int32_t)(p - u0);
      if (p >= 0) ++ch_off[lpar[i] + 1];
    }
    for (int32_t i = 0; i < m; ++i) ch_off[i + 1] += ch_off[i];
    ch.assign(std::max(ch_off[m], 1), 0);
    fill.assign(ch_off.begin(), ch_off.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      if (lpar[i] >= 0) ch[fill[lpar[i]]++] = i;
    fin.assign(m, 0);
    heavy.assign(m, -1);
    for (int32_t i = m - 1; i >= 0; --i) {
      int32_t h = -1;
      for (int32_t e = ch_off[i]; e < ch_off[i + 1]; ++e)
        if (h < 0 || fin[ch[e]] > fin[h]) h = ch[e];  // last to finish; the smallest index on ties
      heavy[i] = h;
      fin[i] = h < 0 ? 0 : fin[h] + 1;
    }
    path_of_top.assign(m, PathInfo{-1, 0});
    int32_t F = 1;
    for (int32_t i = 0; i < m; ++i) {
      if (lpar[i] >= 0 && heavy[lpar[i]] == i) continue;
      int32_t b = i, len = 1;
      while (heavy[b] >= 0) {
        b = heavy[b];
        ++len;
      }
      path_of_top[i] = {b, len};
      if (lpar[i] < 0) F = std::max(F, fin[i] + 1);
    }
    while (!schedule_group(m, lpar, ch_off, ch, heavy, path_of_top, F, placed)) F += std::max(1, F / 32);
    if (F > 65535) {
      err = "resident schedule longer than 65535 steps";
      return ERR_TOO_BIG;
    }
    G.makespan = F;
    G.npath = (int32_t)placed.size();
    // records lane by lane in step order
    std::stable_sort(placed.begin(), placed.end(), [](const Placed& a, const Placed& b) {
      return a.lane != b.lane ? a.lane < b.lane : a.start < b.start;
    });
    std::fill(lane_count.begin(), lane_count.end(), 0);
    for (const Placed& p : placed) ++lane_count[p.lane + 1];
    for (int l = 0; l < kSchedLanes; ++l) lane_count[l + 1] += lane_count[l];
    const int64_t root_bytes = (2 * (int64_t)G.nroot + 15) & ~(int64_t)15;
    const int64_t rec_bytes = (8 * (int64_t)G.npath + 15) & ~(int64_t)15;
    const int64_t bytes = kResLaneTab + root_bytes + rec_bytes;
    G.blob_units = (int32_t)(bytes / 16);
    G.blob = (int64_t)out.blob.size() / 16;
    const size_t b0 = out.blob.size();
    out.blob.resize(b0 + bytes, 0);
    uint8_t* bp = out.blob.data() + b0;
    auto put16 = [&](int64_t off, uint16_t v) { std::memcpy(bp + off, &v, 2); };
    for (int l = 0; l <= kSchedLanes; ++l) put16(2 * l, (uint16_t)lane_count[l]);
    for (int32_t c = 0; c < G.nroot; ++c)
      put16(kResLaneTab + 2 * c, (uint16_t)(cell_offsets[gc[g] + c] - G.lo));
    for (int32_t k = 0; k < G.npath; ++k) {
      const Placed& p = placed[k];
      KResRec r;
      r.slot = (uint16_t)(p.bottom + G.first);
      r.t0 = (uint16_t)p.start;
      r.len = (uint16_t)p.len;
      r.aux = lpar[p.top] >= 0 ? 1 : 0;
      std::memcpy(bp + kResLaneTab + root_bytes + 8 * k, &r, 8);
    }
    for (int32_t i = 0; i < m; ++i)
      out.par[u0 + i] = (uint16_t)(lpar[i] < 0 ? G.nslot : lpar[i] + G.first);
    G.lds_bytes = (int32_t)res_lds_bytes(G.nslot, G.blob_units);
    if (G.lds_bytes > kLdsLimitBytes) {
      err = "a group of " + std::to_string(m) + " compartments exceeds LDS in the resident kernel";
      return ERR_TOO_BIG;
    }
    out.max_lds = std::max<int64_t>(out.max_lds, G.lds_bytes);
    out.groups.push_back(G);
  }
  out.built = true;
  return OK;
}

bool check_resident(const ResPlan& R, const int32_t* parent, int64_t n, std::string& why) {
  std::vector<int32_t> step, lane_of;
  std::vector<uint8_t> leaf;
  for (size_t g = 0; g < R.groups.size(); ++g) {
    const KResGroup& G = R.groups[g];
    const std::string gs = "resident group " + std::to_string(g);
    if (G.lo < 0 || (G.lo & 1) || G.first < 0 || G.first > 1 || G.count < 1 || G.nslot < G.first + G.count ||
        (G.nslot & 1) || G.nslot > kResMaxSlots || G.ndma < G.first + G.count || G.ndma > G.nslot ||
        G.lo + G.ndma > n || G.makespan < 1 || G.makespan > 65535 || G.blob < 0 ||
        16 * (G.blob + G.blob_units) > (int64_t)R.blob.size() || G.lds_bytes > kLdsLimitBytes ||
        G.lds_bytes != res_lds_bytes(G.nslot, G.blob_units)) {
      why = gs + ": record out of range";
      return false;
    }
    const uint8_t* bp = R.blob.data() + 16 * G.blob;
    auto get16 = [&](int64_t off) {
      uint16_t v;
      std::memcpy(&v, bp + off, 2);
      return (int32_t)v;
    };
    const int64_t root_bytes = (2 * (int64_t)G.nroot + 15) & ~(int64_t)15;
    if (kResLaneTab + root_bytes + 8 * (int64_t)G.npath > 16 * (int64_t)G.blob_units || get16(0) != 0 ||
        get16(2 * kSchedLanes) != G.npath) {
      why = gs + ": blob size";
      return false;
    }
    const int32_t s0 = G.first, s1 = G.first + G.count;
    step.assign(G.nslot, -1);
    leaf.assign(G.nslot, 1);
    for (int32_t s = s0; s < s1; ++s) {
      const int64_t i = G.lo + s;
      const int32_t ps = R.par[i];
      if (parent[i] < 0) {
        if (ps != G.nslot) {
          why = gs + ": root parent slot";
          return false;
        }
      } else {
        if (ps != parent[i] - G.lo || ps < s0 || ps >= s) {
          why = gs + ": parent slot";
          return false;
        }
        leaf[ps] = 0;
      }
    }
    for (int32_t c = 0; c < G.nroot; ++c) {
      const int32_t r = get16(kResLaneTab + 2 * c);
      if (r < s0 || r >= s1 || parent[G.lo + r] >= 0) {
        why = gs + ": root list";
        return false;
      }
    }
    for (int l = 0; l < kSchedLanes; ++l) {
      const int32_t a = get16(2 * l), b = get16(2 * l + 2);
      if (a > b || b > G.npath) {
        why = gs + ": lane offsets";
        return false;
      }
      int32_t busy_until = 0;
      for (int32_t k = a; k < b; ++k) {
        KResRec r;
        std::memcpy(&r, bp + kResLaneTab + root_bytes + 8 * k, 8);
        if (r.len < 1 || r.t0 < busy_until || (int32_t)r.t0 + r.len > G.makespan || r.slot < s0 || r.slot >= s1 ||
            !leaf[r.slot] || r.aux > 1) {
          why = gs + ": path record";
          return false;
        }
        busy_until = r.t0 + r.len;
        int32_t j = r.slot;
        for (int32_t q = 0; q < r.len; ++q) {
          if (j < s0 || j >= s1 || step[j] >= 0) {
            why = gs + ": path walk";
            return false;
          }
          step[j] = r.t0 + q;
          const int32_t pj = R.par[G.lo + j];
          if (q + 1 < r.len) {
            if (pj == G.nslot) {
              why = gs + ": path runs past a root";
              return false;
            }
            j = pj;
          } else if ((r.aux == 1) != (pj != G.nslot)) {
            why = gs + ": push flag";
            return false;
          }
        }
      }
    }
    for (int32_t s = s0; s < s1; ++s) {
      if (step[s] < 0) {
        why = gs + ": compartment not scheduled";
        return false;
      }
      const int32_t ps = R.par[G.lo + s];
      if (ps != G.nslot && step[ps] <= step[s]) {
        why = gs + ": a parent is eliminated before its child";
        return false;
      }
    }
  }
  return true;
}

}  // namespace hines
