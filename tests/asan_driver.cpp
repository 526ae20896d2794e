// Host-side table builders under AddressSanitizer / UndefinedBehaviorSanitizer.
// Reads a forest (n, ncells, parent[n], cell_offsets[ncells+1]) and option
// values from a binary file, builds the plan tables, the cell-lane tables (depth-
// first or index order) and the resident tables, runs their replay checks, and writes every exported
// table (int64, with its count) to the output file.  Built and run by
// tests/test_sanitizers.py with g++ only (no device code).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_1810_12742_amd/csrc/setup.hpp"

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[2], opts[8];
  if (std::fread(hdr, 8, 2, f) != 2) return 2;
  const int64_t n = hdr[0], nc = hdr[1];
  std::vector<int32_t> par(n);
  std::vector<int64_t> off(nc + 1);
  if ((int64_t)std::fread(par.data(), 4, n, f) != n || (int64_t)std::fread(off.data(), 8, nc + 1, f) != nc + 1 ||
      std::fread(opts, 8, 8, f) != 8)
    return 2;
  std::fclose(f);
  hines::Options o;
  o.host_only = 1;
  o.rebalance_root = (int32_t)opts[0];
  o.split_branches = (int32_t)opts[1];
  o.group_width = (int32_t)opts[2];
  o.cell_order = (int32_t)opts[3];
  o.max_group_unknowns = (int32_t)opts[4];
  o.level_balance = (int32_t)opts[5];
  o.scheduler = opts[6] ? 0 : 1;  // a cell-lane plan builds no flow schedule
  hines::HostPlan P;
  std::string err;
  hines::Status s = hines::build_plan(par.data(), n, nullptr, 0, off.data(), nc, o, P, err);
  if (s != hines::OK) {
    std::printf("build_plan: %d %s\n", (int)s, err.c_str());
    return 3;
  }
  if (opts[6] == 1) {
    s = hines::build_cell_lanes(par.data(), n, off.data(), nc, P.cl, err);
    if (s != hines::OK) {
      std::printf("build_cell_lanes: %d %s\n", (int)s, err.c_str());
      return 3;
    }
  } else if (opts[6] == 2) {
    s = hines::build_seq_lanes(par.data(), n, off.data(), nc, P.sq, err);
    if (s == hines::OK && !hines::check_seq_lanes(P.sq, par.data(), n, off.data(), nc, err)) s = hines::ERR_STATE;
    if (s != hines::OK) {
      std::printf("build_seq_lanes: %d %s\n", (int)s, err.c_str());
      return 3;
    }
  }
  if (opts[7]) {
    s = hines::build_resident(par.data(), n, off.data(), nc, P.res, err);
    if (s == hines::OK && !hines::check_resident(P.res, par.data(), n, err)) s = hines::ERR_STATE;
    if (s != hines::OK) {
      std::printf("build_resident: %d %s\n", (int)s, err.c_str());
      return 3;
    }
  }
  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  for (int32_t id = 0; id < hines::T_NUM; ++id) {
    const int64_t cnt = hines::export_table(P, id, nullptr, 0);
    std::vector<int64_t> v(cnt > 0 ? cnt : 0);
    if (cnt > 0) hines::export_table(P, id, v.data(), cnt);
    std::fwrite(&cnt, 8, 1, out);
    if (cnt > 0) std::fwrite(v.data(), 8, cnt, out);
  }
  std::fclose(out);
  return 0;
}
